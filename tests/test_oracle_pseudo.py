"""Pins of the oracle's pseudo-random neutrino sampling (the baseline the
paper compares its quasi-random shells with, Sec. 3): the inverse of the
cumulative number distribution against independent quadrature and a closed
moment, and the assembly of the initial conditions (site + bulk displacement;
thermal momentum = speed x direction from the uniforms)."""
import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from paper_2007_13394_amd import inputs as I


def _fd_int(y):
    """int_0^y t^2 / (e^t + 1) dt by adaptive quadrature."""
    return integrate.quad(lambda t: t * t * special.expit(-t), 0.0, y, epsabs=0, epsrel=1e-13, limit=200)[0]


def _fd_cdf(q, qmax=30.0):
    return _fd_int(q) / _fd_int(qmax)


@pytest.mark.parametrize("u", [1e-4, 0.01, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99, 0.9999])
def test_inverse_cdf_degenerate_against_quadrature(u):
    q = O.orc.fd_qinv(3, np.ones(3), u)
    assert abs(_fd_cdf(q) - u) < 1e-10


def test_inverse_cdf_ends_and_monotone():
    us = np.linspace(0, 1, 41)
    qs = [O.orc.fd_qinv(3, np.ones(3), u) for u in us]
    assert qs[0] == 0.0 and qs[-1] == 30.0
    assert np.all(np.diff(qs) > 0)


def test_inverse_cdf_of_three_masses_is_a_mixture():
    """For unequal masses the number distribution is a sum of Fermi-Dirac
    terms in alpha_j q; its cumulative is the alpha_j-weighted mixture of the
    one-species integrals at alpha_j q (cut-off at 30 / min alpha)."""
    alpha = np.array([1.0, 0.175, 0.024])
    qmax = 30.0 / alpha.min()
    tot = sum(aj * _fd_int(aj * qmax) for aj in alpha)
    for u in (0.05, 0.3, 0.6, 0.95):
        q = O.orc.fd_qinv(3, alpha, u)
        c = sum(aj * _fd_int(aj * q) for aj in alpha) / tot
        assert abs(c - u) < 1e-9


def test_mean_square_speed_of_the_samples():
    """The mean of Q(u)^2 over uniform u equals int q^4 f / int q^2 f =
    15 zeta(5) / zeta(3) for Fermi-Dirac (the cut-off at q = 30 changes it by
    ~e^-30)."""
    q2 = lambda u: O.orc.fd_qinv(3, np.ones(3), u) ** 2  # noqa: E731
    m2 = sum(integrate.quad(q2, a, b, epsabs=1e-12, epsrel=1e-9, limit=400)[0]
             for a, b in ((0.0, 0.99), (0.99, 0.99999), (0.99999, 1.0)))
    assert abs(m2 / (15 * special.zeta(5) / special.zeta(3)) - 1) < 1e-7


def test_pseudo_random_initial_conditions_assembly():
    cfg = dict(I.config("C1p"), n_mesh=16, n_cdm=8, n_sites=8)
    sim = O.make_sim(cfg)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((8, 8, 8)).astype(np.float32)
    ns = 8 ** 3
    u = rng.random((3, ns))
    x, p = O.ic_pseudo(sim, w, u)
    # the bulk displacement at the sites, and G/D, from the quasi-random path on the same noise
    _, _, dcdm, dnu = O.ic(sim, w, want_disp=True)
    P, nc, nn = O.num_particles(sim)
    assert nn == ns
    xc, pc = x[:, :nc], p[:, :nc]
    vfac = np.sum(pc * dcdm) / np.sum(dcdm * dcdm)
    assert np.allclose(pc, vfac * dcdm, rtol=1e-12, atol=1e-14)
    n = cfg["n_mesh"]
    j = np.arange(ns)
    site = np.stack([((j // 64) + 0.5) * 2.0, ((j // 8) % 8 + 0.5) * 2.0, (j % 8 + 0.5) * 2.0])
    dx = np.mod(x[:, nc:] - site - dnu + n / 2, n) - n / 2
    assert np.max(np.abs(dx)) < 1e-10
    th = p[:, nc:] - vfac * dnu
    speed = np.linalg.norm(th, axis=0)
    qs = np.array([O.orc.fd_qinv(3, np.ones(3), v) for v in u[0]])
    ratio = speed / qs
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    assert np.allclose(th[2] / speed, 2 * u[1] - 1, atol=1e-12)
    phi = np.mod(np.arctan2(th[1], th[0]), 2 * np.pi)
    assert np.allclose(np.cos(phi - 2 * np.pi * u[2]), 1.0, atol=1e-10)
