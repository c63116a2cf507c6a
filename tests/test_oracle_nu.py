"""Pins of the quasi-random Fermi-Dirac sampling (Sec. 2.1, Appendix A)."""
import json
import os

import numpy as np
from scipy import integrate
from scipy.special import zeta

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
f = lambda q: 1.0 / (np.exp(q) + 1.0)


def test_shell_masses_and_moments_degenerate():
    e, q, m = O.fd_shells([1.0], 10)
    assert e[0] == 0 and e[-1] == 30.0 and np.all(np.diff(e) > 0)
    assert abs(m.sum() - 1) < 1e-13
    # sum m q^2 = int q^4 f / int q^2 f -> 15 zeta(5)/zeta(3) (tail beyond 30 < 1e-9)
    assert abs((m * q ** 2).sum() / (15 * zeta(5) / zeta(3)) - 1) < 1e-8
    # each shell speed lies inside its shell; RMS per shell >= mean speed overall
    assert np.all((q > e[:-1]) & (q < e[1:]))
    mean_q = (7 * np.pi ** 4 / 120) / (1.5 * zeta(3))    # int q^3 f / int q^2 f = 3.1514
    assert abs(mean_q - 3.15137) < 1e-5
    assert (m * q).sum() > mean_q                         # RMS per shell >= mean (Jensen)


def test_shells_equal_area_of_kernel_q_f_independent_quadrature():
    e, q, m = O.fd_shells([1.0], 10)
    tot = integrate.quad(lambda t: t * f(t), 0, 30, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs(tot - np.pi ** 2 / 12) < 1e-10          # int_0^inf q f = pi^2/12
    n2 = integrate.quad(lambda t: t * t * f(t), 0, 30, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs(n2 - 1.5 * zeta(3)) < 1e-9
    for i in range(10):
        g = integrate.quad(lambda t: t * f(t), e[i], e[i + 1], epsabs=0, epsrel=1e-13)[0]
        assert abs(g / (tot / 10) - 1) < 1e-9
        q2 = integrate.quad(lambda t: t ** 2 * f(t), e[i], e[i + 1], epsabs=0, epsrel=1e-13)[0]
        q4 = integrate.quad(lambda t: t ** 4 * f(t), e[i], e[i + 1], epsabs=0, epsrel=1e-13)[0]
        assert abs(q[i] / np.sqrt(q4 / q2) - 1) < 1e-10
        assert abs(m[i] / (q2 / n2) - 1) < 1e-9


def test_effective_distribution_degenerate_limit_and_mass_conservation():
    # degenerate limit reproduces f (Appendix A, last paragraph)
    e1, q1, m1 = O.fd_shells([1.0], 10)
    e3, q3, m3 = O.fd_shells([1.0, 1.0, 1.0], 10)
    assert np.abs(e1 - e3).max() < 1e-12 and np.abs(q1 - q3).max() < 1e-12
    # int q^2 f~ = sum_j alpha_j^4 int q^2 f(alpha q) = 1.5 zeta(3) sum_j alpha_j
    alpha = [1.0, 0.1754126379477057, 0.024234911725705265]
    tot = integrate.quad(lambda t: t * t * O.fd_tilde(alpha, t), 0, 30 / alpha[2],
                         epsabs=0, epsrel=1e-12, limit=500)[0]
    assert abs(tot / (1.5 * zeta(3) * sum(alpha)) - 1) < 1e-8
    e, q, m = O.fd_shells(alpha, 10)
    assert abs(e[-1] - 30 / alpha[2]) < 1e-9 and abs(m.sum() - 1) < 1e-12
    # light eigenstates add slow tails: the last shell reaches far beyond the degenerate one
    assert q[-1] > q1[-1] * 3


def test_fibonacci_directions():
    for nf in (3, 20):
        d = O.fibonacci(nf)
        assert d.shape == (2 * nf + 1, 3)
        assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-14
        assert abs(d[:, 1].sum()) < 1e-12 and abs(d[:, 2].sum()) < 1e-12
        # equal-area bands: z equally spaced
        assert np.abs(np.diff(d[:, 2]) - 2 / (2 * nf + 1)).max() < 1e-12
    d = O.fibonacci(20)
    cov = d.T @ d / len(d)
    assert np.abs(np.diag(cov) - 1 / 3).max() < 5e-3
    assert abs(O.fibonacci(3)[:, 0].sum() - 0.357) < 1e-3   # the x sum does not vanish


def _count(cfg):
    s = O.make_sim(dict(box=1000.0, n_mesh=16, n_cdm=cfg.get("n_cdm", 8), n_sites=cfg["n_sites"],
                        n_shell=cfg["n_shell"], n_fib=cfg["n_fib"], omega_m=0.3, h=0.7, n_s=0.96,
                        sigma8=0.8, m_nu=[0.1 / 3] * 3, a0=0.01))
    return O.num_particles(s)


def test_particle_counts_printed_in_paper():
    g = GOLD["pseudo_vs_quasi_count_ratio"]
    _, _, nn = _count(g["inputs"])
    assert round(nn / g["inputs"]["n_pseudo_side"] ** 3, g["decimals"]) == g["value"]
    for key in ("nu_to_cdm_count_NC512_NF3", "nu_to_cdm_count_NC512_NF20"):
        g = GOLD[key]
        _, nc, nn = _count(g["inputs"])
        assert nc == g["inputs"]["n_cdm"] ** 3
        assert round(nn / nc, g["decimals"]) == g["value"]
