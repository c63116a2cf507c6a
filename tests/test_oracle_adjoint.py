"""Pins of the oracle reverse mode (the adjoint PM step, the density transpose
and the initial-condition transpose) against central finite differences of the
oracle's own FP64 forward model on 16^3 and 32^3 instances.

Each check compares <grad, v> with (L(z + h v) - L(z - h v)) / 2h along random
directions v.  The model is piecewise polynomial in the positions (cloud-in-cell
weights), so the difference quotient is exact up to O(h^2) as long as no
particle crosses a cell face between the two evaluations; positions are kept
away from faces, and the chained check resamples a direction that makes a
particle cross.  Position differences are unwrapped (the periodic wrap has unit
derivative)."""
import numpy as np
import pytest

import oracle as O
from paper_2007_13394_amd import inputs as I


def _sim(name):
    return O.make_sim(I.config(name))


def _away_from_faces(rng, n, P, lo=0.05, hi=0.95):
    cells = rng.integers(0, n, size=(3, P))
    return cells + rng.uniform(lo, hi, size=(3, P))


def _unwrap(dx, n):
    return (dx + n / 2) % n - n / 2


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_force_vjp_matches_finite_differences(name):
    sim = _sim(name)
    n = sim.n_mesh
    P, _, _ = O.num_particles(sim)
    rng = np.random.default_rng(11)
    x = _away_from_faces(rng, n, P)
    g = rng.standard_normal((3, P))
    xbar = O.force_vjp(sim, x, g)
    h = 1e-6
    for _ in range(4):
        v = rng.standard_normal((3, P))
        fd = (np.sum(g * O.force_cont(sim, x + h * v)) - np.sum(g * O.force_cont(sim, x - h * v))) / (2 * h)
        assert _rel(fd, np.sum(xbar * v)) < 1e-6


def test_force_vjp_paint_term_is_needed():
    """A dropped paint transpose (readout derivative only) fails the check:
    the two terms are of comparable size for a clustered state."""
    sim = _sim("C5_fd16")
    n = sim.n_mesh
    P, _, _ = O.num_particles(sim)
    rng = np.random.default_rng(12)
    x = _away_from_faces(rng, n, P)
    g = rng.standard_normal((3, P))
    full = O.force_vjp(sim, x, g)
    # readout-only part: derivative of sum_i g_i . interp(Phi)(x_i) with Phi frozen
    delta = O.density_cont(sim, x)
    F = O.force_mesh_from_delta(delta, sim.cosmo.omega_m)
    h = 1e-6
    v = rng.standard_normal((3, P))
    fd_frozen = (np.sum(g * O.readout(F, x + h * v)) - np.sum(g * O.readout(F, x - h * v))) / (2 * h)
    assert _rel(fd_frozen, np.sum(full * v)) > 1e-3


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_step_vjp_matches_finite_differences(name):
    sim = _sim(name)
    n = sim.n_mesh
    P, _, _ = O.num_particles(sim)
    rng = np.random.default_rng(13)
    x = _away_from_faces(rng, n, P)
    p = 0.05 * rng.standard_normal((3, P))
    kick, drift = 0.7, 1.3
    a, b = rng.standard_normal((3, P)), rng.standard_normal((3, P))

    def fwd(x0, p0):
        xx, pp = np.ascontiguousarray(x0), np.ascontiguousarray(p0.copy())
        xx = xx.copy()
        O.step_cont(sim, xx, pp, kick, drift)
        return xx, pp

    xb, pb = O.step_vjp(sim, x, kick, drift, a, b)
    h = 1e-6
    for _ in range(3):
        vx, vp = rng.standard_normal((3, P)), rng.standard_normal((3, P))
        x1, p1 = fwd(x + h * vx, p + h * vp)
        x2, p2 = fwd(x - h * vx, p - h * vp)
        fd = (np.sum(a * _unwrap(x1 - x2, n)) + np.sum(b * (p1 - p2))) / (2 * h)
        assert _rel(fd, np.sum(xb * vx) + np.sum(pb * vp)) < 1e-6


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_density_vjp_matches_finite_differences(name):
    sim = _sim(name)
    n = sim.n_mesh
    P, _, _ = O.num_particles(sim)
    rng = np.random.default_rng(14)
    x = _away_from_faces(rng, n, P)
    A = rng.standard_normal((n, n, n))
    xbar = O.density_vjp(sim, x, A)
    h = 1e-6
    for _ in range(3):
        v = rng.standard_normal((3, P))
        fd = (np.sum(A * O.density_cont(sim, x + h * v)) - np.sum(A * O.density_cont(sim, x - h * v))) / (2 * h)
        assert _rel(fd, np.sum(xbar * v)) < 1e-6


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_ic_vjp_matches_finite_differences(name):
    """Positions and momenta are linear in the white noise (up to the wrap)."""
    sim = _sim(name)
    n = sim.n_mesh
    P, _, _ = O.num_particles(sim)
    rng = np.random.default_rng(15)
    w = rng.standard_normal((sim.n_cdm,) * 3)
    a, b = rng.standard_normal((3, P)), rng.standard_normal((3, P))
    wbar = O.ic_vjp(sim, a, b)
    h = 1e-3
    for _ in range(3):
        v = rng.standard_normal(w.shape)
        x1, p1 = O.ic_w64(sim, w + h * v)
        x2, p2 = O.ic_w64(sim, w - h * v)
        fd = (np.sum(a * _unwrap(x1 - x2, n)) + np.sum(b * (p1 - p2))) / (2 * h)
        assert _rel(fd, np.sum(wbar * v)) < 1e-9


def _chain(sim, cfg, w, target, keep=False):
    """w -> initial conditions -> KDK run -> density -> L2 loss."""
    a, half = O.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"])
    calls = O.kdk_calls(a, half)
    kick, drift = O.kdk_factors(sim.cosmo, *[list(c) for c in zip(*calls)])
    x, p = O.ic_w64(sim, w)
    x, p = np.ascontiguousarray(x), np.ascontiguousarray(p)
    cps = []
    for i in range(len(calls)):
        cps.append(x.copy())
        O.step_cont(sim, x, p, kick[i], drift[i])
    d = O.density_cont(sim, x)
    loss = float(np.sum((d - target) ** 2))
    return (loss, x, cps, kick, drift, d) if keep else (loss, x, cps)


def _chain_grad(sim, cfg, w, target):
    loss, x, cps, kick, drift, d = _chain(sim, cfg, w, target, keep=True)
    xbar = O.density_vjp(sim, x, 2.0 * (d - target))
    pbar = np.zeros_like(xbar)
    for i in reversed(range(len(cps))):
        xbar, pbar = O.step_vjp(sim, cps[i], kick[i], drift[i], xbar, pbar)
    return loss, O.ic_vjp(sim, xbar, pbar)


@pytest.mark.parametrize("name", ["C5_fd16", "C5_fd32"])
def test_full_chain_gradient_wrt_initial_modes(name):
    cfg = I.config(name)
    sim = O.make_sim(cfg)
    nc = cfg["n_cdm"]
    w = I.white_noise(cfg["seed"] + 100, nc).astype(np.float64)
    target = O.density_cont(sim, _chain(sim, cfg, I.white_noise(cfg["seed"], nc).astype(np.float64),
                                        np.zeros((cfg["n_mesh"],) * 3))[1])
    loss, wbar = _chain_grad(sim, cfg, w, target)
    assert loss > 0
    rng = np.random.default_rng(16)
    h = 1e-6
    checked = 0
    for _ in range(12):
        v = rng.standard_normal(w.shape)
        l1, x1, c1 = _chain(sim, cfg, w + h * v, target)
        l2, x2, c2 = _chain(sim, cfg, w - h * v, target)
        if any((np.floor(a) != np.floor(b)).any() for a, b in zip(c1 + [x1], c2 + [x2])):
            continue    # a particle crossed a cell face: resample the direction
        fd = (l1 - l2) / (2 * h)
        assert _rel(fd, np.sum(wbar * v)) < 1e-6
        checked += 1
        if checked == 3:
            break
    assert checked == 3
