"""GPU pseudo-random neutrino initial conditions (pm_ic_pseudo through the C
ABI) against the FP64 oracle on the same white noise and uniforms.  Positions
within float32 ulps as for the quasi-random path; momenta by relative L2: the
GPU inverts the cumulative speed distribution from a 4097-point table
(search plus linear interpolation), the oracle by bisection on the integral.
The two initial-condition entry points refuse each other's contexts."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _setup(dev):
    from paper_2007_13394_amd import pm
    cfg = I.config("C1p")
    return pm, cfg, pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NU_PSEUDO))


def test_pseudo_ic_vs_oracle(dev):
    pm, cfg, ctx = _setup(dev)
    n, nc, ns = cfg["n_mesh"], cfg["n_cdm"] ** 3, cfg["n_sites"] ** 3
    assert ctx.P == nc + ns
    w = I.white_noise(cfg["seed"], cfg["n_cdm"])
    u = np.random.default_rng(12).random((3, ns)).astype(np.float32)
    x, p = ctx.particles()
    pm.pm_ic_pseudo(ctx, torch.from_numpy(w).to(dev), torch.from_numpy(u).to(dev), x, p)
    ox, op = O.ic_pseudo(O.make_sim(cfg), w, u.astype(np.float64))
    gx, gp = x.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    ulp = np.spacing(np.float32(n))
    dx = np.abs(gx - ox.astype(np.float32).astype(np.float64))
    dx = np.minimum(dx, n - dx)
    e_c, e_n = rel_l2(gp[:, :nc], op[:, :nc]), rel_l2(gp[:, nc:], op[:, nc:])
    say("pseudo ic: momentum rel L2 CDM", e_c, "neutrinos", e_n, "max |dx| / ulp", dx.max() / ulp)
    assert e_c < 1e-5 and e_n < 1e-4
    assert dx[:, :nc].max() <= ulp and dx[:, nc:].max() <= 2 * ulp
    assert np.all((gx >= 0) & (gx < n))
    # the speeds span the distribution (thermal motion dominates at z = 99)
    sp = np.linalg.norm(gp[:, nc:], axis=0)
    assert np.std(sp) > 0.2 * np.mean(sp)


def test_entry_points_refuse_the_other_sampling(dev):
    pm, cfg, ctx = _setup(dev)
    w = torch.from_numpy(I.white_noise(1, cfg["n_cdm"])).to(dev)
    x, p = ctx.particles()
    with pytest.raises(pm.PMError) as e:
        pm.pm_ic(ctx, w, x, p)
    assert e.value.status == -6
    cq = pm.Ctx(pm.make_config(I.config("C1")))
    xq, pq = cq.particles()
    u = torch.rand((3, I.config("C1")["n_sites"] ** 3), device=dev)
    with pytest.raises(pm.PMError) as e:
        pm.pm_ic_pseudo(cq, torch.from_numpy(I.white_noise(1, 32)).to(dev), u, xq, pq)
    assert e.value.status == -6


def test_pseudo_run_steps(dev):
    """A full tile-sorted run from pseudo-random initial conditions keeps the
    state finite and in the box."""
    pm, cfg, ctx = _setup(dev)
    from paper_2007_13394_amd import run as R
    ns = cfg["n_sites"] ** 3
    w = torch.from_numpy(I.white_noise(cfg["seed"], cfg["n_cdm"])).to(dev)
    u = torch.from_numpy(np.random.default_rng(13).random((3, ns)).astype(np.float32)).to(dev)
    x, p = ctx.particles()
    pm.pm_ic_pseudo(ctx, w, u, x, p)
    a, half = R.schedule(cfg["a0"], cfg["n_lin"])
    for c in R.kdk_calls(a, half):
        pm.pm_step(ctx, x, p, *c)
    n = cfg["n_mesh"]
    assert bool(torch.isfinite(x).all()) and bool(torch.isfinite(p).all())
    assert bool(((x >= 0) & (x < n)).all())
    k, pnu, nm = pm.pm_power(ctx, x, 1, ctx.nseg, 1, ctx.nseg, nbins=n // 2)
    say("P_nu at the lowest and highest bins", pnu[1:3], pnu[-2:])
    assert np.all(np.isfinite(pnu)) and np.all(pnu[nm > 0] > 0)


def test_sampling_comparison_small(dev):
    """The quasi- vs pseudo-random comparison on a small instance (8^3 sites x
    510 against 64^3 x 1 neutrinos, ratio 0.996): the pseudo-random spectrum
    sits near its shot-noise level V / N at high k, the quasi-random one lies
    below it between the largest scales and the grid wavenumber, and only the
    quasi-random run shows an excess at the grid wavenumber at z = 2."""
    from paper_2007_13394_amd import sampling
    import numpy as np
    res = sampling.compare("E7s_qr", "E7s_pr", z_out=(2.0, 0.0))
    assert abs(res["n_nu_ratio_qr_over_pr"] - 0.99609375) < 1e-12
    kn = res["k_n_hMpc"]
    for row in res["rows"]:
        say("z", row["z"], "high-k QR", row["p_nu_high_k_qr"], "PR", row["p_nu_high_k_pr"], "shot", row["shot_noise_pr"],
            "grid excess QR", row["grid_excess_qr"].get("k_n"), "PR", row["grid_excess_pr"].get("k_n"))
        assert 0.7 < row["p_nu_high_k_pr"] / row["shot_noise_pr"] < 1.6
    s = res["spectra"]["2.0"]
    k, q, p = (np.array(s[x]) for x in ("k", "p_nu_qr", "p_nu_pr"))
    m = (k > 0.3 * kn) & (k < 0.8 * kn) & (q > 0)
    assert np.median(q[m]) < np.median(p[m])
    assert res["rows"][0]["grid_excess_qr"]["k_n"] > 2.0 > res["rows"][0]["grid_excess_pr"]["k_n"]
