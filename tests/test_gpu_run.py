"""A full run on the GPU against a full oracle run from the same white noise:
matter power spectrum within 0.1 % at k < k_Nyquist / 2 after z = 99 -> 0."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_full_run_C1_power_spectrum(dev):
    from paper_2007_13394_amd import pm
    from paper_2007_13394_amd import run as R
    cfg = I.config("C1")
    n = cfg["n_mesh"]
    ctx = pm.Ctx(pm.make_config(cfg))
    w = I.white_noise(cfg["seed"], cfg["n_cdm"])
    x, p = ctx.particles()
    pm.pm_ic(ctx, torch.from_numpy(w).to(dev), x, p)
    a, half = R.schedule(cfg["a0"], cfg["n_lin"])
    R.run(ctx, x, p, a, half)
    nb = n // 2
    k, pk, nm = pm.pm_power(ctx, x, 0, ctx.nseg, nbins=nb)
    kc, pkc, _ = pm.pm_power(ctx, x, 0, 1, nbins=nb)
    s = O.make_sim(cfg)
    ox, op = O.ic(s, w)
    oa, ohalf = O.schedule(cfg["a0"], cfg["n_lin"])
    O.run(s, ox, op, oa, ohalf)
    ok, opk, onm = O.power(O.delta_of(s, ox, 0, ctx.nseg), None, cfg["box"], nb)
    okc, opkc, _ = O.power(O.delta_of(s, ox, 0, 1), None, cfg["box"], nb)
    kny = np.pi * n / cfg["box"]
    sel = (onm > 0) & (ok < kny / 2)
    em = np.abs(pk[sel] / opk[sel] - 1).max()
    ec = np.abs(pkc[sel] / opkc[sel] - 1).max()
    print("full run C1: max |P/P_oracle - 1| matter", em, "cdm", ec, flush=True)
    sys.stdout.flush()
    assert em < 1e-3 and ec < 1e-3
    assert np.all(np.isfinite(x.cpu().numpy()))
