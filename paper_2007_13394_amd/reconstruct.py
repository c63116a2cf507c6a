"""Reconstruction of initial modes from a final density: gradient descent on
the white noise through the hand-written reverse mode (the use the paper's
introduction gives for a differentiable forward model).

Orchestration only: the forward model is pm_ic -> pm_step calls ->
pm_density and the gradient pm_density_vjp -> pm_step_vjp -> pm_ic_vjp
(through paper_2007_13394_amd.diff); the update is pm_adam.  PyTorch
evaluates the loss L = sum (S delta - S delta_target)^2 / sum (S delta_target)^2,
S an average over blocks of pool^3 cells (a low-pass that keeps the loss off
the scales a few-step run cannot match), and its derivative with respect to
delta.  The correlation of the estimate with
the true modes is computed on the host.
"""
import time

import numpy as np
import torch

from . import diff
from . import inputs as I
from . import pm
from . import run as R


def _corr(a, b):
    a, b = a.ravel().astype(np.float64), b.ravel().astype(np.float64)
    return float(np.dot(a, b) / np.sqrt(np.dot(a, a) * np.dot(b, b)))


def _corr_smoothed(a, b, kmax_frac):
    """Correlation of the two fields keeping modes |k| < kmax_frac k_Nyq."""
    n = a.shape[0]
    fa, fb = np.fft.rfftn(a), np.fft.rfftn(b)
    k0 = np.fft.fftfreq(n) * 2
    k2 = np.fft.rfftfreq(n) * 2
    kk = np.sqrt(k0[:, None, None] ** 2 + k0[None, :, None] ** 2 + k2[None, None, :] ** 2)
    keep = kk < kmax_frac
    num = np.sum((fa * np.conj(fb)).real[keep])
    return float(num / np.sqrt(np.sum(np.abs(fa[keep]) ** 2) * np.sum(np.abs(fb[keep]) ** 2)))


def _pool(d, pool):
    if pool <= 1:
        return d
    return torch.nn.functional.avg_pool3d(d[None, None], pool)[0, 0]


def reconstruct(cfg_name="C5", target_seed=301, iters=100, lr=0.01, pool=4, device="cuda", log=print):
    """Start from zero modes and descend on the density loss against the run of
    `target_seed`.  Returns the loss history, correlations with the true modes
    and the mean forward / backward times per iteration."""
    cfg = I.config(cfg_name)
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    calls = [tuple(c) for c in R.kdk_calls(*R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"]))]
    nc = cfg["n_cdm"]
    w_true = torch.from_numpy(I.white_noise(target_seed, nc)).to(device)
    with torch.no_grad():
        target = _pool(diff.final_density(ctx, w_true, calls), pool).clone()
    norm = float((target.double() ** 2).sum())
    w = torch.zeros_like(w_true)
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    hist, t_fwd, t_bwd = [], [], []
    for it in range(1, iters + 1):
        wl = w.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        delta = _pool(diff.final_density(ctx, wl, calls), pool)
        loss = ((delta - target) ** 2).sum() / norm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pm.pm_adam(w, m, v, wl.grad.contiguous(), lr, 0.9, 0.999, 1e-8, it)
        hist.append(float(loss.detach()))
        t_fwd.append(t1 - t0)
        t_bwd.append(t2 - t1)
        if it == 1 or it % 10 == 0:
            log(f"[reconstruct] iteration {it}: loss {hist[-1]:.4f}")
    wt, we = w_true.cpu().numpy(), w.cpu().numpy()
    out = {"config": cfg_name, "particles": ctx.P, "mesh": cfg["n_mesh"], "calls": len(calls), "iters": iters,
           "lr": lr, "pool": pool,
           "loss": hist, "corr_modes": _corr(we, wt), "corr_modes_k_below_quarter_nyquist": _corr_smoothed(we, wt, 0.25),
           "forward_ms": 1e3 * float(np.median(t_fwd[1:] or t_fwd)),
           "backward_ms": 1e3 * float(np.median(t_bwd[1:] or t_bwd))}
    del ctx
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="reconstruct the initial modes of a seeded run from its final density")
    ap.add_argument("--config", default="C5")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration under rocprofv3 --pmc)")
    a = ap.parse_args()
    if a.copy_calibration:
        pm.copy_calibration()
    res = reconstruct(cfg_name=a.config, iters=a.iters, log=lambda *m: print(*m, file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)
