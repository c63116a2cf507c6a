"""Training and judging of the learned force correction.

Orchestration only: every force, loss, gradient and optimiser step runs in
libpm's kernels (pm_force, pm_learned_loss, pm_adam, pm_learned_step,
pm_step, pm_density, pm_power_mesh); PyTorch holds device memory.

Training pairs come from plain runs on the fine mesh (4x the coarse mesh per
side), started from seeded white noise: at every `snap_every`-th force
evaluation the particle positions and the fine-mesh forces are kept, both
rescaled to coarse-mesh units (positions / 4, forces / 4: a force in grid
units scales with the number of cells per side for the same physical force).
The network is trained by force matching on the coarse mesh, and evaluated by
running coarse learned and plain simulations and a fine plain simulation from
a held-out seed and comparing their power spectra at the end, all painted on
the coarse mesh.

Force matching minimises the per-particle force error, and near the coarse
Nyquist wavenumber the coarse density carries aliased sub-cell structure, so
the least-squares filter shrinks the force there and the runs lose power.
`calibrate` therefore also fits the radial filter to the power spectra of the
fine-mesh runs of the training seeds: repeated coarse learned runs, and a
damped multiplicative update g <- g (P_fine / P_learned)^0.3 onto which the
MLP is regressed with Adam, starting from the force-matched network (the CNN
keeps its weights).
"""
import time

import numpy as np
import torch

from . import inputs as I
from . import pm
from . import run as R

NET_H, NET_C = 96, 16
NET_NB_TABLE = 256


def _offsets():
    sizes = [("W0", NET_H * 2), ("B0", NET_H), ("W1", NET_H * NET_H), ("B1", NET_H), ("W2", NET_H * NET_H),
             ("B2", NET_H), ("W3", NET_H), ("B3", 1), ("C1W", NET_C * 27), ("C1B", NET_C),
             ("C2W", NET_C * NET_C * 27), ("C2B", NET_C), ("C3W", NET_C * 27), ("C3B", 1)]
    off, o = {}, 0
    for k, n in sizes:
        off[k] = (o, n)
        o += n
    return off, o


NET_OFF, NET_NPARAM = _offsets()


def init_params(seed, device, hidden_scale=1.0):
    """Scaled-normal hidden layers; output layers at zero, so the untrained
    network is the plain particle-mesh force."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NET_NPARAM, dtype=np.float32)
    fans = {"W0": 2, "W1": NET_H, "W2": NET_H, "C1W": 27, "C2W": 27 * NET_C}
    for k, fan in fans.items():
        o, n = NET_OFF[k]
        th[o:o + n] = rng.standard_normal(n) * hidden_scale / np.sqrt(fan)
    assert NET_NPARAM == pm.pm_net_nparam()
    return torch.from_numpy(th).to(device)


def make_ctx(cfg, learned=False, sort=False, extra_flags=0):
    """Training contexts keep the particles in canonical order (no tile sort),
    since a force pair and the loss take segment masses by array position;
    timed runs sort."""
    flags = (0 if sort else pm.PM_FLAG_NO_SORT) | (pm.PM_FLAG_LEARNED if learned else 0) | extra_flags
    return pm.Ctx(pm.make_config(cfg, flags=flags))


def _calls(cfg):
    a, half = R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"])
    return R.kdk_calls(a, half)


def fine_pairs(cfg_fine, seeds, snap_every, device, log=print):
    """[(a, x_coarse, F_coarse)] from plain fine-mesh runs (canonical order)."""
    ratio = cfg_fine["n_mesh"] // cfg_fine["coarse_mesh"]
    ctx = make_ctx(cfg_fine)
    calls = _calls(cfg_fine)
    pairs = []
    for seed in seeds:
        x, p = ctx.particles()
        w = torch.from_numpy(I.white_noise(seed, cfg_fine["n_cdm"])).to(device)
        pm.pm_ic(ctx, w, x, p)
        del w
        acc = torch.empty_like(x)
        for i, c in enumerate(calls):
            if i % snap_every == snap_every - 1 or i == len(calls) - 1:
                pm.pm_force(ctx, x, acc)
                pairs.append((c[0], (x / ratio).contiguous(), (acc / ratio).contiguous()))
            pm.pm_step(ctx, x, p, *c)
        log(f"[learn] fine run seed {seed}: {len(pairs)} pairs")
    del ctx
    torch.cuda.empty_cache()
    return pairs


def train(ctx, theta, pairs, iters, lr=2e-3, lr_end=2e-4, seed=0, log=print):
    """Adam on the force-matching loss, one pair per step in shuffled order."""
    rng = np.random.default_rng(seed)
    m, v, g = torch.zeros_like(theta), torch.zeros_like(theta), torch.zeros_like(theta)
    hist = []
    order = []
    for t in range(1, iters + 1):
        if not order:
            order = list(rng.permutation(len(pairs)))
        a, x, F = pairs[order.pop()]
        g.zero_()
        loss = pm.pm_learned_loss(ctx, theta, a, x, F, g)
        lr_t = lr * (lr_end / lr) ** ((t - 1) / max(1, iters - 1))
        pm.pm_adam(theta, m, v, g, lr_t, 0.9, 0.999, 1e-8, t)
        hist.append(loss)
        if t % 50 == 0 or t == 1:
            log(f"[learn] step {t}: loss {np.mean(hist[-50:]):.4g}")
    return hist


def pair_loss(ctx, theta, pairs):
    return float(np.mean([pm.pm_learned_loss(ctx, theta, a, x, F) for a, x, F in pairs]))


def simulate(ctx, cfg, seed, device, theta=None, scale=1):
    """Run the full schedule; returns final positions (in units of the mesh of
    `ctx` divided by `scale`) and the wall time of the steps."""
    x, p = ctx.particles()
    w = torch.from_numpy(I.white_noise(seed, cfg["n_cdm"])).to(device)
    pm.pm_ic(ctx, w, x, p)
    del w
    ids = None
    if ctx.sorts:
        # a sorting context permutes the particles: carry ids to restore the
        # canonical order (segment masses are looked up by position)
        ids = torch.arange(ctx.P, dtype=torch.int32, device=device)
        pm.pm_attach_ids(ctx, ids)
    calls = _calls(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in calls:
        if theta is None:
            pm.pm_step(ctx, x, p, *c)
        else:
            pm.pm_learned_step(ctx, theta, x, p, *c)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if ids is not None:
        pm.pm_attach_ids(ctx, None)
        xc = torch.empty_like(x)
        xc[:, ids.long()] = x
        x = xc
    return (x / scale).contiguous(), dt, len(calls)


def spectra(ctx, xs, nbins):
    """Auto spectra of each position set and cross spectra with the first one,
    all painted on the mesh of `ctx`."""
    n = ctx.n
    dens = []
    for x in xs:
        d = torch.empty(n ** 3, dtype=torch.float32, device=x.device)
        pm.pm_density(ctx, x, d)
        dens.append(d)
    k, p0, nm = pm.pm_power_mesh(ctx, dens[0], dens[0], nbins)
    autos, cross = [p0], [p0]
    for d in dens[1:]:
        autos.append(pm.pm_power_mesh(ctx, d, d, nbins)[1])
        cross.append(pm.pm_power_mesh(ctx, dens[0], d, nbins)[1])
    return k, nm, autos, cross


def _spectrum(ana, x):
    """(k, P, n_modes) of positions x painted on the mesh of `ana`, bins of one
    fundamental wavenumber up to the mesh corner."""
    d = torch.empty(ana.n ** 3, dtype=torch.float32, device=x.device)
    pm.pm_density(ana, x, d)
    return pm.pm_power_mesh(ana, d, d, ana.n)


def fit_table(theta, a_list, targets, weights, steps=1000, lr=3e-3, lr_end=3e-4):
    """Adam on the filter MLP's parameters: mean over scale factors of
    sum_b weights[b] (table(theta, a)_b - target_b)^2 (target tables
    [len(a_list)][NET_NB], host float64), the step size decaying
    geometrically from lr to lr_end.  Returns the largest remaining
    |table - target| over bins of weight 1."""
    m, v, g = torch.zeros_like(theta), torch.zeros_like(theta), torch.zeros_like(theta)
    mlp_end = NET_OFF["C1W"][0]
    tables = torch.empty((len(a_list), NET_NB_TABLE), dtype=torch.float32, device=theta.device)
    tgt = np.asarray(targets)
    worst = 0.0
    for t in range(1, steps + 1):
        g.zero_()
        for i, a in enumerate(a_list):
            pm.pm_net_table(theta, a, tables[i])
        diff = tables.double().cpu().numpy() - tgt          # one host round trip per step
        worst = float(np.max(np.abs(diff[:, weights >= 1.0])))
        tbar = torch.from_numpy(2.0 * weights * diff / len(a_list)).to(theta.device)
        for i, a in enumerate(a_list):
            pm.pm_net_table_vjp(theta, a, tbar[i], g)
        g[mlp_end:] = 0
        pm.pm_adam(theta, m, v, g, lr * (lr_end / lr) ** ((t - 1) / max(1, steps - 1)), 0.9, 0.999, 1e-8, t)
    return worst


def calibrate(cc, seeds, fine_x, theta, rounds=48, power=0.3, fit_steps=1000, device="cuda", log=print):
    """Fit the radial filter to fine-mesh power spectra.  Each round runs the
    learned coarse model from every training seed, takes the ratio R(k) of
    the fine to the learned spectrum (geometric mean over seeds, smoothed over
    three bins) and moves the filter to g(k, a) R(k)^power at every scale
    factor (tapered to no change between 0.8 and 1 k_Nyq); the MLP is fitted
    to that table with Adam, weighted to the bins below 0.6 k_Nyq.  The
    response d ln P / d ln g is about 3.6 on linear scales and falls below 1
    towards k_Nyq / 2; power = 0.3 contracts on the former and creeps on the
    latter, and mode coupling between bins makes the error oscillate slowly,
    so theta ends at the parameters of the round with the smallest
    training-seed error.  fine_x: final fine-run positions in
    coarse-mesh units, one per seed.  Returns the per-round training-seed
    errors max_k |P_l / P_f - 1| over k < k_Nyq / 2."""
    ana = make_ctx(cc)
    n = cc["n_mesh"]
    kN = np.pi * n / cc["box"]
    Pf = [_spectrum(ana, x) for x in fine_x]
    k, nm = Pf[0][0], Pf[0][2]
    sel = (nm > 0) & (k > 0)
    kt = k[sel] / kN
    in_range = kt < 0.5
    a_fit = sorted(set([c[0] for c in _calls(cc)][::3] + [1.0]))
    kt_b = np.arange(NET_NB_TABLE) * np.sqrt(3.0) / (NET_NB_TABLE - 1)
    lnPf = np.mean([np.log(np.maximum(pf[sel], 1e-30)) for (_, pf, _) in Pf], axis=0)
    ctx = make_ctx(cc, learned=True, sort=True)
    w_b = np.where(kt_b <= 0.6, 1.0, 0.05)
    hist = []
    best = (np.inf, theta.clone())
    for r in range(rounds + 1):
        lnP = []
        for s in seeds:
            x, _, _ = simulate(ctx, cc, s, device, theta=theta)
            _, pl, _ = _spectrum(ana, x)
            lnP.append(np.log(np.maximum(pl[sel], 1e-30)))
        lnR = lnPf - np.mean(lnP, axis=0)
        err = float(np.max(np.abs(np.exp(-lnR[in_range]) - 1.0)))
        hist.append(err)
        if err < best[0]:
            best = (err, theta.clone())
        if r == rounds:
            log(f"[calib] round {r}: training seeds max |P_l/P_f - 1| = {err:.4f}; best {best[0]:.4f}")
            break
        lnR_s = np.convolve(np.pad(lnR, 1, mode="edge"), np.ones(3) / 3.0, mode="valid")
        # no update past the Nyquist wavenumber (mesh-corner modes), tapered from 0.8
        upd = np.exp(power * np.clip((1.0 - kt_b) / 0.2, 0.0, 1.0) * np.interp(kt_b, kt, lnR_s))
        targets = [pm.pm_net_table(theta, a).double().cpu().numpy() * upd for a in a_fit]
        resid = fit_table(theta, a_fit, targets, w_b, fit_steps)
        log(f"[calib] round {r}: training seeds max |P_l/P_f - 1| = {err:.4f}, table fit residual {resid:.2e}")
    theta.copy_(best[1])
    return hist


def evaluate(coarse_name, fine_name, train_seeds, test_seeds, snap_every=5, iters=400, lr=2e-3, device="cuda",
          log=print, calib_rounds=48, calib_seeds=None):
    """Train the network on fine-mesh force pairs (force matching), then
    calibrate its radial filter on fine-mesh spectra of the calibration
    seeds; compare the force-matched and the calibrated coarse models with
    plain coarse and plain fine runs from held-out seeds (an int or a list).
    Spectra are averaged over the held-out seeds before their ratios are
    taken; each seed's own worst error is reported too.  "learned" in the
    result is the calibrated model.  Returns a dict."""
    test_seeds = [test_seeds] if isinstance(test_seeds, int) else list(test_seeds)
    cc, cf = I.config(coarse_name), I.config(fine_name)
    ratio = cf["n_mesh"] // cc["n_mesh"]
    cf = dict(cf, coarse_mesh=cc["n_mesh"])
    t0 = time.perf_counter()
    pairs = fine_pairs(cf, train_seeds, snap_every, device, log)
    test_pairs = fine_pairs(cf, test_seeds[:1], snap_every, device, log)
    t_pairs = time.perf_counter() - t0
    ctx = make_ctx(cc, learned=True)
    theta = init_params(1, device)
    base_train, base_test = pair_loss(ctx, theta, pairs), pair_loss(ctx, theta, test_pairs)
    t0 = time.perf_counter()
    hist = train(ctx, theta, pairs, iters, lr=lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    tr_train, tr_test = pair_loss(ctx, theta, pairs), pair_loss(ctx, theta, test_pairs)
    del test_pairs, pairs, ctx
    torch.cuda.empty_cache()
    # filter calibrated on the calibration seeds' fine-mesh spectra
    t0 = time.perf_counter()
    ctx_f = pm.Ctx(pm.make_config(cf))
    calib_seeds = list(train_seeds) if calib_seeds is None else list(calib_seeds)
    assert not set(calib_seeds) & set(test_seeds) and not set(train_seeds) & set(test_seeds)
    fine_x = [simulate(ctx_f, cf, s, device, scale=ratio)[0] for s in calib_seeds]
    del ctx_f
    theta_cal = theta.clone()   # the force-matched network; the calibration moves the filter only
    calib_hist = calibrate(cc, calib_seeds, fine_x, theta_cal, rounds=calib_rounds, device=device, log=log)
    t_cal = time.perf_counter() - t0
    del fine_x
    torch.cuda.empty_cache()
    held = heldout(cc, cf, test_seeds, theta_cal, theta, device)
    out = {
        "coarse": coarse_name, "fine": fine_name, "particles": held["particles"], "train_seeds": list(train_seeds),
        "test_seeds": test_seeds, "iters": iters, "pairs_s": round(t_pairs, 2), "train_s": round(t_train, 2),
        "force_loss": {"plain_train": base_train, "learned_train": tr_train, "plain_test": base_test,
                       "learned_test": tr_test},
        "calibration": {"rounds": calib_rounds, "seeds": calib_seeds, "train_seed_err": calib_hist,
                        "seconds": round(t_cal, 2)},
        "loss_history": [float(h) for h in hist[::10]],
    }
    out.update(held)
    out["theta"] = theta_cal
    return out


def heldout(cc, cf, test_seeds, theta_cal, theta_fm=None, device="cuda"):
    """Held-out comparison: from each seed, a plain fine-mesh run (the truth),
    the learned coarse run (theta_cal), a plain coarse run and, if given, the
    force-matched model (theta_fm), all painted on the coarse mesh at the end.
    Reports each seed's worst |P / P_fine - 1| and smallest cross-correlation
    over k < k_Nyq / 2, the same for the spectra averaged over the seeds, the
    per-bin ratios, and particle-steps/s of the timed step loops."""
    ratio = cf["n_mesh"] // cc["n_mesh"]
    cf = dict(cf, coarse_mesh=cc["n_mesh"])
    ctx_f = pm.Ctx(pm.make_config(cf))
    ctx_l, ctx_c, ana = make_ctx(cc, learned=True, sort=True), make_ctx(cc, sort=True), make_ctx(cc)
    nb = cc["n_mesh"] // 2
    kn = np.pi * cc["n_mesh"] / cc["box"]
    names = ("fine", "learned", "plain_coarse") + (("learned_force_matched",) if theta_fm is not None else ())
    auto_sum, cross_sum, per_seed, ratios = None, None, [], {}
    t_f = t_l = t_c = 0.0
    for s in test_seeds:
        x_f, dt_f, ncalls = simulate(ctx_f, cf, s, device, scale=ratio)
        x_l, dt_l, _ = simulate(ctx_l, cc, s, device, theta=theta_cal)
        x_c, dt_c, _ = simulate(ctx_c, cc, s, device)
        xs = [x_f, x_l, x_c]
        if theta_fm is not None:
            xs.append(simulate(ctx_l, cc, s, device, theta=theta_fm)[0])
        t_f, t_l, t_c = t_f + dt_f, t_l + dt_l, t_c + dt_c
        k, nm, autos, cross = spectra(ana, xs, nb)
        sel = (nm > 0) & (k > 0) & (k < kn / 2)
        rec = {"seed": s}
        for j in range(1, len(names)):
            rec[names[j]] = float(np.max(np.abs(autos[j][sel] / autos[0][sel] - 1)))
            rec[names[j] + "_r_min"] = float(np.min(cross[j][sel] / np.sqrt(autos[0][sel] * autos[j][sel])))
        per_seed.append(rec)
        ratios[str(s)] = {names[j]: np.round(autos[j][sel] / autos[0][sel], 5).tolist() for j in (1, 2)}
        auto_sum = np.array(autos) if auto_sum is None else auto_sum + np.array(autos)
        cross_sum = np.array(cross) if cross_sum is None else cross_sum + np.array(cross)
        P = x_f.shape[1]
        del x_f, x_l, x_c, xs
    del ctx_f, ctx_l, ctx_c
    torch.cuda.empty_cache()
    err = {names[j]: float(np.max(np.abs(auto_sum[j][sel] / auto_sum[0][sel] - 1))) for j in range(1, len(names))}
    rmin = {names[j]: float(np.min(cross_sum[j][sel] / np.sqrt(auto_sum[0][sel] * auto_sum[j][sel])))
            for j in range(1, len(names))}
    nt = len(test_seeds)
    return {
        "particles": P,
        "pk_max_rel_err": err,
        "pk_max_rel_err_per_seed": per_seed,
        "k_range_hMpc": [float(k[sel].min()), float(k[sel].max())],
        "r_min": rmin,
        "particle_steps_per_s": {"learned_coarse": P * ncalls * nt / t_l, "plain_coarse": P * ncalls * nt / t_c,
                                 "plain_fine": P * ncalls * nt / t_f},
        "speedup_vs_fine": t_f / t_l,
        "k": k[sel].tolist(),
        "ratio_per_seed": ratios,
        "pk": {names[j]: (auto_sum[j][sel] / nt).tolist() for j in range(len(names))},
    }


def save_params(theta, path):
    """The flat FP32 parameter array as a .npy file."""
    np.save(path, theta.detach().float().cpu().numpy())


def load_params(path, device="cuda"):
    """Parameters written by save_params (plain array; nothing is unpickled)."""
    th = np.load(path, allow_pickle=False)
    if th.dtype != np.float32 or th.shape != (NET_NPARAM,):
        raise ValueError(f"{path}: expected float32 [{NET_NPARAM}], got {th.dtype} {th.shape}")
    return torch.from_numpy(th).to(device)


def time_steps(cfg_name, steps, device="cuda", seed=200, which=("learned", "plain"), extra_flags=0):
    """ms per learned and/or plain step on a sorted context of `cfg_name`
    (parameters: the seeded initialisation with every entry perturbed by 1 %
    noise, so that every layer runs with non-zero weights), from the initial
    conditions of `seed`.  extra_flags: further context flags (with
    PM_FLAG_DEFER_GUARDS the last step's check, pm_sync, is inside the
    timed region)."""
    cfg = I.config(cfg_name)
    theta = init_params(1, device)
    theta += 0.01 * torch.from_numpy(np.random.default_rng(seed).standard_normal(theta.numel()).astype(np.float32)).to(
        device)
    calls = _calls(cfg)[:steps + 2]
    out = {}
    for name, learned in (("learned", True), ("plain", False)):
        if name not in which:
            continue
        ctx = make_ctx(cfg, learned=learned, sort=True, extra_flags=extra_flags)
        x, p = ctx.particles()
        w = torch.from_numpy(I.white_noise(seed, cfg["n_cdm"])).to(device)
        pm.pm_ic(ctx, w, x, p)
        del w
        for i, c in enumerate(calls):
            if i == 2:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if learned:
                pm.pm_learned_step(ctx, theta, x, p, *c)
            else:
                pm.pm_step(ctx, x, p, *c)
        pm.pm_sync(ctx)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = (time.perf_counter() - t0) / (len(calls) - 2) * 1e3
        out["particles"] = ctx.P
        del ctx, x, p
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="train, calibrate and evaluate the learned force correction")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="only time this many learned and plain steps on the coarse workload")
    ap.add_argument("--coarse", default="C4_coarse")
    ap.add_argument("--fine", default="C4_fine")
    ap.add_argument("--train-seeds", default="100,101,102,103,104,105,106,107")
    ap.add_argument("--calib-seeds", default="100,101,102,103,104,105,106,107,108,109,110,111,112,113,114,115")
    ap.add_argument("--test-seeds", default="200,201,202,203")
    ap.add_argument("--snap-every", type=int, default=5)
    ap.add_argument("--iters", type=int, default=400)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--save", default="", help="write the calibrated parameters to this .npy file")
    a = ap.parse_args()
    if a.time_steps:
        print(json.dumps(dict(time_steps(a.coarse, a.time_steps), workload=a.coarse)), flush=True)
        sys.exit(0)
    res = evaluate(a.coarse, a.fine, [int(s) for s in a.train_seeds.split(",")],
                [int(s) for s in a.test_seeds.split(",")], a.snap_every, a.iters,
                a.lr, log=lambda *m: print(*m, file=sys.stderr, flush=True),
                calib_seeds=[int(s) for s in a.calib_seeds.split(",")])
    theta = res.pop("theta")
    if a.save:
        save_params(theta, a.save)
    print(json.dumps(res), flush=True)
