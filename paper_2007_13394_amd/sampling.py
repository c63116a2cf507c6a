"""Quasi-random against pseudo-random neutrino sampling (the paper's
neutrino power-spectrum comparison, Sec. 3).

Orchestration only: initial conditions, steps and spectra run in libpm
(pm_ic / pm_ic_pseudo, pm_step, pm_power).  Two runs share the CDM lattice,
the mesh, the step schedule and the white noise:
  * quasi-random: N_sites^(1/3) sites, N_shell shells x (2 N_fib + 1)
    Fibonacci directions per site;
  * pseudo-random: one neutrino per site on a finer site grid, each with a
    random speed from the Fermi-Dirac number distribution and a random
    direction (uniforms drawn on the device from a seeded generator),
with close to the same number of neutrino particles.  At the schedule points
nearest to the requested redshifts the neutrino auto power (cloud-in-cell
window divided out) is measured for both.
"""
import time

import numpy as np
import torch

from . import inputs as I
from . import pm
from . import run as R


def _run(cfg, pseudo, z_out, device, nbins):
    flags = pm.PM_FLAG_NU_PSEUDO if pseudo else 0
    ctx = pm.Ctx(pm.make_config(cfg, flags=flags))
    gen = torch.Generator(device=device)
    gen.manual_seed(cfg["seed"])
    nc = cfg["n_cdm"]
    white = torch.randn((nc, nc, nc), generator=gen, device=device, dtype=torch.float32)
    x, p = ctx.particles()
    if pseudo:
        ugen = torch.Generator(device=device)
        ugen.manual_seed(cfg["seed"] + 1)
        u = torch.rand((3, cfg["n_sites"] ** 3), generator=ugen, device=device, dtype=torch.float32)
        pm.pm_ic_pseudo(ctx, white, u, x, p)
        del u
    else:
        pm.pm_ic(ctx, white, x, p)
    del white
    a, half = R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"])
    calls = R.kdk_calls(a, half)
    # after call i the positions are at a[i + 1] (the last call ends at a = 1)
    a_after = [c[3] for c in calls]
    want = {}
    for z in z_out:
        i = int(np.argmin([abs(1.0 / aa - 1.0 - z) for aa in a_after]))
        want.setdefault(i, []).append(z)
    out = {}
    t0 = time.perf_counter()
    for i, c in enumerate(calls):
        pm.pm_step(ctx, x, p, *c)
        if i in want:
            k, pnu, nm = pm.pm_power(ctx, x, 1, ctx.nseg, 1, ctx.nseg, nbins=nbins, compensate=1)
            _, pcdm, _ = pm.pm_power(ctx, x, 0, 1, 0, 1, nbins=nbins, compensate=1)
            for z in want[i]:
                out[z] = {"a": a_after[i], "z_actual": 1.0 / a_after[i] - 1.0, "k": k, "p_nu": pnu, "p_cdm": pcdm,
                          "n_modes": nm}
    torch.cuda.synchronize()
    n_nu = ctx.P - nc ** 3
    res = {"particles": ctx.P, "n_nu": n_nu, "seconds": time.perf_counter() - t0, "spectra": out}
    del ctx, x, p
    torch.cuda.empty_cache()
    return res


def _grid_excess(k, pk, nm, kn, width=3):
    """P in the bin holding kn over the median of the `width` bins on each side."""
    b = int(np.argmin(np.abs(k - kn)))
    side = [j for j in range(b - width, b + width + 1) if j != b and 0 <= j < len(k) and nm[j] > 0]
    return float(pk[b] / np.median(pk[side]))


def compare(qr_name="E7_qr", pr_name="E7_pr", z_out=(2.0, 1.0, 0.0), device="cuda"):
    cq, cp = I.config(qr_name), I.config(pr_name)
    n = cq["n_mesh"]
    nbins = n // 2
    rq = _run(cq, False, z_out, device, nbins)
    rp = _run(cp, True, z_out, device, nbins)
    box = cq["box"]
    kf = 2 * np.pi / box
    kn = kf * cq["n_sites"]
    shot_pr = box ** 3 / rp["n_nu"]
    rows = []
    for z in z_out:
        sq, sp = rq["spectra"][z], rp["spectra"][z]
        k, nm = sq["k"], sq["n_modes"]
        ok = nm > 0
        hi = ok & (k > 0.75 * kf * n / 2) & (k < kf * n / 2)         # top quarter below the mesh Nyquist
        mid = ok & (k > 0.08) & (k < 0.12)
        rows.append({
            "z": z, "z_actual_qr": sq["z_actual"], "z_actual_pr": sp["z_actual"],
            "p_nu_high_k_qr": float(np.mean(sq["p_nu"][hi])), "p_nu_high_k_pr": float(np.mean(sp["p_nu"][hi])),
            "shot_noise_pr": shot_pr,
            "pr_over_qr_0.08_0.12": float(np.mean(sp["p_nu"][mid] / sq["p_nu"][mid])),
            "pr_over_qr_scatter_0.08_0.12": float(np.std(sp["p_nu"][mid] / sq["p_nu"][mid])),
            "grid_excess_qr": {m: _grid_excess(k, sq["p_nu"], nm, f * kn) for m, f in
                               (("k_n", 1.0), ("sqrt2_k_n", 2 ** 0.5), ("sqrt3_k_n", 3 ** 0.5), ("2_k_n", 2.0))
                               if f * kn < kf * n / 2},
            "grid_excess_pr": {m: _grid_excess(k, sp["p_nu"], nm, f * kn) for m, f in
                               (("k_n", 1.0), ("sqrt2_k_n", 2 ** 0.5), ("sqrt3_k_n", 3 ** 0.5), ("2_k_n", 2.0))
                               if f * kn < kf * n / 2},
        })
    return {"quasi_random": {"config": qr_name, "n_nu": rq["n_nu"], "seconds": rq["seconds"]},
            "pseudo_random": {"config": pr_name, "n_nu": rp["n_nu"], "seconds": rp["seconds"]},
            "n_nu_ratio_qr_over_pr": rq["n_nu"] / rp["n_nu"], "k_n_hMpc": kn, "rows": rows,
            "spectra": {str(z): {"k": rq["spectra"][z]["k"].tolist(), "p_nu_qr": rq["spectra"][z]["p_nu"].tolist(),
                                 "p_nu_pr": rp["spectra"][z]["p_nu"].tolist(),
                                 "p_cdm_qr": rq["spectra"][z]["p_cdm"].tolist()} for z in z_out}}


if __name__ == "__main__":
    import json
    import sys
    res = compare()
    brief = {k: v for k, v in res.items() if k != "spectra"}
    print(json.dumps(brief), flush=True)
    if len(sys.argv) > 1:
        with open(sys.argv[1], "w") as f:
            json.dump(res, f)
