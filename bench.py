#!/usr/bin/env python
"""Benchmark of the FastPM-with-neutrinos particle-mesh step on one MI355X.

A step is one pm_step call of a kick-drift-kick run: paint of all CDM and
neutrino particles, forward FFT, gradient of the inverse Laplacian, three
inverse FFTs, readout, kick and drift.  The workload is the paper-scale
configuration: 1024^3 CDM + 128^3 x 70 neutrino particles on a 2048^3 mesh in
a 1024 Mpc/h box, M_nu = 0.06 eV normal hierarchy as one effective species,
z = 99 -> 0 in 5 log + 20 linear steps, Zel'dovich initial conditions from
seeded white noise generated on the GPU.  The default run warms up with the
first call of the schedule and times the remaining 25 calls.

Prints one JSON line (rank 0) with particle-steps/s, the roofline position of
the dominant kernel (durations from HIP events recorded around every launch
on the launch stream during the timed region) and, unless --no-cpu-baseline,
the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import re
import os
import sys
import time

METRIC = "particle-steps/s at 1024^3 CDM; learned vs plain PM at equal 1% P(k) error"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# on this workload, each scaled by what the counter reads for a plain device
# copy of known size (profiles/ has the summaries and the commands).  A figure
# is reported only while the kernel's source file and the layout lines of the
# header (tile sizes, row and plane strides) still hash as they did when the
# counters were taken.
LAYOUT_HEADER = "paper_2007_13394_amd/csrc/pm_internal.h"
# the lines of the layout header that place data in HBM: tile sizes, row and
# plane paddings and strides, the momentum record
_LAYOUT_RE = re.compile(r"^(constexpr int(64_t)? (TILE_W|TILE|half_cols|half_pad|force_plane)\b|"
                        r"#define PM_(ROW_PAD|PAD_FROM|PLANE_PAD)\b|struct Mom3|    float x, y, z;)")


def layout_lines(root):
    with open(os.path.join(root, LAYOUT_HEADER)) as f:
        return "".join(l for l in f if _LAYOUT_RE.match(l)).encode()


MEASURED_TRAFFIC = {
    # profiles/c3_step_hbm_counters.md (averages over the profiled launches;
    # the scatter's include the first sort from canonical order)
    "c2r_x0": {"bytes_per_launch": 69351596441, "source": "paper_2007_13394_amd/csrc/fft.hip",
               "sha256_16": "4ee3c29a55226413"},
    "cols_inv": {"bytes_per_launch": 70472608091, "source": "paper_2007_13394_amd/csrc/fft.hip",
                 "sha256_16": "4ee3c29a55226413"},
    "cols_fwd": {"bytes_per_launch": 70586034592, "source": "paper_2007_13394_amd/csrc/fft.hip",
                 "sha256_16": "4ee3c29a55226413"},
    "x0_green": {"bytes_per_launch": 103884468952, "source": "paper_2007_13394_amd/csrc/fft.hip",
                 "sha256_16": "4ee3c29a55226413"},
    "r2c_x0": {"bytes_per_launch": 69053273764, "source": "paper_2007_13394_amd/csrc/fft.hip",
               "sha256_16": "4ee3c29a55226413"},
    "readout_kick_drift": {"bytes_per_launch": 191412978182, "source": "paper_2007_13394_amd/csrc/particles.hip",
                           "sha256_16": "4b421d94095c9950"},
    "paint": {"bytes_per_launch": 54963058920, "source": "paper_2007_13394_amd/csrc/paint.hip",
              "sha256_16": "7bb63e5c5ffc2155"},
    "sort_scatter": {"bytes_per_launch": 77764017512, "source": "paper_2007_13394_amd/csrc/sort.hip",
                     "sha256_16": "2dfc1c338c0bebb6"},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch of `kernel`, or None when no counter
    figure exists or its source changed since the counters were taken."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(root, rec["source"]), "rb") as f:
        data = f.read()
    if hashlib.sha256(data + layout_lines(root)).hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["bytes_per_launch"]


def model_bytes(P, n):
    """Algorithmic HBM bytes per launch of each kernel kind as implemented
    (one read and one write of what the kernel must move), the paint's per
    step, and the step's model-A bytes 60 P + 40 M + 128 Mc (fused minimum
    passes with an int64 mesh written and read once), against which the step
    is placed on the roofline."""
    M = n ** 3
    Mc = n * n * (n // 2 + 1)
    per_launch = {
        "r2c_rows": 8 * M + 8 * Mc,       # int64 density in, half spectrum out
        "cols_fwd": 16 * Mc,
        "axis0": 8 * Mc + 24 * Mc,        # spectrum in, three force spectra out
        "r2c_x0": 4 * M + 8 * Mc,         # float32 density contrast in, half spectrum out (16-point pass fused)
        "x0_green": 8 * Mc + 16 * Mc,     # spectrum in, k0 T and T out (k1, k2 applied by the column passes)
        "c2r_x0": 8 * Mc + 4 * M,         # half spectrum in, real force mesh out (16-point pass fused)
        "cols_inv": 16 * Mc,
        "c2r_rows": 8 * Mc + 4 * M,
        "readout_kick_drift": 12 * M + 48 * P,
        "sort_count": 12 * P,             # positions in (counts per key only)
        "sort_scatter": 50 * P,           # x, p, tag in (key recomputed); sorted x, p, tag out
    }
    paint_step = 12 * P + 4 * M           # positions in, float32 density contrast written once
    step = 60 * P + 40 * M + 128 * Mc
    return per_launch, paint_step, step


def cpu_baseline(P_target, n_target):
    """The oracle as it stands: one FP64 orc_step (paint, FFT, Green's
    function, three inverse FFTs, readout, kick and drift) on synthetic
    evolved states of the C1, C5, C4-coarse and C2 shapes, timed on the host
    cores, and a least-squares fit t = c + a P + b M ln M over the four (relative
    residuals), extrapolated to the target workload, whose 2048^3 FP64 mesh
    does not fit in host memory."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import numpy as np
    import oracle as O
    from paper_2007_13394_amd import inputs as I
    rows = []
    for name in ("C1", "C5", "C4_coarse", "C2"):
        cfg = I.config(name)
        s = O.make_sim(cfg)
        x32, p32 = I.synthetic_state(cfg, seed=99)
        x, p = x32.astype(np.float64), p32.astype(np.float64)
        kick, drift = O.kdk_factors(s.cosmo, [0.5], [0.48], [0.52], [0.54])
        t0 = time.perf_counter()
        O.step(s, x, p, float(kick[0]), float(drift[0]))
        dt = time.perf_counter() - t0
        M = cfg["n_mesh"] ** 3
        rows.append((name, x.shape[1], M, dt))
        del x, p
    A = np.array([[1.0 / t, P / t, M * math.log(M) / t] for _, P, M, t in rows])
    coef, *_ = np.linalg.lstsq(A, np.ones(len(rows)), rcond=None)
    c0, a, b = (float(v) for v in coef)
    resid = [(c0 + a * P + b * M * math.log(M)) / t - 1.0 for _, P, M, t in rows]
    Mt = n_target ** 3
    t_target = c0 + a * P_target + b * Mt * math.log(Mt)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    meas = ", ".join(f"{nm} {P} particles {round(M ** (1 / 3))}^3 mesh {t:.2f} s ({P / t:.3g}/s, fit {r:+.1%})"
                     for (nm, P, M, t), r in zip(rows, resid))
    return {
        "value": P_target / t_target,
        "unit": "particle-steps/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"one FP64 oracle step (orc_step, synthetic evolved state) each: {meas}; fit t = c + a P + b M ln M, "
                   f"c = {c0:.3g} s, a = {a:.3g} s, b = {b:.3g} s, extrapolated to {P_target} particles on a {n_target}^3 mesh "
                   f"(t = {t_target:.1f} s/step)"),
    }


# Table 1 shapes: (name, CDM per side, mesh per side, N_fib, the paper's runtime increase on Cori CPU nodes)
RUNTIME_SHAPES = [("NC512_NF3", 512, 1024, 3, 25.0), ("NC512_NF20", 512, 1024, 20, 115.0),
                  ("NC1024_NF3", 1024, 2048, 3, 6.0), ("NC1024_NF20", 1024, 2048, 20, 20.0)]


def runtime_increase():
    """Runtime-per-step increase from the neutrino particles (Sec. 4 and
    Table 1): the whole 5 log + 20 linear step schedule from z = 99 with
    neutrino particles (128^3 sites, 10 shells, 2 N_fib + 1 directions) and
    without (same CDM, mesh and steps; no neutrino particles), timed on the
    GPU after the initial conditions.  L = 1024 Mpc/h, M_nu = 0.1 eV
    (degenerate) for the massive runs; the step cost does not depend on
    either.  A shape whose workspace, particles and white noise do not fit in
    the free device memory (with 2 GiB to spare) is reported as not run;
    NC1024_NF20 (1.93e9 particles) needs about 275 GiB."""
    import torch
    from paper_2007_13394_amd import inputs as I
    from paper_2007_13394_amd import pm
    from paper_2007_13394_amd import run as R
    rows, not_run = [], {}
    for name, nc, nmesh, nfib, paper in RUNTIME_SHAPES:
        res = {"name": name, "n_cdm": nc, "mesh": nmesh, "n_fib": nfib, "paper_increase_pct": paper}
        for kind in ("massive", "massless"):
            cfg = I.config("C3", n_cdm=nc, n_mesh=nmesh, n_fib=nfib, box=1024.0, m_nu=(0.1 / 3,) * 3)
            if kind == "massless":
                cfg = dict(cfg, n_sites=0, m_nu=(0.0, 0.0, 0.0))
            c = pm.make_config(cfg)
            P, _, ws = pm.pm_sizes(c)
            need = ws + 24 * P + 4 * nc ** 3 + (2 << 30)
            torch.cuda.empty_cache()
            free = torch.cuda.mem_get_info()[0]
            if need > free:
                not_run[name] = f"{kind} run needs {need / 2**30:.1f} GiB, {free / 2**30:.1f} GiB free"
                log(f"[bench] {name}: {not_run[name]}")
                break
            ctx = pm.Ctx(c)
            gen = torch.Generator(device="cuda")
            gen.manual_seed(cfg["seed"])
            white = torch.randn((nc, nc, nc), generator=gen, device="cuda", dtype=torch.float32)
            x, p = ctx.particles()
            pm.pm_ic(ctx, white, x, p)
            del white
            calls = R.kdk_calls(*R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in calls:
                pm.pm_step(ctx, x, p, *c)
            torch.cuda.synchronize()
            res[kind + "_particles"] = ctx.P
            res[kind + "_ms_per_step"] = round((time.perf_counter() - t0) / len(calls) * 1e3, 3)
            log(f"[bench] {name} {kind}: {ctx.P} particles, {res[kind + '_ms_per_step']:.2f} ms/step")
            del ctx, x, p
            torch.cuda.empty_cache()
        if name in not_run:
            continue
        res["increase_pct"] = round(100.0 * (res["massive_ms_per_step"] / res["massless_ms_per_step"] - 1.0), 1)
        rows.append(res)
    return {"experiment": "runtime-per-step increase from neutrino particles (Table 1 shapes), 26 pm_step calls "
                          "(5 log + 20 linear steps) from z=99, one MI355X",
            "shapes": rows, "not_run": not_run}


def learned_vs_plain(steps=10, seeds=(200, 201, 202, 203)):
    """Both halves of the learned-vs-plain comparison on C4 (19 070 976
    particles, 25 linear steps from z = 19).  Speed: learned steps on the
    256^3 mesh against plain steps on the 256^3 and 1024^3 meshes, sorted
    contexts, `steps` calls after two untimed ones.  Accuracy: the committed
    parameters (trained and calibrated by `python -m paper_2007_13394_amd.learn`
    on seeds 100-115, loaded with allow_pickle=False) run full learned coarse
    runs from held-out seeds; each is compared with the plain fine-mesh run
    and the plain coarse run from the same seed, painted on the coarse mesh,
    by max |P / P_fine - 1| and min r(k) over k < k_Nyq / 2, per seed and for
    the spectra averaged over the seeds."""
    from paper_2007_13394_amd import inputs as I
    from paper_2007_13394_amd import learn
    from paper_2007_13394_amd import pm
    co = learn.time_steps("C4_coarse", steps)
    fi = learn.time_steps("C4_fine", steps, which=("plain",))
    # the same steps with each call's guard flags checked by the next call
    # (PM_FLAG_DEFER_GUARDS): no host wait between calls
    cod = learn.time_steps("C4_coarse", steps, extra_flags=pm.PM_FLAG_DEFER_GUARDS)
    theta = learn.load_params(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2007_13394_amd",
                                           "c4_learned_theta.npy"))
    held = learn.heldout(I.config("C4_coarse"), I.config("C4_fine"), list(seeds), theta)
    per_seed = [{"seed": r["seed"], "learned_max_err": round(r["learned"], 5),
                 "learned_r_min": round(r["learned_r_min"], 4),
                 "plain_coarse_max_err": round(r["plain_coarse"], 5),
                 "plain_coarse_r_min": round(r["plain_coarse_r_min"], 4)} for r in held["pk_max_rel_err_per_seed"]]
    worst = max(r["learned_max_err"] for r in per_seed)
    return {"workload": "C4: 256^3 CDM + 32^3 sites x 70 neutrinos, L=256 Mpc/h, 25 linear steps from z=19; learned "
                        "correction on a 256^3 mesh vs plain PM on a 1024^3 mesh",
            "particles": co["particles"], "steps_timed": steps,
            "learned_coarse_ms_per_step": round(co["learned_ms_per_step"], 3),
            "plain_coarse_ms_per_step": round(co["plain_ms_per_step"], 3),
            "plain_fine_ms_per_step": round(fi["plain_ms_per_step"], 3),
            "deferred_guards": {"learned_coarse_ms_per_step": round(cod["learned_ms_per_step"], 3),
                                "plain_coarse_ms_per_step": round(cod["plain_ms_per_step"], 3),
                                "speedup_vs_fine": round(fi["plain_ms_per_step"] / cod["learned_ms_per_step"], 2)},
            "learned_particle_steps_per_s": co["particles"] / (co["learned_ms_per_step"] * 1e-3),
            "speedup_vs_fine": round(fi["plain_ms_per_step"] / co["learned_ms_per_step"], 2),
            "accuracy": {"k_range_hMpc": [round(v, 4) for v in held["k_range_hMpc"]], "held_out_seeds": per_seed,
                         "mean_spectrum_learned_max_err": round(held["pk_max_rel_err"]["learned"], 5),
                         "mean_spectrum_plain_coarse_max_err": round(held["pk_max_rel_err"]["plain_coarse"], 5),
                         "mean_spectrum_learned_r_min": round(held["r_min"]["learned"], 4),
                         "mean_spectrum_plain_coarse_r_min": round(held["r_min"]["plain_coarse"], 4),
                         "every_seed_within_1pct": bool(worst <= 0.01)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain step timing (C4)")
    ap.add_argument("--runtime-increase", action="store_true",
                    help="only run the runtime-increase experiment (massive vs massless neutrinos, Table 1 shapes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU slab "
              "decomposition is a design, not part of this library)", file=sys.stderr)
        sys.exit(2)

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    if args.runtime_increase:
        print(json.dumps(runtime_increase()), flush=True)
        return
    import numpy as np
    import torch
    from paper_2007_13394_amd import inputs as I
    from paper_2007_13394_amd import pm
    from paper_2007_13394_amd import run as R

    if args.copy_calibration:
        pm.copy_calibration()
        log("[bench] copy calibration: 1 GiB device-to-device copy done")
    cfg = I.config(args.config)
    n = cfg["n_mesh"]
    log(f"[bench] config {args.config}: mesh {n}^3, CDM {cfg['n_cdm']}^3, sites {cfg['n_sites']}^3")
    ctx = pm.Ctx(pm.make_config(cfg))
    P = ctx.P
    log(f"[bench] particles {P}, workspace {ctx.workspace.numel() / 2**30:.1f} GiB")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(cfg["seed"])
    nc = cfg["n_cdm"]
    white = torch.randn((nc, nc, nc), generator=gen, device="cuda", dtype=torch.float32)
    x, p = ctx.particles()
    t = time.perf_counter()
    pm.pm_ic(ctx, white, x, p)
    torch.cuda.synchronize()
    del white
    log(f"[bench] initial conditions {time.perf_counter() - t:.2f} s")
    a, half = R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"])
    calls = R.kdk_calls(a, half)
    for i in range(args.warmup):
        pm.pm_step(ctx, x, p, *calls[i % len(calls)])
        torch.cuda.synchronize()
        log(f"[bench] warmup call {i}")
    pm.pm_trace_begin(ctx, capacity=64 * max(1, args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        pm.pm_step(ctx, x, p, *calls[i % len(calls)])
        if (i - args.warmup) % 5 == 4:
            log(f"[bench] timed call {i}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    trace = pm.pm_trace_end(ctx)
    if not bool(torch.isfinite(x).all()) or not bool(torch.isfinite(p).all()):
        raise RuntimeError("non-finite particle state after the timed steps")

    per_launch, paint_step, step_bytes = model_bytes(P, n)
    tot = {}
    cnt = {}
    for name, ms in trace:
        tot[name] = tot.get(name, 0.0) + ms
        cnt[name] = cnt.get(name, 0) + 1
    K = args.steps
    kernels = {k: {"ms_per_step": tot[k] / K, "launches_per_step": cnt[k] / K, "avg_ms": tot[k] / cnt[k]}
               for k in tot}
    # paint = zero fill + one launch per segment: one unit per step
    paint_ms = (tot.get("paint", 0.0) + tot.get("fill", 0.0)) / K
    candidates = {k: v["ms_per_step"] for k, v in kernels.items() if k in per_launch}
    candidates["paint"] = paint_ms
    dom = max(candidates, key=candidates.get)
    if dom == "paint":
        bytes_unit, ms_unit = paint_step, paint_ms
    else:
        bytes_unit, ms_unit = per_launch[dom], kernels[dom]["avg_ms"]
    achieved = bytes_unit / (ms_unit * 1e-3) / 1e9
    for k, v in kernels.items():
        b = per_launch.get(k)
        if b:
            v["gbs"] = round(b / (v["avg_ms"] * 1e-3) / 1e9, 1)
        t = measured_traffic(k) if args.config == "C3" else None
        if t:
            v["traffic_gb"] = round(t / 1e9, 2)
    ms_per_step = elapsed / K * 1e3
    value = P * K / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "cdm_only_particle_steps_per_s": cfg["n_cdm"] ** 3 * K / elapsed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['n_cdm']}^3 CDM + {cfg['n_sites']}^3 sites x 70 neutrinos "
                               f"on a {n}^3 mesh, L={cfg['box']:g} Mpc/h, M_nu={sum(cfg['m_nu']):g} eV, "
                               f"{cfg['n_log']} log + {cfg['n_lin']} linear steps from z=99, int64 fixed-point paint",
                   "particles": P, "mesh": n},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom) if args.config == "C3" else None},
        "step_roofline": {"model_bytes_per_step": step_bytes,
                          "frac": round(step_bytes / (HBM_PEAK_GBS * 1e9) / (ms_per_step * 1e-3), 4)},
        "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in sorted(kernels.items())},
    }
    del ctx, x, p
    torch.cuda.empty_cache()
    if not args.no_learned and args.config == "C3":
        log("[bench] learned (256^3 mesh) vs plain (256^3, 1024^3 meshes) on C4: step timing, held-out runs")
        out["learned_vs_plain"] = learned_vs_plain()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(P, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
