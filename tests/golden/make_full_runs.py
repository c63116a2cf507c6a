"""Write the oracle's power spectra after full runs (z = 99 -> 0) to JSON
fixtures for the GPU full-run tests.

Calls only the FP64 oracle and the seeded white-noise generator: the
initial conditions of each workload's seed (Sec. 2.1-2.2), the merged-kick
KDK loop on the workload's schedule (Sec. 2.3, Sec. 3), then the total-matter,
CDM, neutrino and CDM x neutrino spectra (Sec. 3) with n_mesh / 2 bins of
width 2 pi / L, without window compensation.

    python tests/golden/make_full_runs.py C5 C2
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2007_13394_amd import inputs as I  # noqa: E402


def full_run(name):
    cfg = I.config(name)
    s = O.make_sim(cfg)
    n = cfg["n_mesh"]
    w = I.white_noise(cfg["seed"], cfg["n_cdm"])
    x, p = O.ic(s, w)
    a, half = O.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"])
    t0 = time.time()

    def progress(i, c, x, p):
        print(f"{name}: call {i} at a = {c[0]:.4f} ({time.time() - t0:.0f} s)", flush=True)

    O.run(s, x, p, a, half, callback=progress)
    off, _, _ = O.segments(s)
    nseg = len(off) - 1
    nb = n // 2
    dm = O.delta_of(s, x, 0, nseg)
    k, pm_, nm = O.power(dm, None, cfg["box"], nb)
    del dm
    dc = O.delta_of(s, x, 0, 1)
    _, pc, _ = O.power(dc, None, cfg["box"], nb)
    out = {"workload": name, "n_mesh": n, "box": cfg["box"], "seed": cfg["seed"], "nbins": nb,
           "n_calls": len(a), "k_mean": k.tolist(), "n_modes": nm.tolist(), "p_matter": pm_.tolist(),
           "p_cdm": pc.tolist()}
    if nseg > 1:
        dn = O.delta_of(s, x, 1, nseg)
        _, pn, _ = O.power(dn, None, cfg["box"], nb)
        _, pcn, _ = O.power(dc, dn, cfg["box"], nb)
        out["p_nu"] = pn.tolist()
        out["p_cdm_nu"] = pcn.tolist()
    out["_source"] = ("FP64 oracle full run from seeded white noise (tests/golden/make_full_runs.py); "
                      "no value comes from the GPU library")
    path = os.path.join(HERE, f"full_run_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    for nm_ in sys.argv[1:] or ["C5", "C2"]:
        full_run(nm_)
