"""Write the oracle's learned force (radial-filter MLP + 3^3 CNN correction
of the particle-mesh force) at 4096 sampled particles of a 256^3-mesh
instance to a JSON fixture for the GPU test of the two-pass (axis-0 split)
learned transforms, which run only on meshes of 256^3 and more.

Calls only the FP64 oracle and the seeded input generators: a synthetic
evolved state of the C5 shape with 64^3 CDM and 8^3 sites, and parameters
drawn from a seeded normal distribution (hidden layers scaled by
1/sqrt(fan-in), output layers small), a = 0.5.  About six minutes on eight
cores.

    python tests/golden/make_learned_force.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2007_13394_amd import inputs as I  # noqa: E402

CFG = dict(name="C5", n_cdm=64, n_sites=8)
STATE_SEED, THETA_SEED, A, NSAMPLE = 907, 908, 0.5, 4096


def params(seed):
    rng = np.random.default_rng(seed)
    th = np.zeros(O.NET_NPARAM)
    fan = {"W0": 2, "W1": O.NET_H, "W2": O.NET_H, "W3": O.NET_H, "C1W": 27, "C2W": 27 * O.NET_C, "C3W": 27 * O.NET_C}
    for k, (o, n) in O.NET_OFF.items():
        scale = 0.3 if k.startswith(("W", "B")) else 0.15
        if k in ("W3", "B3", "C3W", "C3B"):
            scale *= 0.2
        th[o:o + n] = rng.standard_normal(n) * scale / np.sqrt(fan.get(k, 1))
    return th.astype(np.float32)


if __name__ == "__main__":
    cfg = I.config(CFG["name"], n_cdm=CFG["n_cdm"], n_sites=CFG["n_sites"])
    s = O.make_sim(cfg)
    x, _ = I.synthetic_state(cfg, seed=STATE_SEED)
    th = params(THETA_SEED)
    t0 = time.time()
    F = O.learned_force(s, th.astype(np.float64), A, x.astype(np.float64))
    plain = O.force(s, x.astype(np.float64))
    idx = np.sort(np.random.default_rng(909).choice(x.shape[1], NSAMPLE, replace=False))
    out = {"config": CFG, "state_seed": STATE_SEED, "theta_seed": THETA_SEED, "a": A, "index": idx.tolist(),
           "force": F[:, idx].tolist(), "plain_force": plain[:, idx].tolist(),
           "_source": "FP64 oracle (orc_learned_force, orc_force) on seeded inputs; no value comes from the GPU library"}
    with open(os.path.join(HERE, "learned_force_256.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote learned_force_256.json in {time.time() - t0:.0f} s", flush=True)
