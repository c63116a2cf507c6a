"""The hot path at the benchmark's full size (C3: 1024^3 CDM + 128^3 x 70
neutrinos on a 2048^3 mesh, 1.22e9 particles), in the launch configuration
the benchmark times (tile sort, tile paint, fused transforms, tile readout
with kick and drift), checked on a million sampled particles against the
library's unsorted path (global-atomic paint, gather readout).  The int64
paint is bit-exact under any particle order, so both paths see the same
force meshes: the step's momentum change over the kick factor must equal the
unsorted force up to float32 rounding, and the drift must follow.  (The FP64
oracle cannot run a 2048^3 mesh in test time; the transforms themselves are
checked at 2048^3 by closed forms in test_gpu_large.py.)  Peak device memory
is about 262 GB."""
import gc
import sys

import numpy as np
import pytest
import torch

from paper_2007_13394_amd import inputs as I
from paper_2007_13394_amd import run as R
from cell_oracle import oracle_cells

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def free_device_memory():
    gc.collect()
    torch.cuda.empty_cache()
    yield
    gc.collect()
    torch.cuda.empty_cache()


def test_c3_sorted_step_matches_unsorted_force(dev, free_device_memory):
    from paper_2007_13394_amd import pm
    cfg = I.config("C3")
    ctx = pm.Ctx(pm.make_config(cfg))
    assert ctx.sorts
    P, n, nc = ctx.P, cfg["n_mesh"], cfg["n_cdm"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"])
    white = torch.randn((nc, nc, nc), generator=gen, device=dev, dtype=torch.float32)
    x, p = ctx.particles()
    pm.pm_ic(ctx, white, x, p)
    del white
    say("C3 initial conditions done,", P, "particles")
    rng = np.random.default_rng(3)
    sample = torch.from_numpy(np.sort(rng.choice(P, 1_000_000, replace=False))).to(dev)
    acc = torch.empty_like(x)
    pm.pm_force(ctx, x, acc)
    acc_s, p_s, x_s = acc[:, sample].double(), p[:, sample].double(), x[:, sample].double()
    del acc
    torch.cuda.empty_cache()
    call = R.kdk_calls(*R.schedule(cfg["a0"], cfg["n_lin"], cfg["n_log"], cfg["a_mid"]))[0]
    kick, drift = pm.pm_kdk_factors(ctx, *call)
    ids = torch.arange(P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    pm.pm_step(ctx, x, p, *call)
    pm.pm_attach_ids(ctx, None)
    say("C3 sorted step done")
    assert bool(torch.isfinite(x).all()) and bool(torch.isfinite(p).all())
    assert bool(((x >= 0) & (x < n)).all())
    assert int(ids.sum(dtype=torch.int64)) == P * (P - 1) // 2
    # slot of every original particle, built in chunks (no P-sized int64 temporary)
    inv = torch.empty_like(ids)
    step = 1 << 26
    for lo in range(0, P, step):
        hi = min(P, lo + step)
        inv[ids[lo:hi].long()] = torch.arange(lo, hi, dtype=torch.int32, device=dev)
    slots = inv[sample].long()
    del inv, ids
    p_new, x_new = p[:, slots].double(), x[:, slots].double()
    # CDM: the force itself, from the momentum change over the kick factor
    cdm = sample < nc ** 3
    f_step = (p_new[:, cdm] - p_s[:, cdm]) / kick
    e_f = float(torch.linalg.vector_norm(f_step - acc_s[:, cdm]) / torch.linalg.vector_norm(acc_s[:, cdm]))
    # neutrinos: thermal momenta at z = 99 dwarf the kick, so check the update to float32 rounding of |p|
    nu = ~cdm
    pred = p_s[:, nu] + kick * acc_s[:, nu]
    e_nu = float(((p_new[:, nu] - pred).abs().amax(dim=0) / pred.abs().amax(dim=0).clamp_min(1e-30)).max())
    dx = torch.remainder(x_s + drift * p_new - x_new + n / 2, n) - n / 2
    e_x = float(dx.abs().max())
    say("C3 sampled:", int(cdm.sum()), "CDM, force from the sorted step vs unsorted force rel L2", e_f, ";",
        int(nu.sum()), "neutrinos, max momentum deviation / |p|", e_nu, "; drift max |dx|", e_x, "cells")
    del x, p, ctx
    assert e_f < 1e-5
    assert e_nu < 1e-6
    assert e_x < 2e-3


def test_c3_tile_paint_equals_atomic_paint(dev, free_device_memory):
    """At the full 2048^3 size (8 x 128^3 tile keys, Morton tile indices up
    to 2^21) the tile paint and the global-atomic paint give the same
    integers: the mesh painted through the tile sort, minus every segment
    painted again with global atomics and the negated quantum (the paint is
    odd in the quantum: rint(-v) = -rint(v) and the remainder corner
    follows), is zero in every cell.  Before that, 9500 sampled cells (random,
    and on tile faces and the wrap) equal the FP64 oracle's integers.  Device
    memory: workspace, positions and one int64 mesh, about 281 GiB."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C3")
    ctx = pm.Ctx(pm.make_config(cfg))
    assert ctx.sorts
    P, n, nc = ctx.P, cfg["n_mesh"], cfg["n_cdm"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg["seed"] + 1)
    white = torch.randn((nc, nc, nc), generator=gen, device=dev, dtype=torch.float32)
    x, p = ctx.particles()
    pm.pm_ic(ctx, white, x, p)
    del white, p
    gc.collect()
    torch.cuda.empty_cache()
    # move the neutrinos off their shells so that tile faces and wraps are hit everywhere
    off, _, q = pm.pm_segments(ctx)
    u = torch.empty(3, P - nc ** 3, dtype=torch.float32, device=dev)
    u.uniform_(0.0, float(n), generator=gen)
    x[:, nc ** 3:] = torch.where(u < n, u, torch.zeros_like(u))
    del u
    torch.cuda.empty_cache()
    mesh = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    say("C3 paint check: tile paint of", P, "particles")
    pm.pm_paint(ctx, x, 0, ctx.nseg, mesh)
    # the FP64 oracle on sampled cells of the full mesh: random cells, and
    # cells on tile faces and on the wrap (coordinates 0, 15, 16, 2047)
    rng = np.random.default_rng(31)
    special = np.array([0, 15, 16, 1023, 1024, n - 16, n - 1], dtype=np.int64)
    cells = np.concatenate([rng.integers(0, n, size=(8000, 3)), rng.choice(special, size=(1500, 3))])
    want, nfound = oracle_cells(x, off, q, n, cells, dev)
    lin = torch.from_numpy((cells[:, 0] * n + cells[:, 1]) * n + cells[:, 2]).to(dev)
    got = mesh[lin].cpu().numpy()
    say("C3 paint check:", len(cells), "sampled cells from", nfound, "particles;", int(np.sum(got != want)),
        "differ from the oracle; nonzero cells", int(np.sum(want != 0)))
    assert np.array_equal(got, want)
    for g in range(ctx.nseg):
        pm.pm_paint_q(ctx, x, int(off[g]), int(off[g + 1] - off[g]), -int(q[g]), mesh)
    nz, step = 0, 1 << 28
    for lo in range(0, n ** 3, step):
        nz += int(torch.count_nonzero(mesh[lo:lo + step]))
    say("C3 paint check: cells where tile and atomic paints differ:", nz)
    del mesh, x, ctx
    assert nz == 0
