"""The hot-path paint (tile sort by 16^3-cell block and face flags, then one
workgroup per tile summing its own particles and the corners that cross in
from the 19 lower-neighbour ranges in LDS) against the FP64 oracle's
cloud-in-cell paint, bit for bit, with no fallback.

Cloud-in-cell assignment of every species (Sec. 2.2, "Om_pois" eq.: CDM and
neutrinos both source the potential) in int64 fixed point: the oracle paints
each segment with that segment's integer mass quantum as the library holds
it (pm_segments; the library's and the oracle's independently computed
quanta agree to one unit, checked here too), so the integer meshes must be
identical.  Inputs: the synthetic evolved state with a quarter of every
segment replaced by tile-face cases (last cell of a tile on every
combination of axes, the last cell of the mesh whose upper corner wraps to
cell 0, cell faces, u = N - eps, single-point clumps).  Shapes: 64^3 (C1),
256^3 (C5), 512^3 (C2).  Repeated after shuffling each segment, on segment
subsets, and against the global-atomic paint of an unsorted context."""
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


def _state(cfg, seed):
    x, _ = I.synthetic_state(cfg, seed=seed)
    n = cfg["n_mesh"]
    nc, nn, per = I.counts(cfg)
    segs = [(0, nc)] + [(nc + s * per, nc + (s + 1) * per) for s in range(cfg["n_shell"])] if nn else [(0, nc)]
    for g, (lo, hi) in enumerate(segs):
        m = (hi - lo) // 4
        if m:
            x[:, lo:lo + m] = I.tile_face_positions(n, m, seed=seed * 100 + g)
    return np.ascontiguousarray(x)


def _oracle_mesh(x, off, q, n, lo, hi):
    mesh = np.zeros((n, n, n), dtype=np.int64)
    for g in range(lo, hi):
        O.paint_q(x, int(off[g]), int(off[g + 1] - off[g]), int(q[g]), n, mesh)
    return mesh


@pytest.mark.parametrize("name", ["C1", "C5", "C2"])
def test_tile_paint_bit_exact_vs_oracle(dev, name):
    from paper_2007_13394_amd import pm
    cfg = I.config(name)
    n = cfg["n_mesh"]
    ctx = pm.Ctx(pm.make_config(cfg))
    assert ctx.sorts
    off, _, q = pm.pm_segments(ctx)
    _, _, oq = O.segments(O.make_sim(cfg))
    assert np.all(np.abs(q - oq) <= 1)
    say(name, "quanta differing from the oracle's by one unit:", int(np.sum(q != oq)), "of", len(q))
    x = _state(cfg, seed=61)
    xd = torch.from_numpy(x).to(dev)
    x64 = x.astype(np.float64)
    mesh = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    nseg = ctx.nseg
    for lo, hi in ((0, nseg), (0, 1), (1, nseg), (3, 5)):
        if hi > nseg or lo >= hi:
            continue
        mesh.zero_()
        say(name, "tile paint segments", lo, hi)
        pm.pm_paint(ctx, xd, lo, hi, mesh)
        got = mesh.cpu().numpy().reshape(n, n, n)
        ref = _oracle_mesh(x64, off, q, n, lo, hi)
        assert np.array_equal(got, ref), f"{name} segments [{lo}, {hi}): {int(np.sum(got != ref))} cells differ"
        total = sum(int(off[g + 1] - off[g]) * int(q[g]) for g in range(lo, hi))   # exact, Python ints
        assert int(got.sum(dtype=np.uint64)) == total % 2 ** 64   # the mesh total wraps like the sum
        del got, ref
    # full paint again after shuffling every segment: identical mesh
    mesh.zero_()
    pm.pm_paint(ctx, xd, 0, nseg, mesh)
    rng = np.random.default_rng(62)
    xs = x.copy()
    for g in range(nseg):
        perm = rng.permutation(np.arange(off[g], off[g + 1]))
        xs[:, off[g]:off[g + 1]] = x[:, perm]
    mesh2 = torch.zeros_like(mesh)
    pm.pm_paint(ctx, torch.from_numpy(xs).to(dev), 0, nseg, mesh2)
    assert torch.equal(mesh, mesh2)
    # the global-atomic paint of an unsorted context gives the same integers
    ctx_u = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    mesh3 = torch.zeros_like(mesh)
    pm.pm_paint(ctx_u, xd, 0, nseg, mesh3)
    assert torch.equal(mesh, mesh3)
    say(name, "tile paint bit-exact against the oracle, after a shuffle and against the atomic paint")


def test_tile_paint_after_sorted_steps_vs_oracle(dev):
    """After sorted steps the arrays are permuted and carry segment tags; the
    tile paint of the permuted state equals the oracle paint of the same
    particles in canonical order."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C5")
    n = cfg["n_mesh"]
    ctx = pm.Ctx(pm.make_config(cfg))
    x, p = I.synthetic_state(cfg, seed=63)
    ids = torch.arange(ctx.P, dtype=torch.int32, device=dev)
    pm.pm_attach_ids(ctx, ids)
    xd, pd = torch.from_numpy(x).to(dev), torch.from_numpy(p).to(dev)
    pm.pm_step(ctx, xd, pd, 0.406, 0.3565, 0.4555, 0.505)
    pm.pm_step(ctx, xd, pd, 0.505, 0.4555, 0.5545, 0.604)
    pm.pm_attach_ids(ctx, None)
    mesh = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    pm.pm_paint(ctx, xd, 0, ctx.nseg, mesh)
    order = np.argsort(ids.cpu().numpy())
    xc = xd.cpu().numpy()[:, order].astype(np.float64)
    off, _, q = pm.pm_segments(ctx)
    ref = _oracle_mesh(np.ascontiguousarray(xc), off, q, n, 0, ctx.nseg)
    got = mesh.cpu().numpy().reshape(n, n, n)
    assert np.array_equal(got, ref)
