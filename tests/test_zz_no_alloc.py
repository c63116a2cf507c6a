"""The no-allocation paint entry point (pm_paint_static: pm_paint's tile path
with its sort scratch in the library's fixed device array) against pm_paint
through the C ABI: identical int64 meshes on two calls in a row, the second
on a smaller input (the fixed array keeps the first call's contents), the
size limits and the state error."""
import sys

import numpy as np
import pytest
import torch

from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _paint_both(pm, dev, cfg, seed, lo=0, hi=None):
    ctx = pm.Ctx(pm.make_config(cfg))
    hi = ctx.nseg if hi is None else hi
    x, _ = I.synthetic_state(cfg, seed=seed)
    n = cfg["n_mesh"]
    m = (x.shape[1]) // 5
    x[:, :m] = I.tile_face_positions(n, m, seed=seed + 1)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    ref = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
    pm.pm_paint(ctx, xd, lo, hi, ref)
    got = torch.full_like(ref, 5)          # the call adds into the mesh
    pm.pm_paint_static(ctx, xd, lo, hi, got)
    torch.cuda.synchronize()
    return torch.equal(got - 5, ref), int((got - 5 != ref).sum())


def test_paint_static_matches_paint_on_two_calls(dev):
    from paper_2007_13394_amd import pm
    say("no-alloc paint: C5 (256^3, 2.38M particles)")
    ok, nd = _paint_both(pm, dev, I.config("C5"), seed=81)
    assert ok, f"{nd} cells differ on the first call"
    say("no-alloc paint: C1 (64^3, 68608 particles), after the larger call")
    ok, nd = _paint_both(pm, dev, I.config("C1"), seed=82)
    assert ok, f"{nd} cells differ on the second, smaller call"
    ok, nd = _paint_both(pm, dev, I.config("C1"), seed=83, lo=1, hi=4)
    assert ok, f"{nd} cells differ on a segment subset"


def test_paint_static_limits(dev):
    from paper_2007_13394_amd import pm
    big = pm.Ctx(pm.make_config(I.config("C1", n_mesh=1024, n_cdm=8, n_sites=0)))
    x = torch.zeros((3, big.P), dtype=torch.float32, device=dev)
    mesh = torch.zeros(8, dtype=torch.int64, device=dev)
    with pytest.raises(pm.PMError) as e:
        pm._check(pm._lib.pm_paint_static(big.h, pm.C.c_void_p(x.data_ptr()), 0, 1,
                                          pm.C.c_void_p(mesh.data_ptr()), pm._stream()))
    assert e.value.status == pm.PM_ERR_SIZE
    small = pm.Ctx(pm.make_config(I.config("C1", n_mesh=16, n_cdm=8, n_sites=0)))
    x = torch.zeros((3, small.P), dtype=torch.float32, device=dev)
    mesh = torch.zeros(16 ** 3, dtype=torch.int64, device=dev)
    with pytest.raises(pm.PMError) as e:
        pm.pm_paint_static(small, x, 0, 1, mesh)
    assert e.value.status == pm.PM_ERR_STATE
