"""Large-mesh checks of the GPU transforms by closed forms that hold at any
size (the oracle cannot run 1024^3 or 2048^3 meshes in test time).

A single real Fourier mode cos(2 pi n.u / N) has a half spectrum with one
nonzero entry, N^3 / 2, and its force mesh is -1.5 Omega_m A (k / k^2)
sin(k.u) (the single-mode pin of the oracle)."""
import sys

import numpy as np
import pytest
import torch

from paper_2007_13394_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_single_mode_force_mesh(dev, n):
    """Axis-0 frequency n0 = -(3n/10 + 1) lands off the first digit of the
    two-pass axis-0 transform (k0 mod 16 and k0 / 16 both nonzero)."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C1", n_mesh=n, n_cdm=8, n_sites=0)
    ctx = pm.Ctx(pm.make_config(cfg))
    nv = (-(3 * n // 10 + 1), 77, 13)
    A = 0.25
    out = torch.empty(3 * n ** 3, dtype=torch.float32, device=dev)
    # the density is built inside `out` (consumed before out is written)
    q = out[:2 * n ** 3].view(torch.int64).view(n, n, n)
    i = torch.arange(n, device=dev, dtype=torch.float64)
    for a in range(n):
        ph = (2 * np.pi / n) * (nv[0] * a + nv[1] * i[:, None] + nv[2] * i[None, :])
        q[a] = torch.round((1.0 + A * torch.cos(ph)) * 2.0 ** 40).to(torch.int64)
    say("single-mode force", n, nv, "mesh built")
    pm.pm_force_mesh(ctx, q.reshape(-1), out)
    kv = 2 * np.pi * np.array(nv) / n
    k2 = float((kv ** 2).sum())
    o = out.view(3, n, n, n)
    # errors relative to the amplitude of the force vector, 1.5 Omega_m A / |k|
    # (a component's own amplitude can be ~50x smaller than the vector's)
    fmax = 1.5 * 0.3 * A / np.sqrt(k2)
    for d in range(3):
        amp = -1.5 * 0.3 * A * kv[d] / k2
        err = 0.0
        for a in list(range(0, n, max(1, n // 24))) + [n - 1]:
            ph = (2 * np.pi / n) * (nv[0] * a + nv[1] * i[:, None] + nv[2] * i[None, :])
            err = max(err, float((o[d, a].double() - amp * torch.sin(ph)).abs().max()) / fmax)
        say("single-mode force", n, "component", d, "max error / |F|", err)
        assert err < 1e-5


def test_single_mode_fft_2048(dev):
    from paper_2007_13394_amd import pm
    n = 2048
    cfg = I.config("C3", n_sites=0, n_cdm=8)
    ctx = pm.Ctx(pm.make_config(cfg))
    nv = (5, 1021, 13)
    real = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    i = torch.arange(n, device=dev, dtype=torch.float64)
    for a in range(n):   # plane by plane: small temporaries
        ph = (2 * np.pi / n) * (nv[0] * a + nv[1] * i[:, None] + nv[2] * i[None, :])
        real[a] = torch.cos(ph).to(torch.float32)
    spec = torch.empty(n * n * (n // 2 + 1), dtype=torch.complex64, device=dev)
    pm.pm_fft_r2c(ctx, real, spec)
    spec3 = spec.reshape(n, n, n // 2 + 1)
    peak = spec3[nv[0], nv[1], nv[2]].item()
    tot = 0.0
    for a in range(n):   # plane by plane: no mesh-sized temporaries
        pl = spec3[a]
        tot += float((pl.real.double() ** 2 + pl.imag.double() ** 2).sum())
    say("fft 2048 peak", peak, "norm^2 ratio", tot / abs(peak) ** 2)
    assert abs(peak - n ** 3 / 2) < 2e-6 * n ** 3 / 2
    assert abs(tot / abs(peak) ** 2 - 1) < 1e-5
    # inverse: back to N^3 times the field
    pm.pm_fft_c2r(ctx, spec, real.reshape(-1))
    del spec, spec3
    torch.cuda.empty_cache()
    err = 0.0
    for a in range(0, n, 97):
        ph = (2 * np.pi / n) * (nv[0] * a + nv[1] * i[:, None] + nv[2] * i[None, :])
        err = max(err, float((real[a].double() / n ** 3 - torch.cos(ph)).abs().max()))
    say("fft 2048 round trip max error", err)
    assert err < 2e-6
