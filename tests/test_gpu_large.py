"""Large-mesh checks of the GPU transforms by closed forms that hold at any
size (the oracle cannot run 1024^3 or 2048^3 meshes in test time).

A single real Fourier mode cos(2 pi n.u / N) has a half spectrum with one
nonzero entry, N^3 / 2, and its force mesh is -1.5 Omega_m A (k / k^2)
sin(k.u) (the single-mode pin of the oracle)."""
import gc
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


def _modes(n, rng):
    """About 16 real Fourier modes per 8-column block of the half spectrum,
    with the 16 residues of n0 mod 16 in each block: after the forward rows
    every tile of every pass holds data, a skipped or misplaced tile shows.
    Column blocks 0 and the last carry k2 = 0 and k2 = N/2, which the inverse
    real transform treats apart (the k = 0 / Nyquist pair of each row)."""
    ncb = (n // 2 + 1 + 7) // 8
    seen, modes = set(), []
    for cb in range(ncb):
        for c in range(16):
            for _ in range(100):
                k2 = 0 if cb == 0 else (n // 2 if cb == ncb - 1 else min(8 * cb + int(rng.integers(0, 8)), n // 2))
                n0 = c + 16 * int(rng.integers(-(n // 32), n // 32))
                n1 = int(rng.integers(-(n // 2) + 1, n // 2))
                if n0 <= -(n // 2) or n0 >= n // 2:
                    continue
                key = (n0, n1, k2)
                if k2 in (0, n // 2):   # (n0, n1) and (-n0, -n1) are one real mode there
                    key = max(key, (-n0, -n1, k2))
                if key in seen or (n0, n1, k2) == (0, 0, 0):
                    continue
                seen.add(key)
                modes.append((n0, n1, k2))
                break
    return np.array(modes, dtype=np.int64)


@pytest.mark.parametrize("n", [512, 2048])
def test_multi_mode_force_mesh(dev, n):
    """Force mesh of a sum of ~16 (N/16 + 1) random-phase modes against the
    sum of their closed forms -1.5 Omega_m A_m (k_d / k^2) sin(k.u + psi_m),
    the component along an axis at its Nyquist frequency being zero, on one
    output plane of every group of 16 planes the axis-0 passes combine."""
    from paper_2007_13394_amd import pm
    # the context (mesh + three spectra) and `out` take ~257 GiB at 2048^3:
    # cached segments of earlier tests would not merge into them
    gc.collect()
    torch.cuda.empty_cache()
    rng = np.random.default_rng(2048 + n)
    cfg = I.config("C1", n_mesh=n, n_cdm=8, n_sites=0)
    ctx = pm.Ctx(pm.make_config(cfg))
    modes = _modes(n, rng)
    M = len(modes)
    amp = 0.005
    psi = torch.from_numpy(rng.uniform(0, 2 * np.pi, M)).to(dev)
    kv = torch.from_numpy(2 * np.pi * modes / n).to(dev)                      # (M, 3)
    k2 = (kv ** 2).sum(1)
    idx = torch.arange(n, device=dev, dtype=torch.float64)
    V1 = torch.exp(1j * idx[:, None] * kv[None, :, 1])                         # (n, M): axis 1
    V2 = torch.exp(1j * kv[:, 2, None] * idx[None, :]).contiguous()           # (M, n): axis 2
    say("multi-mode force", n, M, "modes")

    def field(planes, coef):
        # Re sum_m coef_m exp(i (psi_m + k0_m a)) exp(i k1_m i) exp(i k2_m j) on planes a
        a = torch.as_tensor(planes, device=dev, dtype=torch.float64)
        c = coef[None, :] * torch.exp(1j * (psi[None, :] + a[:, None] * kv[None, :, 0]))   # (B, M)
        return torch.matmul((V1[None] * c[:, None, :]).contiguous(), V2).real

    out = torch.empty(3 * n ** 3, dtype=torch.float32, device=dev)
    q = out[:2 * n ** 3].view(torch.int64).view(n, n, n)
    ones = torch.full((M,), amp, dtype=torch.complex128, device=dev)
    B = 8
    for a0 in range(0, n, B):
        q[a0:a0 + B] = torch.round((1.0 + field(range(a0, a0 + B), ones)) * 2.0 ** 40).to(torch.int64)
    say("multi-mode force", n, "mesh built")
    pm.pm_force_mesh(ctx, q.reshape(-1), out)
    o = out.view(3, n, n, n)
    n2 = n // 16
    planes = [j + n2 * (j % 16) for j in range(n2)]
    nyq = torch.from_numpy(np.abs(modes) == n // 2).to(dev)
    err, ss, cnt = [0.0] * 3, 0.0, 0
    for d in range(3):
        # F_d = Re[-1.5 Omega_m A (k_d / k^2) (-i) e^{i theta}]
        g = torch.where(nyq[:, d], torch.zeros_like(k2), -1.5 * 0.3 * amp * kv[:, d] / k2)
        coef = (-1j) * g.to(torch.complex128)
        for b0 in range(0, len(planes), B):
            pl = planes[b0:b0 + B]
            ref = field(pl, coef)
            got = o[d, pl].double()
            err[d] = max(err[d], float((got - ref).abs().max()))
            ss += float((ref ** 2).sum())
            cnt += ref.numel()
    rms = (ss / cnt * 3) ** 0.5     # rms of the force vector
    say("multi-mode force", n, "max error / rms |F| per component", [e / rms for e in err])
    del out, q, o, ctx
    gc.collect()
    torch.cuda.empty_cache()
    assert max(err) / rms < 5e-5


@pytest.mark.parametrize("n", [1024, 2048])
def test_power_mesh_single_mode_closed_form(dev, n):
    """Binned power (Sec. 3) of one real mode A cos(2 pi n.u / N) at full
    size: the modes +n and -n of the full mesh land in bin floor(|n|), which
    holds P n_modes = A^2 L^3 / 2; every other bin is empty up to float32
    rounding of the transform."""
    from paper_2007_13394_amd import pm
    cfg = I.config("C3", n_mesh=n, n_sites=0, n_cdm=8)
    ctx = pm.Ctx(pm.make_config(cfg))
    nv = (-(3 * n // 10 + 1), 77, 13)
    A, L = 0.25, cfg["box"]
    d = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    i = torch.arange(n, device=dev, dtype=torch.float64)
    for a in range(n):
        ph = (2 * np.pi / n) * (nv[0] * a + nv[1] * i[:, None] + nv[2] * i[None, :])
        d[a] = (A * torch.cos(ph)).to(torch.float32)
    nb = 1024
    k, pk, nm = pm.pm_power_mesh(ctx, d.reshape(-1), d.reshape(-1), nb)
    b = int(np.floor(np.sqrt(sum(v * v for v in nv))))
    expect = A * A / 2 * L ** 3
    others = np.delete(np.abs(pk * nm), b)
    say("power_mesh", n, "bin", b, "P n_modes / (A^2 L^3 / 2) - 1 =", pk[b] * nm[b] / expect - 1,
        "largest other bin / expected", others.max() / expect)
    assert abs(pk[b] * nm[b] / expect - 1) < 1e-5
    assert others.max() < 1e-6 * expect
    if n == nb:   # bins up to |n| < N cover every mode of the mesh once
        assert nm.sum() == n ** 3 - 1
    kf = 2 * np.pi / L
    assert b * kf <= k[b] < (b + 1) * kf


def test_power_particle_comb_closed_form_1024(dev):
    """pm_power of particles at every even lattice point (spacing 2 cells):
    the cloud-in-cell paint puts each on one cell, so delta is 7 on those
    cells and -1 elsewhere, whose only nonzero modes are the 7 corners with
    every n_d in {0, N/2} except k = 0, each |delta_k| = M: power L^3 per
    mode, three modes in bin N/2, three in bin floor(sqrt(2) N/2), one in bin
    floor(sqrt(3) N/2)."""
    from paper_2007_13394_amd import pm
    n = 1024
    cfg = I.config("C3", n_mesh=n, n_cdm=n // 2, n_sites=0)
    ctx = pm.Ctx(pm.make_config(cfg, flags=pm.PM_FLAG_NO_SORT))
    h = n // 2
    x = torch.empty((3, ctx.P), dtype=torch.float32, device=dev)
    j = torch.arange(ctx.P, device=dev, dtype=torch.int64)
    x[0] = (2 * (j // (h * h))).to(torch.float32)
    x[1] = (2 * ((j // h) % h)).to(torch.float32)
    x[2] = (2 * (j % h)).to(torch.float32)
    del j
    L = cfg["box"]
    k, pk, nm = pm.pm_power(ctx, x, 0, 1, nbins=2048)
    tot = pk * nm / L ** 3
    b1, b2, b3 = h, int(np.floor(np.sqrt(2) * h)), int(np.floor(np.sqrt(3) * h))
    say("comb power, modes per bin at", (b1, b2, b3), ":", tot[b1], tot[b2], tot[b3])
    assert abs(tot[b1] - 3) < 1e-5 and abs(tot[b2] - 3) < 1e-5 and abs(tot[b3] - 1) < 1e-5
    assert np.abs(np.delete(tot, [b1, b2, b3])).max() < 1e-6


def test_force_vjp_finite_differences_2048(dev):
    """Reverse mode of the force at 2048^3, whose force meshes have padded
    planes: L(x) = <g, F(x)> is quadratic in one coordinate while every
    cloud-in-cell corner stays put (the painted density and the readout
    weights are both affine in it), so a central difference with steps that
    stay inside the cell is exact up to rounding.  The particles sit at
    fractions 0.3-0.7 of their cells and the steps are 1/8 cell (exact in
    float32 at these coordinates)."""
    from paper_2007_13394_amd import pm
    gc.collect()
    torch.cuda.empty_cache()
    n = 2048
    # 64^3 particles carry 2^15 cells of mass each (a few point masses of
    # 2^24 cells would dominate the float32 force meshes around them): a
    # shift of 36 keeps their quanta (2^51) and any cell sum inside int64
    cfg = I.config("C1", n_mesh=n, n_cdm=64, n_sites=0, shift=36)
    ctx = pm.Ctx(pm.make_config(cfg))
    P = ctx.P
    rng = np.random.default_rng(4096)
    # a loose clump so that the particles feel each other, cells and
    # in-cell fractions drawn separately
    cells = rng.integers(960, 1088, size=(3, P))
    frac = rng.uniform(0.3, 0.7, size=(3, P))
    x = torch.from_numpy((cells + frac).astype(np.float32)).to(dev)
    # a sparse cotangent: the float32 rounding of the transforms changes
    # from one force evaluation to the next, and a dense one would sum it
    # over every particle into the differences
    S = rng.choice(P, size=32, replace=False)
    g32 = np.zeros((3, P), dtype=np.float32)
    g32[:, S] = rng.standard_normal((3, 32)).astype(np.float32)
    g = torch.from_numpy(g32).to(dev)
    xb = torch.zeros_like(x)
    pm.pm_force_vjp(ctx, x, g, xb)
    acc = torch.empty_like(x)

    def loss(xx):
        pm.pm_force(ctx, xx, acc)
        return float((acc.double() * g.double()).sum())

    eps = 0.125
    # coordinates of particles inside the cotangent's support (readout and
    # density terms) and outside it (density term only)
    picks = [(int(rng.integers(0, 3)), int(i)) for i in S[:4]]
    picks += [(int(rng.integers(0, 3)), int(rng.integers(0, P))) for _ in range(4)]
    got, want = [], []
    for d, i in picks:
        xp, xm = x.clone(), x.clone()
        xp[d, i] += eps
        xm[d, i] -= eps
        want.append((loss(xp) - loss(xm)) / (2 * eps))
        got.append(float(xb[d, i]))
    got, want = np.array(got), np.array(want)
    scale = np.abs(want).max()
    say("force VJP at 2048^3: reverse mode", got, "central differences", want,
        "max |diff| / max |FD|", np.abs(got - want).max() / scale)
    del ctx, x, g, xb, acc
    gc.collect()
    torch.cuda.empty_cache()
    assert scale > 0
    assert np.abs(got - want).max() < 1e-3 * scale
