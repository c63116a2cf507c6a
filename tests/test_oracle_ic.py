"""Pins of the oracle initial conditions."""
import numpy as np
from scipy import integrate

import oracle as O
from paper_2007_13394_amd import inputs as I


def _sim(name="C1", **over):
    return O.make_sim(I.config(name, **over))


def test_sigma8_normalisation_independent_quadrature():
    s = _sim()
    A = O.pk_amplitude(s)
    W = lambda x: 3 * (np.sin(x) - x * np.cos(x)) / x ** 3

    def integrand(lnk):
        k = np.exp(lnk)
        q = k / (0.3 * 0.7)
        T = np.log(1 + 2.34 * q) / (2.34 * q) * (1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25
        return k ** 3 * A * k ** 0.96 * T * T * W(8 * k) ** 2 / (2 * np.pi ** 2)

    s2 = integrate.quad(integrand, np.log(1e-6), np.log(1e3), limit=400, epsabs=0, epsrel=1e-11)[0]
    assert abs(np.sqrt(s2) / 0.8 - 1) < 1e-7
    assert abs(O.bbks_T(1e-8) - 1) < 1e-6


def test_cdm_ic_power_matches_input_spectrum():
    s = _sim(n_sites=0)
    w = I.white_noise(11, s.n_cdm)
    x, p, dc, dn = O.ic(s, w, want_disp=True)
    assert np.abs(dc.mean(axis=1)).max() < 1e-12
    # p = (G/D)(a0) s
    D, G = O.growth(s.cosmo, [s.a0])
    assert np.allclose(p, G[0] / D[0] * dc, rtol=1e-12, atol=0)
    # the displacement divergence reproduces the input spectrum in linear theory
    n = s.n_cdm
    L = s.box
    sk = [np.fft.fftn(dc[d].reshape(n, n, n)) * (L / s.n_mesh) for d in range(3)]
    kk = np.fft.fftfreq(n, d=L / n) * 2 * np.pi
    kv = np.meshgrid(kk, kk, kk, indexing="ij")
    div = sum(1j * kv[d] * sk[d] for d in range(3))
    delta = -np.real(np.fft.ifftn(div))
    k, pk, nm = O.power(delta, None, L, n // 2)
    amp = O.pk_amplitude(s) * (D[0] / O.growth(s.cosmo, [1.0])[0][0]) ** 2
    ok = (nm > 30) & (np.arange(len(pk)) < n // 2 - 1)
    ref = np.array([amp * O.pk_unnorm(s, kb) for kb in k[ok]])
    z = (pk[ok] / ref - 1) / np.sqrt(2.0 / nm[ok])
    assert np.abs(z).max() < 5
    assert abs(np.mean(pk[ok] / ref) - 1) < 0.1


def test_neutrino_sites_staggered_shells_disjoint_and_momentum_balanced():
    s = _sim()
    w = I.white_noise(12, s.n_cdm)
    P, nc, nn = O.num_particles(s)
    x, p, dc, dn = O.ic(s, w, want_disp=True)
    xn = x[:, nc:] - np.repeat(dn, 7, axis=1).reshape(3, -1)[:, :0].sum() if False else x[:, nc:]
    # remove each site's bulk displacement to recover the shells
    per = 8 ** 3 * 7
    sh = np.arange(nn) // per
    site = (np.arange(nn) % per) // 7
    rel = (xn - dn[:, site]) % 64
    centre = (np.indices((8, 8, 8)).reshape(3, -1)[:, site] * 4 + 2 + 0.5) * 2.0
    r = np.linalg.norm((rel - centre + 32) % 64 - 32, axis=0)
    e, q, m = O.fd_shells([1.0, 1.0, 1.0], 10)
    expect = 0.4 * 8.0 * q / q[-1]
    assert np.abs(r - expect[sh]).max() < 1e-9
    assert expect.max() < 0.5 * 8.0                     # neighbouring sites' shells never touch
    # sites are never on the CDM lattice (spacing 2 cells): offset is 0.5 lattice units
    assert np.all(np.abs((centre / 2.0) % 1 - 0.5) < 1e-12)
    # thermal momenta: +-v on even/odd sites cancel exactly in the sum
    pth = p[:, nc:] - (O.growth(s.cosmo, [s.a0])[1][0] / O.growth(s.cosmo, [s.a0])[0][0]) * dn[:, site]
    assert np.abs(pth.sum(axis=1)).max() < 1e-9 * np.abs(pth).sum()
    # speed per unit q: k_B T_nu0 c / (100 m_1) Mpc/h, in mesh units (64 / 256)
    speed = np.linalg.norm(pth, axis=0) / q[sh]
    assert np.allclose(speed, s.cosmo.kT_nu / (0.1 / 3) * 299792.458 / 100 * 0.25, rtol=1e-12)
    assert abs(s.cosmo.kT_nu / (0.1 / 3) * 2997.92458 - 15.13) < 0.01


def test_neutrino_site_displacement_is_the_field_half_a_cell_off():
    # brute force: evaluate the band-limited neutrino displacement at a site by a direct sum
    s = _sim(n_cdm=8, n_sites=2, n_mesh=16, box=64.0)
    w = I.white_noise(13, 8)
    x, p, dc, dn = O.ic(s, w, want_disp=True)
    n, L = 8, 64.0
    W = np.fft.fftn(w.astype(np.float64))
    D, _ = O.growth(s.cosmo, [s.a0, 1.0])
    amp = O.pk_amplitude(s) * (D[0] / D[1]) ** 2
    m1 = s.cosmo.m_nu[0]
    a0 = s.a0
    kfs = 0.82 * np.sqrt(s.cosmo.omega_L + 0.3 / a0 ** 3) * a0 ** 2 * m1
    site = np.array([1 * 4 + 2 + 0.5, 0 * 4 + 2 + 0.5, 1 * 4 + 2 + 0.5]) * (L / n)   # Mpc/h
    tot = np.zeros(3)
    for t in np.ndindex(n, n, n):
        kn = np.array([v if v < n // 2 else v - n for v in t])
        if np.any(np.abs(kn) == n // 2) or not kn.any():
            continue
        kv = 2 * np.pi * kn / L
        k = np.linalg.norm(kv)
        dl = W[t] * np.sqrt(amp * O.pk_unnorm(s, k) / (L / n) ** 3) / (1 + (k / kfs) ** 2)
        tot += np.real(1j * kv / k ** 2 * dl * np.exp(1j * kv @ site))
    tot = tot / n ** 3 * (16 / 64.0)
    j = (1 * 2 + 0) * 2 + 1
    assert np.allclose(dn[:, j], tot, rtol=1e-10, atol=1e-14)


def test_free_streaming_transfer_against_a_hand_computed_k_fs():
    """The neutrino displacement is the CDM one times 1 / (1 + (k / k_fs)^2)
    (the configurations' neutrino spectrum is the CDM spectrum times
    [1 + (k / k_fs)^2]^-2), with k_fs the free-streaming wavenumber of
    Lesgourgues & Pastor (2006), 0.82 sqrt(Omega_L + Omega_m (1+z)^3) /
    (1+z)^2 (m / 1 eV) h/Mpc.  Worked by hand for Omega_m = 0.3, z = 99,
    m = 0.1 / 3 eV: Omega_L = 0.69995 after radiation and neutrinos, so
    sqrt(0.69995 + 0.3e6) = 547.72320, times 0.82 = 449.13302, over
    (1+z)^2 = 1e4 and times 1 / 30 eV: k_fs = 1.4971101e-3 h/Mpc.  A box of
    4096 Mpc/h puts its fundamental mode (1.5339808e-3 h/Mpc) near k_fs,
    where the suppression is 0.4878376 and moves with k_fs one to one."""
    s = _sim(n_cdm=8, n_sites=2, n_mesh=16, box=4096.0)
    n = 8
    i0 = np.arange(n)
    w = np.broadcast_to(np.cos(2 * np.pi * i0 / n)[:, None, None], (n, n, n)).astype(np.float32)
    x, p, dc, dn = O.ic(s, w, want_disp=True)
    # CDM displacement along axis 0 on the lattice: alpha cos + beta sin of the mode
    th = 2 * np.pi / n
    f0 = dc[0].reshape(n, n, n)[:, 0, 0]
    alpha, beta = 2 * np.mean(f0 * np.cos(th * i0)), 2 * np.mean(f0 * np.sin(th * i0))
    assert np.allclose(dc[0].reshape(n, n, n), f0[:, None, None], rtol=0, atol=1e-15 * np.abs(f0).max())
    assert np.abs(dc[1:]).max() < 1e-15 * np.abs(f0).max()
    # sites sit half a lattice cell off the lattice points: g = j R + R / 2 + 1/2 (R = 4)
    g = (np.arange(2) * 4 + 2 + 0.5)
    pred = alpha * np.cos(th * g) + beta * np.sin(th * g)
    got = dn[0].reshape(2, 2, 2)
    T = np.sum(got * pred[:, None, None]) / np.sum(4 * pred ** 2)
    assert np.allclose(got, T * pred[:, None, None], rtol=1e-12, atol=1e-16)
    k = 2 * np.pi / 4096.0
    assert abs(k - 1.5339808e-3) < 1e-10
    assert abs(T / (1.0 / (1.0 + (k / 1.4971101e-3) ** 2)) - 1) < 1e-6
    assert abs(T - 0.4878376) < 1e-6
