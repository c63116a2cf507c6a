"""Pins of the oracle background, growth and FastPM factors against closed
forms and independent quadrature (scipy), not against the oracle's own code."""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import zeta

import oracle as O


def test_fd_integral_closed_forms():
    # F(0) = int x^3/(1+e^x) = 7 pi^4 / 120
    assert abs(O.fd_F(0.0) / (7 * np.pi ** 4 / 120) - 1) < 1e-13
    # y >> 1: F = 1.5 zeta(3) y + 11.25 zeta(5) / y + O(y^-3)
    y = 1e4
    assert abs(O.fd_F(y) / (1.5 * zeta(3) * y + 11.25 * zeta(5) / y) - 1) < 1e-12
    # dF/dy against a central difference of F
    for y in (0.3, 5.0, 80.0):
        h = 1e-4 * max(1.0, y)
        fd = (O.fd_F(y + h) - O.fd_F(y - h)) / (2 * h)
        assert abs(O.fd_dF(y) - fd) < 1e-7 * abs(fd)


def test_neutrino_density_today_and_massless_limit():
    c = O.make_cosmo(0.3, 0.7, [0.1 / 3] * 3)
    printed = 0.1 / (93.14 * 0.7 ** 2)          # Omega_nu0 formula of the Introduction
    assert abs(c.omega_nu0 - printed) < 1e-15
    assert abs(O.omega_nu_E2(c, 1.0) / printed - 1) < 2e-3
    # massless: N_eff (7/8)(4/11)^(4/3) Omega_gamma a^-4, standard radiation
    c0 = O.make_cosmo(0.3, 0.7, [0.0] * 3)
    for a in (1e-3, 0.1, 1.0):
        ref = 3.046 * 7 / 8 * (4 / 11) ** (4 / 3) * c0.omega_g / a ** 4
        assert abs(O.omega_nu_E2(c0, a) / ref - 1) < 1e-12
    # photons: Omega_gamma h^2 = 2.47e-5 at T = 2.7255 K
    assert abs(c0.omega_g * 0.49 / 2.4728e-5 - 1) < 1e-3
    # T_nu0 = (4/11)^(1/3) T_gamma for N_eff = 3
    c3 = O.make_cosmo(0.3, 0.7, [0.0] * 3, N_eff=3.0)
    assert abs(c3.kT_nu / 8.617333262e-5 / 1.9454 - 1) < 1e-4
    # flat
    E1 = O.E(c, 1.0)
    assert abs(E1 - 1) < 1e-14


def test_growth_einstein_de_sitter_is_a():
    c = O.make_cosmo(1.0, 0.7, [0.0, 0.0, 0.0], T_cmb=0.0, n_nu=0)
    a = np.array([0.01, 0.1, 0.37, 1.0])
    D, G = O.growth(c, a)
    assert np.abs(D / a - 1).max() < 1e-12
    assert np.abs(G / a ** 1.5 - 1).max() < 1e-12       # G = a^2 E dD/dlna = a^(3/2)


def test_growth_lcdm_matches_heath_integral():
    # no radiation, no neutrinos: D ~ E(a) int_0^a da' / (a' E)^3
    c = O.make_cosmo(0.3, 0.7, [0.0, 0.0, 0.0], T_cmb=0.0, n_nu=0)
    Ef = lambda a: np.sqrt(0.3 / a ** 3 + 0.7)
    heath = lambda a: Ef(a) * integrate.quad(lambda b: 1.0 / (b * Ef(b)) ** 3, 0, a, epsabs=0, epsrel=1e-13)[0]
    a = np.array([0.05, 0.3, 0.6, 1.0])
    D, _ = O.growth(c, a)
    ref = np.array([heath(v) for v in a])
    assert np.abs(D / D[-1] - ref / ref[-1]).max() < 2e-7


def test_G_is_the_canonical_momentum_growth():
    # Zel'dovich: p = G s and dp/da = F/(a^2 E) with F = 1.5 Om D s  =>  dG/da = 1.5 Om D / (a^2 E)
    c = O.make_cosmo(0.3, 0.7, [0.1 / 3] * 3)
    for a in (0.02, 0.2, 0.8):
        h = 1e-4 * a
        D, G = O.growth(c, [a - h, a, a + h], dlna_max=2e-4)
        dGda = (G[2] - G[0]) / (2 * h)
        assert abs(dGda / (1.5 * 0.3 * D[1] / (a * a * O.E(c, a))) - 1) < 1e-6


def test_fastpm_factors_reduce_to_leapfrog_for_small_steps():
    # kick -> int da/(a^2 E), drift -> int da/(a^3 E) for short steps around a_r
    c = O.make_cosmo(0.3, 0.7, [0.1 / 3] * 3)
    for a in (0.05, 0.5):
        h = 1e-3 * a
        kick, drift = O.kdk_factors(c, [a], [a - h], [a + h], [a + h])
        assert abs(kick[0] / (2 * h / (a * a * O.E(c, a))) - 1) < 1e-5
        # drift from a to a+h with the momentum at a+h
        ref = integrate.quad(lambda b: 1 / (b ** 3 * O.E(c, b)), a, a + h, epsrel=1e-12)[0]
        assert abs(drift[0] / ref - 1) < 5e-3   # first order in h (momentum taken at the end)
        kick2, drift2 = O.kdk_factors(c, [a], [a], [a], [a + h])
        assert kick2[0] == 0.0


@pytest.mark.parametrize("n_log", [0, 5])
def test_schedule_ends_at_one(n_log):
    a, half = O.schedule(0.01, 20, n_log, 0.05 if n_log else None)
    assert abs(a[-1] - 1.0) < 1e-15 and len(a) == 21 + n_log
    calls = O.kdk_calls(a, half)
    # kick intervals tile [a0, 1]
    assert calls[0][1] == a[0] and calls[-1][2] == 1.0
    for i in range(len(calls) - 1):
        assert calls[i][2] == calls[i + 1][1]
    if n_log:
        assert abs(a[5] - 0.05) < 1e-15 and abs(half[0] - np.sqrt(a[0] * a[1])) < 1e-17
