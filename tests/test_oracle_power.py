"""Pins of the oracle power-spectrum estimator."""
import json
import os

import numpy as np

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_single_mode_lands_in_one_bin_with_exact_power():
    n, L, A = 16, 100.0, 0.3
    u = np.indices((n, n, n))
    nv = np.array([2, 1, 2])                       # |n| = 3
    d = A * np.cos(2 * np.pi * (nv[:, None, None, None] * u).sum(0) / n)
    k, pk, nm = O.power(d, None, L, 12)
    nz = np.nonzero(np.abs(pk) > 1e-20)[0]
    assert list(nz) == [3]
    assert abs(pk[3] * nm[3] / (A * A / 2 * L ** 3) - 1) < 1e-12
    assert 3 * 2 * np.pi / L <= k[3] < 4 * 2 * np.pi / L


def test_mode_count_and_white_noise_level():
    n, L = 16, 50.0
    d = np.random.default_rng(7).normal(scale=0.5, size=(n, n, n))
    k, pk, nm = O.power(d, None, L, 40)
    assert nm.sum() == n ** 3 - 1
    ok = nm > 20
    expect = 0.25 * L ** 3 / n ** 3
    z = (pk[ok] / expect - 1) / np.sqrt(1.0 / nm[ok])       # Gaussian error of a mean of |d|^2
    assert np.abs(z).max() < 5
    # cross with itself is the auto power; cross with its negative flips sign
    _, pc, _ = O.power(d, d.copy(), L, 40)
    assert np.allclose(pc, pk, rtol=1e-13, atol=0)
    _, pm, _ = O.power(d, -d, L, 40)
    assert np.allclose(pm, -pk, rtol=1e-13, atol=0)


def test_k_grid_matches_printed_neutrino_grid_wavenumber():
    # k_n = 2 pi N_sites^(1/3) / L printed as ~0.8 h/Mpc for 128 sites in 1 Gpc/h;
    # the same k on a small mesh: a mode n = 8 in a box of 1000 * 8 / 128 Mpc/h
    g = GOLD["k_nu_grid_hMpc"]
    L = g["inputs"]["box"] * 8 / g["inputs"]["n_sites"]
    n = 32
    d = np.cos(2 * np.pi * 8 * np.indices((n, n, n))[2] / n)
    k, pk, nm = O.power(d, None, L, 20)
    b = int(np.argmax(np.abs(pk)))
    kf = 2 * np.pi / L
    assert b == 8 and kf * b <= k[b] < kf * (b + 1)          # bin b holds |k| in [b, b+1) k_f
    assert round(kf * b, g["decimals"]) == g["value"] and abs(kf * b - 0.80425) < 1e-4
