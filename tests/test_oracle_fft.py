"""Pins of the oracle FFT: the DFT definition, Parseval, inversion, symmetry."""
import numpy as np

import oracle as O


def _rand_c(n, seed):
    r = np.random.default_rng(seed)
    return r.normal(size=(n, n, n)) + 1j * r.normal(size=(n, n, n))


def test_fft_matches_naive_dft_8cubed():
    a = _rand_c(8, 1)
    for sign in (-1, +1):
        ref = O.dft3d_naive(a, sign)
        got = O.fft3d(a, sign)
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13


def test_fft_matches_independent_library_and_roundtrip():
    a = _rand_c(16, 2)
    got = O.fft3d(a, -1)
    assert np.abs(got - np.fft.fftn(a)).max() / np.abs(got).max() < 1e-13
    back = O.fft3d(got, +1) / a.size
    assert np.abs(back - a).max() < 1e-14 * np.abs(a).max() * 10


def test_parseval():
    a = _rand_c(16, 3)
    A = O.fft3d(a, -1)
    assert abs((np.abs(A) ** 2).sum() / a.size / (np.abs(a) ** 2).sum() - 1) < 1e-13


def test_rfft_half_spectrum_and_hermitian_planes():
    r = np.random.default_rng(4).normal(size=(16, 16, 16))
    h = O.rfft3d(r)
    assert h.shape == (16, 16, 9)
    assert np.abs(h - np.fft.rfftn(r)).max() / np.abs(h).max() < 1e-13
    # planes k2 = 0 and k2 = n/2 are Hermitian in (k0, k1)
    for k2 in (0, 8):
        p = h[:, :, k2]
        flip = np.conj(np.roll(p[::-1, ::-1], 1, axis=(0, 1)))
        assert np.abs(p - flip).max() < 1e-12 * np.abs(p).max()
    back = O.irfft3d(h) / r.size
    assert np.abs(back - r).max() < 1e-13
