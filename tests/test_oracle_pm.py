"""Pins of the oracle paint, Poisson force and readout: exact arithmetic of the
cloud-in-cell assignment, closed-form single-mode forces, Newton's third law."""
from fractions import Fraction

import numpy as np

import oracle as O
from paper_2007_13394_amd import inputs as I


def test_paint_conserves_mass_exactly_and_rounds_each_corner():
    n = 16
    x = np.random.default_rng(0).uniform(0, n, size=(3, 500)).astype(np.float32).astype(np.float64)
    Qm = 3 * 2 ** 40 + 12345
    mesh = O.paint_q(x, 0, 500, Qm, n)
    assert mesh.sum() == 500 * Qm
    # brute force with exact rationals for a few particles: each of the first
    # seven corners is the nearest integer to the exact weight times Qm
    for i in range(5):
        one = O.paint_q(x[:, i:i + 1], 0, 1, Qm, n)
        u = [Fraction(float(v)) for v in x[:, i]]
        f = [int(np.floor(float(v))) for v in x[:, i]]
        d = [u[k] - f[k] for k in range(3)]
        t = 0
        for c0 in (0, 1):
            for c1 in (0, 1):
                for c2 in (0, 1):
                    w = Fraction(1)
                    for k, c in zip(range(3), (c0, c1, c2)):
                        w *= d[k] if c else 1 - d[k]
                    cell = ((f[0] + c0) % n, (f[1] + c1) % n, (f[2] + c2) % n)
                    exact = w * Qm
                    if t < 7:
                        assert abs(one[cell] - exact) <= Fraction(1, 2) + Fraction(1, 1000)
                    t += 1
        assert one.sum() == Qm


def test_paint_lattice_point_centre_and_translation():
    n = 8
    Qm = 2 ** 40
    m = O.paint_q(np.array([[3.0], [5.0], [7.0]]), 0, 1, Qm, n)
    assert m[3, 5, 7] == Qm and np.count_nonzero(m) == 1
    m = O.paint_q(np.array([[3.5], [5.5], [7.5]]), 0, 1, Qm, n)
    v = m[m != 0]
    assert len(v) == 8 and np.all(np.abs(v - Qm // 8) <= 1) and m.sum() == Qm
    assert m[3, 5, 7] != 0 and m[4, 6, 0] != 0                # wraps across the boundary
    x = I.adversarial_positions(n, 64, 1).astype(np.float64)
    a = O.paint_q(x, 0, 64, Qm, n)
    b = O.paint_q(np.mod(x + np.array([[1.0], [2.0], [3.0]]), n), 0, 64, Qm, n)
    assert np.array_equal(np.roll(a, (1, 2, 3), axis=(0, 1, 2)), b)


def test_single_mode_force_closed_form():
    n, om, A = 16, 0.3, 0.01
    u = np.indices((n, n, n)).astype(np.float64)
    kv = 2 * np.pi * np.array([1, 2, -3]) / n
    arg = (kv[:, None, None, None] * u).sum(0)
    F = O.force_mesh_from_delta(A * np.cos(arg), om)
    k2 = (kv ** 2).sum()
    for d in range(3):
        ref = -1.5 * om * A * kv[d] / k2 * np.sin(arg)
        assert np.abs(F[d] - ref).max() < 1e-14
    # mode on the Nyquist plane of component 0 has no component-0 force
    arg = np.pi * u[0] + 2 * np.pi * u[1] / n
    F = O.force_mesh_from_delta(np.cos(arg), om)
    assert np.abs(F[0]).max() < 1e-14 and np.abs(F[1]).max() > 1e-3


def _sim(n=32):
    return O.make_sim(dict(box=128.0, n_mesh=n, n_cdm=n // 2, n_sites=2, n_shell=2, n_fib=1,
                           omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8, m_nu=[0.1 / 3] * 3, a0=0.01))


def test_momentum_conservation_and_third_law():
    n = 32
    x = np.random.default_rng(3).uniform(0, n, size=(3, 300))
    m = np.random.default_rng(4).uniform(0.5, 2.0, size=300)
    rho = np.zeros((n, n, n))
    for i in range(300):
        O.paint_d(x[:, i:i + 1], 0, 1, m[i], n, rho)
    F = O.force_mesh_from_delta(rho / rho.mean() - 1, 0.3)
    acc = O.readout(F, x)
    tot = (acc * m).sum(axis=1)
    assert np.abs(tot).max() < 1e-12 * np.abs(acc * m).sum(axis=1).max()
    # self force of one particle vanishes; two particles pull equally
    for pos in ([[3.3], [7.9], [12.5]], [[0.0], [31.99], [16.5]]):
        pos = np.array(pos)
        rho = O.paint_d(pos, 0, 1, 1.0, n)
        acc = O.readout(O.force_mesh_from_delta(rho - rho.mean(), 0.3), pos)
        assert np.abs(acc).max() < 1e-14
    pos = np.array([[3.3, 9.1], [7.9, 8.2], [12.5, 14.0]])
    rho = O.paint_d(pos[:, :1], 0, 1, 1.0, n) + O.paint_d(pos[:, 1:], 0, 1, 2.0, n)
    acc = O.readout(O.force_mesh_from_delta(rho - rho.mean(), 0.3), pos)
    assert np.abs(acc[:, 0] * 1.0 + acc[:, 1] * 2.0).max() < 1e-14
    # attraction points from 0 towards 1
    assert np.dot(acc[:, 0], pos[:, 1] - pos[:, 0]) > 0


def test_smooth_mass_far_field_is_newtonian():
    # lap phi = 1.5 Om delta: outside a compact unit mass |F| = 1.5 Om / (4 pi r^2).
    # (A one-cell point source rings at the mesh scale under the exact spectral
    # kernel, so the source is a Gaussian blob of width 1.5 cells.)
    n = 64
    u = np.indices((n, n, n)).astype(np.float64)
    r2 = (u[0] - 20.0) ** 2 + (u[1] - 32.0) ** 2 + (u[2] - 32.0) ** 2
    rho = np.exp(-r2 / (2 * 1.5 ** 2))
    rho /= rho.sum()
    F = O.force_mesh_from_delta(rho - rho.mean(), 0.3)
    for r in (8, 10):
        ref = -1.5 * 0.3 / (4 * np.pi * r * r)
        assert abs(F[0, 20 + r, 32, 32] / ref - 1) < 0.03
        assert abs(F[0, 20 - r, 32, 32] / ref + 1) < 0.03
        assert abs(F[1, 20 + r, 32, 32]) < 1e-6 * abs(ref)


def test_readout_constant_and_linear_fields():
    n = 16
    x = np.random.default_rng(5).uniform(1, n - 2, size=(3, 100))
    F = np.empty((3, n, n, n))
    F[0] = 2.5
    F[1] = np.indices((n, n, n))[1] * 0.75          # linear along axis 1
    F[2] = np.indices((n, n, n))[0] - 3.0
    acc = O.readout(F, x)
    assert np.abs(acc[0] - 2.5).max() < 1e-14
    assert np.abs(acc[1] - 0.75 * x[1]).max() < 1e-13
    assert np.abs(acc[2] - (x[0] - 3.0)).max() < 1e-13


def test_segment_masses_sum_to_mesh():
    s = O.make_sim(I.config("C1"))
    off, mass, q = O.segments(s)
    P, nc, nn = O.num_particles(s)
    assert off[-1] == P and off[1] == nc and nn == 8 ** 3 * 70
    total = (np.diff(off) * mass).sum()
    assert abs(total / 64 ** 3 - 1) < 1e-12
    assert abs(mass[1:].sum() * 7 * 8 ** 3 / 64 ** 3 - s.cosmo.omega_nu0 / 0.3) < 1e-12
