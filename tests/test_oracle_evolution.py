"""End-to-end pin of the oracle evolution: a Zel'dovich pancake.

Before shell crossing a single plane wave evolves exactly along x = q + D(a) s
for any expansion history (the planar force is 1.5 Omega_m0 D s exactly), and
FastPM's modified factors make the time integration exact on that trajectory
(Sec. 2.3).  What remains is the mesh discretisation, which must vanish at
first order in the cell size.  The run starts once the displacement spans a
few cells; from sub-cell displacements the cloud-in-cell assignment of a
lattice dominates the force error (see the design notes).
"""
import numpy as np

import oracle as O


def _pancake(N, nc1, nsteps=5, a0=0.2, af=0.5):
    cfg = dict(box=N * 2.0, n_mesh=N, n_cdm=nc1, n_sites=0, n_shell=10, n_fib=3, omega_m=0.3,
               h=0.7, n_s=0.96, sigma8=0.8, m_nu=[0, 0, 0], a0=a0)
    s = O.make_sim(cfg)
    a = np.linspace(a0, af, nsteps + 1)
    half = 0.5 * (a[1:] + a[:-1])
    D, G = O.growth(s.cosmo, [a0, af, 1.0])
    B, k = 1.0 / D[2], 2 * np.pi / N              # shell crossing at a = 1
    q = np.indices((nc1,) * 3).reshape(3, -1).astype(float) * (N / nc1)
    sq = np.zeros_like(q)
    sq[0] = -(B / k) * np.sin(k * q[0])
    x = np.ascontiguousarray(np.mod(q + D[0] * sq, N))
    p = np.ascontiguousarray(G[0] * sq)
    O.run(s, x, p, a, half)
    dx = (x - q + N / 2) % N - N / 2
    ex = np.abs(dx[0] - D[1] * sq[0]).max() / np.abs(D[1] * sq[0]).max()
    ep = np.abs(p[0] - G[1] * sq[0]).max() / np.abs(G[1] * sq[0]).max()
    assert np.abs(dx[1:]).max() < 1e-12 and np.abs(p[1:]).max() < 1e-12
    return ex, ep


def test_pancake_follows_zeldovich_and_converges_with_mesh():
    ex64, ep64 = _pancake(64, 64)
    ex128, ep128 = _pancake(128, 128)
    assert ex64 < 0.01 and ep64 < 0.015
    assert ex128 < 0.005 and ep128 < 0.0075
    assert ex128 < 0.6 * ex64 and ep128 < 0.6 * ep64


def test_pancake_with_two_mesh_cells_per_particle():
    ex, ep = _pancake(64, 32)
    assert ex < 0.02 and ep < 0.04
