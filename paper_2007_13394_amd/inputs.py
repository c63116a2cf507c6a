"""Seeded synthetic inputs and workload parameter sets.

This module holds no arithmetic of the method: it only lists parameter sets
and draws seeded random numbers (white noise for initial conditions, and
synthetic particle states with the structure of the simulated workloads).
Both the GPU path and the CPU oracle consume what it returns.

Workloads (all periodic boxes, Omega_m = 0.3, h = 0.7, n_s = 0.96,
sigma_8 = 0.8, start z = 99; neutrino sites per side = (nominal neutrino
count)^(1/3) / 4, 10 shells, N_fib = 3, i.e. 70 particles per site):

  C1  64^3 mesh,   L = 256 Mpc/h,  32^3 CDM,   8^3 sites,  M_nu = 0.1 eV, 10 linear steps
  C2  512^3 mesh,  L = 512 Mpc/h,  256^3 CDM,  32^3 sites, M_nu = 0.2 eV, 25 linear steps
  C3  2048^3 mesh, L = 1024 Mpc/h, 1024^3 CDM, 128^3 sites, M_nu = 0.06 eV normal
      hierarchy as one effective species, 5 log steps to z = 19 + 20 linear
  C4  256^3 (coarse) / 1024^3 (fine) mesh, L = 256 Mpc/h, 256^3 CDM, 32^3 sites,
      M_nu = 0.1 eV, 25 linear steps, started at z = 19: a mesh four times finer
      than the particle lattice, run from z = 99, builds spurious large-scale
      power from lattice discreteness, so the fine-mesh truth of the learned
      correction starts later (coarse and fine runs alike)
  C5  256^3 mesh, L = 256 Mpc/h, 128^3 CDM, 16^3 sites, M_nu = 0.1 eV, 10 linear steps
  E7  quasi-random (64^3 sites x 10 shells x 51 directions) against pseudo-random
      (512^3 sites x 1) neutrino sampling at 512^3 CDM, 1024^3 mesh,
      L = 1024 Mpc/h, M_nu = 0.2 eV, 5 log + 20 linear steps (C1p: a small
      pseudo-random instance)
"""
import numpy as np

_COMMON = dict(omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8, T_cmb=2.7255, N_eff=3.046,
               n_shell=10, n_fib=3, a0=0.01, flip_odd=1, shift=40)

# normal hierarchy with sum 0.06 eV and the oscillation splittings
# dm21^2 = 7.55e-5 eV^2, |dm31^2| = 2.50e-3 eV^2, heaviest first
NH_006 = (0.0500146897447819, 0.008773208664268256, 0.0012121015909533257)


def _deg(m_tot):
    return (m_tot / 3.0,) * 3


CONFIGS = {
    "C1": dict(_COMMON, box=256.0, n_mesh=64, n_cdm=32, n_sites=8, m_nu=_deg(0.1),
               n_lin=10, n_log=0, a_mid=None, seed=1),
    "C2": dict(_COMMON, box=512.0, n_mesh=512, n_cdm=256, n_sites=32, m_nu=_deg(0.2),
               n_lin=25, n_log=0, a_mid=None, seed=2),
    "C3": dict(_COMMON, box=1024.0, n_mesh=2048, n_cdm=1024, n_sites=128, m_nu=NH_006,
               n_lin=20, n_log=5, a_mid=0.05, seed=3),
    "C4_coarse": dict(_COMMON, box=256.0, n_mesh=256, n_cdm=256, n_sites=32, m_nu=_deg(0.1),
                      n_lin=25, n_log=0, a_mid=None, seed=200, a0=0.05),
    "C4_fine": dict(_COMMON, box=256.0, n_mesh=1024, n_cdm=256, n_sites=32, m_nu=_deg(0.1),
                    n_lin=25, n_log=0, a_mid=None, seed=200, a0=0.05),
    # a small instance of the C4 setting (same box, 4x coarser particles)
    "C4s_coarse": dict(_COMMON, box=256.0, n_mesh=64, n_cdm=64, n_sites=8, m_nu=_deg(0.1),
                       n_lin=10, n_log=0, a_mid=None, seed=150, a0=0.05),
    "C4s_fine": dict(_COMMON, box=256.0, n_mesh=256, n_cdm=64, n_sites=8, m_nu=_deg(0.1),
                     n_lin=10, n_log=0, a_mid=None, seed=150, a0=0.05),
    # pseudo-random neutrino velocities, one neutrino per site (PM_FLAG_NU_PSEUDO)
    "C1p": dict(_COMMON, box=256.0, n_mesh=64, n_cdm=32, n_sites=32, n_shell=1, n_fib=0, m_nu=_deg(0.1),
                n_lin=10, n_log=0, a_mid=None, seed=11),
    # quasi-random vs pseudo-random sampling at equal neutrino counts (64^3 x 10 x 51 vs 512^3, ratio 0.996)
    "E7_qr": dict(_COMMON, box=1024.0, n_mesh=1024, n_cdm=512, n_sites=64, n_shell=10, n_fib=25, m_nu=_deg(0.2),
                  n_lin=20, n_log=5, a_mid=0.05, seed=700),
    "E7_pr": dict(_COMMON, box=1024.0, n_mesh=1024, n_cdm=512, n_sites=512, n_shell=1, n_fib=0, m_nu=_deg(0.2),
                  n_lin=20, n_log=5, a_mid=0.05, seed=700),
    "E7s_qr": dict(_COMMON, box=256.0, n_mesh=128, n_cdm=64, n_sites=8, n_shell=10, n_fib=25, m_nu=_deg(0.2),
                   n_lin=10, n_log=0, a_mid=None, seed=710),
    "E7s_pr": dict(_COMMON, box=256.0, n_mesh=128, n_cdm=64, n_sites=64, n_shell=1, n_fib=0, m_nu=_deg(0.2),
                   n_lin=10, n_log=0, a_mid=None, seed=710),
    "C5": dict(_COMMON, box=256.0, n_mesh=256, n_cdm=128, n_sites=16, m_nu=_deg(0.1),
               n_lin=10, n_log=0, a_mid=None, seed=301),
    "C5_fd16": dict(_COMMON, box=256.0, n_mesh=16, n_cdm=8, n_sites=2, m_nu=_deg(0.1),
                    n_lin=10, n_log=0, a_mid=None, seed=302),
    "C5_fd32": dict(_COMMON, box=256.0, n_mesh=32, n_cdm=16, n_sites=4, m_nu=_deg(0.1),
                    n_lin=10, n_log=0, a_mid=None, seed=303),
}


def config(name, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    return c


def white_noise(seed, n):
    """Unit-variance Gaussian white noise on an n^3 lattice, float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n, n), dtype=np.float32)


def _wrap32(x, n):
    """Reduce into [0, n) and round to float32, keeping every value < n."""
    y = np.mod(x, n).astype(np.float32)
    y[y >= n] = 0.0
    y[y < 0] = 0.0
    return y


def counts(cfg):
    """(n_cdm_particles, n_nu_particles, particles per shell segment)."""
    nc = cfg["n_cdm"] ** 3
    per = cfg["n_sites"] ** 3 * (2 * cfg["n_fib"] + 1)
    return nc, per * cfg["n_shell"], per


def synthetic_state(cfg, seed, clump_frac=0.2, disp_cells=1.5, p_cdm=2.0, p_nu=40.0):
    """A particle state with the structure of an evolved run, float32 SoA [3, P].

    CDM: lattice order, lattice positions plus a smooth random displacement of
    a few cells, with a fraction gathered into tight clumps (halo-like hot
    spots).  Neutrinos: uniform random positions (they are spatially random
    after the first step) and broad random momenta.
    """
    rng = np.random.default_rng(seed)
    n = cfg["n_mesh"]
    nc1 = cfg["n_cdm"]
    nc, nn, _ = counts(cfg)
    P = nc + nn
    dc = n / nc1
    i = np.indices((nc1, nc1, nc1)).reshape(3, -1).astype(np.float64) * dc
    # smooth displacement: a handful of random long-wavelength sinusoids
    disp = np.zeros_like(i)
    for _ in range(6):
        kv = rng.integers(-3, 4, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        amp = rng.normal(size=3) * disp_cells / 3
        arg = 2 * np.pi * (kv[:, None] * i).sum(0) / n + ph
        disp += amp[:, None] * np.sin(arg)[None, :]
    x = i + disp
    # clumps
    ncl = int(clump_frac * nc)
    if ncl:
        centers = rng.uniform(0, n, size=(3, max(1, ncl // 500 + 1)))
        who = rng.choice(nc, size=ncl, replace=False)
        which = rng.integers(0, centers.shape[1], size=ncl)
        x[:, who] = centers[:, which] + rng.normal(scale=0.7, size=(3, ncl))
    p = rng.normal(scale=p_cdm, size=(3, nc)) + 0.5 * disp
    xs = np.empty((3, P), dtype=np.float32)
    ps = np.empty((3, P), dtype=np.float32)
    xs[:, :nc] = _wrap32(x, n)
    ps[:, :nc] = p.astype(np.float32)
    if nn:
        xs[:, nc:] = _wrap32(rng.uniform(0, n, size=(3, nn)), n)
        ps[:, nc:] = rng.normal(scale=p_nu, size=(3, nn)).astype(np.float32)
    return xs, ps


def adversarial_positions(n, count, seed):
    """Paint edge cases: exact cell faces, the largest float below n, cell
    centres and a dense single-point clump."""
    rng = np.random.default_rng(seed)
    k = count // 4
    faces = rng.integers(0, n, size=(3, k)).astype(np.float32)
    top = np.full((3, k), np.nextafter(np.float32(n), np.float32(0)), dtype=np.float32)
    top[:, ::2] = faces[:, ::2]
    centres = rng.integers(0, n, size=(3, k)).astype(np.float32) + np.float32(0.5)
    rest = count - 3 * k
    clump = np.broadcast_to(rng.uniform(0, n, size=(3, 1)).astype(np.float32), (3, rest)).copy()
    x = np.concatenate([faces, top, centres, clump], axis=1)
    x[x >= n] = 0
    return np.ascontiguousarray(x)


def synthetic_density_q(n, seed, shift=40):
    """A clustered int64 fixed-point density mesh (mean about 2^shift per cell):
    lognormal fluctuations on a smooth random field plus a few dense cells."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, n, n))
    # smooth by averaging neighbours a few times (no spectral arithmetic)
    for _ in range(3):
        g = (g + np.roll(g, 1, 0) + np.roll(g, -1, 0) + np.roll(g, 1, 1) + np.roll(g, -1, 1)
             + np.roll(g, 1, 2) + np.roll(g, -1, 2)) / 7.0
    rho = np.exp(2.0 * g)
    rho /= rho.mean()
    idx = rng.integers(0, n, size=(3, 8))
    rho[idx[0], idx[1], idx[2]] += 500.0
    return np.rint(np.ldexp(rho, shift)).astype(np.int64)


def tile_face_positions(n, count, seed, tile=16):
    """Paint edge cases at the faces of the tile^3-cell blocks that a tiled
    paint works on: on each axis independently (so every combination of
    axes occurs) the cell is the last of its block, the last of the mesh
    (its upper corner wraps to cell 0) or a random one, and the offset in the
    cell is 0 (a cell face), 1/2, random, or the largest float32 below the
    next face (N - eps on the last cell).  A tenth of the particles form
    clumps on single points of such cells."""
    rng = np.random.default_rng(seed)
    nt = n // tile
    cell = rng.integers(0, n, size=(3, count))
    kind = rng.integers(0, 4, size=(3, count))
    last_of_tile = rng.integers(0, nt, size=(3, count)) * tile + (tile - 1)
    cell = np.where(kind == 0, last_of_tile, cell)
    cell = np.where(kind == 1, n - 1, cell)
    frac_kind = rng.integers(0, 4, size=(3, count))
    x = cell.astype(np.float32)
    below = np.nextafter((cell + 1).astype(np.float32), np.float32(0))
    x = np.where(frac_kind == 1, x + np.float32(0.5), x)
    x = np.where(frac_kind == 2, (cell + rng.uniform(0, 1, size=(3, count))).astype(np.float32), x)
    x = np.where(frac_kind == 3, below, x)
    x = x.astype(np.float32)
    nclump = count // 10
    if nclump:
        pts = x[:, rng.integers(0, count, size=8)]
        x[:, count - nclump:] = pts[:, rng.integers(0, 8, size=nclump)]
    x[x >= n] = 0
    x[x < 0] = 0
    return np.ascontiguousarray(x)
