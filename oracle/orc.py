"""ctypes binding and run driver for the FP64 oracle (test infrastructure only).

Every function here calls the C oracle in ``liborc.so`` (built from the C
sources beside this file) or restates a step of the paper in plain Python.
Arrays are numpy float64 unless stated; particle arrays are SoA ``[3, P]`` in
mesh-cell units.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_SRC = ["fft.c", "cosmo.c", "nu.c", "ic.c", "pm.c", "power.c", "adj.c", "net.c"]


def build():
    """Compile the oracle (gcc, OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", _SO]
    cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    subprocess.check_call(cmd)


def _load():
    srcs = [os.path.join(_HERE, s) for s in _SRC] + [os.path.join(_HERE, "orc.h")]
    if not os.path.exists(_SO) or max(os.path.getmtime(f) for f in srcs) > os.path.getmtime(_SO):
        build()
    return C.CDLL(_SO)


_lib = _load()

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class Cosmo(C.Structure):
    _fields_ = [("omega_m", C.c_double), ("h", C.c_double), ("T_cmb", C.c_double),
                ("N_eff", C.c_double), ("n_nu", C.c_int), ("m_nu", C.c_double * 3),
                ("omega_g", C.c_double), ("omega_nu0", C.c_double), ("omega_c", C.c_double),
                ("omega_L", C.c_double), ("gamma_nu", C.c_double), ("kT_nu", C.c_double),
                ("a_ini", C.c_double)]


class Sim(C.Structure):
    _fields_ = [("cosmo", Cosmo), ("box", C.c_double), ("n_mesh", C.c_int), ("n_cdm", C.c_int),
                ("n_sites", C.c_int), ("n_shell", C.c_int), ("n_fib", C.c_int),
                ("sigma8", C.c_double), ("n_s", C.c_double), ("a0", C.c_double),
                ("flip_odd", C.c_int), ("shift", C.c_int)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("orc_fft1d", None, [_dp, C.c_long, C.c_int])
_sig("orc_fft3d", None, [_dp, C.c_long, C.c_int])
_sig("orc_dft3d_naive", None, [_dp, _dp, C.c_long, C.c_int])
_sig("orc_rfft3d", None, [_dp, _dp, C.c_long])
_sig("orc_irfft3d", None, [_dp, _dp, C.c_long])
_sig("orc_cosmo_init", C.c_int, [C.POINTER(Cosmo)])
_sig("orc_fd_F", C.c_double, [C.c_double])
_sig("orc_fd_dF", C.c_double, [C.c_double])
_sig("orc_omega_nu_E2", C.c_double, [C.POINTER(Cosmo), C.c_double])
_sig("orc_E", C.c_double, [C.POINTER(Cosmo), C.c_double])
_sig("orc_dlnE_dlna", C.c_double, [C.POINTER(Cosmo), C.c_double])
_sig("orc_growth", C.c_int, [C.POINTER(Cosmo), C.c_int, _dp, _dp, _dp, C.c_double])
_sig("orc_kdk_factors", C.c_int, [C.POINTER(Cosmo), C.c_int, _dp, _dp, _dp, _dp, _dp, _dp])
_sig("orc_fd_tilde", C.c_double, [C.c_int, _dp, C.c_double])
_sig("orc_fd_shells", C.c_int, [C.c_int, _dp, C.c_int, C.c_double, _dp, _dp, _dp])
_sig("orc_fibonacci", None, [C.c_int, _dp])
_sig("orc_num_particles", C.c_long, [C.POINTER(Sim), C.POINTER(C.c_long), C.POINTER(C.c_long)])
_sig("orc_segments", C.c_int, [C.POINTER(Sim), _ip, _dp, _ip])
_sig("orc_bbks_T", C.c_double, [C.c_double])
_sig("orc_pk_unnorm", C.c_double, [C.POINTER(Sim), C.c_double])
_sig("orc_sigma_R", C.c_double, [C.POINTER(Sim), C.c_double, C.c_double])
_sig("orc_pk_amplitude", C.c_double, [C.POINTER(Sim)])
_sig("orc_ic", C.c_int, [C.POINTER(Sim), _fp, _dp, _dp, C.c_void_p, C.c_void_p])
_sig("orc_paint_q", None, [_dp, C.c_long, C.c_long, C.c_long, C.c_int64, C.c_int, _ip])
_sig("orc_paint_d", None, [_dp, C.c_long, C.c_long, C.c_long, C.c_double, C.c_int, _dp])
_sig("orc_force_mesh", None, [_ip, C.c_int, C.c_int, C.c_double, _dp])
_sig("orc_force_mesh_from_delta", None, [_dp, C.c_int, C.c_double, _dp])
_sig("orc_readout", None, [_dp, C.c_int, _dp, C.c_long, _dp])
_sig("orc_force", C.c_int, [C.POINTER(Sim), _dp, _dp])
_sig("orc_step", C.c_int, [C.POINTER(Sim), _dp, _dp, C.c_double, C.c_double, C.c_void_p])
_sig("orc_power", None, [_dp, _dp, C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp])
_sig("orc_ic_w64", C.c_int, [C.POINTER(Sim), _dp, _dp, _dp])
_sig("orc_ic_pseudo", C.c_int, [C.POINTER(Sim), _fp, _dp, _dp, _dp])
_sig("orc_fd_qinv", C.c_double, [C.c_int, _dp, C.c_double])
_sig("orc_ic_vjp", C.c_int, [C.POINTER(Sim), _dp, _dp, _dp])
_sig("orc_density_cont", C.c_int, [C.POINTER(Sim), _dp, _dp])
_sig("orc_force_cont", C.c_int, [C.POINTER(Sim), _dp, _dp])
_sig("orc_step_cont", C.c_int, [C.POINTER(Sim), _dp, _dp, C.c_double, C.c_double])
_sig("orc_force_vjp", C.c_int, [C.POINTER(Sim), _dp, _dp, _dp])
_sig("orc_step_vjp", C.c_int, [C.POINTER(Sim), _dp, C.c_double, C.c_double, _dp, _dp])
_sig("orc_density_vjp", C.c_int, [C.POINTER(Sim), _dp, _dp, _dp])
_sig("orc_net_kt", C.c_double, [C.c_int])
_sig("orc_net_table", None, [_dp, C.c_double, _dp])
_sig("orc_net_table_vjp", None, [_dp, C.c_double, _dp, _dp])
_sig("orc_conv3", None, [_dp, C.c_int, _dp, _dp, C.c_int, C.c_int, _dp])
_sig("orc_conv3_vjp", None, [_dp, C.c_int, _dp, C.c_int, C.c_int, _dp, C.c_void_p, _dp, _dp])
_sig("orc_learned_force", C.c_int, [C.POINTER(Sim), _dp, C.c_double, _dp, _dp])
_sig("orc_learned_loss", C.c_int, [C.POINTER(Sim), _dp, C.c_double, _dp, _dp, C.POINTER(C.c_double), C.c_void_p])


# ---------------------------------------------------------------- FFT
def fft3d(a, sign=-1):
    """Unnormalised 3D complex DFT (sign -1 forward, +1 inverse)."""
    a = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n = a.shape[0]
    _lib.orc_fft3d(a.view(np.float64).reshape(-1), n, sign)
    return a


def dft3d_naive(a, sign=-1):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.empty_like(a)
    _lib.orc_dft3d_naive(a.view(np.float64).reshape(-1), out.view(np.float64).reshape(-1), a.shape[0], sign)
    return out


def rfft3d(real):
    real = np.ascontiguousarray(real, dtype=np.float64)
    n = real.shape[0]
    half = np.empty((n, n, n // 2 + 1), dtype=np.complex128)
    _lib.orc_rfft3d(real.reshape(-1), half.view(np.float64).reshape(-1), n)
    return half


def irfft3d(half):
    """Unnormalised inverse of a half spectrum (n^3 times the field)."""
    half = np.ascontiguousarray(half, dtype=np.complex128)
    n = half.shape[0]
    real = np.empty((n, n, n), dtype=np.float64)
    _lib.orc_irfft3d(half.view(np.float64).reshape(-1), real.reshape(-1), n)
    return real


# ---------------------------------------------------------------- configuration
def make_cosmo(omega_m, h, m_nu=(0.0, 0.0, 0.0), T_cmb=2.7255, N_eff=3.046, n_nu=3):
    c = Cosmo()
    c.omega_m, c.h, c.T_cmb, c.N_eff, c.n_nu = omega_m, h, T_cmb, N_eff, n_nu
    for j in range(3):
        c.m_nu[j] = m_nu[j] if j < len(m_nu) else 0.0
    if _lib.orc_cosmo_init(C.byref(c)) != 0:
        raise ValueError("invalid cosmology")
    return c


def make_sim(cfg):
    """cfg: mapping with box, n_mesh, n_cdm, n_sites, n_shell, n_fib, omega_m, h,
    n_s, sigma8, m_nu (3 masses, eV), a0 and optional T_cmb, N_eff, flip_odd, shift."""
    s = Sim()
    s.cosmo = make_cosmo(cfg["omega_m"], cfg["h"], cfg["m_nu"], cfg.get("T_cmb", 2.7255),
                         cfg.get("N_eff", 3.046))
    s.box = cfg["box"]
    s.n_mesh, s.n_cdm, s.n_sites = cfg["n_mesh"], cfg["n_cdm"], cfg["n_sites"]
    s.n_shell, s.n_fib = cfg["n_shell"], cfg["n_fib"]
    s.sigma8, s.n_s, s.a0 = cfg["sigma8"], cfg["n_s"], cfg["a0"]
    s.flip_odd = int(cfg.get("flip_odd", 1))
    s.shift = int(cfg.get("shift", 40))
    return s


def fd_F(y):
    return _lib.orc_fd_F(y)


def fd_dF(y):
    return _lib.orc_fd_dF(y)


def E(c, a):
    return _lib.orc_E(C.byref(c), a)


def dlnE_dlna(c, a):
    return _lib.orc_dlnE_dlna(C.byref(c), a)


def omega_nu_E2(c, a):
    return _lib.orc_omega_nu_E2(C.byref(c), a)


def growth(c, a, dlna_max=1e-3):
    a = np.ascontiguousarray(np.atleast_1d(a), dtype=np.float64)
    D = np.empty_like(a)
    G = np.empty_like(a)
    if _lib.orc_growth(C.byref(c), len(a), a, D, G, dlna_max) != 0:
        raise ValueError("a below the start of the growth integration")
    return D, G


def kdk_factors(c, a_force, a_k0, a_k1, a_d1):
    arr = [np.ascontiguousarray(np.atleast_1d(v), dtype=np.float64) for v in (a_force, a_k0, a_k1, a_d1)]
    n = len(arr[0])
    kick = np.empty(n)
    drift = np.empty(n)
    if _lib.orc_kdk_factors(C.byref(c), n, *arr, kick, drift) != 0:
        raise ValueError("bad times")
    return kick, drift


def fd_tilde(alpha, q):
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    return _lib.orc_fd_tilde(len(alpha), alpha, q)


def fd_shells(alpha, n_shell, q_max=0.0):
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    edges = np.empty(n_shell + 1)
    q = np.empty(n_shell)
    m = np.empty(n_shell)
    if _lib.orc_fd_shells(len(alpha), alpha, n_shell, q_max, edges, q, m) != 0:
        raise ValueError("bad shell request")
    return edges, q, m


def fibonacci(n_fib):
    d = np.empty((2 * n_fib + 1) * 3)
    _lib.orc_fibonacci(n_fib, d)
    return d.reshape(-1, 3)


def num_particles(sim):
    nc, nn = C.c_long(), C.c_long()
    P = _lib.orc_num_particles(C.byref(sim), C.byref(nc), C.byref(nn))
    return P, nc.value, nn.value


def segments(sim):
    off = np.zeros(66, dtype=np.int64)
    mass = np.zeros(65)
    q = np.zeros(65, dtype=np.int64)
    nseg = _lib.orc_segments(C.byref(sim), off, mass, q)
    if nseg < 1:
        raise ValueError("bad segments")
    return off[: nseg + 1].copy(), mass[:nseg].copy(), q[:nseg].copy()


def bbks_T(q):
    return _lib.orc_bbks_T(q)


def pk_unnorm(sim, k):
    return _lib.orc_pk_unnorm(C.byref(sim), k)


def sigma_R(sim, amp, R):
    return _lib.orc_sigma_R(C.byref(sim), amp, R)


def pk_amplitude(sim):
    return _lib.orc_pk_amplitude(C.byref(sim))


def fd_qinv(n_nu, alpha, u):
    """Inverse cumulative number distribution of the neutrino momenta."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    return _lib.orc_fd_qinv(int(n_nu), a, float(u))


def ic_pseudo(sim, white, u):
    """Initial conditions with pseudo-random neutrino velocities (one per site);
    u: [3, n_sites^3] uniforms."""
    white = np.ascontiguousarray(white, dtype=np.float32).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    P, nc, nn = num_particles(sim)
    if u.size != 3 * nn:
        raise ValueError("u must hold 3 uniforms per neutrino particle")
    x = np.empty(3 * P)
    p = np.empty(3 * P)
    if _lib.orc_ic_pseudo(C.byref(sim), white, u, x, p) != 0:
        raise ValueError("ic_pseudo needs n_shell = 1 and n_fib = 0")
    return x.reshape(3, P), p.reshape(3, P)


def ic(sim, white, want_disp=False):
    """Zel'dovich initial conditions from a float32 white-noise cube."""
    white = np.ascontiguousarray(white, dtype=np.float32).reshape(-1)
    P, nc, nn = num_particles(sim)
    x = np.empty(3 * P)
    p = np.empty(3 * P)
    dc = np.empty(3 * nc) if want_disp else None
    ns = sim.n_sites ** 3
    dn = np.empty(3 * max(ns, 1)) if want_disp else None
    rc = _lib.orc_ic(C.byref(sim), white, x, p,
                     dc.ctypes.data if want_disp else None, dn.ctypes.data if want_disp else None)
    if rc != 0:
        raise ValueError("ic failed")
    x, p = x.reshape(3, P), p.reshape(3, P)
    if want_disp:
        return x, p, dc.reshape(3, nc), dn[: 3 * ns].reshape(3, ns)
    return x, p


# ---------------------------------------------------------------- PM
def paint_q(x, off, cnt, Qm, n, mesh=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    P = x.shape[-1]
    if mesh is None:
        mesh = np.zeros((n, n, n), dtype=np.int64)
    _lib.orc_paint_q(x.reshape(-1), P, off, cnt, int(Qm), n, mesh.reshape(-1))
    return mesh


def paint_d(x, off, cnt, m, n, mesh=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    P = x.shape[-1]
    if mesh is None:
        mesh = np.zeros((n, n, n), dtype=np.float64)
    _lib.orc_paint_d(x.reshape(-1), P, off, cnt, float(m), n, mesh.reshape(-1))
    return mesh


def paint_sim(sim, x, seg_lo=0, seg_hi=None):
    """Fixed-point paint of segments [seg_lo, seg_hi)."""
    off, _, q = segments(sim)
    seg_hi = len(q) if seg_hi is None else seg_hi
    n = sim.n_mesh
    mesh = np.zeros((n, n, n), dtype=np.int64)
    for g in range(seg_lo, seg_hi):
        paint_q(x, int(off[g]), int(off[g + 1] - off[g]), int(q[g]), n, mesh)
    return mesh


def force_mesh(q, S, omega_m):
    q = np.ascontiguousarray(q, dtype=np.int64)
    n = q.shape[0]
    F = np.empty((3, n, n, n))
    _lib.orc_force_mesh(q.reshape(-1), n, S, omega_m, F.reshape(-1))
    return F


def force_mesh_from_delta(delta, omega_m):
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n = delta.shape[0]
    F = np.empty((3, n, n, n))
    _lib.orc_force_mesh_from_delta(delta.reshape(-1), n, omega_m, F.reshape(-1))
    return F


def readout(F, x):
    F = np.ascontiguousarray(F, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    P = x.shape[-1]
    acc = np.empty((3, P))
    _lib.orc_readout(F.reshape(-1), F.shape[1], x.reshape(-1), P, acc.reshape(-1))
    return acc


def force(sim, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    acc = np.empty_like(x)
    if _lib.orc_force(C.byref(sim), x.reshape(-1), acc.reshape(-1)) != 0:
        raise ValueError("force failed")
    return acc


def step(sim, x, p, kick, drift):
    """In place: force at x, p += kick F, x += drift p (periodic).  Returns F."""
    assert x.dtype == np.float64 and p.dtype == np.float64 and x.flags.c_contiguous and p.flags.c_contiguous
    acc = np.empty_like(x)
    if _lib.orc_step(C.byref(sim), x.reshape(-1), p.reshape(-1), kick, drift, acc.ctypes.data) != 0:
        raise ValueError("step failed")
    return acc


def power(da, db, box, nbins, compensate=False):
    da = np.ascontiguousarray(da, dtype=np.float64)
    db = da if db is None else np.ascontiguousarray(db, dtype=np.float64)
    k = np.empty(nbins)
    pk = np.empty(nbins)
    nm = np.empty(nbins)
    _lib.orc_power(da.reshape(-1), db.reshape(-1), da.shape[0], box, nbins, int(compensate), k, pk, nm)
    return k, pk, nm


def delta_of(sim, x, seg_lo, seg_hi):
    """Density contrast of segments [seg_lo, seg_hi), unquantised weights."""
    off, mass, _ = segments(sim)
    n = sim.n_mesh
    rho = np.zeros((n, n, n))
    for g in range(seg_lo, seg_hi):
        paint_d(x, int(off[g]), int(off[g + 1] - off[g]), mass[g], n, rho)
    return rho / rho.mean() - 1.0


# ---------------------------------------------------------------- time stepping
def schedule(a0, n_lin, n_log=0, a_mid=None):
    """Step times: n_log steps uniform in ln a from a0 to a_mid, then n_lin
    steps uniform in a up to 1 (Sec. 3).  Returns (a, a_half) with a_half[i]
    the mid-point of step i (geometric for log steps, arithmetic for linear)."""
    a = [a0]
    half = []
    if n_log:
        l0, l1 = np.log(a0), np.log(a_mid)
        for i in range(1, n_log + 1):
            a.append(float(np.exp(l0 + (l1 - l0) * i / n_log)))
            half.append(float(np.sqrt(a[-2] * a[-1])))
    start = a[-1]
    for i in range(1, n_lin + 1):
        a.append(start + (1.0 - start) * i / n_lin)
        half.append(0.5 * (a[-2] + a[-1]))
    return np.array(a), np.array(half)


def kdk_calls(a, half):
    """(a_force, a_kick0, a_kick1, a_drift1) for the n+1 force evaluations of a
    KDK run with merged kicks: call i kicks from a_{i-1/2} to a_{i+1/2} and
    drifts from a_i to a_{i+1}; the first kick starts at a_0, the last call
    kicks to a_n and does not drift."""
    n = len(a) - 1
    calls = []
    for i in range(n + 1):
        k0 = a[0] if i == 0 else half[i - 1]
        k1 = half[i] if i < n else a[n]
        d1 = a[i + 1] if i < n else a[n]
        calls.append((a[i], k0, k1, d1))
    return calls


def run(sim, x, p, a, half, callback=None):
    """Full KDK run in place on float64 x, p."""
    calls = kdk_calls(a, half)
    cols = list(zip(*calls))
    kick, drift = kdk_factors(sim.cosmo, *cols)
    for i, c in enumerate(calls):
        step(sim, x, p, kick[i], drift[i])
        if callback:
            callback(i, c, x, p)
    return x, p


# ---------------------------------------------------------------- reverse mode
# The differentiable model paints exact segment masses (the fixed-point paint
# agrees with it to 2^-S per cell); see adj.c.
def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def ic_w64(sim, white):
    """Initial conditions from FP64 white noise (same arithmetic as ic)."""
    P, _, _ = num_particles(sim)
    x, p = np.empty(3 * P), np.empty(3 * P)
    if _lib.orc_ic_w64(C.byref(sim), _c64(white).reshape(-1), x, p) != 0:
        raise ValueError("ic failed")
    return x.reshape(3, P), p.reshape(3, P)


def ic_vjp(sim, xbar, pbar):
    """(d(x0, p0)/dw)^T (xbar, pbar) as an n_cdm^3 array."""
    n = sim.n_cdm
    wbar = np.empty(n ** 3)
    if _lib.orc_ic_vjp(C.byref(sim), _c64(xbar).reshape(-1), _c64(pbar).reshape(-1), wbar) != 0:
        raise ValueError("ic_vjp failed")
    return wbar.reshape(n, n, n)


def density_cont(sim, x):
    n = sim.n_mesh
    d = np.empty(n ** 3)
    if _lib.orc_density_cont(C.byref(sim), _c64(x).reshape(-1), d) != 0:
        raise ValueError("density failed")
    return d.reshape(n, n, n)


def force_cont(sim, x):
    x = _c64(x)
    acc = np.empty_like(x)
    if _lib.orc_force_cont(C.byref(sim), x.reshape(-1), acc.reshape(-1)) != 0:
        raise ValueError("force failed")
    return acc


def step_cont(sim, x, p, kick, drift):
    """In place, the differentiable model's step."""
    assert x.dtype == np.float64 and p.dtype == np.float64 and x.flags.c_contiguous and p.flags.c_contiguous
    if _lib.orc_step_cont(C.byref(sim), x.reshape(-1), p.reshape(-1), kick, drift) != 0:
        raise ValueError("step failed")


def force_vjp(sim, x, g):
    xbar = np.zeros(np.shape(x))
    if _lib.orc_force_vjp(C.byref(sim), _c64(x).reshape(-1), _c64(g).reshape(-1), xbar.reshape(-1)) != 0:
        raise ValueError("force_vjp failed")
    return xbar


def step_vjp(sim, x, kick, drift, xbar, pbar):
    """Cotangents of (x', p') -> cotangents of (x, p) for the step taken at x."""
    xb, pb = _c64(xbar).copy(), _c64(pbar).copy()
    if _lib.orc_step_vjp(C.byref(sim), _c64(x).reshape(-1), kick, drift, xb.reshape(-1), pb.reshape(-1)) != 0:
        raise ValueError("step_vjp failed")
    return xb, pb


def density_vjp(sim, x, dmesh):
    xbar = np.zeros(np.shape(x))
    if _lib.orc_density_vjp(C.byref(sim), _c64(x).reshape(-1), _c64(dmesh).reshape(-1), xbar.reshape(-1)) != 0:
        raise ValueError("density_vjp failed")
    return xbar


# ---------------------------------------------------------------- learned correction (net.c)
NET_H, NET_NB, NET_C = 96, 256, 16
_NET_SIZES = [("W0", NET_H * 2), ("B0", NET_H), ("W1", NET_H * NET_H), ("B1", NET_H), ("W2", NET_H * NET_H),
              ("B2", NET_H), ("W3", NET_H), ("B3", 1), ("C1W", NET_C * 27), ("C1B", NET_C),
              ("C2W", NET_C * NET_C * 27), ("C2B", NET_C), ("C3W", NET_C * 27), ("C3B", 1)]
NET_OFF = {}
_o = 0
for _k, _n in _NET_SIZES:
    NET_OFF[_k] = (_o, _n)
    _o += _n
NET_NPARAM = _o


def net_kt(b):
    return _lib.orc_net_kt(b)


def net_table(th, a):
    t = np.empty(NET_NB)
    _lib.orc_net_table(_c64(th), a, t)
    return t


def net_table_vjp(th, a, tbar):
    d = np.zeros(NET_NPARAM)
    _lib.orc_net_table_vjp(_c64(th), a, _c64(tbar), d)
    return d


def conv3(x, W, b):
    """x [ci, n, n, n] -> [co, n, n, n] periodic 3^3 cross-correlation."""
    x = _c64(x)
    ci, n = x.shape[0], x.shape[1]
    co = len(b)
    out = np.empty((co, n, n, n))
    _lib.orc_conv3(x.reshape(-1), ci, _c64(W).reshape(-1), _c64(b), co, n, out.reshape(-1))
    return out


def conv3_vjp(x, W, co, dout, want_dx=True):
    x = _c64(x)
    ci, n = x.shape[0], x.shape[1]
    dx = np.zeros_like(x) if want_dx else None
    dW = np.zeros(co * ci * 27)
    db = np.zeros(co)
    _lib.orc_conv3_vjp(x.reshape(-1), ci, _c64(W).reshape(-1), co, n, _c64(dout).reshape(-1),
                       dx.ctypes.data if want_dx else None, dW, db)
    return dx, dW, db


def learned_force(sim, th, a, x):
    x = _c64(x)
    acc = np.empty_like(x)
    if _lib.orc_learned_force(C.byref(sim), _c64(th), a, x.reshape(-1), acc.reshape(-1)) != 0:
        raise ValueError("learned_force failed")
    return acc


def learned_loss(sim, th, a, x, target, grad=True):
    """(loss, dloss/dth or None) of sum |F - target|^2 / sum |target|^2."""
    loss = C.c_double()
    d = np.zeros(NET_NPARAM) if grad else None
    rc = _lib.orc_learned_loss(C.byref(sim), _c64(th), a, _c64(x).reshape(-1), _c64(target).reshape(-1),
                               C.byref(loss), d.ctypes.data if grad else None)
    if rc != 0:
        raise ValueError("learned_loss failed")
    return loss.value, d

