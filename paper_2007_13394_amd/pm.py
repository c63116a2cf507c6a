"""ctypes binding of libpm (include/pm.h): argument marshalling only.

Every function has the name of the C entry point it calls and takes torch
tensors (device memory) or numpy arrays (host memory).  All device work runs
in libpm's HIP kernels on the current torch stream.  Importing this module
fails if libpm.so has not been built: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np
import torch

_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpm.so")
if not os.path.exists(_SO):
    raise ImportError(f"{_SO} is not built; run __graft_entry__.build()")
_lib = C.CDLL(_SO)

PM_OK, PM_ERR_ARG, PM_ERR_SIZE, PM_ERR_DEVICE, PM_ERR_OVERFLOW, PM_ERR_NAN, PM_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
PM_FLAG_NO_FLIP, PM_FLAG_NO_GUARDS, PM_FLAG_NO_SORT = 1, 2, 4
PM_FLAG_DEFER_GUARDS = 32


class PMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpm status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("n_mesh", C.c_int32), ("n_cdm", C.c_int32), ("n_sites", C.c_int32), ("n_shell", C.c_int32),
                ("n_fib", C.c_int32), ("n_nu", C.c_int32), ("shift", C.c_int32), ("flags", C.c_int32),
                ("box", C.c_double), ("omega_m", C.c_double), ("h", C.c_double), ("n_s", C.c_double),
                ("sigma8", C.c_double), ("T_cmb", C.c_double), ("N_eff", C.c_double),
                ("m_nu", C.c_double * 3), ("a0", C.c_double)]


def make_config(d, flags=0):
    """Config from a parameter mapping (keys as in paper_2007_13394_amd.inputs)."""
    c = Config()
    c.n_mesh, c.n_cdm, c.n_sites = d["n_mesh"], d["n_cdm"], d["n_sites"]
    c.n_shell, c.n_fib = d["n_shell"], d["n_fib"]
    c.n_nu = d.get("n_nu", 3)
    c.shift = d.get("shift", 40)
    c.flags = flags | (0 if d.get("flip_odd", 1) else PM_FLAG_NO_FLIP)
    c.box, c.omega_m, c.h, c.n_s, c.sigma8 = d["box"], d["omega_m"], d["h"], d["n_s"], d["sigma8"]
    c.T_cmb, c.N_eff = d.get("T_cmb", 2.7255), d.get("N_eff", 3.046)
    for j in range(3):
        c.m_nu[j] = d["m_nu"][j]
    c.a0 = d["a0"]
    return c


_vp, _i32, _i64, _dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_cfgp = C.POINTER(Config)


def _sig(name, args):
    f = getattr(_lib, name)
    f.restype = C.c_int
    f.argtypes = args
    return f


_lib.pm_last_error.restype = C.c_char_p
_lib.pm_last_error.argtypes = []
_lib.pm_free.restype = None
_lib.pm_free.argtypes = [_vp]
_sig("pm_sizes", [_cfgp, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(C.c_size_t)])
_sig("pm_init", [_cfgp, _vp, C.c_size_t, _vp, C.POINTER(_vp)])
_sig("pm_segments", [_vp, _vp, _vp, _vp])
_sig("pm_shells", [_vp, _vp, _vp, _vp])
_sig("pm_growth", [_vp, _i32, _vp, _vp, _vp])
_sig("pm_kdk_factors", [_vp, _dbl, _dbl, _dbl, _dbl, C.POINTER(_dbl), C.POINTER(_dbl)])
_sig("pm_ic", [_vp, _vp, _vp, _vp, _vp])
_sig("pm_ic_pseudo", [_vp, _vp, _vp, _vp, _vp, _vp])
_sig("pm_paint_q", [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp])
_sig("pm_paint", [_vp, _vp, _i32, _i32, _vp, _vp])
_sig("pm_paint_static", [_vp, _vp, _i32, _i32, _vp, _vp])
_sig("pm_fft_r2c", [_vp, _vp, _vp, _vp])
_sig("pm_fft_c2r", [_vp, _vp, _vp, _vp])
_sig("pm_force_mesh", [_vp, _vp, _vp, _vp])
_sig("pm_force", [_vp, _vp, _vp, _vp])
_sig("pm_step", [_vp, _vp, _vp, _dbl, _dbl, _dbl, _dbl, _vp])
_sig("pm_density", [_vp, _vp, _vp, _vp])
_sig("pm_density_vjp", [_vp, _vp, _vp, _vp, _vp])
_sig("pm_force_vjp", [_vp, _vp, _vp, _vp, _vp])
_sig("pm_step_vjp", [_vp, _vp, _dbl, _dbl, _dbl, _dbl, _vp, _vp, _vp])
_sig("pm_ic_vjp", [_vp, _vp, _vp, _vp, _vp])
_sig("pm_learned_force", [_vp, _vp, _dbl, _vp, _vp, _vp])
_sig("pm_learned_step", [_vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _dbl, _vp])
_sig("pm_learned_loss", [_vp, _vp, _dbl, _vp, _vp, C.POINTER(C.c_double), _vp, _vp])
_sig("pm_adam", [_vp, _vp, _vp, _vp, _i64, _dbl, _dbl, _dbl, _dbl, _i32, _vp])
_sig("pm_net_table", [_vp, _dbl, _vp, _vp])
_sig("pm_net_table_vjp", [_vp, _dbl, _vp, _vp, _vp])
_sig("pm_power_mesh", [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp])
_lib.pm_net_nparam.restype = C.c_int32
_lib.pm_net_nparam.argtypes = []
_sig("pm_power", [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp])
_sig("pm_trace_begin", [_vp, _i32])
_sig("pm_attach_ids", [_vp, _vp])
_sig("pm_segment_tags", [_vp, _vp, _vp])
_sig("pm_reset_order", [_vp])
_sig("pm_sync", [_vp])
_sig("pm_trace_end", [_vp, _i32, _vp, _vp, C.POINTER(_i32)])
_lib.pm_kernel_name.restype = C.c_char_p
_lib.pm_kernel_name.argtypes = [_i32]

EXPORTS = ["pm_sizes", "pm_init", "pm_free", "pm_last_error", "pm_segments", "pm_shells", "pm_growth",
           "pm_kdk_factors", "pm_ic", "pm_paint_q", "pm_paint", "pm_fft_r2c", "pm_fft_c2r", "pm_force_mesh",
           "pm_force", "pm_step", "pm_power", "pm_trace_begin", "pm_trace_end", "pm_kernel_name", "pm_attach_ids",
           "pm_segment_tags", "pm_reset_order", "pm_density", "pm_density_vjp", "pm_force_vjp", "pm_step_vjp",
           "pm_ic_vjp", "pm_net_nparam", "pm_learned_force", "pm_learned_step", "pm_learned_loss", "pm_adam",
           "pm_power_mesh", "pm_net_table", "pm_net_table_vjp", "pm_ic_pseudo", "pm_paint_static", "pm_sync"]


def _check(st):
    if st != PM_OK:
        raise PMError(st, _lib.pm_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def pm_sizes(cfg):
    P, ns, nb = _i64(), _i32(), C.c_size_t()
    _check(_lib.pm_sizes(C.byref(cfg), C.byref(P), C.byref(ns), C.byref(nb)))
    return P.value, ns.value, nb.value


class Ctx:
    """A libpm context together with the workspace tensor that backs it."""

    def __init__(self, cfg, device="cuda", stream=None):
        self.cfg = cfg
        self.P, self.nseg, nbytes = pm_sizes(cfg)
        self.n = cfg.n_mesh
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        h = _vp()
        _check(_lib.pm_init(C.byref(cfg), C.c_void_p(self._ws_ptr), C.c_size_t(nbytes), _stream(stream), C.byref(h)))
        self.h = h
        self._free = _lib.pm_free   # held here: module globals may be gone at interpreter exit

    @property
    def sorts(self):
        """Whether pm_step tile-sorts (and so permutes) the particles."""
        return self.n // 16 >= 2 and self.P < 2 ** 31 and not (self.cfg.flags & PM_FLAG_NO_SORT)

    def close(self):
        """Release the context (the workspace tensor is freed with the object)."""
        if getattr(self, "h", None) is not None and self.h.value:
            self._free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def particles(self):
        """Fresh (x, p) float32 [3, P] device tensors."""
        return (torch.empty((3, self.P), dtype=torch.float32, device=self.workspace.device),
                torch.empty((3, self.P), dtype=torch.float32, device=self.workspace.device))


def pm_init(cfg, device="cuda", stream=None):
    return Ctx(cfg, device, stream)


def pm_segments(ctx):
    off = np.zeros(ctx.nseg + 1, dtype=np.int64)
    mass = np.zeros(ctx.nseg)
    q = np.zeros(ctx.nseg, dtype=np.int64)
    _check(_lib.pm_segments(ctx.h, off.ctypes.data, mass.ctypes.data, q.ctypes.data))
    return off, mass, q


def pm_shells(ctx):
    ns = ctx.cfg.n_shell
    e, q, m = np.zeros(ns + 1), np.zeros(ns), np.zeros(ns)
    _check(_lib.pm_shells(ctx.h, e.ctypes.data, q.ctypes.data, m.ctypes.data))
    return e, q, m


def pm_growth(ctx, a):
    a = np.ascontiguousarray(np.atleast_1d(a), dtype=np.float64)
    D, G = np.empty_like(a), np.empty_like(a)
    _check(_lib.pm_growth(ctx.h, len(a), a.ctypes.data, D.ctypes.data, G.ctypes.data))
    return D, G


def pm_kdk_factors(ctx, a_force, a_kick0, a_kick1, a_drift1):
    k, d = _dbl(), _dbl()
    _check(_lib.pm_kdk_factors(ctx.h, a_force, a_kick0, a_kick1, a_drift1, C.byref(k), C.byref(d)))
    return k.value, d.value


def pm_ic(ctx, white, x, p, stream=None):
    nc = ctx.cfg.n_cdm ** 3
    _check(_lib.pm_ic(ctx.h, _dev(white, torch.float32, nc, "white"), _dev(x, torch.float32, 3 * ctx.P, "x"),
                      _dev(p, torch.float32, 3 * ctx.P, "p"), _stream(stream)))


def pm_ic_pseudo(ctx, white, u, x, p, stream=None):
    """Initial conditions with pseudo-random neutrino velocities; u: float32
    [3, n_sites^3] device uniforms in [0, 1)."""
    nc, ns = ctx.cfg.n_cdm ** 3, ctx.cfg.n_sites ** 3
    _check(_lib.pm_ic_pseudo(ctx.h, _dev(white, torch.float32, nc, "white"), _dev(u, torch.float32, 3 * ns, "u"),
                             _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(p, torch.float32, 3 * ctx.P, "p"),
                             _stream(stream)))


def pm_paint_q(ctx, x, first, count, quantum, mesh, stream=None):
    """x: float32 [3, stride] device tensor."""
    if x.dim() != 2 or x.shape[0] != 3:
        raise ValueError("x must be [3, stride]")
    n = ctx.n
    _check(_lib.pm_paint_q(ctx.h, _dev(x, torch.float32, name="x"), x.shape[1], first, count, int(quantum),
                           _dev(mesh, torch.int64, n ** 3, "mesh"), _stream(stream)))


def pm_paint(ctx, x, seg_lo, seg_hi, mesh, stream=None):
    _check(_lib.pm_paint(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), seg_lo, seg_hi,
                         _dev(mesh, torch.int64, ctx.n ** 3, "mesh"), _stream(stream)))


def pm_paint_static(ctx, x, seg_lo, seg_hi, mesh, stream=None):
    """pm_paint's tile path with the library's fixed scratch array (no workspace scratch)."""
    _check(_lib.pm_paint_static(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), seg_lo, seg_hi,
                                _dev(mesh, torch.int64, ctx.n ** 3, "mesh"), _stream(stream)))


PM_STATIC_MAX_MESH, PM_STATIC_MAX_PARTICLES = 512, 3145728


def pm_fft_r2c(ctx, real, out, stream=None):
    n = ctx.n
    _check(_lib.pm_fft_r2c(ctx.h, _dev(real, torch.float32, n ** 3, "real"),
                           _dev(out, torch.complex64, n * n * (n // 2 + 1), "out"), _stream(stream)))


def pm_fft_c2r(ctx, spec, real, stream=None):
    n = ctx.n
    _check(_lib.pm_fft_c2r(ctx.h, _dev(spec, torch.complex64, n * n * (n // 2 + 1), "spec"),
                           _dev(real, torch.float32, n ** 3, "real"), _stream(stream)))


def pm_force_mesh(ctx, mesh, out, stream=None):
    n = ctx.n
    _check(_lib.pm_force_mesh(ctx.h, _dev(mesh, torch.int64, n ** 3, "mesh"),
                              _dev(out, torch.float32, 3 * n ** 3, "out"), _stream(stream)))


def pm_force(ctx, x, acc, stream=None):
    _check(_lib.pm_force(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(acc, torch.float32, 3 * ctx.P, "acc"),
                         _stream(stream)))


def pm_step(ctx, x, p, a_force, a_kick0, a_kick1, a_drift1, stream=None):
    _check(_lib.pm_step(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(p, torch.float32, 3 * ctx.P, "p"),
                        a_force, a_kick0, a_kick1, a_drift1, _stream(stream)))


def pm_power(ctx, x, a_lo, a_hi, b_lo=None, b_hi=None, nbins=None, compensate=False, stream=None):
    b_lo = a_lo if b_lo is None else b_lo
    b_hi = a_hi if b_hi is None else b_hi
    nbins = ctx.n // 2 if nbins is None else nbins
    k, pk, nm = np.zeros(nbins), np.zeros(nbins), np.zeros(nbins)
    _check(_lib.pm_power(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), a_lo, a_hi, b_lo, b_hi, nbins,
                         int(bool(compensate)), k.ctypes.data, pk.ctypes.data, nm.ctypes.data, _stream(stream)))
    return k, pk, nm


def pm_trace_begin(ctx, capacity=4096):
    _check(_lib.pm_trace_begin(ctx.h, capacity))


def pm_trace_end(ctx, max_records=65536):
    """[(kernel name, milliseconds)] of the launches recorded since pm_trace_begin."""
    kind = np.zeros(max_records, dtype=np.int32)
    ms = np.zeros(max_records, dtype=np.float32)
    cnt = _i32()
    _check(_lib.pm_trace_end(ctx.h, max_records, kind.ctypes.data, ms.ctypes.data, C.byref(cnt)))
    m = min(cnt.value, max_records)
    return [(pm_kernel_name(int(kind[i])), float(ms[i])) for i in range(m)]


def pm_kernel_name(kind):
    return _lib.pm_kernel_name(kind).decode()


def pm_attach_ids(ctx, ids):
    """Attach a uint32 (stored as int32) device tensor of P ids, or None."""
    if ids is None:
        _check(_lib.pm_attach_ids(ctx.h, None))
        ctx._ids = None
        return
    _check(_lib.pm_attach_ids(ctx.h, _dev(ids, torch.int32, ctx.P, "ids")))
    ctx._ids = ids   # keep the tensor alive while attached


def pm_segment_tags(ctx, out=None, stream=None):
    out = torch.empty(ctx.P, dtype=torch.uint8, device=ctx.workspace.device) if out is None else out
    _check(_lib.pm_segment_tags(ctx.h, _dev(out, torch.uint8, ctx.P, "tags"), _stream(stream)))
    return out


def pm_reset_order(ctx):
    _check(_lib.pm_reset_order(ctx.h))


def pm_sync(ctx):
    _check(_lib.pm_sync(ctx.h))


# ---- reverse mode (device float32 arrays; cotangents accumulate in place)
def pm_density(ctx, x, delta, stream=None):
    n = ctx.n
    _check(_lib.pm_density(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"),
                           _dev(delta, torch.float32, n ** 3, "delta"), _stream(stream)))


def pm_density_vjp(ctx, x, dmesh, xbar, stream=None):
    n = ctx.n
    _check(_lib.pm_density_vjp(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"),
                               _dev(dmesh, torch.float32, n ** 3, "dmesh"),
                               _dev(xbar, torch.float32, 3 * ctx.P, "xbar"), _stream(stream)))


def pm_force_vjp(ctx, x, g, xbar, stream=None):
    _check(_lib.pm_force_vjp(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(g, torch.float32, 3 * ctx.P, "g"),
                             _dev(xbar, torch.float32, 3 * ctx.P, "xbar"), _stream(stream)))


def pm_step_vjp(ctx, x, a_force, a_kick0, a_kick1, a_drift1, xbar, pbar, stream=None):
    _check(_lib.pm_step_vjp(ctx.h, _dev(x, torch.float32, 3 * ctx.P, "x"), a_force, a_kick0, a_kick1, a_drift1,
                            _dev(xbar, torch.float32, 3 * ctx.P, "xbar"), _dev(pbar, torch.float32, 3 * ctx.P, "pbar"),
                            _stream(stream)))


def pm_ic_vjp(ctx, xbar, pbar, wbar, stream=None):
    nc = ctx.cfg.n_cdm ** 3
    _check(_lib.pm_ic_vjp(ctx.h, _dev(xbar, torch.float32, 3 * ctx.P, "xbar"),
                          _dev(pbar, torch.float32, 3 * ctx.P, "pbar"), _dev(wbar, torch.float32, nc, "wbar"),
                          _stream(stream)))


# ---- learned force correction (PM_FLAG_LEARNED contexts)
PM_FLAG_LEARNED = 8
PM_FLAG_NU_PSEUDO = 16


def pm_net_nparam():
    return int(_lib.pm_net_nparam())


def pm_learned_force(ctx, theta, a, x, acc, stream=None):
    _check(_lib.pm_learned_force(ctx.h, _dev(theta, torch.float32, pm_net_nparam(), "theta"), float(a),
                                 _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(acc, torch.float32, 3 * ctx.P, "acc"),
                                 _stream(stream)))


def pm_learned_step(ctx, theta, x, p, a_force, a_kick0, a_kick1, a_drift1, stream=None):
    _check(_lib.pm_learned_step(ctx.h, _dev(theta, torch.float32, pm_net_nparam(), "theta"),
                                _dev(x, torch.float32, 3 * ctx.P, "x"), _dev(p, torch.float32, 3 * ctx.P, "p"),
                                a_force, a_kick0, a_kick1, a_drift1, _stream(stream)))


def pm_learned_loss(ctx, theta, a, x, target, dtheta=None, stream=None):
    """Force-matching loss; dL/dtheta is accumulated into dtheta when given."""
    loss = C.c_double()
    _check(_lib.pm_learned_loss(ctx.h, _dev(theta, torch.float32, pm_net_nparam(), "theta"), float(a),
                                _dev(x, torch.float32, 3 * ctx.P, "x"),
                                _dev(target, torch.float32, 3 * ctx.P, "target"), C.byref(loss),
                                _dev(dtheta, torch.float32, pm_net_nparam(), "dtheta") if dtheta is not None else None,
                                _stream(stream)))
    return loss.value


def pm_adam(theta, m, v, g, lr, beta1, beta2, eps, t, stream=None):
    n = theta.numel()
    _check(_lib.pm_adam(_dev(theta, torch.float32, n, "theta"), _dev(m, torch.float32, n, "m"),
                        _dev(v, torch.float32, n, "v"), _dev(g, torch.float32, n, "g"), n, lr, beta1, beta2, eps,
                        int(t), _stream(stream)))


NET_NB = 256


def pm_net_table(theta, a, table=None, stream=None):
    """Radial filter table [256] (float32 device tensor) at scale factor a."""
    if table is None:
        table = torch.empty(NET_NB, dtype=torch.float32, device=theta.device)
    _check(_lib.pm_net_table(_dev(theta, torch.float32, pm_net_nparam(), "theta"), float(a),
                             _dev(table, torch.float32, NET_NB, "table"), _stream(stream)))
    return table


def pm_net_table_vjp(theta, a, tbar, dtheta, stream=None):
    """dtheta += tbar . d table / d theta (tbar float64 [256])."""
    _check(_lib.pm_net_table_vjp(_dev(theta, torch.float32, pm_net_nparam(), "theta"), float(a),
                                 _dev(tbar, torch.float64, NET_NB, "tbar"),
                                 _dev(dtheta, torch.float32, pm_net_nparam(), "dtheta"), _stream(stream)))


def pm_power_mesh(ctx, da, db, nbins, compensate=False, stream=None):
    """(k_mean, P(k), n_modes) of two density meshes on the context's mesh."""
    n = ctx.n
    k, pk, nm = np.zeros(nbins), np.zeros(nbins), np.zeros(nbins)
    _check(_lib.pm_power_mesh(ctx.h, _dev(da, torch.float32, n ** 3, "da"), _dev(db, torch.float32, n ** 3, "db"),
                              nbins, int(bool(compensate)), k.ctypes.data, pk.ctypes.data, nm.ctypes.data,
                              _stream(stream)))
    return k, pk, nm


def copy_calibration():
    """A plain device-to-device copy of exactly 1 GiB (reads 1 GiB, writes
    1 GiB): the reference against which the FETCH_SIZE and WRITE_SIZE
    counters of the library's kernels are scaled when a command runs under
    rocprofv3 --pmc."""
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
