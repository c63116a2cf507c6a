// C-ABI entry points of libpm: argument checking, workspace layout, and the
// orchestration of the device passes on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <mutex>
#include <new>

#include "pm_internal.h"

struct pm_ctx : pm::Ctx {};

namespace {

// Fixed device scratch of pm_paint_static, for callers that cannot allocate:
// the tile sort's counts / cursors and offsets for up to PM_STATIC_MAX_MESH^3
// meshes (8 keys per 16^3 tile), the scan's block sums, and the sorted
// position records of up to PM_STATIC_MAX_PARTICLES particles.  Each device
// holds its own copy for the life of the process; host code uses only the
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t align256c(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr int64_t STATIC_KEYS = 8LL * (PM_STATIC_MAX_MESH / pm::TILE) * (PM_STATIC_MAX_MESH / pm::TILE) *
                                (PM_STATIC_MAX_MESH / pm::TILE);
constexpr size_t STATIC_CNT = 0, STATIC_KOFF = align256c(4 * (STATIC_KEYS + 1)),
                 STATIC_BSUM = STATIC_KOFF + align256c(4 * (STATIC_KEYS + 1)),
                 STATIC_XS = STATIC_BSUM + align256c(4 * ((STATIC_KEYS + 1 + 2047) / 2048 + 1)),
                 STATIC_BYTES = STATIC_XS + 16 * (size_t)PM_STATIC_MAX_PARTICLES;
static __device__ __align__(256) char scratch[STATIC_BYTES];

std::mutex g_scratch_mu;
char *g_scratch_ptr[64] = {};

// This device's address of `scratch`, looked up once per device (with that
// device current).
hipError_t static_scratch_for_current_device(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

thread_local char g_err[512] = "no error";

pm_status fail(pm_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(PM_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Launch with optional event bracketing for per-kernel timing.
#define LAUNCH(kind, expr)                                                                      \
    do {                                                                                        \
        hipEvent_t b_ = nullptr;                                                                \
        if (c->tracing) HIPCHK(trace_open(c, kind, s, &b_));                                    \
        HIPCHK(expr);                                                                           \
        if (b_) HIPCHK(hipEventRecord(b_, s));                                                  \
    } while (0)

hipError_t trace_open(pm::Ctx *c, int kind, hipStream_t s, hipEvent_t *end)
{
    *end = nullptr;
    if (c->ev_used + 2 > c->ev_pool.size()) return hipSuccess;   // pool full: stop recording
    hipEvent_t a = c->ev_pool[c->ev_used], b = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    c->trace.push_back({kind, a, b});
    *end = b;
    return hipSuccess;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2i(int v)
{
    int r = 0;
    while ((1 << r) < v) r++;
    return r;
}

struct Layout {
    size_t q, f, tw, flag, partial, tables, segtab, xs, ps, tags, ids, koff, cnt, bsum, cnt_next, total;
    size_t net_phif, net_z1, net_a1, net_z2, net_a2, net_g1, net_g2, net_dpsi, net_dk, net_acc, net_table, net_tbar,
        net_red, net_wpk;
    int64_t nkeys;
};

void counts(const pm_config &c, int64_t *P, int64_t *nc, int64_t *nn, int *nseg);

bool sort_capable(const pm_config &c, int64_t P) { return c.n_mesh / pm::TILE >= 2 && P < (int64_t(1) << 31); }

Layout layout(const pm_config &c)
{
    const int64_t n = c.n_mesh, nhp = pm::half_pad(c.n_mesh);
    int64_t P, nc, nn;
    int nseg;
    counts(c, &P, &nc, &nn, &nseg);
    const int64_t nt = n / pm::TILE;
    Layout L;
    L.nkeys = sort_capable(c, P) ? 8 * nt * nt * nt : 0;
    size_t off = 0;
    L.q = off;
    off = align256(off + (size_t)(8 * n * n * n));
    L.f = off;
    // three components of N planes; the force solve's planes may be padded
    const size_t fbytes = (size_t)(3 * n * pm::force_plane((int)n) * 8);
    off = align256(off + fbytes);
    L.tw = off;
    off = align256(off + (size_t)(2 * n * 8));
    L.flag = off;
    off = align256(off + 256);
    L.partial = off;
    off = align256(off + (size_t)(pm::POWER_BLOCKS + 1) * 3 * pm::MAX_BINS * 8);
    L.tables = off;
    off = align256(off + (size_t)(3 * (2 * c.n_fib + 1) + 2 * c.n_shell + ((c.flags & PM_FLAG_NU_PSEUDO) ? 4097 : 0)) * 4);
    L.segtab = off;
    off = align256(off + (size_t)(2 * pm::MAX_SEG + 1) * 8);
    L.xs = L.ps = L.tags = L.ids = L.koff = L.cnt = L.bsum = L.cnt_next = 0;
    if (L.nkeys > 0) {
        // tile-sorted particle records and the tags survive the whole step
        L.xs = off;
        off = align256(off + (size_t)(16 * P));
        L.ps = off;
        off = align256(off + (size_t)(12 * P));
        L.tags = off;
        off = align256(off + (size_t)P);
        L.ids = off;
        off = align256(off + (size_t)(4 * P));
        L.koff = off;
        off = align256(off + (size_t)(4 * (L.nkeys + 1)));
        // counts of the next step's keys, written by the tile readout while it
        // reads the force region: a region of its own
        L.cnt_next = off;
        off = align256(off + (size_t)(4 * (L.nkeys + 1)));
        // sort scratch is dead before the FFT writes the force region: alias it there when it fits
        const size_t nb = (size_t)((L.nkeys + 1 + 2047) / 2048 + 1);
        const size_t scratch = align256(4 * (size_t)(L.nkeys + 1)) + align256(4 * nb);
        size_t s0 = L.f;
        if (scratch > fbytes) {
            s0 = off;
            off = align256(off + scratch);
        }
        L.cnt = s0;
        L.bsum = L.cnt + align256(4 * (size_t)(L.nkeys + 1));
    }
    L.net_phif = L.net_z1 = L.net_a1 = L.net_z2 = L.net_a2 = L.net_g1 = L.net_g2 = L.net_dpsi = L.net_dk = 0;
    L.net_acc = L.net_table = L.net_tbar = L.net_red = L.net_wpk = 0;
    if (c.flags & PM_FLAG_LEARNED) {
        const size_t M = (size_t)(n * n * n);
        auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
        L.net_phif = take((size_t)(n * n * 2 * nhp) * 4);
        L.net_z1 = take(M * pm::NET_C * 4);
        L.net_a1 = take(M * pm::NET_C * 2);
        L.net_z2 = take(M * pm::NET_C * 4);
        L.net_a2 = take(M * pm::NET_C * 2);
        L.net_g1 = take(M * pm::NET_C * 4);
        L.net_g2 = take(M * pm::NET_C * 4);
        L.net_dpsi = take(M * 4);
        L.net_dk = take((size_t)(n * n * nhp) * 8);
        L.net_acc = take((size_t)(3 * P) * 4);
        L.net_table = take(pm::NET_NB * 4);
        L.net_tbar = take(pm::NET_NB * 8);
        L.net_red = take(64);
        L.net_wpk = take(pm::NET_WPK_BYTES);
    }
    L.total = off;
    return L;
}

pm_status check_config(const pm_config *c)
{
    if (!c) return fail(PM_ERR_ARG, "config is NULL");
    if (!pow2(c->n_mesh) || c->n_mesh < 16 || c->n_mesh > 2048)
        return fail(PM_ERR_ARG, "n_mesh must be a power of two in [16, 2048], got %d", c->n_mesh);
    if (!pow2(c->n_cdm) || c->n_cdm < 8 || c->n_cdm > c->n_mesh)
        return fail(PM_ERR_ARG, "n_cdm must be a power of two in [8, n_mesh], got %d", c->n_cdm);
    if (c->n_sites < 0 || (c->n_sites > 0 && (!pow2(c->n_sites) || c->n_sites > c->n_cdm)))
        return fail(PM_ERR_ARG, "n_sites must be 0 or a power of two dividing n_cdm, got %d", c->n_sites);
    if (c->n_shell < 1 || c->n_shell > pm::MAX_SEG - 1)
        return fail(PM_ERR_ARG, "n_shell must be in [1, %d]", pm::MAX_SEG - 1);
    if (c->n_fib < 0 || c->n_fib > 1000) return fail(PM_ERR_ARG, "n_fib must be in [0, 1000]");
    if ((c->flags & PM_FLAG_NU_PSEUDO) && (c->n_sites < 1 || c->n_shell != 1 || c->n_fib != 0))
        return fail(PM_ERR_ARG, "PM_FLAG_NU_PSEUDO needs neutrino sites, n_shell = 1 and n_fib = 0");
    if (c->n_nu < 0 || c->n_nu > 3) return fail(PM_ERR_ARG, "n_nu must be in [0, 3]");
    if (c->shift < 16 || c->shift > 52) return fail(PM_ERR_ARG, "shift must be in [16, 52]");
    if (!(c->box > 0) || !(c->omega_m > 0) || !(c->h > 0) || !(c->a0 > 1.0 / 160.0) || !(c->a0 <= 1.0))
        return fail(PM_ERR_ARG, "box, omega_m, h must be positive and a0 in (1/160, 1]");
    if (!(c->T_cmb >= 0) || !(c->N_eff >= 0)) return fail(PM_ERR_ARG, "T_cmb and N_eff must be >= 0");
    double m1 = 0;
    for (int j = 0; j < c->n_nu; j++) {
        if (!(c->m_nu[j] >= 0)) return fail(PM_ERR_ARG, "neutrino masses must be >= 0");
        m1 = fmax(m1, c->m_nu[j]);
    }
    if (c->n_sites > 0 && !(m1 > 0))
        return fail(PM_ERR_ARG, "neutrino particles need a positive neutrino mass");
    double Mnu = 0;
    for (int j = 0; j < c->n_nu; j++) Mnu += c->m_nu[j];
    if (!(c->omega_m - Mnu / (93.14 * c->h * c->h) > 0)) return fail(PM_ERR_ARG, "omega_m below omega_nu");
    return PM_OK;
}

void counts(const pm_config &c, int64_t *P, int64_t *nc, int64_t *nn, int *nseg)
{
    *nc = (int64_t)c.n_cdm * c.n_cdm * c.n_cdm;
    *nn = (int64_t)c.n_sites * c.n_sites * c.n_sites * c.n_shell * (2 * c.n_fib + 1);
    *P = *nc + *nn;
    *nseg = c.n_sites > 0 ? 1 + c.n_shell : 1;
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// The guard bits of a flag word read back as a status.
static pm_status guard_status(int h, const char *which)
{
    if (h & pm::FLAG_NAN) return fail(PM_ERR_NAN, "a particle position or momentum became non-finite%s", which);
    if (h & pm::FLAG_OVERFLOW) return fail(PM_ERR_OVERFLOW, "a density cell left the fixed-point range%s", which);
    return PM_OK;
}

// PM_FLAG_DEFER_GUARDS: waits for the previous guarded call's flag copy (that
// call's end only) and returns its status.
static pm_status settle_guard(pm_ctx *c)
{
    if (!c->guard_pending) return PM_OK;
    c->guard_pending = false;
    HIPCHK(hipEventSynchronize(c->guard_ev[c->guard_slot]));
    return guard_status(c->guard_host[c->guard_slot], " (in the previous call)");
}

pm_status check_guards(pm_ctx *c, hipStream_t s)
{
    if (c->cfg.flags & PM_FLAG_NO_GUARDS) return PM_OK;
    if (c->cfg.flags & PM_FLAG_DEFER_GUARDS) {
        // this call's word goes to the other pinned slot and is cleared on the
        // device behind the copy, so each copy holds one call's bits; then the
        // previous call's copy, long done, is read
        const int slot = c->guard_slot ^ 1;
        HIPCHK(hipMemcpyAsync(c->guard_host + slot, c->ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        LAUNCH(pm::K_FILL, pm::launch_fill_i32(c->ws.flag, 1, s));
        HIPCHK(hipEventRecord(c->guard_ev[slot], s));
        const pm_status prev = settle_guard(c);
        c->guard_slot = slot;
        c->guard_pending = true;
        return prev;
    }
    // through the pinned word (free here: a deferred sort verification is
    // settled before any readout)
    HIPCHK(hipMemcpyAsync(c->verify_host, c->ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int h = *c->verify_host;
    if (h) {
        HIPCHK(hipMemsetAsync(c->ws.flag, 0, sizeof(int), s));
        HIPCHK(hipStreamSynchronize(s));
        return guard_status(h, "");
    }
    return PM_OK;
}

bool sorting_on(const pm_ctx *c) { return c->nkeys > 0 && !(c->cfg.flags & PM_FLAG_NO_SORT); }

// Paint segments [lo, hi) of x (in the context's current particle order)
// into `mesh` with global atomics; the caller zeroes the mesh.
pm_status paint_atomic(pm_ctx *c, const float *x, int lo, int hi, int64_t *mesh, hipStream_t s)
{
    if (c->permuted) {
        LAUNCH(pm::K_PAINT, pm::launch_paint_tagged(x, c->P, c->ws.tags, lo, hi, c->ws.quanta, c->n, mesh, s));
    } else {
        for (int g = lo; g < hi; g++)
            LAUNCH(pm::K_PAINT, pm::launch_paint(x, c->P, c->seg_off[g], c->seg_off[g + 1] - c->seg_off[g],
                                                 c->seg_q[g], c->n, mesh, s));
    }
    return PM_OK;
}

// Counting sort of (x, p, tags, ids) by tile key into the workspace records
// xs (position and tag), ps, ids_tmp and the key offsets koff.  p may be
// NULL.  The tag array itself keeps the caller's order until a readout
// writes the particles back in sorted order.
//
// When the last tile readout wrote x, it also counted the keys of the
// positions it wrote (cnt_next): the sort then skips its count pass, and a
// check after the scatter (every key's cursor must end at the next key's
// offset) confirms that the counts still describe x.  If the caller changed
// x in between, the check fails and the sort is redone from a fresh count
// (the scatter never writes past the record arrays).  The check waits for the
// stream, so it is used only when the end-of-call guards wait anyway.
// With `defer`, a verification of taken-over counts is left in flight (the
// flag word on its way to pinned host memory) and finish_sort settles it: the
// caller may queue work that writes only the workspace in between, which is
// redone when the counts were stale.
pm_status tile_sort(pm_ctx *c, const float *x, const float *p, hipStream_t s, bool defer = false)
{
    const int64_t K = c->nkeys;
    const uint8_t *tin = c->permuted ? c->ws.tags : nullptr;
    c->verify_pending = false;
    if (c->counts_ready && x == c->counts_x && !(c->cfg.flags & PM_FLAG_NO_GUARDS)) {
        LAUNCH(pm::K_SORT_SCAN, pm::launch_scan(c->ws.cnt_next, c->ws.koff, K + 1, c->ws.bsum, s, c->ws.cnt));
        LAUNCH(pm::K_SORT_SCATTER,
               pm::launch_sort_scatter(x, p, tin, c->P, c->nseg, c->ws.seg_off, c->n, c->ws.cnt, c->ws.xs,
                                       p ? c->ws.ps : nullptr, c->ids, c->ids ? c->ws.ids_tmp : nullptr, s));
        LAUNCH(pm::K_SORT_VERIFY, pm::launch_sort_verify(c->ws.cnt, c->ws.koff, K, c->ws.flag, s));
        if (defer) {
            HIPCHK(hipMemcpyAsync(c->verify_host, c->ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(c->verify_ev, s));
            c->verify_pending = true;
            return PM_OK;
        }
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, c->ws.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!(h & pm::FLAG_STALE)) return PM_OK;
        h &= ~pm::FLAG_STALE;
        HIPCHK(hipMemcpyAsync(c->ws.flag, &h, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        c->counts_ready = false;
    }
    LAUNCH(pm::K_FILL, pm::launch_fill_i32(c->ws.cnt, K + 1, s));
    LAUNCH(pm::K_SORT_COUNT, pm::launch_sort_count(x, c->P, c->n, c->ws.cnt, s));
    // koff <- exclusive scan of the counts; cnt <- the same, as cursors
    LAUNCH(pm::K_SORT_SCAN, pm::launch_scan(c->ws.cnt, c->ws.koff, K + 1, c->ws.bsum, s, c->ws.cnt));
    LAUNCH(pm::K_SORT_SCATTER,
           pm::launch_sort_scatter(x, p, tin, c->P, c->nseg, c->ws.seg_off, c->n, c->ws.cnt, c->ws.xs,
                                   p ? c->ws.ps : nullptr, c->ids, c->ids ? c->ws.ids_tmp : nullptr, s));
    return PM_OK;
}

// Settles a deferred verification.  Stale counts: the stale bit is cleared
// (with any guard bit that the work queued on the stale sort set) and the
// particles are sorted again from a fresh count; *redo tells the caller to
// queue that work again.  The flag value restored is the one read at the
// verification, so guard bits from before it survive.
pm_status finish_sort(pm_ctx *c, const float *x, const float *p, hipStream_t s, bool *redo)
{
    *redo = false;
    if (!c->verify_pending) return PM_OK;
    c->verify_pending = false;
    HIPCHK(hipEventSynchronize(c->verify_ev));
    int h = *c->verify_host;
    if (!(h & pm::FLAG_STALE)) return PM_OK;
    h &= ~pm::FLAG_STALE;
    HIPCHK(hipMemcpyAsync(c->ws.flag, &h, sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    c->counts_ready = false;
    *redo = true;
    return tile_sort(c, x, p, s);
}

// Paint every segment of x into the Q mesh (overwritten).
pm_status paint_all(pm_ctx *c, const float *x, hipStream_t s)
{
    const int64_t n = c->n;
    LAUNCH(pm::K_FILL, pm::launch_fill_i64(c->ws.q, n * n * n, s));
    return paint_atomic(c, x, 0, c->nseg, c->ws.q, s);
}

// From the int64 density at `src` (row stride n int64) to the three real
// force meshes in the F region (row stride 2 Nhp floats).  The forward
// spectrum is written into F0 (row stride Nhp, not a power of two, so strided
// passes do not camp on a few HBM channels) and the axis-0 pass works in
// place on it.
// With `delta` set, the source is instead the float32 density contrast [N]^3
// written by the tile paint (src unused).
pm_status solve(pm_ctx *c, const int64_t *src, hipStream_t s, const float *delta = nullptr)
{
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    float2 *F = c->ws.f;
    // component stride: N planes of force_plane(N) (N half_pad rows below the
    // padding threshold, which the row path below relies on)
    const int64_t plane = pm::force_plane(n), cs = n * plane;
    const double scale = ldexp(1.0, -c->cfg.shift);
    const double coef = 1.5 * c->cfg.omega_m / ((double)n2 * n);
    if (lg >= 8) {
        // axis 0 as 16 x N/16 (four-step): the 16-point pass rides on the row
        // transforms, the N/16-point pass on the gradient of the inverse
        // Laplacian; the spectrum stays digit-reversed along axis 0 in between
        if (delta)
            LAUNCH(pm::K_R2C_X0, pm::launch_r2c_x0_f32(lg, delta, n, F, (int)nhp, plane, c->ws.tw, s));
        else
            LAUNCH(pm::K_R2C_X0,
                   pm::launch_r2c_x0(lg, src, F, (int)nhp, plane, scale, -1.0, c->ws.tw, c->ws.flag, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, plane, n, ncb, c->ws.tw, s));
        // F0 <- k0 T, F1 <- T; the inverse column passes apply the k2 and
        // k1 factors: component 2 from F1 into F2 first, then 1 in place
        LAUNCH(pm::K_X0_GREEN, pm::launch_x0_green(lg, F, F, F + cs, plane, (int)nhp, coef, c->ws.tw, s));
        for (int d = 2; d >= 0; d--) {
            LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, d == 0 ? F : F + cs, nhp, plane, n, ncb, c->ws.tw, s,
                                                   d, F + d * cs));
            LAUNCH(pm::K_C2R_X0, pm::launch_c2r_x0(lg, F + d * cs, reinterpret_cast<float *>(F + d * cs), 2 * nhp,
                                                   2 * plane, (int)nhp, plane, c->ws.tw, s));
        }
        return PM_OK;
    }
    if (plane != n * nhp) return fail(PM_ERR_STATE, "padded planes on the row path");
    // axis 2: density contrast, real-to-complex rows
    if (delta)
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, delta, n, F, nhp, n2, c->ws.tw, s));
    else
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_i64(lg, src, n, F, nhp, n2, scale, -1.0, c->ws.tw, c->ws.flag, s));
    // axis 1
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
    // axis 0 forward, gradient of the inverse Laplacian, axis 0 inverses (in place on F0)
    LAUNCH(pm::K_AXIS0, pm::launch_axis0(lg, pm::MULT_FORCE, F, n * nhp, nhp, F, F + cs, F + 2 * cs, n * nhp, nhp,
                                         ncb, coef, nullptr, c->ws.tw, s));
    for (int d = 0; d < 3; d++) {
        LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F + d * cs, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F + d * cs, nhp, reinterpret_cast<float *>(F + d * cs), 2 * nhp,
                                              n2, c->ws.tw, s));
    }
    return PM_OK;
}

// Forward spectrum of a density painted into the int64 mesh `q` (in place,
// row stride n complex), contrast delta = Q scale - 1.
pm_status forward_density(pm_ctx *c, int64_t *q, double scale, hipStream_t s)
{
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    float2 *S = reinterpret_cast<float2 *>(q);
    LAUNCH(pm::K_R2C, pm::launch_r2c_rows_i64(lg, q, n, S, n, n2, scale, -1.0, c->ws.tw, c->ws.flag, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, S, n, n2, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_AXIS0, pm::launch_axis0(lg, pm::MULT_NONE, S, n2, n, S, nullptr, nullptr, n2, n, ncb, 0.0, nullptr, c->ws.tw, s));
    return PM_OK;
}

// xbar += gscale (d acc / d x)^T g for the differentiable model (exact
// segment masses, cloud-in-cell weights): the readout-derivative term from the
// force meshes at x, then the cotangents painted with the readout weights,
// the transpose of the gradient of the inverse Laplacian (minus itself) and
// the paint-derivative term.  Natural-order transforms on the F region.
pm_status force_vjp(pm_ctx *c, const float *x, const float *g, double gscale, float *xbar, hipStream_t s)
{
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n, cs = n2 * nhp;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    float2 *F = c->ws.f;
    float *Fr = reinterpret_cast<float *>(F);
    // With the tile-sort workspace, the particles and their cotangents are
    // first sorted into the record arrays (the caller's order is untouched;
    // the count scratch aliases the F region, written only by the solve that
    // follows): the density and each cotangent component are then painted
    // by tile.  Otherwise both use global atomics.  Either way the integers
    // are the same.
    const bool tiles = c->nkeys > 0;
    pm_status st = PM_OK;
    if (tiles) {
        const int64_t K = c->nkeys;
        LAUNCH(pm::K_FILL, pm::launch_fill_i32(c->ws.cnt, K + 1, s));
        LAUNCH(pm::K_SORT_COUNT, pm::launch_sort_count(x, c->P, c->n, c->ws.cnt, s));
        LAUNCH(pm::K_SORT_SCAN, pm::launch_scan(c->ws.cnt, c->ws.koff, K + 1, c->ws.bsum, s, c->ws.cnt));
        LAUNCH(pm::K_SORT_SCATTER,
               pm::launch_sort_scatter(x, g, c->permuted ? c->ws.tags : nullptr, c->P, c->nseg, c->ws.seg_off, c->n,
                                       c->ws.cnt, c->ws.xs, c->ws.ps, nullptr, nullptr, s));
        LAUNCH(pm::K_PAINT, pm::launch_paint_tiles(c->ws.xs, c->ws.koff, c->ws.quanta, c->nseg, 0, c->nseg, c->n,
                                                   c->ws.q, s));
    } else {
        st = paint_all(c, x, s);
    }
    if (st == PM_OK) st = solve(c, c->ws.q, s);
    if (st != PM_OK) return st;
    // cotangent paint in fixed point, one component at a time through Q (free
    // after the solve): a unit of 1/S with S a power of two such that even all
    // particles' largest cotangent in one cell stays below 2^62, so the mesh
    // and the gradient are bit-reproducible
    unsigned *gmax = reinterpret_cast<unsigned *>(c->ws.flag) + 8;
    int *unused_flag = c->ws.flag + 9;
    LAUNCH(pm::K_FILL, pm::launch_fill_i32(reinterpret_cast<int *>(gmax), 1, s));
    LAUNCH(pm::K_ADJOINT, pm::launch_absmax(g, 3 * c->P, (float)gscale, gmax, s));
    unsigned mbits = 0;
    HIPCHK(hipMemcpyAsync(&mbits, gmax, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float gm;
    memcpy(&gm, &mbits, sizeof gm);
    if (!std::isfinite(gm)) return fail(PM_ERR_NAN, "a cotangent is not finite");
    const double S = gm > 0 ? ldexp(1.0, 61 - (int)ceil(log2((double)c->P * (double)gm))) : 1.0;
    // a non-finite cotangent is reported before xbar is touched
    const int64_t fp = pm::force_plane(n);   // the force meshes' plane stride
    LAUNCH(pm::K_ADJOINT,
           pm::launch_readout_grad3(x, c->P, g, (float)gscale, Fr, 2 * nhp, 2 * fp, 2 * n * fp, n, xbar, s));
    for (int d = 0; d < 3; d++) {
        float2 *Fd = F + d * cs;
        if (tiles) {
            LAUNCH(pm::K_ADJOINT, pm::launch_paint_q1_tiles(c->ws.xs, c->ws.ps, d, c->ws.koff, (float)gscale, S, n,
                                                            c->ws.q, s));
        } else {
            LAUNCH(pm::K_FILL, pm::launch_fill_i64(c->ws.q, (int64_t)n * n * n, s));
            LAUNCH(pm::K_ADJOINT, pm::launch_paint_q1(x, c->P, g + d * c->P, (float)gscale, S, n, c->ws.q, s));
        }
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_i64(lg, c->ws.q, n, Fd, nhp, n2, 1.0 / S, 0.0, c->ws.tw, unused_flag, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, n * nhp, nhp, n, ncb, c->ws.tw, s));
    }
    const double coef = 1.5 * c->cfg.omega_m / ((double)n2 * n);
    LAUNCH(pm::K_ADJOINT, pm::launch_green_adj(F, nhp, cs, n, coef, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F, nhp, Fr, 2 * nhp, n2, c->ws.tw, s));
    LAUNCH(pm::K_ADJOINT, pm::launch_density_grad(x, c->P, Fr, 2 * nhp, n, c->nseg, c->ws.seg_off,
                                                  c->permuted ? c->ws.tags : nullptr, c->ws.quanta,
                                                  (float)ldexp(1.0, -c->cfg.shift), 1.0f, xbar, s));
    return PM_OK;
}

// Learned force meshes into the F region (real rows of stride 2 Nhp) from
// the density in Q: natural-order transforms.  With keep, the filtered
// potential, every CNN pre-activation and activation and the density
// spectrum stay in the workspace for the reverse mode; without, the fused
// inference CNN keeps only the filtered potential and a2.
// With `delta` (inference only), the density comes as the float32 contrast
// the tile paint writes instead of the int64 mesh in Q.
pm_status learned_solve(pm_ctx *c, const float *th, double a, bool keep, hipStream_t s, const float *delta = nullptr)
{
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n, cs = n2 * nhp, rs = 2 * nhp;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    const double M = (double)n2 * n;
    float2 *F = c->ws.f;
    const double qs = ldexp(1.0, -c->cfg.shift);
    const bool two_pass = !keep && lg >= 8;
    if (!two_pass) {
        // natural-order forward transform of the density
        if (delta)
            LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, delta, n, F, nhp, n2, c->ws.tw, s));
        else
            LAUNCH(pm::K_R2C, pm::launch_r2c_rows_i64(lg, c->ws.q, n, F, nhp, n2, qs, -1.0, c->ws.tw, c->ws.flag, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
    }
    if (keep) LAUNCH(pm::K_COPY, hipMemcpyAsync(c->ws.net_dk, F, (size_t)cs * 8, hipMemcpyDeviceToDevice, s));
    LAUNCH(pm::K_NET, pm::launch_mlp_fwd(th, a, c->ws.net_table, s));
    float *Fr = reinterpret_cast<float *>(F);
    if (keep) {
        // the reverse mode needs phi_f in real space and every pre-activation
        // and activation of the CNN
        LAUNCH(pm::K_NET, pm::launch_spec_filter(F, F + cs, nhp, n, c->ws.net_table, -1.5 * c->cfg.omega_m / M, s));
        LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F + cs, n * nhp, nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F + cs, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F + cs, nhp, c->ws.net_phif, rs, n2, c->ws.tw, s));
        LAUNCH(pm::K_NET, pm::launch_cnn_fwd(c->ws.q, qs, n, th, c->ws.net_z1, c->ws.net_a1, c->ws.net_z2,
                                             c->ws.net_a2, c->ws.net_dpsi, s));
        LAUNCH(pm::K_NET, pm::launch_combine(c->ws.net_phif, c->ws.net_dpsi, rs, n, Fr, s));
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, Fr, rs, F, nhp, n2, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_NET, pm::launch_grad3(F, nhp, cs, n, 1.0 / M, false, s));
    } else if (two_pass) {
        // inference on the two-pass transforms of the plain solve: rows with
        // the first axis-0 digit and axis 1 for the density and for the CNN
        // output (real rows in field 2, transformed in place); one pass B
        // takes both, forms T = i (g gr S_d - S_c / M) and writes k0 T and T;
        // the inverse passes are the plain solve's
        const int64_t plane = (int64_t)n * nhp;
        if (delta)
            LAUNCH(pm::K_R2C_X0, pm::launch_r2c_x0_f32(lg, delta, n, F, (int)nhp, plane, c->ws.tw, s));
        else
            LAUNCH(pm::K_R2C_X0, pm::launch_r2c_x0(lg, c->ws.q, F, (int)nhp, plane, qs, -1.0, c->ws.tw, c->ws.flag, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
        float *F2r = reinterpret_cast<float *>(F + 2 * cs);
        LAUNCH(pm::K_NET, pm::launch_cnn_inf(c->ws.q, qs, delta, nullptr, rs, n, th, c->ws.net_wpk, c->ws.net_a2,
                                             F2r, s));
        LAUNCH(pm::K_R2C_X0, pm::launch_r2c_x0_f32(lg, F2r, rs, F + 2 * cs, (int)nhp, plane, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F + 2 * cs, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_NET, pm::launch_x0_learned(lg, F, F + 2 * cs, F, F + cs, plane, (int)nhp, 1.5 * c->cfg.omega_m / M,
                                                1.0 / M, c->ws.net_table, c->ws.tw, s));
        for (int d = 2; d >= 0; d--) {
            LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, d == 0 ? F : F + cs, nhp, n * nhp, n, ncb, c->ws.tw, s,
                                                   d, F + d * cs));
            LAUNCH(pm::K_C2R_X0, pm::launch_c2r_x0(lg, F + d * cs, reinterpret_cast<float *>(F + d * cs), 2 * nhp,
                                                   2 * plane, (int)nhp, plane, c->ws.tw, s));
        }
        return PM_OK;
    } else {
        // inference: the filtered potential never leaves spectral space.  The
        // forward transform of phi_f = F^-1[g G delta(k)] / M is g G delta(k)
        // itself, so field 1 holds it with coefficient -1.5 Omega_m (no 1/M);
        // the CNN output goes to field 2 as real rows and is transformed
        // there; the force is -i k (field 1 + field 2) / M.
        LAUNCH(pm::K_NET, pm::launch_spec_filter(F, F + cs, nhp, n, c->ws.net_table, -1.5 * c->cfg.omega_m, s));
        float *F2r = reinterpret_cast<float *>(F + 2 * cs);
        LAUNCH(pm::K_NET, pm::launch_cnn_inf(c->ws.q, qs, delta, nullptr, rs, n, th, c->ws.net_wpk, c->ws.net_a2,
                                             F2r, s));
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, F2r, rs, F + 2 * cs, nhp, n2, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F + 2 * cs, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F + 2 * cs, n * nhp, nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_NET, pm::launch_grad3_sum(F, nhp, cs, n, 1.0 / M, s));
    }
    for (int d = 0; d < 3; d++) {
        float2 *Fd = F + d * cs;
        LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, Fd, n * nhp, nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, Fd, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, Fd, nhp, reinterpret_cast<float *>(Fd), rs, n2, c->ws.tw, s));
    }
    return PM_OK;
}

pm_status learned_ready(pm_ctx *c)
{
    if (!(c->cfg.flags & PM_FLAG_LEARNED)) return fail(PM_ERR_STATE, "configure the context with PM_FLAG_LEARNED");
    if (c->n < 16) return fail(PM_ERR_STATE, "the learned correction needs N >= 16");
    return PM_OK;
}

}  // namespace

extern "C" {

const char *pm_last_error(void) { return g_err; }

pm_status pm_sizes(const pm_config *cfg, int64_t *n_particles, int32_t *n_segments, size_t *workspace_bytes)
{
    pm_status st = check_config(cfg);
    if (st != PM_OK) return st;
    int64_t P, nc, nn;
    int nseg;
    counts(*cfg, &P, &nc, &nn, &nseg);
    if (n_particles) *n_particles = P;
    if (n_segments) *n_segments = nseg;
    if (workspace_bytes) *workspace_bytes = layout(*cfg).total;
    return PM_OK;
}

pm_status pm_init(const pm_config *cfg, void *workspace, size_t workspace_bytes, void *stream, pm_ctx **out)
{
    pm_status st = check_config(cfg);
    if (st != PM_OK) return st;
    if (!out) return fail(PM_ERR_ARG, "out is NULL");
    const Layout L = layout(*cfg);
    if (!workspace) return fail(PM_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(PM_ERR_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(PM_ERR_SIZE, "workspace of %zu bytes is below the %zu required", workspace_bytes, L.total);
    pm_ctx *c = new (std::nothrow) pm_ctx();
    if (!c) return fail(PM_ERR_ARG, "out of host memory");
    c->cfg = *cfg;
    c->n = cfg->n_mesh;
    c->logn = ilog2i(cfg->n_mesh);
    int nseg;
    counts(*cfg, &c->P, &c->nc, &c->nn, &nseg);
    pm::cosmo_setup(*c);
    char *b = reinterpret_cast<char *>(workspace);
    c->ws.base = b;
    c->ws.bytes = workspace_bytes;
    c->ws.q = reinterpret_cast<int64_t *>(b + L.q);
    c->ws.f = reinterpret_cast<float2 *>(b + L.f);
    c->ws.tw = reinterpret_cast<float2 *>(b + L.tw);
    c->ws.flag = reinterpret_cast<int *>(b + L.flag);
    c->ws.partial = reinterpret_cast<double *>(b + L.partial);
    c->ws.tables = reinterpret_cast<float *>(b + L.tables);
    c->ws.seg_off = reinterpret_cast<int64_t *>(b + L.segtab);
    c->ws.quanta = c->ws.seg_off + (pm::MAX_SEG + 1);
    c->nkeys = L.nkeys;
    if (L.nkeys > 0) {
        c->ws.xs = reinterpret_cast<float4 *>(b + L.xs);
        c->ws.ps = reinterpret_cast<pm::Mom3 *>(b + L.ps);
        c->ws.tags = reinterpret_cast<uint8_t *>(b + L.tags);
        c->ws.ids_tmp = reinterpret_cast<uint32_t *>(b + L.ids);
        c->ws.koff = reinterpret_cast<int *>(b + L.koff);
        c->ws.cnt = reinterpret_cast<int *>(b + L.cnt);
        c->ws.bsum = reinterpret_cast<int *>(b + L.bsum);
        c->ws.cnt_next = reinterpret_cast<int *>(b + L.cnt_next);
    }
    if (cfg->flags & PM_FLAG_LEARNED) {
        c->ws.net_phif = reinterpret_cast<float *>(b + L.net_phif);
        c->ws.net_z1 = reinterpret_cast<float *>(b + L.net_z1);
        c->ws.net_a1 = reinterpret_cast<uint16_t *>(b + L.net_a1);
        c->ws.net_z2 = reinterpret_cast<float *>(b + L.net_z2);
        c->ws.net_a2 = reinterpret_cast<uint16_t *>(b + L.net_a2);
        c->ws.net_g1 = reinterpret_cast<float *>(b + L.net_g1);
        c->ws.net_g2 = reinterpret_cast<float *>(b + L.net_g2);
        c->ws.net_dpsi = reinterpret_cast<float *>(b + L.net_dpsi);
        c->ws.net_dk = reinterpret_cast<float2 *>(b + L.net_dk);
        c->ws.net_acc = reinterpret_cast<float *>(b + L.net_acc);
        c->ws.net_table = reinterpret_cast<float *>(b + L.net_table);
        c->ws.net_tbar = reinterpret_cast<double *>(b + L.net_tbar);
        c->ws.net_red = reinterpret_cast<double *>(b + L.net_red);
        c->ws.net_wpk = reinterpret_cast<uint16_t *>(b + L.net_wpk);
    }
    // twiddles for every power-of-two length L <= N: tw[L + m] = exp(-2 pi i m / L)
    const int n = c->n;
    c->tw_host.assign(2 * (size_t)n, make_float2(0.f, 0.f));
    for (int Ln = 1; Ln <= n; Ln *= 2)
        for (int m = 0; m < Ln; m++) {
            const double ang = -2.0 * M_PI * (double)m / (double)Ln;
            c->tw_host[Ln + m] = make_float2((float)cos(ang), (float)sin(ang));
        }
    hipStream_t s = S(stream);
    std::vector<float> tables(c->dirs);
    if (c->nn > 0) {
        const double spacing = (double)n / cfg->n_sites;   // mesh cells between sites
        const double qlast = c->q_shell.back();
        const double pth_unit = c->kT_nu / c->m1 * 299792.458 / 100.0 * n / cfg->box;
        for (int s2 = 0; s2 < cfg->n_shell; s2++) tables.push_back((float)(0.4 * spacing * c->q_shell[s2] / qlast));
        for (int s2 = 0; s2 < cfg->n_shell; s2++) tables.push_back((float)(c->q_shell[s2] * pth_unit));
        for (double v : c->q_cdf) tables.push_back((float)v);   // pseudo-random sampling only
    }
    hipError_t e = hipMemcpyAsync(c->ws.tw, c->tw_host.data(), sizeof(float2) * c->tw_host.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !tables.empty())
        e = hipMemcpyAsync(c->ws.tables, tables.data(), sizeof(float) * tables.size(), hipMemcpyHostToDevice, s);
    c->segtab_host.assign(2 * pm::MAX_SEG + 1, 0);
    for (int g = 0; g <= c->nseg; g++) c->segtab_host[g] = c->seg_off[g];
    for (int g = 0; g < c->nseg; g++) c->segtab_host[pm::MAX_SEG + 1 + g] = c->seg_q[g];
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws.seg_off, c->segtab_host.data(), sizeof(int64_t) * c->segtab_host.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws.flag, 0, 256, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete c;
        return fail(PM_ERR_DEVICE, "uploading tables: %s", hipGetErrorString(e));
    }
    e = static_scratch_for_current_device(&c->static_scratch);
    if (e != hipSuccess) {
        delete c;
        return fail(PM_ERR_DEVICE, "address of the static scratch array: %s", hipGetErrorString(e));
    }
    e = hipHostMalloc(reinterpret_cast<void **>(&c->verify_host), sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->verify_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->guard_host), 2 * sizeof(int), hipHostMallocDefault);
    for (int k = 0; k < 2 && e == hipSuccess; k++) e = hipEventCreateWithFlags(&c->guard_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        pm_free(c);
        return fail(PM_ERR_DEVICE, "pinned flag copy: %s", hipGetErrorString(e));
    }
    *out = c;
    return PM_OK;
}

void pm_free(pm_ctx *ctx)
{
    if (!ctx) return;
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    // a flag copy queued into the pinned words may still be in flight
    if (ctx->verify_ev) {
        (void)hipEventSynchronize(ctx->verify_ev);
        (void)hipEventDestroy(ctx->verify_ev);
    }
    for (hipEvent_t e : ctx->guard_ev)
        if (e) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
    if (ctx->verify_host) (void)hipHostFree(ctx->verify_host);
    if (ctx->guard_host) (void)hipHostFree(ctx->guard_host);
    delete ctx;
}

static const char *kKernelNames[pm::K_COUNT] = {
    "fill",      "paint",        "r2c_rows",     "cols_fwd",   "axis0",      "cols_inv",   "c2r_rows",
    "readout_kick_drift", "readout", "power_bin", "power_reduce", "ic_particles", "copy", "sort_count",
    "sort_scan", "sort_scatter", "x0_green", "r2c_x0", "c2r_x0", "adjoint", "net", "sort_verify"};

const char *pm_kernel_name(int32_t kind)
{
    return (kind >= 0 && kind < pm::K_COUNT) ? kKernelNames[kind] : "unknown";
}

pm_status pm_trace_begin(pm_ctx *c, int32_t capacity)
{
    if (!c || capacity < 1 || capacity > (1 << 20)) return fail(PM_ERR_ARG, "capacity must be in [1, 2^20]");
    while ((int64_t)c->ev_pool.size() < 2 * (int64_t)capacity) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    c->ev_used = 0;
    c->trace.clear();
    c->tracing = true;
    return PM_OK;
}

pm_status pm_trace_end(pm_ctx *c, int32_t max, int32_t *kind, float *ms, int32_t *count)
{
    if (!c || max < 0 || (max > 0 && (!kind || !ms)) || !count) return fail(PM_ERR_ARG, "bad trace arguments");
    if (!c->tracing) return fail(PM_ERR_STATE, "no trace in progress");
    c->tracing = false;
    *count = (int32_t)c->trace.size();
    for (size_t i = 0; i < c->trace.size(); i++) {
        const pm::TraceRec &r = c->trace[i];
        HIPCHK(hipEventSynchronize(r.b));
        if ((int32_t)i < max) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            kind[i] = r.kind;
            ms[i] = t;
        }
    }
    c->trace.clear();
    c->ev_used = 0;
    return PM_OK;
}

pm_status pm_segments(const pm_ctx *c, int64_t *offsets, double *mass, int64_t *quantum)
{
    if (!c) return fail(PM_ERR_ARG, "ctx is NULL");
    for (int g = 0; g < c->nseg; g++) {
        if (offsets) offsets[g] = c->seg_off[g];
        if (mass) mass[g] = c->seg_mass[g];
        if (quantum) quantum[g] = c->seg_q[g];
    }
    if (offsets) offsets[c->nseg] = c->seg_off[c->nseg];
    return PM_OK;
}

pm_status pm_shells(const pm_ctx *c, double *edges, double *q_shell, double *m_shell)
{
    if (!c) return fail(PM_ERR_ARG, "ctx is NULL");
    if (c->q_shell.empty()) return fail(PM_ERR_STATE, "configuration has no neutrino particles");
    const int ns = c->cfg.n_shell;
    for (int s = 0; s < ns; s++) {
        if (q_shell) q_shell[s] = c->q_shell[s];
        if (m_shell) m_shell[s] = c->m_shell[s];
    }
    if (edges)
        for (int s = 0; s <= ns; s++) edges[s] = c->edges[s];
    return PM_OK;
}

pm_status pm_growth(const pm_ctx *c, int32_t n, const double *a, double *D, double *G)
{
    if (!c || n < 0 || (n > 0 && (!a || !D || !G))) return fail(PM_ERR_ARG, "bad growth arguments");
    for (int i = 0; i < n; i++) {
        if (!(a[i] >= 1.0 / 160.0) || !(a[i] <= 2.0)) return fail(PM_ERR_ARG, "a out of [1/160, 2]");
        D[i] = pm::growth_D(*c, a[i]);
        G[i] = pm::growth_G(*c, a[i]);
    }
    return PM_OK;
}

pm_status pm_kdk_factors(const pm_ctx *c, double a_force, double a_kick0, double a_kick1, double a_drift1,
                         double *kick, double *drift)
{
    if (!c || !kick || !drift) return fail(PM_ERR_ARG, "bad factor arguments");
    const double a[4] = {a_force, a_kick0, a_kick1, a_drift1};
    for (double v : a)
        if (!(v >= 1.0 / 160.0) || !(v <= 2.0)) return fail(PM_ERR_ARG, "scale factor out of [1/160, 2]");
    const double Df = pm::growth_D(*c, a_force);
    *kick = (pm::growth_G(*c, a_kick1) - pm::growth_G(*c, a_kick0)) / (1.5 * c->cfg.omega_m * Df);
    *drift = (pm::growth_D(*c, a_drift1) - Df) / pm::growth_G(*c, a_kick1);
    return PM_OK;
}

static pm_status ic_impl(pm_ctx *c, const float *white, const float *u, float *x, float *p, void *stream)
{
    c->permuted = false;
    c->counts_ready = false;
    hipStream_t s = S(stream);
    const pm_config &g = c->cfg;
    const int nic = g.n_cdm, lg = ilog2i(nic), n = c->n;
    const int64_t nhp = pm::half_pad(nic), n2 = (int64_t)nic * nic;
    const int ncb = (int)(pm::half_cols(nic) / pm::TILE_W);
    float2 *S0 = reinterpret_cast<float2 *>(c->ws.q);
    float2 *F = c->ws.f;
    const int64_t cs = n2 * nhp;
    // white-noise spectrum (rows, then axis 1); axis 0 is done per output
    LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, white, nic, S0, nic, n2, c->ws.tw, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, S0, nic, n2, nic, ncb, c->ws.tw, s));
    const double a0 = g.a0;
    const double D0 = pm::growth_D(*c, a0), D1 = pm::growth_D(*c, 1.0), G0 = pm::growth_G(*c, a0);
    pm::IcParams ip{};
    ip.amp_over_vcell = pm::pk_amplitude(*c) * (D0 / D1) * (D0 / D1) / pow(g.box / nic, 3);
    ip.box = g.box;
    ip.omh = g.omega_m * g.h;
    ip.n_s = g.n_s;
    ip.kfs = 0;
    ip.half_cell = 0;
    ip.scale = ((double)n / g.box) / ((double)n2 * nic);
    const double vfac = G0 / D0;
    for (int pass = 0; pass < (c->nn > 0 ? 2 : 1); pass++) {
        if (pass == 1) {
            ip.kfs = 0.82 * sqrt(c->omega_L + g.omega_m / (a0 * a0 * a0)) * a0 * a0 * c->m1;
            ip.half_cell = 0.5 * g.box / nic;
        }
        LAUNCH(pm::K_AXIS0, pm::launch_axis0(lg, pm::MULT_IC, S0, n2, nic, F, F + cs, F + 2 * cs, nic * nhp, nhp, ncb, 0.0, &ip,
                                c->ws.tw, s));
        for (int d = 0; d < 3; d++) {
            LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F + d * cs, nhp, nic * nhp, nic, ncb, c->ws.tw, s));
            LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F + d * cs, nhp, reinterpret_cast<float *>(F + d * cs), 2 * nhp, n2,
                                       c->ws.tw, s));
        }
        if (pass == 0)
            LAUNCH(pm::K_IC_PARTICLES, pm::launch_ic_cdm(F, nhp, cs, nic, n, vfac, x, p, c->P, s));
        else if (u) {
            const double pth_unit = c->kT_nu / c->m1 * 299792.458 / 100.0 * n / g.box;
            const float *cdf = c->ws.tables + 3 + 2;   // after one direction, one radius, one speed
            LAUNCH(pm::K_IC_PARTICLES,
                   pm::launch_ic_nu_pseudo(F, nhp, cs, nic, n, g.n_sites, cdf, (int)c->q_cdf.size() - 1, c->q_cdf_h,
                                           pth_unit, vfac, u, x, p, c->P, c->nc, s));
        } else
            LAUNCH(pm::K_IC_PARTICLES, pm::launch_ic_nu(F, nhp, cs, nic, n, g.n_sites, 2 * g.n_fib + 1, g.n_shell, c->ws.tables, vfac,
                                    (g.flags & PM_FLAG_NO_FLIP) ? 0 : 1, x, p, c->P, c->nc, s));
    }
    return PM_OK;
}

pm_status pm_ic(pm_ctx *c, const float *white, float *x, float *p, void *stream)
{
    if (!c || !white || !x || !p) return fail(PM_ERR_ARG, "NULL argument to pm_ic");
    if (c->cfg.flags & PM_FLAG_NU_PSEUDO)
        return fail(PM_ERR_STATE, "a PM_FLAG_NU_PSEUDO context takes its initial conditions from pm_ic_pseudo");
    return ic_impl(c, white, nullptr, x, p, stream);
}

pm_status pm_ic_pseudo(pm_ctx *c, const float *white, const float *u, float *x, float *p, void *stream)
{
    if (!c || !white || !u || !x || !p) return fail(PM_ERR_ARG, "NULL argument to pm_ic_pseudo");
    if (!(c->cfg.flags & PM_FLAG_NU_PSEUDO) || c->q_cdf.size() < 2)
        return fail(PM_ERR_STATE, "pm_ic_pseudo needs a context configured with PM_FLAG_NU_PSEUDO");
    return ic_impl(c, white, u, x, p, stream);
}

pm_status pm_paint_q(pm_ctx *c, const float *x, int64_t stride, int64_t first, int64_t count, int64_t quantum,
                     int64_t *mesh_q, void *stream)
{
    if (!c || !x || !mesh_q) return fail(PM_ERR_ARG, "NULL argument to pm_paint_q");
    if (first < 0 || count < 0 || first + count > stride) return fail(PM_ERR_ARG, "particle range outside stride");
    hipStream_t s = S(stream);
    LAUNCH(pm::K_PAINT, pm::launch_paint(x, stride, first, count, quantum, c->n, mesh_q, s));
    return PM_OK;
}

pm_status pm_paint(pm_ctx *c, const float *x, int32_t seg_lo, int32_t seg_hi, int64_t *mesh_q, void *stream)
{
    if (!c || !x || !mesh_q) return fail(PM_ERR_ARG, "NULL argument to pm_paint");
    if (seg_lo < 0 || seg_hi > c->nseg || seg_lo > seg_hi) return fail(PM_ERR_ARG, "bad segment range");
    hipStream_t s = S(stream);
    if (seg_lo == seg_hi) return PM_OK;
    if (sorting_on(c) && mesh_q != c->ws.q) {
        // tile sort into the workspace copies, tile paint into Q, add into the caller's mesh
        pm_status st = tile_sort(c, x, nullptr, s);
        if (st != PM_OK) return st;
        const int64_t n = c->n;
        LAUNCH(pm::K_PAINT, pm::launch_paint_tiles(c->ws.xs, c->ws.koff, c->ws.quanta, c->nseg, seg_lo, seg_hi,
                                                   c->n, c->ws.q, s));
        LAUNCH(pm::K_COPY, pm::launch_add_i64(c->ws.q, mesh_q, n * n * n, s));
        return PM_OK;
    }
    return paint_atomic(c, x, seg_lo, seg_hi, mesh_q, s);
}

pm_status pm_paint_static(pm_ctx *c, const float *x, int32_t seg_lo, int32_t seg_hi, int64_t *mesh_q, void *stream)
{
    if (!c || !x || !mesh_q) return fail(PM_ERR_ARG, "NULL argument to pm_paint_static");
    if (seg_lo < 0 || seg_hi > c->nseg || seg_lo > seg_hi) return fail(PM_ERR_ARG, "bad segment range");
    if (c->nkeys == 0) return fail(PM_ERR_STATE, "pm_paint_static needs a configuration that can tile-sort (N >= 32)");
    if (c->n > PM_STATIC_MAX_MESH || c->P > PM_STATIC_MAX_PARTICLES)
        return fail(PM_ERR_SIZE, "pm_paint_static takes meshes up to %d^3 and up to %d particles (got %d^3, %lld)",
                    PM_STATIC_MAX_MESH, PM_STATIC_MAX_PARTICLES, c->n, (long long)c->P);
    if (!c->static_scratch) return fail(PM_ERR_STATE, "no static scratch address for this context");
    hipStream_t s = S(stream);
    if (seg_lo == seg_hi) return PM_OK;
    const int64_t K = c->nkeys;
    int *cnt = reinterpret_cast<int *>(c->static_scratch + STATIC_CNT);
    int *koff = reinterpret_cast<int *>(c->static_scratch + STATIC_KOFF);
    int *bsum = reinterpret_cast<int *>(c->static_scratch + STATIC_BSUM);
    float4 *xs = reinterpret_cast<float4 *>(c->static_scratch + STATIC_XS);
    // the counts start at zero (a fill kernel, which a graph capture may hold)
    LAUNCH(pm::K_FILL, pm::launch_fill_i32(cnt, K + 1, s));
    LAUNCH(pm::K_SORT_COUNT, pm::launch_sort_count(x, c->P, c->n, cnt, s));
    LAUNCH(pm::K_SORT_SCAN, pm::launch_scan(cnt, koff, K + 1, bsum, s, cnt));
    LAUNCH(pm::K_SORT_SCATTER, pm::launch_sort_scatter(x, nullptr, c->permuted ? c->ws.tags : nullptr, c->P, c->nseg,
                                                       c->ws.seg_off, c->n, cnt, xs, nullptr, nullptr, nullptr, s));
    LAUNCH(pm::K_PAINT, pm::launch_paint_tiles_add(xs, koff, c->ws.quanta, c->nseg, seg_lo, seg_hi, c->n, mesh_q, s));
    return PM_OK;
}

pm_status pm_fft_r2c(pm_ctx *c, const float *real, float *out, void *stream)
{
    if (!c || !real || !out) return fail(PM_ERR_ARG, "NULL argument to pm_fft_r2c");
    hipStream_t s = S(stream);
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    float2 *S0 = reinterpret_cast<float2 *>(c->ws.q);
    LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, real, n, S0, n, n2, c->ws.tw, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, S0, n, n2, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, S0, n2, n, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COPY, pm::launch_copy_half(S0, n, n, reinterpret_cast<float2 *>(out), s));
    return PM_OK;
}

pm_status pm_fft_c2r(pm_ctx *c, const float *spec, float *real, void *stream)
{
    if (!c || !spec || !real) return fail(PM_ERR_ARG, "NULL argument to pm_fft_c2r");
    hipStream_t s = S(stream);
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    float2 *F = c->ws.f;
    LAUNCH(pm::K_COPY, pm::launch_load_half(reinterpret_cast<const float2 *>(spec), n, F, nhp, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F, nhp, reinterpret_cast<float *>(F), 2 * nhp, n2, c->ws.tw, s));
    LAUNCH(pm::K_COPY, pm::launch_copy_real(reinterpret_cast<const float *>(F), 2 * nhp, 2 * n * nhp, n, real, s));
    return PM_OK;
}

pm_status pm_force_mesh(pm_ctx *c, const int64_t *mesh_q, float *out, void *stream)
{
    if (!c || !mesh_q || !out) return fail(PM_ERR_ARG, "NULL argument to pm_force_mesh");
    hipStream_t s = S(stream);
    pm_status st = solve(c, mesh_q, s);
    if (st != PM_OK) return st;
    const int64_t n = c->n, nhp = pm::half_pad(c->n), fp = pm::force_plane(c->n), cs = n * fp;
    for (int d = 0; d < 3; d++)
        LAUNCH(pm::K_COPY, pm::launch_copy_real(reinterpret_cast<const float *>(c->ws.f + d * cs), 2 * nhp, 2 * fp,
                                                c->n, out + d * n * n * n, s));
    return check_guards(c, s);
}

pm_status pm_force(pm_ctx *c, const float *x, float *acc, void *stream)
{
    if (!c || !x || !acc) return fail(PM_ERR_ARG, "NULL argument to pm_force");
    hipStream_t s = S(stream);
    pm_status st = paint_all(c, x, s);
    if (st == PM_OK) st = solve(c, c->ws.q, s);
    if (st != PM_OK) return st;
    const int64_t n = c->n, nhp = pm::half_pad(c->n), fp = pm::force_plane(c->n);
    LAUNCH(pm::K_READOUT, pm::launch_readout(x, c->P, c->ws.f, nhp, fp, n * fp, c->n, acc, s));
    return check_guards(c, s);
}

pm_status pm_step(pm_ctx *c, float *x, float *p, double a_force, double a_kick0, double a_kick1, double a_drift1,
                  void *stream)
{
    if (!c || !x || !p) return fail(PM_ERR_ARG, "NULL argument to pm_step");
    double kick, drift;
    pm_status st = pm_kdk_factors(c, a_force, a_kick0, a_kick1, a_drift1, &kick, &drift);
    if (st != PM_OK) return st;
    hipStream_t s = S(stream);
    const int64_t n = c->n, nhp = pm::half_pad(c->n), fp = pm::force_plane(c->n);
    if (sorting_on(c)) {
        // sort by tile, paint tile by tile, solve, read out tile by tile into
        // the caller's arrays, which then hold the particles in sorted order
        // the tile paint stores each cell's exact int64 sum as its float32
        // density contrast, the value the transform would form from it
        // the paint and the solve write only the workspace, so they are queued
        // before a deferred check of taken-over counts and redone if stale
        st = tile_sort(c, x, p, s, true);
        if (st != PM_OK) return st;
        float *delta = reinterpret_cast<float *>(c->ws.q);
        for (bool redo = true; redo;) {
            LAUNCH(pm::K_PAINT, pm::launch_paint_tiles_delta(c->ws.xs, c->ws.koff, c->ws.quanta, c->nseg, c->n,
                                                             ldexp(1.0, -c->cfg.shift), -1.0, delta, c->ws.flag, s));
            st = solve(c, nullptr, s, delta);
            if (st == PM_OK) st = finish_sort(c, x, p, s, &redo);
            if (st != PM_OK) return st;
        }
        int *cnt_next = (c->cfg.flags & PM_FLAG_NO_GUARDS) ? nullptr : c->ws.cnt_next;
        if (cnt_next) LAUNCH(pm::K_FILL, pm::launch_fill_i32(cnt_next, c->nkeys + 1, s));
        LAUNCH(pm::K_READOUT_KD,
               pm::launch_readout_kd_tiles(c->ws.xs, c->ws.ps, c->P, c->ws.koff, c->ws.f, nhp, fp, n * fp, c->n,
                                           (float)kick, (float)drift, x, p, c->ws.tags, c->ws.ids_tmp, c->ids,
                                           c->ws.flag, cnt_next, s));
        c->permuted = true;
        c->counts_ready = cnt_next != nullptr;
        c->counts_x = x;
        return check_guards(c, s);
    }
    st = paint_all(c, x, s);
    if (st == PM_OK) st = solve(c, c->ws.q, s);
    if (st != PM_OK) return st;
    LAUNCH(pm::K_READOUT_KD, pm::launch_readout_kick_drift(x, p, c->P, c->ws.f, nhp, fp, n * fp, c->n, (float)kick,
                                                           (float)drift, c->ws.flag, s));
    return check_guards(c, s);
}

pm_status pm_attach_ids(pm_ctx *c, uint32_t *ids)
{
    if (!c) return fail(PM_ERR_ARG, "ctx is NULL");
    if (ids && c->nkeys == 0) return fail(PM_ERR_STATE, "ids need a configuration that supports tile sorting");
    c->ids = ids;
    return PM_OK;
}

pm_status pm_segment_tags(pm_ctx *c, uint8_t *tags, void *stream)
{
    if (!c || !tags) return fail(PM_ERR_ARG, "NULL argument to pm_segment_tags");
    hipStream_t s = S(stream);
    if (c->permuted)
        LAUNCH(pm::K_COPY, hipMemcpyAsync(tags, c->ws.tags, (size_t)c->P, hipMemcpyDeviceToDevice, s));
    else
        LAUNCH(pm::K_COPY, pm::launch_tags_canonical(tags, c->P, c->nseg, c->ws.seg_off, s));
    return PM_OK;
}

pm_status pm_sync(pm_ctx *c)
{
    if (!c) return fail(PM_ERR_ARG, "ctx is NULL");
    return settle_guard(c);
}

pm_status pm_reset_order(pm_ctx *c)
{
    if (!c) return fail(PM_ERR_ARG, "ctx is NULL");
    c->permuted = false;
    c->counts_ready = false;
    return PM_OK;
}

pm_status pm_power(pm_ctx *c, const float *x, int32_t a_lo, int32_t a_hi, int32_t b_lo, int32_t b_hi,
                   int32_t nbins, int32_t compensate, double *k_mean, double *pk, double *n_modes, void *stream)
{
    if (!c || !x || !k_mean || !pk || !n_modes) return fail(PM_ERR_ARG, "NULL argument to pm_power");
    if (nbins < 1 || nbins > pm::MAX_BINS) return fail(PM_ERR_ARG, "nbins must be in [1, %d]", pm::MAX_BINS);
    if (a_lo < 0 || a_hi > c->nseg || a_lo >= a_hi || b_lo < 0 || b_hi > c->nseg || b_lo >= b_hi)
        return fail(PM_ERR_ARG, "bad segment ranges");
    hipStream_t s = S(stream);
    const int n = c->n;
    const int64_t M = (int64_t)n * n * n;
    auto scale_of = [&](int lo, int hi) {
        double tot = 0;
        for (int g = lo; g < hi; g++) tot += (double)(c->seg_off[g + 1] - c->seg_off[g]) * (double)c->seg_q[g];
        return (double)M / tot;
    };
    LAUNCH(pm::K_FILL, pm::launch_fill_i64(c->ws.q, M, s));
    pm_status st = paint_atomic(c, x, a_lo, a_hi, c->ws.q, s);
    if (st == PM_OK) st = forward_density(c, c->ws.q, scale_of(a_lo, a_hi), s);
    if (st != PM_OK) return st;
    const float2 *A = reinterpret_cast<const float2 *>(c->ws.q), *B = A;
    if (a_lo != b_lo || a_hi != b_hi) {
        int64_t *qb = reinterpret_cast<int64_t *>(c->ws.f);
        LAUNCH(pm::K_FILL, pm::launch_fill_i64(qb, M, s));
        st = paint_atomic(c, x, b_lo, b_hi, qb, s);
        if (st == PM_OK) st = forward_density(c, qb, scale_of(b_lo, b_hi), s);
        if (st != PM_OK) return st;
        B = reinterpret_cast<const float2 *>(qb);
    }
    const double V = pow(c->cfg.box, 3);
    double *out = c->ws.partial + (size_t)pm::POWER_BLOCKS * 3 * pm::MAX_BINS;
    LAUNCH(pm::K_POWER_BIN, pm::launch_power_bin(A, B, n, n, nbins, compensate, V / ((double)M * (double)M), 2.0 * M_PI / c->cfg.box,
                                c->ws.partial, s));
    LAUNCH(pm::K_POWER_REDUCE, pm::launch_power_reduce(c->ws.partial, nbins, out, s));
    std::vector<double> h(3 * (size_t)nbins);
    HIPCHK(hipMemcpyAsync(h.data(), out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < nbins; b++) {
        const double w = h[3 * b + 2];
        n_modes[b] = w;
        pk[b] = w > 0 ? h[3 * b] / w : 0.0;
        k_mean[b] = w > 0 ? h[3 * b + 1] / w : 0.0;
    }
    return check_guards(c, s);
}

pm_status pm_power_mesh(pm_ctx *c, const float *da, const float *db, int32_t nbins, int32_t compensate,
                        double *k_mean, double *pk, double *n_modes, void *stream)
{
    if (!c || !da || !db || !k_mean || !pk || !n_modes) return fail(PM_ERR_ARG, "NULL argument to pm_power_mesh");
    if (nbins < 1 || nbins > pm::MAX_BINS) return fail(PM_ERR_ARG, "nbins must be in [1, %d]", pm::MAX_BINS);
    hipStream_t s = S(stream);
    const int n = c->n, lg = c->logn;
    const int64_t M = (int64_t)n * n * n, n2 = (int64_t)n * n, nhp = pm::half_pad(n);
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    auto spectrum = [&](const float *d, float2 *S) -> pm_status {
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, d, n, S, n, n2, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, S, n, n2, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_AXIS0, pm::launch_axis0(lg, pm::MULT_NONE, S, n2, n, S, nullptr, nullptr, n2, n, ncb, 0.0,
                                             nullptr, c->ws.tw, s));
        return PM_OK;
    };
    float2 *A = reinterpret_cast<float2 *>(c->ws.q), *B = A;
    pm_status st = spectrum(da, A);
    if (st == PM_OK && db != da) {
        B = reinterpret_cast<float2 *>(c->ws.f);
        st = spectrum(db, B);
    }
    if (st != PM_OK) return st;
    const double V = pow(c->cfg.box, 3);
    double *out = c->ws.partial + (size_t)pm::POWER_BLOCKS * 3 * pm::MAX_BINS;
    LAUNCH(pm::K_POWER_BIN, pm::launch_power_bin(A, B, n, n, nbins, compensate, V / ((double)M * (double)M),
                                                 2.0 * M_PI / c->cfg.box, c->ws.partial, s));
    LAUNCH(pm::K_POWER_REDUCE, pm::launch_power_reduce(c->ws.partial, nbins, out, s));
    std::vector<double> h(3 * (size_t)nbins);
    HIPCHK(hipMemcpyAsync(h.data(), out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < nbins; b++) {
        const double w = h[3 * b + 2];
        n_modes[b] = w;
        pk[b] = w > 0 ? h[3 * b] / w : 0.0;
        k_mean[b] = w > 0 ? h[3 * b + 1] / w : 0.0;
    }
    return PM_OK;
}

// ---- reverse mode

pm_status pm_density(pm_ctx *c, const float *x, float *delta, void *stream)
{
    if (!c || !x || !delta) return fail(PM_ERR_ARG, "NULL argument to pm_density");
    hipStream_t s = S(stream);
    pm_status st = paint_all(c, x, s);
    if (st != PM_OK) return st;
    const int64_t n = c->n;
    LAUNCH(pm::K_COPY, pm::launch_q_to_delta(c->ws.q, n * n * n, ldexp(1.0, -c->cfg.shift), delta, s));
    return check_guards(c, s);
}

pm_status pm_density_vjp(pm_ctx *c, const float *x, const float *dmesh, float *xbar, void *stream)
{
    if (!c || !x || !dmesh || !xbar) return fail(PM_ERR_ARG, "NULL argument to pm_density_vjp");
    hipStream_t s = S(stream);
    LAUNCH(pm::K_ADJOINT, pm::launch_density_grad(x, c->P, dmesh, c->n, c->n, c->nseg, c->ws.seg_off,
                                                  c->permuted ? c->ws.tags : nullptr, c->ws.quanta,
                                                  (float)ldexp(1.0, -c->cfg.shift), 1.0f, xbar, s));
    return PM_OK;
}

pm_status pm_force_vjp(pm_ctx *c, const float *x, const float *g, float *xbar, void *stream)
{
    if (!c || !x || !g || !xbar) return fail(PM_ERR_ARG, "NULL argument to pm_force_vjp");
    hipStream_t s = S(stream);
    pm_status st = force_vjp(c, x, g, 1.0, xbar, s);
    return st == PM_OK ? check_guards(c, s) : st;
}

pm_status pm_step_vjp(pm_ctx *c, const float *x, double a_force, double a_kick0, double a_kick1, double a_drift1,
                      float *xbar, float *pbar, void *stream)
{
    if (!c || !x || !xbar || !pbar) return fail(PM_ERR_ARG, "NULL argument to pm_step_vjp");
    if (sorting_on(c))
        return fail(PM_ERR_STATE, "the reverse mode needs PM_FLAG_NO_SORT: particles must keep their order");
    double kick, drift;
    pm_status st = pm_kdk_factors(c, a_force, a_kick0, a_kick1, a_drift1, &kick, &drift);
    if (st != PM_OK) return st;
    hipStream_t s = S(stream);
    // x' = x + drift p', p' = p + kick F(x):  pbar += drift xbar, then
    // xbar += kick (dF/dx)^T pbar
    LAUNCH(pm::K_ADJOINT, pm::launch_axpy(pbar, xbar, (float)drift, 3 * c->P, s));
    st = force_vjp(c, x, pbar, kick, xbar, s);
    return st == PM_OK ? check_guards(c, s) : st;
}

pm_status pm_ic_vjp(pm_ctx *c, const float *xbar, const float *pbar, float *wbar, void *stream)
{
    if (!c || !xbar || !pbar || !wbar) return fail(PM_ERR_ARG, "NULL argument to pm_ic_vjp");
    if (c->permuted) return fail(PM_ERR_STATE, "cotangents must be in the canonical particle order");
    hipStream_t s = S(stream);
    const pm_config &g = c->cfg;
    const int nic = g.n_cdm, lg = ilog2i(nic), n = c->n;
    const int64_t nhp = pm::half_pad(nic), n2 = (int64_t)nic * nic, cs = n2 * nhp;
    const int ncb = (int)(pm::half_cols(nic) / pm::TILE_W);
    float2 *F = c->ws.f;
    float *Fr = reinterpret_cast<float *>(F);
    float2 *A = reinterpret_cast<float2 *>(c->ws.q);
    const double a0 = g.a0;
    const double D0 = pm::growth_D(*c, a0), D1 = pm::growth_D(*c, 1.0), G0 = pm::growth_G(*c, a0);
    pm::IcParams ip{};
    ip.amp_over_vcell = pm::pk_amplitude(*c) * (D0 / D1) * (D0 / D1) / pow(g.box / nic, 3);
    ip.box = g.box;
    ip.omh = g.omega_m * g.h;
    ip.n_s = g.n_s;
    ip.scale = ((double)n / g.box) / ((double)n2 * nic);
    const float vfac = (float)(G0 / D0);
    for (int pass = 0; pass < (c->nn > 0 ? 2 : 1); pass++) {
        if (pass == 1) {
            ip.kfs = 0.82 * sqrt(c->omega_L + g.omega_m / (a0 * a0 * a0)) * a0 * a0 * c->m1;
            ip.half_cell = 0.5 * g.box / nic;
        }
        LAUNCH(pm::K_FILL, pm::launch_fill_i64(reinterpret_cast<int64_t *>(F), 3 * cs, s));
        if (pass == 0)
            LAUNCH(pm::K_ADJOINT, pm::launch_ic_adj_gather_cdm(xbar, pbar, c->P, nic, vfac, Fr, 2 * nhp, 2 * cs, s));
        else
            LAUNCH(pm::K_ADJOINT, pm::launch_ic_adj_gather_nu(xbar, pbar, c->P, c->nc, nic, g.n_sites, 2 * g.n_fib + 1,
                                                              g.n_shell, vfac, Fr, 2 * nhp, 2 * cs, s));
        for (int d = 0; d < 3; d++) {
            float2 *Fd = F + d * cs;
            LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, reinterpret_cast<float *>(Fd), 2 * nhp, Fd, nhp, n2,
                                                      c->ws.tw, s));
            LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, nhp, nic * nhp, nic, ncb, c->ws.tw, s));
            LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, nic * nhp, nhp, nic, ncb, c->ws.tw, s));
        }
        LAUNCH(pm::K_ADJOINT, pm::launch_ic_adj_mult(F, nhp, cs, nic, &ip, A, pass > 0, s));
    }
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, A, nic * nhp, nhp, nic, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, A, nhp, nic * nhp, nic, ncb, c->ws.tw, s));
    LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, A, nhp, reinterpret_cast<float *>(A), 2 * nhp, n2, c->ws.tw, s));
    LAUNCH(pm::K_COPY, pm::launch_copy_real(reinterpret_cast<const float *>(A), 2 * nhp, 2 * nic * nhp, nic, wbar, s));
    return PM_OK;
}

// ---- learned force correction

int32_t pm_net_nparam(void) { return pm::NET_NPARAM; }

pm_status pm_learned_force(pm_ctx *c, const float *th, double a, const float *x, float *acc, void *stream)
{
    if (!c || !th || !x || !acc) return fail(PM_ERR_ARG, "NULL argument to pm_learned_force");
    pm_status st = learned_ready(c);
    if (st != PM_OK) return st;
    hipStream_t s = S(stream);
    st = paint_all(c, x, s);
    if (st == PM_OK) st = learned_solve(c, th, a, false, s);
    if (st != PM_OK) return st;
    const int64_t n = c->n, nhp = pm::half_pad(c->n);
    LAUNCH(pm::K_READOUT, pm::launch_readout(x, c->P, c->ws.f, nhp, n * nhp, n * n * nhp, c->n, acc, s));
    return check_guards(c, s);
}

pm_status pm_learned_step(pm_ctx *c, const float *th, float *x, float *p, double a_force, double a_kick0,
                          double a_kick1, double a_drift1, void *stream)
{
    if (!c || !th || !x || !p) return fail(PM_ERR_ARG, "NULL argument to pm_learned_step");
    pm_status st = learned_ready(c);
    if (st != PM_OK) return st;
    double kick, drift;
    st = pm_kdk_factors(c, a_force, a_kick0, a_kick1, a_drift1, &kick, &drift);
    if (st != PM_OK) return st;
    hipStream_t s = S(stream);
    const int64_t n = c->n, nhp = pm::half_pad(c->n);
    if (sorting_on(c)) {
        // as pm_step: tile sort, tile paint (float32 density contrast),
        // (learned) solve, tile readout counting the next step's keys
        st = tile_sort(c, x, p, s, true);
        if (st != PM_OK) return st;
        float *delta = reinterpret_cast<float *>(c->ws.q);
        for (bool redo = true; redo;) {
            LAUNCH(pm::K_PAINT, pm::launch_paint_tiles_delta(c->ws.xs, c->ws.koff, c->ws.quanta, c->nseg, c->n,
                                                             ldexp(1.0, -c->cfg.shift), -1.0, delta, c->ws.flag, s));
            st = learned_solve(c, th, a_force, false, s, delta);
            if (st == PM_OK) st = finish_sort(c, x, p, s, &redo);
            if (st != PM_OK) return st;
        }
        int *cnt_next = (c->cfg.flags & PM_FLAG_NO_GUARDS) ? nullptr : c->ws.cnt_next;
        if (cnt_next) LAUNCH(pm::K_FILL, pm::launch_fill_i32(cnt_next, c->nkeys + 1, s));
        LAUNCH(pm::K_READOUT_KD,
               pm::launch_readout_kd_tiles(c->ws.xs, c->ws.ps, c->P, c->ws.koff, c->ws.f, nhp, n * nhp, n * n * nhp, c->n,
                                           (float)kick, (float)drift, x, p, c->ws.tags, c->ws.ids_tmp, c->ids,
                                           c->ws.flag, cnt_next, s));
        c->permuted = true;
        c->counts_ready = cnt_next != nullptr;
        c->counts_x = x;
        return check_guards(c, s);
    }
    st = paint_all(c, x, s);
    if (st == PM_OK) st = learned_solve(c, th, a_force, false, s);
    if (st != PM_OK) return st;
    LAUNCH(pm::K_READOUT_KD, pm::launch_readout_kick_drift(x, p, c->P, c->ws.f, nhp, n * nhp, n * n * nhp, c->n, (float)kick,
                                                           (float)drift, c->ws.flag, s));
    return check_guards(c, s);
}

pm_status pm_learned_loss(pm_ctx *c, const float *th, double a, const float *x, const float *target, double *loss,
                          float *dth, void *stream)
{
    if (!c || !th || !x || !target || !loss) return fail(PM_ERR_ARG, "NULL argument to pm_learned_loss");
    pm_status st = learned_ready(c);
    if (st != PM_OK) return st;
    hipStream_t s = S(stream);
    const int n = c->n, lg = c->logn;
    const int64_t nhp = pm::half_pad(n), n2 = (int64_t)n * n, cs = n2 * nhp, rs = 2 * nhp;
    const int ncb = (int)(pm::half_cols(n) / pm::TILE_W);
    const double M = (double)n2 * n;
    float2 *F = c->ws.f;
    float *Fr = reinterpret_cast<float *>(F);
    st = paint_all(c, x, s);
    if (st == PM_OK) st = learned_solve(c, th, a, dth != nullptr, s);
    if (st != PM_OK) return st;
    LAUNCH(pm::K_READOUT, pm::launch_readout(x, c->P, F, nhp, n * nhp, cs, n, c->ws.net_acc, s));
    LAUNCH(pm::K_NET, pm::launch_force_loss(c->ws.net_acc, target, 3 * c->P, c->ws.net_red, s));
    double red[2];
    if (hipMemcpyAsync(red, c->ws.net_red, sizeof(red), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(PM_ERR_DEVICE, "reading the loss back failed");
    if (!(red[1] > 0)) return fail(PM_ERR_ARG, "the target forces are all zero");
    *loss = red[0] / red[1];
    if (!dth) return check_guards(c, s);
    // readout transpose, gradient transpose, CNN and filter reverse mode
    LAUNCH(pm::K_FILL, pm::launch_fill_i64(reinterpret_cast<int64_t *>(F), 3 * cs, s));
    LAUNCH(pm::K_ADJOINT, pm::launch_paint_vec3(x, c->P, c->ws.net_acc, (float)(2.0 / red[1]), Fr, rs, 2 * cs, n, s));
    for (int d = 0; d < 3; d++) {
        float2 *Fd = F + d * cs;
        LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, reinterpret_cast<float *>(Fd), rs, Fd, nhp, n2, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, nhp, n * nhp, n, ncb, c->ws.tw, s));
        LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, Fd, n * nhp, nhp, n, ncb, c->ws.tw, s));
    }
    LAUNCH(pm::K_NET, pm::launch_grad3(F, nhp, cs, n, 1.0 / M, true, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_INV, pm::launch_cols(lg, true, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_C2R, pm::launch_c2r_rows(lg, F, nhp, Fr, rs, n2, c->ws.tw, s));
    LAUNCH(pm::K_NET, pm::launch_cnn_bwd(c->ws.q, ldexp(1.0, -c->cfg.shift), Fr, rs, n, th, c->ws.net_z1,
                                         c->ws.net_a1, c->ws.net_z2, c->ws.net_a2, c->ws.net_g1, c->ws.net_g2, dth, s));
    LAUNCH(pm::K_R2C, pm::launch_r2c_rows_f32(lg, Fr, rs, F, nhp, n2, c->ws.tw, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, nhp, n * nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_COLS_FWD, pm::launch_cols(lg, false, F, n * nhp, nhp, n, ncb, c->ws.tw, s));
    LAUNCH(pm::K_NET, pm::launch_spec_filter_bwd(c->ws.net_dk, F, nhp, n, -1.5 * c->cfg.omega_m / M,
                                                 c->ws.net_tbar, s));
    LAUNCH(pm::K_NET, pm::launch_mlp_bwd(th, a, c->ws.net_tbar, dth, s));
    return check_guards(c, s);
}

pm_status pm_net_table(const float *th, double a, float *table, void *stream)
{
    if (!th || !table) return fail(PM_ERR_ARG, "NULL argument to pm_net_table");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    if (pm::launch_mlp_fwd(th, a, table, s) != hipSuccess) return fail(PM_ERR_DEVICE, "filter table launch failed");
    return PM_OK;
}

pm_status pm_net_table_vjp(const float *th, double a, const double *tbar, float *dth, void *stream)
{
    if (!th || !tbar || !dth) return fail(PM_ERR_ARG, "NULL argument to pm_net_table_vjp");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    if (pm::launch_mlp_bwd(th, a, tbar, dth, s) != hipSuccess)
        return fail(PM_ERR_DEVICE, "filter table reverse-mode launch failed");
    return PM_OK;
}

pm_status pm_adam(float *th, float *m, float *v, const float *g, int64_t n, double lr, double beta1, double beta2,
                  double eps, int32_t t, void *stream)
{
    if (!th || !m || !v || !g || n < 0 || t < 1) return fail(PM_ERR_ARG, "bad argument to pm_adam");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    if (pm::launch_adam(th, m, v, g, n, lr, beta1, beta2, eps, t, s) != hipSuccess)
        return fail(PM_ERR_DEVICE, "adam launch failed");
    return PM_OK;
}

}  // extern "C"
