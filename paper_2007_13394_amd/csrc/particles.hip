// Particle-side kernels: force readout fused with the FastPM kick and drift,
// Zel'dovich initial conditions, power-spectrum binning and layout copies.
#include "pm_internal.h"

namespace pm {
namespace {

inline unsigned grid_for(int64_t n, int block, int64_t cap = 65536LL * 16)
{
    int64_t b = (n + block - 1) / block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

__global__ void k_fill_i64(int64_t *p, int64_t count)
{
    const int64_t n2 = count / 2;
    longlong2 *q = reinterpret_cast<longlong2 *>(p);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        q[i] = make_longlong2(0, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (count & 1)) p[count - 1] = 0;
}

// Cloud-in-cell interpolation of the three force meshes at u (float32
// weights; the force field is float32).
__device__ __forceinline__ void cic_gather(const float *__restrict__ F, int64_t rs, int64_t ps, int64_t cs, int n,
                                           float u0, float u1, float u2, float out[3])
{
    const int mask = n - 1;
    const float f0 = floorf(u0), f1 = floorf(u1), f2 = floorf(u2);
    const float d0 = u0 - f0, d1 = u1 - f1, d2 = u2 - f2;
    const int a0 = (int)f0 & mask, a1 = (int)f1 & mask, a2 = (int)f2 & mask;
    const int b0 = (a0 + 1) & mask, b1 = (a1 + 1) & mask, b2 = (a2 + 1) & mask;
    const float w0[2] = {1.f - d0, d0}, w1[2] = {1.f - d1, d1}, w2[2] = {1.f - d2, d2};
    const int i0[2] = {a0, b0}, i1[2] = {a1, b1}, i2[2] = {a2, b2};
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int64_t row = (int64_t)i0[a] * ps + (int64_t)i1[b] * rs;
            const float wab = w0[a] * w1[b];
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const int64_t idx = row + i2[c];
                const float w = wab * w2[c];
                s0 += w * F[idx];
                s1 += w * F[cs + idx];
                s2 += w * F[2 * cs + idx];
            }
        }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
}

__device__ __forceinline__ float wrapf(float v, float nf)
{
    float t = fmodf(v, nf);
    if (t < 0.f) t += nf;
    if (t >= nf) t -= nf;
    return t;
}

__global__ __launch_bounds__(256) void k_readout(const float *__restrict__ x, int64_t P, const float *__restrict__ F,
                                                 int64_t rs, int64_t ps, int64_t cs, int n, float *acc)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        float f[3];
        cic_gather(F, rs, ps, cs, n, x[i], x[P + i], x[2 * P + i], f);
        acc[i] = f[0];
        acc[P + i] = f[1];
        acc[2 * P + i] = f[2];
    }
}

// p += kick F(x); x += drift p; x wrapped into [0, n).
__global__ __launch_bounds__(256) void k_readout_kick_drift(float *x, float *p, int64_t P,
                                                            const float *__restrict__ F, int64_t rs, int64_t ps,
                                                            int64_t cs, int n, float kick, float drift, int *flag)
{
    const float nf = (float)n;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const float u0 = x[i], u1 = x[P + i], u2 = x[2 * P + i];
        float f[3];
        cic_gather(F, rs, ps, cs, n, u0, u1, u2, f);
        const float p0 = p[i] + kick * f[0];
        const float p1 = p[P + i] + kick * f[1];
        const float p2 = p[2 * P + i] + kick * f[2];
        const float x0 = wrapf(u0 + drift * p0, nf);
        const float x1 = wrapf(u1 + drift * p1, nf);
        const float x2 = wrapf(u2 + drift * p2, nf);
        bad |= !(isfinite(p0) && isfinite(p1) && isfinite(p2) && isfinite(x0) && isfinite(x1) && isfinite(x2));
        p[i] = p0;
        p[P + i] = p1;
        p[2 * P + i] = p2;
        x[i] = x0;
        x[P + i] = x1;
        x[2 * P + i] = x2;
    }
    if (bad) atomicOr(flag, FLAG_NAN);
}

// One workgroup per TILE^3 tile: the three force meshes over the tile and its
// +1 halo are staged in LDS, then every particle sorted into the tile is read
// out from LDS, kicked and drifted; results go to the caller's arrays at the
// particle's sorted index (with its id, when ids are attached).
// 1024 threads: the 77 KB LDS tile allows two workgroups per CU, so the
// workgroup itself must carry enough waves to hide memory latency (the LDS
// fill has four loads per thread; 1024 threads took the C3 readout from 46.0
// to 45.3 ms against 512).  The
// particle range and each thread's first particle are loaded before the LDS
// fill, and the next particle is loaded before the current one is stored.
constexpr int READOUT_T = 1024;

__global__ __launch_bounds__(READOUT_T) void k_readout_kd_tiles(const float4 *__restrict__ xs,
                                                                const Mom3 *__restrict__ ps, int64_t P,
                                                                const int *__restrict__ koff,
                                                                const float *__restrict__ F, int64_t rs,
                                                                int64_t fps, int64_t cs, int n, float kick, float drift,
                                                                float *x, float *p, uint8_t *tags,
                                                                const uint32_t *__restrict__ ids_tmp,
                                                                uint32_t *ids, int *flag, int *cnt_next)
{
    // LDS: the (TILE + 1)^3 cells of the tile and its +1 halo, the three
    // force components of a cell interleaved in one float4
    constexpr int H = TILE + 1, ROWS = H * H, NB = 27 * 8;
    __shared__ float4 fl[ROWS * H];
    __shared__ int hist[NB];   // next-step key counts of this tile and its neighbours (cnt_next)
    const int nt = n / TILE, mask = n - 1;
    // workgroups walk the tiles in row-major order (consecutive tiles share
    // rows of the force mesh); particle ranges are looked up by Morton index
    const int bt = xcd_tile(blockIdx.x, gridDim.x);
    const int t0 = bt / (nt * nt), t1 = (bt / nt) % nt, t2 = bt % nt;
    const int t = tile_index(t0, t1, t2);
    const int o0 = t0 * TILE, o1 = t1 * TILE, o2 = t2 * TILE;
    const int beg = koff[t * 8], end = koff[t * 8 + 8];
    int i = beg + threadIdx.x;
    float4 ur = make_float4(0.f, 0.f, 0.f, 0.f);
    Mom3 vr{0.f, 0.f, 0.f};
    if (i < end) {
        ur = xs[i];
        vr = ps[i];
    }
    // (row, quad) tasks: one 16-byte load per component (rows start 64-byte
    // aligned), four cells written; then one task per row for the halo cell
    for (int e = threadIdx.x; e < ROWS * 4; e += READOUT_T) {
        const int rr = e >> 2, j = e & 3, a = rr / H, b = rr % H;
        const float *src = F + (int64_t)((o0 + a) & mask) * fps + (int64_t)((o1 + b) & mask) * rs + o2 + 4 * j;
        const float4 fx = *reinterpret_cast<const float4 *>(src);
        const float4 fy = *reinterpret_cast<const float4 *>(src + cs);
        const float4 fz = *reinterpret_cast<const float4 *>(src + 2 * cs);
        float4 *dst = fl + rr * H + 4 * j;
        dst[0] = make_float4(fx.x, fy.x, fz.x, 0.f);
        dst[1] = make_float4(fx.y, fy.y, fz.y, 0.f);
        dst[2] = make_float4(fx.z, fy.z, fz.z, 0.f);
        dst[3] = make_float4(fx.w, fy.w, fz.w, 0.f);
    }
    for (int rr = threadIdx.x; rr < ROWS; rr += READOUT_T) {
        const int a = rr / H, b = rr % H;
        const float *src = F + (int64_t)((o0 + a) & mask) * fps + (int64_t)((o1 + b) & mask) * rs + ((o2 + TILE) & mask);
        fl[rr * H + TILE] = make_float4(src[0], src[cs], src[2 * cs], 0.f);
    }
    if (threadIdx.x < NB) hist[threadIdx.x] = 0;
    __syncthreads();
    const float nf = (float)n;
    bool bad = false;
    while (i < end) {
        const float u0 = ur.x, u1 = ur.y, u2 = ur.z;
        const int tag = __float_as_int(ur.w);
        const float f0 = floorf(u0), f1 = floorf(u1), f2 = floorf(u2);
        const float d0 = u0 - f0, d1 = u1 - f1, d2 = u2 - f2;
        const int a0 = ((int)f0 - o0) & mask, a1 = ((int)f1 - o1) & mask, a2 = ((int)f2 - o2) & mask;
        const float w0[2] = {1.f - d0, d0}, w1[2] = {1.f - d1, d1}, w2[2] = {1.f - d2, d2};
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int row = ((a0 + a) * H + (a1 + b)) * H + a2;
                const float wab = w0[a] * w1[b];
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const float w = wab * w2[c];
                    const float4 f = fl[row + c];
                    s0 += w * f.x;
                    s1 += w * f.y;
                    s2 += w * f.z;
                }
            }
        const float p0 = vr.x + kick * s0;
        const float p1 = vr.y + kick * s1;
        const float p2 = vr.z + kick * s2;
        const float x0 = wrapf(u0 + drift * p0, nf);
        const float x1 = wrapf(u1 + drift * p1, nf);
        const float x2 = wrapf(u2 + drift * p2, nf);
        bad |= !(isfinite(p0) && isfinite(p1) && isfinite(p2) && isfinite(x0) && isfinite(x1) && isfinite(x2));
        if (cnt_next) {
            // the next step's sort counts: keys in this tile or its 26
            // neighbours go to the LDS histogram, the rest (mostly neutrinos
            // that streamed far) straight to the global counts
            const int c0 = (int)floorf(x0) & mask, c1 = (int)floorf(x1) & mask, c2 = (int)floorf(x2) & mask;
            const int s0 = c0 / TILE, s1 = c1 / TILE, s2 = c2 / TILE;
            const int f = ((c0 % TILE) == TILE - 1 ? 1 : 0) | ((c1 % TILE) == TILE - 1 ? 2 : 0) |
                          ((c2 % TILE) == TILE - 1 ? 4 : 0);
            const int e0 = (s0 - t0 + 1 + nt) & (nt - 1), e1 = (s1 - t1 + 1 + nt) & (nt - 1),
                      e2 = (s2 - t2 + 1 + nt) & (nt - 1);
            if (e0 < 3 && e1 < 3 && e2 < 3)
                atomicAdd(&hist[((e0 * 3 + e1) * 3 + e2) * 8 + f], 1);
            else
                atomicAdd(cnt_next + tile_index(s0, s1, s2) * 8 + f, 1);
        }
        const int inext = i + READOUT_T;
        if (inext < end) {
            ur = xs[inext];
            vr = ps[inext];
        }
        p[i] = p0;
        p[P + i] = p1;
        p[2 * P + i] = p2;
        x[i] = x0;
        x[P + i] = x1;
        x[2 * P + i] = x2;
        tags[i] = (uint8_t)tag;
        if (ids) ids[i] = ids_tmp[i];
        i = inext;
    }
    if (bad) atomicOr(flag, FLAG_NAN);
    if (cnt_next) {
        __syncthreads();
        if (threadIdx.x < NB && hist[threadIdx.x] > 0) {
            const int b = threadIdx.x, e = b / 8, f = b % 8;
            const int s0 = (t0 + e / 9 - 1 + nt) & (nt - 1), s1 = (t1 + (e / 3) % 3 - 1 + nt) & (nt - 1),
                      s2 = (t2 + e % 3 - 1 + nt) & (nt - 1);
            atomicAdd(cnt_next + tile_index(s0, s1, s2) * 8 + f, hist[b]);
        }
    }
}

__global__ void k_fill_i32(int *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_add_i64(const int64_t *src, int64_t *dst, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] += src[i];
}

__global__ void k_tags_canonical(uint8_t *tags, int64_t P, int nseg, const int64_t *seg_off)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t t = 0;
        for (int g = 1; g < nseg; g++) t += (i >= seg_off[g]) ? 1 : 0;
        tags[i] = t;
    }
}

__global__ void k_copy_real(const float *src, int64_t rs, int64_t ps, int n, float *dst)
{
    const int64_t m = (int64_t)n * n * n, n2 = (int64_t)n * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[(t / n2) * ps + ((t / n) % n) * rs + t % n];
}

__global__ void k_copy_half(const float2 *src, int64_t rs, int n, float2 *dst)
{
    const int nh = n / 2 + 1;
    const int64_t m = (int64_t)n * n * nh;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[(t / nh) * rs + t % nh];
}

__global__ void k_load_half(const float2 *src, int n, float2 *dst, int64_t rs)
{
    const int nh = n / 2 + 1;
    const int64_t m = (int64_t)n * n * rs;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / rs;
        const int k = (int)(t % rs);
        dst[t] = k < nh ? src[row * nh + k] : make_float2(0.f, 0.f);
    }
}

__device__ __forceinline__ float wrap_to_float(double v, int n)
{
    double t = fmod(v, (double)n);
    if (t < 0) t += n;
    float r = (float)t;
    if (r >= (float)n) r = 0.f;
    return r;
}

// CDM: lattice point + displacement; p = vfac s (mesh units).
__global__ void k_ic_cdm(const float *__restrict__ F, int64_t rs, int64_t cs, int nic, int n, double vfac,
                         float *x, float *p, int64_t P)
{
    const int64_t m = (int64_t)nic * nic * nic;
    const double dc = (double)n / nic;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int i0 = (int)(t / ((int64_t)nic * nic)), i1 = (int)((t / nic) % nic), i2 = (int)(t % nic);
        const int64_t idx = ((int64_t)i0 * nic + i1) * rs + i2;
        const int ii[3] = {i0, i1, i2};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double s = F[d * cs + idx];
            x[d * P + t] = wrap_to_float(ii[d] * dc + s, n);
            p[d * P + t] = (float)(vfac * s);
        }
    }
}

// Neutrinos: shell s, site j (row-major), direction t: position = site +
// r_s v_t + s_nu(site), momentum = p_s v_t + vfac s_nu(site), with the
// direction set reversed on odd sites when `flip`.
// tables: dirs[n_dir][3], radius[n_shell], pth[n_shell].
__global__ void k_ic_nu(const float *__restrict__ F, int64_t rs, int64_t cs, int nic, int n, int ns, int n_dir,
                        int n_shell, const float *__restrict__ tables, double vfac, int flip, float *x, float *p,
                        int64_t P, int64_t nc)
{
    const int64_t nsites = (int64_t)ns * ns * ns;
    const int64_t per = nsites * n_dir;
    const int64_t total = per * n_shell;
    const int R = nic / ns;
    const double dc = (double)n / nic;
    const float *dirs = tables, *radius = tables + 3 * n_dir, *pth = radius + n_shell;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int sh = (int)(t / per);
        const int64_t rem = t % per;
        const int64_t site = rem / n_dir;
        const int dir = (int)(rem % n_dir);
        const int j0 = (int)(site / ((int64_t)ns * ns)), j1 = (int)((site / ns) % ns), j2 = (int)(site % ns);
        const int jj[3] = {j0, j1, j2};
        const double sign = (flip && ((j0 + j1 + j2) & 1)) ? -1.0 : 1.0;
        const int64_t g = ((int64_t)(j0 * R + R / 2) * nic + (j1 * R + R / 2)) * rs + (j2 * R + R / 2);
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double s = F[d * cs + g];
            const double v = sign * (double)dirs[dir * 3 + d];
            const double centre = (jj[d] * R + R / 2 + 0.5) * dc;
            x[d * P + nc + t] = wrap_to_float(centre + (double)radius[sh] * v + s, n);
            p[d * P + nc + t] = (float)((double)pth[sh] * v + vfac * s);
        }
    }
}

// Pseudo-random neutrinos (one per site): x = site + s, p = q pth_unit n + vfac s,
// q = C^-1(u0) from the cumulative table cdf[0..nq] at q = i hq (search, then
// linear interpolation inside the cell), n = (sin t cos f, sin t sin f, cos t)
// with cos t = 2 u1 - 1, f = 2 pi u2.
__global__ void k_ic_nu_pseudo(const float *__restrict__ F, int64_t rs, int64_t cs, int nic, int n, int ns,
                               const float *__restrict__ cdf, int nq, double hq, double pth_unit, double vfac,
                               const float *__restrict__ u, float *x, float *p, int64_t P, int64_t nc)
{
    const int64_t nsites = (int64_t)ns * ns * ns;
    const int R = nic / ns;
    const double dc = (double)n / nic;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nsites; t += (int64_t)gridDim.x * blockDim.x) {
        const int j0 = (int)(t / ((int64_t)ns * ns)), j1 = (int)((t / ns) % ns), j2 = (int)(t % ns);
        const int jj[3] = {j0, j1, j2};
        const int64_t g = ((int64_t)(j0 * R + R / 2) * nic + (j1 * R + R / 2)) * rs + (j2 * R + R / 2);
        const float u0 = u[t];
        int lo = 0, hi = nq;   // cdf[lo] <= u0 < cdf[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid] <= u0) lo = mid; else hi = mid;
        }
        const double c0 = cdf[lo], c1 = cdf[lo + 1];
        const double q = hq * (lo + (c1 > c0 ? ((double)u0 - c0) / (c1 - c0) : 0.0));
        const double ct = 2.0 * (double)u[nsites + t] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double ph = 6.283185307179586 * (double)u[2 * nsites + t];
        const double v[3] = {st * cos(ph), st * sin(ph), ct};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const double s = F[d * cs + g];
            const double centre = (jj[d] * R + R / 2 + 0.5) * dc;
            x[d * P + nc + t] = wrap_to_float(centre + s, n);
            p[d * P + nc + t] = (float)(q * pth_unit * v[d] + vfac * s);
        }
    }
}

__device__ __forceinline__ int isqrt_i(int64_t v)
{
    int64_t b = (int64_t)sqrt((double)v);
    while (b * b > v) b--;
    while ((b + 1) * (b + 1) <= v) b++;
    return (int)b;
}

__device__ __forceinline__ double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// Per-block partial sums over the half spectrum: (sum w P, sum w |k|, sum w)
// per bin, w = 2 for 0 < k2 < N/2 (the mode and its conjugate), else 1.
__global__ __launch_bounds__(256) void k_power_bin(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                   int64_t rs, int n, int nbins, int compensate, double norm,
                                                   double kf, double *partial)
{
    __shared__ double sh[3 * MAX_BINS];
    for (int i = threadIdx.x; i < 3 * nbins; i += blockDim.x) sh[i] = 0.0;
    __syncthreads();
    const int nh = n / 2 + 1;
    const int64_t m = (int64_t)n * n * nh;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int k2 = (int)(t % nh);
        const int64_t row = t / nh;
        const int k1 = (int)(row % n), k0 = (int)(row / n);
        const int64_t n0 = k0 < n / 2 ? k0 : k0 - n, n1 = k1 < n / 2 ? k1 : k1 - n, n2 = k2;
        const int64_t nn2 = n0 * n0 + n1 * n1 + n2 * n2;
        if (nn2 == 0) continue;
        const int b = isqrt_i(nn2);
        if (b >= nbins) continue;
        const double w = (k2 == 0 || k2 == n / 2) ? 1.0 : 2.0;
        const float2 a = A[row * rs + k2], c = B[row * rs + k2];
        double v = ((double)a.x * c.x + (double)a.y * c.y) * norm;
        if (compensate) {
            const double pi_n = 3.141592653589793238 / n;
            const double s0 = sinc(pi_n * n0), s1 = sinc(pi_n * n1), s2 = sinc(pi_n * n2);
            const double win = s0 * s0 * s1 * s1 * s2 * s2;
            v /= win * win;
        }
        atomicAdd(&sh[3 * b], w * v);
        atomicAdd(&sh[3 * b + 1], w * kf * sqrt((double)nn2));
        atomicAdd(&sh[3 * b + 2], w);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * nbins; i += blockDim.x) partial[(int64_t)blockIdx.x * 3 * nbins + i] = sh[i];
}

// Sum the block partials in block order (deterministic).
__global__ void k_power_reduce(const double *partial, int nblocks, int nbins, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * nbins) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; b++) s += partial[(int64_t)b * 3 * nbins + i];
    out[i] = s;
}

}  // namespace

hipError_t launch_fill_i64(int64_t *p, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(count / 2, 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_readout(const float *x, int64_t P, const float2 *f, int64_t rs_f, int64_t ps_f, int64_t comp_stride,
                          int n, float *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_readout, dim3(grid_for(P, 256)), dim3(256), 0, s, x, P,
                       reinterpret_cast<const float *>(f), 2 * rs_f, 2 * ps_f, 2 * comp_stride, n, acc);
    return hipGetLastError();
}

hipError_t launch_readout_kick_drift(float *x, float *p, int64_t P, const float2 *f, int64_t rs_f, int64_t ps_f,
                                     int64_t comp_stride, int n, float kick, float drift, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_readout_kick_drift, dim3(grid_for(P, 256)), dim3(256), 0, s, x, p, P,
                       reinterpret_cast<const float *>(f), 2 * rs_f, 2 * ps_f, 2 * comp_stride, n, kick, drift, flag);
    return hipGetLastError();
}

hipError_t launch_readout_kd_tiles(const float4 *xs, const Mom3 *ps, int64_t P, const int *koff, const float2 *f,
                                   int64_t rs_f, int64_t ps_f, int64_t comp_stride, int n, float kick, float drift,
                                   float *x, float *p, uint8_t *tags, const uint32_t *ids_tmp, uint32_t *ids, int *flag,
                                   int *cnt_next, hipStream_t s)
{
    const int nt = n / TILE;
    if (nt < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_readout_kd_tiles, dim3((unsigned)(nt * nt * nt)), dim3(READOUT_T), 0, s, xs, ps, P, koff,
                       reinterpret_cast<const float *>(f), 2 * rs_f, 2 * ps_f, 2 * comp_stride, n, kick, drift, x, p, tags,
                       ids_tmp, ids, flag, cnt_next);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_add_i64(const int64_t *src, int64_t *dst, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_i64, dim3(grid_for(count, 256)), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_tags_canonical(uint8_t *tags, int64_t P, int nseg, const int64_t *seg_off, hipStream_t s)
{
    hipLaunchKernelGGL(k_tags_canonical, dim3(grid_for(P, 256)), dim3(256), 0, s, tags, P, nseg, seg_off);
    return hipGetLastError();
}

hipError_t launch_copy_real(const float *src, int64_t rs, int64_t ps, int n, float *dst, hipStream_t s)
{
    const int64_t m = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_copy_real, dim3(grid_for(m, 256)), dim3(256), 0, s, src, rs, ps, n, dst);
    return hipGetLastError();
}

hipError_t launch_copy_half(const float2 *src, int64_t rs, int n, float2 *dst, hipStream_t s)
{
    const int64_t m = (int64_t)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_copy_half, dim3(grid_for(m, 256)), dim3(256), 0, s, src, rs, n, dst);
    return hipGetLastError();
}

hipError_t launch_load_half(const float2 *src, int n, float2 *dst, int64_t rs, hipStream_t s)
{
    const int64_t m = (int64_t)n * n * rs;
    hipLaunchKernelGGL(k_load_half, dim3(grid_for(m, 256)), dim3(256), 0, s, src, n, dst, rs);
    return hipGetLastError();
}

hipError_t launch_ic_cdm(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, double vfac, float *x,
                         float *p, int64_t P, hipStream_t s)
{
    const int64_t m = (int64_t)nic * nic * nic;
    hipLaunchKernelGGL(k_ic_cdm, dim3(grid_for(m, 256)), dim3(256), 0, s, reinterpret_cast<const float *>(f),
                       2 * rs, 2 * comp_stride, nic, n, vfac, x, p, P);
    return hipGetLastError();
}

hipError_t launch_ic_nu(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, int ns, int n_dir,
                        int n_shell, const float *tables, double vfac, int flip, float *x, float *p, int64_t P,
                        int64_t nc, hipStream_t s)
{
    const int64_t total = (int64_t)ns * ns * ns * n_dir * n_shell;
    hipLaunchKernelGGL(k_ic_nu, dim3(grid_for(total, 256)), dim3(256), 0, s, reinterpret_cast<const float *>(f),
                       2 * rs, 2 * comp_stride, nic, n, ns, n_dir, n_shell, tables, vfac, flip, x, p, P, nc);
    return hipGetLastError();
}

hipError_t launch_ic_nu_pseudo(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, int ns,
                               const float *cdf, int nq, double hq, double pth_unit, double vfac, const float *u,
                               float *x, float *p, int64_t P, int64_t nc, hipStream_t s)
{
    if (nq < 1 || ns < 1 || nic % ns) return hipErrorInvalidValue;
    const int64_t nsites = (int64_t)ns * ns * ns;
    hipLaunchKernelGGL(k_ic_nu_pseudo, dim3(grid_for(nsites, 256)), dim3(256), 0, s, reinterpret_cast<const float *>(f),
                       2 * rs, 2 * comp_stride, nic, n, ns, cdf, nq, hq, pth_unit, vfac, u, x, p, P, nc);
    return hipGetLastError();
}

hipError_t launch_power_bin(const float2 *A, const float2 *B, int64_t rs, int n, int nbins, int compensate,
                            double norm, double kf, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_bin, dim3(POWER_BLOCKS), dim3(256), 0, s, A, B, rs, n, nbins, compensate, norm, kf,
                       partial);
    return hipGetLastError();
}

hipError_t launch_power_reduce(const double *partial, int nbins, double *out, hipStream_t s)
{
    const int m = 3 * nbins;
    hipLaunchKernelGGL(k_power_reduce, dim3((m + 255) / 256), dim3(256), 0, s, partial, POWER_BLOCKS, nbins, out);
    return hipGetLastError();
}

}  // namespace pm
