// Reverse mode of the particle-mesh step and of the initial conditions.
//
// Differentiable model (the reconstruction use of the method, Sec. 1 and the
// conclusions of the paper): each particle deposits its segment mass with
// cloud-in-cell weights W(x, c) = prod_e w_e, w_e = 1 - f_e on cell floor(u_e)
// and f_e on the next one (f_e = u_e - floor u_e); the fixed-point paint
// equals this to 2^-S per cell and its rounding has zero derivative.  With
// Phi_d = L_d delta the force meshes and g the cotangent of the force on the
// particles,
//   xbar_i += sum_d g_{i,d} sum_c dW(x_i, c)/dx_i Phi_d(c)        (readout term)
//   psi = sum_d L_d^T G_d = -sum_d L_d G_d,  G_d = sum_i g_{i,d} W(x_i, .)
//   xbar_j += m_j sum_c psi(c) dW(x_j, c)/dx_j                      (paint term)
// since L_d (multiplier 1.5 Omega_m0 i k_d / k^2) is a real convolution with an
// odd kernel.  dW/dx_e takes -1 / +1 for the lower / upper cell along e (the
// right derivative at cell faces).  Kick and drift are linear.
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

struct Cic {
    int64_t row[2][2];   // (c0, c1) row offsets
    int c2[2];
    float w[3][2];
};

// Row offsets on a mesh of row stride rs and plane stride ps.
__device__ __forceinline__ Cic cic_at(float u0, float u1, float u2, int n, int64_t rs, int64_t ps)
{
    Cic r;
    const int mask = n - 1;
    const float u[3] = {u0, u1, u2};
    int c[3][2];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const float f = floorf(u[d]);
        const int i = (int)f;
        r.w[d][1] = u[d] - f;
        r.w[d][0] = 1.f - r.w[d][1];
        c[d][0] = i & mask;
        c[d][1] = (i + 1) & mask;
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) r.row[a][b] = (int64_t)c[0][a] * ps + (int64_t)c[1][b] * rs;
    r.c2[0] = c[2][0];
    r.c2[1] = c[2][1];
    return r;
}

// Gradient of sum_d v_d interp(mesh_d)(x): out_e = sum_c dW/dx_e sum_d v_d mesh_d(c).
template <int ND>
__device__ __forceinline__ void interp_grad(const Cic &q, const float *mesh, int64_t cs, const float *v, float out[3])
{
    out[0] = out[1] = out[2] = 0.f;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int e = 0; e < 2; e++) {
                const int64_t idx = q.row[a][b] + q.c2[e];
                float s = 0.f;
#pragma unroll
                for (int d = 0; d < ND; d++) s += v[d] * mesh[d * cs + idx];
                const float s0 = a ? 1.f : -1.f, s1 = b ? 1.f : -1.f, s2 = e ? 1.f : -1.f;
                out[0] += s0 * q.w[1][b] * q.w[2][e] * s;
                out[1] += q.w[0][a] * s1 * q.w[2][e] * s;
                out[2] += q.w[0][a] * q.w[1][b] * s2 * s;
            }
}

__device__ __forceinline__ int segment_of(int64_t i, int nseg, const int64_t *seg_off, const uint8_t *tags)
{
    if (tags) return tags[i];
    int g = 0;
    for (int k = 1; k < nseg; k++) g += (i >= seg_off[k]) ? 1 : 0;
    return g;
}

__global__ void k_axpy(float *y, const float *x, float a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

// Readout term: xbar_i += gscale * sum_d g_{i,d} grad interp(F_d)(x_i).
__global__ __launch_bounds__(256) void k_readout_grad3(const float *__restrict__ x, int64_t P,
                                                       const float *__restrict__ g, float gscale,
                                                       const float *__restrict__ F, int64_t rs, int64_t ps,
                                                       int64_t cs, int n, float *xbar)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const Cic q = cic_at(x[i], x[P + i], x[2 * P + i], n, rs, ps);
        const float v[3] = {gscale * g[i], gscale * g[P + i], gscale * g[2 * P + i]};
        float out[3];
        interp_grad<3>(q, F, cs, v, out);
        xbar[i] += out[0];
        xbar[P + i] += out[1];
        xbar[2 * P + i] += out[2];
    }
}

// G_d(c) += gscale g_{i,d} W(x_i, c) (float atomics: summation order varies).
__global__ __launch_bounds__(256) void k_paint_vec3(const float *__restrict__ x, int64_t P,
                                                    const float *__restrict__ g, float gscale, float *G, int64_t rs,
                                                    int64_t cs, int n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const Cic q = cic_at(x[i], x[P + i], x[2 * P + i], n, rs, (int64_t)n * rs);
        const float v[3] = {gscale * g[i], gscale * g[P + i], gscale * g[2 * P + i]};
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const float w = (q.w[0][a] * q.w[1][b]) * q.w[2][e];
                    const int64_t idx = q.row[a][b] + q.c2[e];
#pragma unroll
                    for (int d = 0; d < 3; d++) unsafeAtomicAdd(G + d * cs + idx, w * v[d]);
                }
    }
}

// Largest |gscale g| over count values, as the bits of a non-negative float,
// atomicMax'ed into *out (zeroed by the caller).
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ g, int64_t count, float gscale,
                                                unsigned *out)
{
    // The bits of |v| order like the values themselves (sign bit clear), with
    // +inf above every finite value and NaN above +inf, so an integer maximum
    // reports a NaN or an infinity anywhere in g.  One atomic per workgroup.
    __shared__ unsigned wm[256 / 64];
    unsigned m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(fabsf(gscale * g[i])));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(out, max(max(wm[0], wm[1]), max(wm[2], wm[3])));
}

// One cotangent component in fixed point: Q(c) += llrint(S w_c gscale g_i)
// with the cloud-in-cell weight w_c of particle i (the float products of the
// FP32 form).  Integer sums do not depend on the order of the atomics, so the
// cotangent mesh, and the gradient built from it, is the same on every run.
__global__ __launch_bounds__(256) void k_paint_q1(const float *__restrict__ x, int64_t P,
                                                  const float *__restrict__ gd, float gscale, double S, int n,
                                                  unsigned long long *Q)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const Cic q = cic_at(x[i], x[P + i], x[2 * P + i], n, n, (int64_t)n * n);
        const double v = (double)(gscale * gd[i]) * S;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const float w = (q.w[0][a] * q.w[1][b]) * q.w[2][e];
                    const long long iq = (long long)__builtin_rint((double)w * v);
                    atomicAdd(Q + q.row[a][b] + q.c2[e], (unsigned long long)iq);
                }
    }
}

// The same integers by 16^3 tile, from the tile-sorted records (positions
// xs, cotangent components vals): one workgroup per tile sums, in LDS, the
// corners of its own particles and of the 19 neighbour ranges whose face
// flags say a +1 corner crosses in, then writes the tile once (no zero fill,
// no global atomics).  Each corner value is formed exactly as in k_paint_q1.
constexpr int PQT = 512;
__global__ __launch_bounds__(PQT) void k_paint_q1_tiles(const float4 *__restrict__ xs, const Mom3 *__restrict__ vals,
                                                       int comp, const int *__restrict__ koff, float gscale, double S,
                                                       int n, unsigned long long *Q)
{
    __shared__ unsigned long long acc[TILE * TILE * TILE];
    __shared__ int rbeg[NRANGE], rpre[NRANGE + 1];
    const int nt = n / TILE, mask = n - 1;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int t2 = (int)morton_compact((unsigned)t), t1 = (int)morton_compact((unsigned)t >> 1),
              t0 = (int)morton_compact((unsigned)t >> 2);
    for (int i = threadIdx.x; i < TILE * TILE * TILE; i += PQT) acc[i] = 0;
    tile_ranges(koff, t, t0, t1, t2, nt, rbeg, rpre);
    const int total = rpre[NRANGE];
    const int o[3] = {t0 * TILE, t1 * TILE, t2 * TILE};
    for (int k = threadIdx.x; k < total; k += PQT) {
        const int idx = tile_range_index(k, rbeg, rpre);
        const float4 r = xs[idx];
        const Mom3 g = vals[idx];
        const float gd = comp == 0 ? g.x : (comp == 1 ? g.y : g.z);
        const double v = (double)(gscale * gd) * S;
        const float u[3] = {r.x, r.y, r.z};
        float w[3][2];
        int l[3][2];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float f = floorf(u[d]);
            const int i = (int)f;
            w[d][1] = u[d] - f;
            w[d][0] = 1.f - w[d][1];
            l[d][0] = ((i & mask) - o[d]) & mask;
            l[d][1] = (((i + 1) & mask) - o[d]) & mask;
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    if (l[0][a] < TILE && l[1][b] < TILE && l[2][e] < TILE) {
                        const float wc = (w[0][a] * w[1][b]) * w[2][e];
                        const long long iq = (long long)__builtin_rint((double)wc * v);
                        atomicAdd(&acc[(l[0][a] * TILE + l[1][b]) * TILE + l[2][e]], (unsigned long long)iq);
                    }
                }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TILE * TILE * TILE; i += PQT) {
        const int a = i / (TILE * TILE), b = (i / TILE) % TILE, e = i % TILE;
        Q[((int64_t)(o[0] + a) * n + (o[1] + b)) * n + (o[2] + e)] = acc[i];
    }
}

// psi(k) = -coef sum_d i k_d / k^2 G_d(k) into field 0 (natural-order half
// spectra, row stride nhp, field stride fs); zero at k = 0 and, per term, on
// the Nyquist plane of component d.
__global__ void k_green_adj(float2 *F, int64_t nhp, int64_t fs, int n, float coef)
{
    const int64_t tot = (int64_t)n * n * nhp;
    const float sc = 6.28318530717958648f / (float)n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int k2 = (int)(t % nhp);
        const int64_t r = t / nhp;
        const int i1 = (int)(r % n), i0 = (int)(r / n);
        const int n0 = i0 <= n / 2 ? i0 : i0 - n, n1 = i1 <= n / 2 ? i1 : i1 - n;
        const float k0 = sc * n0, k1 = sc * n1, kz = sc * k2;
        const float kk = k0 * k0 + k1 * k1 + kz * kz;
        float2 out = make_float2(0.f, 0.f);
        if (k2 <= n / 2 && kk > 0.f) {
            const float g = coef / kk;
            const float f0 = (i0 == n / 2) ? 0.f : k0, f1 = (i1 == n / 2) ? 0.f : k1, f2 = (k2 == n / 2) ? 0.f : kz;
            const float2 a = F[t], b = F[fs + t], c = F[2 * fs + t];
            // s = sum_d f_d G_d;  psi = -i g s
            const float sx = f0 * a.x + f1 * b.x + f2 * c.x, sy = f0 * a.y + f1 * b.y + f2 * c.y;
            out = make_float2(g * sy, -g * sx);
        }
        F[t] = out;
    }
}

// xbar_j += scale m_j grad interp(mesh)(x_j), m_j = quanta[segment] 2^-S.
__global__ __launch_bounds__(256) void k_density_grad(const float *__restrict__ x, int64_t P,
                                                      const float *__restrict__ mesh, int64_t rs, int n, int nseg,
                                                      const int64_t *__restrict__ seg_off,
                                                      const uint8_t *__restrict__ tags,
                                                      const int64_t *__restrict__ quanta, float qscale, float scale,
                                                      float *xbar)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = segment_of(i, nseg, seg_off, tags);
        const float m = (float)quanta[g] * qscale * scale;
        const Cic q = cic_at(x[i], x[P + i], x[2 * P + i], n, rs, (int64_t)n * rs);
        const float v[1] = {m};
        float out[3];
        interp_grad<1>(q, mesh, 0, v, out);
        xbar[i] += out[0];
        xbar[P + i] += out[1];
        xbar[2 * P + i] += out[2];
    }
}

// delta = Q scale - 1 into a dense float mesh.
__global__ void k_q_to_delta(const int64_t *q, int64_t m, double scale, float *delta)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        delta[i] = (float)((double)q[i] * scale - 1.0);
}

// Initial-condition transpose, CDM: sbar_d(t) = xbar_{d,t} + vfac pbar_{d,t}
// on the IC lattice (particle t sits at lattice site t), real rows of stride rs.
__global__ void k_ic_adj_gather_cdm(const float *xbar, const float *pbar, int64_t P, int nic, float vfac, float *F,
                                    int64_t rs, int64_t cs)
{
    const int64_t m = (int64_t)nic * nic * nic;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * m; t += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(t / m);
        const int64_t i = t % m;
        F[d * cs + (i / nic) * rs + i % nic] = xbar[d * P + i] + vfac * pbar[d * P + i];
    }
}

// Neutrinos: the 70 particles of a site share its displacement, sampled at
// lattice point (j R + R/2) per axis; sbar there is the sum over them.
__global__ void k_ic_adj_gather_nu(const float *xbar, const float *pbar, int64_t P, int64_t nc, int nic, int ns,
                                   int nd, int n_shell, float vfac, float *F, int64_t rs, int64_t cs)
{
    const int64_t nsites = (int64_t)ns * ns * ns, per = nsites * nd;
    const int R = nic / ns;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * nsites;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(t / nsites);
        const int64_t j = t % nsites;
        float sum = 0.f;
        for (int sh = 0; sh < n_shell; sh++)
            for (int u = 0; u < nd; u++) {
                const int64_t idx = nc + sh * per + j * nd + u;
                sum += xbar[d * P + idx] + vfac * pbar[d * P + idx];
            }
        const int64_t j0 = j / ((int64_t)ns * ns), j1 = (j / ns) % ns, j2 = j % ns;
        const int64_t g0 = j0 * R + R / 2, g1 = j1 * R + R / 2, g2 = j2 * R + R / 2;
        F[d * cs + (g0 * nic + g1) * rs + g2] = sum;
    }
}

}  // namespace

hipError_t launch_axpy(float *y, const float *x, float a, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, s, y, x, a, n);
    return hipGetLastError();
}

hipError_t launch_readout_grad3(const float *x, int64_t P, const float *g, float gscale, const float *F, int64_t rs,
                                int64_t ps, int64_t cs, int n, float *xbar, hipStream_t s)
{
    hipLaunchKernelGGL(k_readout_grad3, dim3(grid_for(P, 256)), dim3(256), 0, s, x, P, g, gscale, F, rs, ps, cs, n,
                       xbar);
    return hipGetLastError();
}

hipError_t launch_paint_vec3(const float *x, int64_t P, const float *g, float gscale, float *G, int64_t rs,
                             int64_t cs, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_paint_vec3, dim3(grid_for(P, 256)), dim3(256), 0, s, x, P, g, gscale, G, rs, cs, n);
    return hipGetLastError();
}

hipError_t launch_absmax(const float *g, int64_t count, float gscale, unsigned *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_absmax, dim3(grid_for(count, 256, 1024)), dim3(256), 0, s, g, count, gscale, out);
    return hipGetLastError();
}

hipError_t launch_paint_q1(const float *x, int64_t P, const float *gd, float gscale, double S, int n, int64_t *Q,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_paint_q1, dim3(grid_for(P, 256)), dim3(256), 0, s, x, P, gd, gscale, S, n,
                       reinterpret_cast<unsigned long long *>(Q));
    return hipGetLastError();
}

hipError_t launch_paint_q1_tiles(const float4 *xs, const Mom3 *vals, int comp, const int *koff, float gscale,
                                 double S, int n, int64_t *Q, hipStream_t s)
{
    const int nt = n / TILE;
    if (nt < 2 || comp < 0 || comp > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_paint_q1_tiles, dim3((unsigned)(nt * nt * nt)), dim3(PQT), 0, s, xs, vals, comp, koff, gscale,
                       S, n, reinterpret_cast<unsigned long long *>(Q));
    return hipGetLastError();
}

hipError_t launch_green_adj(float2 *F, int64_t nhp, int64_t fs, int n, double coef, hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    hipLaunchKernelGGL(k_green_adj, dim3(grid_for(tot, 256)), dim3(256), 0, s, F, nhp, fs, n, (float)coef);
    return hipGetLastError();
}

hipError_t launch_density_grad(const float *x, int64_t P, const float *mesh, int64_t rs, int n, int nseg,
                               const int64_t *seg_off, const uint8_t *tags, const int64_t *quanta, float qscale,
                               float scale, float *xbar, hipStream_t s)
{
    hipLaunchKernelGGL(k_density_grad, dim3(grid_for(P, 256)), dim3(256), 0, s, x, P, mesh, rs, n, nseg, seg_off, tags,
                       quanta, qscale, scale, xbar);
    return hipGetLastError();
}

hipError_t launch_q_to_delta(const int64_t *q, int64_t m, double scale, float *delta, hipStream_t s)
{
    hipLaunchKernelGGL(k_q_to_delta, dim3(grid_for(m, 256)), dim3(256), 0, s, q, m, scale, delta);
    return hipGetLastError();
}

hipError_t launch_ic_adj_gather_cdm(const float *xbar, const float *pbar, int64_t P, int nic, float vfac, float *F,
                                    int64_t rs, int64_t cs, hipStream_t s)
{
    const int64_t m = (int64_t)nic * nic * nic;
    hipLaunchKernelGGL(k_ic_adj_gather_cdm, dim3(grid_for(3 * m, 256)), dim3(256), 0, s, xbar, pbar, P, nic, vfac, F,
                       rs, cs);
    return hipGetLastError();
}

hipError_t launch_ic_adj_gather_nu(const float *xbar, const float *pbar, int64_t P, int64_t nc, int nic, int ns,
                                   int nd, int n_shell, float vfac, float *F, int64_t rs, int64_t cs, hipStream_t s)
{
    const int64_t nsites = (int64_t)ns * ns * ns;
    hipLaunchKernelGGL(k_ic_adj_gather_nu, dim3(grid_for(3 * nsites, 256)), dim3(256), 0, s, xbar, pbar, P, nc, nic,
                       ns, nd, n_shell, vfac, F, rs, cs);
    return hipGetLastError();
}

}  // namespace pm
