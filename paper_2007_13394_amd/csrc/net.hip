// Learned force correction: kernels of the forward model and its reverse mode.
//
// Model (an addition to the method; the paper's introduction motivates
// learned corrections of fast particle-mesh codes): a radial filter
// g(k, a) = 1 + MLP(|k| / k_Nyq, a) on the potential spectrum, tabulated at
// NET_NB radial bins and interpolated linearly, and a 3-layer periodic 3^3
// CNN (1 -> 16 -> 16 -> 1 channels, SiLU) on the density contrast (read from
// the int64 mesh); the force is minus the spectral gradient of phi_f + cnn.
// Parameters: one flat FP32 array (offsets in pm_internal.h).  The CNN takes
// BF16 activations and weights and accumulates in FP32; the 16 -> 16 layer,
// 89 % of the network's arithmetic, runs on MFMA (16x16x16 BF16 tiles).
#include <type_traits>

#include "pm_internal.h"

namespace pm {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// sum + a.lo b.lo + a.hi b.hi for BF16 pairs, FP32 accumulation
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float sum)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(v2bf, a), __builtin_bit_cast(v2bf, b), sum, false);
}

inline unsigned grid_for(int64_t n, int block, int64_t cap = 65536LL * 16)
{
    int64_t b = (n + block - 1) / block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = 1.f / (1.f + __expf(-z));
    return s + z * s * (1.f - s);
}
// round to the nearest BF16 (ties to even; the hardware conversion) and back
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16r(float f) { return from_bf16(to_bf16(f)); }

__device__ __forceinline__ float bin_kt(int b) { return (float)b * 1.7320508075688772f / (float)(NET_NB - 1); }

// ---------------------------------------------------------------- radial MLP table
// One workgroup per bin, one thread per hidden unit.
__global__ __launch_bounds__(128) void k_mlp_fwd(const float *__restrict__ th, float a, float *table)
{
    __shared__ float h[NET_H], red[128];
    const int b = blockIdx.x, j = threadIdx.x;
    const float kt = bin_kt(b);
    float z = 0.f;
    if (j < NET_H) h[j] = silu(th[NB0 + j] + th[NW0 + 2 * j] * kt + th[NW0 + 2 * j + 1] * a);
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < 2; l++) {
        const int W = l == 0 ? NW1 : NW2, B = l == 0 ? NB1 : NB2;
        if (j < NET_H) {
            z = th[B + j];
            for (int i = 0; i < NET_H; i++) z += th[W + j * NET_H + i] * h[i];
        }
        __syncthreads();
        if (j < NET_H) h[j] = silu(z);
        __syncthreads();
    }
    red[j] = j < NET_H ? th[NW3 + j] * h[j] : 0.f;
    __syncthreads();
    for (int s = 64; s >= 1; s >>= 1) {
        if (j < s) red[j] += red[j + s];
        __syncthreads();
    }
    if (j == 0) table[b] = 1.f + th[NB3] + red[0];
}

// dth += tbar[b] d table[b] / d th (float atomics across bins).
__global__ __launch_bounds__(128) void k_mlp_bwd(const float *__restrict__ th, float a, const double *tbar,
                                                 float *dth)
{
    __shared__ float h0[NET_H], h1[NET_H], h2[NET_H], dd[NET_H];
    const int b = blockIdx.x, j = threadIdx.x;
    const float g = (float)tbar[b];
    if (g == 0.f) return;   // uniform over the workgroup
    const float kt = bin_kt(b);
    float z0 = 0.f, z1 = 0.f, z2 = 0.f;
    if (j < NET_H) {
        z0 = th[NB0 + j] + th[NW0 + 2 * j] * kt + th[NW0 + 2 * j + 1] * a;
        h0[j] = silu(z0);
    }
    __syncthreads();
    if (j < NET_H) {
        z1 = th[NB1 + j];
        for (int i = 0; i < NET_H; i++) z1 += th[NW1 + j * NET_H + i] * h0[i];
        h1[j] = silu(z1);
    }
    __syncthreads();
    if (j < NET_H) {
        z2 = th[NB2 + j];
        for (int i = 0; i < NET_H; i++) z2 += th[NW2 + j * NET_H + i] * h1[i];
        h2[j] = silu(z2);
    }
    __syncthreads();
    if (j == 0) atomicAdd(dth + NB3, g);
    if (j < NET_H) {
        atomicAdd(dth + NW3 + j, g * h2[j]);
        dd[j] = g * th[NW3 + j] * dsilu(z2);
    }
    __syncthreads();
    float d = 0.f;
    if (j < NET_H) {
        atomicAdd(dth + NB2 + j, dd[j]);
        for (int i = 0; i < NET_H; i++) atomicAdd(dth + NW2 + j * NET_H + i, dd[j] * h1[i]);
        for (int k = 0; k < NET_H; k++) d += dd[k] * th[NW2 + k * NET_H + j];
        d *= dsilu(z1);
    }
    __syncthreads();
    if (j < NET_H) dd[j] = d;
    __syncthreads();
    d = 0.f;
    if (j < NET_H) {
        atomicAdd(dth + NB1 + j, dd[j]);
        for (int i = 0; i < NET_H; i++) atomicAdd(dth + NW1 + j * NET_H + i, dd[j] * h0[i]);
        for (int k = 0; k < NET_H; k++) d += dd[k] * th[NW1 + k * NET_H + j];
        d *= dsilu(z0);
        atomicAdd(dth + NB0 + j, d);
        atomicAdd(dth + NW0 + 2 * j, d * kt);
        atomicAdd(dth + NW0 + 2 * j + 1, d * a);
    }
}

// ---------------------------------------------------------------- spectral parts
// Natural-order half spectra [n][n][nhp]; mode t -> wave vector in grid units.
struct Mode {
    float k0, k1, k2, kk;
    bool pad, nyq0, nyq1, nyq2;
    int kz;
};
__device__ __forceinline__ Mode mode_of(int64_t t, int64_t nhp, int n)
{
    Mode m;
    const int kz = (int)(t % nhp);
    const int64_t r = t / nhp;
    const int i1 = (int)(r % n), i0 = (int)(r / n);
    const float sc = 6.28318530717958648f / (float)n;
    m.k0 = sc * (i0 <= n / 2 ? i0 : i0 - n);
    m.k1 = sc * (i1 <= n / 2 ? i1 : i1 - n);
    m.k2 = sc * kz;
    m.kk = m.k0 * m.k0 + m.k1 * m.k1 + m.k2 * m.k2;
    m.pad = kz > n / 2;
    m.nyq0 = i0 == n / 2;
    m.nyq1 = i1 == n / 2;
    m.nyq2 = kz == n / 2;
    m.kz = kz;
    return m;
}


// out = g(|k|) coef / k^2 in (k = 0 and padding -> 0).
__global__ void k_spec_filter(const float2 *in, float2 *out, int64_t nhp, int n, const float *table, float coef)
{
    __shared__ float tab[NET_NB];
    for (int i = threadIdx.x; i < NET_NB; i += blockDim.x) tab[i] = table[i];
    __syncthreads();
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(t, nhp, n);
        float2 o = make_float2(0.f, 0.f);
        if (!m.pad && m.kk > 0.f) {
            int b;
            float w;
            const float g = table_at(tab, sqrtf(m.kk) * 0.31830988618379067f, b, w) * coef / m.kk;
            const float2 v = in[t];
            o = make_float2(g * v.x, g * v.y);
        }
        out[t] = o;
    }
}

// tbar[b] += sum over modes of the bin weights times Re[coef / k^2 dk conj(pf)],
// each half-spectrum mode standing for its conjugate too (weight 2) except on
// the planes kz = 0 and kz = n/2.
__global__ __launch_bounds__(256) void k_spec_filter_bwd(const float2 *dk, const float2 *pf, int64_t nhp, int n,
                                                         float coef, double *tbar)
{
    __shared__ double hist[NET_NB];
    for (int i = threadIdx.x; i < NET_NB; i += blockDim.x) hist[i] = 0.0;
    __syncthreads();
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(t, nhp, n);
        if (m.pad || m.kk == 0.f) continue;
        const float2 a = dk[t], c = pf[t];
        const float mult = (m.kz == 0 || m.nyq2) ? 1.f : 2.f;
        const float dg = mult * coef / m.kk * (a.x * c.x + a.y * c.y);
        int b;
        float w;
        const float kt = sqrtf(m.kk) * 0.31830988618379067f;
        const float tt = kt * (float)(NET_NB - 1) / 1.7320508075688772f;
        b = (int)floorf(tt);
        if (b > NET_NB - 2) b = NET_NB - 2;
        w = tt - (float)b;
        atomicAdd(&hist[b], (double)((1.f - w) * dg));
        atomicAdd(&hist[b + 1], (double)(w * dg));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NET_NB; i += blockDim.x)
        if (hist[i] != 0.0) atomicAdd(tbar + i, hist[i]);
}

// F_d = -i k_d phi scale (field 0 holds phi on entry; fields fs apart).
__global__ void k_grad3(float2 *F, int64_t nhp, int64_t fs, int n, float scale)
{
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(t, nhp, n);
        const float2 v = F[t];
        const float f0 = (m.pad || m.nyq0) ? 0.f : m.k0 * scale, f1 = (m.pad || m.nyq1) ? 0.f : m.k1 * scale,
                    f2 = (m.pad || m.nyq2) ? 0.f : m.k2 * scale;
        F[t] = make_float2(f0 * v.y, -f0 * v.x);
        F[fs + t] = make_float2(f1 * v.y, -f1 * v.x);
        F[2 * fs + t] = make_float2(f2 * v.y, -f2 * v.x);
    }
}

// F_d = -i k_d (A + B) scale for the sum of two spectra A (field 1) and B
// (field 2), written to fields 0, 1, 2 (fields fs apart); zero on the
// Nyquist plane of d.
__global__ void k_grad3_sum(float2 *F, int64_t nhp, int64_t fs, int n, float scale)
{
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(t, nhp, n);
        const float2 a = F[fs + t], b = F[2 * fs + t];
        const float2 v = make_float2(a.x + b.x, a.y + b.y);
        const float f0 = (m.pad || m.nyq0) ? 0.f : m.k0 * scale, f1 = (m.pad || m.nyq1) ? 0.f : m.k1 * scale,
                    f2 = (m.pad || m.nyq2) ? 0.f : m.k2 * scale;
        F[t] = make_float2(f0 * v.y, -f0 * v.x);
        F[fs + t] = make_float2(f1 * v.y, -f1 * v.x);
        F[2 * fs + t] = make_float2(f2 * v.y, -f2 * v.x);
    }
}

// Transpose: phibar = sum_d i k_d Fbar_d scale into field 0.
__global__ void k_grad3_t(float2 *F, int64_t nhp, int64_t fs, int n, float scale)
{
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const Mode m = mode_of(t, nhp, n);
        const float f0 = (m.pad || m.nyq0) ? 0.f : m.k0 * scale, f1 = (m.pad || m.nyq1) ? 0.f : m.k1 * scale,
                    f2 = (m.pad || m.nyq2) ? 0.f : m.k2 * scale;
        const float2 a = F[t], b = F[fs + t], c = F[2 * fs + t];
        const float sx = f0 * a.x + f1 * b.x + f2 * c.x, sy = f0 * a.y + f1 * b.y + f2 * c.y;
        F[t] = make_float2(-sy, sx);
    }
}

// ---------------------------------------------------------------- convolutions
// Voxel v = (i0 n + i1) n + i2; tap t = (t0 3 + t1) 3 + t2, offset t_e - 1.
__device__ __forceinline__ int64_t nb_voxel(int i0, int i1, int i2, int t, int n)
{
    const int m = n - 1;
    return ((int64_t)((i0 + t / 9 - 1) & m) * n + ((i1 + (t / 3) % 3 - 1) & m)) * n + ((i2 + t % 3 - 1) & m);
}

// The CNN input: density contrast q 2^-S - 1 of the int64 mesh, rounded to BF16.
__device__ __forceinline__ uint16_t delta_bf16(int64_t q, double qs) { return to_bf16((float)((double)q * qs - 1.0)); }

// conv1: delta (int64 mesh q, quantum qs) rounded to BF16 -> z1 (FP32),
// a1 = SiLU(z1) (BF16), 16 channels per voxel.
__global__ __launch_bounds__(256) void k_conv1_fwd(const int64_t *__restrict__ q, double qs, int n,
                                                   const float *__restrict__ th, float *z1, uint16_t *a1)
{
    __shared__ float W[NET_C * 27], B[NET_C];
    for (int i = threadIdx.x; i < NET_C * 27; i += blockDim.x) W[i] = bf16r(th[NC1W + i]);
    if (threadIdx.x < NET_C) B[threadIdx.x] = th[NC1B + threadIdx.x];
    __syncthreads();
    const int64_t M = (int64_t)n * n * n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < M; v += (int64_t)gridDim.x * blockDim.x) {
        const int i2 = (int)(v % n), i1 = (int)((v / n) % n), i0 = (int)(v / ((int64_t)n * n));
        float x[27];
#pragma unroll
        for (int t = 0; t < 27; t++) {
            x[t] = from_bf16(delta_bf16(q[nb_voxel(i0, i1, i2, t, n)], qs));
        }
        float z[NET_C];
#pragma unroll
        for (int co = 0; co < NET_C; co++) {
            float acc = B[co];
#pragma unroll
            for (int t = 0; t < 27; t++) acc += W[co * 27 + t] * x[t];
            z[co] = acc;
        }
#pragma unroll
        for (int co = 0; co < NET_C; co += 4) {
            *reinterpret_cast<float4 *>(z1 + v * NET_C + co) = make_float4(z[co], z[co + 1], z[co + 2], z[co + 3]);
            const uint32_t lo = (uint32_t)to_bf16(silu(z[co])) | ((uint32_t)to_bf16(silu(z[co + 1])) << 16);
            const uint32_t hi = (uint32_t)to_bf16(silu(z[co + 2])) | ((uint32_t)to_bf16(silu(z[co + 3])) << 16);
            *reinterpret_cast<uint2 *>(a1 + v * NET_C + co) = make_uint2(lo, hi);
        }
    }
}

// conv2 (16 -> 16) on MFMA.  Workgroup tile: 16 (axis 2) x 8 (axis 1) x 4
// (axis 0) voxels with its one-voxel halo in LDS as BF16 [z][y][x][16]; the
// weights as BF16 [tap][co][ci].  Per 16-voxel row and tap one
// v_mfma_f32_16x16x16_bf16: D[co][vox] += W_t[co][ci] X_t[ci][vox] (lane l
// holds A[co = l % 16][ci = 4 (l / 16) + r], B[ci = 4 (l / 16) + r][vox = l % 16]
// and D[co = 4 (l / 16) + r][vox = l % 16]).
constexpr int C2X = 16, C2Y = 8, C2Z = 4, C2HX = C2X + 2, C2HY = C2Y + 2, C2HZ = C2Z + 2;
constexpr int C2HALO = C2HX * C2HY * C2HZ;

__global__ __launch_bounds__(256) void k_conv2_fwd(const uint16_t *__restrict__ a1, int n,
                                                   const float *__restrict__ th, float *z2, uint16_t *a2)
{
    __shared__ __align__(16) uint16_t X[C2HALO * NET_C];
    __shared__ __align__(16) uint16_t W[27 * NET_C * NET_C];
    __shared__ float B[NET_C];
    const int tid = threadIdx.x;
    const int ntx = n / C2X, nty = n / C2Y;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * C2X, y0 = ty * C2Y, z0 = tz * C2Z, m = n - 1;
    // weights [co][ci][t] (FP32) -> LDS [t][co][ci] (BF16)
    for (int e = tid; e < 27 * NET_C * NET_C; e += 256) {
        const int t = e / (NET_C * NET_C), co = (e / NET_C) % NET_C, ci = e % NET_C;
        W[e] = to_bf16(th[NC2W + (co * NET_C + ci) * 27 + t]);
    }
    if (tid < NET_C) B[tid] = th[NC2B + tid];
    // halo tile: two 16-byte chunks per voxel
    for (int e = tid; e < C2HALO * 2; e += 256) {
        const int hv = e >> 1, half = e & 1;
        const int hx = hv % C2HX, hy = (hv / C2HX) % C2HY, hz = hv / (C2HX * C2HY);
        const int64_t g = ((int64_t)((z0 + hz - 1) & m) * n + ((y0 + hy - 1) & m)) * n + ((x0 + hx - 1) & m);
        reinterpret_cast<uint4 *>(X)[hv * 2 + half] = reinterpret_cast<const uint4 *>(a1 + g * NET_C)[half];
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kg = lane >> 4;   // voxel within the row / co and ci group
    for (int row = wave; row < C2Y * C2Z; row += 4) {
        const int ry = row % C2Y, rz = row / C2Y;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
        for (int t = 0; t < 27; t++) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const v4s wa = *reinterpret_cast<const v4s *>(W + (t * NET_C + col) * NET_C + 4 * kg);
            const int hv = ((rz + dz) * C2HY + (ry + dy)) * C2HX + (col + dx);
            const v4s xb = *reinterpret_cast<const v4s *>(X + hv * NET_C + 4 * kg);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa, xb, acc, 0, 0, 0);
        }
        // lane holds D[co = 4 kg + r][vox = col]
        const int64_t v = ((int64_t)(z0 + rz) * n + (y0 + ry)) * n + (x0 + col);
        float zz[4];
        uint16_t aa[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            zz[r] = acc[r] + B[4 * kg + r];
            aa[r] = to_bf16(silu(zz[r]));
        }
        *reinterpret_cast<float4 *>(z2 + v * NET_C + 4 * kg) = make_float4(zz[0], zz[1], zz[2], zz[3]);
        *reinterpret_cast<uint2 *>(a2 + v * NET_C + 4 * kg) =
            make_uint2((uint32_t)aa[0] | ((uint32_t)aa[1] << 16), (uint32_t)aa[2] | ((uint32_t)aa[3] << 16));
    }
}

// conv3 (16 -> 1): out(v) = b + sum_{ci,t} W[ci][t] a2[v + o(t)][ci].
__global__ __launch_bounds__(256) void k_conv3_fwd(const uint16_t *__restrict__ a2, int n,
                                                   const float *__restrict__ th, float *out)
{
    __shared__ float W[27 * NET_C];   // [t][ci]
    for (int e = threadIdx.x; e < 27 * NET_C; e += blockDim.x) {
        const int t = e / NET_C, ci = e % NET_C;
        W[e] = bf16r(th[NC3W + ci * 27 + t]);
    }
    __syncthreads();
    const float b = th[NC3B];
    const int64_t M = (int64_t)n * n * n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < M; v += (int64_t)gridDim.x * blockDim.x) {
        const int i2 = (int)(v % n), i1 = (int)((v / n) % n), i0 = (int)(v / ((int64_t)n * n));
        float acc = b;
        for (int t = 0; t < 27; t++) {
            const int64_t u = nb_voxel(i0, i1, i2, t, n);
            const uint4 *p = reinterpret_cast<const uint4 *>(a2 + u * NET_C);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint4 q = p[h];
                const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int ci = h * 8 + 2 * k;
                    acc += W[t * NET_C + ci] * from_bf16((uint16_t)(w4[k] & 0xffff)) +
                           W[t * NET_C + ci + 1] * from_bf16((uint16_t)(w4[k] >> 16));
                }
            }
        }
        out[v] = acc;
    }
}

// ---- inference path: no pre-activations kept, a1 never leaves LDS
// conv1 + conv2 on v_mfma_f32_16x16x32_bf16 (K = 32; lane l holds
// A[row l % 16][k 8 (l / 16) + j], B[k 8 (l / 16) + j][col l % 16] and
// D[row 4 (l / 16) + r][col l % 16]).  The 16 x 8 x IZ output tile of conv2
// needs a1 on the tile and its one-voxel halo (IHALO voxels); conv1 computes
// those from delta on a two-voxel halo staged in LDS as BF16, one MFMA per 16
// halo voxels: D[co][vox] = W1[co][tap] U[tap][vox] over 32 taps (27 real,
// weights zero past 26).  a1 sits in LDS as two planes of 8 channels (16 bytes
// per voxel), so the 16 lanes of a K group read 256 contiguous bytes.  conv2
// takes two taps per MFMA: k = 8 kg + j is tap 2 p + kg / 2, channel
// 8 (kg % 2) + j, so 14 MFMAs cover 27 taps (the 28th has zero weights); the
// 14 weight fragments live in registers.  Only a2 (BF16) is written.
#ifndef INF_Z
#define INF_Z 8
#endif
// Inference tile: 16 x 8 x IZ outputs on IZ wavefronts (one per z plane of
// conv2's output); the deeper the tile, the less of conv1's two-voxel halo is
// recomputed (2.1x the tile's voxels at IZ = 4, 1.76x at IZ = 8).
constexpr int IZ = INF_Z, INF_T = 64 * IZ, IHZ = IZ + 2, IHALO = C2HX * C2HY * IHZ;
constexpr int U1X = C2X + 4, U1Y = C2Y + 4, U1Z = IZ + 4, U1N = U1X * U1Y * U1Z;
constexpr int NG1 = (IHALO + 15) / 16, NPAIR = 14;
// Inference weights repacked once per call (byte offsets in wpk): conv2 as
// MFMA A fragments [pair][co][kg][8] BF16, conv1 [co][32 taps] BF16, conv3
// [t][ci] BF16.
constexpr int WPK_W2 = 0, WPK_W1 = NPAIR * NET_C * 4 * 8 * 2, WPK_W3 = WPK_W1 + NET_C * 32 * 2,
              WPK_END = WPK_W3 + 27 * NET_C * 2;
static_assert(WPK_END <= NET_WPK_BYTES && WPK_W1 % 16 == 0 && WPK_W3 % 16 == 0, "packed weight layout");

// A grid of PACK_BLOCKS workgroups (one would wait on its strided weight
// reads for 32 rounds).
constexpr int PACK_BLOCKS = 32;
__global__ __launch_bounds__(256) void k_pack_w(const float *__restrict__ th, uint16_t *wpk)
{
    uint16_t *w2 = wpk + WPK_W2 / 2, *w1 = wpk + WPK_W1 / 2, *w3 = wpk + WPK_W3 / 2;
    const int e0 = blockIdx.x * 256 + threadIdx.x, es = PACK_BLOCKS * 256;
    for (int e = e0; e < NPAIR * NET_C * 4 * 8; e += es) {
        const int pr = e / (NET_C * 32), co = (e / 32) % NET_C, kg = (e / 8) % 4, j = e % 8;
        const int t = 2 * pr + kg / 2, ci = 8 * (kg % 2) + j;
        w2[e] = t < 27 ? to_bf16(th[NC2W + (co * NET_C + ci) * 27 + t]) : (uint16_t)0;
    }
    for (int e = e0; e < NET_C * 32; e += es) {
        const int co = e / 32, t = e % 32;
        w1[e] = t < 27 ? to_bf16(th[NC1W + co * 27 + t]) : (uint16_t)0;
    }
    for (int e = e0; e < 27 * NET_C; e += es) {
        const int t = e / NET_C, ci = e % NET_C;
        w3[e] = to_bf16(th[NC3W + ci * 27 + t]);
    }
}

// x / D for 0 <= x < N as one 24-bit multiply and a shift: v_mul_u32_u24 is
// full rate, while the 32-bit multiplies that a division by a constant
// otherwise becomes are quarter rate.  Exactness on the range is checked at
// compile time.
template <unsigned D, unsigned N>
struct Div24 {
    static constexpr unsigned M = (65536u + D - 1) / D;
    static constexpr bool exact()
    {
        for (unsigned x = 0; x < N; x++)
            if (((x * M) >> 16) != x / D) return false;
        return (unsigned long long)N * M < (1ull << 32);
    }
    static_assert(exact(), "multiply-shift division not exact on the range");
    __device__ static __forceinline__ int div(int x)
    {
        // written out, since the compiler turns a 24-bit multiply whose
        // operands it can bound back into the quarter-rate v_mul_lo_u32
        unsigned r;
        asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "s"(M), "v"((unsigned)x));
        return (int)(r >> 16);
    }
};

// Index of voxel (z, y, x) of an n^3 mesh (n <= 4096): the row index in 24-bit
// arithmetic, then one 64-bit multiply-add.
__device__ __forceinline__ int64_t vox_index(int z, int y, int x, int n)
{
    return (int64_t)(unsigned)(__mul24(z, n) + y) * (unsigned)n + (unsigned)x;
}

__device__ __forceinline__ int u1_off(int t) { return ((t / 9) * U1Y + (t / 3) % 3) * U1X + t % 3; }
__device__ __forceinline__ int x_off(int t) { return ((t / 9) * C2HY + (t / 3) % 3) * C2HX + t % 3; }

// SRC int64_t: the fixed-point density, delta = q qs - 1 formed here; SRC
// float: the density contrast as the tile paint stores it (the same value).
template <typename SRC>
__global__ __launch_bounds__(INF_T) void k_cnn12_inf(const SRC *__restrict__ q, double qs, int n,
                                                   const float *__restrict__ th, const uint16_t *__restrict__ wpk,
                                                   uint16_t *a2)
{
    __shared__ __align__(16) uint16_t U[U1N];
    __shared__ __align__(16) uint4 X[2 * IHALO];   // channel planes 0-7 and 8-15
    const int tid = threadIdx.x;
    const int ntx = n / C2X, nty = n / C2Y;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * C2X, y0 = ty * C2Y, z0 = tz * IZ, m = n - 1;
    const int lane = tid & 63, wave = tid >> 6;
    constexpr int NW = INF_T / 64;   // wavefronts
    const int col = lane & 15, kg = lane >> 4;
    // weight fragments straight from the packed buffer (L2-resident)
    const v8bf w1 = *reinterpret_cast<const v8bf *>(wpk + WPK_W1 / 2 + col * 32 + 8 * kg);
    v8bf wa[NPAIR];
#pragma unroll
    for (int pr = 0; pr < NPAIR; pr++)
        wa[pr] = *reinterpret_cast<const v8bf *>(wpk + WPK_W2 / 2 + ((pr * NET_C + col) * 4 + kg) * 8);
    {
        // every load of the halo fill issued before the first LDS store (one
        // memory round trip per tile rather than one per round); indices past
        // the end are clamped, and the empty asm keeps the loads from being
        // sunk into the guarded stores
        constexpr int NU = (U1N + INF_T - 1) / INF_T;
        SRC qv[NU];
#pragma unroll
        for (int k = 0; k < NU; k++) {
            const int e = min(tid + INF_T * k, U1N - 1);
            const int eq = Div24<U1X, U1N>::div(e), uz = Div24<U1Y, U1N / U1X>::div(eq);
            const int ux = e - __mul24(eq, U1X), uy = eq - __mul24(uz, U1Y);
            qv[k] = q[vox_index((z0 + uz - 2) & m, (y0 + uy - 2) & m, (x0 + ux - 2) & m, n)];
        }
#pragma unroll
        for (int k = 0; k < NU; k++) asm volatile("" : "+v"(qv[k]));
#pragma unroll
        for (int k = 0; k < NU; k++) {
            const int e = tid + INF_T * k;
            if constexpr (std::is_same<SRC, int64_t>::value) {
                if (e < U1N) U[e] = delta_bf16(qv[k], qs);
            } else {
                if (e < U1N) U[e] = to_bf16(qv[k]);
            }
        }
    }
    __syncthreads();
    {
        // taps 27..31 read a real voxel (tap 26's) against zero weights, so
        // every lane's eight reads are unconditional (no exec-mask branches)
        int ou[8];
#pragma unroll
        for (int j = 0; j < 8; j++) ou[j] = u1_off(8 * kg + j < 27 ? 8 * kg + j : 26);
        float bias[4];
#pragma unroll
        for (int r = 0; r < 4; r++) bias[r] = th[NC1B + 4 * kg + r];
        for (int g = wave; g < NG1; g += NW) {
            const int hv = g * 16 + col;
            const int hc = hv < IHALO ? hv : IHALO - 1;
            const int hq = Div24<C2HX, IHALO>::div(hc), hz = Div24<C2HY, IHALO / C2HX>::div(hq);
            const int hx = hc - __mul24(hq, C2HX), hy = hq - __mul24(hz, C2HY);
            const int base = __mul24(__mul24(hz, U1Y) + hy, U1X) + hx;
            v8bf b;
#pragma unroll
            for (int j = 0; j < 8; j++) b[j] = __builtin_bit_cast(__bf16, U[base + ou[j]]);
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, b, acc, 0, 0, 0);
            // lane holds D[co = 4 kg + r][vox = col]: channels 4 kg .. 4 kg + 3
            if (hv < IHALO) {
                uint16_t aa[4];
#pragma unroll
                for (int r = 0; r < 4; r++) aa[r] = to_bf16(silu(acc[r] + bias[r]));
                reinterpret_cast<uint2 *>(X + (kg >> 1) * IHALO + hv)[kg & 1] =
                    make_uint2((uint32_t)aa[0] | ((uint32_t)aa[1] << 16), (uint32_t)aa[2] | ((uint32_t)aa[3] << 16));
            }
        }
    }
    __syncthreads();
    int ox[NPAIR];
#pragma unroll
    for (int pr = 0; pr < NPAIR; pr++) {
        const int t = 2 * pr + (kg >> 1);
        ox[pr] = x_off(t < 27 ? t : 26);   // the 28th tap reads real data against zero weights
    }
    // wavefront w computes the output rows y = w of every z plane: with the
    // loop unrolled, a row's LDS offsets are the loop-invariant lane offsets
    // plus an immediate, and the output pointer steps by one plane
    static_assert(NW == C2Y, "one wavefront per output row of a plane");
    const uint4 *Xp = X + (kg & 1) * IHALO + wave * C2HX + col;
    float bias[4];
#pragma unroll
    for (int r = 0; r < 4; r++) bias[r] = th[NC2B + 4 * kg + r];
    uint16_t *out = a2 + ((((int64_t)z0 * n + (y0 + wave)) * n + (x0 + col)) * NET_C + 4 * kg);
    const int64_t plane_step = (int64_t)n * n * NET_C;
#pragma unroll
    for (int rz = 0; rz < IZ; rz++) {
        const uint4 *xr = Xp + rz * (C2HY * C2HX);
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int pr = 0; pr < NPAIR; pr++) {
            const v8bf xb = __builtin_bit_cast(v8bf, xr[ox[pr]]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[pr], xb, acc, 0, 0, 0);
        }
        uint16_t aa[4];
#pragma unroll
        for (int r = 0; r < 4; r++) aa[r] = to_bf16(silu(acc[r] + bias[r]));
        *reinterpret_cast<uint2 *>(out) =
            make_uint2((uint32_t)aa[0] | ((uint32_t)aa[1] << 16), (uint32_t)aa[2] | ((uint32_t)aa[3] << 16));
        out += plane_step;
    }
}

// conv3 fused with the combination: out = phi_f + b3 + conv3(a2) on
// real rows of stride rs.  Tile 16 x 16 x 4 with a2's one-voxel halo in LDS;
// a thread owns a column of 4 voxels along axis 0, so each halo voxel it reads
// feeds up to three taps.
// Tile 16 x TY x TZ with a2's one-voxel halo in LDS; 256 threads, each owning
// ZPT consecutive voxels along axis 0 of one (axis 1, axis 2) column, so each
// halo voxel it reads feeds up to three taps.
template <int TY, int TZ, int ZPT>
__global__ __launch_bounds__(256) void k_conv3_inf(const uint16_t *__restrict__ a2, int n,
                                                   const float *__restrict__ th, const uint16_t *__restrict__ wpk,
                                                   const float *__restrict__ phif, int64_t rs, float *out)
{
    static_assert(16 * TY * (TZ / ZPT) == 256 && TZ % ZPT == 0, "conv3 tile shape");
    constexpr int HX = 18, HY = TY + 2, HZ = TZ + 2, HALO = HX * HY * HZ;
    // channel halves of each halo voxel in two planes: 16-byte rows, no bank conflicts
    // + one slot per lane after the two planes (stores of idle fill tasks)
    __shared__ __align__(16) uint4 X[2 * HALO + 64];
    __shared__ __align__(16) uint32_t W[27 * NET_C / 2];   // BF16 pairs [t][ci / 2]
    const int tid = threadIdx.x;
    const int ntx = n / 16, nty = n / TY;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * 16, y0 = ty * TY, z0 = tz * TZ, m = n - 1;
    const int lx = tid % 16, ly = (tid / 16) % TY, zg = tid / (16 * TY);
    // phi_f of the thread's voxels, loaded now rather than after the sums
    float pf[ZPT];
#pragma unroll
    for (int z = 0; z < ZPT; z++)
        pf[z] = phif ? phif[((int64_t)(z0 + zg * ZPT + z) * n + (y0 + ly)) * rs + (x0 + lx)] : 0.f;
    {
        // Every load of the halo fill is issued before the first LDS store
        // (one memory round trip per tile, not one per round).  Indices past
        // the end are clamped, and those lanes store to their own slot after
        // the tile, so no store is guarded (a guarded store would let the
        // compiler sink its load into the guard).
        constexpr int NX = (HALO * 2 + 255) / 256;
        uint4 xv[NX];
#pragma unroll
        for (int k = 0; k < NX; k++) {
            const int e = min(tid + 256 * k, HALO * 2 - 1);
            const int hv = e >> 1, half = e & 1;
            const int hq = Div24<HX, HALO>::div(hv), hz = Div24<HY, HALO / HX>::div(hq);
            const int hx = hv - __mul24(hq, HX), hy = hq - __mul24(hz, HY);
            const int64_t g = vox_index((z0 + hz - 1) & m, (y0 + hy - 1) & m, (x0 + hx - 1) & m, n);
            xv[k] = reinterpret_cast<const uint4 *>(a2 + g * NET_C)[half];
        }
        // the conv3 weights, one 16-byte row per thread, unconditional like
        // the halo (lanes past the last row store to their slot after the tile)
        constexpr int NW = 27 * NET_C / 8;
        static_assert(NW <= 256, "one weight row per thread");
        const uint4 wv = reinterpret_cast<const uint4 *>(wpk + WPK_W3 / 2)[min(tid, NW - 1)];
        *(tid < NW ? reinterpret_cast<uint4 *>(W) + tid : X + 2 * HALO + (tid & 63)) = wv;
#pragma unroll
        for (int k = 0; k < NX; k++) {
            const int e = tid + 256 * k;
            X[e < HALO * 2 ? (e & 1) * HALO + (e >> 1) : 2 * HALO + (tid & 63)] = xv[k];
        }
    }
    __syncthreads();
    const float b = th[NC3B];
    float acc[ZPT];
#pragma unroll
    for (int z = 0; z < ZPT; z++) acc[z] = b;
#pragma unroll 1
    for (int t2 = 0; t2 < 9; t2++) {
        const int dy = t2 / 3, dx = t2 % 3;
        uint32_t w[3][NET_C / 2];
#pragma unroll
        for (int dz = 0; dz < 3; dz++)
#pragma unroll
            for (int k = 0; k < NET_C / 2; k++) w[dz][k] = W[(dz * 9 + t2) * (NET_C / 2) + k];
        const int h0 = (zg * ZPT * HY + ly + dy) * HX + lx + dx;
#pragma unroll
        for (int j = 0; j < ZPT + 2; j++) {
            const int hv = h0 + j * HY * HX;
            const uint4 q0 = X[hv], q1 = X[HALO + hv];
            const uint32_t xv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int dz = 0; dz < 3; dz++) {
                const int lz = j - dz;
                if (lz < 0 || lz >= ZPT) continue;
                float sum = acc[lz];
#pragma unroll
                for (int k = 0; k < NET_C / 2; k++) sum = dot2_bf16(w[dz][k], xv[k], sum);
                acc[lz] = sum;
            }
        }
    }
#pragma unroll
    for (int z = 0; z < ZPT; z++) {
        const int64_t o = ((int64_t)(z0 + zg * ZPT + z) * n + (y0 + ly)) * rs + (x0 + lx);
        out[o] = pf[z] + acc[z];
    }
}

// Measured at 256^3 (one MI355X): 16 x 8 x 4 with two voxels per thread
// (35 KB of LDS, four workgroups per CU) 306 us; 16 x 16 x 4 with four per
// thread (63 KB, two per CU) 418 us; one voxel per thread 360 us.
constexpr int C3TY = 8, C3TZ = 4, C3ZPT = 2;

// phi = phi_f + dpsi on real rows of stride rs.
__global__ void k_combine(const float *phif, const float *dpsi, int64_t rs, int n, float *out)
{
    const int64_t M = (int64_t)n * n * n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < M; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (v / n) * rs + v % n;
        out[o] = phif[o] + dpsi[v];
    }
}

// ---- reverse mode of the CNN
// conv3 data: g2[v][ci] = dsilu(z2[v][ci]) sum_t W3[ci][t] phibar(v - o(t)),
// phibar on real rows of stride rs.
__global__ __launch_bounds__(256) void k_conv3_bwd_data(const float *__restrict__ phibar, int64_t rs, int n,
                                                        const float *__restrict__ th,
                                                        const float *__restrict__ z2, float *g2)
{
    __shared__ float W[27 * NET_C];   // [t][ci]
    for (int e = threadIdx.x; e < 27 * NET_C; e += blockDim.x) {
        const int t = e / NET_C, ci = e % NET_C;
        W[e] = bf16r(th[NC3W + ci * 27 + t]);
    }
    __syncthreads();
    const int64_t M = (int64_t)n * n * n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < M; v += (int64_t)gridDim.x * blockDim.x) {
        const int i2 = (int)(v % n), i1 = (int)((v / n) % n), i0 = (int)(v / ((int64_t)n * n));
        float acc[NET_C];
#pragma unroll
        for (int c = 0; c < NET_C; c++) acc[c] = 0.f;
        for (int t = 0; t < 27; t++) {
            const int64_t u = nb_voxel(i0, i1, i2, 26 - t, n);   // v - o(t)
            const float d = phibar[(u / n) * rs + u % n];
#pragma unroll
            for (int c = 0; c < NET_C; c++) acc[c] += W[t * NET_C + c] * d;
        }
#pragma unroll
        for (int c = 0; c < NET_C; c += 4) {
            const float4 z = *reinterpret_cast<const float4 *>(z2 + v * NET_C + c);
            *reinterpret_cast<float4 *>(g2 + v * NET_C + c) =
                make_float4(acc[c] * dsilu(z.x), acc[c + 1] * dsilu(z.y), acc[c + 2] * dsilu(z.z),
                            acc[c + 3] * dsilu(z.w));
        }
    }
}

// conv2 data: g1[v][ci] = dsilu(z1[v][ci]) sum_{co,t} W2[co][ci][t] g2[v - o(t)][co].
__global__ __launch_bounds__(256) void k_conv2_bwd_data(const float *__restrict__ g2, int n,
                                                        const float *__restrict__ th,
                                                        const float *__restrict__ z1, float *g1)
{
    __shared__ float W[27 * NET_C * NET_C];   // [t][co][ci]
    for (int e = threadIdx.x; e < 27 * NET_C * NET_C; e += blockDim.x) {
        const int t = e / (NET_C * NET_C), co = (e / NET_C) % NET_C, ci = e % NET_C;
        W[e] = bf16r(th[NC2W + (co * NET_C + ci) * 27 + t]);
    }
    __syncthreads();
    const int64_t M = (int64_t)n * n * n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < M; v += (int64_t)gridDim.x * blockDim.x) {
        const int i2 = (int)(v % n), i1 = (int)((v / n) % n), i0 = (int)(v / ((int64_t)n * n));
        float acc[NET_C];
#pragma unroll
        for (int c = 0; c < NET_C; c++) acc[c] = 0.f;
        for (int t = 0; t < 27; t++) {
            const int64_t u = nb_voxel(i0, i1, i2, 26 - t, n);
            const float4 *gp = reinterpret_cast<const float4 *>(g2 + u * NET_C);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 gv = gp[q];
                const float gg[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int co = 4 * q + r;
#pragma unroll
                    for (int c = 0; c < NET_C; c++) acc[c] += W[(t * NET_C + co) * NET_C + c] * gg[r];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NET_C; c += 4) {
            const float4 z = *reinterpret_cast<const float4 *>(z1 + v * NET_C + c);
            *reinterpret_cast<float4 *>(g1 + v * NET_C + c) =
                make_float4(acc[c] * dsilu(z.x), acc[c + 1] * dsilu(z.y), acc[c + 2] * dsilu(z.z),
                            acc[c + 3] * dsilu(z.w));
        }
    }
}

// Weight gradients dW[co][ci][t] += sum_v in_ci(v + o(t)) dout_co(v), db[co] += sum_v dout_co(v).
// in: KIN 0 = the int64 density mesh as BF16 delta (quantum qs: the conv1 input),
//     KIN 1 = BF16 [v][16]; dout: KOUT 0 = real rows of stride rs_out (conv3), KOUT 1 = FP32 [v][16].
// A workgroup walks tiles of 16 x 8 x 4 voxels with LDS copies of the input
// halo and the output gradient; each thread owns CO CI 27 / 256 entries.
template <int CI, int CO, int KIN, int KOUT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const void *in_, double qs, const void *dout_, int64_t rs_out,
                                                    int n, float *dW, float *db)
{
    constexpr int NE = CO * CI * 27, PER = (NE + 255) / 256;
    __shared__ float Xs[C2HALO * CI];
    __shared__ float Gs[C2X * C2Y * C2Z * CO];
    const int tid = threadIdx.x, m = n - 1;
    const int ntx = n / C2X, nty = n / C2Y, ntz = n / C2Z, ntiles = ntx * nty * ntz;
    float acc[PER], bacc = 0.f;
#pragma unroll
    for (int k = 0; k < PER; k++) acc[k] = 0.f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
        const int x0 = tx * C2X, y0 = ty * C2Y, z0 = tz * C2Z;
        __syncthreads();
        for (int e = tid; e < C2HALO * CI; e += 256) {
            const int hv = e / CI, ci = e % CI;
            const int hx = hv % C2HX, hy = (hv / C2HX) % C2HY, hz = hv / (C2HX * C2HY);
            const int64_t g = ((int64_t)((z0 + hz - 1) & m) * n + ((y0 + hy - 1) & m)) * n + ((x0 + hx - 1) & m);
            float val;
            if constexpr (KIN == 0)
                val = from_bf16(delta_bf16(reinterpret_cast<const int64_t *>(in_)[g], qs));
            else
                val = from_bf16(reinterpret_cast<const uint16_t *>(in_)[g * CI + ci]);
            Xs[e] = val;
        }
        for (int e = tid; e < C2X * C2Y * C2Z * CO; e += 256) {
            const int lv = e / CO, co = e % CO;
            const int lx = lv % C2X, ly = (lv / C2X) % C2Y, lz = lv / (C2X * C2Y);
            const int64_t g = ((int64_t)(z0 + lz) * n + (y0 + ly)) * n + (x0 + lx);
            float val;
            if constexpr (KOUT == 0)
                val = reinterpret_cast<const float *>(dout_)[(g / n) * rs_out + g % n];
            else
                val = reinterpret_cast<const float *>(dout_)[g * CO + co];
            Gs[e] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int e = tid + 256 * k;
            if (e < NE) {
                const int co = e / (CI * 27), ci = (e / 27) % CI, t = e % 27;
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                float s = 0.f;
                for (int lz = 0; lz < C2Z; lz++)
                    for (int ly = 0; ly < C2Y; ly++)
                        for (int lx = 0; lx < C2X; lx++) {
                            const int hv = ((lz + dz) * C2HY + (ly + dy)) * C2HX + (lx + dx);
                            const int lv = (lz * C2Y + ly) * C2X + lx;
                            s += Xs[hv * CI + ci] * Gs[lv * CO + co];
                        }
                acc[k] += s;
            }
        }
        if (tid < CO) {
            float s = 0.f;
            for (int lv = 0; lv < C2X * C2Y * C2Z; lv++) s += Gs[lv * CO + tid];
            bacc += s;
        }
    }
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int e = tid + 256 * k;
        if (e < NE) atomicAdd(dW + e, acc[k]);
    }
    if (tid < CO) atomicAdd(db + tid, bacc);
}

// ---- loss and optimiser
// red[0] += sum (acc - target)^2, red[1] += sum target^2; acc -= target.
__global__ __launch_bounds__(256) void k_force_loss(float *acc, const float *target, int64_t n3, double *red)
{
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = acc[i] - target[i];
        a += (double)d * d;
        b += (double)target[i] * target[i];
        acc[i] = d;
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(red, sa[0]);
        atomicAdd(red + 1, sb[0]);
    }
}

// Adam with bias correction (FP32 master weights).
__global__ void k_adam(float *th, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_zero_f64(double *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

}  // namespace

hipError_t launch_mlp_fwd(const float *th, double a, float *table, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_fwd, dim3(NET_NB), dim3(128), 0, s, th, (float)a, table);
    return hipGetLastError();
}

hipError_t launch_mlp_bwd(const float *th, double a, const double *tbar, float *dth, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_bwd, dim3(NET_NB), dim3(128), 0, s, th, (float)a, tbar, dth);
    return hipGetLastError();
}

hipError_t launch_spec_filter(const float2 *in, float2 *out, int64_t nhp, int n, const float *table, double coef,
                              hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    hipLaunchKernelGGL(k_spec_filter, dim3(grid_for(tot, 256, 4096)), dim3(256), 0, s, in, out, nhp, n, table,
                       (float)coef);
    return hipGetLastError();
}

hipError_t launch_spec_filter_bwd(const float2 *dk, const float2 *pf, int64_t nhp, int n, double coef, double *tbar,
                                  hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, tbar, NET_NB);
    hipLaunchKernelGGL(k_spec_filter_bwd, dim3(grid_for(tot, 256, 1024)), dim3(256), 0, s, dk, pf, nhp, n,
                       (float)coef, tbar);
    return hipGetLastError();
}

hipError_t launch_grad3_sum(float2 *F, int64_t nhp, int64_t fs, int n, double scale, hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    hipLaunchKernelGGL(k_grad3_sum, dim3(grid_for(tot, 256)), dim3(256), 0, s, F, nhp, fs, n, (float)scale);
    return hipGetLastError();
}

hipError_t launch_grad3(float2 *F, int64_t nhp, int64_t fs, int n, double scale, bool transpose, hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    if (transpose)
        hipLaunchKernelGGL(k_grad3_t, dim3(grid_for(tot, 256)), dim3(256), 0, s, F, nhp, fs, n, (float)scale);
    else
        hipLaunchKernelGGL(k_grad3, dim3(grid_for(tot, 256)), dim3(256), 0, s, F, nhp, fs, n, (float)scale);
    return hipGetLastError();
}

hipError_t launch_cnn_fwd(const int64_t *q, double qs, int n, const float *th, float *z1, uint16_t *a1, float *z2,
                          uint16_t *a2, float *dpsi, hipStream_t s)
{
    if (n < C2X || n % C2X) return hipErrorInvalidValue;
    const int64_t M = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_conv1_fwd, dim3(grid_for(M, 256)), dim3(256), 0, s, q, qs, n, th, z1, a1);
    hipLaunchKernelGGL(k_conv2_fwd, dim3((unsigned)(M / (C2X * C2Y * C2Z))), dim3(256), 0, s, a1, n, th, z2, a2);
    hipLaunchKernelGGL(k_conv3_fwd, dim3(grid_for(M, 256)), dim3(256), 0, s, a2, n, th, dpsi);
    return hipGetLastError();
}

hipError_t launch_cnn_inf(const int64_t *q, double qs, const float *delta, const float *phif, int64_t rs, int n,
                          const float *th, uint16_t *wpk, uint16_t *a2, float *out, hipStream_t s)
{
    if (n < 16 || n % 16 || n > 4096) return hipErrorInvalidValue;
    const int64_t M = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_pack_w, dim3(PACK_BLOCKS), dim3(256), 0, s, th, wpk);
    if (delta)
        hipLaunchKernelGGL(k_cnn12_inf<float>, dim3((unsigned)(M / (C2X * C2Y * IZ))), dim3(INF_T), 0, s, delta, qs, n,
                           th, wpk, a2);
    else
        hipLaunchKernelGGL(k_cnn12_inf<int64_t>, dim3((unsigned)(M / (C2X * C2Y * IZ))), dim3(INF_T), 0, s, q, qs, n,
                           th, wpk, a2);
    hipLaunchKernelGGL((k_conv3_inf<C3TY, C3TZ, C3ZPT>), dim3((unsigned)(M / (16 * C3TY * C3TZ))), dim3(256), 0, s, a2,
                       n, th, wpk, phif, rs, out);
    return hipGetLastError();
}

hipError_t launch_combine(const float *phif, const float *dpsi, int64_t rs, int n, float *out, hipStream_t s)
{
    const int64_t M = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(M, 256)), dim3(256), 0, s, phif, dpsi, rs, n, out);
    return hipGetLastError();
}

hipError_t launch_cnn_bwd(const int64_t *q, double qs, const float *phibar, int64_t rs, int n, const float *th,
                          const float *z1, const uint16_t *a1, const float *z2, const uint16_t *a2, float *g1,
                          float *g2, float *dth, hipStream_t s)
{
    if (n < C2X || n % C2X) return hipErrorInvalidValue;
    const int64_t M = (int64_t)n * n * n;
    const int ntiles = (int)(M / (C2X * C2Y * C2Z));
    const unsigned gw = (unsigned)(ntiles < 2048 ? ntiles : 2048);
    // conv3: dW3, db3 from a2 and phibar; g2 = dsilu(z2) W3^T phibar
    hipLaunchKernelGGL((k_conv_bwd_w<NET_C, 1, 1, 0>), dim3(gw), dim3(256), 0, s, (const void *)a2, 0.0,
                       (const void *)phibar, rs, n, dth + NC3W, dth + NC3B);
    hipLaunchKernelGGL(k_conv3_bwd_data, dim3(grid_for(M, 256)), dim3(256), 0, s, phibar, rs, n, th, z2, g2);
    // conv2
    hipLaunchKernelGGL((k_conv_bwd_w<NET_C, NET_C, 1, 1>), dim3(gw), dim3(256), 0, s, (const void *)a1, 0.0,
                       (const void *)g2, (int64_t)0, n, dth + NC2W, dth + NC2B);
    hipLaunchKernelGGL(k_conv2_bwd_data, dim3(grid_for(M, 256)), dim3(256), 0, s, g2, n, th, z1, g1);
    // conv1 weights from delta; delta does not depend on the parameters
    hipLaunchKernelGGL((k_conv_bwd_w<1, NET_C, 0, 1>), dim3(gw), dim3(256), 0, s, (const void *)q, qs,
                       (const void *)g1, (int64_t)0, n, dth + NC1W, dth + NC1B);
    return hipGetLastError();
}

hipError_t launch_force_loss(float *acc, const float *target, int64_t n3, double *red, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, red, 2);
    hipLaunchKernelGGL(k_force_loss, dim3(grid_for(n3, 256, 2048)), dim3(256), 0, s, acc, target, n3, red);
    return hipGetLastError();
}

hipError_t launch_adam(float *th, float *m, float *v, const float *g, int64_t n, double lr, double b1, double b2,
                       double eps, int t, hipStream_t s)
{
    const float c1 = (float)(1.0 - pow(b1, t)), c2 = (float)(1.0 - pow(b2, t));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256)), dim3(256), 0, s, th, m, v, g, n, (float)lr, (float)b1,
                       (float)b2, (float)eps, c1, c2);
    return hipGetLastError();
}

}  // namespace pm
