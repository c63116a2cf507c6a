// Mesh FFT passes for the particle-mesh Poisson solve on gfx950.
//
// The 3D transform of an N^3 mesh (i0, i1, i2; i2 contiguous) is done as
// three passes, each one HBM read and one HBM write of the mesh:
//   * rows (axis 2): real-to-complex of every contiguous row, computed as an
//     N/2-point complex FFT of the even/odd samples packed as (re, im) plus a
//     split step; the int64 fixed-point density is converted to the density
//     contrast on the fly.  The complex-to-real inverse mirrors it.
//   * columns (axis 1): tiles of TILE_W contiguous complex columns (64 bytes)
//     x N rows are staged in LDS and transformed along the strided axis.
//   * axis 0: the same column tiles, forward transform, then for each output
//     a per-mode multiplier (the gradient of the inverse Laplacian, or the
//     initial-condition transfer function) and an inverse transform, so the
//     forward spectrum is read once and the k-space multiply never touches
//     HBM on its own.  For the force solve at N >= 256, where a 64-byte
//     column tile would touch a different 2 MiB page on every row, axis 0 is
//     instead split into a 16-point pass over strided planes and an N/16-point
//     pass over consecutive planes fused with the multiplier (see below).
// Transforms inside LDS are Stockham autosort stages of radix 2..16 held in
// registers (two barriers per stage, in place), twiddles from an FP64-derived
// table.  Consecutive workgroups are spread over the eight XCDs by the
// hardware, so tiles are renumbered to give each XCD a contiguous run of
// tiles (neighbouring 64-byte half lines then meet in the same L2).
#include <type_traits>

#include "pm_internal.h"

namespace pm {
namespace {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// cos(2 pi j / 64), exact quarter-wave symmetry
constexpr float c64q(int j)
{
    switch (j) {
    case 0: return 1.0f;
    case 1: return 0.99518472667219693f;
    case 2: return 0.98078528040323043f;
    case 3: return 0.95694033573220882f;
    case 4: return 0.92387953251128674f;
    case 5: return 0.88192126434835505f;
    case 6: return 0.83146961230254524f;
    case 7: return 0.77301045336273699f;
    case 8: return 0.70710678118654757f;
    case 9: return 0.63439328416364549f;
    case 10: return 0.55557023301960229f;
    case 11: return 0.47139673682599781f;
    case 12: return 0.38268343236508984f;
    case 13: return 0.29028467725446233f;
    case 14: return 0.19509032201612833f;
    case 15: return 0.09801714032956077f;
    default: return 0.0f;
    }
}
constexpr float c64(int j)
{
    j &= 63;
    return j <= 16 ? c64q(j) : (j <= 32 ? -c64q(32 - j) : (j <= 48 ? -c64q(j - 32) : c64q(64 - j)));
}

// a * exp(-/+ 2 pi i j / 64) (minus for the forward transform)
template <bool INV>
__device__ __forceinline__ float2 rot64(float2 a, int j)
{
    j &= 63;
    if (j == 0) return a;
    if (j == 32) return make_float2(-a.x, -a.y);
    if (j == 16) return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    if (j == 48) return INV ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    const float c = c64(j), s = INV ? c64(j - 16) : -c64(j - 16);
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// In-register DFT of size R <= 64 (natural order in and out), radix-2 recursion.
template <int R, bool INV>
struct Dft {
    __device__ __forceinline__ static void run(float2 *v)
    {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; i++) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2, INV>::run(e);
        Dft<R / 2, INV>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; k++) {
            const float2 t = rot64<INV>(o[k], k * (64 / R));
            v[k] = cadd(e[k], t);
            v[k + R / 2] = csub(e[k], t);
        }
    }
};
template <bool INV>
struct Dft<1, INV> {
    __device__ __forceinline__ static void run(float2 *) {}
};

// LDS index of element i.  PS > 0: one pad slot per 2^PS elements.  A
// Stockham stage writes its outputs R elements apart; with 8-byte elements
// and a stride of 16 every lane of a wavefront would hit the same bank pair.
// PS < 0 (tiles of 8 columns, element (c, l) at 8 l + c): bits 0-1 of the row
// l are XORed with bits -PS-3 .. -PS-2 of it.  The first stage's writes, rows
// R apart (-PS = 3 + log2 R), then spread over four groups of eight bank
// pairs, and aligned groups of four rows only permute, so consecutive
// accesses stay conflict-free; no extra LDS.
//
// PS == SWZ_ROWS (rows of N/2 complex, one per Stockham transform, radix
// 16/8/8): bits 0-4 of i are XORed with bits 4-8 and bit 4 also with bit 7.
// Within aligned groups of 32 elements this only permutes, so consecutive
// accesses stay conflict-free, and the strided writes of every stage spread
// over all bank pairs, with no extra LDS.
constexpr int SWZ_ROWS = 32;
template <int PS>
__device__ __forceinline__ int pad(int i)
{
    if constexpr (PS == SWZ_ROWS) return i ^ ((i >> 4) & 31) ^ (((i >> 7) & 1) << 4);
    else if constexpr (PS > 0) return i + (i >> PS);
    else if constexpr (PS < 0) return i ^ (((i >> (-PS)) & 3) << 3);
    else return i;
}
constexpr int padded(int n, int ps) { return ps > 0 && ps != SWZ_ROWS ? n + (n >> ps) + 1 : n; }

// One Stockham stage of radix R over NC independent transforms of length L
// held in LDS: element (c, l) at buf[c * SC + l * SL].  NS = product of the
// radices already applied.  All butterflies of a thread are read before the
// barrier and written after it, so the stage runs in place.
template <int L, int R, int NS, int NC, int T, bool COLMAJ, int SL, int SC, bool INV, int PS = 0>
__device__ __forceinline__ void stage(float2 *buf, const float2 *__restrict__ twL)
{
    constexpr int NB = NC * (L / R);
    constexpr int PER = (NB + T - 1) / T;
    float2 v[PER][R];
    int dst[PER];
    const int tid = threadIdx.x;
#pragma unroll
    for (int b = 0; b < PER; b++) {
        const int bf = tid + b * T;
        if ((NB % T == 0) || bf < NB) {
            int c, j;
            if (COLMAJ) {
                c = bf % NC;
                j = bf / NC;
            } else {
                j = bf % (L / R);
                c = bf / (L / R);
            }
            const int k = j & (NS - 1);
#pragma unroll
            for (int r = 0; r < R; r++) v[b][r] = buf[pad<PS>(c * SC + (j + r * (L / R)) * SL)];
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; r++) {
                    float2 w = twL[r * k * (L / (NS * R))];
                    if (INV) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            Dft<R, INV>::run(v[b]);
            dst[b] = c * SC + ((j / NS) * NS * R + k) * SL;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; b++) {
        const int bf = tid + b * T;
        if ((NB % T == 0) || bf < NB) {
#pragma unroll
            for (int r = 0; r < R; r++) buf[pad<PS>(dst[b] + r * NS * SL)] = v[b][r];
        }
    }
    __syncthreads();
}

// Full transform: stages of at most 2^MAXB, bits split as evenly as possible.
template <int L, int NS, int NC, int T, bool COLMAJ, int SL, int SC, bool INV, int MAXB, int PS = 0>
__device__ __forceinline__ void fft_from(float2 *buf, const float2 *__restrict__ twL)
{
    if constexpr (NS < L) {
        constexpr int rem = ilog2c(L / NS);
        constexpr int nst = (rem + MAXB - 1) / MAXB;
        constexpr int bits = (rem + nst - 1) / nst;
        constexpr int R = 1 << bits;
        stage<L, R, NS, NC, T, COLMAJ, SL, SC, INV, PS>(buf, twL);
        fft_from<L, NS * R, NC, T, COLMAJ, SL, SC, INV, MAXB, PS>(buf, twL);
    }
}

template <int LOGN>
struct RowCfg {
    static constexpr int N = 1 << LOGN, L = N / 2;
    static constexpr int RB = (8192 / N) < (N * N) ? (8192 / N) : (N * N);
    static constexpr int T = 256;
};

template <int LOGN, int WW = TILE_W>
struct ColCfg {
    static constexpr int N = 1 << LOGN, W = WW, E = N * W;
    // 16 elements per thread (at least one wavefront): keeps a tile's
    // register footprint below the 128-VGPR budget of 16 waves per CU.
    static constexpr int T = (E / 16) > 64 ? ((E / 16) < 1024 ? (E / 16) : 1024) : 64;
    static constexpr int PER = E / T;
    // log2 of the first stage's radix (stages of at most 2^4, bits split evenly)
    static constexpr int R1 = (LOGN + (LOGN + 3) / 4 - 1) / ((LOGN + 3) / 4);
};

// The axis-0 pass keeps part of a spectrum in registers across an inverse
// transform; stages of radix <= 8 (AX0_MAXB) and 16 elements per thread keep
// it within the 128-VGPR budget of 16 waves per CU.
template <int LOGN>
struct Ax0Cfg {
    static constexpr int N = 1 << LOGN, W = TILE_W, E = N * W;
    static constexpr int T = (E / 16) > 64 ? ((E / 16) < 1024 ? (E / 16) : 1024) : 64;
    static constexpr int PER = E / T;
};
constexpr int AX0_MAXB = 3;

// ---------------------------------------------------------------- rows
template <int LOGN, typename SRC>
__global__ __launch_bounds__(256) void k_r2c_rows(const SRC *src, int64_t src_stride,
                                                  float2 *dst, int64_t dst_stride, double scale,
                                                  double offset, const float2 *__restrict__ tw, int *flag)
{
    using C = RowCfg<LOGN>;
    constexpr int N = C::N, L = C::L, RB = C::RB, T = C::T;
    __shared__ float2 buf[RB * L];
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    const int tid = threadIdx.x;
    bool bad = false;
#pragma unroll 8
    for (int e = tid; e < RB * L; e += T) {
        const int r = e / L, m = e % L;
        const SRC *s = src + (row0 + r) * src_stride + 2 * m;
        float a, b;
        if constexpr (std::is_same<SRC, int64_t>::value) {
            const longlong2 q = *reinterpret_cast<const longlong2 *>(s);
            bad |= (q.x < GUARD_MIN_Q) | (q.y < GUARD_MIN_Q);
            a = (float)((double)q.x * scale + offset);
            b = (float)((double)q.y * scale + offset);
        } else {
            const float2 q = *reinterpret_cast<const float2 *>(s);
            a = q.x;
            b = q.y;
        }
        buf[e] = make_float2(a, b);
    }
    if (bad) atomicOr(flag, FLAG_OVERFLOW);
    __syncthreads();
    fft_from<L, 1, RB, T, false, 1, L, false, 4>(buf, tw + L);
    // X_k = (Z_k + conj Z_{L-k}) / 2 - i w^k (Z_k - conj Z_{L-k}) / 2, w = exp(-2 pi i / N)
    for (int e = tid; e < RB * (L + 1); e += T) {
        const int r = e / (L + 1), k = e % (L + 1);
        const float2 zk = buf[r * L + (k & (L - 1))];
        const float2 zc = cconj(buf[r * L + ((L - k) & (L - 1))]);
        const float2 w = tw[N + k];
        const float2 sum = cadd(zk, zc), t = cmul(w, csub(zk, zc));
        dst[(row0 + r) * dst_stride + k] = make_float2(0.5f * (sum.x + t.y), 0.5f * (sum.y - t.x));
    }
    constexpr int PADC = (int)half_cols(N) - (L + 1);   // the last column tile's unused columns
    for (int e = tid; e < RB * PADC; e += T) {
        const int r = e / PADC, k = L + 1 + e % PADC;
        dst[(row0 + r) * dst_stride + k] = make_float2(0.f, 0.f);
    }
}

template <int LOGN>
__global__ __launch_bounds__(256) void k_c2r_rows(const float2 *src, int64_t src_stride, float *dst,
                                                  int64_t dst_stride, const float2 *__restrict__ tw)
{
    using C = RowCfg<LOGN>;
    constexpr int N = C::N, L = C::L, RB = C::RB, T = C::T, LS = L + 1;
    __shared__ float2 buf[RB * LS];
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    const int tid = threadIdx.x;
#pragma unroll 8
    for (int e = tid; e < RB * LS; e += T) {
        const int r = e / LS, k = e % LS;
        buf[e] = src[(row0 + r) * src_stride + k];
    }
    __syncthreads();
    // Z_k = A + i B, A = X_k + conj X_{L-k}, B = (X_k - conj X_{L-k}) exp(+2 pi i k / N);
    // Z_{L-k} = conj A + i conj B.
    for (int e = tid; e < RB * (L / 2 + 1); e += T) {
        const int r = e / (L / 2 + 1), k = e % (L / 2 + 1);
        const float2 X = buf[r * LS + k], Y = cconj(buf[r * LS + L - k]);
        const float2 A = cadd(X, Y), B = cmul(cconj(tw[N + k]), csub(X, Y));
        buf[r * LS + k] = make_float2(A.x - B.y, A.y + B.x);
        if (k != 0 && k != L / 2) buf[r * LS + L - k] = make_float2(A.x + B.y, B.x - A.y);
    }
    __syncthreads();
    fft_from<L, 1, RB, T, false, 1, LS, true, 4>(buf, tw + L);
#pragma unroll 8
    for (int e = tid; e < RB * L; e += T) {
        const int r = e / L, m = e % L;
        *reinterpret_cast<float2 *>(dst + (row0 + r) * dst_stride + 2 * m) = buf[r * LS + m];
    }
}

// ---------------------------------------------------------------- columns
// Column factor of the force components (the k1 and k2 parts of the
// gradient of the inverse Laplacian), applied on load: 1 -> 2 pi n1 / N with
// n1 the signed row frequency, 2 -> 2 pi k2 / N with k2 the column; zero on
// the component's own Nyquist frequency.  The row and column are the axis-1
// and axis-2 frequencies when the pass runs along axis 1.
template <int N>
__device__ __forceinline__ float col_factor(int mul, int row, int col)
{
    const float sc = 6.28318530717958648f / (float)N;
    if (mul == 1) {
        const int r1 = row <= N / 2 ? row : row - N;
        return (r1 == N / 2 || r1 == -N / 2) ? 0.f : sc * r1;
    }
    return col >= N / 2 ? 0.f : sc * col;
}

// V2: a thread moves two adjacent columns of a row per access (16 bytes;
// base and dst 16-byte aligned, strides even), else one (8 bytes).
// mul != 0 scales every element by col_factor before the transform; the
// result goes to dst (the same offsets; dst == base: in place).
template <int LOGN, bool INV, int WW, bool V2>
__global__ __launch_bounds__((ColCfg<LOGN, WW>::T)) void k_cols(float2 *base, int64_t stride_l, int64_t stride_o,
                                                              int n_cb, const float2 *__restrict__ tw, int mul,
                                                              float2 *dst)
{
    using C = ColCfg<LOGN, WW>;
    constexpr int N = C::N, W = C::W, E = C::E, T = C::T;
    __shared__ float2 buf[E];
    // the stages' twiddles, staged once: read from global memory after each
    // stage's barrier, their latency would stall every wave at once
    __shared__ float2 twl[N];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int o = tile / n_cb, cb = tile % n_cb;
    const int tid = threadIdx.x;
    constexpr int SW = W == 8 ? -(3 + ColCfg<LOGN, WW>::R1) : 0;
    for (int i = tid; i < N; i += T) twl[i] = tw[N + i];
    if constexpr (V2) {
        // thread owns columns 2 (tid % (W/2)) + {0, 1} and rows tid / (W/2) + i 2T / W;
        // element (row, col) sits at row W + col, and the swizzle keeps a pair adjacent
        static_assert(C::PER % 2 == 0 && T % (W / 2) == 0, "pairs per thread");
        constexpr int HW = W / 2;
        const int64_t off = (int64_t)o * stride_o + cb * W + 2 * (tid % HW) + (int64_t)(tid / HW) * stride_l;
        const float2 *p = base + off;
        float2 *q = dst + off;
        const int64_t step = (int64_t)(T / HW) * stride_l;
#pragma unroll
        for (int i = 0; i < C::PER / 2; i++) {
            const float4 v = *reinterpret_cast<const float4 *>(p + i * step);
            const int e = 2 * (tid + i * T);
            float fa = 1.f, fb = 1.f;
            if (mul) {
                fa = col_factor<N>(mul, e / W, cb * W + e % W);
                fb = col_factor<N>(mul, e / W, cb * W + e % W + 1);
            }
            buf[pad<SW>(e)] = make_float2(fa * v.x, fa * v.y);
            buf[pad<SW>(e + 1)] = make_float2(fb * v.z, fb * v.w);
        }
        __syncthreads();
        fft_from<N, 1, W, T, true, W, 1, INV, 4, SW>(buf, twl);
#pragma unroll
        for (int i = 0; i < C::PER / 2; i++) {
            const int e = 2 * (tid + i * T);
            const float2 a = buf[pad<SW>(e)], b = buf[pad<SW>(e + 1)];
            *reinterpret_cast<float4 *>(q + i * step) = make_float4(a.x, a.y, b.x, b.y);
        }
    } else {
        // thread owns column tid % W and rows tid / W + i T / W (T is a multiple of W)
        const int64_t off = (int64_t)o * stride_o + cb * W + (tid % W) + (int64_t)(tid / W) * stride_l;
        const float2 *p = base + off;
        float2 *q = dst + off;
        const int64_t step = (int64_t)(T / W) * stride_l;
#pragma unroll
        for (int i = 0; i < C::PER; i++) {
            const int e = tid + i * T;
            const float f = mul ? col_factor<N>(mul, e / W, cb * W + e % W) : 1.f;
            const float2 v = p[i * step];
            buf[pad<SW>(e)] = make_float2(f * v.x, f * v.y);
        }
        __syncthreads();
        fft_from<N, 1, W, T, true, W, 1, INV, 4, SW>(buf, twl);
#pragma unroll
        for (int i = 0; i < C::PER; i++) q[i * step] = buf[pad<SW>(tid + i * T)];
    }
}

// ---------------------------------------------------------------- axis 0 + multiplier
__device__ __forceinline__ int signed_mode(int k, int n) { return k <= n / 2 ? k : k - n; }

// Zel'dovich displacement of component d from a white-noise mode (FP64):
// i k_d / k^2 sqrt(A P(k) / V_cell) [1 + (k/k_fs)^2]^-1 exp(i k.h) / M_ic,
// P(k) = k^n_s T_BBKS^2(k / (Omega_m h)); zero at k = 0 and on every Nyquist plane.
__device__ __forceinline__ float2 mult_ic(float2 v, int d, int l, int o, int k2, int n, const IcParams &p)
{
    if (k2 >= n / 2) return make_float2(0.f, 0.f);
    const int n0 = signed_mode(l, n), n1 = signed_mode(o, n), n2 = k2;
    if (n0 == -n / 2 || n0 == n / 2 || n1 == -n / 2 || n1 == n / 2) return make_float2(0.f, 0.f);
    if (n0 == 0 && n1 == 0 && n2 == 0) return make_float2(0.f, 0.f);
    const double s = 6.283185307179586476925 / p.box;
    const double k0 = s * n0, k1 = s * n1, kz = s * n2;
    const double kk = k0 * k0 + k1 * k1 + kz * kz, k = sqrt(kk);
    const double q = k / p.omh;
    const double poly = 1.0 + 3.89 * q + (16.1 * q) * (16.1 * q) + (5.46 * q) * (5.46 * q) * (5.46 * q) +
                        (6.71 * q) * (6.71 * q) * (6.71 * q) * (6.71 * q);
    const double T = log(1.0 + 2.34 * q) / (2.34 * q) * pow(poly, -0.25);
    double amp = sqrt(p.amp_over_vcell * pow(k, p.n_s)) * T * p.scale;
    if (p.kfs > 0) amp /= 1.0 + (k / p.kfs) * (k / p.kfs);
    const double kd = d == 0 ? k0 : (d == 1 ? k1 : kz);
    const double g = amp * kd / kk;
    double re = -g * v.y, im = g * v.x;   // i g v
    if (p.half_cell != 0) {
        const double ph = (k0 + k1 + kz) * p.half_cell;
        const double c = cos(ph), sn = sin(ph);
        const double r2 = re * c - im * sn, i2 = re * sn + im * c;
        re = r2;
        im = i2;
    }
    return make_float2((float)re, (float)im);
}

// Transpose of the initial-condition transfer: acc (+)= sum_d conj(M_d) G_d
// over three natural-order half spectra G_d (row stride nhp, field stride
// fs); conj(M) v = conj(M conj(v)).
__global__ void k_ic_adj_mult(const float2 *G, int64_t nhp, int64_t fs, int n, IcParams icp, float2 *acc,
                              int accumulate)
{
    const int64_t tot = (int64_t)n * n * nhp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int k2 = (int)(t % nhp);
        const int64_t r = t / nhp;
        const int i1 = (int)(r % n), i0 = (int)(r / n);
        float2 s = accumulate ? acc[t] : make_float2(0.f, 0.f);
        for (int d = 0; d < 3; d++) {
            const float2 m = mult_ic(cconj(G[d * fs + t]), d, i0, i1, k2, n, icp);
            s = cadd(s, cconj(m));
        }
        acc[t] = s;
    }
}

template <int LOGN, int MODE, int NOUT>
__global__ __launch_bounds__(Ax0Cfg<LOGN>::T) void k_axis0(const float2 *src, int64_t s_l, int64_t s_o,
                                                           float2 *out0, float2 *out1, float2 *out2,
                                                           int64_t o_l, int64_t o_o, int n_cb, float coef,
                                                           IcParams icp, const float2 *__restrict__ tw)
{
    using C = Ax0Cfg<LOGN>;
    constexpr int N = C::N, W = C::W, E = C::E, T = C::T, PER = C::PER;
    __shared__ float2 buf[E];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int o = tile / n_cb, cb = tile % n_cb;
    const int tid = threadIdx.x;
    const int col = tid % W, row0 = tid / W;
    constexpr int RSTEP = T / W;
    {
        const float2 *p = src + (int64_t)o * s_o + cb * W + col + (int64_t)row0 * s_l;
#pragma unroll
        for (int i = 0; i < PER; i++) buf[tid + i * T] = p[i * (RSTEP * s_l)];
    }
    __syncthreads();
    fft_from<N, 1, W, T, true, W, 1, false, AX0_MAXB>(buf, tw + N);
    const int64_t out_off = (int64_t)o * o_o + cb * W + col + (int64_t)row0 * o_l;
    const int64_t ostep = (int64_t)RSTEP * o_l;
    if constexpr (NOUT == 0) {
        float2 *q = out0 + out_off;
#pragma unroll
        for (int i = 0; i < PER; i++) q[i * ostep] = buf[tid + i * T];
    } else if constexpr (MODE == MULT_FORCE) {
        // Within a column (k1, k2) the axis-1 and axis-2 components are k1 and
        // k2 times one common transform of T(k) = coef i S / k^2, and the
        // axis-0 component is the transform of k0 T: two inverse FFTs give
        // all three outputs.  The inverses run on one half of the tile's
        // columns at a time while the forward spectrum of the other half waits
        // in LDS, so a thread keeps only its half's T values in registers.
        constexpr int HW = W / 2, HE = N * HW, HPER = HE / T > 0 ? HE / T : 1;
        constexpr int HSTEP = T / HW;
        if constexpr (HE % T == 0 && T % HW == 0) {
        const int hcol = tid % HW, hrow0 = tid / HW;
        const int n1 = signed_mode(o, N);
        const float s = 6.28318530717958648f / (float)N;
        const float k1 = s * n1;
        const float f1 = (n1 == N / 2 || n1 == -N / 2) ? 0.f : k1;
        const int64_t hstep = (int64_t)HSTEP * o_l;
#pragma unroll 1
        for (int h = 0; h < 2; h++) {
            const int k2 = cb * W + h * HW + hcol;
            const float kz = s * k2;
            const float kperp = k1 * k1 + kz * kz;
            float2 *hb = buf + h * HW;
            float2 keep[HPER];
#pragma unroll
            for (int i = 0; i < HPER; i++) {
                const int row = hrow0 + i * HSTEP;
                const int n0 = signed_mode(row, N);
                const float k0 = s * n0;
                const float kk = k0 * k0 + kperp;
                const float2 v = hb[row * W + hcol];
                const float g = (k2 > N / 2 || kk == 0.f) ? 0.f : coef / kk;
                keep[i] = make_float2(-g * v.y, g * v.x);                       // T = i g S
                const float g0 = (n0 == N / 2 || n0 == -N / 2) ? 0.f : k0;
                hb[row * W + hcol] = make_float2(g0 * keep[i].x, g0 * keep[i].y);   // k0 T
            }
            __syncthreads();
            fft_from<N, 1, HW, T, true, W, 1, true, AX0_MAXB>(hb, tw + N);
            const int64_t hoff = (int64_t)o * o_o + cb * W + h * HW + hcol + (int64_t)hrow0 * o_l;
            {
                float2 *q = out0 + hoff;
#pragma unroll
                for (int i = 0; i < HPER; i++) q[i * hstep] = hb[(hrow0 + i * HSTEP) * W + hcol];
            }
#pragma unroll
            for (int i = 0; i < HPER; i++) hb[(hrow0 + i * HSTEP) * W + hcol] = keep[i];
            __syncthreads();
            fft_from<N, 1, HW, T, true, W, 1, true, AX0_MAXB>(hb, tw + N);
            const float f2 = (k2 >= N / 2) ? 0.f : kz;
            float2 *q1 = out1 + hoff, *q2 = out2 + hoff;
#pragma unroll
            for (int i = 0; i < HPER; i++) {
                const float2 v = hb[(hrow0 + i * HSTEP) * W + hcol];
                q1[i * hstep] = make_float2(f1 * v.x, f1 * v.y);
                q2[i * hstep] = make_float2(f2 * v.x, f2 * v.y);
            }
        }
        }  // meshes below 16^3 never take the force path (launch_axis0 rejects them)
    } else {
        float2 keep[PER];
#pragma unroll
        for (int i = 0; i < PER; i++) keep[i] = buf[tid + i * T];
#pragma unroll 1
        for (int d = 0; d < NOUT; d++) {
#pragma unroll
            for (int i = 0; i < PER; i++)
                buf[tid + i * T] = mult_ic(keep[i], d, row0 + i * RSTEP, o, cb * W + col, N, icp);
            __syncthreads();
            fft_from<N, 1, W, T, true, W, 1, true, AX0_MAXB>(buf, tw + N);
            float2 *q = (d == 0 ? out0 : (d == 1 ? out1 : out2)) + out_off;
#pragma unroll
            for (int i = 0; i < PER; i++) q[i * ostep] = buf[tid + i * T];
        }
    }
}


// ---------------------------------------------------------------- axis 0 in two passes
// At N >= 256 one plane of the half spectrum (N x nhp complex, contiguous)
// spans several 2 MiB pages, and a column tile that reads 64 bytes from each
// of N planes takes an address-translation miss on nearly every access.  The
// axis-0 transform is therefore split as N = 16 x N2 (four-step FFT) into two
// passes whose wavefronts each read 512 contiguous bytes of one plane:
//   pass A: for every j1 < N2, a 16-point DFT over the planes j1 + N2 j2
//           (j2 < 16) and the twiddle w_N^(j1 m); Y_m[j1] is stored in place,
//           in plane j1 + N2 m;
//   pass B: for every m < 16, an N2-point DFT over the consecutive planes
//           N2 m + j1, which leaves frequency k0 = m + 16 k in plane N2 m + k
//           (digit-reversed along axis 0).
// Pass A rides on the row transforms (k_r2c_x0, k_c2r_x0 below, which hold
// the 16 rows j2 < 16 of one x1 in LDS).  The force kernel fuses pass B with
// the gradient of the inverse Laplacian and the inverse of pass B for two
// fields; the inverse column passes apply the k1 and k2 factors (they do not
// depend on k0, so they commute with the axis-0 inverse), and the inverse of
// pass A, inside the complex-to-real rows, restores natural order.  Plane offsets e (0 <= e < N nhp) index
// (k1, k2) = (e / nhp, e % nhp).

// Pass B of the force solve: grid (N nhp / 64, 16), 64 R2 threads with
// R2 = N2 / 16, each thread one of 64 consecutive plane offsets.  The N2-point
// DFT is itself split as N2 = R2 x 16: step 1 (thread (c, g), g < R2) takes a
// 16-point DFT over j1 = g + R2 i and the twiddle w_N2^(g a), step 2 (thread
// (c, q), after an LDS exchange) the R2-point DFTs over g for a = q + R2 s,
// giving k = a + 16 l.  T = coef i S / k^2 is kept in registers; k0 T and T
// go through the inverse steps; outputs k0 T -> out0 (which may alias src,
// zero on the k0 Nyquist plane) and T -> out1, both zero at k = 0.  Writing T
// once instead of k1 T and k2 T saves a third of the pass's writes.
template <int N>
struct X0Cfg {
    static constexpr int N2 = N / 16, R2 = N2 / 16, C = 64, T = C * R2, SPT = 16 / R2;
    static_assert(N >= 256 && R2 >= 1, "two-pass axis-0 transform needs N >= 256");
};

// Inverse of pass B on one thread's 16 values (step-2 slots in, j1 = g + R2 i
// out); the caller's LDS tile is free on entry and on return.
template <int N>
__device__ __forceinline__ void x0_inverse_b(float2 (&w)[16], float2 *lds, int c, int g,
                                             const float2 *__restrict__ twN2)
{
    using X = X0Cfg<N>;
    constexpr int R2 = X::R2, C = X::C, SPT = X::SPT;
#pragma unroll
    for (int s = 0; s < SPT; s++) {
        Dft<R2, true>::run(w + s * R2);
        const int a = g + R2 * s;
#pragma unroll
        for (int l = 0; l < R2; l++) lds[(a * R2 + l) * C + c] = w[s * R2 + l];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 16; a++) w[a] = lds[(a * R2 + g) * C + c];
    __syncthreads();
    if constexpr (R2 > 1) {
#pragma unroll
        for (int a = 1; a < 16; a++) w[a] = cmul(w[a], cconj(twN2[g * a]));
    }
    Dft<16, true>::run(w);
}

template <int N>
__global__ __launch_bounds__(X0Cfg<N>::T, 4) void k_x0_green(const float2 *src, float2 *out0, float2 *out1,
                                                          int64_t plane, int nhp, float coef,
                                                          const float2 *__restrict__ tw)
{
    using X = X0Cfg<N>;
    constexpr int N2 = X::N2, R2 = X::R2, C = X::C, SPT = X::SPT;
    __shared__ float2 lds[16 * R2 * C];
    const int m = blockIdx.y;
    static_assert(C == 64, "one wavefront per g: g and the twiddles it selects are wave-uniform");
    // step 1: g; step 2: q = g.  Uniform per wavefront, so the twiddles
    // twN2[g a] come through the scalar cache instead of the vector loads
    // that carry the spectrum.
    const int c = threadIdx.x % C, g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / C);
    const int64_t e = (int64_t)blockIdx.x * C + c;
    const int64_t pbase = (int64_t)(N2 * m + g) * plane + e;
    const int64_t pstep = (int64_t)R2 * plane;
    const float2 *twN2 = tw + N2;
    float2 v[16];
#pragma unroll
    for (int i = 0; i < 16; i++) v[i] = src[pbase + i * pstep];
    Dft<16, false>::run(v);
    if constexpr (R2 > 1) {
#pragma unroll
        for (int a = 1; a < 16; a++) v[a] = cmul(v[a], twN2[g * a]);
    }
#pragma unroll
    for (int a = 0; a < 16; a++) lds[(a * R2 + g) * C + c] = v[a];
    __syncthreads();
    // step 2: slot s R2 + l holds frequency k = q + R2 s + 16 l
#pragma unroll
    for (int s = 0; s < SPT; s++) {
        const int a = g + R2 * s;
#pragma unroll
        for (int l = 0; l < R2; l++) v[s * R2 + l] = lds[(a * R2 + l) * C + c];
        Dft<R2, false>::run(v + s * R2);
    }
    __syncthreads();
    const float sc = 6.28318530717958648f / (float)N;
    const int k1i = (int)(e / nhp), k2 = (int)(e % nhp);
    const int n1 = signed_mode(k1i, N);
    const float k1 = sc * n1, kz = sc * k2, kperp = k1 * k1 + kz * kz;
    float2 keep[16];
#pragma unroll
    for (int s = 0; s < SPT; s++)
#pragma unroll
        for (int l = 0; l < R2; l++) {
            const int k = g + R2 * s + 16 * l;
            const int n0 = signed_mode(m + 16 * k, N);
            const float k0 = sc * n0, kk = k0 * k0 + kperp;
            const float gr = (k2 > N / 2 || kk == 0.f) ? 0.f : coef / kk;
            const float2 x = v[s * R2 + l];
            const float2 t = make_float2(-gr * x.y, gr * x.x);                 // T = i g S
            keep[s * R2 + l] = t;
            const float g0 = (n0 == N / 2 || n0 == -N / 2) ? 0.f : k0;
            v[s * R2 + l] = make_float2(g0 * t.x, g0 * t.y);                  // k0 T
        }
    // walking output pointers; the empty asm keeps the compiler from
    // materialising all sixteen 64-bit addresses while T is live
    x0_inverse_b<N>(v, lds, c, g, twN2);
    {
        float2 *q = out0 + pbase;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            asm volatile("" : "+v"(q));
            *q = v[i];
            q += pstep;
        }
    }
    x0_inverse_b<N>(keep, lds, c, g, twN2);
    {
        float2 *q1 = out1 + pbase;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            asm volatile("" : "+v"(q1));
            *q1 = keep[i];
            q1 += pstep;
        }
    }
}

// Pass B of the learned force (the two-pass form of the potential of the
// learned correction): the same completion of the axis-0 transform on two
// spectra, the density srcd and the CNN output srcc (both after the rows,
// the first axis-0 digit and axis 1), then T = i (g(|k|) gr S_d - S_c / M)
// with gr = coef / k^2, coef = 1.5 Omega_m / M and g the radial filter
// table: the force of the potential phi_f + cnn is F_d = k_d T, as for the
// plain force.  Writes k0 T and T after the inverse of pass B, like
// k_x0_green; zero at k = 0 for the filtered part and in the padding.
template <int N>
__global__ __launch_bounds__(X0Cfg<N>::T, 2) void k_x0_learned(const float2 *srcd, const float2 *srcc,
                                                            float2 *out0, float2 *out1, int64_t plane, int nhp,
                                                            float coef, float inv_m, const float *__restrict__ table,
                                                            const float2 *__restrict__ tw)
{
    using X = X0Cfg<N>;
    constexpr int N2 = X::N2, R2 = X::R2, C = X::C, SPT = X::SPT;
    __shared__ float2 lds[16 * R2 * C];
    __shared__ float tab[NET_NB];
    const int m = blockIdx.y;
    static_assert(C == 64, "one wavefront per g: g and the twiddles it selects are wave-uniform");
    const int c = threadIdx.x % C, g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / C);
    for (int i = threadIdx.x; i < NET_NB; i += X::T) tab[i] = table[i];
    const int64_t e = (int64_t)blockIdx.x * C + c;
    const int64_t pbase = (int64_t)(N2 * m + g) * plane + e;
    const int64_t pstep = (int64_t)R2 * plane;
    const float2 *twN2 = tw + N2;
    float2 v[16], w[16];
    // pass B forward on one field: step 1 through LDS, step 2 in registers
    auto forward = [&](const float2 *src, float2 (&u)[16]) {
#pragma unroll
        for (int i = 0; i < 16; i++) u[i] = src[pbase + i * pstep];
        Dft<16, false>::run(u);
        if constexpr (R2 > 1) {
#pragma unroll
            for (int a = 1; a < 16; a++) u[a] = cmul(u[a], twN2[g * a]);
        }
#pragma unroll
        for (int a = 0; a < 16; a++) lds[(a * R2 + g) * C + c] = u[a];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SPT; s++) {
            const int a = g + R2 * s;
#pragma unroll
            for (int l = 0; l < R2; l++) u[s * R2 + l] = lds[(a * R2 + l) * C + c];
            Dft<R2, false>::run(u + s * R2);
        }
        __syncthreads();
    };
    forward(srcc, w);
    forward(srcd, v);
    const float sc = 6.28318530717958648f / (float)N;
    const int k1i = (int)(e / nhp), k2 = (int)(e % nhp);
    const int n1 = signed_mode(k1i, N);
    const float k1 = sc * n1, kz = sc * k2, kperp = k1 * k1 + kz * kz;
#pragma unroll
    for (int s = 0; s < SPT; s++)
#pragma unroll
        for (int l = 0; l < R2; l++) {
            const int k = g + R2 * s + 16 * l;
            const int n0 = signed_mode(m + 16 * k, N);
            const float k0 = sc * n0, kk = k0 * k0 + kperp;
            int b;
            float wt;
            const float filt = table_at(tab, sqrtf(kk) * 0.31830988618379067f, b, wt);
            const float gr = (k2 > N / 2 || kk == 0.f) ? 0.f : filt * coef / kk;
            const float cm = k2 > N / 2 ? 0.f : inv_m;
            const float2 x = v[s * R2 + l], y = w[s * R2 + l];
            const float2 u = make_float2(gr * x.x - cm * y.x, gr * x.y - cm * y.y);
            const float2 t = make_float2(-u.y, u.x);                             // T = i (g gr S_d - S_c / M)
            w[s * R2 + l] = t;
            const float g0 = (n0 == N / 2 || n0 == -N / 2) ? 0.f : k0;
            v[s * R2 + l] = make_float2(g0 * t.x, g0 * t.y);                  // k0 T
        }
    x0_inverse_b<N>(v, lds, c, g, twN2);
    {
        float2 *q = out0 + pbase;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            asm volatile("" : "+v"(q));
            *q = v[i];
            q += pstep;
        }
    }
    x0_inverse_b<N>(w, lds, c, g, twN2);
    {
        float2 *q1 = out1 + pbase;
#pragma unroll
        for (int i = 0; i < 16; i++) {
            asm volatile("" : "+v"(q1));
            *q1 = w[i];
            q1 += pstep;
        }
    }
}

// Rows fused with pass A: one workgroup takes the 16 rows (plane j1 + N2 j,
// row x1), j < 16, of a field, so the 16-point axis-0 DFT across them costs
// no HBM pass of its own.  Forward: real-to-complex of the 16 int64 rows,
// then for every column k the DFT over j and the twiddle w_N^(j1 m), stored
// in plane j1 + N2 m.  Inverse: for every column the twiddle conj(w_N^(j1 m))
// and the inverse DFT over m, then the 16 complex-to-real rows.  The x1
// transform commutes with both, so it may run before or after.  L = N/2
// threads, 16 rows of L complex in LDS (128 KiB at N = 2048).
// SRC int64_t: the fixed-point density, converted to delta = Q scale + offset
// on load (overflow flag as in the row transform); SRC float: the density
// contrast itself, written by the tile paint.
template <int LOGN, typename SRC>
__global__ __launch_bounds__(1 << (LOGN - 1)) void k_r2c_x0(const SRC *src, int64_t src_rs, float2 *dst, int nhp,
                                                            int64_t plane, double scale, double offset,
                                                            const float2 *__restrict__ tw, int *flag)
{
    constexpr int N = 1 << LOGN, L = N / 2, T = L, N2 = N / 16, RB = 16, PS = SWZ_ROWS;
    __shared__ float2 buf[padded(RB * L, PS)];
    __shared__ float2 twl[L];   // the row stages' twiddles (one per thread)
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int j1 = tile / N, x1 = tile % N;
    const int tid = threadIdx.x;
    twl[tid] = tw[L + tid];
    // the split's twiddles for column k = tid and (thread 0) k = L, loaded
    // with the rows rather than after the last barrier
    const float2 wk = tw[N + tid], wl = tw[N + L];
    float2 tj[16];
#pragma unroll
    for (int m = 1; m < 16; m++) tj[m] = tw[N + j1 * m];
    bool bad = false;
    // thread tid moves element tid of each of the 16 rows; all 16 loads are
    // issued before the first LDS write (one workgroup per CU: a
    // load-then-store loop would keep only a few requests in flight)
    static_assert(RB * L == 16 * T, "one element per row and thread");
    const SRC *row0 = src + ((int64_t)j1 * N + x1) * src_rs + 2 * tid;
    const int64_t rstep = (int64_t)N2 * N * src_rs;
    if constexpr (std::is_same<SRC, int64_t>::value) {
        longlong2 q[16];
#pragma unroll
        for (int r = 0; r < 16; r++) q[r] = *reinterpret_cast<const longlong2 *>(row0 + r * rstep);
#pragma unroll
        for (int r = 0; r < 16; r++) {
            bad |= (q[r].x < GUARD_MIN_Q) | (q[r].y < GUARD_MIN_Q);
            buf[pad<PS>(r * L + tid)] =
                make_float2((float)((double)q[r].x * scale + offset), (float)((double)q[r].y * scale + offset));
        }
    } else {
        float2 q[16];
#pragma unroll
        for (int r = 0; r < 16; r++) q[r] = *reinterpret_cast<const float2 *>(row0 + r * rstep);
#pragma unroll
        for (int r = 0; r < 16; r++) buf[pad<PS>(r * L + tid)] = q[r];
    }
    if (bad) atomicOr(flag, FLAG_OVERFLOW);
    __syncthreads();
    fft_from<L, 1, RB, T, false, 1, L, false, 4, PS>(buf, twl);
    float2 *d0 = dst + (int64_t)j1 * plane + (int64_t)x1 * nhp;
    const int64_t pstep = (int64_t)N2 * plane;
    for (int k = tid; k <= L; k += T) {
        const float2 w = k == tid ? wk : wl;
        float2 v[16];
#pragma unroll
        for (int r = 0; r < 16; r++) {
            // X_k = (Z_k + conj Z_{L-k}) / 2 - i w^k (Z_k - conj Z_{L-k}) / 2
            const float2 zk = buf[pad<PS>(r * L + (k & (L - 1)))];
            const float2 zc = cconj(buf[pad<PS>(r * L + ((L - k) & (L - 1)))]);
            const float2 sum = cadd(zk, zc), t = cmul(w, csub(zk, zc));
            v[r] = make_float2(0.5f * (sum.x + t.y), 0.5f * (sum.y - t.x));
        }
        Dft<16, false>::run(v);
#pragma unroll
        for (int m = 1; m < 16; m++) v[m] = cmul(v[m], tj[m]);
#pragma unroll
        for (int m = 0; m < 16; m++) d0[m * pstep + k] = v[m];
    }
    const int padc = nhp - (L + 1);
    for (int e = tid; e < 16 * padc; e += T) {
        const int m = e / padc, k = L + 1 + e % padc;
        d0[m * pstep + k] = make_float2(0.f, 0.f);
    }
}

template <int LOGN>
__global__ __launch_bounds__(1 << (LOGN - 1)) void k_c2r_x0(const float2 *src, float *dst, int64_t dst_stride,
                                                            int64_t dst_plane, int nhp, int64_t plane,
                                                            const float2 *__restrict__ tw)
{
    constexpr int N = 1 << LOGN, L = N / 2, T = L, N2 = N / 16, RB = 16, LS = L, PS = SWZ_ROWS;
    __shared__ float2 buf[padded(RB * LS, PS)];
    __shared__ float2 twl[L];   // the row stages' twiddles (one per thread)
    __shared__ float2 xnq[RB];  // the Nyquist column X_L of the 16 rows
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int j1 = tile / N, x1 = tile % N;
    const int tid = threadIdx.x;
    const float2 *twN = tw + N;
    const float2 *s0 = src + (int64_t)j1 * plane + (int64_t)x1 * nhp;
    const int64_t pstep = (int64_t)N2 * plane;
    // the Hermitian pre-step below: thread tid takes k = 1 + tid % (L/2) on
    // rows (tid / (L/2)) RB/2 .. + RB/2 - 1, with one twiddle, loaded here
    // with the columns
    const int hk = 1 + tid % (L / 2), hr = (tid / (L / 2)) * (RB / 2);
    const float2 hw = cconj(twN[hk]);
    twl[tid] = tw[L + tid];
    {
        // column k = tid, and the Nyquist column k = L on thread 0, whose
        // loads are issued with the others (a second round would leave the
        // whole workgroup waiting on one thread's loads)
        float2 v[16], vn[16];
#pragma unroll
        for (int m = 0; m < 16; m++) v[m] = s0[m * pstep + tid];
        if (tid == 0) {
#pragma unroll
            for (int m = 0; m < 16; m++) vn[m] = s0[m * pstep + L];
        }
#pragma unroll
        for (int m = 1; m < 16; m++) v[m] = cmul(v[m], cconj(twN[j1 * m]));
        Dft<16, true>::run(v);
#pragma unroll
        for (int r = 0; r < 16; r++) buf[pad<PS>(r * LS + tid)] = v[r];
        if (tid == 0) {
#pragma unroll
            for (int m = 1; m < 16; m++) vn[m] = cmul(vn[m], cconj(twN[j1 * m]));
            Dft<16, true>::run(vn);
#pragma unroll
            for (int r = 0; r < 16; r++) xnq[r] = vn[r];
        }
    }
    __syncthreads();
    // Z_k = A + i B, A = X_k + conj X_{L-k}, B = (X_k - conj X_{L-k}) exp(+2 pi i k / N);
    // Z_{L-k} = conj A + i conj B.  k = 1 .. L/2 here (T = L threads), k = 0
    // (B = X_0 - conj X_L, no twiddle) on threads 0 .. RB-1, one row each.
#pragma unroll
    for (int i = 0; i < RB / 2; i++) {
        const int r = hr + i;
        const float2 X = buf[pad<PS>(r * LS + hk)], Y = cconj(buf[pad<PS>(r * LS + L - hk)]);
        const float2 A = cadd(X, Y), B = cmul(hw, csub(X, Y));
        buf[pad<PS>(r * LS + hk)] = make_float2(A.x - B.y, A.y + B.x);
        if (hk != L / 2) buf[pad<PS>(r * LS + L - hk)] = make_float2(A.x + B.y, B.x - A.y);
    }
    if (tid < RB) {
        const float2 X = buf[pad<PS>(tid * LS)], Y = cconj(xnq[tid]);
        const float2 A = cadd(X, Y), B = csub(X, Y);
        buf[pad<PS>(tid * LS)] = make_float2(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    fft_from<L, 1, RB, T, false, 1, LS, true, 4, PS>(buf, twl);
    // 16-byte stores: two complex (four reals) per thread per round
#pragma unroll 4
    for (int e = tid; e < RB * L / 2; e += T) {
        const int r = e / (L / 2), m = 2 * (e % (L / 2));
        const float2 a = buf[pad<PS>(r * LS + m)], b = buf[pad<PS>(r * LS + m + 1)];
        *reinterpret_cast<float4 *>(dst + (int64_t)(j1 + N2 * r) * dst_plane + (int64_t)x1 * dst_stride + 2 * m) =
            make_float4(a.x, a.y, b.x, b.y);
    }
}

}  // namespace

#define PM_DISPATCH_LOGN(logn, MACRO) \
    switch (logn) {                    \
    case 3: MACRO(3); break;           \
    case 4: MACRO(4); break;           \
    case 5: MACRO(5); break;           \
    case 6: MACRO(6); break;           \
    case 7: MACRO(7); break;           \
    case 8: MACRO(8); break;           \
    case 9: MACRO(9); break;           \
    case 10: MACRO(10); break;         \
    case 11: MACRO(11); break;         \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_r2c_rows_i64(int logn, const int64_t *src, int64_t src_stride, float2 *dst,
                               int64_t dst_stride, int64_t nrows, double scale, double offset,
                               const float2 *tw, int *flag, hipStream_t s)
{
#define R2C_I64(LG)                                                                                  \
    {                                                                                                \
        const int64_t nb = nrows / RowCfg<LG>::RB;                                                   \
        hipLaunchKernelGGL((k_r2c_rows<LG, int64_t>), dim3((unsigned)nb), dim3(256), 0, s, src,      \
                           src_stride, dst, dst_stride, scale, offset, tw, flag);                   \
    }
    PM_DISPATCH_LOGN(logn, R2C_I64)
    return hipGetLastError();
}

hipError_t launch_r2c_rows_f32(int logn, const float *src, int64_t src_stride, float2 *dst,
                               int64_t dst_stride, int64_t nrows, const float2 *tw, hipStream_t s)
{
#define R2C_F32(LG)                                                                                  \
    {                                                                                                \
        const int64_t nb = nrows / RowCfg<LG>::RB;                                                   \
        hipLaunchKernelGGL((k_r2c_rows<LG, float>), dim3((unsigned)nb), dim3(256), 0, s, src,        \
                           src_stride, dst, dst_stride, 1.0, 0.0, tw, nullptr);                     \
    }
    PM_DISPATCH_LOGN(logn, R2C_F32)
    return hipGetLastError();
}

hipError_t launch_c2r_rows(int logn, const float2 *src, int64_t src_stride, float *dst, int64_t dst_stride,
                           int64_t nrows, const float2 *tw, hipStream_t s)
{
#define C2R(LG)                                                                                      \
    {                                                                                                \
        const int64_t nb = nrows / RowCfg<LG>::RB;                                                   \
        hipLaunchKernelGGL((k_c2r_rows<LG>), dim3((unsigned)nb), dim3(256), 0, s, src, src_stride,   \
                           dst, dst_stride, tw);                                                     \
    }
    PM_DISPATCH_LOGN(logn, C2R)
    return hipGetLastError();
}

hipError_t launch_cols(int logn, bool inverse, float2 *base, int64_t stride_l, int64_t stride_o, int n_o,
                       int n_cb, const float2 *tw, hipStream_t s, int mul, float2 *dst)
{
    const unsigned nb = (unsigned)n_o * (unsigned)n_cb;
    if (mul < 0 || mul > 2) return hipErrorInvalidValue;
    if (!dst) dst = base;
    // 16-byte accesses where the layout allows them
    const bool v2 = logn >= 4 && ((reinterpret_cast<uintptr_t>(base) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0 &&
                    stride_l % 2 == 0 && stride_o % 2 == 0;
#define COLS_V(LG, V)                                                                                \
    {                                                                                                \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((k_cols<LG, true, TILE_W, V>), dim3(nb), dim3(ColCfg<LG>::T), 0, s, base, \
                               stride_l, stride_o, n_cb, tw, mul, dst);                             \
        else                                                                                         \
            hipLaunchKernelGGL((k_cols<LG, false, TILE_W, V>), dim3(nb), dim3(ColCfg<LG>::T), 0, s, base, \
                               stride_l, stride_o, n_cb, tw, mul, dst);                             \
    }
#define COLS(LG)                                                                                     \
    {                                                                                                \
        if constexpr (LG >= 4) {                                                                     \
            if (v2) COLS_V(LG, true) else COLS_V(LG, false)                                          \
        } else {                                                                                     \
            COLS_V(LG, false)                                                                        \
        }                                                                                            \
    }
    PM_DISPATCH_LOGN(logn, COLS)
    return hipGetLastError();
}

hipError_t launch_axis0(int logn, int mode, const float2 *src, int64_t s_l, int64_t s_o, float2 *out0,
                        float2 *out1, float2 *out2, int64_t o_l, int64_t o_o, int n_cb, double coef,
                        const IcParams *ic, const float2 *tw, hipStream_t s)
{
    const int n = 1 << logn;
    if (mode == MULT_FORCE && n < 16) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)n * (unsigned)n_cb;
    if (mode == MULT_FORCE && logn >= 8) return hipErrorInvalidValue;   // two-pass path (launch_x0_*)
    IcParams icp{};
    if (ic) icp = *ic;
    const float fc = (float)coef;
#define AX0(LG)                                                                                      \
    {                                                                                                \
        const dim3 g(nb), b(Ax0Cfg<LG>::T);                                                          \
        if (mode == MULT_FORCE)                                                                      \
            hipLaunchKernelGGL((k_axis0<LG, MULT_FORCE, 3>), g, b, 0, s, src, s_l, s_o, out0, out1,  \
                               out2, o_l, o_o, n_cb, fc, icp, tw);                                  \
        else if (mode == MULT_IC)                                                                    \
            hipLaunchKernelGGL((k_axis0<LG, MULT_IC, 3>), g, b, 0, s, src, s_l, s_o, out0, out1,     \
                               out2, o_l, o_o, n_cb, fc, icp, tw);                                  \
        else                                                                                         \
            hipLaunchKernelGGL((k_axis0<LG, MULT_NONE, 0>), g, b, 0, s, src, s_l, s_o, out0, out1,   \
                               out2, o_l, o_o, n_cb, fc, icp, tw);                                  \
    }
    PM_DISPATCH_LOGN(logn, AX0)
    return hipGetLastError();
}

hipError_t launch_x0_green(int logn, const float2 *src, float2 *out0, float2 *out1, int64_t plane, int nhp,
                           double coef, const float2 *tw, hipStream_t s)
{
    // planes hold N rows of nhp values and may be followed by padding
    if (logn < 8 || logn > 11 || plane < ((int64_t)nhp << logn)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(((int64_t)nhp << logn) / 64), 16);
    const float fc = (float)coef;
#define X0B(NN)                                                                                      \
    hipLaunchKernelGGL((k_x0_green<NN>), grid, dim3(X0Cfg<NN>::T), 0, s, src, out0, out1, plane, nhp, fc, tw)
    switch (logn) {
    case 8: X0B(256); break;
    case 9: X0B(512); break;
    case 10: X0B(1024); break;
    default: X0B(2048); break;
    }
#undef X0B
    return hipGetLastError();
}

hipError_t launch_x0_learned(int logn, const float2 *srcd, const float2 *srcc, float2 *out0, float2 *out1,
                             int64_t plane, int nhp, double coef, double inv_m, const float *table, const float2 *tw,
                             hipStream_t s)
{
    if (logn < 8 || logn > 11 || plane < ((int64_t)nhp << logn)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(((int64_t)nhp << logn) / 64), 16);
    const float fc = (float)coef, fm = (float)inv_m;
#define X0L(NN)                                                                                      \
    hipLaunchKernelGGL((k_x0_learned<NN>), grid, dim3(X0Cfg<NN>::T), 0, s, srcd, srcc, out0, out1, plane, nhp, fc, fm, \
                       table, tw)
    switch (logn) {
    case 8: X0L(256); break;
    case 9: X0L(512); break;
    case 10: X0L(1024); break;
    default: X0L(2048); break;
    }
#undef X0L
    return hipGetLastError();
}

hipError_t launch_r2c_x0(int logn, const int64_t *src, float2 *dst, int nhp, int64_t plane, double scale,
                         double offset, const float2 *tw, int *flag, hipStream_t s)
{
    if (logn < 8 || logn > 11 || plane < ((int64_t)nhp << logn)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((1 << logn) / 16) << logn;
#define R2CX(LG)                                                                                     \
    hipLaunchKernelGGL((k_r2c_x0<LG, int64_t>), dim3(nb), dim3(1 << (LG - 1)), 0, s, src, (int64_t)1 << LG, dst, nhp, \
                       plane, scale, offset, tw, flag)
    switch (logn) {
    case 8: R2CX(8); break;
    case 9: R2CX(9); break;
    case 10: R2CX(10); break;
    default: R2CX(11); break;
    }
#undef R2CX
    return hipGetLastError();
}

hipError_t launch_r2c_x0_f32(int logn, const float *src, int64_t src_rs, float2 *dst, int nhp, int64_t plane,
                             const float2 *tw, hipStream_t s)
{
    if (logn < 8 || logn > 11 || plane < ((int64_t)nhp << logn) || src_rs < ((int64_t)1 << logn))
        return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((1 << logn) / 16) << logn;
#define R2CX(LG)                                                                                     \
    hipLaunchKernelGGL((k_r2c_x0<LG, float>), dim3(nb), dim3(1 << (LG - 1)), 0, s, src, src_rs, dst, nhp, plane, 1.0, \
                       0.0, tw, static_cast<int *>(nullptr))
    switch (logn) {
    case 8: R2CX(8); break;
    case 9: R2CX(9); break;
    case 10: R2CX(10); break;
    default: R2CX(11); break;
    }
#undef R2CX
    return hipGetLastError();
}

hipError_t launch_c2r_x0(int logn, const float2 *src, float *dst, int64_t dst_stride, int64_t dst_plane, int nhp,
                         int64_t plane, const float2 *tw, hipStream_t s)
{
    if (logn < 8 || logn > 11 || plane < ((int64_t)nhp << logn)) return hipErrorInvalidValue;
    // the rows are stored 16 bytes at a time
    if ((reinterpret_cast<uintptr_t>(dst) & 15) != 0 || dst_stride % 4 != 0 || dst_plane % 4 != 0 ||
        dst_plane < (dst_stride << logn))
        return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((1 << logn) / 16) << logn;
#define C2RX(LG)                                                                                     \
    hipLaunchKernelGGL((k_c2r_x0<LG>), dim3(nb), dim3(1 << (LG - 1)), 0, s, src, dst, dst_stride, dst_plane, nhp, \
                       plane, tw)
    switch (logn) {
    case 8: C2RX(8); break;
    case 9: C2RX(9); break;
    case 10: C2RX(10); break;
    default: C2RX(11); break;
    }
#undef C2RX
    return hipGetLastError();
}

hipError_t launch_ic_adj_mult(const float2 *G, int64_t nhp, int64_t fs, int n, const IcParams *ic, float2 *acc,
                              bool accumulate, hipStream_t s)
{
    const int64_t tot = (int64_t)n * n * nhp;
    int64_t b = (tot + 255) / 256;
    if (b > 65536 * 16) b = 65536 * 16;
    hipLaunchKernelGGL(k_ic_adj_mult, dim3((unsigned)b), dim3(256), 0, s, G, nhp, fs, n, *ic, acc, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace pm
