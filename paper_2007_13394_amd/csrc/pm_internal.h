// Private declarations shared by the libpm translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pm.h"

namespace pm {

// Strided FFT passes work on tiles of TILE_W contiguous complex columns.
constexpr int TILE_W = 8;
// Complex columns of a half-spectrum row (N/2 + 1 values) rounded up to whole
// column tiles: the columns the strided passes transform.  Layouts with a
// compact row stride of N (the white-noise and power spectra) hold them for
// every N >= 8.
constexpr int64_t half_cols(int n) { return ((n / 2 + 1 + TILE_W - 1) / TILE_W) * TILE_W; }
// Row stride of the half spectra and force meshes: half_cols plus PM_ROW_PAD
// columns for N >= PM_PAD_FROM (none by default).
#ifndef PM_ROW_PAD
#define PM_ROW_PAD 0
#endif
#ifndef PM_PAD_FROM
#define PM_PAD_FROM 2048
#endif
constexpr int64_t half_pad(int n) { return half_cols(n) + (n >= PM_PAD_FROM ? PM_ROW_PAD : 0); }
// Plane stride (complex values) of the force solve's spectra and real force
// meshes: N rows of half_pad(N), plus PM_PLANE_PAD values for N >= PM_PAD_FROM.
// Every other use of the F region keeps N half_pad rows per plane.  The
// strides decide how rows and planes fall on HBM channels and banks.  At
// N = 2048 (C3 step, 8 timed steps per variant, two sweeps on two boxes):
//   rows 1032, planes unpadded   248.8 ms
//   rows 1040, planes unpadded   238.2 ms (readout 48.4 -> 40.3 ms, Green
//                                pass 25.8 -> 21.0 ms, column passes 67.4 -> 72.3 ms)
//   rows 1032, planes + 16384    233.0 ms
//   rows 1032, planes + 81920    231.0 ms
//   rows 1032, planes + 163840   228.4 ms (the default; 1.25 MB per plane)
//   rows 1032, planes + 245760   232.2 ms
// Row strides of 1048 to 1152 were no better than 1040.  At N = 256 a padded
// row cost 2 % of the learned step, so smaller meshes keep the bare layout.
#ifndef PM_PLANE_PAD
#define PM_PLANE_PAD 163840
#endif
static_assert(PM_PLANE_PAD % 64 == 0, "planes stay whole 64-value groups");
constexpr int64_t force_plane(int n) { return (int64_t)n * half_pad(n) + (n >= PM_PAD_FROM ? PM_PLANE_PAD : 0); }

// Particles are sorted by TILE^3-cell blocks of the mesh for the tiled paint
// and readout (meshes of at least 2 TILE cells per side).
constexpr int TILE = 16;

constexpr int MAX_SEG = 65;
constexpr int MAX_BINS = 2048;
constexpr int POWER_BLOCKS = 512;

// Workgroups are dispatched round-robin over the eight XCDs (b mod 8), each
// with its own L2.  Renumbering them so that each XCD owns a contiguous range
// of tiles lets neighbouring tiles share cache lines in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Sort keys number the tiles in Morton (Z) order, bits of (t0, t1, t2)
// interleaved with t2 fastest: a particle that crosses a tile face then
// usually lands a few tiles away in the sorted arrays.  Tile counts per side
// are powers of two up to 2^10.
__device__ __forceinline__ unsigned morton_spread(unsigned v)
{
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ int tile_index(int t0, int t1, int t2)
{
    return (int)(morton_spread((unsigned)t2) | (morton_spread((unsigned)t1) << 1) |
                 (morton_spread((unsigned)t0) << 2));
}
// Inverse of morton_spread: every third bit of v, packed.
__device__ __forceinline__ unsigned morton_compact(unsigned v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Sort key of a position: 8 * (Morton index of the TILE^3-cell block holding
// floor(u)) + face flags, bit d set when floor(u_d) is the last cell of the
// block along axis d (its +1 cloud-in-cell corner lies in the next block).
__device__ __forceinline__ int tile_key(float u0, float u1, float u2, int n)
{
    const int mask = n - 1;
    const int c0 = (int)floorf(u0) & mask, c1 = (int)floorf(u1) & mask, c2 = (int)floorf(u2) & mask;
    const int t = tile_index(c0 / TILE, c1 / TILE, c2 / TILE);
    const int f = ((c0 % TILE) == TILE - 1 ? 1 : 0) | ((c1 % TILE) == TILE - 1 ? 2 : 0) |
                  ((c2 % TILE) == TILE - 1 ? 4 : 0);
    return t * 8 + f;
}

// Particle ranges of a tile paint: range 0 is the tile's own particles (all
// flags), ranges 1..19 the particles of the lower neighbour e != 0 (bit d of
// e: one tile lower along axis d) whose face flags f contain e, in (e, f)
// order: exactly those with a +1 corner inside this tile.  rbeg[r] is the
// first sorted index of range r, rpre the exclusive prefix of the lengths
// (rpre[NRANGE] = total).  Called by the whole workgroup; ends with a barrier.
constexpr int NRANGE = 20;
__device__ __forceinline__ void tile_ranges(const int *__restrict__ koff, int t, int t0, int t1, int t2, int nt,
                                            int *rbeg, int *rpre)
{
    if (threadIdx.x < 64) {
        const int e = threadIdx.x >> 3, f = threadIdx.x & 7;
        int slot = -1, b = 0, len = 0;
        if (e == 0 && f == 0) {
            slot = 0;
            b = koff[t * 8];
            len = koff[t * 8 + 8] - b;
        } else if (e != 0 && (f & e) == e) {
            slot = 1;
            for (int ee = 1; ee < e; ee++) slot += 1 << (3 - __popc(ee));
            for (int ff = 0; ff < f; ff++) slot += ((ff & e) == e) ? 1 : 0;
            const int s0 = (t0 - (e & 1) + nt) % nt, s1 = (t1 - ((e >> 1) & 1) + nt) % nt,
                      s2 = (t2 - ((e >> 2) & 1) + nt) % nt;
            const int tn = tile_index(s0, s1, s2);
            b = koff[tn * 8 + f];
            len = koff[tn * 8 + f + 1] - b;
        }
        if (slot >= 0) {
            rbeg[slot] = b;
            rpre[slot + 1] = len;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        rpre[0] = 0;
        for (int r = 1; r <= NRANGE; r++) rpre[r] += rpre[r - 1];
    }
    __syncthreads();
}

// Sorted index of the k-th particle (0 <= k < rpre[NRANGE]) of the ranges.
__device__ __forceinline__ int tile_range_index(int k, const int *rbeg, const int *rpre)
{
    int r = 0;   // last range whose prefix is <= k
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1)
        if (r + step < NRANGE && rpre[r + step] <= k) r += step;
    return rbeg[r] + (k - rpre[r]);
}

// Lanes of the wavefront that share this lane's key: the mask and its
// lowest lane (ballot loop, no memory traffic).
__device__ __forceinline__ void key_group(bool live, int k, uint64_t &group, int &leader)
{
    uint64_t todo = __ballot(live);
    group = 0;
    leader = 0;
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const int lk = __shfl(k, l);
        const uint64_t same = __ballot(live && k == lk);
        if (live && k == lk) {
            group = same;
            leader = l;
        }
        todo &= ~same;
    }
}

// Device-side guard bits (workspace flag word).  FLAG_STALE: tile counts
// taken over from the previous step did not match the positions.
enum { FLAG_OVERFLOW = 1, FLAG_NAN = 2, FLAG_STALE = 4 };
// A painted cell below this many quanta has wrapped past 2^63.  Cells are
// sums of positive particle quanta, but a particle's remainder corner (its
// quantum minus seven rounded corners) can be a few units negative when its
// true weight is nearly zero, so an otherwise empty cell may read -1..-3 per
// such particle; the threshold leaves room for far more of those than there
// can be particles, independent of the fixed-point shift.
constexpr long long GUARD_MIN_Q = -(1LL << 36);

// A sorted momentum record: three floats, 12 bytes (no padding lane), moved
// with one dwordx3 access.
struct Mom3 {
    float x, y, z;
};
static_assert(sizeof(Mom3) == 12, "packed momentum record");

struct Workspace {
    char *base = nullptr;
    size_t bytes = 0;
    int64_t *q = nullptr;        // int64 [N]^3 density; spectrum in place, row stride N complex
    float2 *f = nullptr;         // 3 x [N][N][Nhp] complex spectra / real force meshes
    float2 *tw = nullptr;        // twiddles: length L at tw + L, tw[L + m] = exp(-2 pi i m / L)
    int *flag = nullptr;         // guard bits
    double *partial = nullptr;   // power-spectrum block partials
    float *tables = nullptr;     // small per-run tables (IC directions, shells)
    int64_t *seg_off = nullptr;  // device copy of the segment offsets (MAX_SEG + 1)
    int64_t *quanta = nullptr;   // device copy of the segment mass quanta (MAX_SEG)
    float4 *xs = nullptr;        // tile-sorted records (u0, u1, u2, segment tag as int bits) [P]
    Mom3 *ps = nullptr;          // tile-sorted momenta (p0, p1, p2) [P], 12 bytes each
    uint8_t *tags = nullptr;     // segment tag per particle in the caller's current order [P]
    uint32_t *ids_tmp = nullptr; // tile-sorted ids [P]
    int *cnt = nullptr;          // counts per key (K + 1), then the scatter's cursors (aliases the F region)
    int *cnt_next = nullptr;     // counts per key of the positions the last tile readout wrote (K + 1)
    int *koff = nullptr;         // exclusive offsets per key (K + 1)
    int *bsum = nullptr;         // scan block sums
    // learned force correction (PM_FLAG_LEARNED)
    float *net_phif = nullptr;   // filtered potential, real rows of stride 2 Nhp
    float *net_z1 = nullptr, *net_z2 = nullptr;      // CNN pre-activations [N^3][16] FP32
    uint16_t *net_a1 = nullptr, *net_a2 = nullptr;   // CNN activations [N^3][16] BF16
    float *net_g1 = nullptr, *net_g2 = nullptr;      // reverse-mode buffers [N^3][16]
    float *net_dpsi = nullptr;   // CNN output [N^3]
    float2 *net_dk = nullptr;    // density spectrum kept for the reverse mode
    float *net_acc = nullptr;    // forces on the particles [3][P]
    float *net_table = nullptr;  // radial filter table [NET_NB]
    double *net_tbar = nullptr;  // its cotangent [NET_NB]
    double *net_red = nullptr;   // loss reductions [2]
    uint16_t *net_wpk = nullptr; // inference weights in LDS layout [NET_WPK_BYTES]
};

// Learned force correction: MLP width, radial table bins, CNN channels, and
// offsets into the flat parameter array.
constexpr int NET_H = 96, NET_NB = 256, NET_C = 16;

// The learned radial filter at kt = |k| / k_Nyq: linear interpolation in the
// table of NET_NB bins kt_b = b sqrt(3) / (NET_NB - 1); b and w receive the
// lower bin and the weight of the upper one.
__device__ __forceinline__ float table_at(const float *table, float kt, int &b, float &w)
{
    const float tt = kt * (float)(NET_NB - 1) / 1.7320508075688772f;
    b = (int)floorf(tt);
    if (b > NET_NB - 2) b = NET_NB - 2;
    w = tt - (float)b;
    return (1.f - w) * table[b] + w * table[b + 1];
}
constexpr int NET_WPK_BYTES = 32768;
constexpr int NW0 = 0, NB0 = NW0 + NET_H * 2, NW1 = NB0 + NET_H, NB1 = NW1 + NET_H * NET_H, NW2 = NB1 + NET_H,
              NB2 = NW2 + NET_H * NET_H, NW3 = NB2 + NET_H, NB3 = NW3 + NET_H, NC1W = NB3 + 1,
              NC1B = NC1W + NET_C * 27, NC2W = NC1B + NET_C, NC2B = NC2W + NET_C * NET_C * 27,
              NC3W = NC2B + NET_C, NC3B = NC3W + NET_C * 27, NET_NPARAM = NC3B + 1;

// Kernel kinds recorded by the launch trace (pm_trace_begin / pm_trace_end).
enum KernelKind {
    K_FILL = 0, K_PAINT, K_R2C, K_COLS_FWD, K_AXIS0, K_COLS_INV, K_C2R, K_READOUT_KD, K_READOUT,
    K_POWER_BIN, K_POWER_REDUCE, K_IC_PARTICLES, K_COPY, K_SORT_COUNT, K_SORT_SCAN, K_SORT_SCATTER,
    K_X0_GREEN, K_R2C_X0, K_C2R_X0, K_ADJOINT, K_NET, K_SORT_VERIFY, K_COUNT
};

struct TraceRec {
    int kind;
    hipEvent_t a, b;
};

struct Ctx {
    pm_config cfg;
    int n;                        // mesh size
    int logn;
    int64_t P, nc, nn;            // particles, CDM, neutrinos
    int nseg;
    std::vector<int64_t> seg_off; // nseg + 1
    std::vector<double> seg_mass;
    std::vector<int64_t> seg_q;
    // background / growth tables (host, FP64)
    double omega_g, omega_nu0, omega_c, omega_L, kT_nu, m1;
    std::vector<double> gx, gD, gDp, gDpp;  // growth on a uniform ln a grid
    double gx0, gdx;
    // neutrino shells
    std::vector<double> edges, q_shell, m_shell;
    std::vector<float> dirs;      // (2 n_fib + 1) x 3
    std::vector<double> q_cdf;    // pseudo-random sampling: cumulative of q^2 f~ at q = i q_cdf_h
    double q_cdf_h = 0;
    Workspace ws;
    std::vector<float2> tw_host;
    // particle order: canonical (segments at seg_off) or permuted by the last
    // tile-sorted step (segment of particle i = tags[i])
    bool permuted = false;
    int64_t nkeys = 0;            // 8 x tiles when tile sorting is available, else 0
    std::vector<int64_t> segtab_host;
    uint32_t *ids = nullptr;      // caller's id array, permuted along with the particles
    // tile counts of the positions written by the last tile readout (into the
    // array counts_x); the next sort takes them over and verifies them
    bool counts_ready = false;
    const float *counts_x = nullptr;
    // a verification of taken-over counts still in flight: the flag word is
    // copied to pinned verify_host and verify_ev marks the copy's end
    bool verify_pending = false;
    int *verify_host = nullptr;
    hipEvent_t verify_ev = nullptr;
    // PM_FLAG_DEFER_GUARDS: the flag word of the last guarded call, on its way
    // to pinned guard_host[guard_slot] behind guard_ev[guard_slot]
    bool guard_pending = false;
    int guard_slot = 0;
    int *guard_host = nullptr;   // two words
    hipEvent_t guard_ev[2] = {nullptr, nullptr};
    char *static_scratch = nullptr;   // this device's fixed scratch array (pm_paint_static)
    // launch trace
    bool tracing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<TraceRec> trace;
};

// ---- host numerics (host_cosmo.cpp)
void cosmo_setup(Ctx &c);                         // background, growth table, shells, masses
double growth_D(const Ctx &c, double a);
double growth_G(const Ctx &c, double a);
double E_of_a(const Ctx &c, double a);
double pk_amplitude(const Ctx &c);                // sigma8 normalisation of k^ns T^2

// ---- launchers (fft.hip)
struct IcParams {
    double amp_over_vcell;   // A (D0/D1)^2 / V_cell
    double box;              // Mpc/h
    double omh;              // Omega_m h
    double n_s;
    double kfs;              // free-streaming wavenumber (h/Mpc), <= 0: none
    double half_cell;        // phase shift (Mpc/h) or 0
    double scale;            // 1/M_ic x mesh cells per Mpc/h
};

hipError_t launch_r2c_rows_i64(int logn, const int64_t *src, int64_t src_stride, float2 *dst,
                               int64_t dst_stride, int64_t nrows, double scale, double offset,
                               const float2 *tw, int *flag, hipStream_t s);
hipError_t launch_r2c_rows_f32(int logn, const float *src, int64_t src_stride, float2 *dst,
                               int64_t dst_stride, int64_t nrows, const float2 *tw, hipStream_t s);
hipError_t launch_c2r_rows(int logn, const float2 *src, int64_t src_stride, float *dst,
                           int64_t dst_stride, int64_t nrows, const float2 *tw, hipStream_t s);
// mul: 0, or the k1 (1) / k2 (2) factor of a force component applied before
// the transform; dst: output at the same offsets (nullptr: in place).
hipError_t launch_cols(int logn, bool inverse, float2 *base, int64_t stride_l, int64_t stride_o,
                       int n_o, int n_cb, const float2 *tw, hipStream_t s, int mul = 0, float2 *dst = nullptr);
// axis-0 pass: forward FFT, then per output a multiplier and an inverse FFT.
enum { MULT_FORCE = 0, MULT_IC = 1, MULT_NONE = 2 };
hipError_t launch_axis0(int logn, int mode, const float2 *src, int64_t s_l, int64_t s_o, float2 *out0,
                        float2 *out1, float2 *out2, int64_t o_l, int64_t o_o, int n_cb, double coef,
                        const IcParams *ic, const float2 *tw, hipStream_t s);
// Axis 0 of the force solve at N >= 256 as two passes (N = 16 x N/16), on
// fields of nhp-padded half spectra whose planes hold `plane` = N nhp complex:
// pass A (16-point DFTs over planes N/16 apart, twiddled; or its inverse) on
// nf fields field_stride apart, and pass B fused with the gradient of the
// inverse Laplacian: out0 <- k0 T, out1 <- T, T = coef i S / k^2 (src may
// alias out0; the k1 and k2 factors are applied by the inverse column passes,
// launch_cols mul 1 and 2; outputs digit-reversed until the inverse of pass A).
hipError_t launch_x0_green(int logn, const float2 *src, float2 *out0, float2 *out1, int64_t plane, int nhp,
                           double coef, const float2 *tw, hipStream_t s);
// Row transforms fused with pass A (forward: int64 density rows -> twiddled
// pass-A output; inverse: pass-A inverse -> real rows, in place allowed).
hipError_t launch_r2c_x0(int logn, const int64_t *src, float2 *dst, int nhp, int64_t plane, double scale,
                         double offset, const float2 *tw, int *flag, hipStream_t s);
// The same pass on a float32 density contrast mesh (already offset and scaled).
hipError_t launch_r2c_x0_f32(int logn, const float *src, int64_t src_rs, float2 *dst, int nhp, int64_t plane,
                             const float2 *tw, hipStream_t s);
// Pass B of the learned force on two fields after rows, first digit and axis
// 1: the density spectrum srcd and the CNN output's srcc; writes k0 T and T
// with T = i (g(|k|) coef / k^2 S_d - inv_m S_c) (table: the radial filter).
hipError_t launch_x0_learned(int logn, const float2 *srcd, const float2 *srcc, float2 *out0, float2 *out1,
                             int64_t plane, int nhp, double coef, double inv_m, const float *table, const float2 *tw,
                             hipStream_t s);
hipError_t launch_c2r_x0(int logn, const float2 *src, float *dst, int64_t dst_stride, int64_t dst_plane, int nhp,
                         int64_t plane, const float2 *tw, hipStream_t s);

hipError_t launch_ic_adj_mult(const float2 *G, int64_t nhp, int64_t fs, int n, const IcParams *ic, float2 *acc,
                              bool accumulate, hipStream_t s);

// ---- launchers (adjoint.hip)
hipError_t launch_axpy(float *y, const float *x, float a, int64_t n, hipStream_t s);
hipError_t launch_readout_grad3(const float *x, int64_t P, const float *g, float gscale, const float *F, int64_t rs, int64_t ps,
                                int64_t cs, int n, float *xbar, hipStream_t s);
hipError_t launch_paint_vec3(const float *x, int64_t P, const float *g, float gscale, float *G, int64_t rs,
                             int64_t cs, int n, hipStream_t s);
// max |gscale g| over count values into *out as float bits (zero *out first).
hipError_t launch_absmax(const float *g, int64_t count, float gscale, unsigned *out, hipStream_t s);
// Q (int64 [N]^3, added to) += llrint(S w gscale g_d) per particle and corner.
hipError_t launch_paint_q1_tiles(const float4 *xs, const Mom3 *vals, int comp, const int *koff, float gscale,
                                 double S, int n, int64_t *Q, hipStream_t s);
hipError_t launch_paint_q1(const float *x, int64_t P, const float *gd, float gscale, double S, int n, int64_t *Q,
                           hipStream_t s);
hipError_t launch_green_adj(float2 *F, int64_t nhp, int64_t fs, int n, double coef, hipStream_t s);
hipError_t launch_density_grad(const float *x, int64_t P, const float *mesh, int64_t rs, int n, int nseg,
                               const int64_t *seg_off, const uint8_t *tags, const int64_t *quanta, float qscale,
                               float scale, float *xbar, hipStream_t s);
hipError_t launch_q_to_delta(const int64_t *q, int64_t m, double scale, float *delta, hipStream_t s);
hipError_t launch_ic_adj_gather_cdm(const float *xbar, const float *pbar, int64_t P, int nic, float vfac, float *F,
                                    int64_t rs, int64_t cs, hipStream_t s);
hipError_t launch_ic_adj_gather_nu(const float *xbar, const float *pbar, int64_t P, int64_t nc, int nic, int ns,
                                   int nd, int n_shell, float vfac, float *F, int64_t rs, int64_t cs, hipStream_t s);

// ---- launchers (net.hip)
hipError_t launch_mlp_fwd(const float *th, double a, float *table, hipStream_t s);
hipError_t launch_mlp_bwd(const float *th, double a, const double *tbar, float *dth, hipStream_t s);
hipError_t launch_spec_filter(const float2 *in, float2 *out, int64_t nhp, int n, const float *table, double coef,
                              hipStream_t s);
hipError_t launch_spec_filter_bwd(const float2 *dk, const float2 *pf, int64_t nhp, int n, double coef, double *tbar,
                                  hipStream_t s);
hipError_t launch_grad3(float2 *F, int64_t nhp, int64_t fs, int n, double scale, bool transpose, hipStream_t s);
// F_d = -i k_d (F_1 + F_2) scale into fields 0, 1, 2 (the potential given as two spectra).
hipError_t launch_grad3_sum(float2 *F, int64_t nhp, int64_t fs, int n, double scale, hipStream_t s);
// CNN input: the int64 density mesh q with quantum qs (delta = q qs - 1).
hipError_t launch_cnn_fwd(const int64_t *q, double qs, int n, const float *th, float *z1, uint16_t *a1, float *z2,
                          uint16_t *a2, float *dpsi, hipStream_t s);
hipError_t launch_combine(const float *phif, const float *dpsi, int64_t rs, int n, float *out, hipStream_t s);
// Inference CNN fused with the combination: out = phi_f + cnn(delta) on real
// rows; a2: BF16 [n^3][16] scratch, wpk: NET_WPK_BYTES scratch for the
// repacked weights.  n a multiple of 16.
// delta (optional): the float32 density contrast to use instead of q; phif
// (optional): added to the CNN output (none: the output is the CNN alone).
hipError_t launch_cnn_inf(const int64_t *q, double qs, const float *delta, const float *phif, int64_t rs, int n,
                          const float *th, uint16_t *wpk, uint16_t *a2, float *out, hipStream_t s);
hipError_t launch_cnn_bwd(const int64_t *q, double qs, const float *phibar, int64_t rs, int n, const float *th,
                          const float *z1, const uint16_t *a1, const float *z2, const uint16_t *a2, float *g1,
                          float *g2, float *dth, hipStream_t s);
hipError_t launch_force_loss(float *acc, const float *target, int64_t n3, double *red, hipStream_t s);
hipError_t launch_adam(float *th, float *m, float *v, const float *g, int64_t n, double lr, double b1, double b2,
                       double eps, int t, hipStream_t s);

// ---- launchers (paint.hip)
hipError_t launch_paint(const float *x, int64_t stride, int64_t first, int64_t count, int64_t quantum,
                        int n, int64_t *mesh, hipStream_t s);
hipError_t launch_paint_tagged(const float *x, int64_t P, const uint8_t *tags, int seg_lo, int seg_hi,
                               const int64_t *quanta, int n, int64_t *mesh, hipStream_t s);
hipError_t launch_paint_tiles(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int seg_lo,
                              int seg_hi, int n, int64_t *mesh, hipStream_t s);
// The same, added to mesh (int64 [N]^3) instead of overwriting its tiles.
hipError_t launch_paint_tiles_add(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int seg_lo,
                                  int seg_hi, int n, int64_t *mesh, hipStream_t s);
// Tile paint of every segment, stored as the float32 density contrast
// (float)(Q scale + offset) of each cell's exact int64 sum (overflow flag as
// the transforms raise it).
hipError_t launch_paint_tiles_delta(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int n,
                                    double scale, double offset, float *delta, int *flag, hipStream_t s);

// ---- launchers (sort.hip)
// Counting sort by tile key: counts per key (cnt zeroed by the caller), an
// exclusive scan (out2: a second copy, the scatter's cursors), and the
// scatter of particles to their cursor slots (cursor advanced by the counts).
hipError_t launch_sort_count(const float *x, int64_t P, int n, int *cnt, hipStream_t s);
hipError_t launch_scan(const int *in, int *out, int64_t n, int *block_sums, hipStream_t s, int *out2 = nullptr);
hipError_t launch_sort_scatter(const float *x, const float *p, const uint8_t *tag_in, int64_t P, int nseg,
                               const int64_t *seg_off, int n, int *cursor, float4 *xs, Mom3 *ps,
                               const uint32_t *ids_in, uint32_t *ids_out, hipStream_t s);
// FLAG_STALE unless cursor[k] == koff[k + 1] for every key k < K.
hipError_t launch_sort_verify(const int *cursor, const int *koff, int64_t K, int *flag, hipStream_t s);

// ---- launchers (particles.hip)
hipError_t launch_fill_i64(int64_t *p, int64_t count, hipStream_t s);
// rs_f, ps_f, comp_stride: row, plane and component strides of the force
// meshes in complex values (real rows of 2 rs_f floats).
hipError_t launch_readout(const float *x, int64_t P, const float2 *f, int64_t rs_f, int64_t ps_f, int64_t comp_stride,
                          int n, float *acc, hipStream_t s);
hipError_t launch_readout_kick_drift(float *x, float *p, int64_t P, const float2 *f, int64_t rs_f, int64_t ps_f,
                                     int64_t comp_stride, int n, float kick, float drift, int *flag,
                                     hipStream_t s);
// cnt_next (optional): counts per sort key of the positions written, added to.
hipError_t launch_readout_kd_tiles(const float4 *xs, const Mom3 *ps, int64_t P, const int *koff, const float2 *f,
                                   int64_t rs_f, int64_t ps_f, int64_t comp_stride, int n, float kick, float drift,
                                   float *x, float *p, uint8_t *tags, const uint32_t *ids_tmp, uint32_t *ids, int *flag,
                                   int *cnt_next, hipStream_t s);
hipError_t launch_fill_i32(int *p, int64_t count, hipStream_t s);
hipError_t launch_add_i64(const int64_t *src, int64_t *dst, int64_t count, hipStream_t s);
hipError_t launch_tags_canonical(uint8_t *tags, int64_t P, int nseg, const int64_t *seg_off, hipStream_t s);
hipError_t launch_copy_real(const float *src, int64_t rs, int64_t ps, int n, float *dst, hipStream_t s);
hipError_t launch_copy_half(const float2 *src, int64_t rs, int n, float2 *dst, hipStream_t s);
hipError_t launch_load_half(const float2 *src, int n, float2 *dst, int64_t rs, hipStream_t s);
hipError_t launch_ic_cdm(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, double vfac,
                         float *x, float *p, int64_t P, hipStream_t s);
hipError_t launch_ic_nu(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, int ns,
                        int n_dir, int n_shell, const float *tables, double vfac, int flip, float *x,
                        float *p, int64_t P, int64_t nc, hipStream_t s);
// Pseudo-random neutrinos: one per site, speed from the cumulative table cdf
// [nq + 1] at q = i hq, direction from the uniforms u [3][ns^3].
hipError_t launch_ic_nu_pseudo(const float2 *f, int64_t rs, int64_t comp_stride, int nic, int n, int ns,
                               const float *cdf, int nq, double hq, double pth_unit, double vfac, const float *u,
                               float *x, float *p, int64_t P, int64_t nc, hipStream_t s);
hipError_t launch_power_bin(const float2 *A, const float2 *B, int64_t rs, int n, int nbins, int compensate,
                            double norm, double kf, double *partial, hipStream_t s);
hipError_t launch_power_reduce(const double *partial, int nbins, double *out, hipStream_t s);

}  // namespace pm
