// Counting sort of particles by mesh tile, done at the start of every step
// so that the paint and the readout can work tile by tile out of LDS.
//
// Key of a particle = 8 * tile + face flags: tile is the Morton index of the
// TILE^3-cell block holding floor(u); bit d of the flags is set when floor(u_d) is the last
// cell of the tile along axis d (its +1 cloud-in-cell corner then lies in the
// next tile).  Counting: one atomic per distinct key per wavefront (lanes
// sharing a key are grouped by ballot), so lattice-ordered CDM, where most of
// a wavefront falls in one tile, costs few atomics.  Offsets come from an
// exclusive scan of the counts, which also leaves a copy of them as per-key
// cursors; the scatter recomputes each particle's key from its position,
// takes its slot from the cursor (one returning atomic per key and
// wavefront, lanes ranked by ballot), and writes the position record (with
// the segment tag), the momentum and the optional id there.  The order of
// particles within a key depends on the order of the atomics.
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


// Each workgroup takes SORT_CH consecutive particles, workgroups numbered so
// that each XCD owns a contiguous run of chunks (the scatter of a nearly
// sorted state then writes whole cache lines from one L2).
constexpr int SORT_T = 256, SORT_CH = SORT_T * 8;
// particles per batch in the scatter: two keep it at 38 VGPRs; four and eight
// (66, 114 VGPRs) gain nothing at 2048^3 and lose at 256^3 (lower occupancy)
constexpr int SCATTER_SB = 2;


__global__ __launch_bounds__(SORT_T) void k_sort_count(const float *__restrict__ x, int64_t P, int n, int *cnt)
{
    const int lane = threadIdx.x & 63;
    const int64_t c0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * SORT_CH;
    const int64_t c1 = c0 + SORT_CH < P ? c0 + SORT_CH : P;
    if (c0 >= c1) return;
    // All rounds' positions are loaded up front (8 per thread; indices past
    // the chunk are clamped to c0, a valid particle); the atomics return
    // nothing, so no round waits on memory after the first.
    constexpr int NR = SORT_CH / SORT_T;
    float a0[NR], a1[NR], a2[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int64_t i = c0 + threadIdx.x + r * SORT_T, ic = i < c1 ? i : c0;
        a0[r] = x[ic];
        a1[r] = x[P + ic];
        a2[r] = x[2 * P + ic];
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const bool live = c0 + threadIdx.x + r * SORT_T < c1;
        const int k = live ? tile_key(a0[r], a1[r], a2[r], n) : -1;
        uint64_t group;
        int leader;
        key_group(live, k, group, leader);
        if (live && lane == leader) atomicAdd(cnt + k, __popcll(group));
    }
}

// Exclusive scan in blocks of SCAN_B = 2048 values (256 threads x 8).
constexpr int SCAN_T = 256, SCAN_PER = 8, SCAN_B = SCAN_T * SCAN_PER;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh)
{
    // sh: SCAN_T ints; returns the exclusive prefix of v over the block, total in sh[SCAN_T - 1] + last v
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        const int t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    const int incl = sh[tid];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(const int *in, int *out, int64_t n, int *block_sums)
{
    __shared__ int sh[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B + (int64_t)threadIdx.x * SCAN_PER;
    int v[SCAN_PER], s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    const int pre = block_exclusive_scan(s, sh);
    int run = pre;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == SCAN_T - 1) block_sums[blockIdx.x] = run;
}

// Single block: exclusive scan of up to SCAN_B * 4 block sums, in place.
__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int *sums, int nb)
{
    __shared__ int sh[SCAN_T];
    int carry = 0;
    for (int start = 0; start < nb; start += SCAN_B) {
        const int base = start + threadIdx.x * SCAN_PER;
        int v[SCAN_PER], s = 0;
#pragma unroll
        for (int j = 0; j < SCAN_PER; j++) {
            v[j] = base + j < nb ? sums[base + j] : 0;
            s += v[j];
        }
        const int pre = block_exclusive_scan(s, sh);
        int run = carry + pre;
#pragma unroll
        for (int j = 0; j < SCAN_PER; j++) {
            if (base + j < nb) sums[base + j] = run;
            run += v[j];
        }
        // total of this chunk = inclusive value of the last thread
        if (threadIdx.x == SCAN_T - 1) sh[0] = run;
        __syncthreads();
        carry = sh[0];
        __syncthreads();
    }
}

// out2 (optional): a second copy of the result.
__global__ void k_scan_add(int *out, int64_t n, const int *sums, int *out2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int v = out[i] + sums[i / SCAN_B];
        out[i] = v;
        if (out2) out2[i] = v;
    }
}

// Scatter into float4 records: one 16-byte store for the position and the
// segment tag, one for the momentum, so a particle that moves far in the
// order costs two stores instead of seven partial ones.  The optional arrays
// are template flags.  A thread takes its eight particles in batches of SB:
// a batch's particles are loaded at once, then its cursor atomics are issued
// back to back, then its stores (two memory round trips per batch).  The
// pointers do not alias (caller arrays in, workspace records out).
template <bool HP, bool HT, bool HI, int SB>
__device__ __forceinline__ void scatter_chunk(int64_t c0, int64_t c1, const float *__restrict__ x,
                                              const float *__restrict__ p, const uint8_t *__restrict__ tag_in,
                                              int64_t P, int nseg, const int64_t *__restrict__ seg_off, int n,
                                              int *cursor, float4 *__restrict__ xs, Mom3 *__restrict__ ps,
                                              const uint32_t *__restrict__ ids_in, uint32_t *__restrict__ ids_out)
{
    constexpr int NR = SORT_CH / SORT_T;
    static_assert(NR % SB == 0, "whole batches");
    const int lane = threadIdx.x & 63;
    for (int r0 = 0; r0 < NR; r0 += SB) {
        // indices past the chunk are clamped to c0, a valid particle, and dropped
        float a0[SB], a1[SB], a2[SB], b0[SB], b1[SB], b2[SB];
        int t[SB];
        uint32_t id[SB];
#pragma unroll
        for (int r = 0; r < SB; r++) {
            const int64_t i = c0 + threadIdx.x + (r0 + r) * SORT_T, ic = i < c1 ? i : c0;
            a0[r] = x[ic];
            a1[r] = x[P + ic];
            a2[r] = x[2 * P + ic];
            if constexpr (HP) {
                b0[r] = p[ic];
                b1[r] = p[P + ic];
                b2[r] = p[2 * P + ic];
            } else {
                b0[r] = b1[r] = b2[r] = 0.f;
            }
            if constexpr (HT) {
                t[r] = tag_in[ic];
            } else {   // canonical order: segment from the offsets
                int g0 = 0;
                for (int g = 1; g < nseg; g++) g0 += (ic >= seg_off[g]) ? 1 : 0;
                t[r] = g0;
            }
            id[r] = 0;
            if constexpr (HI) id[r] = ids_in[ic];
        }
        uint64_t group[SB];
        int leader[SB], base[SB];
#pragma unroll
        for (int r = 0; r < SB; r++) {
            const bool live = c0 + threadIdx.x + (r0 + r) * SORT_T < c1;
            const int k = live ? tile_key(a0[r], a1[r], a2[r], n) : -1;
            key_group(live, k, group[r], leader[r]);
            base[r] = 0;
            if (live && lane == leader[r]) base[r] = atomicAdd(cursor + k, __popcll(group[r]));
        }
#pragma unroll
        for (int r = 0; r < SB; r++) {
            const bool live = c0 + threadIdx.x + (r0 + r) * SORT_T < c1;
            const int b = __shfl(base[r], leader[r]);
            const int64_t d = (int64_t)b + __popcll(group[r] & ((1ull << lane) - 1));
            if (live && d < P) {   // d >= P only with counts that do not match x (k_sort_verify reports it)
                xs[d] = make_float4(a0[r], a1[r], a2[r], __int_as_float(t[r]));
                if constexpr (HP) ps[d] = Mom3{b0[r], b1[r], b2[r]};
                if constexpr (HI) ids_out[d] = id[r];
            }
        }
    }
}

__global__ __launch_bounds__(SORT_T) void k_sort_scatter(const float *__restrict__ x, const float *__restrict__ p,
                                                         const uint8_t *__restrict__ tag_in, int64_t P, int nseg,
                                                         const int64_t *__restrict__ seg_off, int n, int *cursor,
                                                         float4 *xs, Mom3 *ps, const uint32_t *ids_in,
                                                         uint32_t *ids_out)
{
    const int64_t c0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * SORT_CH;
    const int64_t c1 = c0 + SORT_CH < P ? c0 + SORT_CH : P;
    if (c0 >= c1) return;
#define SCATTER(HP, HT, HI) \
    scatter_chunk<HP, HT, HI, SCATTER_SB>(c0, c1, x, p, tag_in, P, nseg, seg_off, n, cursor, xs, ps, ids_in, ids_out)
    if (p) {
        if (tag_in) {
            if (ids_in) SCATTER(true, true, true);
            else SCATTER(true, true, false);
        } else {
            if (ids_in) SCATTER(true, false, true);
            else SCATTER(true, false, false);
        }
    } else {
        if (tag_in) {
            if (ids_in) SCATTER(false, true, true);
            else SCATTER(false, true, false);
        } else {
            if (ids_in) SCATTER(false, false, true);
            else SCATTER(false, false, false);
        }
    }
#undef SCATTER
}

// After a scatter from counts computed elsewhere (the previous readout):
// every key's cursor must have reached the next key's offset, else the
// counts did not describe x and FLAG_STALE is raised.
__global__ __launch_bounds__(256) void k_sort_verify(const int *__restrict__ cursor, const int *__restrict__ koff,
                                                     int64_t K, int *flag)
{
    bool bad = false;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x)
        bad |= cursor[k] != koff[k + 1];
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, FLAG_STALE);
}

}  // namespace

hipError_t launch_sort_verify(const int *cursor, const int *koff, int64_t K, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_verify, dim3(grid_for(K, 256, 65536)), dim3(256), 0, s, cursor, koff, K, flag);
    return hipGetLastError();
}

hipError_t launch_sort_count(const float *x, int64_t P, int n, int *cnt, hipStream_t s)
{
    const int64_t nb = (P + SORT_CH - 1) / SORT_CH;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_count, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SORT_T), 0, s, x, P, n, cnt);
    return hipGetLastError();
}

hipError_t launch_scan(const int *in, int *out, int64_t n, int *block_sums, hipStream_t s, int *out2)
{
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb > (int64_t)SCAN_B * 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, block_sums, (int)nb);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n, 256)), dim3(256), 0, s, out, n, block_sums, out2);
    return hipGetLastError();
}

hipError_t launch_sort_scatter(const float *x, const float *p, const uint8_t *tag_in, int64_t P, int nseg,
                               const int64_t *seg_off, int n, int *cursor, float4 *xs, Mom3 *ps,
                               const uint32_t *ids_in, uint32_t *ids_out, hipStream_t s)
{
    const int64_t nb = (P + SORT_CH - 1) / SORT_CH;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SORT_T), 0, s, x, p, tag_in, P, nseg,
                       seg_off, n, cursor, xs, ps, ids_in, ids_out);
    return hipGetLastError();
}

}  // namespace pm
