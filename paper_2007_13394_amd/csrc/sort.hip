// Counting sort of particles by mesh tile, done at the start of every step
// so that the paint and the readout can work tile by tile out of LDS.
//
// Key of a particle = 8 * tile + face flags: tile is the Morton index of the
// TILE^3-cell block holding floor(u); bit d of the flags is set when floor(u_d) is the last
// cell of the tile along axis d (its +1 cloud-in-cell corner then lies in the
// next tile).  Counting: one atomic per distinct key per wavefront (lanes
// sharing a key are ranked by ballot), so lattice-ordered CDM, where most of
// a wavefront falls in one tile, costs few atomics.  Offsets come from an
// exclusive scan of the counts; the scatter writes the position record (with
// the segment tag), the momentum and the optional id of particle i to
// offset[key_i] + rank_i.
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

__device__ __forceinline__ int tile_key(float u0, float u1, float u2, int n)
{
    const int mask = n - 1;
    const int c0 = (int)floorf(u0) & mask, c1 = (int)floorf(u1) & mask, c2 = (int)floorf(u2) & mask;
    const int t = tile_index(c0 / TILE, c1 / TILE, c2 / TILE);
    const int f = ((c0 % TILE) == TILE - 1 ? 1 : 0) | ((c1 % TILE) == TILE - 1 ? 2 : 0) |
                  ((c2 % TILE) == TILE - 1 ? 4 : 0);
    return t * 8 + f;
}

// Each workgroup takes SORT_CH consecutive particles, workgroups numbered so
// that each XCD owns a contiguous run of chunks (the scatter of a nearly
// sorted state then writes whole cache lines from one L2).
constexpr int SORT_T = 256, SORT_CH = SORT_T * 8;

__global__ __launch_bounds__(SORT_T) void k_sort_count(const float *__restrict__ x, int64_t P, int n, int *cnt,
                                                       int *key, int *rank)
{
    const int lane = threadIdx.x & 63;
    const int64_t c0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * SORT_CH;
    const int64_t c1 = c0 + SORT_CH < P ? c0 + SORT_CH : P;
    if (c0 >= c1) return;
    // The next round's position is loaded before this round's atomic, so the
    // two memory round trips of a round overlap.  Indices past the chunk are
    // clamped to c0, a valid particle.
    int64_t i = c0 + threadIdx.x;
    float a0, a1, a2;
    {
        const int64_t ic = i < c1 ? i : c0;
        a0 = x[ic];
        a1 = x[P + ic];
        a2 = x[2 * P + ic];
        // taken here, the first loads leave nothing for the loop head to wait
        // on (a wait there would also hold for the previous round's stores)
        asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2));
    }
    for (int64_t base = c0; base < c1; base += SORT_T, i += SORT_T) {
        const bool live = i < c1;
        const int k = live ? tile_key(a0, a1, a2, n) : -1;
        {
            const int64_t in = i + SORT_T, ic = in < c1 ? in : c0;
            a0 = x[ic];
            a1 = x[P + ic];
            a2 = x[2 * P + ic];
        }
        // group lanes with equal keys (ballot loop: no memory traffic), then
        // the leader of every group issues its atomic in one instruction
        uint64_t todo = __ballot(live);
        uint64_t group = 0;
        int leader = 0;
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
        int b = 0;
        if (live && lane == leader) b = atomicAdd(cnt + k, __popcll(group));
        b = __shfl(b, leader);
        const int r = b + __popcll(group & ((1ull << lane) - 1));
        if (live) {
            key[i] = k;
            rank[i] = r;
        }
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

__global__ void k_scan_add(int *out, int64_t n, const int *sums)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] += sums[i / SCAN_B];
}

// Scatter into float4 records: one 16-byte store for the position and the
// segment tag, one for the momentum, so a particle that moves far in the
// order costs two stores instead of seven partial ones.  The optional arrays
// are template flags, so every load of a particle is issued at once (one
// round trip, then the dependent offset lookup); the pointers do not alias
// (caller arrays in, workspace records out), which lets unrolled iterations
// overlap.
template <bool HP, bool HT, bool HI>
__device__ __forceinline__ void scatter_chunk(int64_t c0, int64_t c1, const float *__restrict__ x,
                                              const float *__restrict__ p, const uint8_t *__restrict__ tag_in,
                                              int64_t P, int nseg, const int64_t *__restrict__ seg_off,
                                              const int *__restrict__ key, const int *__restrict__ rank,
                                              const int *__restrict__ off, float4 *__restrict__ xs,
                                              float4 *__restrict__ ps, const uint32_t *__restrict__ ids_in,
                                              uint32_t *__restrict__ ids_out)
{
#pragma unroll 2
    for (int64_t i = c0 + threadIdx.x; i < c1; i += SORT_T) {
        const int k = key[i], r = rank[i];
        const float a0 = x[i], a1 = x[P + i], a2 = x[2 * P + i];
        float b0 = 0.f, b1 = 0.f, b2 = 0.f;
        if constexpr (HP) {
            b0 = p[i];
            b1 = p[P + i];
            b2 = p[2 * P + i];
        }
        int t = 0;
        if constexpr (HT) {
            t = tag_in[i];
        } else {   // canonical order: segment from the offsets
            for (int g = 1; g < nseg; g++) t += (i >= seg_off[g]) ? 1 : 0;
        }
        uint32_t id = 0;
        if constexpr (HI) id = ids_in[i];
        const int64_t d = (int64_t)off[k] + r;
        xs[d] = make_float4(a0, a1, a2, __int_as_float(t));
        if constexpr (HP) ps[d] = make_float4(b0, b1, b2, 0.f);
        if constexpr (HI) ids_out[d] = id;
    }
}

__global__ __launch_bounds__(SORT_T) void k_sort_scatter(const float *__restrict__ x, const float *__restrict__ p,
                                                         const uint8_t *__restrict__ tag_in, int64_t P, int nseg,
                                                         const int64_t *__restrict__ seg_off, const int *key,
                                                         const int *rank, const int *off, float4 *xs, float4 *ps,
                                                         const uint32_t *ids_in, uint32_t *ids_out)
{
    const int64_t c0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * SORT_CH;
    const int64_t c1 = c0 + SORT_CH < P ? c0 + SORT_CH : P;
#define SCATTER(HP, HT, HI) \
    scatter_chunk<HP, HT, HI>(c0, c1, x, p, tag_in, P, nseg, seg_off, key, rank, off, xs, ps, ids_in, ids_out)
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

}  // namespace

hipError_t launch_sort_count(const float *x, int64_t P, int n, int *cnt, int *key, int *rank, hipStream_t s)
{
    const int64_t nb = (P + SORT_CH - 1) / SORT_CH;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_count, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SORT_T), 0, s, x, P, n, cnt, key, rank);
    return hipGetLastError();
}

hipError_t launch_scan(const int *in, int *out, int64_t n, int *block_sums, hipStream_t s)
{
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb > (int64_t)SCAN_B * 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, block_sums, (int)nb);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n, 256)), dim3(256), 0, s, out, n, block_sums);
    return hipGetLastError();
}

hipError_t launch_sort_scatter(const float *x, const float *p, const uint8_t *tag_in, int64_t P, int nseg,
                               const int64_t *seg_off, const int *key, const int *rank, const int *off, float4 *xs,
                               float4 *ps, const uint32_t *ids_in, uint32_t *ids_out, hipStream_t s)
{
    const int64_t nb = (P + SORT_CH - 1) / SORT_CH;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(SORT_T), 0, s, x, p, tag_in, P, nseg, seg_off, key,
                       rank, off, xs, ps, ids_in, ids_out);
    return hipGetLastError();
}

}  // namespace pm
