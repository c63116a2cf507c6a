// Cloud-in-cell mass assignment into an int64 fixed-point mesh.
//
// FastPM assigns particle mass to the force mesh with cloud-in-cell weights
// (particle-mesh method, Sec. 1 and 2.3 of the paper).  Here each particle's
// eight corner weights are formed in double precision as products of
// (1 - d, d) per axis, d = u - floor(u) taken exactly in float32, multiplied
// by the particle's integer mass quantum and rounded to the nearest integer;
// the eighth corner receives the quantum minus the other seven.  Every
// particle therefore adds exactly its quantum, and integer addition makes the
// mesh independent of the order in which atomics land: the result is
// bit-identical run to run.  This file is compiled without floating-point
// contraction so that the weight arithmetic is exactly the sequence written.
#include "pm_internal.h"

namespace pm {
namespace {

// Cells and integer quanta of one particle's eight corners (corner order:
// axis 2 fastest).  Every kernel that paints uses this, so a particle's
// split is identical whichever kernel or workgroup computes it.
__device__ __forceinline__ void cic_quanta(float u0, float u1, float u2, long long quantum, int mask,
                                           int c[3][2], long long q[8])
{
    const float u[3] = {u0, u1, u2};
    double w[3][2];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const float f = floorf(u[d]);
        const int id = (int)f;
        const double dd = (double)(u[d] - f);
        w[d][0] = 1.0 - dd;
        w[d][1] = dd;
        c[d][0] = id & mask;
        c[d][1] = (id + 1) & mask;
    }
    const double qd = (double)quantum;
    long long acc = 0;
    int corner = 0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int e = 0; e < 2; e++, corner++) {
                if (corner < 7) {
                    const double wq = ((w[0][a] * w[1][b]) * w[2][e]) * qd;
                    q[corner] = (long long)__builtin_rint(wq);
                    acc += q[corner];
                } else {
                    q[corner] = quantum - acc;
                }
            }
}

__device__ __forceinline__ void add_corners(const int c[3][2], const long long q[8], int n, unsigned long long *mesh)
{
    int corner = 0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int e = 0; e < 2; e++, corner++) {
                const int64_t idx = ((int64_t)c[0][a] * n + c[1][b]) * n + c[2][e];
                __hip_atomic_fetch_add(mesh + idx, (unsigned long long)q[corner], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
}

__global__ __launch_bounds__(256) void k_paint(const float *__restrict__ x, int64_t stride, int64_t first,
                                               int64_t count, long long quantum, int n,
                                               unsigned long long *mesh)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = first + t;
        int c[3][2];
        long long q[8];
        cic_quanta(x[i], x[stride + i], x[2 * stride + i], quantum, n - 1, c, q);
        add_corners(c, q, n, mesh);
    }
}

// Particles in any order, each with its segment tag; segments [lo, hi) only.
__global__ __launch_bounds__(256) void k_paint_tagged(const float *__restrict__ x, int64_t P,
                                                      const uint8_t *__restrict__ tags, int lo, int hi,
                                                      const int64_t *__restrict__ quanta, int n,
                                                      unsigned long long *mesh)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = tags[i];
        if (g < lo || g >= hi) continue;
        int c[3][2];
        long long q[8];
        cic_quanta(x[i], x[P + i], x[2 * P + i], (long long)quanta[g], n - 1, c, q);
        add_corners(c, q, n, mesh);
    }
}

// One workgroup per TILE^3 tile of the mesh, particles sorted by tile and
// face flags (koff: offsets per key 8 * tile + flags).  The tile's cells get
// corners from its own particles and from particles of the seven lower
// neighbour tiles whose flags say a +1 corner crosses into this tile.  The
// sums are formed with LDS atomics and the tile is written once with plain
// stores, so the mesh needs no zero fill and no global atomics.  The own
// tile's particles (one contiguous range) and the 19 neighbour ranges are
// walked as one flat index space, two particles per thread per round, so
// that the global loads of a thread are independent of each other.
// Output modes.  PAINT_STORE: the int64 sums overwrite the tile.  PAINT_ADD:
// they are added to the tile (tiles are disjoint, so plain loads and stores).
// PAINT_DELTA: the exact int64 sums are not stored; each cell is written as
// the float32 density contrast (float)(Q scale + offset), the value the
// real-to-complex pass would form from the int64 cell, and cells below
// GUARD_MIN_Q raise the overflow flag (half the bytes of an int64 mesh,
// written once and read once by the transform).
enum { PAINT_STORE = 0, PAINT_ADD = 1, PAINT_DELTA = 2 };
// 512 threads, two particles each per round: the 33 KB of LDS allow four workgroups per CU, and eight
// waves each hide the latency of the range, particle and store phases.  At C3 (2048^3) this takes
// 16.7 ms against 18.6 ms for four particles per thread, 19.1 ms for 256 threads with four each and
// 24.1 ms for 1024 threads with two; at 256^3 (19 M particles) the same order holds.
constexpr int PAINT_T = 512, NPT = 2;   // NPT particles per thread per round

template <int MODE>
__global__ __launch_bounds__(PAINT_T) void k_paint_tiles(const float4 *__restrict__ xs,
                                                         const int *__restrict__ koff,
                                                         const int64_t *__restrict__ quanta, int nseg, int lo,
                                                         int hi, int n, void *out, double scale, double offset,
                                                         int *flag)
{
    __shared__ unsigned long long acc[TILE * TILE * TILE];
    __shared__ long long qtab[MAX_SEG];
    __shared__ int rbeg[NRANGE], rpre[NRANGE + 1];
    const int nt = n / TILE, mask = n - 1;
    // workgroups walk the tiles in Morton order (the sort keys' order, nt a
    // power of two): the neighbour ranges a tile reads were mostly just read
    // by the tiles around it
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int t2 = (int)morton_compact((unsigned)t), t1 = (int)morton_compact((unsigned)t >> 1),
              t0 = (int)morton_compact((unsigned)t >> 2);
    for (int i = threadIdx.x; i < TILE * TILE * TILE; i += PAINT_T) acc[i] = 0;
    for (int i = threadIdx.x; i < nseg; i += PAINT_T) qtab[i] = quanta[i];
    tile_ranges(koff, t, t0, t1, t2, nt, rbeg, rpre);
    const int total = rpre[NRANGE];
    const int ox = t0 * TILE, oy = t1 * TILE, oz = t2 * TILE;
    for (int k0 = threadIdx.x; k0 < total; k0 += NPT * PAINT_T) {
        int idx[NPT];
        bool ok[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            const int k = k0 + u * PAINT_T;
            ok[u] = k < total;
            idx[u] = ok[u] ? tile_range_index(k, rbeg, rpre) : 0;
        }
        // All loads unconditional (idx 0, a valid particle whenever the loop
        // runs, stands in past the end) and issued back to back: a load under
        // a branch is joined with the other path's value, and the join waits
        // for it.  The empty asm takes every loaded value, so no load can be
        // sunk into the branch that uses it (one memory round trip per round).
        float4 r[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) r[u] = xs[idx[u]];
#pragma unroll
        for (int u = 0; u < NPT; u++) asm volatile("" : "+v"(r[u].x), "+v"(r[u].y), "+v"(r[u].z), "+v"(r[u].w));
        float u0[NPT], u1[NPT], u2[NPT];
        int g[NPT];
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            u0[u] = r[u].x;
            u1[u] = r[u].y;
            u2[u] = r[u].z;
            g[u] = ok[u] ? __float_as_int(r[u].w) : -1;
        }
#pragma unroll
        for (int u = 0; u < NPT; u++) {
            if (!ok[u] || g[u] < lo || g[u] >= hi) continue;
            int c[3][2];
            long long q[8];
            cic_quanta(u0[u], u1[u], u2[u], (long long)qtab[g[u]], mask, c, q);
            int corner = 0;
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int d = 0; d < 2; d++, corner++) {
                        const int l0 = c[0][a] - ox, l1 = c[1][b] - oy, l2 = c[2][d] - oz;
                        if ((unsigned)l0 < TILE && (unsigned)l1 < TILE && (unsigned)l2 < TILE)
                            atomicAdd(&acc[(l0 * TILE + l1) * TILE + l2], (unsigned long long)q[corner]);
                    }
        }
    }
    __syncthreads();
    if constexpr (MODE == PAINT_DELTA) {
        // four cells of a row per thread: one 16-byte store
        float *dm = static_cast<float *>(out);
        bool bad = false;
        for (int i = threadIdx.x; i < TILE * TILE * TILE / 4; i += PAINT_T) {
            const int l0 = i / (TILE * TILE / 4), l1 = (i / (TILE / 4)) % TILE, l2 = 4 * (i % (TILE / 4));
            const long long *a = reinterpret_cast<const long long *>(acc) + (l0 * TILE + l1) * TILE + l2;
            float4 v;
            v.x = (float)((double)a[0] * scale + offset);
            v.y = (float)((double)a[1] * scale + offset);
            v.z = (float)((double)a[2] * scale + offset);
            v.w = (float)((double)a[3] * scale + offset);
            bad |= (a[0] < GUARD_MIN_Q) | (a[1] < GUARD_MIN_Q) | (a[2] < GUARD_MIN_Q) | (a[3] < GUARD_MIN_Q);
            *reinterpret_cast<float4 *>(dm + ((int64_t)(ox + l0) * n + (oy + l1)) * n + (oz + l2)) = v;
        }
        if (bad) atomicOr(flag, FLAG_OVERFLOW);
    } else {
        unsigned long long *mesh = static_cast<unsigned long long *>(out);
        for (int i = threadIdx.x; i < TILE * TILE * TILE; i += PAINT_T) {
            const int l0 = i / (TILE * TILE), l1 = (i / TILE) % TILE, l2 = i % TILE;
            unsigned long long *cell = mesh + ((int64_t)(ox + l0) * n + (oy + l1)) * n + (oz + l2);
            if constexpr (MODE == PAINT_ADD)
                *cell += acc[i];
            else
                *cell = acc[i];
        }
    }
}

}  // namespace

hipError_t launch_paint(const float *x, int64_t stride, int64_t first, int64_t count, int64_t quantum, int n,
                        int64_t *mesh, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536 * 8) blocks = 65536 * 8;
    hipLaunchKernelGGL(k_paint, dim3((unsigned)blocks), dim3(256), 0, s, x, stride, first, count,
                       (long long)quantum, n, reinterpret_cast<unsigned long long *>(mesh));
    return hipGetLastError();
}

hipError_t launch_paint_tagged(const float *x, int64_t P, const uint8_t *tags, int seg_lo, int seg_hi,
                               const int64_t *quanta, int n, int64_t *mesh, hipStream_t s)
{
    int64_t blocks = (P + 255) / 256;
    if (blocks > 65536 * 8) blocks = 65536 * 8;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_paint_tagged, dim3((unsigned)blocks), dim3(256), 0, s, x, P, tags, seg_lo, seg_hi, quanta,
                       n, reinterpret_cast<unsigned long long *>(mesh));
    return hipGetLastError();
}

hipError_t launch_paint_tiles(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int seg_lo,
                              int seg_hi, int n, int64_t *mesh, hipStream_t s)
{
    const int nt = n / TILE;
    if (nt < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_paint_tiles<PAINT_STORE>, dim3((unsigned)(nt * nt * nt)), dim3(PAINT_T), 0, s, xs, koff, quanta,
                       nseg, seg_lo, seg_hi, n, static_cast<void *>(mesh), 0.0, 0.0, static_cast<int *>(nullptr));
    return hipGetLastError();
}

hipError_t launch_paint_tiles_add(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int seg_lo,
                                  int seg_hi, int n, int64_t *mesh, hipStream_t s)
{
    const int nt = n / TILE;
    if (nt < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_paint_tiles<PAINT_ADD>, dim3((unsigned)(nt * nt * nt)), dim3(PAINT_T), 0, s, xs, koff, quanta,
                       nseg, seg_lo, seg_hi, n, static_cast<void *>(mesh), 0.0, 0.0, static_cast<int *>(nullptr));
    return hipGetLastError();
}

hipError_t launch_paint_tiles_delta(const float4 *xs, const int *koff, const int64_t *quanta, int nseg, int n,
                                    double scale, double offset, float *delta, int *flag, hipStream_t s)
{
    const int nt = n / TILE;
    if (nt < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_paint_tiles<PAINT_DELTA>, dim3((unsigned)(nt * nt * nt)), dim3(PAINT_T), 0, s, xs, koff, quanta,
                       nseg, 0, nseg, n, static_cast<void *>(delta), scale, offset, flag);
    return hipGetLastError();
}

}  // namespace pm
