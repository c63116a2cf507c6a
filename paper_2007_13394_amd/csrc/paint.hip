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

__global__ __launch_bounds__(256) void k_paint(const float *__restrict__ x, int64_t stride, int64_t first,
                                               int64_t count, long long quantum, int n,
                                               unsigned long long *mesh)
{
    const double qd = (double)quantum;
    const int mask = n - 1;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = first + t;
        int c[3][2];
        double w[3][2];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const float u = x[d * stride + i];
            const float f = floorf(u);
            const int id = (int)f;
            const double dd = (double)(u - f);
            w[d][0] = 1.0 - dd;
            w[d][1] = dd;
            c[d][0] = id & mask;
            c[d][1] = (id + 1) & mask;
        }
        long long acc = 0;
        int corner = 0;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int e = 0; e < 2; e++, corner++) {
                    long long q;
                    if (corner < 7) {
                        const double wq = ((w[0][a] * w[1][b]) * w[2][e]) * qd;
                        q = (long long)__builtin_rint(wq);
                        acc += q;
                    } else {
                        q = quantum - acc;
                    }
                    const int64_t idx = ((int64_t)c[0][a] * n + c[1][b]) * n + c[2][e];
                    __hip_atomic_fetch_add(mesh + idx, (unsigned long long)q, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
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

}  // namespace pm
