/*
 * Oracle FFT (test infrastructure only; see orc.h).
 *
 * A textbook radix-2 decimation-in-time transform with bit reversal and
 * twiddles evaluated directly with cos/sin in double precision.  The 3D
 * transform applies it along each axis in turn.  The real-to-complex and
 * complex-to-real variants are defined through the full complex transform so
 * that they are correct by construction: the half spectrum is the slice
 * 0 <= k2 <= n/2 of the full spectrum, and the inverse rebuilds the full
 * spectrum from Hermitian symmetry X(-k) = conj X(k).
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static void fft_inplace(cplx *a, long n, int sign)
{
    /* bit-reversal permutation */
    for (long i = 1, j = 0; i < n; i++) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (long len = 2; len <= n; len <<= 1) {
        long half = len >> 1;
        for (long k = 0; k < half; k++) {
            double ang = sign * 2.0 * M_PI * (double)k / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (long s = 0; s < n; s += len) {
                cplx u = a[s + k];
                cplx v = a[s + k + half] * w;
                a[s + k] = u + v;
                a[s + k + half] = u - v;
            }
        }
    }
}

void orc_fft1d(double *c, long n, int sign)
{
    fft_inplace((cplx *)c, n, sign);
}

/* Transform along every axis of an n^3 complex array (index (i0*n+i1)*n+i2). */
void orc_fft3d(double *c, long n, int sign)
{
    cplx *a = (cplx *)c;
    long n2 = n * n;
    /* axis 2: contiguous rows */
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < n2; r++) fft_inplace(a + r * n, n, sign);
    /* axis 1 */
    #pragma omp parallel
    {
        cplx *col = malloc(sizeof(cplx) * n);
        #pragma omp for schedule(static)
        for (long t = 0; t < n2; t++) {
            long i0 = t / n, i2 = t % n;
            for (long i1 = 0; i1 < n; i1++) col[i1] = a[(i0 * n + i1) * n + i2];
            fft_inplace(col, n, sign);
            for (long i1 = 0; i1 < n; i1++) a[(i0 * n + i1) * n + i2] = col[i1];
        }
        free(col);
    }
    /* axis 0 */
    #pragma omp parallel
    {
        cplx *col = malloc(sizeof(cplx) * n);
        #pragma omp for schedule(static)
        for (long t = 0; t < n2; t++) {
            for (long i0 = 0; i0 < n; i0++) col[i0] = a[i0 * n2 + t];
            fft_inplace(col, n, sign);
            for (long i0 = 0; i0 < n; i0++) a[i0 * n2 + t] = col[i0];
        }
        free(col);
    }
}

/* The definition itself, O(n^6): only for tiny meshes (pins the FFT). */
void orc_dft3d_naive(const double *in, double *out, long n, int sign)
{
    const cplx *x = (const cplx *)in;
    cplx *X = (cplx *)out;
    long m = n * n * n;
    #pragma omp parallel for schedule(static)
    for (long k = 0; k < m; k++) {
        long k0 = k / (n * n), k1 = (k / n) % n, k2 = k % n;
        cplx s = 0;
        for (long j = 0; j < m; j++) {
            long j0 = j / (n * n), j1 = (j / n) % n, j2 = j % n;
            long ph = (k0 * j0 + k1 * j1 + k2 * j2) % n;
            double ang = sign * 2.0 * M_PI * (double)ph / (double)n;
            s += x[j] * (cos(ang) + I * sin(ang));
        }
        X[k] = s;
    }
}

/* half[i0][i1][k2], k2 = 0..n/2: forward transform of a real n^3 field. */
void orc_rfft3d(const double *real, double *half, long n)
{
    long m = n * n * n, nh = n / 2 + 1;
    cplx *full = malloc(sizeof(cplx) * m);
    for (long i = 0; i < m; i++) full[i] = real[i];
    orc_fft3d((double *)full, n, -1);
    cplx *h = (cplx *)half;
    for (long r = 0; r < n * n; r++)
        for (long k2 = 0; k2 < nh; k2++) h[r * nh + k2] = full[r * n + k2];
    free(full);
}

/* Unnormalised inverse of a half spectrum to a real field (result is n^3 times
 * the field whose forward transform is `half`). */
void orc_irfft3d(const double *half, double *real, long n)
{
    long m = n * n * n, nh = n / 2 + 1;
    const cplx *h = (const cplx *)half;
    cplx *full = malloc(sizeof(cplx) * m);
    for (long i0 = 0; i0 < n; i0++)
        for (long i1 = 0; i1 < n; i1++)
            for (long k2 = 0; k2 < n; k2++) {
                cplx v;
                if (k2 < nh) {
                    v = h[(i0 * n + i1) * nh + k2];
                } else {
                    long j0 = (n - i0) % n, j1 = (n - i1) % n, j2 = n - k2;
                    v = conj(h[(j0 * n + j1) * nh + j2]);
                }
                full[(i0 * n + i1) * n + k2] = v;
            }
    orc_fft3d((double *)full, n, +1);
    for (long i = 0; i < m; i++) real[i] = creal(full[i]);
    free(full);
}
