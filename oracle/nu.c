/*
 * Oracle quasi-random Fermi-Dirac sampling of neutrino thermal velocities
 * (test infrastructure only; see orc.h).
 *
 * Paper passages followed (Sec. 2.1):
 *   - f(q) = 1/(e^q + 1), dn = q^2 f(q) dq dOmega              ("fd", "dn" eqs.)
 *   - shell speed q_shell = sqrt(int q^4 f / int q^2 f) over
 *     the shell, shell mass fraction m_shell = int_shell q^2 f
 *     / int_0^qmax q^2 f                                        ("q_shell", "m_shell" eqs.)
 *   - shell edges with equal area under the kernel g(q) = q f(q) ("N_shell" eq. and text)
 *   - non-degenerate masses carried by one effective
 *     distribution f~(q) = sum_j alpha_j^4 f(alpha_j q),
 *     alpha_j = m_j / m_1, m_1 the heaviest                      ("FD_deg" eq., Appendix A)
 *   - 2 N_fib + 1 directions per shell on a Fibonacci sphere      (Sec. 2.1, after "FD_deg")
 *
 * Readings: the kernel for the effective distribution is g = q f~; the cut-off
 * is q_max = 30 / min(alpha) (q^2 f~ is below 1e-10 of its peak there);
 * Fibonacci lattice points i = -N_fib..N_fib at latitude asin(2i/(2N_fib+1))
 * and longitude 2 pi i / golden ratio, with the polar axis on mesh axis 2.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>

/* Gauss-Kronrod 7/15 nodes and weights (QUADPACK qk15). */
static const double xgk[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double wgk[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double wg[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

static void gk15(double (*f)(double, void *), void *ctx, double a, double b, double *K, double *err)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c, ctx);
    double rk = fc * wgk[7], rg = fc * wg[3];
    for (int j = 0; j < 7; j++) {
        double dx = h * xgk[j];
        double f1 = f(c - dx, ctx), f2 = f(c + dx, ctx);
        rk += wgk[j] * (f1 + f2);
        if (j % 2 == 1) rg += wg[j / 2] * (f1 + f2);
    }
    *K = rk * h;
    *err = fabs((rk - rg) * h);
}

static double adapt(double (*f)(double, void *), void *ctx, double a, double b, double eps, int depth)
{
    double K, err;
    gk15(f, ctx, a, b, &K, &err);
    if (err <= eps || depth > 40) return K;
    double m = 0.5 * (a + b);
    return adapt(f, ctx, a, m, 0.5 * eps, depth + 1) + adapt(f, ctx, m, b, 0.5 * eps, depth + 1);
}

/* Adaptive Gauss-Kronrod quadrature to a relative tolerance `tol`. */
double orc_integrate(double (*f)(double, void *), void *ctx, double a, double b, double tol)
{
    if (b <= a) return 0.0;
    double K, err;
    gk15(f, ctx, a, b, &K, &err);
    double scale = fabs(K);
    /* a coarse first estimate can underrate a peaked integrand: refine it once */
    double K2 = 0;
    int nsub = 64;
    for (int i = 0; i < nsub; i++) {
        double e;
        double lo = a + (b - a) * i / nsub, hi = a + (b - a) * (i + 1) / nsub;
        double Ki;
        gk15(f, ctx, lo, hi, &Ki, &e);
        K2 += Ki;
    }
    if (fabs(K2) > scale) scale = fabs(K2);
    double eps = tol * (scale > 0 ? scale : 1e-300);
    double s = 0;
    for (int i = 0; i < nsub; i++) {
        double lo = a + (b - a) * i / nsub, hi = a + (b - a) * (i + 1) / nsub;
        s += adapt(f, ctx, lo, hi, eps / nsub, 0);
    }
    return s;
}

double orc_fd_tilde(int n_nu, const double *alpha, double q)
{
    double s = 0;
    for (int j = 0; j < n_nu; j++) {
        double aj = alpha[j];
        s += aj * aj * aj * aj / (exp(aj * q) + 1.0);
    }
    return s;
}

typedef struct { int n_nu; const double *alpha; int power; } moment_ctx;

static double moment_integrand(double q, void *p)
{
    moment_ctx *m = (moment_ctx *)p;
    return pow(q, m->power) * orc_fd_tilde(m->n_nu, m->alpha, q);
}

static double moment(int n_nu, const double *alpha, int power, double a, double b)
{
    moment_ctx m = {n_nu, alpha, power};
    return orc_integrate(moment_integrand, &m, a, b, 1e-13);
}

/* Shell edges (n_shell+1 values), speeds and mass fractions.  q_max <= 0
 * selects the default cut-off 30 / min(alpha). */
int orc_fd_shells(int n_nu, const double *alpha, int n_shell, double q_max,
                  double *edges, double *q_shell, double *m_shell)
{
    if (n_nu < 1 || n_shell < 1) return -1;
    if (q_max <= 0) {
        double amin = alpha[0];
        for (int j = 1; j < n_nu; j++) if (alpha[j] < amin) amin = alpha[j];
        q_max = 30.0 / amin;
    }
    double g_tot = moment(n_nu, alpha, 1, 0.0, q_max);
    edges[0] = 0.0;
    edges[n_shell] = q_max;
    double below = 0.0; /* int_0^{edges[i-1]} g */
    for (int i = 1; i < n_shell; i++) {
        double target = g_tot * (double)i / (double)n_shell;
        double lo = edges[i - 1], hi = q_max;
        for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; it++) {
            double mid = 0.5 * (lo + hi);
            double v = below + moment(n_nu, alpha, 1, edges[i - 1], mid);
            if (v < target) lo = mid; else hi = mid;
        }
        edges[i] = 0.5 * (lo + hi);
        below += moment(n_nu, alpha, 1, edges[i - 1], edges[i]);
    }
    double n_tot = moment(n_nu, alpha, 2, 0.0, q_max);
    for (int i = 0; i < n_shell; i++) {
        double m2 = moment(n_nu, alpha, 2, edges[i], edges[i + 1]);
        double m4 = moment(n_nu, alpha, 4, edges[i], edges[i + 1]);
        q_shell[i] = sqrt(m4 / m2);
        m_shell[i] = m2 / n_tot;
    }
    return 0;
}

/* Inverse of the cumulative number distribution of the neutrino momenta,
 * C(q) = int_0^q q'^2 f~ dq' / int_0^q_max q'^2 f~ dq' (q_max = 30 / min alpha):
 * the q with C(q) = u, by bisection with the integral carried along (the
 * pseudo-random sampling of thermal speeds that the paper compares against). */
double orc_fd_qinv(int n_nu, const double *alpha, double u)
{
    double amin = alpha[0];
    for (int j = 1; j < n_nu; j++) if (alpha[j] < amin) amin = alpha[j];
    double q_max = 30.0 / amin;
    if (u <= 0.0) return 0.0;
    if (u >= 1.0) return q_max;
    double target = u * moment(n_nu, alpha, 2, 0.0, q_max);
    double lo = 0.0, hi = q_max, below = 0.0;   /* below = int_0^lo */
    for (int it = 0; it < 200 && hi - lo > 1e-15 * q_max; it++) {
        double mid = 0.5 * (lo + hi);
        double piece = moment(n_nu, alpha, 2, lo, mid);
        if (below + piece < target) { lo = mid; below += piece; } else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* dirs[(i + n_fib) * 3 + d], i = -n_fib..n_fib: unit vectors (axis 0, 1, 2). */
void orc_fibonacci(int n_fib, double *dirs)
{
    double phi = 0.5 * (1.0 + sqrt(5.0));
    int n = 2 * n_fib + 1;
    for (int i = -n_fib; i <= n_fib; i++) {
        double lat = asin(2.0 * i / (double)n);
        double lon = 2.0 * M_PI * i / phi;
        double *v = dirs + (i + n_fib) * 3;
        v[0] = cos(lat) * cos(lon);
        v[1] = cos(lat) * sin(lon);
        v[2] = sin(lat);
    }
}
