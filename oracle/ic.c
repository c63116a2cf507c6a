/*
 * Oracle simulation set-up: particle counts and masses, linear power spectrum,
 * Zel'dovich initial conditions for CDM and neutrino particles
 * (test infrastructure only; see orc.h).
 *
 * Paper passages followed:
 *   - N_c CDM lattice sites with one particle each; N_sites neutrino sites with
 *     N_shell x (2 N_fib + 1) particles each                    (Sec. 2.1, "N_n" eq.)
 *   - neutrino grid staggered with respect to the CDM grid, particles placed on
 *     spherical shells of radius proportional to their speed, shells of
 *     neighbouring sites not overlapping                          (Sec. 2.1, Fig. 1 caption)
 *   - Zel'dovich displacements at the starting redshift          (Sec. 2.2)
 *   - neutrino speeds scale with 1/m_1 for the effective species (Appendix A)
 *   - mean density: total matter Omega_c0 + Omega_nu0, neutrinos non-relativistic
 *                                                               (Sec. 2.2, "Om_pois" eq.)
 * Readings (the paper initialises with the reps two-fluid transfer functions,
 * which are not available here): BBKS transfer function with Gamma = Omega_m h,
 * sigma_8 normalising the CDM spectrum at z = 0, back-scaled with the growth
 * factor D; neutrino density transfer = CDM x 1/(1 + (k/k_fs)^2) with the
 * Lesgourgues-Pastor free-streaming scale; the same white noise drives both;
 * the IC grid is the CDM lattice; Nyquist planes are zeroed; a neutrino site
 * sits half an IC cell off the lattice along each axis and its displacement is
 * the band-limited field evaluated there (a phase shift before the inverse
 * transform); shell radius 0.4 x site spacing x q_shell / q_shell(last);
 * canonical thermal momentum q_shell k_B T_nu0 c / m_1, in mesh units.
 */
#include "orc.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>

typedef double complex cplx;
#define C_KMS 299792.458

long orc_num_particles(const orc_sim *s, long *n_cdm, long *n_nu)
{
    long nc = (long)s->n_cdm * s->n_cdm * s->n_cdm;
    long nn = (long)s->n_sites * s->n_sites * s->n_sites * s->n_shell * (2 * s->n_fib + 1);
    if (n_cdm) *n_cdm = nc;
    if (n_nu) *n_nu = nn;
    return nc + nn;
}

static double heaviest(const orc_cosmo *c)
{
    double m1 = 0;
    for (int j = 0; j < c->n_nu; j++) if (c->m_nu[j] > m1) m1 = c->m_nu[j];
    return m1;
}

static int shells_for(const orc_sim *s, double *edges, double *q_shell, double *m_shell)
{
    double alpha[3], m1 = heaviest(&s->cosmo);
    for (int j = 0; j < s->cosmo.n_nu; j++) alpha[j] = s->cosmo.m_nu[j] / m1;
    return orc_fd_shells(s->cosmo.n_nu, alpha, s->n_shell, 0.0, edges, q_shell, m_shell);
}

/* Segment 0 is CDM; segment 1 + i holds neutrino shell i.  Masses give a mean
 * of one mass unit per mesh cell for all matter; seg_q = llrint(mass 2^S). */
int orc_segments(const orc_sim *s, long *seg_off, double *seg_mass, int64_t *seg_q)
{
    long nc, nn;
    orc_num_particles(s, &nc, &nn);
    double M = (double)s->n_mesh * s->n_mesh * s->n_mesh;
    const orc_cosmo *c = &s->cosmo;
    seg_off[0] = 0;
    seg_off[1] = nc;
    seg_mass[0] = c->omega_c / c->omega_m * M / (double)nc;
    int nseg = 1;
    if (s->n_sites > 0) {
        double edges[65], q_shell[64], m_shell[64];
        if (s->n_shell > 64 || shells_for(s, edges, q_shell, m_shell)) return -1;
        long nsites = (long)s->n_sites * s->n_sites * s->n_sites;
        long per = nsites * (2 * s->n_fib + 1);
        for (int i = 0; i < s->n_shell; i++) {
            seg_off[2 + i] = nc + (i + 1) * per;
            seg_mass[1 + i] = c->omega_nu0 / c->omega_m * (M / (double)nsites) * m_shell[i] / (2 * s->n_fib + 1);
        }
        nseg += s->n_shell;
    }
    for (int i = 0; i < nseg; i++) seg_q[i] = llrint(ldexp(seg_mass[i], s->shift));
    return nseg;
}

double orc_bbks_T(double q)
{
    if (q <= 0) return 1.0;
    double x = 2.34 * q;
    double poly = 1.0 + 3.89 * q + pow(16.1 * q, 2) + pow(5.46 * q, 3) + pow(6.71 * q, 4);
    return log(1.0 + x) / x * pow(poly, -0.25);
}

/* k^n_s T^2(k / (Omega_m h)), k in h/Mpc. */
double orc_pk_unnorm(const orc_sim *s, double k)
{
    double T = orc_bbks_T(k / (s->cosmo.omega_m * s->cosmo.h));
    return pow(k, s->n_s) * T * T;
}

typedef struct { const orc_sim *s; double amp, R; } sig_ctx;

static double tophat(double x)
{
    if (x < 1e-3) return 1.0 - x * x / 10.0;
    return 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
}

static double sigma_integrand(double lnk, void *p)
{
    sig_ctx *c = (sig_ctx *)p;
    double k = exp(lnk);
    double W = tophat(k * c->R);
    return k * k * k * c->amp * orc_pk_unnorm(c->s, k) * W * W / (2.0 * M_PI * M_PI);
}

/* sigma(R) = [ 1/(2 pi^2) int k^2 P(k) W^2(kR) dk ]^(1/2) for P = amp x pk_unnorm. */
double orc_sigma_R(const orc_sim *s, double amp, double R)
{
    sig_ctx c = {s, amp, R};
    return sqrt(orc_integrate(sigma_integrand, &c, log(1e-6), log(1e3), 1e-12));
}

double orc_pk_amplitude(const orc_sim *s)
{
    double sig = orc_sigma_R(s, 1.0, 8.0);
    return s->sigma8 * s->sigma8 / (sig * sig);
}

static double wrap(double u, double n)
{
    u = fmod(u, n);
    if (u < 0) u += n;
    if (u >= n) u -= n;
    return u;
}

static long sgn_mode(long k, long n) { return k <= n / 2 ? k : k - n; }

/* Multiplier of mode t (full n^3 spectrum) that turns the white-noise spectrum
 * into displacement component d (Mpc/h): i k_d / k^2 sqrt(A P(k) / V_cell),
 * zero at k = 0 and on every Nyquist plane.  kind 0: CDM at lattice points;
 * kind 1: neutrinos, free-streaming suppressed and evaluated half a cell off
 * the lattice (phase exp(i k.h)). */
static cplx ic_mult(const orc_sim *s, long t, long n, int d, int kind, double amp, double kfs)
{
    double L = s->box, vcell = pow(L / n, 3);
    long k[3] = {sgn_mode(t / (n * n), n), sgn_mode((t / n) % n, n), sgn_mode(t % n, n)};
    for (int e = 0; e < 3; e++) if (labs(k[e]) == n / 2) return 0;
    double kv[3], k2 = 0;
    for (int e = 0; e < 3; e++) { kv[e] = 2.0 * M_PI * k[e] / L; k2 += kv[e] * kv[e]; }
    if (k2 == 0) return 0;
    double kk = sqrt(k2);
    cplx mult = sqrt(amp * orc_pk_unnorm(s, kk) / vcell);
    if (kind == 1) {
        double r = kk / kfs;
        mult /= (1.0 + r * r);
        double ph = 0.5 * (L / n) * (kv[0] + kv[1] + kv[2]);
        mult *= cos(ph) + I * sin(ph);
    }
    return I * kv[d] / k2 * mult;
}

/* Displacement (Mpc/h) of one component from the white-noise spectrum W:
 * inverse transform of the multiplied spectrum, normalised by 1/n^3. */
static void displacement(const orc_sim *s, const cplx *W, long n, int d, int kind, double amp,
                         double kfs, cplx *out)
{
    long m = n * n * n;
    for (long t = 0; t < m; t++) out[t] = ic_mult(s, t, n, d, kind, amp, kfs) * W[t];
    orc_fft3d((double *)out, n, +1);
    for (long t = 0; t < m; t++) out[t] /= (double)m;
}

/* x, p: [3][P] in mesh units.  disp_cdm [3][N_c], disp_nu [3][N_sites] (mesh
 * units) are optional outputs of the displacement fields used. */
static int ic_impl(const orc_sim *s, const float *white32, const double *white64, const double *uni, double *x,
                   double *p, double *disp_cdm, double *disp_nu)
{
    long n = s->n_cdm, m = n * n * n, nc, nn;
    long P = orc_num_particles(s, &nc, &nn);
    const orc_cosmo *c = &s->cosmo;
    double a2[2] = {s->a0, 1.0}, D[2], G[2];
    if (orc_growth(c, 2, a2, D, G, 1e-3)) return -1;
    double amp = orc_pk_amplitude(s) * pow(D[0] / D[1], 2);
    double vfac = G[0] / D[0];
    double to_mesh = s->n_mesh / s->box;
    double dc = (double)s->n_mesh / n;

    cplx *W = malloc(sizeof(cplx) * m), *S = malloc(sizeof(cplx) * m);
    for (long t = 0; t < m; t++) W[t] = white32 ? (double)white32[t] : white64[t];
    orc_fft3d((double *)W, n, -1);

    for (int d = 0; d < 3; d++) {
        displacement(s, W, n, d, 0, amp, 0.0, S);
        for (long t = 0; t < m; t++) {
            long i[3] = {t / (n * n), (t / n) % n, t % n};
            double sd = creal(S[t]) * to_mesh;
            x[d * P + t] = wrap(i[d] * dc + sd, s->n_mesh);
            p[d * P + t] = vfac * sd;
            if (disp_cdm) disp_cdm[d * nc + t] = sd;
        }
    }

    if (nn > 0) {
        double edges[65], q_shell[64], m_shell[64];
        if (s->n_shell > 64 || shells_for(s, edges, q_shell, m_shell)) { free(W); free(S); return -1; }
        int nd = 2 * s->n_fib + 1;
        double *dirs = malloc(sizeof(double) * 3 * nd);
        orc_fibonacci(s->n_fib, dirs);
        long ns = s->n_sites, nsites = ns * ns * ns, R = n / ns;
        double m1 = heaviest(c);
        double a0 = s->a0;
        double kfs = 0.82 * sqrt(c->omega_L + c->omega_m / (a0 * a0 * a0)) * a0 * a0 * m1;
        double spacing = R * dc;
        double pth_unit = c->kT_nu / m1 * C_KMS / 100.0 * to_mesh;
        double *snu = malloc(sizeof(double) * 3 * nsites);
        for (int d = 0; d < 3; d++) {
            displacement(s, W, n, d, 1, amp, kfs, S);
            for (long j = 0; j < nsites; j++) {
                long jj[3] = {j / (ns * ns), (j / ns) % ns, j % ns};
                long g[3];
                for (int e = 0; e < 3; e++) g[e] = jj[e] * R + R / 2;
                snu[d * nsites + j] = creal(S[(g[0] * n + g[1]) * n + g[2]]) * to_mesh;
                if (disp_nu) disp_nu[d * nsites + j] = snu[d * nsites + j];
            }
        }
        if (uni) {
            /* pseudo-random: one particle per site at the site, random speed and direction */
            double alpha[3];
            for (int j = 0; j < c->n_nu; j++) alpha[j] = c->m_nu[j] / m1;
            for (long j = 0; j < nsites; j++) {
                long jj[3] = {j / (ns * ns), (j / ns) % ns, j % ns};
                double q = orc_fd_qinv(c->n_nu, alpha, uni[j]);
                double ct = 2.0 * uni[nsites + j] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
                double ph = 2.0 * M_PI * uni[2 * nsites + j];
                double v[3] = {st * cos(ph), st * sin(ph), ct};
                for (int d = 0; d < 3; d++) {
                    double site = (jj[d] * R + R / 2 + 0.5) * dc;
                    x[d * P + nc + j] = wrap(site + snu[d * nsites + j], s->n_mesh);
                    p[d * P + nc + j] = q * pth_unit * v[d] + vfac * snu[d * nsites + j];
                }
            }
            free(snu);
            free(dirs);
            free(W);
            free(S);
            return 0;
        }
        long per = nsites * nd;
        for (int sh = 0; sh < s->n_shell; sh++) {
            double r = 0.4 * spacing * q_shell[sh] / q_shell[s->n_shell - 1];
            double pth = q_shell[sh] * pth_unit;
            for (long j = 0; j < nsites; j++) {
                long jj[3] = {j / (ns * ns), (j / ns) % ns, j % ns};
                double sign = (s->flip_odd && ((jj[0] + jj[1] + jj[2]) & 1)) ? -1.0 : 1.0;
                for (int t = 0; t < nd; t++) {
                    long idx = nc + sh * per + j * nd + t;
                    for (int d = 0; d < 3; d++) {
                        double site = (jj[d] * R + R / 2 + 0.5) * dc;
                        double v = sign * dirs[t * 3 + d];
                        x[d * P + idx] = wrap(site + r * v + snu[d * nsites + j], s->n_mesh);
                        p[d * P + idx] = pth * v + vfac * snu[d * nsites + j];
                    }
                }
            }
        }
        free(snu);
        free(dirs);
    }
    free(W);
    free(S);
    return 0;
}

int orc_ic(const orc_sim *s, const float *white, double *x, double *p, double *disp_cdm, double *disp_nu)
{
    return ic_impl(s, white, NULL, NULL, x, p, disp_cdm, disp_nu);
}

/* The same initial conditions from FP64 white noise (for derivative checks). */
int orc_ic_w64(const orc_sim *s, const double *white, double *x, double *p)
{
    return ic_impl(s, NULL, white, NULL, x, p, NULL, NULL);
}

int orc_ic_pseudo(const orc_sim *s, const float *white, const double *u, double *x, double *p)
{
    if (s->n_shell != 1 || s->n_fib != 0 || s->n_sites < 1) return -1;
    return ic_impl(s, white, NULL, u, x, p, NULL, NULL);
}

/* Vector-Jacobian product of the initial conditions with respect to the white
 * noise: wbar = (d(x, p)/dw)^T (xbar, pbar).  Positions and momenta are linear
 * in the displacement fields (x = q + s, p = (G/D) s; a neutrino site's 70
 * particles share its displacement), and each field is A w with
 * A = F^-1 diag(M) F for the unnormalised forward transform F; its transpose is
 * F^-1 diag(conj M) F, the same transforms with the multiplier conjugated. */
int orc_ic_vjp(const orc_sim *s, const double *xbar, const double *pbar, double *wbar)
{
    long n = s->n_cdm, m = n * n * n, nc, nn;
    long P = orc_num_particles(s, &nc, &nn);
    const orc_cosmo *c = &s->cosmo;
    double a2[2] = {s->a0, 1.0}, D[2], G[2];
    if (orc_growth(c, 2, a2, D, G, 1e-3)) return -1;
    double amp = orc_pk_amplitude(s) * pow(D[0] / D[1], 2);
    double vfac = G[0] / D[0];
    double to_mesh = s->n_mesh / s->box;
    cplx *acc = calloc(m, sizeof(cplx)), *F = malloc(sizeof(cplx) * m);
    for (int d = 0; d < 3; d++) {
        for (long t = 0; t < m; t++) F[t] = (xbar[d * P + t] + vfac * pbar[d * P + t]) * to_mesh;
        orc_fft3d((double *)F, n, -1);
        for (long t = 0; t < m; t++) acc[t] += conj(ic_mult(s, t, n, d, 0, amp, 0.0)) * F[t];
    }
    if (nn > 0) {
        long ns = s->n_sites, nsites = ns * ns * ns, R = n / ns;
        int nd = 2 * s->n_fib + 1;
        long per = nsites * nd;
        double m1 = 0;
        for (int j = 0; j < c->n_nu; j++) if (c->m_nu[j] > m1) m1 = c->m_nu[j];
        double a0 = s->a0;
        double kfs = 0.82 * sqrt(c->omega_L + c->omega_m / (a0 * a0 * a0)) * a0 * a0 * m1;
        for (int d = 0; d < 3; d++) {
            for (long t = 0; t < m; t++) F[t] = 0;
            for (long j = 0; j < nsites; j++) {
                long jj[3] = {j / (ns * ns), (j / ns) % ns, j % ns};
                double sum = 0;
                for (int sh = 0; sh < s->n_shell; sh++)
                    for (int t = 0; t < nd; t++) {
                        long idx = nc + sh * per + j * nd + t;
                        sum += xbar[d * P + idx] + vfac * pbar[d * P + idx];
                    }
                long g[3];
                for (int e = 0; e < 3; e++) g[e] = jj[e] * R + R / 2;
                F[(g[0] * n + g[1]) * n + g[2]] = sum * to_mesh;
            }
            orc_fft3d((double *)F, n, -1);
            for (long t = 0; t < m; t++) acc[t] += conj(ic_mult(s, t, n, d, 1, amp, kfs)) * F[t];
        }
    }
    orc_fft3d((double *)acc, n, +1);
    for (long t = 0; t < m; t++) wbar[t] = creal(acc[t]) / (double)m;
    free(acc);
    free(F);
    return 0;
}

