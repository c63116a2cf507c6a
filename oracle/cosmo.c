/*
 * Oracle background cosmology, linear growth and FastPM step factors
 * (test infrastructure only; see orc.h).
 *
 * Paper passages followed:
 *   - Omega_nu0 = M_nu / (93.14 h^2 eV)                       (Introduction)
 *   - E(a) with photons, CDM, exact Fermi-Dirac neutrino
 *     density and Lambda; the F(y) integral                    (Sec. 2.3, "Hubble" eq.)
 *   - matter-only Poisson / growth source, neutrinos counted
 *     as matter                                                (Sec. 2.2, "Om_pois" eq.)
 *   - growth ODE in ln a with D = D' = a_ini at z_ini = 159    (Sec. 2.3, "growthDE" eq.)
 *   - modified kick/drift factors that make the Zel'dovich
 *     trajectory x = q + D(a) s exact                          (Sec. 2.3, first paragraph)
 *
 * Readings where the paper is silent:
 *   - Omega_gamma from T_cmb through the Stefan-Boltzmann law; Gamma_nu =
 *     (4/11)^(1/3) (N_eff/3)^(1/4).
 *   - the configured Omega_m includes neutrinos: Omega_c0 = Omega_m - Omega_nu0.
 *   - flat closure Omega_L = 1 - Omega_g - Omega_c0 - (Omega_nu E^2)(a=1), with
 *     the exact integral for today's neutrino density.
 *   - the printed source (Omega_c0+Omega_nu0) a^-3 is a density in units of
 *     today's critical density; in the ODE it enters divided by E^2(a) (only
 *     then is D = a a solution in matter domination).
 *   - with p the canonical momentum (dx/da = p/(a^3 E), dp/da = F/(a^2 E),
 *     F = -grad phi, lap phi = 1.5 Omega_m0 delta), let G(a) = a^2 E dD/dlna.
 *     On the Zel'dovich trajectory p = G s and F = 1.5 Omega_m0 D s, so the
 *     drift from a_i to a_j with momentum taken at a_r is (D_j - D_i)/G(a_r)
 *     and the kick from a_i to a_j with force taken at a_r is
 *     (G_j - G_i)/(1.5 Omega_m0 D(a_r)).
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>

/* physical constants (SI, CODATA 2018) */
#define SIGMA_SB 5.670374419e-8
#define C_LIGHT  299792458.0
#define G_NEWTON 6.67430e-11
#define MPC_M    3.0856775814913673e22
#define KB_EV    8.617333262e-5

static double F_integrand(double x, void *ctx)
{
    double y = *(double *)ctx;
    return x * x * sqrt(x * x + y * y) / (1.0 + exp(x));
}

static double dF_integrand(double x, void *ctx)
{
    double y = *(double *)ctx;
    double r = sqrt(x * x + y * y);
    return r > 0 ? x * x * y / r / (1.0 + exp(x)) : 0.0;
}

/* F(y) = int_0^inf x^2 sqrt(x^2+y^2) / (1 + e^x) dx; the tail beyond x = 100
 * is below 1e-38 of the value for every y used here. */
double orc_fd_F(double y)
{
    return orc_integrate(F_integrand, &y, 0.0, 100.0, 1e-14);
}

double orc_fd_dF(double y)
{
    if (y == 0.0) return 0.0;
    return orc_integrate(dF_integrand, &y, 0.0, 100.0, 1e-14);
}

int orc_cosmo_init(orc_cosmo *c)
{
    if (c->n_nu < 0 || c->n_nu > 3 || c->h <= 0 || c->omega_m <= 0) return -1;
    double H100 = 1.0e5 / MPC_M;                                     /* s^-1 */
    double rho_crit100 = 3.0 * H100 * H100 / (8.0 * M_PI * G_NEWTON); /* kg m^-3 */
    double rho_g = 4.0 * SIGMA_SB * pow(c->T_cmb, 4) / (C_LIGHT * C_LIGHT * C_LIGHT);
    c->omega_g = rho_g / rho_crit100 / (c->h * c->h);
    c->gamma_nu = cbrt(4.0 / 11.0) * pow(c->N_eff / 3.0, 0.25);
    c->kT_nu = KB_EV * c->T_cmb * c->gamma_nu;
    double Mnu = 0;
    for (int j = 0; j < c->n_nu; j++) Mnu += c->m_nu[j];
    c->omega_nu0 = Mnu / (93.14 * c->h * c->h);
    c->omega_c = c->omega_m - c->omega_nu0;
    c->omega_L = 0.0;
    c->omega_L = 1.0 - c->omega_g - c->omega_c - orc_omega_nu_E2(c, 1.0);
    c->a_ini = 1.0 / 160.0;
    return 0;
}

/* Neutrino term of E^2 and its derivative with respect to ln a.  The F
 * integrals are evaluated once per distinct mass (degenerate masses repeat). */
static void nu_terms(const orc_cosmo *c, double a, double *e2nu, double *de2nu)
{
    double pref = 15.0 / pow(M_PI, 4) * pow(c->gamma_nu, 4) * c->omega_g / pow(a, 4);
    double s = 0, ds = 0, F = 0, dF = 0;
    for (int j = 0; j < c->n_nu; j++) {
        double y = c->m_nu[j] * a / c->kT_nu;
        if (j == 0 || c->m_nu[j] != c->m_nu[j - 1]) {
            F = orc_fd_F(y);
            dF = de2nu ? orc_fd_dF(y) : 0.0;
        }
        s += F;
        ds += -4.0 * F + y * dF;
    }
    *e2nu = pref * s;
    if (de2nu) *de2nu = pref * ds;
}

double orc_omega_nu_E2(const orc_cosmo *c, double a)
{
    double e2nu;
    nu_terms(c, a, &e2nu, NULL);
    return e2nu;
}

static void background(const orc_cosmo *c, double a, double *E2, double *dE2)
{
    double e2nu, de2nu;
    nu_terms(c, a, &e2nu, dE2 ? &de2nu : NULL);
    *E2 = c->omega_g / pow(a, 4) + c->omega_c / pow(a, 3) + e2nu + c->omega_L;
    if (dE2) *dE2 = -4.0 * c->omega_g / pow(a, 4) - 3.0 * c->omega_c / pow(a, 3) + de2nu;
}

double orc_E(const orc_cosmo *c, double a)
{
    double E2;
    background(c, a, &E2, NULL);
    return sqrt(E2);
}

double orc_dlnE_dlna(const orc_cosmo *c, double a)
{
    double E2, dE2;
    background(c, a, &E2, &dE2);
    return dE2 / (2.0 * E2);
}

/* Right-hand side in x = ln a for y = (D, dD/dlna). */
static void growth_rhs(const orc_cosmo *c, double x, const double *y, double *dy)
{
    double a = exp(x);
    double E2, dE2;
    background(c, a, &E2, &dE2);
    double om_a = c->omega_m / (a * a * a) / E2;
    dy[0] = y[1];
    dy[1] = -(2.0 + dE2 / (2.0 * E2)) * y[1] + 1.5 * om_a * y[0];
}

static const double *cmp_a;
static int cmp_by_a(const void *p, const void *q)
{
    double u = cmp_a[*(const int *)p], v = cmp_a[*(const int *)q];
    return (u > v) - (u < v);
}

/* Integrate the growth ODE with classical RK4 from a_ini, landing exactly on
 * every requested a (steps no longer than dlna_max in ln a).  Returns D(a) and
 * G(a) = a^2 E(a) dD/dlna. */
int orc_growth(const orc_cosmo *c, int n, const double *a, double *D, double *G, double dlna_max)
{
    int *idx = malloc(sizeof(int) * n);
    for (int i = 0; i < n; i++) {
        idx[i] = i;
        if (!(a[i] >= c->a_ini)) { free(idx); return -1; }
    }
    cmp_a = a;
    qsort(idx, n, sizeof(int), cmp_by_a);
    double x = log(c->a_ini);
    double y[2] = {c->a_ini, c->a_ini};
    for (int t = 0; t < n; t++) {
        int i = idx[t];
        double xt = log(a[i]);
        while (x < xt) {
            double h = xt - x;
            if (h > dlna_max) h = dlna_max;
            double k1[2], k2[2], k3[2], k4[2], yt[2];
            growth_rhs(c, x, y, k1);
            yt[0] = y[0] + 0.5 * h * k1[0]; yt[1] = y[1] + 0.5 * h * k1[1];
            growth_rhs(c, x + 0.5 * h, yt, k2);
            yt[0] = y[0] + 0.5 * h * k2[0]; yt[1] = y[1] + 0.5 * h * k2[1];
            growth_rhs(c, x + 0.5 * h, yt, k3);
            yt[0] = y[0] + h * k3[0]; yt[1] = y[1] + h * k3[1];
            growth_rhs(c, x + h, yt, k4);
            y[0] += h / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]);
            y[1] += h / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]);
            x = (xt - x <= dlna_max) ? xt : x + h;
        }
        D[i] = y[0];
        double E = orc_E(c, a[i]);
        G[i] = a[i] * a[i] * E * y[1];
    }
    free(idx);
    return 0;
}

/* FastPM factors for a list of KDK calls: kick from a_k0 to a_k1 with the
 * force taken at a_force, drift from a_force to a_d1 with the momentum taken
 * at a_k1. */
int orc_kdk_factors(const orc_cosmo *c, int n, const double *a_force, const double *a_k0,
                    const double *a_k1, const double *a_d1, double *kick, double *drift)
{
    int m = 4 * n;
    double *a = malloc(sizeof(double) * m), *D = malloc(sizeof(double) * m), *G = malloc(sizeof(double) * m);
    for (int i = 0; i < n; i++) {
        a[4 * i + 0] = a_force[i];
        a[4 * i + 1] = a_k0[i];
        a[4 * i + 2] = a_k1[i];
        a[4 * i + 3] = a_d1[i];
    }
    int rc = orc_growth(c, m, a, D, G, 1e-3);
    if (rc == 0) {
        for (int i = 0; i < n; i++) {
            double Df = D[4 * i], Gk0 = G[4 * i + 1], Gk1 = G[4 * i + 2], Dd1 = D[4 * i + 3];
            kick[i] = (Gk1 - Gk0) / (1.5 * c->omega_m * Df);
            drift[i] = (Dd1 - Df) / Gk1;
        }
    }
    free(a); free(D); free(G);
    return rc;
}
