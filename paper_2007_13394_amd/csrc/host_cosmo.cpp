// Host-side numerics of libpm (FP64): background expansion with the exact
// Fermi-Dirac neutrino density, linear growth, FastPM factors, quasi-random
// Fermi-Dirac shells and particle masses.
//
//   * Omega_nu0 = M_nu / (93.14 h^2 eV) (Introduction); CDM takes the rest of
//     the configured Omega_m; flat closure with the exact neutrino density today.
//   * E^2(a) = Omega_g a^-4 + Omega_c0 a^-3 + Omega_nu(a) E^2 + Omega_L, with
//     Omega_nu(a) E^2 = 15/pi^4 Gamma_nu^4 Omega_g a^-4 sum_j F(m_j a / k T_nu0),
//     F(y) = int x^2 sqrt(x^2 + y^2) / (1 + e^x) dx          (Sec. 2.3, "Hubble" eq.)
//   * D'' + (2 + dlnE/dlna) D' = 1.5 Omega_m a^-3 / E^2 D in ln a, with
//     D = D' = a_ini at z = 159                               (Sec. 2.3, "growthDE" eq.)
//     The matter-only source of the "Om_pois" equation is a density in units
//     of today's critical density, hence the division by E^2.
//   * Shell edges with equal area of q f~(q), speeds sqrt(<q^4>/<q^2>) and
//     mass fractions over each shell, f~ = sum_j alpha_j^4 f(alpha_j q)
//                                                 (Sec. 2.1, "q_shell", "m_shell",
//                                                  "N_shell", "FD_deg" eqs.)
// F(y) is tabulated once on a logarithmic grid and interpolated with cubic
// Hermite polynomials; the growth ODE is integrated once with RK4 on a uniform
// ln a grid and D, dD/dlna are Hermite-interpolated from it.
#include <math.h>

#include <algorithm>
#include <functional>

#include "pm_internal.h"

namespace pm {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kZeta3 = 1.2020569031595942854;
constexpr double kZeta5 = 1.0369277551433699263;
constexpr double kKb = 8.617333262e-5;         // eV / K
constexpr double kHbarC = 1.973269804e-7;      // eV m
constexpr double kEv = 1.602176634e-19;        // J
constexpr double kC = 299792458.0;             // m / s
constexpr double kG = 6.67430e-11;             // m^3 kg^-1 s^-2
constexpr double kMpc = 3.0856775814913673e22; // m

// Composite Simpson over [a, b] with n (even) intervals.
double simpson(const std::function<double(double)> &f, double a, double b, int n)
{
    const double h = (b - a) / n;
    double s = f(a) + f(b);
    for (int i = 1; i < n; i++) s += f(a + i * h) * ((i & 1) ? 4.0 : 2.0);
    return s * h / 3.0;
}

double asimp_rec(const std::function<double(double)> &f, double a, double b, double fa, double fm, double fb,
                 double whole, double eps, int depth)
{
    const double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    const double flm = f(lm), frm = f(rm);
    const double left = (m - a) / 6.0 * (fa + 4 * flm + fm), right = (b - m) / 6.0 * (fm + 4 * frm + fb);
    const double diff = left + right - whole;
    if (depth <= 0 || fabs(diff) <= 15.0 * eps) return left + right + diff / 15.0;
    return asimp_rec(f, a, m, fa, flm, fm, left, 0.5 * eps, depth - 1) +
           asimp_rec(f, m, b, fm, frm, fb, right, 0.5 * eps, depth - 1);
}

// Adaptive Simpson to a relative tolerance `rel` of the integral (the scale
// comes from a 64-panel composite estimate), at most 2^30 subdivisions deep.
double asimpson(const std::function<double(double)> &f, double a, double b, double rel)
{
    if (b <= a) return 0.0;
    const double scale = fabs(simpson(f, a, b, 64));
    const double eps = rel * scale + 1e-300;
    const double fa = f(a), fb = f(b), fm = f(0.5 * (a + b));
    const double whole = (b - a) / 6.0 * (fa + 4 * fm + fb);
    return asimp_rec(f, a, b, fa, fm, fb, whole, eps, 30);
}

struct FTable {
    double l0 = 0, dl = 0;
    std::vector<double> F, dF;  // F(y), y dF/dy on the grid
    double F0 = 0;
};

FTable &ftable()
{
    static FTable t;
    if (t.F.empty()) {
        const int n = 800;
        t.l0 = log(1e-3);
        t.dl = (log(1e5) - t.l0) / (n - 1);
        t.F.resize(n);
        t.dF.resize(n);
        for (int i = 0; i < n; i++) {
            const double y = exp(t.l0 + i * t.dl);
            t.F[i] = simpson([y](double x) { return x * x * sqrt(x * x + y * y) / (1.0 + exp(x)); }, 0.0, 60.0, 12000);
            t.dF[i] = y * simpson([y](double x) { return x * x * y / sqrt(x * x + y * y) / (1.0 + exp(x)); }, 1e-300,
                                  60.0, 12000);
        }
        t.F0 = 7.0 * pow(kPi, 4) / 120.0;
    }
    return t;
}

// F(y) and dF/dy.
void fd_F(double y, double *F, double *dF)
{
    const FTable &t = ftable();
    if (y < 1e-3) {
        *F = t.F0 + y * y * kPi * kPi / 24.0;
        *dF = y * kPi * kPi / 12.0;
        return;
    }
    if (y > 1e5) {
        *F = 1.5 * kZeta3 * y + 11.25 * kZeta5 / y;
        *dF = 1.5 * kZeta3 - 11.25 * kZeta5 / (y * y);
        return;
    }
    const double l = log(y);
    double u = (l - t.l0) / t.dl;
    int i = (int)u;
    if (i >= (int)t.F.size() - 1) i = (int)t.F.size() - 2;
    const double s = u - i, h = t.dl;
    const double h00 = 2 * s * s * s - 3 * s * s + 1, h10 = s * s * s - 2 * s * s + s;
    const double h01 = -2 * s * s * s + 3 * s * s, h11 = s * s * s - s * s;
    *F = h00 * t.F[i] + h10 * h * t.dF[i] + h01 * t.F[i + 1] + h11 * h * t.dF[i + 1];
    // derivative of the Hermite cubic with respect to ln y, divided by y
    const double d00 = 6 * s * s - 6 * s, d10 = 3 * s * s - 4 * s + 1, d01 = -6 * s * s + 6 * s, d11 = 3 * s * s - 2 * s;
    const double dl = (d00 * t.F[i] + d10 * h * t.dF[i] + d01 * t.F[i + 1] + d11 * h * t.dF[i + 1]) / h;
    *dF = dl / y;
}

void background(const Ctx &c, double a, double *E2, double *dE2)
{
    const pm_config &g = c.cfg;
    const double pref = 15.0 / pow(kPi, 4) * pow(g.N_eff / 3.0, 1.0) * pow(4.0 / 11.0, 4.0 / 3.0) * c.omega_g / pow(a, 4);
    double s = 0, ds = 0;
    for (int j = 0; j < g.n_nu; j++) {
        const double y = g.m_nu[j] * a / c.kT_nu;
        double F, dF;
        fd_F(y, &F, &dF);
        s += F;
        ds += -4.0 * F + y * dF;
    }
    *E2 = c.omega_g / pow(a, 4) + c.omega_c / pow(a, 3) + pref * s + c.omega_L;
    *dE2 = -4.0 * c.omega_g / pow(a, 4) - 3.0 * c.omega_c / pow(a, 3) + pref * ds;
}

void rhs(const Ctx &c, double x, const double y[2], double dy[2])
{
    const double a = exp(x);
    double E2, dE2;
    background(c, a, &E2, &dE2);
    dy[0] = y[1];
    dy[1] = -(2.0 + 0.5 * dE2 / E2) * y[1] + 1.5 * c.cfg.omega_m / (a * a * a) / E2 * y[0];
}

double ftilde(const std::vector<double> &alpha, double q)
{
    double s = 0;
    for (double aj : alpha) s += aj * aj * aj * aj / (exp(aj * q) + 1.0);
    return s;
}

}  // namespace

double E_of_a(const Ctx &c, double a)
{
    double E2, dE2;
    background(c, a, &E2, &dE2);
    return sqrt(E2);
}

static void growth_interp(const Ctx &c, double a, double *D, double *Dp)
{
    const double x = log(a);
    double u = (x - c.gx0) / c.gdx;
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i >= (int)c.gD.size() - 1) i = (int)c.gD.size() - 2;
    const double s = u - i, h = c.gdx;
    const double h00 = 2 * s * s * s - 3 * s * s + 1, h10 = s * s * s - 2 * s * s + s;
    const double h01 = -2 * s * s * s + 3 * s * s, h11 = s * s * s - s * s;
    *D = h00 * c.gD[i] + h10 * h * c.gDp[i] + h01 * c.gD[i + 1] + h11 * h * c.gDp[i + 1];
    *Dp = h00 * c.gDp[i] + h10 * h * c.gDpp[i] + h01 * c.gDp[i + 1] + h11 * h * c.gDpp[i + 1];
}

double growth_D(const Ctx &c, double a)
{
    double D, Dp;
    growth_interp(c, a, &D, &Dp);
    return D;
}

double growth_G(const Ctx &c, double a)
{
    double D, Dp;
    growth_interp(c, a, &D, &Dp);
    return a * a * E_of_a(c, a) * Dp;
}

double pk_amplitude(const Ctx &c)
{
    const pm_config &g = c.cfg;
    const double omh = g.omega_m * g.h;
    auto integrand = [&](double lnk) {
        const double k = exp(lnk), q = k / omh, x = 8.0 * k;
        const double T = log(1.0 + 2.34 * q) / (2.34 * q) *
                         pow(1.0 + 3.89 * q + pow(16.1 * q, 2) + pow(5.46 * q, 3) + pow(6.71 * q, 4), -0.25);
        const double W = x < 1e-3 ? 1.0 - x * x / 10.0 : 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
        return k * k * k * pow(k, g.n_s) * T * T * W * W / (2.0 * kPi * kPi);
    };
    const double s2 = simpson(integrand, log(1e-6), log(1e3), 400000);
    return g.sigma8 * g.sigma8 / s2;
}

void cosmo_setup(Ctx &c)
{
    const pm_config &g = c.cfg;
    // photons: rho_g c^2 = pi^2/15 (k T)^4 / (hbar c)^3
    const double kT = kKb * g.T_cmb;
    const double rho_g = kPi * kPi / 15.0 * pow(kT, 4) / pow(kHbarC, 3) * kEv / (kC * kC);   // kg / m^3
    const double H100 = 1.0e5 / kMpc;
    const double rho_c = 3.0 * H100 * H100 / (8.0 * kPi * kG);
    c.omega_g = rho_g / rho_c / (g.h * g.h);
    c.kT_nu = kT * cbrt(4.0 / 11.0) * pow(g.N_eff / 3.0, 0.25);
    double Mnu = 0, m1 = 0;
    for (int j = 0; j < g.n_nu; j++) {
        Mnu += g.m_nu[j];
        m1 = std::max(m1, g.m_nu[j]);
    }
    c.m1 = m1;
    c.omega_nu0 = Mnu / (93.14 * g.h * g.h);
    c.omega_c = g.omega_m - c.omega_nu0;
    c.omega_L = 0.0;
    {
        double E2, dE2;
        background(c, 1.0, &E2, &dE2);
        c.omega_L = 1.0 - E2;   // E2 here excludes Lambda
    }
    // growth table
    c.gx0 = log(1.0 / 160.0);
    c.gdx = 1e-3;
    const int n = (int)ceil((log(2.0) - c.gx0) / c.gdx) + 1;
    c.gD.resize(n);
    c.gDp.resize(n);
    c.gDpp.resize(n);
    double y[2] = {1.0 / 160.0, 1.0 / 160.0};
    for (int i = 0; i < n; i++) {
        const double x = c.gx0 + i * c.gdx;
        double dy[2];
        rhs(c, x, y, dy);
        c.gD[i] = y[0];
        c.gDp[i] = y[1];
        c.gDpp[i] = dy[1];
        if (i == n - 1) break;
        const double h = c.gdx;
        double k1[2], k2[2], k3[2], k4[2], t[2];
        k1[0] = dy[0];
        k1[1] = dy[1];
        t[0] = y[0] + 0.5 * h * k1[0];
        t[1] = y[1] + 0.5 * h * k1[1];
        rhs(c, x + 0.5 * h, t, k2);
        t[0] = y[0] + 0.5 * h * k2[0];
        t[1] = y[1] + 0.5 * h * k2[1];
        rhs(c, x + 0.5 * h, t, k3);
        t[0] = y[0] + h * k3[0];
        t[1] = y[1] + h * k3[1];
        rhs(c, x + h, t, k4);
        y[0] += h / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0]);
        y[1] += h / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1]);
    }

    // neutrino shells
    c.edges.clear();
    c.q_shell.clear();
    c.m_shell.clear();
    c.dirs.clear();
    if (g.n_sites > 0 && g.n_nu > 0 && m1 > 0) {
        std::vector<double> alpha;
        double amin = 1.0;
        for (int j = 0; j < g.n_nu; j++) {
            alpha.push_back(g.m_nu[j] / m1);
            amin = std::min(amin, alpha.back());
        }
        const double qmax = 30.0 / amin;
        auto gq = [&](double q) { return q * ftilde(alpha, q); };
        // cumulative of g on a fine grid, then bisection inside the bracketing cell
        const int ng = 4096;
        const double hq = qmax / ng;
        std::vector<double> cum(ng + 1, 0.0);
        for (int i = 0; i < ng; i++) cum[i + 1] = cum[i] + simpson(gq, i * hq, (i + 1) * hq, 16);
        const double gtot = cum[ng];
        const int ns = g.n_shell;
        c.edges.assign(ns + 1, 0.0);
        c.edges[ns] = qmax;
        for (int s = 1; s < ns; s++) {
            const double target = gtot * s / ns;
            const int i = (int)(std::upper_bound(cum.begin(), cum.end(), target) - cum.begin()) - 1;
            double lo = i * hq, hi = (i + 1) * hq;
            for (int it = 0; it < 100; it++) {
                const double mid = 0.5 * (lo + hi);
                const double v = cum[i] + asimpson(gq, i * hq, mid, 1e-14);
                (v < target ? lo : hi) = mid;
            }
            c.edges[s] = 0.5 * (lo + hi);
        }
        double ntot = 0;
        std::vector<double> m2(ns), m4(ns);
        for (int s = 0; s < ns; s++) {
            auto f2 = [&](double q) { return q * q * ftilde(alpha, q); };
            auto f4 = [&](double q) { return q * q * q * q * ftilde(alpha, q); };
            m2[s] = asimpson(f2, c.edges[s], c.edges[s + 1], 1e-14);
            m4[s] = asimpson(f4, c.edges[s], c.edges[s + 1], 1e-14);
            ntot += m2[s];
        }
        for (int s = 0; s < ns; s++) {
            c.q_shell.push_back(sqrt(m4[s] / m2[s]));
            c.m_shell.push_back(m2[s] / ntot);
        }
        // pseudo-random sampling: cumulative number distribution C(q) on the same grid
        c.q_cdf.clear();
        if (g.flags & PM_FLAG_NU_PSEUDO) {
            auto f2 = [&](double q) { return q * q * ftilde(alpha, q); };
            c.q_cdf.assign(ng + 1, 0.0);
            for (int i = 0; i < ng; i++) c.q_cdf[i + 1] = c.q_cdf[i] + simpson(f2, i * hq, (i + 1) * hq, 16);
            const double tot = c.q_cdf[ng];
            for (double &v : c.q_cdf) v /= tot;
            c.q_cdf_h = hq;
        }
        // Fibonacci sphere: latitude asin(2i/(2 n_fib + 1)), longitude 2 pi i / golden ratio
        const double phi = 0.5 * (1.0 + sqrt(5.0));
        for (int i = -g.n_fib; i <= g.n_fib; i++) {
            const double lat = asin(2.0 * i / (2.0 * g.n_fib + 1.0)), lon = 2.0 * kPi * i / phi;
            c.dirs.push_back((float)(cos(lat) * cos(lon)));
            c.dirs.push_back((float)(cos(lat) * sin(lon)));
            c.dirs.push_back((float)sin(lat));
        }
    }

    // segments and masses (mean of one mass unit per cell)
    const double M = (double)g.n_mesh * g.n_mesh * g.n_mesh;
    c.seg_off.assign(1, 0);
    c.seg_mass.clear();
    c.seg_q.clear();
    c.seg_off.push_back(c.nc);
    c.seg_mass.push_back(c.omega_c / g.omega_m * M / (double)c.nc);
    if (c.nn > 0) {
        const int64_t nsites = (int64_t)g.n_sites * g.n_sites * g.n_sites;
        const int64_t per = nsites * (2 * g.n_fib + 1);
        for (int s = 0; s < g.n_shell; s++) {
            c.seg_off.push_back(c.nc + (s + 1) * per);
            c.seg_mass.push_back(c.omega_nu0 / g.omega_m * (M / (double)nsites) * c.m_shell[s] /
                                 (2.0 * g.n_fib + 1.0));
        }
    }
    c.nseg = (int)c.seg_mass.size();
    for (double m : c.seg_mass) c.seg_q.push_back(llrint(ldexp(m, g.shift)));
}

}  // namespace pm
