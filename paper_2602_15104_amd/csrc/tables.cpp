// Host-side background, recombination and thermodynamics tables (CPU).
//
// Shared input of the device kernels for one cosmology, following arXiv
// 2602.15104:
//   * derived parameters and species densities: App. A.2 (derived
//     parameters), Sec. 2.4 (eq. Neffdef, neutrino temperatures), App. C;
//     flatness fixes Lambda so that Hc(a = 1) = H0;
//   * free-electron fraction: helium in Saha equilibrium (App. B.1, both
//     stages), hydrogen by Saha (eq. SahaH) while x_p >= 0.99 and then by the
//     Peebles three-level atom (the TLA App. B.1 uses at late times) with the
//     Pequignot-Petitjean-Boisson case-B rate (1.14 fudge of Seager et al.
//     1999); matter temperature quasi-static above z = 700, by its ODE below
//     (App. B.1); tanh reionisation patched on (App. B.2) with z_reion from
//     tau_reio (App. A.2, eq. tau_reion);
//   * Thomson rate a n_e sigma_T, optical depth kappa, baryon sound speed
//     (App. B.4, App. C baryons), conformal time;
//   * start time per mode from R_tc and R_large (App. A.2);
//   * output times and line-of-sight trapezoid weights in ln a (App. B.6).
// Discretisation: uniform ln a grid of n_tab intervals from
// ln(min a_i) - 1/2 to 0; classical RK4 per interval for the recombination
// ODEs; Simpson per interval for conformal time; trapezoid for kappa;
// natural cubic splines of ln(1/tau_c), kappa, ln c_s^2, ln tau, stored as
// per-interval cubic polynomials for the device.
#include "cmbhip_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

namespace cmbhip {

// CODATA 2018 / AME 2016
static const double kC = 299792458.0;               // m/s
static const double kG = 6.67430e-11;               // m^3 kg^-1 s^-2
static const double kHbarcEvCm = 1.973269804e-5;    // eV cm
static const double kEvJ = 1.602176634e-19;         // J
static const double kMpcM = 3.0856775814913673e22;  // m
static const double kSigmaT = 6.6524587321e-25;     // cm^2
static const double kMe = 0.51099895000e6;          // eV
static const double kAmu = 931.49410242e6;          // eV
static const double kMH = 1.00782503223 * kAmu;     // eV, hydrogen atom
static const double kMHe = 4.00260325413 * kAmu;    // eV, helium-4 atom
static const double kEH = 13.598434599702;          // eV
static const double kEHe1 = 24.587387;              // eV
static const double kEHe2 = 54.417760;              // eV
static const double kL2s = 8.2245809;               // 1/s
static const double kPi = 3.14159265358979323846;

static inline double cube(double x) { return x * x * x; }

struct Model {
    double H0 = 0, rt_g0 = 0, rt_ur0 = 0, rt_c0 = 0, rt_b0 = 0, rt_L = 0, rt_m0 = 0, rt_rad_early = 0;
    double pref_n = 0, m_over_T = 0, N_n = 0;
    std::vector<double> q, W;
    double T0 = 0, Y = 0, fHe = 0, nH0 = 0, dk_pref = 0, R_nu = 0, N_ml = 0, Neff = 0;
    cmb_cosmo c{};

    void ncdm(double a, double &rho, double &p) const {
        rho = p = 0.0;
        if (N_n <= 0) return;
        double x = a * m_over_T, sr = 0, sp = 0;
        for (size_t i = 0; i < q.size(); ++i) {
            double e = std::sqrt(q[i] * q[i] + x * x);
            sr += W[i] * e;
            sp += W[i] * q[i] * q[i] / e;
        }
        double a4 = a * a * a * a;
        rho = pref_n * sr / a4;
        p = pref_n * sp / (3.0 * a4);
    }
    void tot(double a, double &rho, double &p) const {
        double rn, pn;
        ncdm(a, rn, pn);
        double a3 = a * a * a;
        double rr = (rt_g0 + rt_ur0) / (a3 * a);
        rho = rr + rt_m0 / a3 + rt_L + rn;
        p = rr / 3.0 - rt_L + pn;
    }
    double Hc(double a) const {
        double r, p;
        tot(a, r, p);
        return a * std::sqrt(r);
    }
    double Hcp(double a) const {
        double r, p;
        tot(a, r, p);
        return a * std::sqrt(r) * (1.0 - 1.5 * (r + p) / r);
    }
    double Hs(double a) const { return Hc(a) / a * kC / kMpcM; }
};

static double inv_hbarc3() { return 1.0 / cube(kHbarcEvCm); }

// ---------------------------------------------------------------------------
// n-node Gauss rule for  int_0^inf dq q^2/(e^q+1) g(q)  (the massive-neutrino
// momentum integrals of App. B.3, eq. mnu_sum, with more nodes than the paper's
// rules).  The weight is discretised by composite Gauss-Legendre on [0, 120]
// (beyond, q^(2n+2) e^-q is below 1e-17 of its peak for n <= 16); the
// recurrence coefficients of its monic orthogonal polynomials come from the
// discretised Stieltjes procedure (Gautschi 1982), and nodes and weights from
// the eigen-decomposition of the Jacobi matrix (Golub & Welsch 1969) by the
// implicit QL method with Wilkinson shifts.  All in long double.
// ---------------------------------------------------------------------------
static void gauss_legendre(int m, std::vector<long double> &x, std::vector<long double> &w) {
    x.assign(m, 0.0L);
    w.assign(m, 0.0L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < m; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (m + 0.5L)), dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;  // P_0, P_1
            for (int j = 2; j <= m; ++j) {
                long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0L);  // P_m'
            long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

void gauss_legendre_nodes(int m, std::vector<double> &x, std::vector<double> &w) {
    std::vector<long double> xl, wl;
    gauss_legendre(m, xl, wl);
    x.assign(xl.begin(), xl.end());
    w.assign(wl.begin(), wl.end());
}

// eigenvalues d and first eigenvector components z0 of the symmetric
// tridiagonal matrix (d on the diagonal, e[i] between i and i+1)
static bool tridiag_eigen(std::vector<long double> &d, std::vector<long double> e, std::vector<long double> &z0) {
    const int n = (int)d.size();
    std::vector<long double> Z((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0L;
    e.resize(n, 0.0L);
    e[n - 1] = 0.0L;
    const long double eps = std::numeric_limits<long double>::epsilon();
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            int mm = l;
            for (; mm < n - 1; ++mm) {
                long double dd = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
                if (std::fabs(e[mm]) <= eps * dd) break;
            }
            if (mm == l) break;
            if (iter > 200) return false;
            // Wilkinson shift from the leading 2x2 block, then a chase of
            // plane rotations from the bottom of the unreduced block upwards
            long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            long double r = std::hypot(g, 1.0L);
            g = d[mm] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            long double s = 1.0L, c = 1.0L, p = 0.0L;
            int i = mm - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                long double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {
                    d[i + 1] -= p;
                    e[mm] = 0.0L;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int kq = 0; kq < n; ++kq) {
                    long double t = Z[(size_t)kq * n + i + 1];
                    Z[(size_t)kq * n + i + 1] = s * Z[(size_t)kq * n + i] + c * t;
                    Z[(size_t)kq * n + i] = c * Z[(size_t)kq * n + i] - s * t;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0L;
        }
    }
    z0.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) z0[i] = Z[i];  // first row of Z: first components of the eigenvectors
    return true;
}

static bool fermi_dirac_rule(int n, std::vector<double> &q, std::vector<double> &W) {
    // discretised weight
    std::vector<long double> gx, gw, x, w;
    gauss_legendre(24, gx, gw);
    const int panels = 120;
    for (int pnl = 0; pnl < panels; ++pnl)
        for (int i = 0; i < 24; ++i) {
            long double t = pnl + 0.5L * (gx[i] + 1.0L);
            x.push_back(t);
            w.push_back(0.5L * gw[i] * t * t / (std::exp(t) + 1.0L));
        }
    // Stieltjes: p_{j+1} = (x - alpha_j) p_j - beta_j p_{j-1}
    const size_t M = x.size();
    std::vector<long double> pm(M, 0.0L), pc(M, 1.0L), alpha(n), beta(n);
    long double norm_prev = 1.0L;
    for (int j = 0; j < n; ++j) {
        long double nrm = 0.0L, xn = 0.0L;
        for (size_t k = 0; k < M; ++k) {
            long double v = w[k] * pc[k] * pc[k];
            nrm += v;
            xn += v * x[k];
        }
        alpha[j] = xn / nrm;
        beta[j] = (j == 0) ? nrm : nrm / norm_prev;
        norm_prev = nrm;
        for (size_t k = 0; k < M; ++k) {
            long double pn = (x[k] - alpha[j]) * pc[k] - (j == 0 ? 0.0L : beta[j]) * pm[k];
            pm[k] = pc[k];
            pc[k] = pn;
        }
    }
    std::vector<long double> d(alpha), e(n, 0.0L), z0;
    for (int j = 0; j + 1 < n; ++j) e[j] = std::sqrt(beta[j + 1]);
    if (!tridiag_eigen(d, e, z0)) return false;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    q.resize(n);
    W.resize(n);
    for (int i = 0; i < n; ++i) {
        q[i] = (double)d[order[i]];
        W[i] = (double)(beta[0] * z0[order[i]] * z0[order[i]]);
    }
    return true;
}

// root of x^2 + B x - C = 0 with C >= 0, stable form
static double pos_root(double B, double C) { return 2.0 * C / (B + std::sqrt(B * B + 4.0 * C)); }

static double saha(double mu, double T, double E, double nH) {
    return std::pow(mu * T / (2.0 * kPi), 1.5) * inv_hbarc3() * std::exp(-E / T) / nH;
}

static const double kMuH = kMe * (kMH - kMe) / kMH;
static const double kMuHe2 = kMe * (kMHe - 2 * kMe) / (kMHe - kMe);
static const double kMuHe1 = kMe * (kMHe - kMe) / kMHe;

static double he_electrons(const Model &m, double a) {
    double T = m.T0 / a, nH = m.nH0 / cube(a), f = m.fHe;
    double s2 = saha(kMuHe2, T, kEHe2, nH);
    double x3 = pos_root(1.0 + f + s2, s2 * f);  // x(1+f+x)/(f-x) = s2
    if (x3 >= 1e-9) return f + x3;
    double s1 = 4.0 * saha(kMuHe1, T, kEHe1, nH);
    return pos_root(1.0 + s1, s1 * f);  // x(1+x)/(f-x) = 4 s
}

static double h_saha(const Model &m, double a) {
    double s = saha(kMuH, m.T0 / a, kEH, m.nH0 / cube(a));
    return s > 0 ? 2.0 / (1.0 + std::sqrt(1.0 + 4.0 / s)) : 0.0;
}

static double alphaB(double T) {  // cm^3/s, T in eV
    double t = T / 8.617333262e-5 / 1.0e4;
    return 1.14e-13 * 4.309 * std::pow(t, -0.6166) / (1.0 + 0.6703 * std::pow(t, 0.5300));
}

static double gamma_c(const Model &m, double a, double xe) {
    double T = m.T0 / a;
    double rho_g = (kPi * kPi / 15.0) * T * T * T * T * inv_hbarc3();
    return 8.0 * kSigmaT * rho_g * (kC * 100.0) / (3.0 * kMe) * xe / (1.0 + m.fHe + xe);
}

static double tm_qs(const Model &m, double a, double xe) { return m.T0 / a * (1.0 - m.Hs(a) / gamma_c(m, a, xe)); }

static double dxp_dlna(const Model &m, double a, double xp, double Tm) {
    double Tr = m.T0 / a, nH = m.nH0 / cube(a), H = m.Hs(a);
    double xe = xp + he_electrons(m, a);
    double beta = alphaB(Tr) * std::pow(kMe * Tr / (2.0 * kPi), 1.5) * inv_hbarc3() * std::exp(-0.25 * kEH / Tr);
    double lam = 2.0 * kPi * kHbarcEvCm / (0.75 * kEH);
    double K = cube(lam) / (8.0 * kPi * H);
    double n1s = nH * (1.0 - xp);
    double C = (1.0 + K * kL2s * n1s) / (1.0 + K * (kL2s + beta) * n1s);
    return -C * (alphaB(Tm) * nH * xe * xp - beta * (1.0 - xp) * std::exp(-0.75 * kEH / Tr)) / H;
}

static double dtm_dlna(const Model &m, double a, double xp, double Tm) {
    double xe = xp + he_electrons(m, a), H = m.Hs(a);
    return (-2.0 * H * Tm + gamma_c(m, a, xe) * (m.T0 / a - Tm)) / H;
}

struct Reion {
    double yre, dy, beta, zHe, dzHe, fHe;
    Reion(const Model &m, double zre) {
        beta = m.c.exp_reio;
        yre = std::pow(1.0 + zre, beta);
        dy = beta * m.c.Delta_z_reio * std::pow(1.0 + zre, beta - 1.0);
        zHe = m.c.z_reio_He;
        dzHe = m.c.Delta_z_reio_He;
        fHe = m.fHe;
    }
    double fracH(double z) const { return 0.5 * (1.0 + std::tanh((yre - std::pow(1.0 + z, beta)) / dy)); }
    double fracHe(double z) const { return 0.5 * (1.0 + std::tanh((zHe - z) / dzHe)); }
    double blend(double z, double xrec) const { return xrec + ((1.0 + fHe) - xrec) * fracH(z) + fHe * fracHe(z); }
    double only(double z) const { return (1.0 + fHe) * fracH(z) + fHe * fracHe(z); }
    double zmax() const {
        return std::max(std::pow(yre + 20.0 * dy, 1.0 / beta) - 1.0, zHe + 20.0 * dzHe);
    }
};

// eq. tau_reion in redshift, Simpson's rule on 2000 intervals
static double tau_reion(const Model &m, double zre) {
    Reion R(m, zre);
    const int n = 2000;
    double zmax = R.zmax(), hz = zmax / n, acc = 0.0;
    for (int i = 0; i <= n; ++i) {
        double z = i * hz;
        double f = m.dk_pref * (1.0 + z) * R.only(z) / m.Hc(1.0 / (1.0 + z));
        double w = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        acc += w * f;
    }
    return acc * hz / 3.0;
}

// Root of f in [lo, hi] (f(lo) <= 0 < f(hi)) by bisection to the last bit.  Once
// the midpoint rounds onto an end point every further halving returns that
// same point, so the search stops there.
static double bisect(const std::function<double(double)> &f, double lo, double hi) {
    for (int it = 0; it < 100; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) return mid;
        if (f(mid) > 0.0)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Root of an increasing f with f(lo) = flo <= 0 < f(hi) = fhi, for an f that is
// expensive to evaluate: Illinois false position (the retained end's value
// halved when the same end is kept twice) while the bracket is wider than
// 1e-10 of its ends, then bisection to the last bit.
static double root_bracketed(const std::function<double(double)> &f, double lo, double hi, double flo, double fhi) {
    int keep = 0;  // -1: hi was moved last, +1: lo was moved last
    for (int it = 0; it < 60 && hi - lo > 1e-10 * (1.0 + std::fabs(lo) + std::fabs(hi)); ++it) {
        double x = (lo * fhi - hi * flo) / (fhi - flo);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        const double fx = f(x);
        if (fx > 0.0) {
            hi = x;
            fhi = fx;
            if (keep == -1) flo *= 0.5;
            keep = -1;
        } else {
            lo = x;
            flo = fx;
            if (keep == 1) fhi *= 0.5;
            keep = 1;
        }
    }
    return bisect(f, lo, hi);
}

// second derivatives of the natural cubic spline on a uniform grid (Thomas algorithm)
static void natural_spline(const std::vector<double> &f, double h, std::vector<double> &M) {
    int n = (int)f.size() - 1;
    M.assign(n + 1, 0.0);
    if (n < 2) return;
    std::vector<double> cp(n + 1), dp(n + 1);
    // rows j = 1..n-1: M_{j-1} + 4 M_j + M_{j+1} = 6 (f_{j+1} - 2 f_j + f_{j-1}) / h^2
    double inv_h2 = 6.0 / (h * h);
    for (int j = 1; j < n; ++j) {
        double d = inv_h2 * (f[j + 1] - 2.0 * f[j] + f[j - 1]);
        double b = 4.0;
        if (j > 1) {
            b -= cp[j - 1];
            d -= dp[j - 1];
        }
        cp[j] = 1.0 / b;
        dp[j] = d / b;
    }
    // cp holds 1/b'_j; convert forward sweep to the standard form
    // (upper entries are 1): x_j = dp_j - cp_j x_{j+1}
    M[n - 1] = dp[n - 1];
    for (int j = n - 2; j >= 1; --j) M[j] = dp[j] - cp[j] * M[j + 1];
}

void set_error(const std::string &msg);

static int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

int build_tables(const cmb_cosmo &cin, const cmb_prec &p, const double *k, int n_k, int n_tau, Tables &T) {
    if (n_k < 1 || n_tau < 3) return fail(CMB_E_INVALID, "n_k must be >= 1 and n_tau >= 3");
    for (int i = 0; i < n_k; ++i) {
        if (!finite_pos(k[i])) return fail(CMB_E_INVALID, "k must be finite and positive");
        if (i > 0 && !(k[i] > k[i - 1])) return fail(CMB_E_INVALID, "k must be strictly increasing");
    }
    const cmb_cosmo &c = cin;
    if (!finite_pos(c.h) || !finite_pos(c.omega_b) || !finite_pos(c.omega_cdm) || !finite_pos(c.A_s) ||
        !std::isfinite(c.n_s) || !finite_pos(c.TCMB0) || !finite_pos(c.YHe) || !(c.YHe < 1.0) ||
        !finite_pos(c.T_nu_massless) || !finite_pos(c.Delta_z_reio) || !finite_pos(c.Delta_z_reio_He) ||
        !finite_pos(c.exp_reio) || !std::isfinite(c.z_reio_He))
        return fail(CMB_E_INVALID, "cosmological parameter NaN or out of range");
    if (p.ell_gamma < 3 || p.ell_nu < 3 || (p.ell_pol != 0 && p.ell_pol < 3) || p.n_tab < 16 || p.max_steps < 1 ||
        !finite_pos(p.rtol_small) || !finite_pos(p.rtol_large) || !finite_pos(p.atol_small) ||
        !finite_pos(p.atol_large) || !finite_pos(p.R_tc) || !finite_pos(p.R_large) || !finite_pos(p.k_pivot))
        return fail(CMB_E_INVALID, "precision options out of range");
    if (std::isfinite(c.Neff) && std::isfinite(c.N_nu_massless))
        return fail(CMB_E_CONFLICT, "Neff and N_nu_massless both given");
    if (std::isfinite(c.tau_reio) && std::isfinite(c.z_reio))
        return fail(CMB_E_CONFLICT, "tau_reio and z_reio both given");
    if (!std::isfinite(c.tau_reio) && !std::isfinite(c.z_reio))
        return fail(CMB_E_INVALID, "one of tau_reio, z_reio must be given");
    const bool massive = c.N_nu_massive > 0;
    if (massive && (!(p.n_q >= 1 && p.n_q <= kMaxQ) || p.ell_ncdm < 3 || !std::isfinite(c.m_nu_massive) ||
                    c.m_nu_massive < 0 || !finite_pos(c.T_nu_massive)))
        return fail(CMB_E_INVALID, "massive neutrinos need 1 <= n_q <= 16, ell_ncdm >= 3, m >= 0 and T > 0");

    Model m;
    m.c = c;
    const double H100s = 1.0e5 / kMpcM;  // 1/s
    const double H100 = 1.0e5 / kC;      // 1/Mpc
    const double rho_crit_h2 = 3.0 * H100s * H100s * kC * kC / (8.0 * kPi * kG) / kEvJ * 1.0e-6;  // eV/cm^3
    const double rho_crit_h2_eV4 = rho_crit_h2 * cube(kHbarcEvCm);
    const double to_rt = H100 * H100 / rho_crit_h2_eV4;
    m.H0 = c.h * H100;
    m.T0 = c.TCMB0;
    double T4 = c.TCMB0 * c.TCMB0 * c.TCMB0 * c.TCMB0;
    m.rt_g0 = kPi * kPi / 15.0 * T4 * to_rt;
    m.rt_c0 = c.omega_cdm * H100 * H100;
    m.rt_b0 = c.omega_b * H100 * H100;
    m.rt_m0 = m.rt_c0 + m.rt_b0;
    const double tinst = std::cbrt(4.0 / 11.0);
    double per_ml = std::pow(c.T_nu_massless / tinst, 4);
    double per_m = std::pow(c.T_nu_massive / tinst, 4);
    m.N_n = c.N_nu_massive > 0 ? c.N_nu_massive : 0.0;
    if (std::isfinite(c.Neff)) {
        m.N_ml = (c.Neff - m.N_n * per_m) / per_ml;
        if (m.N_ml < 0) return fail(CMB_E_NEG_NMASSLESS, "Neff requires a negative number of massless neutrinos");
    } else {
        m.N_ml = std::isfinite(c.N_nu_massless) ? c.N_nu_massless : 3.0;
        if (m.N_ml < 0) return fail(CMB_E_INVALID, "N_nu_massless < 0");
    }
    m.Neff = m.N_ml * per_ml + m.N_n * per_m;
    if (massive) {
        // rho = (N / pi^2) T^4 a^-4 sum_i W_i eps_i  (two helicity states per species)
        if (!fermi_dirac_rule(p.n_q, m.q, m.W)) return fail(CMB_E_INVALID, "momentum rule did not converge");
        const double Tm = c.T_nu_massive * c.TCMB0;
        m.m_over_T = c.m_nu_massive / Tm;
        m.pref_n = m.N_n / (kPi * kPi) * Tm * Tm * Tm * Tm * to_rt;
    }
    double Tml = c.T_nu_massless * c.TCMB0;
    m.rt_ur0 = m.N_ml * 7.0 * kPi * kPi / 120.0 * Tml * Tml * Tml * Tml * to_rt;
    {
        double rn, pn;
        m.ncdm(1.0, rn, pn);
        m.rt_L = m.H0 * m.H0 - (m.rt_g0 + m.rt_ur0 + m.rt_m0 + rn);
    }
    // early-time radiation, with the massive species still relativistic
    double ncdm_rel = 0.0;
    for (size_t i = 0; i < m.q.size(); ++i) ncdm_rel += m.pref_n * m.W[i] * m.q[i];
    m.rt_rad_early = m.rt_g0 + m.rt_ur0 + ncdm_rel;
    m.R_nu = (m.rt_ur0 + ncdm_rel) / m.rt_rad_early;
    m.Y = c.YHe;
    m.fHe = c.YHe * kMH / ((1.0 - c.YHe) * kMHe);
    m.nH0 = (1.0 - c.YHe) * c.omega_b * rho_crit_h2 / kMH;
    m.dk_pref = m.nH0 * kSigmaT * kMpcM * 100.0;

    // reionisation redshift
    double zre = c.z_reio;
    if (std::isfinite(c.tau_reio)) {
        auto f = [&](double z) { return tau_reion(m, z) - c.tau_reio; };
        const double f0 = f(0.0), f50 = f(50.0);
        if (!(f0 < 0.0 && f50 > 0.0)) return fail(CMB_E_ROOT, "tau_reio not bracketed by z_reion in [0, 50]");
        zre = root_bracketed(f, 0.0, 50.0, f0, f50);
    }
    Reion R(m, zre);

    // start times
    const double lmin = std::log(1e-12);
    auto xe_early = [&](double a) { return R.blend(1.0 / a - 1.0, h_saha(m, a) + he_electrons(m, a)); };
    auto ftc = [&](double l) {
        double a = std::exp(l);
        return m.Hc(a) / (xe_early(a) * m.dk_pref / (a * a)) - p.R_tc;
    };
    double lhi = std::log(1.0 / 1601.0);
    if (!(ftc(lmin) < 0.0 && ftc(lhi) > 0.0)) return fail(CMB_E_ROOT, "R_tc start time not bracketed");
    double lna_tc = bisect(ftc, lmin, lhi);
    double lna_hmin = 0.0;
    {
        auto fh = [&](double l) { return m.Hcp(std::exp(l)); };
        if (fh(0.0) > 0.0) lna_hmin = bisect(fh, std::log(0.01), 0.0);
    }
    std::vector<double> lna_i(n_k);
    for (int i = 0; i < n_k; ++i) {
        double kk = k[i];
        auto fl = [&](double l) { return kk / m.Hc(std::exp(l)) - p.R_large; };
        if (fl(lna_hmin) <= 0.0) {
            lna_i[i] = lna_tc;
            continue;
        }
        if (fl(lmin) >= 0.0) return fail(CMB_E_ROOT, "k too large for the start-time search");
        lna_i[i] = std::min(lna_tc, bisect(fl, lmin, lna_hmin));
    }

    // grid
    const int n = p.n_tab;
    double L0 = *std::min_element(lna_i.begin(), lna_i.end()) - 0.5;
    double dl = -L0 / n;
    std::vector<double> lna(n + 1);
    for (int j = 0; j < n; ++j) lna[j] = L0 + j * dl;
    lna[n] = 0.0;

    // recombination
    std::vector<double> xrec(n + 1), Tm(n + 1), dlnT(n + 1);
    const double zsw = 700.0;
    int j = 0;
    for (; j <= n; ++j) {
        double a = std::exp(lna[j]);
        double xp = h_saha(m, a);
        if (xp < 0.99) break;
        double xe = xp + he_electrons(m, a);
        xrec[j] = xe;
        Tm[j] = tm_qs(m, a, xe);
        dlnT[j] = -1.0;
    }
    if (j > n) return fail(CMB_E_ROOT, "hydrogen never leaves Saha equilibrium");
    double xp, tm;
    {
        double a = std::exp(lna[j]);
        xp = h_saha(m, a);
        xrec[j] = xp + he_electrons(m, a);
        tm = tm_qs(m, a, xrec[j]);
        Tm[j] = tm;
        dlnT[j] = (1.0 / a - 1.0 >= zsw) ? -1.0 : dtm_dlna(m, a, xp, tm) / tm;
    }
    for (; j < n; ++j) {
        double l0 = lna[j], h = lna[j + 1] - lna[j], lm = l0 + 0.5 * h, l1 = l0 + h;
        if (1.0 / std::exp(l0) - 1.0 >= zsw) {
            auto g = [&](double l, double x) {
                double a = std::exp(l);
                return dxp_dlna(m, a, x, tm_qs(m, a, x + he_electrons(m, a)));
            };
            double k1 = g(l0, xp), k2 = g(lm, xp + 0.5 * h * k1), k3 = g(lm, xp + 0.5 * h * k2), k4 = g(l1, xp + h * k3);
            xp += h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
            double a1 = std::exp(lna[j + 1]);
            tm = tm_qs(m, a1, xp + he_electrons(m, a1));
        } else {
            auto gx = [&](double l, double x, double t) { return dxp_dlna(m, std::exp(l), x, t); };
            auto gt = [&](double l, double x, double t) { return dtm_dlna(m, std::exp(l), x, t); };
            double x1 = gx(l0, xp, tm), t1 = gt(l0, xp, tm);
            double x2 = gx(lm, xp + 0.5 * h * x1, tm + 0.5 * h * t1), t2 = gt(lm, xp + 0.5 * h * x1, tm + 0.5 * h * t1);
            double x3 = gx(lm, xp + 0.5 * h * x2, tm + 0.5 * h * t2), t3 = gt(lm, xp + 0.5 * h * x2, tm + 0.5 * h * t2);
            double x4 = gx(l1, xp + h * x3, tm + h * t3), t4 = gt(l1, xp + h * x3, tm + h * t3);
            xp += h / 6.0 * (x1 + 2.0 * x2 + 2.0 * x3 + x4);
            tm += h / 6.0 * (t1 + 2.0 * t2 + 2.0 * t3 + t4);
        }
        double a1 = std::exp(lna[j + 1]);
        xrec[j + 1] = xp + he_electrons(m, a1);
        Tm[j + 1] = tm;
        dlnT[j + 1] = (1.0 / a1 - 1.0 >= zsw) ? -1.0 : dtm_dlna(m, a1, xp, tm) / tm;
    }

    // thermodynamics columns
    T.xe.resize(n + 1);
    T.tm = Tm;
    std::vector<double> ldk(n + 1), lcs(n + 1), ltau(n + 1), kap(n + 1), integ(n + 1);
    const double mH_mHe = kMH / kMHe;
    for (int i = 0; i <= n; ++i) {
        double a = std::exp(lna[i]);
        double xe = R.blend(1.0 / a - 1.0, xrec[i]);
        T.xe[i] = xe;
        double dk = xe * m.dk_pref / (a * a);
        ldk[i] = std::log(dk);
        double mu = kMH / ((1.0 + xe) * (1.0 - m.Y) + mH_mHe * m.Y);
        lcs[i] = std::log(Tm[i] / mu * (1.0 - dlnT[i] / 3.0));
        integ[i] = dk / m.Hc(a);
    }
    std::vector<double> tau(n + 1);
    {
        double a0 = std::exp(L0);
        tau[0] = 2.0 / m.rt_m0 * (std::sqrt(m.rt_rad_early + m.rt_m0 * a0) - std::sqrt(m.rt_rad_early));
        for (int i = 0; i < n; ++i) {
            double h = lna[i + 1] - lna[i];
            double fa = 1.0 / m.Hc(std::exp(lna[i])), fm = 1.0 / m.Hc(std::exp(lna[i] + 0.5 * h)),
                   fb = 1.0 / m.Hc(std::exp(lna[i + 1]));
            tau[i + 1] = tau[i] + h / 6.0 * (fa + 4.0 * fm + fb);
        }
        for (int i = 0; i <= n; ++i) ltau[i] = std::log(tau[i]);
    }
    kap[n] = 0.0;
    for (int i = n - 1; i >= 0; --i) kap[i] = kap[i + 1] + 0.5 * (lna[i + 1] - lna[i]) * (integ[i] + integ[i + 1]);

    T.cosmo = c;
    T.prec = p;
    T.k.assign(k, k + n_k);
    T.lna_start = lna_i;
    T.n_tab = n;
    T.L0 = L0;
    T.dl = dl;
    T.tau0 = tau[n];
    T.z_reio = zre;
    T.lna_tc = lna_tc;
    T.N_massless = m.N_ml;
    T.Neff = m.Neff;
    T.R_nu = m.R_nu;
    T.rt_g0 = m.rt_g0;
    T.rt_ur0 = m.rt_ur0;
    T.rt_c0 = m.rt_c0;
    T.rt_b0 = m.rt_b0;
    T.rt_L = m.rt_L;
    T.pref_ncdm = m.pref_n;
    T.m_over_T = m.m_over_T;
    T.H0 = m.H0;
    T.q = m.q;
    T.W = m.W;
    T.col[0] = ldk;
    T.col[1] = kap;
    T.col[2] = lcs;
    T.col[3] = ltau;
    for (int cidx = 0; cidx < 4; ++cidx) natural_spline(T.col[cidx], dl, T.M[cidx]);
    // per-interval polynomials: on [j, j+1], S(t) = c0 + c1 t + c2 t^2 + c3 t^3
    T.poly.assign((size_t)n * 16, 0.0);
    const double h6 = dl * dl / 6.0;
    for (int s = 0; s < n; ++s) {
        for (int cidx = 0; cidx < 4; ++cidx) {
            const std::vector<double> &f = T.col[cidx], &M = T.M[cidx];
            double *o = &T.poly[(size_t)s * 16 + cidx * 4];
            o[0] = f[s];
            o[1] = f[s + 1] - f[s] - h6 * (2.0 * M[s] + M[s + 1]);
            o[2] = 3.0 * h6 * M[s];
            o[3] = h6 * (M[s + 1] - M[s]);
        }
    }

    // output grid: ceil(0.6 n_tau) uniform in ln a on [ln a(z=2500), ln a(z=400)],
    // the rest uniform on (ln a(z=400), 0]
    int n1 = (int)std::ceil(0.6 * n_tau), n2 = n_tau - n1;
    double la = -std::log(2501.0), lb = -std::log(401.0);
    T.lna_src.resize(n_tau);
    for (int i = 0; i < n1; ++i) T.lna_src[i] = la + (lb - la) * i / (n1 - 1);
    for (int i = 1; i <= n2; ++i) T.lna_src[n1 + i - 1] = lb + (0.0 - lb) * i / n2;
    T.lna_src[n_tau - 1] = 0.0;
    T.tau_src.resize(n_tau);
    T.chi_src.resize(n_tau);
    T.w_src.resize(n_tau);
    std::vector<double> Hsrc(n_tau);
    for (int i = 0; i < n_tau; ++i) {
        T.tau_src[i] = std::exp(T.eval(3, T.lna_src[i]));
        T.chi_src[i] = T.tau0 - T.tau_src[i];
        Hsrc[i] = m.Hc(std::exp(T.lna_src[i]));
    }
    T.chi_src[n_tau - 1] = 0.0;
    for (int i = 0; i < n_tau; ++i) {
        double lo = T.lna_src[i > 0 ? i - 1 : i], hi = T.lna_src[i < n_tau - 1 ? i + 1 : i];
        T.w_src[i] = 0.5 * (hi - lo) / Hsrc[i];
    }

    // lensing (App. B.5): chi_* from the visibility peak g = kappa' e^{-kappa}
    // (conformal time), located on the table knots and refined by the vertex
    // of the parabola through the three knots around the largest value
    {
        int j = 1;
        double gmax = -1.0;
        for (int i = 1; i < n; ++i) {
            double g = std::exp(ldk[i] - kap[i]);
            if (g > gmax) {
                gmax = g;
                j = i;
            }
        }
        double gm = std::exp(ldk[j - 1] - kap[j - 1]), g0 = std::exp(ldk[j] - kap[j]),
               gp = std::exp(ldk[j + 1] - kap[j + 1]);
        double den = gm - 2.0 * g0 + gp;
        double off = den != 0.0 ? 0.5 * (gm - gp) / den : 0.0;
        T.lna_star = lna[j] + off * dl;
        T.tau_star = std::exp(T.eval(3, T.lna_star));
        T.chi_star = T.tau0 - T.tau_star;
    }
    // Limber weights per output time: w_j / chi_j (3/2 a^2 rho_m)^2 ((chi_* - chi_j)/chi_*)^2
    // for 0 < chi_j < chi_*, rho_m over CDM, baryons and massive neutrinos
    T.lens_w.assign(n_tau, 0.0);
    for (int i = 0; i < n_tau; ++i) {
        const double chi = T.chi_src[i];
        if (!(chi > 0.0 && chi < T.chi_star)) continue;
        const double a = std::exp(T.lna_src[i]);
        double rn, pn;
        m.ncdm(a, rn, pn);
        const double src = 1.5 * a * a * (m.rt_m0 / (a * a * a) + rn);
        const double f = (T.chi_star - chi) / T.chi_star;
        T.lens_w[i] = T.w_src[i] / chi * src * src * f * f;
    }
    return CMB_OK;
}

double Tables::eval(int cidx, double lna) const {
    double u = (lna - L0) / dl;
    int s = (int)std::floor(u);
    s = std::min(std::max(s, 0), n_tab - 1);
    double t = u - s;
    const double *o = &poly[(size_t)s * 16 + cidx * 4];
    return ((o[3] * t + o[2]) * t + o[1]) * t + o[0];
}

}  // namespace cmbhip
