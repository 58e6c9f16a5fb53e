// K1: synchronous-gauge perturbations and CMB source functions on gfx950.
//
// One lane integrates one (cosmology, k) mode from its start time to a = 1
// (arXiv 2602.15104, App. B.3 and App. C: CDM, baryons, photon temperature
// F_l and polarisation G_l hierarchies, massless neutrinos, metric h' and
// eta'), with the ESDIRK4(3)6L[2]SA scheme of Kennedy & Carpenter (order 4,
// L-stable, stiffly accurate, embedded order 3), RMS error norm, PID step
// control with (pcoeff, icoeff, dcoeff) and a Hairer-Norsett-Wanner first
// step.  At the output times it evaluates the source functions of App. B.4
// (eq. source_functions) on the cubic Hermite dense output.
//
// Stage solve.  The system is linear, y' = A(ln a) y, so each implicit stage is
// one solve of (I - h gamma A) Y = R.  A is the paper's equations written as
// three tridiagonal chains in the multipole index,
//     [delta_b, theta_b, theta_g, sigma_g, F_3 .. F_lmax]   (photon T + baryons)
//     [G_0 .. G_lmax]                                        (photon P)
//     [delta_nu, theta_nu, sigma_nu, F_3 .. F_lmax]         (neutrinos)
// plus three isolated rows (delta_c, delta_g, eta) and three scalar couplings:
// h' (00 Einstein equation), eta' (0i equation) and Pi = 2 sigma_g + G_0 + G_2.
// delta_g couples only to theta_g and is eliminated into that row.  The
// chains are reduced from the highest multipole upwards; the scalar
// couplings touch only the four lowest rows of each chain, so after the
// upward sweep the lowest rows are affine in (h', eta', Pi); the three
// coupling equations then give a 3x3 system, and one downward sweep
// finishes the stage.  K_s = (Y_s - R_s)/(h gamma) avoids forming A Y.
//
// Memory.  Working vectors (state, stage derivatives, sweep factors) live in
// a structure-of-arrays workspace, element [vector][row][lane], so every
// access by a wavefront is 64 consecutive doubles.  Modes are numbered with
// the cosmology index fastest and the largest k first, so one wavefront holds
// modes with similar step counts and the longest ones start first.
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

namespace {

constexpr int NV = 11;  // workspace vectors per mode
enum Slot { SY = 0, SYN = 1, SK1 = 2, SR = 8, SIB = 9, SRP = 10 };

__device__ constexpr double RKc[6] = {0.0, 0.5, 83.0 / 250.0, 31.0 / 50.0, 17.0 / 20.0, 1.0};
__device__ constexpr double RKa[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.25, 0.25, 0, 0, 0, 0},
    {8611.0 / 62500.0, -1743.0 / 31250.0, 0.25, 0, 0, 0},
    {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, 0.25, 0, 0},
    {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0, 2285395.0 / 8070912.0,
     0.25, 0},
    {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, 0.25}};
// b - bhat (error weights)
__device__ constexpr double RKe[6] = {
    82889.0 / 524892.0 - 4586570599.0 / 29645900160.0, 0.0, 15625.0 / 83664.0 - 178811875.0 / 945068544.0,
    69875.0 / 102672.0 - 814220225.0 / 1159782912.0, -2260.0 / 8211.0 + 3700637.0 / 11593932.0,
    0.25 - 61727.0 / 225920.0};
constexpr double GAM = 0.25;

struct Ws {
    double *base;
    size_t S;  // lane stride
    int N;
    __device__ double &at(int slot, int row) const { return base[((size_t)slot * N + row) * S]; }
};

// Background and thermodynamics at one ln a, plus the per-stage constants.
struct St {
    double a, Hc, Hcp, rg, rur, rc, rb;
    double dk, dkp, kap, cs2, tau;
    // derived
    double invHc, kH, k2H, T, R, trunc, cH1, cH2, cE;
};

__device__ void state_at(const DevTab &tb, const DevPrec &p, double k, double lna, St &s) {
    double a = exp(lna);
    s.a = a;
    double a2 = a * a, a3 = a2 * a, a4 = a2 * a2;
    s.rg = tb.rt_g0 / a4;
    s.rur = tb.rt_ur0 / a4;
    s.rc = tb.rt_c0 / a3;
    s.rb = tb.rt_b0 / a3;
    double rho = s.rg + s.rur + s.rc + s.rb + tb.rt_L;
    double pr = (s.rg + s.rur) * (1.0 / 3.0) - tb.rt_L;
    s.Hc = a * sqrt(rho);
    s.Hcp = s.Hc * (1.0 - 1.5 * (rho + pr) / rho);
    double u = (lna - tb.L0) * tb.inv_dl;
    int j = (int)floor(u);
    j = j < 0 ? 0 : (j > tb.n_tab - 1 ? tb.n_tab - 1 : j);
    double t = u - j;
    const double *o = tb.poly + (size_t)j * 16;
    double l0 = ((o[3] * t + o[2]) * t + o[1]) * t + o[0];
    double d0 = ((3.0 * o[3] * t + 2.0 * o[2]) * t + o[1]) * tb.inv_dl;
    s.dk = exp(l0);
    s.dkp = s.dk * d0;
    s.kap = ((o[7] * t + o[6]) * t + o[5]) * t + o[4];
    s.cs2 = exp(((o[11] * t + o[10]) * t + o[9]) * t + o[8]);
    s.tau = exp(((o[15] * t + o[14]) * t + o[13]) * t + o[12]);
    s.invHc = 1.0 / s.Hc;
    s.kH = k * s.invHc;
    s.k2H = k * s.kH;
    s.T = p.thom * s.dk * s.invHc;
    s.R = (4.0 / 3.0) * s.rg / s.rb;
    s.trunc = s.invHc / s.tau;
    double ih2 = s.invHc * s.invHc;
    s.cH1 = p.grav * 2.0 * k * k * ih2;
    s.cH2 = p.grav * 3.0 * a2 * ih2;
    s.cE = p.grav * 1.5 * a2 * s.invHc / (k * k);
}

struct Co {
    double a, d, c, uH, uE, uP;
};

// Row j of chain CH: y'_j = a y_{j-1} + d y_j + c y_{j+1} + uH h' + uE eta' + uP Pi
template <int CH>
__device__ inline Co coef(int j, int n, const St &s, const DevPrec &p) {
    Co r{0, 0, 0, 0, 0, 0};
    if (CH == 0) {  // delta_b, theta_b, theta_g, sigma_g, F_3..F_lg
        if (j == 0) {
            r.c = -s.invHc;
            r.uH = -0.5;
        } else if (j == 1) {
            r.a = s.cs2 * s.k2H;
            r.d = -1.0 - s.R * s.T;
            r.c = s.R * s.T;
        } else if (j == 2) {
            r.a = s.T;
            r.d = -s.T;
            r.c = -s.k2H;
        } else if (j == 3) {
            r.a = (4.0 / 15.0) * s.invHc;
            r.c = -0.3 * s.kH;
            r.uH = 2.0 / 15.0;
            r.uE = 0.8;
            if (p.lp > 0) {
                r.d = -s.T;
                r.uP = 0.05 * s.T;
            } else {
                r.d = -0.9 * s.T;
            }
        } else {
            int l = j - 1;
            double f2 = (l == 3) ? 2.0 : 1.0;  // F_2 = 2 sigma_g
            if (j == n - 1) {
                r.a = f2 * s.kH;
                r.d = -(l + 1.0) * s.trunc - s.T;
            } else {
                double w = s.kH / (2.0 * l + 1.0);
                r.a = f2 * l * w;
                r.d = -s.T;
                r.c = -(l + 1.0) * w;
            }
        }
    } else if (CH == 1) {  // G_0..G_lp
        int l = j;
        if (j == n - 1) {
            r.a = s.kH;
            r.d = -(l + 1.0) * s.trunc - s.T;
        } else {
            double w = s.kH / (2.0 * l + 1.0);
            r.a = l * w;
            r.d = -s.T;
            r.c = -(l + 1.0) * w;
            if (l == 0) r.uP = 0.5 * s.T;
            if (l == 2) r.uP = 0.1 * s.T;
        }
    } else {  // delta_nu, theta_nu, sigma_nu, F_3..F_ln
        if (j == 0) {
            r.c = -(4.0 / 3.0) * s.invHc;
            r.uH = -2.0 / 3.0;
        } else if (j == 1) {
            r.a = 0.25 * s.k2H;
            r.c = -s.k2H;
        } else if (j == 2) {
            r.a = (4.0 / 15.0) * s.invHc;
            r.c = -0.3 * s.kH;
            r.uH = 2.0 / 15.0;
            r.uE = 0.8;
        } else {
            int l = j;
            double f2 = (l == 3) ? 2.0 : 1.0;
            if (j == n - 1) {
                r.a = f2 * s.kH;
                r.d = -(l + 1.0) * s.trunc;
            } else {
                double w = s.kH / (2.0 * l + 1.0);
                r.a = f2 * l * w;
                r.c = -(l + 1.0) * w;
            }
        }
    }
    return r;
}

struct Layout {
    int N, nF, nG, nV, bF, bG, bV;
};
__device__ inline Layout layout(const DevPrec &p) {
    Layout L;
    L.nF = p.lg + 2;
    L.nG = p.lp > 0 ? p.lp + 1 : 0;
    L.nV = p.ln + 1;
    L.bF = 3;
    L.bG = L.bF + L.nF;
    L.bV = L.bG + L.nG;
    L.N = L.bV + L.nV;
    return L;
}
// isolated rows
constexpr int RDC = 0, RDG = 1, RETA = 2;

// f = A y for a whole vector (slot src -> slot dst).
template <int CH>
__device__ void rhs_chain(const Ws &w, int src, int dst, int base, int n, const St &s, const DevPrec &p, double H,
                          double E, double P) {
    double ym = 0.0, y0 = w.at(src, base);
    for (int j = 0; j < n; ++j) {
        double yp = (j + 1 < n) ? w.at(src, base + j + 1) : 0.0;
        Co c = coef<CH>(j, n, s, p);
        double f = c.a * ym + c.d * y0 + c.c * yp + c.uH * H + c.uE * E + c.uP * P;
        if (CH == 0 && j == 2) f += 0.25 * s.k2H * w.at(src, RDG);
        w.at(dst, base + j) = f;
        ym = y0;
        y0 = yp;
    }
}

__device__ void aux_from_state(const Ws &w, int src, const Layout &L, const St &s, const DevPrec &p, double &H,
                               double &E, double &P) {
    H = s.cH1 * w.at(src, RETA) + s.cH2 * (s.rc * w.at(src, RDC) + s.rb * w.at(src, L.bF) + s.rg * w.at(src, RDG) +
                                           s.rur * w.at(src, L.bV));
    E = s.cE * (s.rb * w.at(src, L.bF + 1) + (4.0 / 3.0) * s.rg * w.at(src, L.bF + 2) +
                (4.0 / 3.0) * s.rur * w.at(src, L.bV + 1));
    P = (p.lp > 0) ? 2.0 * w.at(src, L.bF + 3) + w.at(src, L.bG) + w.at(src, L.bG + 2) : 0.0;
}

__device__ void rhs_full(const Ws &w, int src, int dst, const Layout &L, const St &s, const DevPrec &p) {
    double H, E, P;
    aux_from_state(w, src, L, s, p, H, E, P);
    w.at(dst, RDC) = -0.5 * H;
    w.at(dst, RDG) = -(4.0 / 3.0) * s.invHc * w.at(src, L.bF + 2) - (2.0 / 3.0) * H;
    w.at(dst, RETA) = E;
    rhs_chain<0>(w, src, dst, L.bF, L.nF, s, p, H, E, P);
    if (L.nG) rhs_chain<1>(w, src, dst, L.bG, L.nG, s, p, H, E, P);
    rhs_chain<2>(w, src, dst, L.bV, L.nV, s, p, H, E, P);
}

// Affine value of one of the four lowest chain rows: v0 + vH h' + vE eta' + vP Pi.
struct Aff {
    double v0, vH, vE, vP;
};

// Upward (highest multipole first) elimination of one chain for the stage
// matrix I - g A.  Stores 1/b'_j and rho'_j (rows >= 4 only need these) and
// returns the four lowest rows of the downward solution as affine functions.
template <int CH>
__device__ void sweep_up(const Ws &w, int base, int n, const St &s, const DevPrec &p, double g, Aff top[4]) {
    // rows n-1 .. 4: no scalar couplings
    double bp = 0.0, rp = 0.0, al_below = 0.0;
    for (int j = n - 1; j >= 4; --j) {
        Co c = coef<CH>(j, n, s, p);
        double be = 1.0 - g * c.d, ga = -g * c.c;
        double rho = w.at(SR, base + j);
        if (j < n - 1) {
            double m = ga / bp;
            be -= m * al_below;
            rho -= m * rp;
        }
        bp = be;
        rp = rho;
        al_below = -g * c.a;
        w.at(SIB, base + j) = 1.0 / be;
        w.at(SRP, base + j) = rho;
    }
    // rows 3 .. 0 with the couplings carried as extra right-hand sides
    double eH = 0.0, eE = 0.0, eP = 0.0;
    double ib[4], r0[4], rH[4], rE[4], rP[4], al[4];
    for (int j = 3; j >= 0; --j) {
        Co c = coef<CH>(j, n, s, p);
        double be = 1.0 - g * c.d, ga = -g * c.c;
        double rho = w.at(SR, base + j);
        double xH = -g * c.uH, xE = -g * c.uE, xP = -g * c.uP;
        if (CH == 0 && j == 2) {
            // eliminate the leaf delta_g = R_dg - g (4/3)/Hc theta_g - (2g/3) h'
            double cl = g * 0.25 * s.k2H;
            be += cl * g * (4.0 / 3.0) * s.invHc;
            xH += cl * g * (2.0 / 3.0);
            rho += cl * w.at(SR, RDG);
        }
        if (j < n - 1) {
            double m = ga / bp;
            be -= m * al_below;
            rho -= m * rp;
            xH -= m * eH;
            xE -= m * eE;
            xP -= m * eP;
        }
        bp = be;
        rp = rho;
        eH = xH;
        eE = xE;
        eP = xP;
        al_below = -g * c.a;
        ib[j] = 1.0 / be;
        r0[j] = rho;
        rH[j] = xH;
        rE[j] = xE;
        rP[j] = xP;
        al[j] = -g * c.a;
    }
    // downward substitution of the lowest rows, affine in the couplings
    for (int j = 0; j < 4; ++j) {
        double v0 = r0[j], vH = -rH[j], vE = -rE[j], vP = -rP[j];
        if (j > 0) {
            v0 -= al[j] * top[j - 1].v0;
            vH -= al[j] * top[j - 1].vH;
            vE -= al[j] * top[j - 1].vE;
            vP -= al[j] * top[j - 1].vP;
        }
        top[j].v0 = v0 * ib[j];
        top[j].vH = vH * ib[j];
        top[j].vE = vE * ib[j];
        top[j].vP = vP * ib[j];
    }
}

// Downward sweep of rows >= 4 given the four lowest rows; writes
// K = (Y - R)/g into slot kslot and, if ynew, Y into SYN.
template <int CH>
__device__ void sweep_down(const Ws &w, int base, int n, const St &s, const DevPrec &p, double g, const double y4[4],
                           int kslot, bool ynew) {
    double ig = 1.0 / g;
    for (int j = 0; j < 4; ++j) {
        double y = y4[j];
        w.at(kslot, base + j) = (y - w.at(SR, base + j)) * ig;
        if (ynew) w.at(SYN, base + j) = y;
    }
    double yprev = y4[3];
    for (int j = 4; j < n; ++j) {
        Co c = coef<CH>(j, n, s, p);
        double y = (w.at(SRP, base + j) + g * c.a * yprev) * w.at(SIB, base + j);
        w.at(kslot, base + j) = (y - w.at(SR, base + j)) * ig;
        if (ynew) w.at(SYN, base + j) = y;
        yprev = y;
    }
}

__device__ inline double affv(const Aff &a, double H, double E, double P) { return a.v0 + a.vH * H + a.vE * E + a.vP * P; }

// One implicit stage: solve (I - g A(ts)) Y = R (R in slot SR).
__device__ void stage_solve(const Ws &w, const Layout &L, const St &s, const DevPrec &p, double g, int kslot,
                            bool ynew) {
    Aff tF[4], tG[4], tV[4];
    sweep_up<0>(w, L.bF, L.nF, s, p, g, tF);
    if (L.nG) sweep_up<1>(w, L.bG, L.nG, s, p, g, tG);
    sweep_up<2>(w, L.bV, L.nV, s, p, g, tV);
    // isolated rows as affine functions
    double Rdc = w.at(SR, RDC), Reta = w.at(SR, RETA), Rdg = w.at(SR, RDG);
    Aff dc{Rdc, -0.5 * g, 0.0, 0.0};
    Aff eta{Reta, 0.0, g, 0.0};
    double cg = -g * (4.0 / 3.0) * s.invHc;
    Aff dg{Rdg + cg * tF[2].v0, cg * tF[2].vH - (2.0 / 3.0) * g, cg * tF[2].vE, cg * tF[2].vP};
    // coupling equations X = v + M X
    Aff eqH, eqE, eqP;
    eqH.v0 = s.cH1 * eta.v0 + s.cH2 * (s.rc * dc.v0 + s.rb * tF[0].v0 + s.rg * dg.v0 + s.rur * tV[0].v0);
    eqH.vH = s.cH1 * eta.vH + s.cH2 * (s.rc * dc.vH + s.rb * tF[0].vH + s.rg * dg.vH + s.rur * tV[0].vH);
    eqH.vE = s.cH1 * eta.vE + s.cH2 * (s.rc * dc.vE + s.rb * tF[0].vE + s.rg * dg.vE + s.rur * tV[0].vE);
    eqH.vP = s.cH1 * eta.vP + s.cH2 * (s.rc * dc.vP + s.rb * tF[0].vP + s.rg * dg.vP + s.rur * tV[0].vP);
    const double f43 = 4.0 / 3.0;
    eqE.v0 = s.cE * (s.rb * tF[1].v0 + f43 * s.rg * tF[2].v0 + f43 * s.rur * tV[1].v0);
    eqE.vH = s.cE * (s.rb * tF[1].vH + f43 * s.rg * tF[2].vH + f43 * s.rur * tV[1].vH);
    eqE.vE = s.cE * (s.rb * tF[1].vE + f43 * s.rg * tF[2].vE + f43 * s.rur * tV[1].vE);
    eqE.vP = s.cE * (s.rb * tF[1].vP + f43 * s.rg * tF[2].vP + f43 * s.rur * tV[1].vP);
    double H, E, P;
    if (L.nG) {
        eqP.v0 = 2.0 * tF[3].v0 + tG[0].v0 + tG[2].v0;
        eqP.vH = 2.0 * tF[3].vH + tG[0].vH + tG[2].vH;
        eqP.vE = 2.0 * tF[3].vE + tG[0].vE + tG[2].vE;
        eqP.vP = 2.0 * tF[3].vP + tG[0].vP + tG[2].vP;
        // (I - M) X = v, 3x3, Gaussian elimination with partial pivoting
        double m[3][4] = {{1.0 - eqH.vH, -eqH.vE, -eqH.vP, eqH.v0},
                          {-eqE.vH, 1.0 - eqE.vE, -eqE.vP, eqE.v0},
                          {-eqP.vH, -eqP.vE, 1.0 - eqP.vP, eqP.v0}};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int piv = c;
#pragma unroll
            for (int r = c + 1; r < 3; ++r)
                if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
            if (piv != c) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double t = m[c][q];
                    m[c][q] = m[piv][q];
                    m[piv][q] = t;
                }
            }
#pragma unroll
            for (int r = c + 1; r < 3; ++r) {
                double f = m[r][c] / m[c][c];
#pragma unroll
                for (int q = c; q < 4; ++q) m[r][q] -= f * m[c][q];
            }
        }
        P = m[2][3] / m[2][2];
        E = (m[1][3] - m[1][2] * P) / m[1][1];
        H = (m[0][3] - m[0][1] * E - m[0][2] * P) / m[0][0];
    } else {
        double a11 = 1.0 - eqH.vH, a12 = -eqH.vE, a21 = -eqE.vH, a22 = 1.0 - eqE.vE;
        double det = a11 * a22 - a12 * a21;
        H = (eqH.v0 * a22 - a12 * eqE.v0) / det;
        E = (a11 * eqE.v0 - a21 * eqH.v0) / det;
        P = 0.0;
    }
    // finish: isolated rows, then each chain downward
    double ig = 1.0 / g;
    double ydc = affv(dc, H, E, P), yeta = affv(eta, H, E, P), ydg = affv(dg, H, E, P);
    w.at(kslot, RDC) = (ydc - Rdc) * ig;
    w.at(kslot, RETA) = (yeta - Reta) * ig;
    w.at(kslot, RDG) = (ydg - Rdg) * ig;
    if (ynew) {
        w.at(SYN, RDC) = ydc;
        w.at(SYN, RETA) = yeta;
        w.at(SYN, RDG) = ydg;
    }
    double y4[4];
    for (int j = 0; j < 4; ++j) y4[j] = affv(tF[j], H, E, P);
    sweep_down<0>(w, L.bF, L.nF, s, p, g, y4, kslot, ynew);
    if (L.nG) {
        for (int j = 0; j < 4; ++j) y4[j] = affv(tG[j], H, E, P);
        sweep_down<1>(w, L.bG, L.nG, s, p, g, y4, kslot, ynew);
    }
    for (int j = 0; j < 4; ++j) y4[j] = affv(tV[j], H, E, P);
    sweep_down<2>(w, L.bV, L.nV, s, p, g, y4, kslot, ynew);
}

__device__ double rms_ratio(const Ws &w, int N, int sv, int sy, int sy2, double rtol, double atol) {
    double acc = 0.0;
    for (int r = 0; r < N; ++r) {
        double y = fabs(w.at(sy, r));
        if (sy2 >= 0) y = fmax(y, fabs(w.at(sy2, r)));
        double q = w.at(sv, r) / (atol + rtol * y);
        acc += q * q;
    }
    return sqrt(acc / N);
}

// Source functions at one output time from the interpolated state.
struct SrcState {
    double dc, dg, eta, db, tb, tg, sg, G0, G2, dn, tn, sn;
};

__device__ void sources(const DevTab &tb, const DevPrec &p, double k, double lna, const SrcState &y, double &S0,
                        double &S1, double &S2) {
    St s;
    state_at(tb, p, k, lna, s);
    double k2 = k * k;
    double H = s.cH1 * y.eta + s.cH2 * (s.rc * y.dc + s.rb * y.db + s.rg * y.dg + s.rur * y.dn);
    double E = s.cE * (s.rb * y.tb + (4.0 / 3.0) * s.rg * y.tg + (4.0 / 3.0) * s.rur * y.tn);
    double tbp = s.cs2 * s.k2H * y.db + (-1.0 - s.R * s.T) * y.tb + s.R * s.T * y.tg;
    double ek = exp(-s.kap);
    double g = s.dk * ek;
    double gp = (s.dkp + s.dk * s.dk * s.invHc) * ek;
    double Hc = s.Hc;
    double alpha = Hc * (H + 6.0 * E) / (2.0 * k2);
    double rps = (4.0 / 3.0) * (s.rg * y.sg + s.rur * y.sn);
    double alphap = -2.0 * alpha + (y.eta - 4.5 * s.a * s.a * rps / k2) * s.invHc;
    double Pi = 2.0 * y.sg + (p.lp > 0 ? y.G0 + y.G2 : 0.0);
    S0 = p.sw * g * (0.25 * y.dg + Hc * alphap) +
         p.isw * (g * (y.eta - Hc * alphap - 2.0 * Hc * alpha) + 2.0 * Hc * ek * (E - s.Hcp * alpha - Hc * alphap)) +
         p.dop * Hc * (g * (tbp / k2 + alphap) + gp * (y.tb / k2 + alpha));
    S1 = p.isw * ek * k * (Hc * alphap + 2.0 * Hc * alpha - y.eta);
    S2 = g * Pi * 0.125;
}

__global__ void __launch_bounds__(64) perturb_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k, int n_tau,
                                                     DevPrec p, double *__restrict__ ws, size_t S,
                                                     double *__restrict__ Sout, int *__restrict__ status,
                                                     int *__restrict__ nsteps) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_sys = n_cosmo * n_k;
    if (lane >= n_sys) return;
    // largest k first, cosmology index fastest
    const int sys = n_sys - 1 - lane;
    const int c = sys % n_cosmo;
    const int ik = sys / n_cosmo;
    const DevTab tb = tabs[c];
    const Layout L = layout(p);
    const int N = L.N;
    Ws w{ws + lane, S, N};
    const double k = tb.k[ik];
    const double t0 = tb.lna_start[ik];
    const bool small = k < tb.k_split;
    const double rtol = small ? tb.rtol_small : tb.rtol_large;
    const double atol = small ? tb.atol_small : tb.atol_large;
    double *So = Sout + ((size_t)c * n_k + ik) * 3 * n_tau;
    const double *lo = tb.lna_src;

    // initial conditions: adiabatic growing mode (Ma & Bertschinger 1995), eta -> 1
    St s;
    state_at(tb, p, k, t0, s);
    for (int r = 0; r < N; ++r) w.at(SY, r) = 0.0;
    {
        double x = k * s.tau, Rn = tb.R_nu;
        double dg = -x * x / 3.0, tg = -k * x * x * x / 36.0;
        w.at(SY, RDC) = 0.75 * dg;
        w.at(SY, RDG) = dg;
        w.at(SY, RETA) = 1.0 - (5.0 + 4.0 * Rn) / (12.0 * (15.0 + 4.0 * Rn)) * x * x;
        w.at(SY, L.bF) = 0.75 * dg;
        w.at(SY, L.bF + 1) = tg;
        w.at(SY, L.bF + 2) = tg;
        w.at(SY, L.bV) = dg;
        w.at(SY, L.bV + 1) = (23.0 + 4.0 * Rn) / (15.0 + 4.0 * Rn) * tg;
        w.at(SY, L.bV + 2) = 2.0 / (3.0 * (15.0 + 4.0 * Rn)) * x * x;
    }
    rhs_full(w, SY, SK1, L, s, p);
    int jo = 0;
    while (jo < n_tau && lo[jo] < t0) {
        So[jo] = 0.0;
        So[n_tau + jo] = 0.0;
        So[2 * n_tau + jo] = 0.0;
        ++jo;
    }
    double t = t0;
    // first step (Hairer, Norsett & Wanner), order 4
    double h;
    {
        double d0 = rms_ratio(w, N, SY, SY, -1, rtol, atol);
        double d1 = rms_ratio(w, N, SK1, SY, -1, rtol, atol);
        double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
        if (h0 > -t) h0 = -t;
        for (int r = 0; r < N; ++r) w.at(SR, r) = w.at(SY, r) + h0 * w.at(SK1, r);
        St s1;
        state_at(tb, p, k, t + h0, s1);
        rhs_full(w, SR, SYN, L, s1, p);
        double acc = 0.0;
        for (int r = 0; r < N; ++r) {
            double q = (w.at(SYN, r) - w.at(SK1, r)) / (atol + rtol * fabs(w.at(SY, r)));
            acc += q * q;
        }
        double d2 = sqrt(acc / N) / h0;
        double dm = fmax(d1, d2);
        double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 0.2);
        h = fmin(100.0 * h0, h1);
    }
    const double q = 4.0;
    const double b1 = (p.pcoeff + p.icoeff + p.dcoeff) / q;
    const double b2 = -(p.pcoeff + 2.0 * p.dcoeff) / q;
    const double b3 = p.dcoeff / q;
    double Ep = 1.0, Epp = 1.0;
    int ns = 0, st = CMB_K_OK;

    while (t < 0.0) {
        if (ns >= p.max_steps) {
            st = CMB_K_MAX_STEPS;
            break;
        }
        bool last = false;
        if (h >= -t) {
            h = -t;
            last = true;
        }
        const double g = h * GAM;
        for (int sidx = 1; sidx < 6; ++sidx) {
            double ts = (sidx == 5) ? (last ? 0.0 : t + h) : t + RKc[sidx] * h;
            state_at(tb, p, k, ts, s);
            for (int r = 0; r < N; ++r) {
                double acc = w.at(SY, r);
                for (int j = 0; j < sidx; ++j) acc += h * RKa[sidx][j] * w.at(SK1 + j, r);
                w.at(SR, r) = acc;
            }
            stage_solve(w, L, s, p, g, SK1 + sidx, sidx == 5);
        }
        double acc = 0.0;
        for (int r = 0; r < N; ++r) {
            double e = 0.0;
            for (int j = 0; j < 6; ++j) e += RKe[j] * w.at(SK1 + j, r);
            e *= h;
            double sc = atol + rtol * fmax(fabs(w.at(SY, r)), fabs(w.at(SYN, r)));
            double qq = e / sc;
            acc += qq * qq;
        }
        double E = sqrt(acc / N);
        ++ns;
        if (!isfinite(E)) {
            st = CMB_K_NONFINITE;
            break;
        }
        double fac;
        if (E <= 1.0) {
            double tn = last ? 0.0 : t + h;
            if (tn >= 0.0) tn = 0.0;
            double hh = tn - t;
            while (jo < n_tau && lo[jo] <= tn) {
                double th = hh > 0.0 ? (lo[jo] - t) / hh : 1.0;
                double th2 = th * th, th3 = th2 * th;
                double h00 = 2.0 * th3 - 3.0 * th2 + 1.0, h10 = th3 - 2.0 * th2 + th;
                double h01 = -2.0 * th3 + 3.0 * th2, h11 = th3 - th2;
                auto I = [&](int r) {
                    return h00 * w.at(SY, r) + h10 * hh * w.at(SK1, r) + h01 * w.at(SYN, r) +
                           h11 * hh * w.at(SK1 + 5, r);
                };
                SrcState y;
                y.dc = I(RDC);
                y.dg = I(RDG);
                y.eta = I(RETA);
                y.db = I(L.bF);
                y.tb = I(L.bF + 1);
                y.tg = I(L.bF + 2);
                y.sg = I(L.bF + 3);
                y.G0 = L.nG ? I(L.bG) : 0.0;
                y.G2 = L.nG ? I(L.bG + 2) : 0.0;
                y.dn = I(L.bV);
                y.tn = I(L.bV + 1);
                y.sn = I(L.bV + 2);
                double S0, S1, S2;
                sources(tb, p, k, lo[jo], y, S0, S1, S2);
                So[jo] = S0;
                So[n_tau + jo] = S1;
                So[2 * n_tau + jo] = S2;
                ++jo;
            }
            for (int r = 0; r < N; ++r) {
                w.at(SY, r) = w.at(SYN, r);
                w.at(SK1, r) = w.at(SK1 + 5, r);
            }
            t = tn;
            double Ef = fmax(E, 1e-10);
            fac = 0.9 * pow(Ef, -b1) * pow(Ep, -b2) * pow(Epp, -b3);
            fac = fmin(10.0, fmax(0.2, fac));
            Epp = Ep;
            Ep = Ef;
        } else {
            fac = fmin(0.9, fmax(0.2, 0.9 * pow(E, -0.25)));
        }
        h *= fac;
        if (t < 0.0 && h < 1e-12) {
            st = CMB_K_STEP_UNDERFLOW;
            break;
        }
    }
    for (; jo < n_tau; ++jo) {
        So[jo] = 0.0;
        So[n_tau + jo] = 0.0;
        So[2 * n_tau + jo] = 0.0;
    }
    status[(size_t)c * n_k + ik] = st;
    nsteps[(size_t)c * n_k + ik] = ns;
}

}  // namespace

size_t perturb_ws_doubles(int n_cosmo, int n_k, const DevPrec &p) {
    int N = 3 + (p.lg + 2) + (p.lp > 0 ? p.lp + 1 : 0) + (p.ln + 1);
    size_t lanes = ((size_t)n_cosmo * n_k + 63) / 64 * 64;
    return lanes * N * NV;
}

int launch_perturb(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, double *d_ws,
                   double *d_S, int *d_status, int *d_nsteps, void *stream) {
    size_t lanes = ((size_t)n_cosmo * n_k + 63) / 64 * 64;
    dim3 grid((unsigned)(lanes / 64)), block(64);
    hipLaunchKernelGGL(perturb_kernel, grid, block, 0, (hipStream_t)stream, d_tabs, n_cosmo, n_k, n_tau, p, d_ws,
                       lanes, d_S, d_status, d_nsteps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("perturb launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
