// Device code shared by the perturbation kernel (K1) and its reverse sweep:
// the ESDIRK tableau, the background at one time, the layout of the state
// rows and their multipole chains, the row coefficients of the right-hand side
// y' = A y (App. B.3, App. C), the LDS records of a mode, the couplings h',
// eta', Pi, the initial conditions and the source functions (App. B.4).
#pragma once

#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

namespace {


// ESDIRK: the implicit part of Kennedy & Carpenter's ARK4(3)6L[2]SA (2003):
// six stages, explicit first stage, gamma = 1/4, stiffly accurate (the last
// row is the order-4 solution), Ke = b - bhat with bhat the order-3 weights.
constexpr int NSTG = 6;
static_assert(NSTG == kTrajStages, "trajectory records hold every stage derivative");
__device__ constexpr double Kc[NSTG] = {0.0, 0.5, 83.0 / 250.0, 31.0 / 50.0, 17.0 / 20.0, 1.0};
__device__ constexpr double Ka[NSTG][NSTG] = {
    {0, 0, 0, 0, 0, 0},
    {0.25, 0.25, 0, 0, 0, 0},
    {8611.0 / 62500.0, -1743.0 / 31250.0, 0.25, 0, 0, 0},
    {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, 0.25, 0, 0},
    {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0, 2285395.0 / 8070912.0,
     0.25, 0},
    {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, 0.25}};
__device__ constexpr double Ke[NSTG] = {
    82889.0 / 524892.0 - 4586570599.0 / 29645900160.0, 0.0, 15625.0 / 83664.0 - 178811875.0 / 945068544.0,
    69875.0 / 102672.0 - 814220225.0 / 1159782912.0, -2260.0 / 8211.0 + 3700637.0 / 11593932.0,
    0.25 - 61727.0 / 225920.0};
constexpr double GAMMA = 0.25;
constexpr double ERR_ORDER = 4.0;  // order of the error estimate (step control)

// 1/b: hardware reciprocal refined by two Newton steps (relative error at the
// level of rounding), shorter on the dependent path than IEEE division.
__device__ inline double rcp(double b) {
    // hardware estimate, then x (1 + e + e^2) with e = 1 - b x: the relative
    // error of the estimate enters cubed
    const double x = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, x, 1.0);
    return fma(x, fma(e, e, e), x);
}

// Exchange point between the lanes of a wavefront.  A workgroup is one
// wavefront, and the LDS executes a wavefront's DS instructions in the order
// they are issued, so a value one lane stores is seen by any lane's later
// load; what must not happen is the compiler moving a load or store across
// the exchange (it reasons per lane and would see no dependence).  The
// memory clobber forbids that and emits no instruction: no s_barrier, and no
// wait for outstanding stores (each load still waits for its own data).
// Groups of a wavefront may therefore sit in different branches.
__device__ inline void wsync() { __asm__ volatile("" ::: "memory"); }

// v of another lane of the same 16-lane row, selected by a DPP control word
// (both 32-bit halves moved; every lane of the row is active wherever this is
// used, since a group's lanes take the same branches)
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct Bk {  // background and per-stage constants at one ln a
    double a, Hc, Hcp, rg, rur, rc, rb;
    double dk, dkp, kap, cs2, tau;
    double invHc, kH, k2H, T, R, trunc, cH1, cH2, cE;
    double am, pn4;  // massive nu: a m/T and pref/a^4 (rho = pn4 sum W eps)
};
static_assert(sizeof(Bk) == 23 * sizeof(double), "Bk is a record of 23 doubles");

// massive-neutrino node energy and dln f0/dln q for f0 = 1/(e^q + 1)
__device__ inline double eps_of(double q, double am) { return sqrt(fma(q, q, am * am)); }
__device__ inline double dlnf0(double q) { return -q / (1.0 + exp(-q)); }

// MNU: the hierarchy has massive-neutrino chains (compiled separately, so the
// massless kernel carries none of their code)
template <bool MNU>
__device__ void bk_at(const DevTab &tb, const DevPrec &p, double k, double lna, Bk &s) {
    double a = exp(lna);
    s.a = a;
    const double ia = rcp(a), ia3 = ia * ia * ia, ia4 = ia3 * ia;
    double a2 = a * a;
    s.rg = tb.rt_g0 * ia4;
    s.rur = tb.rt_ur0 * ia4;
    s.rc = tb.rt_c0 * ia3;
    s.rb = tb.rt_b0 * ia3;
    double rho = s.rg + s.rur + s.rc + s.rb + tb.rt_L;
    double pr = (s.rg + s.rur) * (1.0 / 3.0) - tb.rt_L;
    s.am = a * tb.m_over_T;
    s.pn4 = tb.pref_ncdm * ia4;
    if (MNU && p.nq > 0) {  // App. C massive neutrinos, eq. mnu_sum
        double sr = 0.0, sp = 0.0;
        for (int i = 0; i < p.nq; ++i) {
            const double q = tb.q[i], e = eps_of(q, s.am);
            sr += tb.W[i] * e;
            sp += tb.W[i] * q * q * rcp(e);
        }
        rho += s.pn4 * sr;
        pr += s.pn4 * sp * (1.0 / 3.0);
    }
    s.Hc = a * sqrt(rho);
    s.Hcp = s.Hc * (1.0 - 1.5 * (rho + pr) * rcp(rho));
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
    s.invHc = rcp(s.Hc);
    s.kH = k * s.invHc;
    s.k2H = k * s.kH;
    s.T = p.thom * s.dk * s.invHc;
    s.R = (4.0 / 3.0) * s.rg * rcp(s.rb);
    s.trunc = s.invHc * rcp(s.tau);
    double ih2 = s.invHc * s.invHc;
    s.cH1 = p.grav * 2.0 * k * k * ih2;
    s.cH2 = p.grav * 3.0 * a2 * ih2;
    s.cE = p.grav * 1.5 * a2 * s.invHc * rcp(k * k);
}

// Row layout: [F chain | G chain | nu chain | one Psi chain per momentum node |
// delta_c, eta, delta_g], padded.
struct Lay {
    int N, nF, nG, nV, nQ, nPs, bG, bV, bM, rDC, rETA, rDG, nch;
};
__host__ __device__ inline Lay make_lay(const DevPrec &p) {
    Lay L;
    L.nF = p.lg + 2;
    L.nG = p.lp > 0 ? p.lp + 1 : 0;
    L.nV = p.ln + 1;
    L.nQ = p.nq;
    L.nPs = p.nq > 0 ? p.lq + 1 : 0;
    L.bG = L.nF;
    L.bV = L.nF + L.nG;
    L.bM = L.bV + L.nV;
    L.rDC = L.bM + L.nQ * L.nPs;
    L.rETA = L.rDC + 1;
    L.rDG = L.rDC + 2;
    L.N = L.rDC + 3;
    L.nch = (L.nG ? 3 : 2) + L.nQ;
    return L;
}

// A multipole chain: type (0 photon temperature + baryons, 1 photon
// polarisation, 2 massless neutrinos, 3 massive neutrinos at node iq), first
// row and length.
struct Chain {
    int ty, cb, cn, iq;
};
// chain number ch (0 .. nch-1) in row order
__device__ inline Chain chain_by_index(int ch, const Lay &L) {
    const int n0 = L.nG ? 3 : 2;
    if (ch == 0) return Chain{0, 0, L.nF, 0};
    if (ch == 1 && L.nG) return Chain{1, L.bG, L.nG, 0};
    if (ch < n0) return Chain{2, L.bV, L.nV, 0};
    const int iq = ch - n0;
    return Chain{3, L.bM + iq * L.nPs, L.nPs, iq};
}
// chain of a row (false for the isolated rows and the padding)
__device__ inline bool chain_of(int row, const Lay &L, Chain &c) {
    if (row < L.bG) c = Chain{0, 0, L.nF, 0};
    else if (row < L.bV) c = Chain{1, L.bG, L.nG, 0};
    else if (row < L.bM) c = Chain{2, L.bV, L.nV, 0};
    else if (row < L.rDC) {
        const int iq = (row - L.bM) / L.nPs;
        c = Chain{3, L.bM + iq * L.nPs, L.nPs, iq};
    } else
        return false;
    return true;
}

struct RowCo {
    double a, d, c, uH, uE, uP;
};

// y'_row = a y_{row-1} + d y_row + c y_{row+1} + uH h' + uE eta' + uP Pi
// (chain rows; for the isolated rows only the coupling terms are used and
// the delta_g leaf term of the theta_g row is added by the caller).
__device__ RowCo row_coef(int row, const Lay &L, const Bk &s, const DevPrec &p, const DevTab &tb) {
    RowCo r{0, 0, 0, 0, 0, 0};
    Chain cs;
    if (!chain_of(row, L, cs)) {
        if (row == L.rDC) r.uH = -0.5;
        if (row == L.rETA) r.uE = 1.0;
        if (row == L.rDG) r.uH = -2.0 / 3.0;
        return r;
    }
    const int ch = cs.ty, j = row - cs.cb, n = cs.cn;
    if (ch == 3) {  // massive neutrinos at node q (App. C), speed v = q k / (eps Hc)
        const double q = tb.q[cs.iq], v = q * s.kH / eps_of(q, s.am), dl = dlnf0(q);
        if (j == n - 1) {
            r.a = v;
            r.d = -(j + 1.0) * s.trunc;
        } else if (j == 0) {
            r.c = -v;
            r.uH = dl / 6.0;
        } else if (j == 1) {
            r.a = v / 3.0;
            r.c = -2.0 * v / 3.0;
        } else if (j == 2) {
            r.a = 0.4 * v;
            r.c = -0.6 * v;
            r.uH = -dl / 15.0;
            r.uE = -0.4 * dl;
        } else {
            r.a = j / (2.0 * j + 1.0) * v;
            r.c = -(j + 1.0) / (2.0 * j + 1.0) * v;
        }
        return r;
    }
    // generic multipole row: l from the chain, Thomson damping for photons
    int l = (ch == 0) ? j - 1 : j;
    bool thom = ch != 2;
    int low = (ch == 0) ? 4 : (ch == 1 ? 0 : 3);  // first row of the generic form
    if (j >= low) {
        double f2 = (l == 3 && ch != 1) ? 2.0 : 1.0;  // F_2 = 2 sigma
        double damp = thom ? -s.T : 0.0;
        if (j == n - 1) {
            r.a = f2 * s.kH;
            r.d = -(l + 1.0) * s.trunc + damp;
        } else {
            double w = s.kH / (2.0 * l + 1.0);
            r.a = f2 * l * w;
            r.d = damp;
            r.c = -(l + 1.0) * w;
            if (ch == 1 && l == 0) r.uP = 0.5 * s.T;
            if (ch == 1 && l == 2) r.uP = 0.1 * s.T;
        }
        return r;
    }
    if (ch == 0) {
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
        } else {
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
        }
    } else {  // neutrinos
        if (j == 0) {
            r.c = -(4.0 / 3.0) * s.invHc;
            r.uH = -2.0 / 3.0;
        } else if (j == 1) {
            r.a = 0.25 * s.k2H;
            r.c = -s.k2H;
        } else {
            r.a = (4.0 / 15.0) * s.invHc;
            r.c = -0.3 * s.kH;
            r.uH = 2.0 / 15.0;
            r.uE = 0.8;
        }
    }
    return r;
}

// LDS of a workgroup: the rows' time-independent multipliers, one table that
// every mode of the wavefront reads (they depend on the hierarchy only), then
// one slab per mode.  A mode's slab holds a record of STR doubles per row
// (16-byte aligned, so neighbouring fields pair into 128-bit accesses): the
// stage rhs / solution, the scaled continuants M_j, M_{j+1} and S_j of the
// upward sweep; after the pivots are formed, the U_j and V_j of the downward
// recurrence replace S_j and M_{j+1} in place.
constexpr int STR = 4;
constexpr int F_RY = 0, F_M = 1, F_MN = 2, F_U = 3;
constexpr int F_V = F_MN;  // V_j of the downward recurrence (U_j in F_U)
// the multipliers table: SST doubles per row (CC and CP adjacent)
constexpr int SST = 4;
constexpr int S_CC = 0, S_CP = 1, S_CA = 2, S_CD = 3;
// record fields free between steps, one per output time of a batch of dense
// outputs (the next step's stages rewrite them before reading them)
constexpr int OUT_SLOTS = STR;
__device__ inline int out_slot(int b) { return b; }
constexpr int PADR = 8;  // spare records before row 0 and after the last row

struct Slab {
    double *base;  // record of row r at base + (r + PADR) * STR
    const double *st;  // multipliers of row r at st + (r + PADR) * SST (shared by the wavefront's modes)
    double *AX;    // exchange area
    double *BK;    // the current step's stage backgrounds, NBK doubles each
    __device__ double *rec(int row) const { return base + (row + PADR) * STR; }
    __device__ const double *sta(int row) const { return st + (row + PADR) * SST; }
    __device__ double &ry(int row) const { return base[(row + PADR) * STR + F_RY]; }
};

// exchange area per mode: couplings (4) and the 4 x 4 top-row affine maps of
// every chain, rounded to an even count (16-byte alignment of the next slab)
__host__ __device__ constexpr int ax_doubles(int nch) { return (4 + 16 * nch + 1) & ~1; }
// one stage's background record (a Bk, padded to an even count)
constexpr int NBK = 24;
static_assert(NBK * sizeof(double) >= sizeof(Bk), "a stage record holds a Bk");
// doubles of LDS per mode for NP rows: records, exchange area, the
// backgrounds of the implicit stages, and two spare doubles.  The spare
// doubles skew consecutive slabs of a wavefront across the LDS banks: with
// eight slabs per wavefront an unpadded 556-double slab put the same record
// of several slabs in one bank group (0.97 conflict cycles per conflict-free
// LDS cycle at C1 batch 32), and a pad of 2 (mod 8) doubles took the batch's
// perturbation kernel from 127.9 to 122.0 ms (a pad of 4 (mod 8) made it
// slower; the results are the same bits).
__host__ __device__ constexpr int slab_doubles(int NP, int nch) {
    return (NP + 2 * PADR) * STR + ax_doubles(nch) + (NSTG - 1) * NBK + 2;
}
// doubles of the shared multipliers table for NP rows
__host__ __device__ constexpr int stat_doubles(int NP) { return (NP + 2 * PADR) * SST; }

// Time-independent multipliers of a generic chain row (fifth row of its chain
// onward): a = CA v, c = CC v, d = CD trunc - T (photon chains) or CD trunc,
// with the chain's streaming rate v = kH (massive node: q kH / eps),
// and CP = -CC_j CA_{j+1} >= 0, so that -c_j a_{j+1} = (kH)^2 CP_j.  The first
// four rows of each chain and the isolated rows get zeros; their entries come
// from the full row formulas (top_coef).
__device__ void row_static1(int row, const Lay &L, double &ca, double &cc, double &cd) {
    ca = cc = cd = 0.0;
    Chain cs;
    if (!chain_of(row, L, cs)) return;
    const int ch = cs.ty, j = row - cs.cb, n = cs.cn;
    if (j < 4) return;
    const int l = (ch == 0) ? j - 1 : j;
    // the l = 2 neighbour of a photon-temperature or massless-neutrino l = 3 row is sigma = F_2 / 2
    const double f2 = (l == 3 && (ch == 0 || ch == 2)) ? 2.0 : 1.0;
    if (j == n - 1) {
        ca = f2;
        cd = -(l + 1.0);
    } else {
        ca = f2 * l / (2.0 * l + 1.0);
        cc = -(l + 1.0) / (2.0 * l + 1.0);
    }
}

__device__ void row_static(int row, const Lay &L, double &ca, double &cc, double &cd, double &cp) {
    row_static1(row, L, ca, cc, cd);
    double ca1, cc1, cd1;
    row_static1(row + 1, L, ca1, cc1, cd1);
    cp = (cc != 0.0) ? -cc * ca1 : 0.0;  // cc != 0 only when row + 1 is in the same chain
}

// Entries of the first four rows (j = 0..3) of chain type ty (0 photon T +
// baryons, 1 photon polarisation, 2 massless neutrinos, 3 massive neutrinos at
// one momentum node), in the form of row_coef, evaluated for every type and
// selected without branching.
template <bool MNU>
__device__ inline RowCo top_coef(int ty, int j, const Lay &L, const Bk &s, const DevPrec &p, double vq, double dl) {
    RowCo f{0, 0, 0, 0, 0, 0}, gp{0, 0, 0, 0, 0, 0}, v{0, 0, 0, 0, 0, 0}, m{0, 0, 0, 0, 0, 0};
    if (j == 0) {
        f.c = -s.invHc;
        f.uH = -0.5;
        v.c = -(4.0 / 3.0) * s.invHc;
        v.uH = -2.0 / 3.0;
    } else if (j == 1) {
        f.a = s.cs2 * s.k2H;
        f.d = -1.0 - s.R * s.T;
        f.c = s.R * s.T;
        v.a = 0.25 * s.k2H;
        v.c = -s.k2H;
    } else if (j == 2) {
        f.a = s.T;
        f.d = -s.T;
        f.c = -s.k2H;
        v.a = (4.0 / 15.0) * s.invHc;
        v.c = -0.3 * s.kH;
        v.uH = 2.0 / 15.0;
        v.uE = 0.8;
    } else {
        f.a = (4.0 / 15.0) * s.invHc;
        f.c = -0.3 * s.kH;
        f.uH = 2.0 / 15.0;
        f.uE = 0.8;
        f.d = p.lp > 0 ? -s.T : -0.9 * s.T;
        f.uP = p.lp > 0 ? 0.05 * s.T : 0.0;
        // neutrino l = 3 (its l = 2 neighbour is sigma = F_2 / 2)
        const bool vlast = L.nV == 4;
        v.a = vlast ? 2.0 * s.kH : (6.0 / 7.0) * s.kH;
        v.c = vlast ? 0.0 : -(4.0 / 7.0) * s.kH;
        v.d = vlast ? -4.0 * s.trunc : 0.0;
    }
    {  // polarisation, l = j
        const double l = j;
        const bool last = j == L.nG - 1;
        gp.a = last ? s.kH : l / (2.0 * l + 1.0) * s.kH;
        gp.c = last ? 0.0 : -(l + 1.0) / (2.0 * l + 1.0) * s.kH;
        gp.d = last ? -s.T - (l + 1.0) * s.trunc : -s.T;
        gp.uP = (j == 0) ? 0.5 * s.T : (j == 2 ? 0.1 * s.T : 0.0);
    }
    if (MNU) {  // massive neutrinos at one node: rate vq = q kH / eps, dl = dln f0/dln q
        const bool last = j == L.nPs - 1;
        if (j == 0) {
            m.c = -vq;
            m.uH = dl * (1.0 / 6.0);
        } else if (j == 1) {
            m.a = vq * (1.0 / 3.0);
            m.c = vq * (-2.0 / 3.0);
        } else if (j == 2) {
            m.a = 0.4 * vq;
            m.c = -0.6 * vq;
            m.uH = dl * (-1.0 / 15.0);
            m.uE = -0.4 * dl;
        } else {
            m.a = last ? vq : (3.0 / 7.0) * vq;
            m.c = last ? 0.0 : -(4.0 / 7.0) * vq;
            m.d = last ? -4.0 * s.trunc : 0.0;
        }
    }
    auto sel = [&](double a0, double a1, double a2, double a3) {
        return ty == 0 ? a0 : (ty == 1 ? a1 : ((!MNU || ty == 2) ? a2 : a3));
    };
    RowCo r;
    r.a = sel(f.a, gp.a, v.a, m.a);
    r.d = sel(f.d, gp.d, v.d, m.d);
    r.c = sel(f.c, gp.c, v.c, m.c);
    r.uH = sel(f.uH, gp.uH, v.uH, m.uH);
    r.uE = sel(f.uE, gp.uE, v.uE, m.uE);
    r.uP = sel(f.uP, gp.uP, v.uP, m.uP);
    return r;
}

// Massive-neutrino moments of a state held in the records (App. B.3 eq.
// mnu_sum): delta rho, (rho + p) theta and (rho + p) sigma, in the units of rt.
__device__ inline void ncdm_moments(const Slab &m, const Lay &L, const Bk &s, const DevTab &tb, double k,
                                    double &drho, double &rpt, double &rps, int fld = F_RY) {
    drho = rpt = rps = 0.0;
    for (int i = 0; i < L.nQ; ++i) {
        const double q = tb.q[i], e = eps_of(q, s.am), w = s.pn4 * tb.W[i];
        const int b = L.bM + i * L.nPs;
        drho += w * e * m.rec(b)[fld];
        rpt += w * k * q * m.rec(b + 1)[fld];
        rps += w * (2.0 / 3.0) * q * q / e * m.rec(b + 2)[fld];
    }
}

// Couplings (h', eta', Pi) from the state rows held in RY (App. B.3, eqs.
// hprime and etaprime).
__device__ void aux_from_rows(const Slab &m, const Lay &L, const Bk &s, const DevPrec &p, const DevTab &tb,
                              double k, double &H, double &E, double &P) {
    auto y = [&](int r) { return m.ry(r); };
    double drho, rpt, rps;
    ncdm_moments(m, L, s, tb, k, drho, rpt, rps);
    // explicit fused multiply-adds: the rounding must not depend on how the
    // compiler contracts the sums where this is inlined (the launch shapes of
    // the kernel compile it in different contexts and must agree bit for bit)
    double dr = fma(s.rc, y(L.rDC), fma(s.rb, y(0), fma(s.rg, y(L.rDG), fma(s.rur, y(L.bV), drho))));
    H = fma(s.cH1, y(L.rETA), s.cH2 * dr);
    double th = fma(s.rb, y(1), fma((4.0 / 3.0) * s.rg, y(2), fma((4.0 / 3.0) * s.rur, y(L.bV + 1), rpt)));
    E = s.cE * th;
    P = (p.lp > 0) ? 2.0 * y(3) + y(L.bG) + y(L.bG + 2) : 0.0;
}

// Adiabatic growing mode at leading order in k tau (Ma & Bertschinger 1995,
// eqs. 96 and 97), normalised so that eta -> 1: the initial value of state
// row `row` from the background s at the start time.
template <bool MNU>
__device__ __attribute__((always_inline)) double ic_row(int row, const Lay &L, const Bk &s, const DevTab &tb,
                                                        double k) {
    const double x = k * s.tau, Rn = tb.R_nu;
    const double dg = -x * x / 3.0, tg = -k * x * x * x / 36.0;
    double v = 0.0;
    if (row == 0) v = 0.75 * dg;
    if (row == 1 || row == 2) v = tg;
    if (row == L.bV) v = dg;
    if (row == L.bV + 1) v = (23.0 + 4.0 * Rn) / (15.0 + 4.0 * Rn) * tg;
    if (row == L.bV + 2) v = 2.0 / (3.0 * (15.0 + 4.0 * Rn)) * x * x;
    if (row == L.rDC) v = 0.75 * dg;
    if (row == L.rDG) v = dg;
    if (row == L.rETA) v = 1.0 - (5.0 + 4.0 * Rn) / (12.0 * (15.0 + 4.0 * Rn)) * x * x;
    if (MNU && row >= L.bM && row < L.rDC) {  // massive nu from the massless moments via dln f0/dln q
        const int iq = (row - L.bM) / L.nPs, j = row - L.bM - iq * L.nPs;
        const double q = tb.q[iq], dl = dlnf0(q);
        const double tn = (23.0 + 4.0 * Rn) / (15.0 + 4.0 * Rn) * tg;
        const double sn = 2.0 / (3.0 * (15.0 + 4.0 * Rn)) * x * x;
        if (j == 0) v = -0.25 * dg * dl;
        if (j == 1) v = -eps_of(q, s.am) / (3.0 * q * k) * tn * dl;
        if (j == 2) v = -0.5 * sn * dl;
    }
    return v;
}

// The CMB source functions S_T0, S_T1, S_T2 (App. B.4, eq. source_functions)
// at one output time from the state rows y(row), the background `so` there and
// the massive-neutrino moments (zero without them); alpha' from the traceless
// Einstein equation.
template <class Y>
__device__ __attribute__((always_inline)) void source_values(const Bk &so, const Lay &L, const DevPrec &p, double k,
                                                             Y y, double drho, double rpt, double rpsn, double &S0,
                                                             double &S1, double &S2) {
    double k2 = k * k;
    double Hh = so.cH1 * y(L.rETA) + so.cH2 * (so.rc * y(L.rDC) + so.rb * y(0) + so.rg * y(L.rDG) +
                                               so.rur * y(L.bV) + drho);
    double Ee = so.cE * (so.rb * y(1) + (4.0 / 3.0) * so.rg * y(2) + (4.0 / 3.0) * so.rur * y(L.bV + 1) + rpt);
    double tbp = so.cs2 * so.k2H * y(0) + (-1.0 - so.R * so.T) * y(1) + so.R * so.T * y(2);
    double ek = exp(-so.kap);
    double gv = so.dk * ek;
    double gp = (so.dkp + so.dk * so.dk * so.invHc) * ek;
    double Hc = so.Hc;
    double alpha = Hc * (Hh + 6.0 * Ee) / (2.0 * k2);
    double rps = (4.0 / 3.0) * (so.rg * y(3) + so.rur * y(L.bV + 2)) + rpsn;
    double alphap = -2.0 * alpha + (y(L.rETA) - 4.5 * so.a * so.a * rps / k2) * so.invHc;
    double Pi = 2.0 * y(3) + (L.nG ? y(L.bG) + y(L.bG + 2) : 0.0);
    double eta = y(L.rETA);
    S0 = p.sw * gv * (0.25 * y(L.rDG) + Hc * alphap) +
         p.isw * (gv * (eta - Hc * alphap - 2.0 * Hc * alpha) + 2.0 * Hc * ek * (Ee - so.Hcp * alpha - Hc * alphap)) +
         p.dop * Hc * (gv * (tbp / k2 + alphap) + gp * (y(1) / k2 + alpha));
    S1 = p.isw * ek * k * (Hc * alphap + 2.0 * Hc * alpha - eta);
    S2 = gv * Pi * 0.125;
}

template <int R>
struct Rows {
    double y[R], yn[R], K[NSTG][R], rr[R];
};

// f = A y for this lane's rows; y already in the records (all rows), couplings in AX[0..2].
// (explicit fused multiply-adds throughout, so that every launch shape rounds
// alike wherever the compiler places this code)
template <int R>
__device__ __attribute__((always_inline)) void rhs_rows(const Slab &m, const Lay &L, const Bk &s, const DevPrec &p,
                                                        const DevTab &tb, int gl, double *f) {
    double H = m.AX[0], E = m.AX[1], P = m.AX[2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int row = gl * R + r;
        double v = 0.0;
        if (row < L.N) {
            RowCo c = row_coef(row, L, s, p, tb);
            Chain cs;
            if (chain_of(row, L, cs)) {
                double ym = row > cs.cb ? m.ry(row - 1) : 0.0;
                double yp = row + 1 < cs.cb + cs.cn ? m.ry(row + 1) : 0.0;
                v = fma(c.c, yp, fma(c.d, m.ry(row), c.a * ym));
                if (row == 2) v = fma(0.25 * s.k2H, m.ry(L.rDG), v);
            } else if (row == L.rDG) {
                v = (-(4.0 / 3.0) * s.invHc) * m.ry(2);
            }
            v = fma(c.uP, P, fma(c.uE, E, fma(c.uH, H, v)));
        }
        f[r] = v;
    }
}

struct Aff {
    double v0, vH, vE, vP;
};

__device__ inline double aff(const Aff &a, double H, double E, double P) { return a.v0 + a.vH * H + a.vE * E + a.vP * P; }

// Transposed source functions at one point (reverse mode of App. B.4, eq.
// source_functions, with respect to the state): dL/dS_T0, dL/dS_T1, dL/dS_T2
// at output time j of mode ik added into G (the N state rows).  The sources
// are linear in the state at a fixed time (theta_b' enters through the
// baryon row of the right-hand side, h' and eta' through the Einstein
// constraints), so this is the transpose of that linear map, written from the
// source formulas in reverse order.
template <bool MNU>
__device__ void sources_adj_point(const DevTab &tb, const DevPrec &p, const Lay &L, int n_tau, int ik, int j,
                                  const double *__restrict__ gs, double *G) {
    const double lna = tb.lna_src[j];
    if (lna < tb.lna_start[ik]) return;  // no sources before the mode starts
    const double k = tb.k[ik], k2 = k * k;
    const double g0 = gs[j], g1 = gs[n_tau + j], g2 = gs[2 * n_tau + j];
    Bk so;
    bk_at<MNU>(tb, p, k, lna, so);
    const double Hc = so.Hc, ek = exp(-so.kap), gv = so.dk * ek;
    const double gp = (so.dkp + so.dk * so.dk * so.invHc) * ek;
    // adjoints of the intermediate quantities of the forward formulas
    double a_alphap = g0 * (p.sw * gv * Hc - p.isw * gv * Hc - 2.0 * p.isw * Hc * ek * Hc + p.dop * Hc * gv) +
                      g1 * p.isw * ek * k * Hc;
    double a_alpha = g0 * (-2.0 * p.isw * gv * Hc - 2.0 * p.isw * Hc * ek * so.Hcp + p.dop * Hc * gp) +
                     g1 * 2.0 * p.isw * ek * k * Hc;
    const double a_eta = g0 * p.isw * gv - g1 * p.isw * ek * k;
    double a_Ee = g0 * 2.0 * p.isw * Hc * ek;
    const double a_tbp = g0 * p.dop * Hc * gv / k2;
    const double a_Pi = g2 * 0.125 * gv;
    G[1] += g0 * p.dop * Hc * gp / k2;
    G[L.rDG] += g0 * p.sw * gv * 0.25;
    // alpha' = -2 alpha + (eta - 4.5 a^2 rps / k^2) / Hc
    a_alpha += -2.0 * a_alphap;
    G[L.rETA] += a_alphap * so.invHc + a_eta;
    const double a_rps = -a_alphap * 4.5 * so.a * so.a * so.invHc / k2;
    // alpha = Hc (h' + 6 eta') / (2 k^2), with h' = Hh and eta' = Ee below
    const double a_Hh = a_alpha * Hc / (2.0 * k2);
    a_Ee += a_alpha * 6.0 * Hc / (2.0 * k2);
    // (rho + p) sigma, the anisotropic stress
    G[3] += a_rps * (4.0 / 3.0) * so.rg + 2.0 * a_Pi;
    G[L.bV + 2] += a_rps * (4.0 / 3.0) * so.rur;
    if (L.nG) {
        G[L.bG] += a_Pi;
        G[L.bG + 2] += a_Pi;
    }
    // theta_b' of the right-hand side
    G[0] += a_tbp * so.cs2 * so.k2H;
    G[1] += a_tbp * (-1.0 - so.R * so.T);
    G[2] += a_tbp * so.R * so.T;
    // eta' constraint
    G[1] += a_Ee * so.cE * so.rb;
    G[2] += a_Ee * so.cE * (4.0 / 3.0) * so.rg;
    G[L.bV + 1] += a_Ee * so.cE * (4.0 / 3.0) * so.rur;
    // h' constraint
    G[L.rETA] += a_Hh * so.cH1;
    G[L.rDC] += a_Hh * so.cH2 * so.rc;
    G[0] += a_Hh * so.cH2 * so.rb;
    G[L.rDG] += a_Hh * so.cH2 * so.rg;
    G[L.bV] += a_Hh * so.cH2 * so.rur;
    // massive neutrinos: delta rho, (rho + p) theta, (rho + p) sigma of every node
    for (int i = 0; i < (MNU ? L.nQ : 0); ++i) {
        const double q = tb.q[i], e = eps_of(q, so.am), w = so.pn4 * tb.W[i];
        const int b = L.bM + i * L.nPs;
        G[b] += a_Hh * so.cH2 * w * e;
        G[b + 1] += a_Ee * so.cE * w * k * q;
        G[b + 2] += a_rps * w * (2.0 / 3.0) * q * q / e;
    }
}

}  // namespace

// Rows per lane and group size for a hierarchy of N rows: R = 5 and the
// smallest power-of-two group holding the rows (at most one wavefront).
inline void group_shape(const DevPrec &p, int &R, int &G) {
    int N = (p.lg + 2) + (p.lp > 0 ? p.lp + 1 : 0) + (p.ln + 1) + p.nq * (p.nq > 0 ? p.lq + 1 : 0) + 3;
    const int nch = (p.lp > 0 ? 3 : 2) + p.nq;  // one sweeping lane per chain
    R = (N <= 32) ? 2 : 5;
    int need = (N + R - 1) / R;
    if (need < nch) need = nch;
    G = 4;
    while (G < need) G <<= 1;
}

}  // namespace cmbhip
