// Reverse sweep of the perturbation kernel (K1): the discrete adjoint of its
// ESDIRK integration with frozen steps, segment by segment from the step
// trajectories a replay writes (App. A.2 integrator adjoint option; section 3
// of arXiv 2602.15104).
#include <hip/hip_runtime.h>

#include <string>

#include "k1_common.h"

namespace cmbhip {

namespace {

// ---------------------------------------------------------------------------
// Reverse sweep: the discrete adjoint of the ESDIRK integration with frozen
// steps (section 3 and the integrator's adjoint option, App. A.2), one group
// of G lanes per mode as in the forward kernel.
//
// A step n maps (y_n, K_0) to y_{n+1} = Y_5 through the stages
//   R_s = y_n + h sum_{j<s} a_sj K_j,  (I - g A_s) Y_s = R_s,  K_s = A_s Y_s,
// g = h gamma, A_s = A(t_n + c_s h); K_0 is the previous step's K_5, and the
// dense output y(t_o) = h00 y_n + h10 hh K_0 + h01 Y_5 + h11 hh K_5 gives the
// sources.  Backwards, with ybar = dL/dy_n, Kbar_j = dL/dK_j:
//   Ybar_s = [s = 5: dL/dy_{n+1}] + A_s^T Kbar_s,   Rbar_s = (I - g A_s)^-T Ybar_s,
//   ybar += Rbar_s,  Kbar_j += h a_sj Rbar_s (j < s),
// and the matrix A_s itself, through the tables and the background, carries
// dL/dA_s = (Kbar_s + g Rbar_s) Y_s^T.  Its dependence on the parameters
// theta_p is taken from central differences of A_s Y_s between the tables
// built at theta_p (1 +- eps) (the host's table tangents), contracted with
// (Kbar_s + g Rbar_s); so are the sources' own dependence at fixed state and
// the initial conditions'.
//
// The transposed stage matrix has the forward one's structure: the chains'
// tridiagonal blocks transposed (a row's sub-diagonal is the previous row's
// super-diagonal), and the rank-three coupling A = B + u_H w_H^T + u_E w_E^T
// + u_P w_P^T with the roles of u (how h', eta', Pi enter each row) and w
// (how each row enters h', eta', Pi) exchanged.  It is solved as the forward
// one is: each chain eliminated upwards from its highest multipole, its top
// four rows as affine maps of the three coupling unknowns
// zeta = (u_H.x, u_E.x, u_P.x), a 3 x 3 system for zeta, then substitution
// downwards.  The elimination divides by pivots that are those of the
// forward continuants (a transposed tridiagonal block has the same ones),
// all >= 1.
//
// Per mode and launch: the steps of one segment, in reverse, read from the
// step trajectory a segment replay of the forward kernel wrote; the running
// adjoint (dL/dy, dL/dK_0) and the parameter accumulators carry from one
// segment's launch to the previous one's in global memory.

constexpr int NAF = 4;  // adjoint fields per row: right-hand side, solution, elimination U and V
constexpr int AF_B = 0, AF_X = 1, AF_U = 2, AF_V = 3;
// per-row flags of a lane's rows (bit positions)
constexpr unsigned RI_VALID = 1u, RI_TOP = 2u, RI_UP = 4u, RI_DN = 8u, RI_TG = 16u, RI_DG = 32u, RI_DC = 64u,
                   RI_ETA = 128u;
constexpr int RI_WH = 8, RI_WE = 11, RI_WP = 13;
constexpr int NPAR = 4;  // parameters with table tangents: h, omega_b, omega_cdm, tau_reio
// stage backgrounds kept per mode: the 2 NPAR perturbed tables' (slot q) and
// the mode's own (slot 2 NPAR)
constexpr int NBKS = 2 * NPAR + 1;
// record fields (free in the reverse kernel) that cache the current stage's
// chain coefficients of each row: y'_row = a y_{row-1} + d y_row + c y_{row+1} + ...
constexpr int F_A = F_M, F_D = F_MN, F_C = F_U;

// The entries of a chain's top rows and of the isolated rows are linear in
// eight background quantities, the bases 1, 1/Hc, kH, k^2/Hc, T, R T,
// c_s^2 k^2/Hc and the truncation rate (and u_P is T times a constant).  A
// table per wavefront holds, for each such row, the multiplier of every
// basis in its entries a, d, c, and its u_H, u_E and u_P / T; it is filled
// once from the row formulas themselves, at unit backgrounds.
constexpr int NBAS = 8;
constexpr int TBLW = 3 * NBAS + 4;  // a, d, c per basis; u_H, u_E, u_P / T; spare
__device__ inline void bases_of(const Bk &s, double *v) {
    v[0] = 1.0;
    v[1] = s.invHc;
    v[2] = s.kH;
    v[3] = s.k2H;
    v[4] = s.T;
    v[5] = s.R * s.T;
    v[6] = s.cs2 * s.k2H;
    v[7] = s.trunc;
}
// rows of the table: four top rows per chain, then delta_c, eta, delta_g
__host__ __device__ constexpr int top_rows(int nch) { return 4 * nch + 3; }

// how a row enters the couplings: h' = w_H . y, eta' = w_E . y, Pi = w_P . y
// (App. B.3, eqs. hprime and etaprime; Pi = 2 sigma_gamma + G_0 + G_2)
__device__ inline void w_row(int row, const Lay &L, const Bk &s, const DevPrec &p, double &wH, double &wE, double &wP) {
    wH = wE = wP = 0.0;
    if (row == L.rETA) wH = s.cH1;
    if (row == L.rDC) wH = s.cH2 * s.rc;
    if (row == 0) wH = s.cH2 * s.rb;
    if (row == L.rDG) wH = s.cH2 * s.rg;
    if (row == L.bV) wH = s.cH2 * s.rur;
    if (row == 1) wE = s.cE * s.rb;
    if (row == 2) wE = s.cE * (4.0 / 3.0) * s.rg;
    if (row == L.bV + 1) wE = s.cE * (4.0 / 3.0) * s.rur;
    if (p.lp > 0) {
        if (row == 3) wP = 2.0;
        if (row == L.bG || row == L.bG + 2) wP = 1.0;
    }
}

// doubles of LDS per mode of the reverse kernel: the records of the forward
// kernel's slab and its exchange area, the adjoint fields of every row, one
// vector of NP rows (the forcing at an output), the stage backgrounds and
// dL/dK_j of every stage and row (each lane only touches its own rows there).
// The workgroup's LDS starts with the shared multipliers table.
// the forcing vector's area also holds, during the stages, the parameter
// contraction's per-parameter differences (NPAR x (NBAS + 2) doubles)
__host__ __device__ constexpr int gv_doubles(int NP) { return NP > NPAR * (NBAS + 2) ? NP : NPAR * (NBAS + 2); }
__host__ __device__ constexpr int adj_slab_doubles(int NP, int nch) {
    return (NP + 2 * PADR) * STR + ax_doubles(nch) + (NP + 2 * PADR) * NAF + gv_doubles(NP) + NBKS * NBK + NSTG * NP;
}
__host__ __device__ constexpr int adj_lds_doubles(int NP, int nch, int spw) {
    return stat_doubles(NP) + top_rows(nch) * TBLW + spw * adj_slab_doubles(NP, nch);
}

template <int R>
struct AdjRows {
    double y[R];    // the step's start state
    double yb[R];   // dL/dy_n being accumulated
    double Y5b[R];  // dL/dy_{n+1} (seed of the last stage)
};

template <int R>
__global__ void __launch_bounds__(64) adjoint_kernel(const DevTab *__restrict__ tabs, const DevTab *__restrict__ ptabs,
                                                     const double *__restrict__ pden, int n_cosmo, int n_k, int n_tau,
                                                     DevPrec p, int G, const double *__restrict__ traj, int traj_cap,
                                                     const int *__restrict__ hist_n, int seg, int every,
                                                     const double *__restrict__ gS, double *__restrict__ lam,
                                                     double *__restrict__ grad, int first) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int gl = lane % G;
    const int grp = lane / G;
    const int spw = 64 / G;
    const int n_sys = n_cosmo * n_k;
    const int lin = blockIdx.x * spw + grp;
    const Lay L = make_lay(p);
    const int NP = G * R;
    const int N = L.N;
    const int TR = traj_rec(N);
    Slab m;
    double *af, *gv, *bks, *kbb;
    double *const tbl = lds + stat_doubles(NP);  // the top rows' basis multipliers (shared)
    {
        double *stat = lds;
        double *base = lds + stat_doubles(NP) + top_rows(L.nch) * TBLW + (size_t)grp * adj_slab_doubles(NP, L.nch);
        m.base = base;
        m.st = stat;
        m.AX = base + (NP + 2 * PADR) * STR;
        m.BK = nullptr;  // the forward kernel's stage records are not used here
        af = m.AX + ax_doubles(L.nch);
        gv = af + (NP + 2 * PADR) * NAF;
        bks = gv + gv_doubles(NP);
        kbb = bks + NBKS * NBK;
        for (int i = gl; i < adj_slab_doubles(NP, L.nch); i += G) base[i] = 0.0;
        for (int i = gl; i < stat_doubles(NP); i += G) stat[i] = 0.0;
        wsync();
        // the rows' time-independent multipliers (every group writes the same values)
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            double ca, cc, cd, cp;
            row_static(row, L, ca, cc, cd, cp);
            double *q = stat + (row + PADR) * SST;
            q[S_CA] = ca;
            q[S_CC] = cc;
            q[S_CD] = cd;
            q[S_CP] = cp;
        }
        wsync();
    }
    if (lin >= n_sys) return;
    const int c = lin % n_cosmo, ik = lin / n_cosmo;
    const DevTab &tb = tabs[c];
    const double k = tb.k[ik];
    auto afr = [&](int row) { return af + (row + PADR) * NAF; };
    // dL/dK_j of this lane's row r
    auto kbr = [&](int j, int r) __attribute__((always_inline)) -> double & { return kbb[j * NP + gl * R + r]; };
    auto group_sum = [&](double v) __attribute__((always_inline)) {
        v += dpp_f64<0xB1>(v);
        v += dpp_f64<0x4E>(v);
        if (G >= 8) v += dpp_f64<0x141>(v);
        if (G >= 16) v += dpp_f64<0x140>(v);
        for (int o = 16; o < G; o <<= 1) v += __shfl_xor(v, o, G);
        return v;
    };
    const size_t mode = (size_t)c * n_k + ik;
    double *lm = lam + mode * 2 * N;  // dL/dy and dL/dK_0 carried between segments
    double *gr = grad + mode * NPAR;
    const double *den = pden + (size_t)c * NPAR;  // 2 eps theta_p of each parameter
    // tables at theta_p (1 + eps) (q = 2 p) and theta_p (1 - eps) (q = 2 p + 1),
    // one set of n_cosmo per q
    auto pt = [&](int q) -> const DevTab & { return ptabs[(size_t)q * n_cosmo + c]; };
    double acc[NPAR] = {0.0, 0.0, 0.0, 0.0};  // this lane's share of dL/dtheta_p

    // this lane's rows: generic chain rows (fifth of their chain onward, whose
    // entries are multipliers of kH and trunc, and -T on the photon chains)
    // and the rest (the chains' top rows and the isolated rows)
    unsigned gen = 0, pho = 0;
    // and per row what the stage code asks of the layout, found once here:
    // inside the matrix, a chain's top row, the chain neighbours above and
    // below, the theta_g / delta_g link rows, and how the row enters the
    // couplings (which factor of h' = w_H . y, eta' = w_E . y, Pi = w_P . y,
    // as w_row states them)
    unsigned rinfo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = gl * R + r;
        unsigned f = 0;
        Chain cs;
        if (row < N) {
            f |= RI_VALID;
            if (chain_of(row, L, cs)) {
                if (row - cs.cb >= 4) gen |= 1u << r;
                else f |= RI_TOP;
                if (cs.ty <= 1) pho |= 1u << r;
                if (row > cs.cb) f |= RI_UP;
                if (row + 1 < cs.cb + cs.cn) f |= RI_DN;
            }
            if (row == 2) f |= RI_TG;
            if (row == L.rDG) f |= RI_DG;
            if (row == L.rDC) f |= RI_DC;
            if (row == L.rETA) f |= RI_ETA;
            unsigned wh = 0, we = 0, wp = 0;
            if (row == L.rETA) wh = 1;
            if (row == L.rDC) wh = 2;
            if (row == 0) wh = 3;
            if (row == L.rDG) wh = 4;
            if (row == L.bV) wh = 5;
            if (row == 1) we = 1;
            if (row == 2) we = 2;
            if (row == L.bV + 1) we = 3;
            if (p.lp > 0) {
                if (row == 3) wp = 2;
                if (row == L.bG || row == L.bG + 2) wp = 1;
            }
            f |= wh << RI_WH | we << RI_WE | wp << RI_WP;
        }
        rinfo[r] = f;
    }
    // w_row of a row from its flags (the same products)
    auto w_of = [&](unsigned f, const Bk &s, double &wH, double &wE, double &wP) __attribute__((always_inline)) {
        const unsigned wh = (f >> RI_WH) & 7u, we = (f >> RI_WE) & 3u, wp = (f >> RI_WP) & 3u;
        wH = wh == 1 ? s.cH1 : wh == 2 ? s.cH2 * s.rc : wh == 3 ? s.cH2 * s.rb : wh == 4 ? s.cH2 * s.rg
                                                                              : wh == 5 ? s.cH2 * s.rur : 0.0;
        wE = we == 1 ? s.cE * s.rb : we == 2 ? s.cE * (4.0 / 3.0) * s.rg : we == 3 ? s.cE * (4.0 / 3.0) * s.rur : 0.0;
        wP = wp == 2 ? 2.0 : wp == 1 ? 1.0 : 0.0;
    };
    // entries of row `row` of A at background s (as row_coef): the multipliers
    // table for generic rows, the top-row formulas otherwise
    auto coef_at = [&](int row, const Bk &s, bool generic, bool photon) __attribute__((always_inline)) {
        RowCo r{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (row >= N) return r;
        if (generic) {
            const double *q = m.sta(row);
            r.a = q[S_CA] * s.kH;
            r.c = q[S_CC] * s.kH;
            r.d = photon ? fma(q[S_CD], s.trunc, -s.T) : q[S_CD] * s.trunc;
            return r;
        }
        Chain cs;
        if (chain_of(row, L, cs)) return top_coef<false>(cs.ty, row - cs.cb, L, s, p, 0.0, 0.0);
        if (row == L.rDC) r.uH = -0.5;
        if (row == L.rETA) r.uE = 1.0;
        if (row == L.rDG) r.uH = -2.0 / 3.0;
        return r;
    };
    // the table row of a chain's top row or an isolated row (-1 otherwise)
    auto top_index = [&](int row) __attribute__((always_inline)) -> int {
        if (row >= N) return -1;
        if (row == L.rDC) return 4 * L.nch;
        if (row == L.rETA) return 4 * L.nch + 1;
        if (row == L.rDG) return 4 * L.nch + 2;
        for (int ch = 0; ch < L.nch; ++ch) {
            const Chain cs = chain_by_index(ch, L);
            if (row >= cs.cb && row < cs.cb + 4 && row < cs.cb + cs.cn) return 4 * ch + (row - cs.cb);
        }
        return -1;
    };
    // fill the table (every group writes the same values)
    for (int idx = gl; idx < top_rows(L.nch); idx += G) {
        int row = -1;
        if (idx >= 4 * L.nch) {
            row = idx == 4 * L.nch ? L.rDC : (idx == 4 * L.nch + 1 ? L.rETA : L.rDG);
        } else {
            const Chain cs = chain_by_index(idx / 4, L);
            if (idx % 4 < cs.cn) row = cs.cb + idx % 4;
        }
        double *e = tbl + idx * TBLW;
        for (int i = 0; i < TBLW; ++i) e[i] = 0.0;
        if (row < 0) continue;
        const Bk z{};
        const RowCo c0 = coef_at(row, z, false, false);
        auto put = [&](int b, const RowCo &hi, const RowCo &lo_) {
            e[b] = hi.a - lo_.a;
            e[NBAS + b] = hi.d - lo_.d;
            e[2 * NBAS + b] = hi.c - lo_.c;
        };
        put(0, c0, RowCo{0.0, 0.0, 0.0, 0.0, 0.0, 0.0});
        e[3 * NBAS] = c0.uH;
        e[3 * NBAS + 1] = c0.uE;
        Bk sb = z;
        sb.invHc = 1.0;
        put(1, coef_at(row, sb, false, false), c0);
        sb = z;
        sb.kH = 1.0;
        put(2, coef_at(row, sb, false, false), c0);
        sb = z;
        sb.k2H = 1.0;
        const RowCo ck = coef_at(row, sb, false, false);
        put(3, ck, c0);
        sb = z;
        sb.T = 1.0;
        const RowCo cT = coef_at(row, sb, false, false);
        put(4, cT, c0);
        e[3 * NBAS + 2] = cT.uP - c0.uP;
        sb.R = 1.0;
        put(5, coef_at(row, sb, false, false), cT);
        sb = z;
        sb.k2H = 1.0;
        sb.cs2 = 1.0;
        put(6, coef_at(row, sb, false, false), ck);
        sb = z;
        sb.trunc = 1.0;
        put(7, coef_at(row, sb, false, false), c0);
    }
    wsync();
    int cidx[R];  // this lane's rows' table rows (-1 for generic rows)
#pragma unroll
    for (int r = 0; r < R; ++r) cidx[r] = ((gen >> r) & 1u) ? -1 : top_index(gl * R + r);

    AdjRows<R> w;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = gl * R + r;
        const bool in = row < N && !first;
        w.Y5b[r] = in ? lm[row] : 0.0;
        kbr(NSTG - 1, r) = in ? lm[N + row] : 0.0;
    }
    const double *lo = tb.lna_src;
    const bool final_seg = seg == 0;
    int nst = hist_n[mode] - seg * every;  // this mode's steps in the segment
    nst = nst < 0 ? 0 : (nst > every ? every : nst);

    // the backgrounds at ln a = tt of the perturbed tables (slots 0 .. 2 NPAR-1)
    // and of the mode's own (slot 2 NPAR), one per lane
    auto stage_bks = [&](double tt) __attribute__((always_inline)) {
        for (int q = gl; q < NBKS; q += G) {
            Bk b;
            bk_at<false>(q < 2 * NPAR ? pt(q) : tb, p, k, tt, b);
            __builtin_memcpy(bks + q * NBK, &b, sizeof(Bk));
        }
        wsync();
    };
    auto bk_ref = [&](int q) __attribute__((always_inline)) -> const Bk & {
        return *reinterpret_cast<const Bk *>(bks + q * NBK);
    };

    // A^T b for this lane's rows, b in AF_B of every row.  Each lane first
    // caches its rows' entries of A at this stage (chain a, d, c in the
    // records, the couplings' u in the adjoint fields; the transposed solve
    // reads them too) and its share of u . b.
    auto apply_t = [&](const Bk &s, double *out) __attribute__((always_inline)) {
        // the chains' top rows (position j static, type per lane): entries into
        // the records, coupling coefficients into the free adjoint fields
        // (U, V, X) for the row lanes
        if (gl < L.nch) {
            const Chain ch = chain_by_index(gl, L);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j >= ch.cn) continue;
                const RowCo cc = top_coef<false>(ch.ty, j, L, s, p, 0.0, 0.0);
                double *q = m.rec(ch.cb + j);
                q[F_A] = cc.a;
                q[F_D] = cc.d;
                q[F_C] = cc.c;
                double *f = afr(ch.cb + j);
                f[AF_U] = cc.uH;
                f[AF_V] = cc.uE;
                f[AF_X] = cc.uP;
            }
        }
        wsync();
        double zH = 0.0, zE = 0.0, zP = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            const unsigned fl = rinfo[r];
            double uH = 0.0, uE = 0.0, uP = 0.0;
            if ((gen >> r) & 1u) {
                const double *q = m.sta(row);
                double *e = m.rec(row);
                e[F_A] = q[S_CA] * s.kH;
                e[F_C] = q[S_CC] * s.kH;
                e[F_D] = ((pho >> r) & 1u) ? fma(q[S_CD], s.trunc, -s.T) : q[S_CD] * s.trunc;
            } else if (fl & RI_TOP) {
                const double *f = afr(row);
                uH = f[AF_U];
                uE = f[AF_V];
                uP = f[AF_X];
            } else {  // isolated rows and padding: no entries
                double *e = m.rec(row);
                e[F_A] = 0.0;
                e[F_D] = 0.0;
                e[F_C] = 0.0;
                if (fl & RI_DC) uH = -0.5;
                if (fl & RI_ETA) uE = 1.0;
                if (fl & RI_DG) uH = -2.0 / 3.0;
            }
            const double v = afr(row)[AF_B];
            zH = fma(uH, v, zH);
            zE = fma(uE, v, zE);
            zP = fma(uP, v, zP);
        }
        zH = group_sum(zH);
        zE = group_sum(zE);
        zP = group_sum(zP);
        wsync();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            const unsigned fl = rinfo[r];
            double v = 0.0;
            if (fl & RI_VALID) {
                v = m.rec(row)[F_D] * afr(row)[AF_B];
                // (A^T)_{row,row-1} = A_{row-1,row} (c of the row above), (A^T)_{row,row+1} = a of the row below
                if (fl & RI_UP) v = fma(m.rec(row - 1)[F_C], afr(row - 1)[AF_B], v);
                if (fl & RI_DN) v = fma(m.rec(row + 1)[F_A], afr(row + 1)[AF_B], v);
                if (fl & RI_TG) v = fma(-(4.0 / 3.0) * s.invHc, afr(L.rDG)[AF_B], v);  // delta_g' = -(4/3) theta_g / Hc ...
                if (fl & RI_DG) v = fma(0.25 * s.k2H, afr(2)[AF_B], v);          // theta_g' = ... + k^2 delta_g / (4 Hc)
                double wH, wE, wP;
                w_of(fl, s, wH, wE, wP);
                v = fma(wH, zH, fma(wE, zE, fma(wP, zP, v)));
            }
            out[r] = v;
        }
    };

    // x = (I - g A)^-T b: b in AF_B of every row, x into AF_X of every row; the
    // entries of A as apply_t cached them at this stage
    auto solve_t = [&](const Bk &s, double g) __attribute__((always_inline)) {
        // (1) chains, one lane each: upward elimination x_j = U_j + V_j x_{j-1};
        // the top four rows' U as affine maps of zeta (constant, H, E, P parts)
        if (gl < L.nch) {
            const Chain ch = chain_by_index(gl, L);
            double U1 = 0.0, V1 = 0.0;  // of the row below
            // top rows 0..3: affine U, and V (zero beyond a chain shorter than four rows)
            double tU[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}, tV[4] = {0, 0, 0, 0};
            // Generic rows cn-1 .. 4 in continuant form, with no division on the
            // dependent path: M_j = piv_j M_{j+1} - g^2 sup_j sub_{j+1} M_{j+2} (the
            // forward solve's pivots: sup_j sub_{j+1} = a_{j+1} c_j <= 0, so every
            // term is non-negative) and Z_j = rhs_j M_{j+1} + g sup_j Z_{j+1}; then
            // U_j = Z_j / M_j and V_j = g sub_j M_{j+1} / M_j, formed here beside
            // the recurrences (the reciprocal is off their dependent path) and the
            // only values stored.  Rows go in blocks of four with the next block's
            // entries in flight; M and Z are rescaled by 2^-332 at the end of a
            // block whenever M passes 2^332 (U and V are ratios: the same bits).
            // Blocks always run whole: rows above the fifth receive values nobody
            // reads, and reads stay within the record pads.
            if (ch.cn > 4) {
                const int cb = ch.cb;
                double M1 = 1.0, M2 = 0.0, Z1 = 0.0;  // M_{j+1}, M_{j+2}, Z_{j+1}
                double aup = 0.0;                     // a_{j+1}: none below the last row
                // entries of rows j0 .. j0-3 (d, c, a, rhs) and c of row j0-4
                struct Blk {
                    double d[4], c[5], a[4], r[4];
                };
                auto load_blk = [&](int j0, Blk &e) __attribute__((always_inline)) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double *rq = m.rec(cb + j0 - q);
                        e.d[q] = rq[F_D];
                        e.c[q] = rq[F_C];
                        e.a[q] = rq[F_A];
                        e.r[q] = afr(cb + j0 - q)[AF_B];
                    }
                    e.c[4] = m.rec(cb + j0 - 4)[F_C];
                };
                auto up_blk = [&](const Blk &e, Blk &nx, int j0) __attribute__((always_inline)) {
                    load_blk(j0 - 4, nx);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double piv = 1.0 - g * e.d[q];
                        const double gs = g * aup;
                        const double M = fma(piv, M1, (-gs * g * e.c[q]) * M2);
                        const double Z = fma(e.r[q], M1, gs * Z1);
                        const double iM = rcp(M);
                        double *f = afr(cb + j0 - q);
                        f[AF_U] = Z * iM;
                        f[AF_V] = g * e.c[q + 1] * M1 * iM;  // sub_j = c_{j-1}
                        M2 = M1;
                        M1 = M;
                        Z1 = Z;
                        aup = e.a[q];
                    }
                    const double sc = M1 > 0x1p332 ? 0x1p-332 : 1.0;
                    M1 *= sc;
                    M2 *= sc;
                    Z1 *= sc;
                };
                Blk e0, e1;
                load_blk(ch.cn - 1, e0);
                int j0 = ch.cn - 1;
                for (; j0 >= 8; j0 -= 8) {
                    up_blk(e0, e1, j0);
                    up_blk(e1, e0, j0 - 4);
                }
                if (j0 >= 4) up_blk(e0, e1, j0);
                // row 4's U and V for the top rows (sub_4 = c_3), as stored above
                U1 = afr(cb + 4)[AF_U];
                V1 = afr(cb + 4)[AF_V];
            }
            // top rows 3 .. 0 with static indices (every register array index a
            // constant); rows at or past the end of a chain shorter than four
            // rows are skipped, as their affine maps and V stay zero
#pragma unroll
            for (int j = 3; j >= 0; --j) {
                if (j >= ch.cn) continue;
                const int row = ch.cb + j;
                const double dd = m.rec(row)[F_D];
                const double sub = j > 0 ? m.rec(row - 1)[F_C] : 0.0;
                const double sup = j + 1 < ch.cn ? m.rec(row + 1)[F_A] : 0.0;
                double piv = 1.0 - g * dd;
                double rhs = afr(row)[AF_B];
                double xH = 0.0, xE = 0.0, xP = 0.0;  // coupling columns (top rows)
                if (j < 4) {
                    double wH, wE, wP;
                    w_row(row, L, s, p, wH, wE, wP);
                    xH = g * wH;
                    xE = g * wE;
                    xP = g * wP;
                    if (row == 2) {
                        // delta_g = b_dg + g w_H(dg) zeta_H + g k^2/(4 Hc) x_theta_g, eliminated
                        // into the theta_g row through its link -(4/3)/Hc
                        const double lk = g * (4.0 / 3.0) * s.invHc;
                        double wHd, wEd, wPd;
                        w_row(L.rDG, L, s, p, wHd, wEd, wPd);
                        piv = fma(lk, g * 0.25 * s.k2H, piv);
                        rhs = fma(-lk, afr(L.rDG)[AF_B], rhs);
                        xH = fma(-lk, g * wHd, xH);
                    }
                }
                // row j: piv x_j - g sub x_{j-1} - g sup x_{j+1} = rhs + x . zeta,
                // with x_{j+1} = U1 + V1 x_j from below
                const double p2 = fma(-g * sup, V1, piv);
                const double ip = rcp(p2);
                const double V = g * sub * ip;
                {
                    // affine: the row below contributes only through its
                    // constant part (generic rows) or its affine map (top rows)
                    const double gs = g * sup;
                    double a0 = rhs, aH = xH, aE = xE, aP = xP;
                    if (j == 3) {
                        a0 = fma(gs, U1, a0);
                    } else {
                        a0 = fma(gs, tU[j + 1][0], a0);
                        aH = fma(gs, tU[j + 1][1], aH);
                        aE = fma(gs, tU[j + 1][2], aE);
                        aP = fma(gs, tU[j + 1][3], aP);
                    }
                    tU[j][0] = a0 * ip;
                    tU[j][1] = aH * ip;
                    tU[j][2] = aE * ip;
                    tU[j][3] = aP * ip;
                    tV[j] = V;
                }
                V1 = V;
            }
            // downwards through the top rows: x_j as affine maps of zeta
            double x0 = tU[0][0], xh = tU[0][1], xe = tU[0][2], xp = tU[0][3];
            for (int j = 0; j < 4; ++j) {
                if (j > 0) {
                    x0 = fma(tV[j], x0, tU[j][0]);
                    xh = fma(tV[j], xh, tU[j][1]);
                    xe = fma(tV[j], xe, tU[j][2]);
                    xp = fma(tV[j], xp, tU[j][3]);
                }
                double *q = m.AX + 4 + 16 * gl + 4 * j;
                q[0] = x0;
                q[1] = xh;
                q[2] = xe;
                q[3] = xp;
            }
        }
        wsync();
        // (2) one lane: the coupling unknowns zeta = (u_H.x, u_E.x, u_P.x)
        if (gl == 0) {
            double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, d[3] = {0, 0, 0};
            auto add = [&](int idx, double x0, double xh, double xe, double xp) {
                const double *f = tbl + idx * TBLW + 3 * NBAS;
                const double u[3] = {f[0], f[1], f[2] * s.T};
                for (int i = 0; i < 3; ++i) {
                    d[i] = fma(u[i], x0, d[i]);
                    C[i][0] = fma(u[i], xh, C[i][0]);
                    C[i][1] = fma(u[i], xe, C[i][1]);
                    C[i][2] = fma(u[i], xp, C[i][2]);
                }
            };
            for (int ch = 0; ch < L.nch; ++ch) {
                const Chain cs = chain_by_index(ch, L);
                for (int j = 0; j < 4 && j < cs.cn; ++j) {
                    const double *q = m.AX + 4 + 16 * ch + 4 * j;
                    add(4 * ch + j, q[0], q[1], q[2], q[3]);
                }
            }
            double wH, wE, wP;
            w_row(L.rDC, L, s, p, wH, wE, wP);
            add(4 * L.nch, afr(L.rDC)[AF_B], g * wH, 0.0, 0.0);
            w_row(L.rETA, L, s, p, wH, wE, wP);
            add(4 * L.nch + 1, afr(L.rETA)[AF_B], g * wH, 0.0, 0.0);
            w_row(L.rDG, L, s, p, wH, wE, wP);
            {
                const double *q = m.AX + 4 + 4 * 2;  // theta_g, row 2 of the first chain
                const double lk = g * 0.25 * s.k2H;
                add(4 * L.nch + 2, fma(lk, q[0], afr(L.rDG)[AF_B]), fma(lk, q[1], g * wH), lk * q[2], lk * q[3]);
            }
            // (I - C) zeta = d by the adjugate
            const double a00 = 1.0 - C[0][0], a01 = -C[0][1], a02 = -C[0][2];
            const double a10 = -C[1][0], a11 = 1.0 - C[1][1], a12 = -C[1][2];
            const double a20 = -C[2][0], a21 = -C[2][1], a22 = 1.0 - C[2][2];
            const double c00 = fma(a11, a22, -a12 * a21), c01 = fma(a12, a20, -a10 * a22);
            const double c02 = fma(a10, a21, -a11 * a20), c10 = fma(a02, a21, -a01 * a22);
            const double c11 = fma(a00, a22, -a02 * a20), c12 = fma(a01, a20, -a00 * a21);
            const double c20 = fma(a01, a12, -a02 * a11), c21 = fma(a02, a10, -a00 * a12);
            const double c22 = fma(a00, a11, -a01 * a10);
            const double idet = 1.0 / fma(a00, c00, fma(a01, c01, a02 * c02));
            const double zH = fma(c00, d[0], fma(c10, d[1], c20 * d[2])) * idet;
            const double zE = fma(c01, d[0], fma(c11, d[1], c21 * d[2])) * idet;
            const double zP = fma(c02, d[0], fma(c12, d[1], c22 * d[2])) * idet;
            m.AX[0] = zH;
            m.AX[1] = zE;
            m.AX[2] = zP;
            w_row(L.rDC, L, s, p, wH, wE, wP);
            afr(L.rDC)[AF_X] = fma(g * wH, zH, afr(L.rDC)[AF_B]);
            w_row(L.rETA, L, s, p, wH, wE, wP);
            afr(L.rETA)[AF_X] = fma(g * wH, zH, afr(L.rETA)[AF_B]);
            w_row(L.rDG, L, s, p, wH, wE, wP);
            const double *q = m.AX + 4 + 4 * 2;
            const double xtg = fma(q[1], zH, fma(q[2], zE, fma(q[3], zP, q[0])));
            afr(L.rDG)[AF_X] = fma(g * 0.25 * s.k2H, xtg, fma(g * wH, zH, afr(L.rDG)[AF_B]));
        }
        wsync();
        // (3) chains: the top rows from zeta, the others downwards
        if (gl < L.nch) {
            const Chain ch = chain_by_index(gl, L);
            const int cb = ch.cb, cn = ch.cn;
            const double zH = m.AX[0], zE = m.AX[1], zP = m.AX[2];
            double xp = 0.0;
            for (int j = 0; j < 4 && j < cn; ++j) {
                const double *q = m.AX + 4 + 16 * gl + 4 * j;
                xp = fma(q[1], zH, fma(q[2], zE, fma(q[3], zP, q[0])));
                afr(cb + j)[AF_X] = xp;
            }
            // generic rows in blocks of four with the next block's U, V in
            // flight; rows past the chain end go to a spare record
            double pu[4], pv[4], qu[4], qv[4];
            auto load_uv = [&](int j0, double(&u)[4], double(&v)[4]) __attribute__((always_inline)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double *f = afr(cb + j0 + q);
                    u[q] = f[AF_U];
                    v[q] = f[AF_V];
                }
            };
            double *const spare = afr(-1);
            auto down_blk = [&](const double(&u)[4], const double(&v)[4], double(&nu)[4], double(&nv)[4], int j0)
                                __attribute__((always_inline)) {
                load_uv(j0 + 4, nu, nv);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xp = fma(v[q], xp, u[q]);
                    (j0 + q < cn ? afr(cb + j0 + q) : spare)[AF_X] = xp;
                }
            };
            if (cn > 4) {
                load_uv(4, pu, pv);
                int j0 = 4;
                for (; j0 + 4 < cn; j0 += 8) {
                    down_blk(pu, pv, qu, qv, j0);
                    down_blk(qu, qv, pu, pv, j0 + 4);
                }
                if (j0 < cn) down_blk(pu, pv, qu, qv, j0);
            }
        }
        wsync();
    };

    // sum over the perturbed tables q of mu . (A(theta_q) v), differenced into
    // acc: v in the RY records of every row, mu for this lane's rows, the
    // tables' backgrounds in the stage slots.  Every entry of A is a sum of
    // background bases times static multipliers (generic rows: kH, trunc and
    // -T; the other rows from the table), so mu . A v is the bases dotted
    // with sums G_b formed once per stage, plus the couplings (h', eta', Pi)
    // of v at each background (App. B.3, eqs. hprime and etaprime).  The
    // constant basis cancels in the differences and is left out.
    auto theta_stage = [&](const double *mu) __attribute__((always_inline)) {
        double Gb[NBAS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double UH = 0.0, UE = 0.0, UPT = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            if (row >= N) continue;
            const double yr = m.ry(row);
            if ((gen >> r) & 1u) {
                const double *q = m.sta(row);
                Gb[2] = fma(mu[r], fma(q[S_CA], m.ry(row - 1), q[S_CC] * m.ry(row + 1)), Gb[2]);
                Gb[7] = fma(mu[r] * q[S_CD], yr, Gb[7]);
                if ((pho >> r) & 1u) Gb[4] = fma(-mu[r], yr, Gb[4]);
                continue;
            }
            if (cidx[r] < 0) continue;
            const double *e = tbl + cidx[r] * TBLW;
            const double ym = (rinfo[r] & RI_UP) ? m.ry(row - 1) : 0.0;
            const double yp = (rinfo[r] & RI_DN) ? m.ry(row + 1) : 0.0;
#pragma unroll
            for (int bb = 1; bb < NBAS; ++bb)
                Gb[bb] = fma(mu[r], fma(e[bb], ym, fma(e[NBAS + bb], yr, e[2 * NBAS + bb] * yp)), Gb[bb]);
            UH = fma(mu[r], e[3 * NBAS], UH);
            UE = fma(mu[r], e[3 * NBAS + 1], UE);
            UPT = fma(mu[r], e[3 * NBAS + 2], UPT);
            if (rinfo[r] & RI_TG) Gb[3] = fma(0.25 * mu[r], m.ry(L.rDG), Gb[3]);  // theta_g' ... + k^2 delta_g / (4 Hc)
            if (rinfo[r] & RI_DG) Gb[1] = fma(-(4.0 / 3.0) * mu[r], m.ry(2), Gb[1]);  // delta_g' = -(4/3) theta_g / Hc ...
        }
        // mu . (A(theta+) - A(theta-)) v / den is linear in the bases and the
        // couplings h', eta', Pi of v at each background: their differences
        // between the two tables of a parameter, divided by den, are formed once
        // per stage, one parameter per lane, and left in gv (free between
        // output times) for every lane to dot with its own sums.  Differencing
        // the bases before the contraction also cancels the two nearly equal
        // tables on exact inputs rather than on rounded sums.
        constexpr int DVW = NBAS + 2;  // bases 1..7, then H, E, T Pi
        if (gl < NPAR) {
            const int i = gl;
            const Bk &sa = bk_ref(2 * i), &sb = bk_ref(2 * i + 1);
            const double Yeta = m.ry(L.rETA), Ydc = m.ry(L.rDC), Y0 = m.ry(0), Ydg = m.ry(L.rDG), YbV = m.ry(L.bV);
            const double Y1 = m.ry(1), Y2 = m.ry(2), YbV1 = m.ry(L.bV + 1);
            const double Pv = p.lp > 0 ? 2.0 * m.ry(3) + m.ry(L.bG) + m.ry(L.bG + 2) : 0.0;
            auto HE = [&](const Bk &sq, double &H, double &E) __attribute__((always_inline)) {
                H = fma(sq.cH1, Yeta, sq.cH2 * fma(sq.rc, Ydc, fma(sq.rb, Y0, fma(sq.rg, Ydg, sq.rur * YbV))));
                E = sq.cE * fma(sq.rb, Y1, fma((4.0 / 3.0) * sq.rg, Y2, (4.0 / 3.0) * sq.rur * YbV1));
            };
            double va[NBAS], vb[NBAS], Ha, Ea, Hb, Eb;
            bases_of(sa, va);
            bases_of(sb, vb);
            HE(sa, Ha, Ea);
            HE(sb, Hb, Eb);
            const double id = 1.0 / den[i];
            double *dv = gv + i * DVW;
#pragma unroll
            for (int bb = 1; bb < NBAS; ++bb) dv[bb - 1] = (va[bb] - vb[bb]) * id;
            dv[NBAS - 1] = (Ha - Hb) * id;
            dv[NBAS] = (Ea - Eb) * id;
            dv[NBAS + 1] = (sa.T - sb.T) * Pv * id;
        }
        wsync();
#pragma unroll
        for (int i = 0; i < NPAR; ++i) {
            const double *dv = gv + i * DVW;
            double d = 0.0;
#pragma unroll
            for (int bb = 1; bb < NBAS; ++bb) d = fma(Gb[bb], dv[bb - 1], d);
            d = fma(UH, dv[NBAS - 1], fma(UE, dv[NBAS], fma(UPT, dv[NBAS + 1], d)));
            acc[i] += d;
        }
        wsync();
    };

    for (int n = nst - 1; n >= 0; --n) {
        const double *qrec = traj + (mode * traj_cap + n) * TR;
        const double t = qrec[0], h = qrec[1], tn = qrec[2], hh = tn - t;
        const double g = h * GAMMA;
        const bool start = final_seg && n == 0;  // the integration's first step
        // the step's stage derivatives of this lane's rows (from the trajectory)
        double Kr[NSTG][R];
#pragma unroll
        for (int j = 0; j < NSTG; ++j)
#pragma unroll
            for (int r = 0; r < R; ++r) Kr[j][r] = gl * R + r < N ? qrec[3 + (1 + j) * N + gl * R + r] : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            w.y[r] = row < N ? qrec[3 + row] : 0.0;
            w.yb[r] = 0.0;
#pragma unroll
            for (int j = 0; j < NSTG - 1; ++j) kbr(j, r) = 0.0;
        }
        // the output times of this step: (t_n, t_{n+1}], the first step also t_0
        int o0 = 0, o1 = n_tau;
        {
            int lo_i = 0, hi_i = n_tau;  // first index with lo > t (>= t at the start)
            while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i) >> 1;
                if (start ? lo[mid] < t : lo[mid] <= t) lo_i = mid + 1; else hi_i = mid;
            }
            o0 = lo_i;
            lo_i = o0;
            hi_i = n_tau;  // first index with lo > tn
            while (lo_i < hi_i) {
                const int mid = (lo_i + hi_i) >> 1;
                if (lo[mid] <= tn) lo_i = mid + 1; else hi_i = mid;
            }
            o1 = lo_i;
        }
        for (int o = o0; o < o1; ++o) {
            const double th = hh > 0.0 ? (lo[o] - t) / hh : 1.0;
            const double th2 = th * th, th3 = th2 * th;
            const double h00 = 2.0 * th3 - 3.0 * th2 + 1.0, h10 = th3 - 2.0 * th2 + th;
            const double h01 = -2.0 * th3 + 3.0 * th2, h11 = th3 - th2;
            // dL/dy at this output (transposed sources) into gv, zero elsewhere
#pragma unroll
            for (int r = 0; r < R; ++r) gv[gl * R + r] = 0.0;
            // the interpolated state into the RY records (for the sources' own
            // parameter dependence); Y_5 = R_5 + g K_5
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double y5 = w.y[r];
#pragma unroll
                for (int j = 0; j < NSTG - 1; ++j) y5 = fma(h * Ka[NSTG - 1][j], Kr[j][r], y5);
                y5 = fma(g, Kr[NSTG - 1][r], y5);
                m.ry(gl * R + r) = h00 * w.y[r] + h10 * hh * Kr[0][r] + h01 * y5 + h11 * hh * Kr[NSTG - 1][r];
            }
            wsync();
            if (gl == 0) sources_adj_point<false>(tb, p, L, n_tau, ik, o, gS + mode * 3 * n_tau, gv);
            wsync();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double G_ = gv[gl * R + r];
                w.yb[r] = fma(h00, G_, w.yb[r]);
                kbr(0, r) = fma(h10 * hh, G_, kbr(0, r));
                w.Y5b[r] = fma(h01, G_, w.Y5b[r]);
                kbr(NSTG - 1, r) = fma(h11 * hh, G_, kbr(NSTG - 1, r));
            }
            // the sources' own dependence on the parameters at this state: one
            // perturbed table per lane
            for (int q = gl; q < 2 * NPAR; q += G) {
                Bk sp;
                bk_at<false>(pt(q), p, k, lo[o], sp);
                double S0, S1, S2;
                auto yo = [&](int row) { return m.ry(row); };
                source_values(sp, L, p, k, yo, 0.0, 0.0, 0.0, S0, S1, S2);
                const double *gs = gS + mode * 3 * n_tau;
                const double d = (gs[o] * S0 + gs[n_tau + o] * S1 + gs[2 * n_tau + o] * S2) / den[q >> 1];
#pragma unroll
                for (int i = 0; i < NPAR; ++i)
                    if ((q >> 1) == i) acc[i] += (q & 1) ? -d : d;
            }
            wsync();
        }
        // stages, last to first
        for (int si = NSTG - 1; si >= 1; --si) {
            const double ts = (Kc[si] == 1.0) ? tn : t + Kc[si] * h;
            stage_bks(ts);
            const Bk &s = bk_ref(2 * NPAR);
            double Ys[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double rr = w.y[r];
                double ks = Kr[0][r];
#pragma unroll
                for (int j = 0; j < NSTG - 1; ++j)
                    if (j < si) rr = fma(h * Ka[si][j], Kr[j][r], rr);
#pragma unroll
                for (int j = 1; j < NSTG; ++j)
                    if (si == j) ks = Kr[j][r];
                Ys[r] = fma(g, ks, rr);
                afr(gl * R + r)[AF_B] = kbr(si, r);
            }
            wsync();
            double at[R];
            apply_t(s, at);  // A_s^T Kbar_s (and this stage's entries cached)
            wsync();
#pragma unroll
            for (int r = 0; r < R; ++r)
                afr(gl * R + r)[AF_B] = at[r] + (si == NSTG - 1 ? w.Y5b[r] : 0.0);
            wsync();
            solve_t(s, g);  // Rbar_s into AF_X
            double mu[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double rb = gl * R + r < N ? afr(gl * R + r)[AF_X] : 0.0;
                mu[r] = fma(g, rb, kbr(si, r));
                w.yb[r] += rb;
#pragma unroll
                for (int j = 0; j < NSTG - 1; ++j)
                    if (j < si) kbr(j, r) = fma(h * Ka[si][j], rb, kbr(j, r));
                m.ry(gl * R + r) = Ys[r];
            }
            wsync();
            theta_stage(mu);  // the stage matrix's dependence on the parameters
        }
        if (start) {
            // K_0 = A(t_0) y_0 at the start, and y_0 from the initial conditions
            stage_bks(t);
            const Bk &s = bk_ref(2 * NPAR);
            double at[R], mu[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                afr(gl * R + r)[AF_B] = kbr(0, r);
                m.ry(gl * R + r) = w.y[r];
                mu[r] = kbr(0, r);
            }
            wsync();
            apply_t(s, at);
            wsync();
            theta_stage(mu);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                w.yb[r] += at[r];
                kbr(0, r) = 0.0;
            }
            double dq[2 * NPAR];
            for (int q = 0; q < 2 * NPAR; ++q) {
                const Bk &sp = bk_ref(q);
                double d = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int row = gl * R + r;
                    if (row < N) d = fma(w.yb[r], ic_row<false>(row, L, sp, pt(q), k), d);
                }
                dq[q] = d;
            }
#pragma unroll
            for (int i = 0; i < NPAR; ++i) acc[i] += (dq[2 * i] - dq[2 * i + 1]) / den[i];
        }
        // to the previous step: dL/dy_n seeds its last stage, dL/dK_0 its K_5
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w.Y5b[r] = w.yb[r];
            kbr(NSTG - 1, r) = kbr(0, r);
        }
    }
    // carry to the previous segment (or, after the first, dL/dy_0)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = gl * R + r;
        if (row < N) {
            lm[row] = w.Y5b[r];
            lm[N + row] = kbr(NSTG - 1, r);
        }
    }
#pragma unroll
    for (int q = 0; q < NPAR; ++q) {
        const double v = group_sum(acc[q]);
        if (gl == 0) gr[q] = (first ? 0.0 : gr[q]) + v;
    }
}

// The gradient of L = sum dL/dC_l C_l per cosmology, assembled from its
// parts (one workgroup per cosmology): the reverse sweep's per-mode sums for
// (h, omega_b, omega_cdm, tau_reio); the projection's own dependence on them
// from the spectra of the unperturbed sources under the perturbed tables'
// geometry (central differences); ln A_s (C_l is proportional to A_s) and n_s
// (the k quadrature weighted by ln(k / k_pivot)).
constexpr int ASM_THREADS = 256;
__global__ void __launch_bounds__(ASM_THREADS) grad_assemble_kernel(int n_cosmo, int n_k, int n3,
                                                                   const double *__restrict__ gCl,
                                                                   const double *__restrict__ Cl,
                                                                   const double *__restrict__ Cns,
                                                                   const double *__restrict__ Cp,
                                                                   const double *__restrict__ pden,
                                                                   const double *__restrict__ adj,
                                                                   double *__restrict__ grad) {
    __shared__ double red[ASM_THREADS / 64][2 + 2 * NPAR];
    const int c = blockIdx.x, tid = threadIdx.x;
    const double *g = gCl + (size_t)c * n3;
    double v[2 + 2 * NPAR];
    for (int i = 0; i < 2 + 2 * NPAR; ++i) v[i] = 0.0;
    for (int j = tid; j < n3; j += ASM_THREADS) {
        const double gj = g[j];
        v[0] = fma(gj, Cl[(size_t)c * n3 + j], v[0]);
        v[1] = fma(gj, Cns[(size_t)c * n3 + j], v[1]);
        for (int i = 0; i < NPAR; ++i) {
            const double dp = Cp[((size_t)(2 * i) * n_cosmo + c) * n3 + j] - Cp[((size_t)(2 * i + 1) * n_cosmo + c) * n3 + j];
            v[2 + i] = fma(gj, dp, v[2 + i]);
        }
    }
    for (int ik = tid; ik < n_k; ik += ASM_THREADS)
        for (int i = 0; i < NPAR; ++i) v[2 + NPAR + i] += adj[((size_t)c * n_k + ik) * NPAR + i];
    // wavefront sums, then one per wavefront through LDS (fixed order)
    for (int i = 0; i < 2 + 2 * NPAR; ++i)
        for (int o = 32; o >= 1; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
    if ((tid & 63) == 0)
        for (int i = 0; i < 2 + 2 * NPAR; ++i) red[tid >> 6][i] = v[i];
    __syncthreads();
    if (tid == 0) {
        double t[2 + 2 * NPAR];
        for (int i = 0; i < 2 + 2 * NPAR; ++i) {
            t[i] = 0.0;
            for (int w = 0; w < ASM_THREADS / 64; ++w) t[i] += red[w][i];
        }
        // (h, omega_b, omega_cdm, ln A_s, n_s, tau_reio)
        const int slot[NPAR] = {0, 1, 2, 5};
        double *gr = grad + (size_t)c * 6;
        gr[3] = t[0];
        gr[4] = t[1];
        for (int i = 0; i < NPAR; ++i) gr[slot[i]] = t[2 + NPAR + i] + t[2 + i] / pden[(size_t)c * NPAR + i];
    }
}

template <int R>
int launch_adj_r(const DevTab *d_tabs, const DevTab *d_ptabs, const double *d_pden, int n_cosmo, int n_k, int n_tau,
                 const DevPrec &p, int G, const double *d_traj, int traj_cap, const int *d_hist_n, int seg, int every,
                 const double *d_gS, double *d_lam, double *d_grad, int first, size_t lds, hipStream_t s) {
    const int spw = 64 / G;
    const long n_sys = (long)n_cosmo * n_k;
    const long blocks = (n_sys + spw - 1) / spw;
    hipLaunchKernelGGL(adjoint_kernel<R>, dim3((unsigned)blocks), dim3(64), lds, s, d_tabs, d_ptabs, d_pden, n_cosmo,
                       n_k, n_tau, p, G, d_traj, traj_cap, d_hist_n, seg, every, d_gS, d_lam, d_grad, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("reverse sweep launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

// The reverse kernel's group shape: 32 lanes of three rows for hierarchies of
// 65..96 rows (config 1: 79), two modes per wavefront; otherwise the forward
// kernel's narrow shape.  At config 1, batch 32, the 32-lane groups took a
// gradient from 2.80 to 2.52 s against 16 lanes of five rows (64 lanes of
// two: 3.77 s): the row-parallel work per lane shrinks, and the kernel holds
// one wavefront per SIMD in either shape.
void adjoint_shape(const DevPrec &p, int &R, int &G) {
    group_shape(p, R, G);
    const int N = make_lay(p).N;
    if (N > 64 && N <= 96) {
        R = 3;
        G = 32;
    }
}

}  // namespace

bool adjoint_supported(const DevPrec &p) {
    if (p.nq > 0) return false;
    int R, G;
    adjoint_shape(p, R, G);
    const Lay L = make_lay(p);
    if (G > 64 || (R != 2 && R != 3 && R != 5)) return false;
    return (size_t)adj_lds_doubles(G * R, L.nch, 64 / G) * sizeof(double) <= 65536;
}

int launch_adjoint_segment(const DevTab *d_tabs, const DevTab *d_ptabs, const double *d_pden, int n_cosmo, int n_k,
                           int n_tau, const DevPrec &p, const double *d_traj, int traj_cap, const int *d_hist_n,
                           int seg, int every, const double *d_gS, double *d_lam, double *d_grad, int first,
                           void *stream) {
    if (!adjoint_supported(p)) {
        set_error("reverse sweep: massless neutrinos only, and a hierarchy whose records fit 64 KB of LDS per workgroup");
        return CMB_E_UNSUPPORTED;
    }
    if (every < 1 || traj_cap < every || seg < 0 || n_cosmo < 1 || n_k < 1) {
        set_error("reverse sweep: need every >= 1, traj_cap >= every, seg >= 0");
        return CMB_E_INVALID;
    }
    int R, G;
    adjoint_shape(p, R, G);
    const Lay L = make_lay(p);
    const size_t lds = (size_t)adj_lds_doubles(G * R, L.nch, 64 / G) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    if (R == 3)
        return launch_adj_r<3>(d_tabs, d_ptabs, d_pden, n_cosmo, n_k, n_tau, p, G, d_traj, traj_cap, d_hist_n, seg,
                               every, d_gS, d_lam, d_grad, first, lds, s);
    if (R == 2)
        return launch_adj_r<2>(d_tabs, d_ptabs, d_pden, n_cosmo, n_k, n_tau, p, G, d_traj, traj_cap, d_hist_n, seg,
                               every, d_gS, d_lam, d_grad, first, lds, s);
    return launch_adj_r<5>(d_tabs, d_ptabs, d_pden, n_cosmo, n_k, n_tau, p, G, d_traj, traj_cap, d_hist_n, seg, every,
                           d_gS, d_lam, d_grad, first, lds, s);
}

int launch_grad_assemble(int n_cosmo, int n_k, int ell_max, const double *d_gCl, const double *d_Cl,
                         const double *d_Cns, const double *d_Cp, const double *d_pden, const double *d_adj,
                         double *d_grad, void *stream) {
    const int n3 = 3 * (ell_max + 1);
    hipLaunchKernelGGL(grad_assemble_kernel, dim3(n_cosmo), dim3(ASM_THREADS), 0, (hipStream_t)stream, n_cosmo, n_k,
                       n3, d_gCl, d_Cl, d_Cns, d_Cp, d_pden, d_adj, d_grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("gradient assembly launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
