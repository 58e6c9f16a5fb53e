// K1: synchronous-gauge perturbations and CMB sources, one group of G lanes
// per (cosmology, k) mode.
//
// The method: the ESDIRK of ARK4(3)6L[2]SA (Kennedy & Carpenter 2003), RMS
// error norm, PID step control, Hermite dense output and the source
// functions of App. B.4 of arXiv 2602.15104, for the equations of App. B.3 and
// App. C.  The mapping onto the hardware:
//
//  * a mode's state rows are spread over a group of G lanes (G = 16 for the
//    79-row TT/TE/EE hierarchy, R = 5 rows per lane, in full launches; 64
//    lanes with 2 rows or 32 with 3 when the launch has few modes, with the
//    same arithmetic); every working vector
//    (state, six stage derivatives, new state, stage right-hand side) lives
//    in registers of the lane that owns the row, so no workspace traffic;
//  * row-parallel work (stage right-hand sides, matrix entries of
//    I - h gamma A, K = (Y - R)/(h gamma), error norm, dense output) is
//    spread over the group's lanes;
//  * the three multipole chains (photon T + baryons, photon P, neutrinos)
//    are reduced by one lane each, highest multipole first, reading the
//    entries the row lanes left in LDS; the chains share one instruction
//    stream, so they advance in lock-step;
//  * one lane solves the 3x3 system of the couplings h', eta', Pi, then the
//    chain lanes substitute downwards and the row lanes pick up their rows;
//  * a wavefront holds 64/G modes; lanes exchange data through LDS at
//    compiler-only fences (a workgroup is one wavefront, whose DS
//    instructions the LDS executes in order), so modes of one wavefront may
//    branch independently.
#include <hip/hip_runtime.h>

#include "k1_common.h"

namespace cmbhip {

namespace {

// p, made opaque to the optimiser where it is formed: addresses derived from it
// are computed at their use instead of being hoisted as loop invariants.
__device__ inline double *lane_ptr(double *p) {
    __asm__ volatile("" : "+v"(p));
    return p;
}

// Modes: either the whole [n_cosmo][n_k] batch (items == nullptr; outputs in
// Sout/status/nsteps, largest k first) or the work list items[n_items] of
// (cosmology, mode) pairs, each cosmology with its own grids and its own
// output arrays in its DevTab (ragged batches of the serving runtime).
// RN: rows per lane of the groups whose error-norm summation order the
// instance keeps (RN = R, or RN = 5 for wider groups with R = 2 or 3 standing
// in for groups of Gn lanes with five rows each).
template <int R, bool MNU, bool HIST, int RN>
__global__ void __launch_bounds__(64) perturb2_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                      int n_tau_all, DevPrec p, int G, int Gn,
                                                      double *__restrict__ Sout,
                                                      int *__restrict__ status, int *__restrict__ nsteps,
                                                      const int2 *__restrict__ items, int n_items,
                                                      double *__restrict__ Pk, double *__restrict__ Dm) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int gl = lane % G;
    const int grp = lane / G;
    const int spw = 64 / G;
    const int n_sys = items ? n_items : n_cosmo * n_k;
    const int lin = blockIdx.x * spw + grp;
    const Lay L = make_lay(p);
    const int NP = G * R;
    // pivots of the chain rows formed in the upward sweep (groups of five or
    // more rows per lane, several modes per wavefront) or by a row-parallel pass
    // (fewer rows per lane); the same bits
    constexpr bool PIV = R >= 5;
    Slab m;
    {
        double *stat = lds;
        double *base = lds + stat_doubles(NP) + (size_t)grp * slab_doubles(NP, L.nch);
        m.base = base;
        m.st = stat;
        m.AX = base + (NP + 2 * PADR) * STR;
        m.BK = m.AX + ax_doubles(L.nch);
        // every record, pads included, starts from zero, and so does the
        // multipliers table (every group writes the same values into it)
        for (int i = gl; i < (NP + 2 * PADR) * STR; i += G) base[i] = 0.0;
        for (int i = gl; i < stat_doubles(NP); i += G) stat[i] = 0.0;
        wsync();
#pragma unroll
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
    if (lin >= n_sys) return;  // whole group idle (no cross-group dependence)
    int c, ik;
    if (items) {
        c = items[lin].x;
        ik = items[lin].y;
    } else {
        const int sys = n_sys - 1 - lin;  // largest k first, cosmology fastest
        c = sys % n_cosmo;
        ik = sys / n_cosmo;
    }
    const DevTab &tb = tabs[c];
    const int n_tau = items ? tb.n_tau : n_tau_all;
    const double k = tb.k[ik];
    // step history: replay the accepted step sizes hin[1..hin_n] from the
    // start hin[0] without error control, or record this mode's into hout
    // (same start and sizes: the same sequence of times, bit for bit)
    // (compiled in only for the history instances: the plain ones carry no
    // pointers or branches for it)
    const double *hin = (HIST && tb.hist_in) ? tb.hist_in + (size_t)ik * tb.hist_cap : nullptr;
    const int hin_n = hin ? min(tb.hist_in_n[ik], tb.hist_cap - 1) : 0;
    double *hout = (HIST && tb.hist_out) ? tb.hist_out + (size_t)ik * tb.hist_cap : nullptr;
    // trajectory checkpoints: ckp receives (ln a, state rows, carried stage
    // derivative) at the start and after every ck_every-th accepted step;
    // cks, when set, is the checkpoint this mode's segment of the replay
    // starts from (accepted steps na0 + 1 .. na_end)
    const int ck_stride = 1 + 2 * L.N;
    const double *cks = (HIST && hin && tb.ck_in)
                            ? tb.ck_in + ((size_t)ik * tb.ck_cap + tb.ck_seg) * ck_stride
                            : nullptr;
    double *ckp = (HIST && !cks && tb.ck_out) ? tb.ck_out + (size_t)ik * tb.ck_cap * ck_stride : nullptr;
    const int na0 = cks ? tb.ck_seg * tb.ck_every : 0;
    const int na_end = cks ? min(hin_n, na0 + tb.ck_every) : hin_n;
    if (cks && hin_n <= na0) {  // the mode ended before this segment: nothing to do
        if (gl == 0 && items) {
            tb.status[ik] = CMB_K_OK;
            tb.nsteps[ik] = 0;
        } else if (gl == 0) {
            status[(size_t)c * n_k + ik] = CMB_K_OK;
            nsteps[(size_t)c * n_k + ik] = 0;
        }
        return;
    }
    const double t0 = cks ? cks[0] : hin ? hin[0] : tb.lna_start[ik];
    const bool small = k < tb.k_split;
    const double rtol = small ? tb.rtol_small : tb.rtol_large;
    const double atol = small ? tb.atol_small : tb.atol_large;
    double *So = items ? tb.S + (size_t)ik * 3 * n_tau : Sout + ((size_t)c * n_k + ik) * 3 * n_tau;
    // matter density contrast at the output times (batch launches only)
    double *Dmo = (Dm && !items) ? Dm + ((size_t)c * n_k + ik) * n_tau : nullptr;
    const double *lo = tb.lna_src;
    const int ch = gl;  // chain handled by this lane in the sweeps
    const bool sweeper = ch < L.nch;
    const Chain mych = sweeper ? chain_by_index(ch, L) : Chain{2, 0, 0, 0};
    const int cb = mych.cb, cn = mych.cn, ty = mych.ty;  // chain start row, length, type
    const bool photon_chain = ty < 2;
    // massive node of this lane's chain: q and dln f0/dln q
    const double q_ch = (MNU && ty == 3) ? tb.q[mych.iq] : 0.0;
    const double dl_ch = (MNU && ty == 3) ? dlnf0(q_ch) : 0.0;
    const int N = L.N;

    Rows<R> w;
    // every register vector starts at zero: the stage sums below multiply the
    // not-yet-computed derivatives by zero weights, which must not meet NaN bits
#pragma unroll
    for (int r = 0; r < R; ++r) {
        w.y[r] = w.yn[r] = w.rr[r] = 0.0;
#pragma unroll
        for (int j = 0; j < NSTG; ++j) w.K[j][r] = 0.0;
    }
    Bk s;
    bk_at<MNU>(tb, p, k, t0, s);
    // initial conditions (Ma & Bertschinger 1995 growing mode, eta -> 1)
#pragma unroll
    for (int r = 0; r < R; ++r) w.y[r] = ic_row<MNU>(gl * R + r, L, s, tb, k);
    // f0 = A y0
    auto full_rhs = [&](const double *yv, double *f, const Bk &bs) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < R; ++r) m.ry(gl * R + r) = yv[r];
        wsync();
        if (gl == 0) {
            double H, E, P;
            aux_from_rows(m, L, bs, p, tb, k, H, E, P);
            m.AX[0] = H;
            m.AX[1] = E;
            m.AX[2] = P;
        }
        wsync();
        rhs_rows<R>(m, L, bs, p, tb, gl, f);
        wsync();
    };
    full_rhs(w.y, w.K[0], s);
    if (cks) {  // a segment continues from its checkpoint's state and derivative
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = gl * R + r;
            if (row < N) {
                w.y[r] = cks[1 + row];
                w.K[0][r] = cks[1 + N + row];
            }
        }
    }

    // sum over the group's lanes, the same bits in every lane (each step adds
    // two partial sums that every lane of the pair forms in the same order):
    // DPP permutes inside a 16-lane row (swap neighbours, swap pairs, mirror
    // the half row, mirror the row), lane shuffles only for groups above 16
    auto group_sum = [&](double v, int w) __attribute__((always_inline)) {
        v += dpp_f64<0xB1>(v);  // quad_perm [1, 0, 3, 2]
        v += dpp_f64<0x4E>(v);  // quad_perm [2, 3, 0, 1]
        if (w >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
        if (w >= 16) v += dpp_f64<0x140>(v);  // row_mirror
        for (int o = 16; o < w; o <<= 1) v += __shfl_xor(v, o, w);
        return v;
    };
    // RMS error norm.  In a wide launch (a whole wavefront per mode, RN != R)
    // the rows' terms are summed in the order of the narrow groups of Gn
    // lanes with RN rows each, so a mode takes the same steps, bit for bit,
    // in either shape (and so alone or in any batch).
    auto rms = [&](const double *v, const double *y1, const double *y2) __attribute__((always_inline)) {
        auto term = [&](int r) __attribute__((always_inline)) {
            double yy = fabs(y1[r]);
            if (y2) yy = fmax(yy, fabs(y2[r]));
            return v[r] * rcp(fma(rtol, yy, atol));
        };
        double acc = 0.0;
        if constexpr (RN == R) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (gl * R + r < N) {
                    const double q = term(r);
                    acc = fma(q, q, acc);
                }
            }
            acc = group_sum(acc, G);
        } else if constexpr (R == 2 * RN) {
            // groups of G = Gn / 2 lanes with twice the rows: lane g holds the
            // rows of narrow lanes 2g and 2g + 1, whose partial sums it forms
            // in their order and adds (the narrow tree's first level); the
            // narrow tree's later levels pair lanes g ^ 1, g ^ 2 and the two
            // halves of the group (its mirrored quads hold equal values)
            double a2 = 0.0;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                if (gl * R + r < N) {
                    const double q = term(r);
                    acc = fma(q, q, acc);
                }
                if (gl * R + RN + r < N) {
                    const double q = term(RN + r);
                    a2 = fma(q, q, a2);
                }
            }
            acc += a2;
            if (G >= 2) acc += dpp_f64<0xB1>(acc);   // quad_perm [1, 0, 3, 2]
            if (G >= 4) acc += dpp_f64<0x4E>(acc);   // quad_perm [2, 3, 0, 1]
            if (G >= 8) acc += dpp_f64<0x141>(acc);  // row_half_mirror
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) m.rec(gl * R + r)[F_M] = term(r);
            wsync();
            if (gl < Gn)
                for (int r = 0; r < RN; ++r)
                    if (RN * gl + r < N) {
                        const double q = m.rec(RN * gl + r)[F_M];
                        acc = fma(q, q, acc);
                    }
            acc = group_sum(acc, Gn);  // lanes from Gn on carry values nobody uses
            acc = __shfl(acc, 0, G);   // the group's first lane to the group
        }
        return sqrt(acc / N);
    };

    int jo = 0;
    if (cks && na0 > 0) {  // outputs up to the checkpoint belong to earlier segments
        while (jo < n_tau && lo[jo] <= t0) ++jo;
    } else if (gl == 0) {
        while (jo < n_tau && lo[jo] < t0) {
            So[jo] = 0.0;
            So[n_tau + jo] = 0.0;
            So[2 * n_tau + jo] = 0.0;
            if (Dmo) Dmo[jo] = 0.0;
            ++jo;
        }
    } else {
        while (jo < n_tau && lo[jo] < t0) ++jo;
    }
    double t = t0;
    double h = 0.0;
    if (!hin) {
        double d0 = rms(w.y, w.y, nullptr);
        double d1 = rms(w.K[0], w.y, nullptr);
        double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
        if (h0 > -t) h0 = -t;
        double y1[R], f1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) y1[r] = w.y[r] + h0 * w.K[0][r];
        Bk s1;
        bk_at<MNU>(tb, p, k, t + h0, s1);
        full_rhs(y1, f1, s1);
#pragma unroll
        for (int r = 0; r < R; ++r) f1[r] -= w.K[0][r];
        double d2 = rms(f1, w.y, nullptr) / h0;
        double dm = fmax(d1, d2);
        double hh = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / (ERR_ORDER + 1.0));
        h = fmin(100.0 * h0, hh);
    }
    const double b1 = (p.pcoeff + p.icoeff + p.dcoeff) / ERR_ORDER;
    const double b2 = -(p.pcoeff + 2.0 * p.dcoeff) / ERR_ORDER;
    const double b3 = p.dcoeff / ERR_ORDER;
    double lEp = 0.0, lEpp = 0.0;  // logs of the previous two accepted error norms
    int ns = 0, na = na0, st = CMB_K_OK;
    bool seg_open = false;  // a segment stopped at its last step, before a = 1
    if (hout && gl == 0) hout[0] = t0;
    auto put_ck = [&](int slot) __attribute__((always_inline)) {
        if (slot >= tb.ck_cap) return;
        double *q = ckp + (size_t)slot * ck_stride;
        if (gl == 0) q[0] = t;
        // this lane's rows from a base formed here (opaque to the optimiser, so
        // that the per-row addresses are not hoisted out of the step loop and
        // held in registers for the whole integration)
        double *qr = lane_ptr(q + 1 + gl * R);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (gl * R + r < N) {
                qr[r] = w.y[r];
                qr[N + r] = w.K[0][r];
            }
        }
    };
    if (ckp) put_ck(0);

    while (t < 0.0) {
        if (ns >= p.max_steps) {
            st = CMB_K_MAX_STEPS;
            break;
        }
        bool last = false;
        if (hin) {
            if (na >= na_end) {
                seg_open = na_end < hin_n;
                st = seg_open ? CMB_K_OK : CMB_K_MAX_STEPS;
                break;
            }
            h = hin[1 + na];
            last = t + h >= 0.0;
        } else if (h >= -t) {
            h = -t;
            last = true;
        }
        const double g = h * GAMMA;
        // the backgrounds of the step's implicit stages, evaluated at once on
        // as many lanes of the group (instead of one stage after the other on
        // every lane) and read back from LDS stage by stage; the stage at the
        // step's end lands on it exactly
        for (int si = 1 + gl; si < NSTG; si += G) {
            const double ts = (Kc[si] == 1.0) ? (last ? 0.0 : t + h) : t + Kc[si] * h;
            Bk b;
            bk_at<MNU>(tb, p, k, ts, b);
            __builtin_memcpy(m.BK + (si - 1) * NBK, &b, sizeof(Bk));
        }
        wsync();
        for (int si = 1; si < NSTG; ++si) {
            __builtin_memcpy(&s, m.BK + (si - 1) * NBK, sizeof(Bk));
            const double gkH = g * s.kH, gT_ph = g * s.T, gtr = g * s.trunc;
            // (A) stage right-hand sides y_n + sum_{j<s} h a_sj K_j, row-parallel;
            // the weights h a_sj for j >= s are zero: fixed-length sums keep every
            // register index static
            double hA[NSTG - 1];
#pragma unroll
            for (int j = 0; j < NSTG - 1; ++j) hA[j] = (j < si) ? h * Ka[si][j] : 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double acc = w.y[r];
#pragma unroll
                for (int j = 0; j < NSTG - 1; ++j) acc += hA[j] * w.K[j][r];
                w.rr[r] = acc;
                m.ry(gl * R + r) = acc;
            }
            wsync();
            // (B) upward elimination of each chain, one lane per chain.  The top
            // rows' affine maps are set on every lane first: a value that only
            // the sweeping lanes define must not stay undefined in the other
            // lanes while they run the sections in between (the downward pass
            // reads these maps from registers)
            Aff top[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) top[j] = Aff{0.0, 0.0, 0.0, 0.0};
            double vq = 0.0;  // streaming rate of this lane's massive node
            if (sweeper) {
                const double gT = photon_chain ? gT_ph : 0.0;
                if (MNU && ty == 3) vq = q_ch * s.kH * rcp(eps_of(q_ch, s.am));
                const double u = (MNU && ty == 3) ? g * vq : gkH, iu = rcp(u);
                // Generic rows cn-1 .. 4 in continuant form.  With N_cn = 1,
                // N_{cn+1} = 0, N_j = b_j N_{j+1} - c_j a_{j+1} N_{j+2} and
                // T_j = r_j N_{j+1} - c_j T_{j+1}, the eliminated pivot and rhs
                // are N_j / N_{j+1} and T_j / N_{j+1}.  Kept as M_j = N_j u^(j-cn),
                // S_j = T_j u^(j+1-cn) with u = g v (v the chain's streaming rate),
                // both recurrences take two operations a row:
                //   M_j = (b_j / u) M_{j+1} + CP_j M_{j+2},  S_j = r_j M_{j+1} + CC_j S_{j+1}.
                // Every M_j >= M_{j+1} > 0 (b_j >= 1, CP_j >= 0): no cancellation, no
                // division on the dependent path; M, S are rescaled by 2^-332 per
                // block whenever M passes 2^332.  The downward recurrence
                // y_j = U_j - V_j y_{j-1} takes U_j = T_j / N_j = S_j / (u M_j) and
                // V_j = a_j N_{j+1} / N_j = -CA_j M_{j+1} / M_j.  With several modes
                // per wavefront (PIV) both are formed here, beside the recurrences
                // (the reciprocal is off their dependent path), and only they are
                // stored: LDS stores cost a whole wavefront's store bandwidth however
                // few lanes are active, and with four wavefronts per CU they are what
                // this serial section waits on.  With a mode per wavefront or two,
                // the sweep stores M_j, M_{j+1} and S_j / u and the row lanes form
                // U_j, V_j in a pass of their own (D0), with the same operations, so
                // both give the same bits.  Blocks of four rows always run whole: rows
                // above the fifth only receive values nobody reads.
                if (cn >= 5) {
                    const double bq = (1.0 + gT) * iu;
                    double *rl = m.rec(cb + cn - 1);
                    const double *sl = m.sta(cb + cn - 1);
                    double M1 = fma(-gtr, sl[S_CD], 1.0 + gT) * iu, M2 = 1.0, S1 = rl[F_RY];
                    double caP = sl[S_CA];  // CA_{j+1} for the next row j (CP_j = -CC_j CA_{j+1})
                    if constexpr (PIV) {
                        const double iM = rcp(M1);
                        rl[F_U] = (S1 * iu) * iM;
                        rl[F_V] = -sl[S_CA] * M2 * iM;
                    } else {
                        rl[F_M] = M1;
                        rl[F_MN] = M2;
                        rl[F_U] = S1 * iu;
                    }
                    // prefetched RY, CC, CP and CA of the next block, rows j0 .. j0-3
                    double pr[4], pc[4], pp[4], pa[4];
                    const double *pb = m.rec(cb + cn - 5);  // row j0 - 3 of the first block
                    const double *ps = m.sta(cb + cn - 5);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pr[q] = pb[(3 - q) * STR + F_RY];
                        pc[q] = ps[(3 - q) * SST + S_CC];
                        pp[q] = PIV ? 0.0 : ps[(3 - q) * SST + S_CP];
                        pa[q] = PIV ? ps[(3 - q) * SST + S_CA] : 0.0;
                    }
                    // one block: rows j0 .. j0-3 from (cr, cc, cp, ca) while the next
                    // block's values load into (nr, nc, np, na); two blocks per trip
                    // with the buffers alternating, so no register copies between blocks
                    auto up_block = [&](const double(&cr)[4], const double(&cc)[4], const double(&cp)[4],
                                        const double(&ca)[4], double(&nr)[4], double(&nc)[4], double(&np)[4],
                                        double(&na)[4], int j0) {
                        double *cbk = m.rec(j0 - 3 + cb);
                        const double *nb = cbk - 4 * STR;
                        const double *ns = m.sta(j0 - 3 + cb) - 4 * SST;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            nr[q] = nb[(3 - q) * STR + F_RY];
                            nc[q] = ns[(3 - q) * SST + S_CC];
                            if constexpr (!PIV) np[q] = ns[(3 - q) * SST + S_CP];
                            if constexpr (PIV) na[q] = ns[(3 - q) * SST + S_CA];
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // CP_j = -CC_j CA_{j+1}, CA_{j+1} being the row below's
                            const double cpq = PIV ? -cc[q] * caP : cp[q];
                            if constexpr (PIV) caP = ca[q];
                            const double M0 = fma(bq, M1, cpq * M2);
                            const double S0 = fma(cr[q], M1, cc[q] * S1);
                            M2 = M1;
                            M1 = M0;
                            S1 = S0;
                            double *rq = cbk + (3 - q) * STR;
                            if constexpr (PIV) {
                                const double iM = rcp(M1);
                                rq[F_U] = (S1 * iu) * iM;
                                rq[F_V] = -ca[q] * M2 * iM;
                            } else {
                                rq[F_M] = M1;
                                rq[F_MN] = M2;
                                rq[F_U] = S1 * iu;
                            }
                        }
                        const double f = M1 > 0x1p332 ? 0x1p-332 : 1.0;
                        M1 *= f;
                        M2 *= f;
                        S1 *= f;
                    };
                    double qr[4], qc[4], qp[4], qa[4];
                    int j0 = cn - 2;
                    for (; j0 >= 8; j0 -= 8) {
                        up_block(pr, pc, pp, pa, qr, qc, qp, qa, j0);
                        up_block(qr, qc, qp, qa, pr, pc, pp, pa, j0 - 4);
                    }
                    if (j0 >= 4) up_block(pr, pc, pp, pa, qr, qc, qp, qa, j0);
                }
                // top rows 3 .. 0 carry the couplings.  Their elimination goes on
                // in continuant form, with no division on the dependent path: in
                // units of the generic row 4's continuant (N_j / N_4),
                //   Q_j = be_j Q_{j+1} - ga_j b_{j+1} Q_{j+2},  Z_j = z_j Q_{j+1} - ga_j Z_{j+1}
                // for z the rhs and each coupling column, where row 4 enters as
                // Q_4 = 1, b_4 Q_5 = -CA_4 M_5 / M_4 = V_4 and Z_4 = U_4 (zero for the
                // couplings).  Then pivot_j = Q_j / Q_{j+1} and z'_j / pivot_j =
                // Z_j / Q_j: the four reciprocals are independent of one another.
                // (A four-row chain starts from Q_4 = 1, Q_5 = 0, Z_4 = 0.)
                double Q1 = 1.0, Q2 = 0.0, bq1 = 0.0, Z0 = 0.0, ZH = 0.0, ZE = 0.0, ZP = 0.0;
                if (cn >= 5) {
                    const double *r4 = m.rec(cb + 4);
                    bq1 = 1.0;
                    if constexpr (PIV) {
                        Q2 = r4[F_V];
                        Z0 = r4[F_U];
                    } else {  // the operations of the D0 pass below
                        const double iM = rcp(r4[F_M]);
                        Q2 = -m.sta(cb + 4)[S_CA] * r4[F_MN] * iM;
                        Z0 = r4[F_U] * iM;
                    }
                }
                double Qs[5], z0[4], zH[4], zE[4], zP[4], al[4];
                Qs[4] = Q1;
#pragma unroll
                for (int j = 3; j >= 0; --j) {
                    const RowCo cc = top_coef<MNU>(ty, j, L, s, p, vq, dl_ch);
                    double be = 1.0 - g * cc.d, ga = -g * cc.c, rho = m.ry(cb + j);
                    double xH = -g * cc.uH, xE = -g * cc.uE, xP = -g * cc.uP;
                    if (j == 2) {
                        // photon chain: delta_g = R_dg - g (4/3)/Hc theta_g - (2g/3) h'
                        // eliminated into the theta_g row
                        const double cl = ty == 0 ? g * 0.25 * s.k2H : 0.0;
                        be = fma(cl * g * (4.0 / 3.0), s.invHc, be);
                        xH = fma(cl, g * (2.0 / 3.0), xH);
                        rho = fma(cl, m.ry(L.rDG), rho);
                    }
                    const double Q = fma(be, Q1, -(ga * bq1) * Q2);
                    Z0 = fma(-ga, Z0, rho * Q1);
                    ZH = fma(-ga, ZH, xH * Q1);
                    ZE = fma(-ga, ZE, xE * Q1);
                    ZP = fma(-ga, ZP, xP * Q1);
                    Q2 = Q1;
                    Q1 = Q;
                    bq1 = -g * cc.a;
                    Qs[j] = Q;
                    z0[j] = Z0;
                    zH[j] = ZH;
                    zE[j] = ZE;
                    zP[j] = ZP;
                    al[j] = bq1;
                }
                // y_j = (z'_j - b_j y_{j-1} - x'_j . (h', eta', Pi)) / pivot_j as affine maps
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double iQ = rcp(Qs[j]);
                    double v0 = z0[j] * iQ, vH = -zH[j] * iQ, vE = -zE[j] * iQ, vP = -zP[j] * iQ;
                    if (j > 0) {
                        const double c = al[j] * (Qs[j + 1] * iQ);
                        v0 = fma(-c, top[j - 1].v0, v0);
                        vH = fma(-c, top[j - 1].vH, vH);
                        vE = fma(-c, top[j - 1].vE, vE);
                        vP = fma(-c, top[j - 1].vP, vP);
                    }
                    top[j] = Aff{v0, vH, vE, vP};
                    m.AX[4 + 16 * ch + 4 * j + 0] = v0;
                    m.AX[4 + 16 * ch + 4 * j + 1] = vH;
                    m.AX[4 + 16 * ch + 4 * j + 2] = vE;
                    m.AX[4 + 16 * ch + 4 * j + 3] = vP;
                }
            }
            wsync();
            // (D0) row lanes turn the continuants of the generic rows into the
            // downward recurrence y_j = U_j - V_j y_{j-1} (wide shapes only; see
            // the upward sweep): U_j = S_j / (u M_j),  V_j = -CA_j M_{j+1} / M_j
            // (selects rather than a branch per row, so the rows' loads and
            // reciprocals overlap; other rows keep their values)
            if constexpr (!PIV) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double *q = m.rec(gl * R + r);
                    const double ca = m.sta(gl * R + r)[S_CA], fm = q[F_M], fu = q[F_U], fmn = q[F_MN];
                    const double iM = rcp(fm);
                    const bool gen = ca != 0.0;
                    q[F_U] = gen ? fu * iM : fu;
                    q[F_V] = gen ? -ca * fmn * iM : fmn;
                }
            }
            // (C) couplings: 3x3 (2x2 without polarisation) system, one lane
            if (gl == 0) {
                auto T = [&](int chn, int j) {
                    const double *q = m.AX + 4 + 16 * chn + 4 * j;
                    return Aff{q[0], q[1], q[2], q[3]};
                };
                const int cv = L.nG ? 2 : 1;
                Aff F0 = T(0, 0), F1 = T(0, 1), F2 = T(0, 2), F3 = T(0, 3), V0 = T(cv, 0), V1 = T(cv, 1);
                double Rdc = m.ry(L.rDC), Reta = m.ry(L.rETA), Rdg = m.ry(L.rDG);
                Aff dc{Rdc, -0.5 * g, 0.0, 0.0};
                Aff eta{Reta, 0.0, g, 0.0};
                double cg = -g * (4.0 / 3.0) * s.invHc;
                Aff dg{Rdg + cg * F2.v0, cg * F2.vH - (2.0 / 3.0) * g, cg * F2.vE, cg * F2.vP};
                Aff eH, eE;
                eH.v0 = s.cH1 * eta.v0 + s.cH2 * (s.rc * dc.v0 + s.rb * F0.v0 + s.rg * dg.v0 + s.rur * V0.v0);
                eH.vH = s.cH1 * eta.vH + s.cH2 * (s.rc * dc.vH + s.rb * F0.vH + s.rg * dg.vH + s.rur * V0.vH);
                eH.vE = s.cH1 * eta.vE + s.cH2 * (s.rc * dc.vE + s.rb * F0.vE + s.rg * dg.vE + s.rur * V0.vE);
                eH.vP = s.cH1 * eta.vP + s.cH2 * (s.rc * dc.vP + s.rb * F0.vP + s.rg * dg.vP + s.rur * V0.vP);
                const double f43 = 4.0 / 3.0;
                eE.v0 = s.cE * (s.rb * F1.v0 + f43 * s.rg * F2.v0 + f43 * s.rur * V1.v0);
                eE.vH = s.cE * (s.rb * F1.vH + f43 * s.rg * F2.vH + f43 * s.rur * V1.vH);
                eE.vE = s.cE * (s.rb * F1.vE + f43 * s.rg * F2.vE + f43 * s.rur * V1.vE);
                eE.vP = s.cE * (s.rb * F1.vP + f43 * s.rg * F2.vP + f43 * s.rur * V1.vP);
                // massive neutrinos: delta rho from Psi_0, (rho + p) theta from Psi_1 of every node
                for (int i = 0; i < (MNU ? L.nQ : 0); ++i) {
                    const double q = tb.q[i], w = s.pn4 * tb.W[i];
                    const double wh = s.cH2 * w * eps_of(q, s.am), we = s.cE * w * k * q;
                    const Aff P0 = T(cv + 1 + i, 0), P1 = T(cv + 1 + i, 1);
                    eH.v0 = fma(wh, P0.v0, eH.v0);
                    eH.vH = fma(wh, P0.vH, eH.vH);
                    eH.vE = fma(wh, P0.vE, eH.vE);
                    eH.vP = fma(wh, P0.vP, eH.vP);
                    eE.v0 = fma(we, P1.v0, eE.v0);
                    eE.vH = fma(we, P1.vH, eE.vH);
                    eE.vE = fma(we, P1.vE, eE.vE);
                    eE.vP = fma(we, P1.vP, eE.vP);
                }
                double H, E, P;
                if (L.nG) {
                    Aff G0 = T(1, 0), G2 = T(1, 2);
                    Aff eP{2.0 * F3.v0 + G0.v0 + G2.v0, 2.0 * F3.vH + G0.vH + G2.vH, 2.0 * F3.vE + G0.vE + G2.vE,
                           2.0 * F3.vP + G0.vP + G2.vP};
                    // (I - coupling) (h', eta', Pi) = rhs by the adjugate: nine
                    // cofactors, one reciprocal of the determinant (a shorter
                    // dependence chain on this one lane than elimination)
                    const double a00 = 1.0 - eH.vH, a01 = -eH.vE, a02 = -eH.vP;
                    const double a10 = -eE.vH, a11 = 1.0 - eE.vE, a12 = -eE.vP;
                    const double a20 = -eP.vH, a21 = -eP.vE, a22 = 1.0 - eP.vP;
                    const double b0 = eH.v0, b1 = eE.v0, b2 = eP.v0;
                    const double c00 = fma(a11, a22, -a12 * a21), c01 = fma(a12, a20, -a10 * a22);
                    const double c02 = fma(a10, a21, -a11 * a20), c10 = fma(a02, a21, -a01 * a22);
                    const double c11 = fma(a00, a22, -a02 * a20), c12 = fma(a01, a20, -a00 * a21);
                    const double c20 = fma(a01, a12, -a02 * a11), c21 = fma(a02, a10, -a00 * a12);
                    const double c22 = fma(a00, a11, -a01 * a10);
                    const double idet = rcp(fma(a00, c00, fma(a01, c01, a02 * c02)));
                    H = fma(c00, b0, fma(c10, b1, c20 * b2)) * idet;
                    E = fma(c01, b0, fma(c11, b1, c21 * b2)) * idet;
                    P = fma(c02, b0, fma(c12, b1, c22 * b2)) * idet;
                } else {
                    double a11 = 1.0 - eH.vH, a12 = -eH.vE, a21 = -eE.vH, a22 = 1.0 - eE.vE;
                    const double idet = rcp(a11 * a22 - a12 * a21);
                    H = (eH.v0 * a22 - a12 * eE.v0) * idet;
                    E = (a11 * eE.v0 - a21 * eH.v0) * idet;
                    P = 0.0;
                }
                m.AX[0] = H;
                m.AX[1] = E;
                m.AX[2] = P;
                m.ry(L.rDC) = aff(dc, H, E, P);
                m.ry(L.rETA) = aff(eta, H, E, P);
                m.ry(L.rDG) = aff(dg, H, E, P);
            }
            wsync();
            // (D) downward substitution, one lane per chain
            if (sweeper) {
                double H = m.AX[0], E = m.AX[1], P = m.AX[2];
                double yprev = 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    yprev = aff(top[j], H, E, P);
                    m.ry(cb + j) = yprev;
                }
                // generic rows: y_j = U_j - V_j y_{j-1}, four at a time with the
                // next block's U, V already in flight (reads stay inside the slab)
                // (rows past the chain end are computed too and their results
                // sent to a spare record)
                double pu[4], pv[4];
                {
                    const double *pb = m.rec(cb + 4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pu[q] = pb[q * STR + F_U];
                        pv[q] = pb[q * STR + F_V];
                    }
                }
                double *const spare = m.rec(-1);
                // one block from (cu, cv) while the next loads into (nu, nv); two
                // blocks per trip with alternating buffers
                auto down_block = [&](const double(&cu)[4], const double(&cv)[4], double(&nu)[4], double(&nv)[4],
                                      int j0) {
                    double *cbk = m.rec(cb + j0);
                    const double *nb = cbk + 4 * STR;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        nu[q] = nb[q * STR + F_U];
                        nv[q] = nb[q * STR + F_V];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        yprev = fma(-cv[q], yprev, cu[q]);
                        double *dst = (j0 + q < cn) ? cbk + q * STR : spare;
                        dst[F_RY] = yprev;
                    }
                };
                double qu[4], qv[4];
                int j0 = 4;
                for (; j0 + 4 < cn; j0 += 8) {
                    down_block(pu, pv, qu, qv, j0);
                    down_block(qu, qv, pu, pv, j0 + 4);
                }
                if (j0 < cn) down_block(pu, pv, qu, qv, j0);
            }
            wsync();
            // (E) row lanes: K = (Y - R)/g
            const double ig = 1.0 / g;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int row = gl * R + r;
                double y = row < N ? m.ry(row) : 0.0;
                double kv = (y - w.rr[r]) * ig;
#pragma unroll
                for (int j = 1; j < NSTG; ++j)
                    if (si == j) w.K[j][r] = kv;
                if (si == NSTG - 1) w.yn[r] = y;
            }
            wsync();
        }
        // error estimate
        double ev[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double e = 0.0;
#pragma unroll
            for (int j = 0; j < NSTG; ++j) e += Ke[j] * w.K[j][r];
            ev[r] = h * e;
        }
        double E = rms(ev, w.y, w.yn);
        ++ns;
        if (!isfinite(E)) {
            st = CMB_K_NONFINITE;
            break;
        }
        double fac;
        if (hin || E <= 1.0) {
            double tn = last ? 0.0 : t + h;
            if (tn >= 0.0) tn = 0.0;
            if (hout && gl == 0 && na + 1 < tb.hist_cap) hout[1 + na] = h;
            if (HIST && hin && tb.traj_out && na - na0 < tb.traj_cap) {
                // the step's record for the reverse sweep: start, size, end,
                // the state it started from and its stage derivatives
                const int TR = traj_rec(N);
                double *q = tb.traj_out + ((size_t)ik * tb.traj_cap + (na - na0)) * TR;
                if (gl == 0) {
                    q[0] = t;
                    q[1] = h;
                    q[2] = tn;
                }
                double *qr = lane_ptr(q + 3 + gl * R);  // as in put_ck
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (gl * R + r < N) {
                        qr[r] = w.y[r];
#pragma unroll
                        for (int j = 0; j < NSTG; ++j) qr[(1 + j) * N + r] = w.K[j][r];
                    }
                }
            }
            ++na;
            double hh = tn - t;
            // the output times inside this step, in batches of up to OUT_SLOTS:
            // the interpolated rows of output b go to record field out_slot(b)
            // and lane b of the group evaluates its sources (per output the
            // same arithmetic as one output at a time)
            const int nb_max = G < OUT_SLOTS ? G : OUT_SLOTS;
            while (jo < n_tau && lo[jo] <= tn) {
                int nb = 1;
                while (nb < nb_max && jo + nb < n_tau && lo[jo + nb] <= tn) ++nb;
                for (int b = 0; b < nb; ++b) {
                    const int fld = out_slot(b);
                    double th = hh > 0.0 ? (lo[jo + b] - t) / hh : 1.0;
                    double th2 = th * th, th3 = th2 * th;
                    double h00 = 2.0 * th3 - 3.0 * th2 + 1.0, h10 = th3 - 2.0 * th2 + th;
                    double h01 = -2.0 * th3 + 3.0 * th2, h11 = th3 - th2;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        m.rec(gl * R + r)[fld] =
                            h00 * w.y[r] + h10 * hh * w.K[0][r] + h01 * w.yn[r] + h11 * hh * w.K[NSTG - 1][r];
                }
                wsync();
                if (gl < nb) {
                    const int jl = jo + gl, fld = out_slot(gl);
                    Bk so;
                    bk_at<MNU>(tb, p, k, lo[jl], so);
                    auto y = [&](int r) { return m.rec(r)[fld]; };
                    double drho = 0.0, rpt = 0.0, rpsn = 0.0;
                    if (MNU) ncdm_moments(m, L, so, tb, k, drho, rpt, rpsn, fld);
                    source_values(so, L, p, k, y, drho, rpt, rpsn, So[jl], So[n_tau + jl], So[2 * n_tau + jl]);
                    if (Dmo) {
                        // sum rho_i delta_i / sum rho_i over CDM, baryons and massive
                        // nu, scaled by a^3 (massive nu: a^-4 eps against a^-3)
                        double num = tb.rt_c0 * y(L.rDC) + tb.rt_b0 * y(0), den = tb.rt_c0 + tb.rt_b0;
                        if (MNU) {
                            const double ia = rcp(so.a);
                            for (int i = 0; i < L.nQ; ++i) {
                                const double w1 = tb.pref_ncdm * tb.W[i] * eps_of(tb.q[i], so.am) * ia;
                                num = fma(w1, y(L.bM + i * L.nPs), num);
                                den += w1;
                            }
                        }
                        Dmo[jl] = num / den;
                    }
                }
                wsync();
                jo += nb;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                w.y[r] = w.yn[r];
                w.K[0][r] = w.K[NSTG - 1][r];
            }
            t = tn;
            if (ckp && na % tb.ck_every == 0) put_ck(na / tb.ck_every);
            const double lE = log(fmax(E, 1e-10));
            fac = 0.9 * exp(-(b1 * lE + b2 * lEp + b3 * lEpp));
            fac = fmin(10.0, fmax(0.2, fac));
            lEpp = lEp;
            lEp = lE;
        } else {
            fac = fmin(0.9, fmax(0.2, 0.9 * pow(E, -1.0 / ERR_ORDER)));
        }
        h *= fac;
        if (!hin && t < 0.0 && h < 1e-12) {
            st = CMB_K_STEP_UNDERFLOW;
            break;
        }
    }
    // a time that is not a number ends the loop as if the mode had finished:
    // report it instead of a result
    if (st == CMB_K_OK && !seg_open && !(t >= 0.0)) st = CMB_K_NONFINITE;
    // matter power spectrum today (App. B.4, eq. PK) from the state at a = 1:
    // 2 pi^2/k^3 P_R(k) [sum rho_i delta_i / sum rho_i]^2 over CDM, baryons and
    // the massive neutrinos (0 for a mode that did not finish)
    if (Pk) {
#pragma unroll
        for (int r = 0; r < R; ++r) m.ry(gl * R + r) = w.y[r];
        wsync();
        if (gl == 0) {
            double val = 0.0;
            if (st == CMB_K_OK) {
                double num = tb.rt_c0 * m.ry(L.rDC) + tb.rt_b0 * m.ry(0), den = tb.rt_c0 + tb.rt_b0;
                if (MNU)
                    for (int i = 0; i < L.nQ; ++i) {
                        const double w1 = tb.pref_ncdm * tb.W[i] * eps_of(tb.q[i], tb.m_over_T);
                        num = fma(w1, m.ry(L.bM + i * L.nPs), num);
                        den += w1;
                    }
                const double dm = num * rcp(den);
                val = 2.0 * M_PI * M_PI * rcp(k * k * k) * tb.A_s * pow(k / tb.k_pivot, tb.n_s - 1.0) * dm * dm;
            }
            Pk[(size_t)c * n_k + ik] = val;
        }
    }
    if (gl == 0) {
        for (; !seg_open && jo < n_tau; ++jo) {
            So[jo] = 0.0;
            So[n_tau + jo] = 0.0;
            So[2 * n_tau + jo] = 0.0;
            if (Dmo) Dmo[jo] = 0.0;
        }
        if (hout) tb.hist_out_n[ik] = na < tb.hist_cap ? na : tb.hist_cap - 1;
        if (items) {
            tb.status[ik] = st;
            tb.nsteps[ik] = ns;
        } else {
            status[(size_t)c * n_k + ik] = st;
            nsteps[(size_t)c * n_k + ik] = ns;
        }
    }
}


// Transposed source functions (reverse mode of App. B.4, eq. source_functions,
// with respect to the state): for every (cosmology, k, output time) from the
// mode's start on, dL/dy of each state row from dL/dS_T0, dL/dS_T1, dL/dS_T2.
// The sources are linear in the state at a fixed time (theta_b' enters
// through the baryon row of the right-hand side, h' and eta' through the
// Einstein constraints), so this is the transpose of that linear map.  A block
// of 64 lanes takes P consecutive output points: their rows (zero where the
// sources do not read) are formed in LDS, one lane per point, and the block's
// contiguous P N doubles then go out in coalesced 64-wide stores.
constexpr int SADJ_LDS = 8192;  // at most this many doubles of LDS per block
template <bool MNU>
__global__ void __launch_bounds__(64) sources_adj_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                         int n_tau, DevPrec p, int P, const double *__restrict__ gS,
                                                         double *__restrict__ gY) {
    extern __shared__ double sg[];  // P rows-long records
    const Lay L = make_lay(p);
    const long total = (long)n_cosmo * n_k * n_tau;
    const long first = (long)blockIdx.x * P;
    const int np = (int)((total - first) < P ? (total - first) : P);  // points of this block
    const int nd = np * L.N;
    for (int i = threadIdx.x; i < nd; i += 64) sg[i] = 0.0;
    __syncthreads();
    if ((int)threadIdx.x < np) {
        const long id = first + threadIdx.x;
        const int j = (int)(id % n_tau);
        const long ck = id / n_tau;
        const int ik = (int)(ck % n_k), c = (int)(ck / n_k);
        sources_adj_point<MNU>(tabs[c], p, L, n_tau, ik, j, gS + ck * 3 * n_tau, sg + threadIdx.x * L.N);
    }
    __syncthreads();
    double *out = gY + first * L.N;
    for (int i = threadIdx.x; i < nd; i += 64) out[i] = sg[i];
}


}  // namespace

// Few modes: wider groups while the launch still fits one round of the
// chip's 1024 wavefront slots (one wavefront per SIMD), so a step's
// row-parallel work is shorter: a whole wavefront per mode with two rows per
// lane up to 1024 modes, 32 lanes with three rows up to 2048.  Per row, per
// chain and in the error norm the arithmetic is that of the narrow groups,
// so results are the same bits in every shape.  (Massless hierarchies whose
// narrow groups have five rows per lane.)
static void wide_shape(const DevPrec &p, long n_sys, int &R, int &G) {
    if (R != 5 || p.nq > 0) return;
    const int N = (p.lg + 2) + (p.lp > 0 ? p.lp + 1 : 0) + (p.ln + 1) + 3;
    const int nch = p.lp > 0 ? 3 : 2;
    if (n_sys <= 1024 && (N + 1) / 2 <= 64 && nch <= 64) {
        R = 2;
        G = 64;
    } else if (n_sys <= 2048 && (N + 2) / 3 <= 32 && nch <= 32) {
        R = 3;
        G = 32;
    }
}

// Many modes: groups of half the narrow width with twice the rows, so that a
// wavefront carries eight modes and the serial chain sweeps and coupling
// solves serve twice as many modes per instruction (the error norm keeps the
// narrow groups' order).  Massless hierarchies whose narrow groups are 16
// lanes of five rows, in launches of at least kDenseModes modes.
constexpr long kDenseModes = 8192;
static void dense_shape(const DevPrec &p, long n_sys, int &R, int &G) {
    if (R != 5 || G != 16 || p.nq > 0 || n_sys < kDenseModes) return;
    R = 10;
    G = 8;
}

bool perturb2_supported(const DevPrec &p) {
    int R, G;
    group_shape(p, R, G);
    const int nch = (p.lp > 0 ? 3 : 2) + p.nq;
    return G <= 64 && (stat_doubles(G * R) + (64 / G) * slab_doubles(G * R, nch)) * sizeof(double) <= 65536 &&
           p.nq <= kMaxQ;
}

static int launch_perturb2_any(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, double *d_S,
                               int *d_status, int *d_nsteps, const int2 *d_items, int n_items, double *d_Pk,
                               double *d_Dm, bool hist, void *stream) {
    int R, G;
    group_shape(p, R, G);
    if (G > 64) {
        set_error("hierarchy too large for the cooperative perturbation kernel");
        return CMB_E_UNSUPPORTED;
    }
    long n_sys = d_items ? (long)n_items : (long)n_cosmo * n_k;
    if (n_sys <= 0) return CMB_OK;
    const int Gn = G;  // the narrow group, whose error-norm order every shape keeps
    wide_shape(p, n_sys, R, G);
    dense_shape(p, n_sys, R, G);
    int spw = 64 / G;
    dim3 grid((unsigned)((n_sys + spw - 1) / spw)), block(64);
    const int nch = (p.lp > 0 ? 3 : 2) + p.nq;
    size_t lds = ((size_t)stat_doubles(G * R) + (size_t)spw * slab_doubles(G * R, nch)) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    const bool mnu = p.nq > 0;
#define CMB_K1_LAUNCH(R_, M_, H_, RN_)                                                                  \
    hipLaunchKernelGGL((perturb2_kernel<R_, M_, H_, RN_>), grid, block, lds, s, d_tabs, n_cosmo, n_k, n_tau, p, G, \
                       Gn, d_S, d_status, d_nsteps, d_items, n_items, d_Pk, d_Dm)
#define CMB_K1_LAUNCH3(R_, M_, H_) CMB_K1_LAUNCH(R_, M_, H_, R_)
    if (G != Gn && R == 10) {  // dense groups (massless) in the order of narrow groups of five rows
        if (hist) CMB_K1_LAUNCH(10, false, true, 5); else CMB_K1_LAUNCH(10, false, false, 5);
    } else if (G != Gn && R == 2) {  // wide groups (massless hierarchies) in the order of narrow groups of five rows
        if (hist) CMB_K1_LAUNCH(2, false, true, 5); else CMB_K1_LAUNCH(2, false, false, 5);
    } else if (G != Gn) {
        if (hist) CMB_K1_LAUNCH(3, false, true, 5); else CMB_K1_LAUNCH(3, false, false, 5);
    } else if (R == 2 && !mnu) {
        if (hist) CMB_K1_LAUNCH3(2, false, true); else CMB_K1_LAUNCH3(2, false, false);
    } else if (R == 2) {
        if (hist) CMB_K1_LAUNCH3(2, true, true); else CMB_K1_LAUNCH3(2, true, false);
    } else if (!mnu) {
        if (hist) CMB_K1_LAUNCH3(5, false, true); else CMB_K1_LAUNCH3(5, false, false);
    } else {
        if (hist) CMB_K1_LAUNCH3(5, true, true); else CMB_K1_LAUNCH3(5, true, false);
    }
#undef CMB_K1_LAUNCH3
#undef CMB_K1_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("perturb2 launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_perturb2(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, double *d_S,
                    int *d_status, int *d_nsteps, double *d_Pk, double *d_Dm, void *stream, bool hist) {
    return launch_perturb2_any(d_tabs, n_cosmo, n_k, n_tau, p, d_S, d_status, d_nsteps, nullptr, 0, d_Pk, d_Dm, hist,
                               stream);
}

int launch_perturb2_items(const DevTab *d_tabs, const WorkItem *d_items, int n_items, const DevPrec &p, void *stream) {
    static_assert(sizeof(WorkItem) == sizeof(int2), "work item layout");
    return launch_perturb2_any(d_tabs, 0, 0, 0, p, nullptr, nullptr, nullptr, reinterpret_cast<const int2 *>(d_items),
                               n_items, nullptr, nullptr, false, stream);
}

int launch_sources_adjoint(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, const double *d_gS,
                           double *d_gY, void *stream) {
    const long n = (long)n_cosmo * n_k * n_tau;
    if (n <= 0) return CMB_OK;
    const int rows = make_lay(p).N;
    int P = SADJ_LDS / rows;  // output points per block, each one lane
    if (P > 64) P = 64;
    if (P < 1) {
        set_error("state too large for the transposed-source kernel");
        return CMB_E_UNSUPPORTED;
    }
    dim3 grid((unsigned)((n + P - 1) / P)), block(64);
    const size_t lds = sizeof(double) * (size_t)P * rows;
    hipStream_t s = (hipStream_t)stream;
    if (p.nq > 0)
        hipLaunchKernelGGL((sources_adj_kernel<true>), grid, block, lds, s, d_tabs, n_cosmo, n_k, n_tau, p, P, d_gS,
                           d_gY);
    else
        hipLaunchKernelGGL((sources_adj_kernel<false>), grid, block, lds, s, d_tabs, n_cosmo, n_k, n_tau, p, P, d_gS,
                           d_gY);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("sources adjoint launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int state_rows(const DevPrec &p) { return make_lay(p).N; }

}  // namespace cmbhip
