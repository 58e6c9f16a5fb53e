// Internal types shared by the host table builder, the C ABI and the kernel
// launchers of libcmbhip.  Not part of the public interface.
#pragma once

#include <limits>
#include <string>
#include <vector>

#include "../../include/cmbhip.h"

namespace cmbhip {

constexpr int kMaxQ = 16;  // most momentum nodes of the massive-neutrino rule

// Host tables of one cosmology (see tables.cpp).
struct Tables {
    cmb_cosmo cosmo{};
    cmb_prec prec{};
    std::vector<double> k, lna_start;
    int n_tab = 0;
    double L0 = 0, dl = 0, tau0 = 0, z_reio = 0, lna_tc = 0, N_massless = 0, Neff = 0, R_nu = 0;
    double rt_g0 = 0, rt_ur0 = 0, rt_c0 = 0, rt_b0 = 0, rt_L = 0, pref_ncdm = 0, m_over_T = 0, H0 = 0;
    std::vector<double> q, W;
    std::vector<double> xe, tm;
    std::vector<double> col[4], M[4];  // ln dk, kappa, ln cs2, ln tau: knot values, second derivatives
    std::vector<double> poly;          // [n_tab][4 columns][4 coefficients]
    std::vector<double> lna_src, tau_src, chi_src, w_src;
    double lna_star = 0, tau_star = 0, chi_star = 0;  // visibility peak
    std::vector<double> lens_w;                        // [n_tau] Limber weights
    unsigned long long uid = 0;
    double eval(int column, double lna) const;
};

int build_tables(const cmb_cosmo &c, const cmb_prec &p, const double *k, int n_k, int n_tau, Tables &T);
void set_error(const std::string &msg);

// Per-cosmology view the kernels read (device pointers into the context's
// table buffer, plus scalars).
struct DevTab {
    const double *poly;       // [n_tab][16]
    const double *k;          // [n_k]
    const double *lna_start;  // [n_k]
    const double *lna_src;    // [n_tau]
    const double *chi_src;    // [n_tau]
    const double *w_src;      // [n_tau]
    const double *q, *W;      // [n_q] massive-neutrino momentum rule (n_q = 0: none)
    const double *lens_w;     // [n_tau] Limber weights of the lensing potential
    double *S;                // work-list launches only: this cosmology's [n_k][3][n_tau] sources
    int *status, *nsteps;     //   and [n_k] status / step counts
    // accepted-step histories [n_k][hist_cap] (entry 0: start, then the size
    // of every accepted step): replayed from hist_in (no error control)
    // and/or recorded into hist_out with their counts; NULL when unused
    const double *hist_in;
    const int *hist_in_n;
    double *hist_out;
    int *hist_out_n;
    int hist_cap, hist_pad;
    // trajectory checkpoints [n_k][ck_cap][1 + 2 N] (ln a, the N state rows,
    // the stage derivative the next step starts from) at the start and after
    // every ck_every-th accepted step, written to ck_out; with ck_in (and
    // hist_in), each mode replays only its accepted steps
    // ck_seg ck_every + 1 .. (ck_seg + 1) ck_every from checkpoint ck_seg and
    // writes only the outputs those steps reach; NULL when unused
    double *ck_out;
    const double *ck_in;
    int ck_every, ck_cap, ck_seg, ck_pad;
    // step trajectory of a replay (for the reverse sweep): per accepted step
    // of the replayed steps (a segment's, counted from its first), the record
    // [t_n, h, t_{n+1}, y_n (N), K_0 .. K_{s-1} (s N)] in traj_out
    // [n_k][traj_cap][traj_rec(N)]; NULL when unused
    double *traj_out;
    int traj_cap, traj_pad;
    double L0, inv_dl;
    int n_tab, n_k, n_tau, pad;
    double tau0, R_nu;
    double rt_g0, rt_ur0, rt_c0, rt_b0, rt_L;
    double pref_ncdm, m_over_T;  // massive nu: rho = pref a^-4 sum W eps, eps = sqrt(q^2 + (a m/T)^2)
    double A_s, n_s, k_pivot;
    double chi_star;
    double rtol_small, rtol_large, atol_small, atol_large, k_split;
};

// doubles of one step-trajectory record for N state rows (the ESDIRK's six
// stage derivatives)
constexpr int kTrajStages = 6;
constexpr int traj_rec(int N) { return 3 + (1 + kTrajStages) * N; }

// Static options shared by one launch.
struct DevPrec {
    int lg, lp, ln, max_steps;
    int nq, lq;  // massive-neutrino momentum nodes (0: none) and their hierarchy cut-off
    double pcoeff, icoeff, dcoeff;
    double sw, isw, dop, pol, grav, thom;
};

// table arrays of one cosmology packed for the device: count, and packing
// into host staging hp whose device copy will sit at dp (fills the DevTab)
size_t table_doubles(const Tables &t);
void pack_table(const Tables &t, double *hp, const double *dp, DevTab &x);

// The descriptor of table t whose arrays sit one after another from device
// address dp, in the order of the calls put(host array, doubles, device
// address) that this makes (table_doubles(t) doubles in all).
template <class Put>
void describe_table(const Tables &t, const double *dp, DevTab &x, Put put) {
    size_t o = 0;
    auto at = [&](const std::vector<double> &v) {
        const double *r = dp + o;
        put(v.data(), v.size(), r);
        o += v.size();
        return r;
    };
    x = DevTab{};
    x.poly = at(t.poly);
    x.k = at(t.k);
    x.lna_start = at(t.lna_start);
    x.lna_src = at(t.lna_src);
    x.chi_src = at(t.chi_src);
    x.w_src = at(t.w_src);
    x.q = at(t.q);
    x.W = at(t.W);
    x.lens_w = at(t.lens_w);
    x.chi_star = t.chi_star;
    x.pref_ncdm = t.pref_ncdm;
    x.m_over_T = t.m_over_T;
    x.L0 = t.L0;
    x.inv_dl = 1.0 / t.dl;
    x.n_tab = t.n_tab;
    x.n_k = (int)t.k.size();
    x.n_tau = (int)t.lna_src.size();
    x.tau0 = t.tau0;
    x.R_nu = t.R_nu;
    x.rt_g0 = t.rt_g0;
    x.rt_ur0 = t.rt_ur0;
    x.rt_c0 = t.rt_c0;
    x.rt_b0 = t.rt_b0;
    x.rt_L = t.rt_L;
    x.A_s = t.cosmo.A_s;
    x.n_s = t.cosmo.n_s;
    x.k_pivot = t.prec.k_pivot;
    x.rtol_small = t.prec.rtol_small;
    x.rtol_large = t.prec.rtol_large;
    x.atol_small = t.prec.atol_small;
    x.atol_large = t.prec.atol_large;
    x.k_split = t.prec.k_split;
}
// launch options of a hierarchy (nq: momentum nodes actually present)
DevPrec dev_prec(const cmb_prec &p, int nq);

// What the cosmologies of one call share; check_batch validates a batch
// (non-empty, no NULL table, equal n_k, n_tau and static options) and fills
// it, or sets the error text and returns CMB_E_INVALID.
struct Batch {
    int n_k = 0, n_tau = 0;
    DevPrec prec{};
    int polar = 0;
    double s_pol = 1.0;
};
int check_batch(const cmb_tables *const *tabs, int n_cosmo, Batch &b);
const Tables &tables_of(const cmb_tables *t);

// kernel launchers (hipStream_t passed as void*)
int launch_perturb2(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, double *d_S,
                    int *d_status, int *d_nsteps, double *d_Pk, double *d_Dm, void *stream, bool hist = false);
bool perturb2_supported(const DevPrec &p);
// work list of (cosmology, mode) pairs; outputs through each DevTab's S/status/nsteps
struct WorkItem {
    int c, ik;
};
int launch_perturb2_items(const DevTab *d_tabs, const WorkItem *d_items, int n_items, const DevPrec &p, void *stream);
int launch_los(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E, double s_pol,
               const double *d_S, double *d_Delta, void *stream);
int launch_cl(const DevTab *d_tabs, int n_cosmo, int n_k, int ell_max, const double *d_Delta, double *d_Cl,
              void *stream);
int los_max_tau();
// reverse mode of K3 then K2: dL/dC_l -> G = dL/dDelta (workspace, Delta's
// layout) -> dL/dS in the sources' layout
// transposed source functions: gS [n_cosmo][n_k][3][n_tau] -> gY [n_cosmo][n_k][n_tau][state_rows(p)]
int launch_sources_adjoint(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, const DevPrec &p, const double *d_gS,
                           double *d_gY, void *stream);
int state_rows(const DevPrec &p);
// reverse sweep of K1 over segment seg (steps seg*every .. of each mode, in
// reverse) from the step trajectories d_traj [n_cosmo][n_k][traj_cap]
// [traj_rec(N)] of that segment's replay, forced by d_gS (the sources'
// adjoint); carries (dL/dy, dL/dK_0) [n_cosmo][n_k][2N] in d_lam between
// segments and sums dL/dtheta of (h, omega_b, omega_cdm, tau_reio) per mode
// into d_grad [n_cosmo][n_k][4]; first != 0 for the first launch (the last
// segment: nothing carried in).  d_ptabs holds 8 sets of n_cosmo tables,
// set 2p at theta_p (1 + eps), set 2p + 1 at theta_p (1 - eps); d_pden
// [n_cosmo][4] = 2 eps theta_p.  Massless neutrinos only.
bool adjoint_supported(const DevPrec &p);
int launch_adjoint_segment(const DevTab *d_tabs, const DevTab *d_ptabs, const double *d_pden, int n_cosmo, int n_k,
                           int n_tau, const DevPrec &p, const double *d_traj, int traj_cap, const int *d_hist_n,
                           int seg, int every, const double *d_gS, double *d_lam, double *d_grad, int first,
                           void *stream);
// dL/dtheta [n_cosmo][6] = (h, omega_b, omega_cdm, ln A_s, n_s, tau_reio) from
// dL/dC_l, C_l, the n_s-weighted C_l, the spectra of the unperturbed sources
// under the perturbed tables Cp [8][n_cosmo][3][ell_max+1] (sets as d_ptabs),
// d_pden and the reverse sweep's per-mode sums
int launch_grad_assemble(int n_cosmo, int n_k, int ell_max, const double *d_gCl, const double *d_Cl,
                         const double *d_Cns, const double *d_Cp, const double *d_pden, const double *d_adj,
                         double *d_grad, void *stream);
int launch_spectra_adjoint(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E,
                           double s_pol, const double *d_Delta, const double *d_gC, double *d_G, double *d_gS,
                           void *stream);
// K3 with an output stride per cosmology and optionally the ln(k/k_pivot)
// weight (dC/dn_s); finite-difference stencils and replay status merging
int launch_cl_ex(const DevTab *d_tabs, int n_cosmo, int n_k, int ell_max, const double *d_Delta, double *d_Cl,
                 long out_stride, int dlog, void *stream);
int launch_fd(int n_base, int ell_max, int order, const double *d_C, const double *d_e, double *d_J, long j_stride,
              void *stream);
int launch_merge_status(int n_base, int n_k, int n_rep, const int *d_rep, int *d_st, void *stream);
// sources of the perturbation grid interpolated in k onto kt (natural cubic
// splines; elimination factors lo/dinv and intervals seg from the host); M is
// workspace of the size of S
int launch_spline_sources(const double *d_S, double *d_M, const double *d_kg, const double *d_lo,
                          const double *d_dinv, const int *d_seg, const double *d_kt, double *d_St, int n_cosmo,
                          int n_k, int n_tau, int n_kt, void *stream);
int ell_cut(double x);  // host copy of the Bessel cut rule (tests)
// spline second derivatives in k of F[n_cosmo][n_k][nty][n_tau] (one system
// per (cosmology, type, time)) into M of the same layout
int launch_spline_m(const double *d_F, double *d_M, const double *d_kg, const double *d_lo, const double *d_dinv,
                    int n_cosmo, int n_k, int nty, int n_tau, void *stream);
// m-point Gauss-Legendre nodes (descending) and weights on [-1, 1]
void gauss_legendre_nodes(int m, std::vector<double> &x, std::vector<double> &w);
// lensed spectra from full-sky correlation functions: host tables (nodes mu,
// weights w, recurrence coefficients coef[L+1][13][3], X-function factors
// lfac[L+1][4], start values start[13][n_mu]), workspace xi[n_cosmo][4][n_mu]
// and part[n_cosmo][blocks][4][lmax+1]
int lens_back_blocks(int n_mu);
int launch_lensed_cl(int n_cosmo, int L, int lmax, int n_mu, const double *d_Cl, const double *d_Clpp,
                     const double *d_mu, const double *d_w, const double *d_coef, const double *d_lfac,
                     const double *d_start, double *d_xi, double *d_part, double *d_Cll, void *stream);
// lensing potential by Limber's approximation (App. B.5): Clpp[c][0..ell_max]
// from the matter density contrast Dm[c][n_k][n_tau] and its spline M in k
int launch_limber(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, const double *d_Dm,
                  const double *d_M, double *d_Clpp, void *stream);
// three-region Bessel scheme: samples per multipole, table build for
// l_lo..l_hi (x_start[l-1], x_5[l-1] (NaN if not found), tab[l-1][B3_PTS]) and
// the projection with it
constexpr int B3_PTS = 5000;
int launch_bessel3_build(int l_lo, int l_hi, double *d_xs, double *d_x5, double *d_tab, void *stream);
int launch_los3(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E, double s_pol,
                const double *d_S, const double *d_xs, const double *d_x5, const double *d_tab, double *d_Delta,
                void *stream);

}  // namespace cmbhip
