/*
 * cmbhip: FP64 hot path of a linear Einstein-Boltzmann CMB solver on AMD
 * Instinct MI355X (gfx950), after arXiv 2602.15104 (ABCMB).
 *
 * The calls follow the paper's problem statement (App. A.2): cosmological
 * parameters, static precision options, a wavenumber grid and ell_max in;
 * source functions, transfer functions and C_ell^{TT,TE,EE} out.
 *
 * Threading: every call is thread-safe with respect to distinct handles.
 * cmb_last_error() is thread-local.  No exception crosses this boundary; each
 * int-returning call returns CMB_OK (0) or one of the CMB_E_* codes below.
 */
#ifndef CMBHIP_H
#define CMBHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMB_ABI_VERSION 4

/* call-level return codes */
enum {
    CMB_OK = 0,
    CMB_E_INVALID = 1,        /* NULL pointer, NaN/non-positive parameter, bad size, unsorted k */
    CMB_E_CONFLICT = 2,       /* Neff and N_nu_massless both given, or tau_reio and z_reio both
                                 given (Sec. 2.4; App. A.2, tau_reion) */
    CMB_E_NEG_NMASSLESS = 3,  /* Neff too small for the other species (Sec. 2.4) */
    CMB_E_ROOT = 4,           /* a root find was not bracketed (z_reion from tau_reio, start times) */
    CMB_E_DEVICE = 5,         /* HIP runtime error */
    CMB_E_NOMEM = 6,          /* device memory budget of the context exceeded */
    CMB_E_UNSUPPORTED = 7     /* option combination not built into this library */
};

/* per-mode integration status written to the status array by the solver */
enum {
    CMB_K_OK = 0,
    CMB_K_MAX_STEPS = 1,      /* max_steps attempted steps before ln a = 0 */
    CMB_K_NONFINITE = 2,      /* NaN/Inf in the error estimate or the time */
    CMB_K_STEP_UNDERFLOW = 3  /* step size fell below 1e-12 in ln a */
};

/* Cosmological parameters (App. A.2, "Cosmological parameters").  NaN means
 * "not given" for tau_reio/z_reio (exactly one must be given) and for
 * Neff/N_nu_massless (at most one; neither means N_nu_massless = 3). */
typedef struct cmb_cosmo {
    double h, omega_b, omega_cdm, A_s, n_s;
    double tau_reio, z_reio;
    double Delta_z_reio, z_reio_He, Delta_z_reio_He, exp_reio;
    double YHe, TCMB0;               /* TCMB0 in eV */
    double Neff, N_nu_massless, T_nu_massless;
    double N_nu_massive, m_nu_massive, T_nu_massive; /* m in eV */
} cmb_cosmo;

/* Static options (App. A.2, "Initialization options").  ell_pol = 0 means no
 * polarisation hierarchy (temperature only: no E, Pi = 2 sigma_gamma). */
typedef struct cmb_prec {
    int ell_gamma, ell_pol, ell_nu, n_q, ell_ncdm;
    int max_steps, n_tab;
    double rtol_small, rtol_large, atol_small, atol_large, k_split;
    double R_tc, R_large, k_pivot;
    double pcoeff, icoeff, dcoeff;
    double scale_sw, scale_isw, scale_dop, scale_pol;
    double gravity_scale, thomson_scale; /* test knobs: 1 = physical */
} cmb_prec;

/* ABI version integer (CMB_ABI_VERSION). */
int cmb_abi_version(void);

/* Fill *c and *p with the paper's defaults (App. A.2).  Either may be NULL
 * only if the other is not; both NULL -> CMB_E_INVALID. */
int cmb_defaults(cmb_cosmo *c, cmb_prec *p);

/* Message for the last failing call on this thread ("" if none).  The
 * pointer stays valid until the next call on the same thread. */
const char *cmb_last_error(void);

/* ---------------------------------------------------------------- tables */
/* Host-built background, recombination and thermodynamics tables for one
 * cosmology (App. A.2 derived parameters, App. B.1 recombination, App. B.2
 * reionisation, App. B.4 kappa and visibility, App. C species), the start
 * time of every mode (App. A.2, eqs. k_start_small/k_start_large) and the
 * output-time grid with its line-of-sight weights.  CPU only.
 *   k:     n_k >= 1 wavenumbers [Mpc^-1], positive, strictly increasing
 *          (copied; the caller keeps ownership of its array)
 *   n_tau: >= 3 output times
 * On success *out is a library-owned immutable handle, shareable between
 * threads, released by cmb_tables_destroy.  Errors: CMB_E_INVALID,
 * CMB_E_CONFLICT, CMB_E_NEG_NMASSLESS, CMB_E_ROOT, CMB_E_UNSUPPORTED. */
typedef struct cmb_tables cmb_tables;
int cmb_tables_build(const cmb_cosmo *c, const cmb_prec *p, const double *k, int n_k, int n_tau,
                     cmb_tables **out);
void cmb_tables_destroy(cmb_tables *t);

/* Read-only view of a table (no ownership transfer; valid while t lives).
 * Knot arrays have n_tab + 1 entries on the uniform grid
 * ln a_j = L0 + j * dlna (j < n_tab), ln a_n_tab = 0.  Spline columns are
 * natural cubic splines given by knot values and second derivatives. */
typedef struct cmb_table_view {
    int n_k, n_tau, n_tab, n_q;
    double L0, dlna, tau0, z_reio, lna_tc, N_massless, Neff, R_nu;
    const double *k, *lna_start;                      /* [n_k] */
    const double *lna_src, *tau_src, *chi_src, *w_src; /* [n_tau] */
    const double *xe, *tm;                            /* [n_tab+1] */
    const double *ln_dk, *kappa, *ln_cs2, *ln_tau;    /* [n_tab+1] knot values */
    const double *M_ln_dk, *M_kappa, *M_ln_cs2, *M_ln_tau; /* [n_tab+1] second derivatives */
    const double *q, *W;                              /* [n_q] momentum rule */
    double rt_g0, rt_ur0, rt_c0, rt_b0, rt_L, pref_ncdm, m_over_T, H0;
    /* lensing (App. B.5): conformal time of the visibility peak (parabola
     * through the three table knots around the largest kappa' e^-kappa),
     * chi_* = tau0 - tau_star, and the Limber weights per output time
     * w_j / chi_j (3/2 a_j^2 rho_m(a_j))^2 ((chi_* - chi_j)/chi_*)^2 for
     * 0 < chi_j < chi_* (else 0), rho_m over CDM, baryons and massive nu in
     * units where H^2 = sum rho (Mpc^-2) */
    double tau_star, chi_star;
    const double *lens_w; /* [n_tau] */
} cmb_table_view;
int cmb_tables_export(const cmb_tables *t, cmb_table_view *out);

/* ---------------------------------------------------------------- device */
/* A context binds one HIP device and owns the device workspace (table
 * copies, integrator scratch), grown on demand up to hbm_budget_bytes
 * (0 = 16 GiB).  One context per host thread.  Calls on one context may name
 * different streams: each call's device work is queued after the device work
 * of the context's previous call (its stream waits for an event the previous
 * call recorded), because calls reuse and regrow the context's buffers; work
 * on one stream is ordered as usual.  Errors: CMB_E_DEVICE, CMB_E_INVALID. */
typedef struct cmb_ctx cmb_ctx;
int cmb_ctx_create(int device, size_t hbm_budget_bytes, cmb_ctx **out);
void cmb_ctx_destroy(cmb_ctx *ctx);

/* Device bytes cmb_solve needs for this batch (tables + integrator scratch),
 * excluding the caller's output buffers.  Used for admission by footprint. */
size_t cmb_solve_workspace_bytes(const cmb_tables *const *tabs, int n_cosmo);

/*
 * Perturbations and sources (App. B.3, App. C, App. B.4 eq. source_functions)
 * for n_cosmo cosmologies that share n_k, n_tau and the hierarchy sizes.
 *   d_S:      device, [n_cosmo][n_k][3][n_tau] doubles: S_T0, S_T1, S_T2
 *             (S_E = sqrt(6) S_T2), zero before each mode's start time;
 *   d_status: device, [n_cosmo][n_k] int32 (CMB_K_*);
 *   d_nsteps: device, [n_cosmo][n_k] int32 attempted steps (may be NULL).
 * Asynchronous on hip_stream (a hipStream_t; NULL = default stream).  Buffers
 * are caller-owned and must stay valid until the stream reaches this work.
 * Hierarchies of more than 320 state rows (cmb_state_rows) or more than 16
 * momentum nodes: CMB_E_UNSUPPORTED, outputs untouched.
 */
int cmb_perturb(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                int32_t *d_nsteps, void *hip_stream);

/* As cmb_perturb, plus the linear matter power spectrum today (App. B.4,
 * eq. PK): P(k, z=0) = 2 pi^2/k^3 A_s (k/k_pivot)^(n_s-1) [sum_i rho_i delta_i
 * / sum_i rho_i]^2 in Mpc^3, the sums over the non-relativistic species (CDM,
 * baryons and massive neutrinos), from each mode's state at a = 1.
 *   d_Pk: device, [n_cosmo][n_k] doubles, caller-owned (0 for a mode whose
 *         status is not CMB_K_OK).
 * Errors as cmb_perturb; CMB_E_UNSUPPORTED for a hierarchy the cooperative
 * perturbation kernel cannot hold. */
int cmb_perturb_pk(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                   int32_t *d_nsteps, double *d_Pk, void *hip_stream);

/*
 * Line-of-sight projection (App. B.4, transfer integrals; trapezoid in ln a):
 * from sources d_S (layout above, any values) to
 *   d_Delta: device, [n_cosmo][2][n_k][ell_max-1] doubles (Delta_T, Delta_E
 *            for ell = 2..ell_max, ell fastest: each mode's multipoles are
 *            contiguous); the E plane is written as 0 when the tables have
 *            no polarisation hierarchy.
 * Bessel functions by recurrence on the GPU; ell_max in [2, 10000]
 * (else CMB_E_INVALID) and n_tau <= 4096 (else CMB_E_UNSUPPORTED: each
 * 256-lane workgroup holds at most 16 output times per lane).
 */
int cmb_los(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S,
            double *d_Delta, void *hip_stream);

/*
 * k quadrature (eq. c_ell_def, eq. PK_pivot; trapezoid in k on the mode grid):
 *   d_Cl: device, [n_cosmo][3][ell_max+1] doubles (TT, TE, EE; dimensionless;
 *         entries ell < 2 are 0).
 */
int cmb_cl(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Delta,
           double *d_Cl, void *hip_stream);

/*
 * The whole path: cmb_perturb, cmb_los, cmb_cl in order on hip_stream.
 * d_S and d_Delta may be NULL (then context scratch is used).  Cosmologies in
 * one call must share n_k, n_tau and the static options' hierarchy sizes.
 */
int cmb_solve(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, double *d_S, double *d_Delta,
              double *d_Cl, int32_t *d_status, int32_t *d_nsteps, void *hip_stream);

/* ------------------------------------------------------ no allocation */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the whole
 * path of cmb_solve with every intermediate -- table copies, sources,
 * transfer functions, step counts when d_nsteps is NULL -- in a fixed device
 * array of CMB_NOALLOC_SCRATCH_MB MiB that the library holds on each device
 * it runs on, from that device's first call until the process ends.  The
 * call allocates nothing: no hipMalloc, hipFree or pinned staging; it needs
 * no context and runs on the current device.
 *   tabs, n_cosmo: as cmb_solve (cosmologies sharing n_k, n_tau and the
 *     static options); their host arrays are copied into the scratch array
 *     on hip_stream, so the tables must stay alive until the stream has
 *     reached this work;
 *   d_Cl [n_cosmo][3][ell_max+1], d_status [n_cosmo][n_k], d_nsteps
 *     [n_cosmo][n_k] (may be NULL): device, caller-owned, as cmb_solve.
 * Asynchronous on hip_stream.  Every call on one device shares that device's
 * array and leaves the last call's intermediates in it: calls that overlap
 * on one device (other streams, other host threads) race, calls on one
 * stream are ordered.  Errors: CMB_E_INVALID as cmb_solve; CMB_E_NOMEM when
 * the batch's tables, sources and transfer functions exceed the array
 * (cmb_noalloc_scratch_bytes; one config-1 cosmology -- 400 modes, 2000
 * output times, l <= 2500 -- needs 36 MiB); CMB_E_UNSUPPORTED and
 * CMB_E_DEVICE as cmb_solve.  On an error nothing is launched and the
 * outputs are untouched. */
#define CMB_NOALLOC_SCRATCH_MB 160
size_t cmb_noalloc_scratch_bytes(void);
int cmb_solve_noalloc(const cmb_tables *const *tabs, int n_cosmo, int ell_max, double *d_Cl, int32_t *d_status,
                      int32_t *d_nsteps, void *hip_stream);

/* ------------------------------------------------------- transfer k-grid */
/* Transfer k-grid of App. A.2 (eq. k_transfer_spacing):
 *   k_{n+1} = k_n + k_period linstep k_n / (k_n + linstep/logstep),
 *   k_period = 2 pi / (tau0_fid - tau_rec_fid),
 * from max(k_min_tau0 / tau0_fid, k_lo) to min(k_max_tau0_over_l_max ell_max
 * / tau0_fid, k_hi), the last point being that upper end, with the paper's
 * default constants (k_min_tau0 0.1, k_max_tau0_over_l_max 1.8, tau0_fid
 * 14186.68 Mpc, tau_rec_fid 281.040565 Mpc, linstep 0.45, logstep 170).
 * Writes at most cap points to k_out (may be NULL when cap = 0) and returns
 * the number of points of the grid (call once with cap = 0 to size it), or
 * -CMB_E_INVALID. */
int cmb_transfer_kgrid(int ell_max, double k_lo, double k_hi, double *k_out, int cap);

/* Spectra on a transfer k-grid: the sources d_S [n_cosmo][n_k][3][n_tau] of
 * the perturbation grid (all cosmologies sharing it) are interpolated in k
 * by natural cubic splines at every output time onto kt, then projected
 * (App. B.4 transfer integrals) and integrated over kt (eq. Cl) as cmb_los
 * and cmb_cl do on the perturbation grid.
 *   kt:      host [n_kt], strictly increasing inside [k_0, k_{n_k-1}]
 *   d_St:    device [n_cosmo][n_kt][3][n_tau], the interpolated sources
 *   d_Delta: device [n_cosmo][2][n_kt][ell_max-1];  d_Cl: device [n_cosmo][3][ell_max+1]
 * Caller-owned buffers, asynchronous on hip_stream.  Errors: CMB_E_INVALID,
 * CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_spectra_on_grid(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S,
                        const double *kt, int n_kt, double *d_St, double *d_Delta, double *d_Cl, void *hip_stream);

/* ---------------------------------------------------- parameter derivatives */
/* Step histories of the perturbation integration (App. A.2 solver options):
 * cmb_perturb_record runs cmb_perturb and writes, per mode, the start ln a_i
 * and the size of every accepted step into d_hist[n_cosmo][n_k][hist_cap]
 * (entry 0 the start) with the counts in d_hist_n[n_cosmo][n_k];
 * cmb_perturb_replay integrates each mode from its recorded start with
 * exactly those steps and no error control (the same tables replay a run bit
 * for bit; other tables give the frozen-step discrete map, whose finite
 * differences carry no step-control noise).  hist_cap >= max_steps + 1.
 * Errors as cmb_perturb. */
int cmb_perturb_record(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                       int32_t *d_nsteps, double *d_hist, int32_t *d_hist_n, int hist_cap, void *hip_stream);
int cmb_perturb_replay(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, const double *d_hist,
                       const int32_t *d_hist_n, int hist_cap, double *d_S, int32_t *d_status, int32_t *d_nsteps,
                       void *hip_stream);

/* Trajectory checkpoints of the ESDIRK integration (section 3 and the
 * integrator's adjoint option in App. A.2: reverse-mode differentiation
 * through the integrator needs the forward states again, the memory cost the
 * paper notes; checkpoints every few steps bound it to one segment of steps
 * plus the checkpoints, each segment recomputed from its own).
 * cmb_perturb_checkpoint is cmb_perturb_record (replay = 0) or
 * cmb_perturb_replay (replay != 0) that also writes, per mode, the record
 *   d_ck[n_cosmo][n_k][ck_cap][1 + 2 N]  (N = cmb_state_rows):
 *   ln a, the N state rows, and the N rows of the stage derivative the next
 *   step starts from (the last stage of the step just taken),
 * slot j after j * every accepted steps (slot 0 the start); slots past a
 * mode's last step are left unwritten.  Sources, status and counts as the
 * record or replay call.
 * cmb_perturb_segment replays, for every mode, only the accepted steps
 * seg * every + 1 .. (seg + 1) * every of d_hist, starting from checkpoint
 * slot seg, and writes only the source entries of the output times those
 * steps reach (segment 0 also the zeros before the start, the last segment
 * the outputs after an abort): run over every segment into one d_S it
 * reproduces cmb_perturb_replay's sources bit for bit, whatever the order.
 * A mode whose history ends at or before step seg * every is left alone
 * (status 0, count 0); status CMB_K_MAX_STEPS when the history ends inside
 * the segment before a = 1.  d_ck must come from cmb_perturb_checkpoint
 * with the same tables, history, every and ck_cap.
 * Needs every >= 1, ck_cap >= (hist_cap - 1) / every + 1,
 * 0 <= seg < ck_cap and seg * every < hist_cap (else CMB_E_INVALID);
 * otherwise errors as cmb_perturb. */
int cmb_perturb_checkpoint(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int replay, double *d_hist,
                           int32_t *d_hist_n, int hist_cap, int every, double *d_ck, int ck_cap, double *d_S,
                           int32_t *d_status, int32_t *d_nsteps, void *hip_stream);
int cmb_perturb_segment(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, const double *d_hist,
                        const int32_t *d_hist_n, int hist_cap, int every, const double *d_ck, int ck_cap, int seg,
                        double *d_S, int32_t *d_status, int32_t *d_nsteps, void *hip_stream);

/* Spectra and their derivatives with respect to theta = (h, omega_b,
 * omega_cdm, ln A_s, n_s, tau_reio) for a batch of cosmologies sharing one k
 * grid (each with tau_reio given):
 *   d_Cl: device [n_cosmo][3][ell_max+1]  TT, TE, EE as cmb_solve;
 *   d_J:  device [n_cosmo][6][3][ell_max+1]  dC/dtheta_p.
 * For h, omega_b, omega_cdm and tau_reio the host builds the tables at
 * theta_p (1 +- rel) (and +- 2 rel for order 4) on worker threads; every
 * perturbed cosmology replays its base cosmology's recorded steps, and the
 * spectra combine by the central (order 2) or five-point (order 4) stencil
 * with step e = rel theta_p.  dC/d ln A_s = C; dC/dn_s is the k quadrature
 * with P(k) ln(k/k_pivot).  d_status [n_cosmo][n_k]: the base run's status,
 * or a failing replay's.  0 < rel <= 0.01.  Synchronises hip_stream before
 * returning (the perturbed tables are temporary).  Errors: CMB_E_INVALID,
 * CMB_E_UNSUPPORTED, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_jacobian(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, double rel, int order,
                 double *d_Cl, double *d_J, int32_t *d_status, void *hip_stream);

/* Gradient of a scalar L of the spectra with respect to theta = (h, omega_b,
 * omega_cdm, ln A_s, n_s, tau_reio), by the discrete adjoint of the whole
 * path (section 3; App. A.2, the integrator's reverse-mode adjoint with
 * recursive checkpoints): given dL/dC_l, the spectra and dL/dtheta for a
 * batch of cosmologies (each with tau_reio given), in one call:
 *   1. the base run, recording each mode's accepted steps and a checkpoint
 *      (state and carried stage derivative) every 64 of them; projection and
 *      k quadrature to C_l;
 *   2. dL/dS by the transposes of the k quadrature and the projection
 *      (cmb_spectra_adjoint);
 *   3. segment by segment, last first: a replay of the segment's steps from
 *      its checkpoint that keeps every step's stages, then the reverse
 *      sweep over them: per step, the transposed dense output forced by the
 *      transposed source functions at the output times inside it, and per
 *      implicit stage (last to first) the transposed stage solve
 *      (I - h gamma A)^T, the transposed A and the stage weights.  The
 *      steps are frozen (the derivative of the recorded discrete map);
 *   4. the tables' dependence on h, omega_b, omega_cdm and tau_reio as
 *      central differences of the tables at theta_p (1 +- rel), built on
 *      host threads: contracted with the sweep's stage adjoints (the stage
 *      matrices, the sources at fixed state, the initial conditions) and,
 *      for the projection's geometry, as the spectra of the base sources
 *      under the perturbed tables;
 *   5. dL/d ln A_s = sum dL/dC_l C_l, and dL/dn_s from the k quadrature
 *      weighted by ln(k/k_pivot).
 *   d_gCl:   device [n_cosmo][3][ell_max+1] dL/dC_l (TT, TE, EE; l < 2 ignored);
 *   d_Cl:    device [n_cosmo][3][ell_max+1] the spectra (output, as cmb_solve);
 *   d_grad:  device [n_cosmo][6] dL/dtheta (output);
 *   d_status: device [n_cosmo][n_k] the base run's per-mode status, or a
 *            failing segment replay's;
 *   d_dLdy0: device [n_cosmo][n_k][cmb_state_rows] dL/dy at each mode's start
 *            state (before the initial conditions' own dependence on theta),
 *            or NULL.
 * 0 < rel <= 0.01.  Massless neutrinos only (CMB_E_UNSUPPORTED otherwise).
 * Workspace from the context: about 250 MB per cosmology of config-1 size
 * (400 modes, 2000 output times, l <= 2500).  Synchronises hip_stream before
 * returning (the perturbed tables are temporary).  Errors: CMB_E_INVALID,
 * CMB_E_UNSUPPORTED, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_gradient(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_gCl,
                 double rel, double *d_Cl, double *d_grad, int32_t *d_status, double *d_dLdy0, void *hip_stream);

/* Reverse mode of the spectrum side (the first two steps of the discrete
 * adjoint): given dL/dC_l for a scalar L of the spectra, the gradient with
 * respect to the sources, dL/dS, through the transposes of the k quadrature
 * (eq. c_ell_def) and of the line-of-sight projection (App. B.4):
 *   G_T = 4 pi w_k P(k)/k (2 gTT Delta_T + gTE Delta_E),
 *   G_E = 4 pi w_k P(k)/k (gTE Delta_T + 2 gEE Delta_E),
 *   dL/dS_T0 = w_j sum_l G_T j_l,  dL/dS_T1 = w_j sum_l G_T j_l',
 *   dL/dS_T2 = w_j sum_l [s_pol G_T (3 j_l'' + j_l)/2 + c_l sqrt(6) G_E j_l/x^2],
 * with the projection kernel's Bessel recurrence and cut.
 *   d_Delta: device [n_cosmo][2][n_k][ell_max-1] (cmb_los at these sources);
 *   d_gCl:   device [n_cosmo][3][ell_max+1] dL/dC_l (TT, TE, EE; l < 2 ignored);
 *   d_gS:    device [n_cosmo][n_k][3][n_tau] dL/dS.
 * Asynchronous on hip_stream.  Errors: CMB_E_INVALID, CMB_E_UNSUPPORTED,
 * CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_spectra_adjoint(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Delta,
                        const double *d_gCl, double *d_gS, void *hip_stream);

/* Rows of one mode's perturbation state for these tables' hierarchy, in the
 * order the perturbation kernel keeps them (the row index of
 * cmb_sources_adjoint's output):
 *   [delta_b, theta_b, theta_g, F_g2 .. F_g,lmax]     ell_gamma + 2 rows
 *   [G_0 .. G_lpol]                                     ell_pol + 1 (none if 0)
 *   [delta_nu, theta_nu, F_nu2 .. F_nu,lmax]          ell_nu + 1
 *   [Psi_0 .. Psi_lncdm] per momentum node             n_q (ell_ncdm + 1)
 *   [delta_c, eta, delta_g]                             3
 * (F_2 = 2 sigma, photon and neutrino; App. B.3 and App. C variables).
 * Returns that count (> 0), or -CMB_E_INVALID for a NULL table. */
int cmb_state_rows(const cmb_tables *tab);

/* Reverse mode of the source functions (App. B.4, eq. source_functions),
 * the third step of the spectrum's reverse sweep after cmb_spectra_adjoint:
 * at a fixed output time the sources are linear in the state (theta_b'
 * through the right-hand side's baryon row, h' and eta' through the Einstein
 * constraints), so dL/dy = (dS/dy)^T dL/dS at every output time.
 *   d_gS: device [n_cosmo][n_k][3][n_tau]  dL/dS_T0, dL/dS_T1, dL/dS_T2
 *         (cmb_spectra_adjoint's layout);
 *   d_gY: device [n_cosmo][n_k][n_tau][cmb_state_rows] dL/dy, rows as
 *         cmb_state_rows lists; zero before each mode's start time (no
 *         sources there) and in the rows the sources do not read.
 * n_cosmo * n_k * n_tau * rows doubles (506 MB for one config-1 cosmology):
 * callers with large batches pass them in parts.  Asynchronous on
 * hip_stream.  Errors: CMB_E_INVALID, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_sources_adjoint(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, const double *d_gS, double *d_gY,
                        void *hip_stream);

/* ---------------------------------------------------------------- lensing */
/* cmb_perturb plus the matter outputs (App. B.4 eq. PK, App. B.5): either
 * pointer may be NULL, not both.
 *   d_Pk: device [n_cosmo][n_k], P(k, z = 0) in Mpc^3 as cmb_perturb_pk;
 *   d_Dm: device [n_cosmo][n_k][n_tau], the matter density contrast
 *         delta_m = sum rho_i delta_i / sum rho_i over CDM, baryons and
 *         massive neutrinos at every output time (synchronous gauge; zero
 *         before the mode's start time and after a failed integration).
 * Errors as cmb_perturb; CMB_E_UNSUPPORTED for hierarchies the cooperative
 * kernel does not hold. */
int cmb_perturb_matter(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                       int32_t *d_nsteps, double *d_Pk, double *d_Dm, void *hip_stream);

/* Lensing-potential spectrum by Limber's approximation (App. B.5):
 *   C_l^psipsi = 8 pi^2/(l+1/2)^3 sum_j W_j P_R(k_j) delta_m(k_j, tau_j)^2 / k_j^4,
 *   k_j = (l+1/2)/chi_j,
 * W_j the tables' Limber weights (cmb_table_view.lens_w: time quadrature,
 * 1/chi, (3/2 a^2 rho_m)^2 and ((chi_* - chi)/chi_*)^2), delta_m(k, tau_j) the
 * natural cubic spline in k of d_Dm at output time j, zero outside
 * [k_0, k_{n_k-1}].
 *   d_Dm:   device [n_cosmo][n_k][n_tau] from cmb_perturb_matter;
 *   d_Clpp: device [n_cosmo][ell_max+1], zero for l < 2.
 * All cosmologies of one call share the perturbation k grid.  Asynchronous
 * on hip_stream (synchronises it once before staging the spline factors).
 * Errors: CMB_E_INVALID, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_lensing_potential(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Dm,
                          double *d_Clpp, void *hip_stream);

/* Lensed CMB spectra (App. B.5) from full-sky correlation functions, after
 * the correlation-function method the paper implements (Challinor & Lewis
 * 2005): the deflection correlations C_gl and C_gl,2, sigma^2 = C_gl(0) -
 * C_gl(beta), the small-deflection X functions, and the lensed correlation
 * functions xi_T, xi_+, xi_-, xi_x to second order in C_gl,2, transformed back
 * by an n_mu-point Gauss-Legendre rule over the whole range -1 <= cos(beta)
 * <= 1 (the restricted-range "fast" variant is not offered).  Only the lensing
 * change of each correlation function is transformed and added to the
 * unlensed spectra.
 *   d_Cl:   device [n_cosmo][3][L+1] unlensed TT, TE, EE (cmb_cl's layout, l < 2 ignored);
 *   d_Clpp: device [n_cosmo][L+1] lensing-potential spectrum (cmb_lensing_potential);
 *   d_Cll:  device [n_cosmo][4][ell_max+1] lensed TT, TE, EE, BB (zero for l < 2).
 * Multipoles above L are taken as zero, so results near L miss the power
 * that lensing moves down from above it: choose ell_max well below L (several
 * hundred).  2 <= ell_max <= L <= 20000; n_mu of about L + ell_max/2 or more.
 * The first call for a new (L, n_mu) builds the node tables on the host and
 * synchronises hip_stream.  Errors: CMB_E_INVALID, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_lensed_cl(cmb_ctx *ctx, int n_cosmo, int L, const double *d_Cl, const double *d_Clpp, int ell_max, int n_mu,
                  double *d_Cll, void *hip_stream);

/* ------------------------------------------- three-region Bessel variant */
/* The paper's three-region spherical Bessel scheme (App. B.4, below the
 * transfer integrals): for each l >= 1, j_l = 0 up to x_start(l) (the first x
 * where j_l reaches 1e-10), linear interpolation on 5000 equally spaced exact
 * samples over [x_start(l), x_5(l)] (x_5 the fifth local maximum of j_l), and
 * the leading Debye-type asymptotic form above x_5.
 *
 * cmb_bessel3_table: the context's table for 1 <= l <= ell_max, built on the
 * device at the first call that needs it (and rebuilt whole for a larger
 * ell_max), copied to host arrays: h_xs[ell_max] = x_start, h_x5[ell_max] =
 * x_5, h_tab[ell_max][5000] = j_l at x_start + i (x_5 - x_start)/4999 (index
 * l - 1; any pointer may be NULL).  Synchronous.  Errors: CMB_E_INVALID,
 * CMB_E_DEVICE (also when a root search fails), CMB_E_NOMEM (the table takes
 * 8 (5002 ell_max) bytes of the context's budget). */
int cmb_bessel3_table(cmb_ctx *ctx, int ell_max, double *h_xs, double *h_x5, double *h_tab);

/* cmb_los with the three-region scheme in place of the exact recurrence:
 * the same arguments, layouts and errors; j_l' = j_{l-1} - (l+1) j_l / x and
 * j_l'' from Bessel's equation, both from the scheme's values.  A speed and
 * accuracy variant of the projection; the first call for a larger ell_max
 * builds the table and synchronises hip_stream. */
int cmb_los_bessel3(cmb_ctx *ctx, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S,
                    double *d_Delta, void *hip_stream);

/* ---------------------------------------------------------------- serving */
/*
 * Continuous-batching runtime for independent spectrum requests (each one
 * cosmology with its own k grid, output-time count and ell_max; the whole
 * path of App. B.1-B.4 per request).  Requests are submitted from any host
 * thread; host tables are built on a pool of worker threads; a scheduler
 * thread admits ready requests while their device footprint (tables,
 * sources, transfer functions, spectra) fits the server's HBM arena, launches
 * them as one perturbation launch over the work list of all their modes
 * (longest first), then each request's projection and k quadrature, on up to
 * n_streams HIP streams so that consecutive batches overlap on the device.
 * All requests of one server must share the hierarchy options of cmb_prec
 * (ell_gamma, ell_pol, ell_nu, n_q, ell_ncdm, max_steps, controller and
 * switch options) and have n_tau <= 4096.
 */
typedef struct cmb_server cmb_server;
typedef struct cmb_server_opts {
    int n_workers;            /* host table-builder threads (0 = 4) */
    int n_streams;            /* batches in flight on the device (0 = 2, at most 4) */
    int max_batch;            /* requests per batch (0 = 64; 1 = one request at a time) */
    size_t hbm_budget_bytes;  /* device arena (0 = 8 GiB) */
} cmb_server_opts;

/* Timing of one request, seconds on the server's monotonic clock
 * (submit = 0 at cmb_server_create). */
typedef struct cmb_request_times {
    double submit, tables_ready, launched, done;
    int batch_size; /* requests in the batch it ran in */
} cmb_request_times;

/* Create a server on HIP device `device` (opts may be NULL for defaults).
 * Errors: CMB_E_INVALID, CMB_E_DEVICE, CMB_E_NOMEM. */
int cmb_server_create(int device, const cmb_server_opts *opts, cmb_server **out);

/* Queue one request; k[n_k] is copied.  *ticket identifies it in
 * cmb_server_wait.  Returns at once; table-build errors are reported by
 * cmb_server_wait.  Errors now: CMB_E_INVALID (NULL, sizes, options that
 * differ from the server's first request). */
int cmb_server_submit(cmb_server *s, const cmb_cosmo *c, const cmb_prec *p, const double *k, int n_k, int n_tau,
                      int ell_max, uint64_t *ticket);

/* Wait up to timeout_s seconds (< 0: forever) for a request.  On completion
 * copies its spectra to host Cl[3][ell_max+1] (TT, TE, EE), and optionally
 * status[n_k] (CMB_K_* per mode) and *times, then forgets the ticket.
 * Returns CMB_OK, the request's table-build or device error code,
 * CMB_E_NOMEM if it can never fit the arena, or -1 on timeout (the ticket
 * stays valid). */
int cmb_server_wait(cmb_server *s, uint64_t ticket, double timeout_s, double *Cl, int32_t *status,
                    cmb_request_times *times);

/* Drain: waits for every request in flight, then releases the server. */
void cmb_server_destroy(cmb_server *s);

/* Host self-test of the server's device-arena allocator (no GPU used):
 * random allocation/release sequences checked for overlap, bounds and full
 * coalescing.  Returns 0 on success. */
int cmb_server_selftest_arena(unsigned seed, int n_ops);

#ifdef __cplusplus
}
#endif
#endif /* CMBHIP_H */
