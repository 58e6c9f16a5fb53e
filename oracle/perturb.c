/*
 * CPU oracle, part 2: synchronous-gauge perturbations of one Fourier mode.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference the HIP library is
 * checked against.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code with the library.
 *
 * What it computes (arXiv 2602.15104):
 *   - the right-hand side y' = f(ln a, y) exactly as the species equations of
 *     App. C are written (CDM, baryons, photon temperature F_l and
 *     polarisation G_l, massless neutrinos, massive-neutrino Psi_l(q)), with
 *     the metric equations of App. B.3 (eqs. hprime, etaprime) and the
 *     massive-neutrino sums of eq. mnu_sum (here with an n-node Gauss rule
 *     for the weight q^2/(e^q+1));
 *     readings taken where the printed equations are garbled:
 *       * the photon shear Thomson term is -(9/10) sigma_gamma/(Hc tau_c);
 *       * the polarisation source is (1/2)(Pi/(Hc tau_c)) (delta_l0 + delta_l2/5);
 *   - adiabatic superhorizon initial conditions, leading order in k tau
 *     (Ma & Bertschinger 1995, eqs. 96 and 97), normalised to eta -> 1;
 *   - an ESDIRK time stepper: the six-stage, order-4, L-stable, stiffly
 *     accurate implicit part of Kennedy & Carpenter's additive scheme
 *     ARK4(3)6L[2]SA (Appl. Numer. Math. 44, 2003) with its order-3 embedded
 *     estimate; every implicit stage is one linear solve of
 *     (I - h gamma A) Y = R because the system is linear, done here on the
 *     dense matrix A (built column by column from f) by Gaussian elimination
 *     with partial pivoting and two steps of iterative refinement;
 *   - RMS error norm with scale atol + rtol max(|y_n|,|y_n+1|), PID step
 *     controller with coefficients (pcoeff, icoeff, dcoeff) (App. A.2,
 *     perturbation solver options) on error order 4, safety 0.9, step factor
 *     clipped to [0.2, 10] (rejected steps: 0.9 E^-1/4 clipped to [0.2, 0.9]),
 *     Hairer-Norsett-Wanner starting step;
 *   - cubic Hermite dense output at the requested ln a, and there the CMB
 *     source functions of App. B.4 (eq. source_functions), with alpha' from
 *     the traceless Einstein equation (Ma & Bertschinger 1995, eq. 21d):
 *       alpha_dot = -2 Hc alpha + eta - 12 pi G a^2 sum (rho+p) sigma / k^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_MAX_STEPS 1
#define O_NONFINITE 2
#define O_STEP_UNDERFLOW 3
#define O_BAD_INPUT 4

#define MAXQ 32

typedef struct {
    /* closed-form background, rt_i = (8 pi G/3) rho_i today [Mpc^-2] */
    double rt_g0, rt_ur0, rt_c0, rt_b0, rt_L;
    double pref_ncdm, m_over_T; /* massive nu: rho = pref a^-4 sum W eps */
    int n_q;
    const double *q, *W;
    double R_nu;
    /* thermodynamics splines on a uniform ln a grid: f values and second derivatives */
    int n;
    double L0, dl;
    const double *f_ldk, *M_ldk, *f_kap, *M_kap, *f_lcs, *M_lcs, *f_ltau, *M_ltau;
} otab_t;

typedef struct {
    int lg, lp, ln, nq, lq;
    double rtol, atol;
    int max_steps;
    double pcoeff, icoeff, dcoeff;
    double sw, isw, dop, pol;
    double grav, thom;
} oprec_t;

typedef struct {
    int N, dc, db, tb, g0, p0, n0, m0, eta;
} olayout_t;

static void make_layout(const oprec_t *p, olayout_t *L) {
    L->dc = 0;
    L->db = 1;
    L->tb = 2;
    L->g0 = 3;
    L->p0 = L->g0 + p->lg + 1;
    L->n0 = L->p0 + (p->lp > 0 ? p->lp + 1 : 0);
    L->m0 = L->n0 + p->ln + 1;
    L->eta = L->m0 + p->nq * (p->lq + 1);
    L->N = L->eta + 1;
}

/* Linear matter power spectrum today (App. B.4, eq. PK) from the state y at
   a = 1: P = 2 pi^2/k^3 * A_s (k/k_pivot)^(n_s - 1) * [sum_i rho_i delta_i /
   sum_i rho_i]^2, the sums over the non-relativistic species -- CDM, baryons
   and the massive neutrinos (their density contrast from Psi_0 through the
   momentum rule, eq. mnu_sum).  Units Mpc^3. */
double oracle_matter_pk(const otab_t *t, const oprec_t *p, double k, const double *y, double A_s, double n_s,
                        double k_pivot) {
    olayout_t L;
    make_layout(p, &L);
    double num = t->rt_c0 * y[L.dc] + t->rt_b0 * y[L.db];
    double den = t->rt_c0 + t->rt_b0;
    for (int i = 0; i < p->nq; ++i) {
        double e = sqrt(t->q[i] * t->q[i] + t->m_over_T * t->m_over_T); /* a = 1 */
        num += t->pref_ncdm * t->W[i] * e * y[L.m0 + i * (p->lq + 1)];
        den += t->pref_ncdm * t->W[i] * e;
    }
    double dm = num / den;
    double prim = A_s * pow(k / k_pivot, n_s - 1.0);
    const double pi = 3.14159265358979323846;
    return 2.0 * pi * pi / (k * k * k) * prim * dm * dm;
}

/* Matter density contrast at ln a (App. B.4 eq. PK, App. B.5): sum rho_i
   delta_i / sum rho_i over CDM, baryons and massive neutrinos, with rho_c,b
   proportional to a^-3 and the massive species' rho to a^-4 sum W eps. */
double oracle_delta_m(const otab_t *t, const oprec_t *p, double lna, const double *y) {
    olayout_t L;
    make_layout(p, &L);
    double a = exp(lna);
    double num = t->rt_c0 / (a * a * a) * y[L.dc] + t->rt_b0 / (a * a * a) * y[L.db];
    double den = (t->rt_c0 + t->rt_b0) / (a * a * a);
    for (int i = 0; i < p->nq; ++i) {
        double x = a * t->m_over_T;
        double rho_i = t->pref_ncdm * t->W[i] * sqrt(t->q[i] * t->q[i] + x * x) / (a * a * a * a);
        num += rho_i * y[L.m0 + i * (p->lq + 1)];
        den += rho_i;
    }
    return num / den;
}

int oracle_state_size(const oprec_t *p) {
    olayout_t L;
    make_layout(p, &L);
    return L.N;
}

/* natural cubic spline value and derivative, textbook form */
static double spl(const double *f, const double *M, int n, double x0, double h, double x, double *deriv) {
    double u = (x - x0) / h;
    int j = (int)floor(u);
    if (j < 0) j = 0;
    if (j > n - 1) j = n - 1;
    double B = u - j, A = 1.0 - B;
    double v = A * f[j] + B * f[j + 1] + ((A * A * A - A) * M[j] + (B * B * B - B) * M[j + 1]) * h * h / 6.0;
    if (deriv)
        *deriv = (f[j + 1] - f[j]) / h - (3.0 * A * A - 1.0) / 6.0 * h * M[j] + (3.0 * B * B - 1.0) / 6.0 * h * M[j + 1];
    return v;
}

typedef struct {
    double a, Hc, Hcp, rt_g, rt_ur, rt_c, rt_b, rho_n, p_n;
    double dk, kap, cs2, tau, dkp;
    double eps[MAXQ];
} obg_t;

static void background_at(const otab_t *t, double lna, obg_t *b) {
    double a = exp(lna);
    b->a = a;
    double a3 = a * a * a, a4 = a3 * a;
    b->rt_g = t->rt_g0 / a4;
    b->rt_ur = t->rt_ur0 / a4;
    b->rt_c = t->rt_c0 / a3;
    b->rt_b = t->rt_b0 / a3;
    double sr = 0.0, sp = 0.0;
    for (int i = 0; i < t->n_q; ++i) {
        double x = a * t->m_over_T;
        double e = sqrt(t->q[i] * t->q[i] + x * x);
        b->eps[i] = e;
        sr += t->W[i] * e;
        sp += t->W[i] * t->q[i] * t->q[i] / e;
    }
    b->rho_n = t->pref_ncdm * sr / a4;
    b->p_n = t->pref_ncdm * sp / (3.0 * a4);
    double rho = b->rt_g + b->rt_ur + b->rt_c + b->rt_b + t->rt_L + b->rho_n;
    double p = (b->rt_g + b->rt_ur) / 3.0 - t->rt_L + b->p_n;
    b->Hc = a * sqrt(rho);
    b->Hcp = b->Hc * (1.0 - 1.5 * (rho + p) / rho);
    double dlog;
    double ldk = spl(t->f_ldk, t->M_ldk, t->n, t->L0, t->dl, lna, &dlog);
    b->dk = exp(ldk);
    b->dkp = b->dk * dlog;
    b->kap = spl(t->f_kap, t->M_kap, t->n, t->L0, t->dl, lna, NULL);
    b->cs2 = exp(spl(t->f_lcs, t->M_lcs, t->n, t->L0, t->dl, lna, NULL));
    b->tau = exp(spl(t->f_ltau, t->M_ltau, t->n, t->L0, t->dl, lna, NULL));
}

static double dlnf0(double q) { return -q / (1.0 + exp(-q)); }

/* y' = f(ln a, y), species by species as App. C writes them. */
static void rhs(const otab_t *t, const oprec_t *p, const olayout_t *L, double k, const obg_t *b, const double *y,
                double *dy, double *hp_out, double *ep_out) {
    double a = b->a, H = b->Hc, k2 = k * k, a2 = a * a;
    double a4 = a2 * a2;
    /* metric: h' from the 00 equation, eta' from the 0i equation */
    double drho = b->rt_c * y[L->dc] + b->rt_b * y[L->db] + b->rt_g * y[L->g0] + b->rt_ur * y[L->n0];
    double rpt = b->rt_b * y[L->tb] + (4.0 / 3.0) * b->rt_g * y[L->g0 + 1] + (4.0 / 3.0) * b->rt_ur * y[L->n0 + 1];
    for (int i = 0; i < p->nq; ++i) {
        const double *psi = y + L->m0 + i * (p->lq + 1);
        drho += t->pref_ncdm / a4 * t->W[i] * b->eps[i] * psi[0];
        rpt += t->pref_ncdm / a4 * k * t->W[i] * t->q[i] * psi[1];
    }
    double hp = p->grav * (2.0 * k2 * y[L->eta] / (H * H) + 3.0 * a2 * drho / (H * H));
    double ep = p->grav * (1.5 * a2 * rpt / (H * k2));
    double T = p->thom * b->dk / H; /* 1/(Hc tau_c) */

    /* CDM */
    dy[L->dc] = -0.5 * hp;
    /* baryons */
    double Rgb = 4.0 * b->rt_g / (3.0 * b->rt_b);
    double dg = y[L->g0], tg = y[L->g0 + 1], sg = y[L->g0 + 2];
    dy[L->db] = -y[L->tb] / H - 0.5 * hp;
    dy[L->tb] = -y[L->tb] + b->cs2 * k2 * y[L->db] / H + Rgb * T * (tg - y[L->tb]);
    /* photons, temperature */
    int lg = p->lg;
    double G0 = 0.0, G2 = 0.0;
    if (p->lp > 0) {
        G0 = y[L->p0];
        G2 = y[L->p0 + 2];
    }
    dy[L->g0] = -4.0 * tg / (3.0 * H) - (2.0 / 3.0) * hp;
    dy[L->g0 + 1] = k2 / H * (0.25 * dg - sg) + T * (y[L->tb] - tg);
    dy[L->g0 + 2] = 4.0 * tg / (15.0 * H) - 0.3 * k / H * y[L->g0 + 3] + (2.0 / 15.0) * hp + 0.8 * ep - 0.9 * T * sg +
                    0.05 * T * (G0 + G2);
    for (int l = 3; l < lg; ++l) {
        double Fm = (l == 3) ? 2.0 * sg : y[L->g0 + l - 1];
        dy[L->g0 + l] = k / ((2.0 * l + 1.0) * H) * (l * Fm - (l + 1.0) * y[L->g0 + l + 1]) - T * y[L->g0 + l];
    }
    {
        int l = lg;
        double Fm = (l == 3) ? 2.0 * sg : y[L->g0 + l - 1];
        dy[L->g0 + l] = k / H * Fm - (l + 1.0) / (H * b->tau) * y[L->g0 + l] - T * y[L->g0 + l];
    }
    /* photons, polarisation */
    if (p->lp > 0) {
        int lp = p->lp;
        double Pi = 2.0 * sg + G0 + G2;
        for (int l = 0; l < lp; ++l) {
            double Gm = (l == 0) ? 0.0 : y[L->p0 + l - 1];
            double src = (l == 0) ? 1.0 : ((l == 2) ? 0.2 : 0.0);
            dy[L->p0 + l] = k / ((2.0 * l + 1.0) * H) * (l * Gm - (l + 1.0) * y[L->p0 + l + 1]) - T * y[L->p0 + l] +
                            0.5 * T * Pi * src;
        }
        dy[L->p0 + lp] = k / H * y[L->p0 + lp - 1] - (lp + 1.0) / (H * b->tau) * y[L->p0 + lp] - T * y[L->p0 + lp];
    }
    /* massless neutrinos */
    {
        int ln = p->ln;
        double dn = y[L->n0], tn = y[L->n0 + 1], sn = y[L->n0 + 2];
        dy[L->n0] = -4.0 * tn / (3.0 * H) - (2.0 / 3.0) * hp;
        dy[L->n0 + 1] = k2 / H * (0.25 * dn - sn);
        dy[L->n0 + 2] = 4.0 * tn / (15.0 * H) - 0.3 * k / H * y[L->n0 + 3] + (2.0 / 15.0) * hp + 0.8 * ep;
        for (int l = 3; l < ln; ++l) {
            double Fm = (l == 3) ? 2.0 * sn : y[L->n0 + l - 1];
            dy[L->n0 + l] = k / ((2.0 * l + 1.0) * H) * (l * Fm - (l + 1.0) * y[L->n0 + l + 1]);
        }
        double Fm = (ln == 3) ? 2.0 * sn : y[L->n0 + ln - 1];
        dy[L->n0 + ln] = k / H * Fm - (ln + 1.0) / (H * b->tau) * y[L->n0 + ln];
    }
    /* massive neutrinos, one hierarchy per momentum node */
    for (int i = 0; i < p->nq; ++i) {
        int lq = p->lq;
        const double *psi = y + L->m0 + i * (lq + 1);
        double *dpsi = dy + L->m0 + i * (lq + 1);
        double v = t->q[i] * k / (b->eps[i] * H);
        double dl = dlnf0(t->q[i]);
        dpsi[0] = -v * psi[1] + hp / 6.0 * dl;
        dpsi[1] = v / 3.0 * (psi[0] - 2.0 * psi[2]);
        dpsi[2] = v / 5.0 * (2.0 * psi[1] - 3.0 * psi[3]) - (hp / 15.0 + 0.4 * ep) * dl;
        for (int l = 3; l < lq; ++l) dpsi[l] = v / (2.0 * l + 1.0) * (l * psi[l - 1] - (l + 1.0) * psi[l + 1]);
        dpsi[lq] = v * psi[lq - 1] - (lq + 1.0) / (H * b->tau) * psi[lq];
    }
    dy[L->eta] = ep;
    if (hp_out) *hp_out = hp;
    if (ep_out) *ep_out = ep;
}

/* Adiabatic growing mode, leading order (Ma & Bertschinger 1995, eqs. 96-97)
   with C = 1/2 so that eta -> 1. */
static void initial_conditions(const otab_t *t, const oprec_t *p, const olayout_t *L, double k, const obg_t *b,
                               double *y) {
    memset(y, 0, sizeof(double) * L->N);
    double tau = b->tau, x = k * tau, Rn = t->R_nu;
    double dg = -x * x / 3.0;
    double tg = -k * x * x * x / 36.0;
    y[L->dc] = 0.75 * dg;
    y[L->db] = 0.75 * dg;
    y[L->tb] = tg;
    y[L->g0] = dg;
    y[L->g0 + 1] = tg;
    double tn = (23.0 + 4.0 * Rn) / (15.0 + 4.0 * Rn) * tg;
    double sn = 2.0 / (3.0 * (15.0 + 4.0 * Rn)) * x * x;
    y[L->n0] = dg;
    y[L->n0 + 1] = tn;
    y[L->n0 + 2] = sn;
    for (int i = 0; i < p->nq; ++i) {
        double *psi = y + L->m0 + i * (p->lq + 1);
        double dl = dlnf0(t->q[i]);
        psi[0] = -0.25 * dg * dl;
        psi[1] = -b->eps[i] / (3.0 * t->q[i] * k) * tn * dl;
        psi[2] = -0.5 * sn * dl;
    }
    y[L->eta] = 1.0 - (5.0 + 4.0 * Rn) / (12.0 * (15.0 + 4.0 * Rn)) * x * x;
}

/* ------------------------------------------------------------------------- */
/* Dense linear algebra                                                       */
/* ------------------------------------------------------------------------- */
static void build_A(const otab_t *t, const oprec_t *p, const olayout_t *L, double k, const obg_t *b, double *A,
                    double *e, double *col) {
    int N = L->N;
    for (int j = 0; j < N; ++j) {
        memset(e, 0, sizeof(double) * N);
        e[j] = 1.0;
        rhs(t, p, L, k, b, e, col, NULL, NULL);
        for (int i = 0; i < N; ++i) A[i * N + j] = col[i];
    }
}

static void matvec(int N, const double *A, const double *x, double *y) {
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += A[i * N + j] * x[j];
        y[i] = s;
    }
}

/* Gaussian elimination with partial pivoting: M (N x N, row major) is
   overwritten by its LU factors, piv records the row swaps. */
static int lu_factor(int N, double *M, int *piv) {
    for (int c = 0; c < N; ++c) {
        int p = c;
        double best = fabs(M[c * N + c]);
        for (int i = c + 1; i < N; ++i)
            if (fabs(M[i * N + c]) > best) {
                best = fabs(M[i * N + c]);
                p = i;
            }
        if (best == 0.0) return -1;
        piv[c] = p;
        if (p != c)
            for (int j = 0; j < N; ++j) {
                double t = M[c * N + j];
                M[c * N + j] = M[p * N + j];
                M[p * N + j] = t;
            }
        for (int i = c + 1; i < N; ++i) {
            double m = M[i * N + c] / M[c * N + c];
            M[i * N + c] = m;
            if (m == 0.0) continue;
            for (int j = c + 1; j < N; ++j) M[i * N + j] -= m * M[c * N + j];
        }
    }
    return 0;
}

static void lu_apply(int N, const double *LU, const int *piv, double *r) {
    /* P r (the swaps in the order they were made), then L and U */
    for (int c = 0; c < N; ++c)
        if (piv[c] != c) {
            double t = r[c];
            r[c] = r[piv[c]];
            r[piv[c]] = t;
        }
    for (int c = 0; c < N; ++c)
        for (int i = c + 1; i < N; ++i) r[i] -= LU[i * N + c] * r[c];
    for (int i = N - 1; i >= 0; --i) {
        double s = r[i];
        for (int j = i + 1; j < N; ++j) s -= LU[i * N + j] * r[j];
        r[i] = s / LU[i * N + i];
    }
}

/* Solve M x = r (x returned in r): LU with partial pivoting followed by two
   steps of iterative refinement with residuals accumulated in long double.
   The stage matrices are badly scaled (the eta' row carries 1/k^2), and the
   refinement brings the solve to rounding level. */
static int lu_solve(int N, const double *M, double *r, double *LU, int *piv, double *res) {
    memcpy(LU, M, sizeof(double) * N * N);
    if (lu_factor(N, LU, piv) != 0) return -1;
    double *b = res + N;
    memcpy(b, r, sizeof(double) * N);
    lu_apply(N, LU, piv, r);
    for (int it = 0; it < 2; ++it) {
        for (int i = 0; i < N; ++i) {
            long double acc = b[i];
            for (int j = 0; j < N; ++j) acc -= (long double)M[i * N + j] * r[j];
            res[i] = (double)acc;
        }
        lu_apply(N, LU, piv, res);
        for (int i = 0; i < N; ++i) r[i] += res[i];
    }
    return 0;
}

/* Solve M x = r again with the factors lu_solve left in LU, piv (same two
   refinement steps). */
static void lu_resolve(int N, const double *M, const double *LU, const int *piv, double *r, double *res) {
    double *b = res + N;
    memcpy(b, r, sizeof(double) * N);
    lu_apply(N, LU, piv, r);
    for (int it = 0; it < 2; ++it) {
        for (int i = 0; i < N; ++i) {
            long double acc = b[i];
            for (int j = 0; j < N; ++j) acc -= (long double)M[i * N + j] * r[j];
            res[i] = (double)acc;
        }
        lu_apply(N, LU, piv, res);
        for (int i = 0; i < N; ++i) r[i] += res[i];
    }
}

/* ------------------------------------------------------------------------- */
/* ESDIRK: implicit part of ARK4(3)6L[2]SA (Kennedy & Carpenter 2003), gamma = 1/4 */
/* ------------------------------------------------------------------------- */
static const double RK_c[6] = {0.0, 0.5, 83.0 / 250.0, 31.0 / 50.0, 17.0 / 20.0, 1.0};
static const double RK_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.25, 0.25, 0, 0, 0, 0},
    {8611.0 / 62500.0, -1743.0 / 31250.0, 0.25, 0, 0, 0},
    {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, 0.25, 0, 0},
    {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0, 2285395.0 / 8070912.0,
     0.25, 0},
    {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, 0.25}};
static const double RK_bh[6] = {4586570599.0 / 29645900160.0, 0.0, 178811875.0 / 945068544.0,
                                814220225.0 / 1159782912.0, -3700637.0 / 11593932.0, 61727.0 / 225920.0};

static double rms_norm(int N, const double *v, const double *y0, const double *y1, double rtol, double atol) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        double sc = atol + rtol * (y1 ? fmax(fabs(y0[i]), fabs(y1[i])) : fabs(y0[i]));
        double r = v[i] / sc;
        s += r * r;
    }
    return sqrt(s / N);
}

/* Source functions at ln a = t from the state y (App. B.4). */
static void sources_at(const otab_t *tb, const oprec_t *p, const olayout_t *L, double k, double t, const double *y,
                       double *dy, double *S0, double *S1, double *S2, double *diag) {
    obg_t b;
    background_at(tb, t, &b);
    double hp, ep;
    rhs(tb, p, L, k, &b, y, dy, &hp, &ep);
    double H = b.Hc, k2 = k * k, a2 = b.a * b.a, a4 = a2 * a2;
    double expk = exp(-b.kap);
    double g = b.dk * expk;
    double gp = (b.dkp + b.dk * b.dk / H) * expk;
    double eta = y[L->eta];
    double alpha = H * (hp + 6.0 * ep) / (2.0 * k2);
    double rps = (4.0 / 3.0) * (b.rt_g * y[L->g0 + 2] + b.rt_ur * y[L->n0 + 2]);
    for (int i = 0; i < p->nq; ++i)
        rps += tb->pref_ncdm / a4 * (2.0 / 3.0) * tb->W[i] * tb->q[i] * tb->q[i] / b.eps[i] *
               y[L->m0 + i * (p->lq + 1) + 2];
    double alphap = -2.0 * alpha + (eta - 4.5 * a2 * rps / k2) / H;
    double thb = y[L->tb], thbp = dy[L->tb];
    double Pi = 2.0 * y[L->g0 + 2];
    if (p->lp > 0) Pi += y[L->p0] + y[L->p0 + 2];
    *S0 = p->sw * g * (0.25 * y[L->g0] + H * alphap) +
          p->isw * (g * (eta - H * alphap - 2.0 * H * alpha) + 2.0 * H * expk * (ep - b.Hcp * alpha - H * alphap)) +
          p->dop * H * (g * (thbp / k2 + alphap) + gp * (thb / k2 + alpha));
    *S1 = p->isw * expk * k * (H * alphap + 2.0 * H * alpha - eta);
    *S2 = g * Pi / 8.0;
    if (diag) {
        diag[0] = hp;
        diag[1] = ep;
        diag[2] = alpha;
        diag[3] = alphap;
    }
}

/*
 * Integrate one mode from ln a = lna0 to 0.
 *   S: [3][n_out] (T0, T1, T2), zero before lna0 and after an abort.
 *   yout (optional): [n_out][N] dense-output states.
 *   y0 (optional): initial state overriding the adiabatic one.
 *   acc_lna (optional): accepted step end points, up to acc_cap of them.
 *   acc_h (optional): accepted step sizes, up to acc_cap of them.
 *   fixed (optional): replay; fixed[0] is the start (overriding lna0) and
 *     fixed[1..n_fixed] the step sizes, taken without error control (the
 *     recorded start and acc_h of another run).
 * Returns a status code; nsteps = attempted steps, naccept = accepted.
 */
int oracle_perturb(const otab_t *tb, const oprec_t *p, double k, double lna0, int n_out, const double *lna_out,
                   double *S, double *yout, const double *y0, int *nsteps, int *naccept, double *acc_lna,
                   int acc_cap, double *diag, double *acc_h,
                   const double *fixed, int n_fixed) {
    olayout_t L;
    make_layout(p, &L);
    int N = L.N;
    if (p->lg < 3 || p->ln < 3 || (p->lp != 0 && p->lp < 3) || (p->nq > 0 && p->lq < 3) || p->nq > MAXQ || k <= 0)
        return O_BAD_INPUT;
    double *work = (double *)calloc((size_t)N * N * 3 + (size_t)N * 22, sizeof(double));
    int *piv = (int *)calloc((size_t)N, sizeof(int));
    double *A = work, *Mm = A + N * N;
    double *y = Mm + N * N, *f = y + N, *ynew = f + N, *R = ynew + N, *err = R + N, *e = err + N, *col = e + N;
    double *K = col + N; /* 6 vectors */
    double *tmp = K + 6 * N, *ytmp = tmp + N, *dyt = ytmp + N;
    double *LU = dyt + N, *res = LU + (size_t)N * N; /* res holds 2N */
    for (int i = 0; i < 3 * n_out; ++i) S[i] = 0.0;
    int status = O_OK;
    int ns = 0, na = 0;
    double t = fixed ? fixed[0] : lna0;
    obg_t b;
    background_at(tb, t, &b);
    if (y0)
        memcpy(y, y0, sizeof(double) * N);
    else
        initial_conditions(tb, p, &L, k, &b, y);
    build_A(tb, p, &L, k, &b, A, e, col);
    matvec(N, A, y, f);
    int jo = 0;
    while (jo < n_out && lna_out[jo] < t) ++jo;

    /* starting step (Hairer, Norsett & Wanner, Sec. II.4), order 4 */
    double h = 0.0;
    if (!fixed) {
        double d0 = rms_norm(N, y, y, NULL, p->rtol, p->atol);
        double d1 = rms_norm(N, f, y, NULL, p->rtol, p->atol);
        double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
        if (h0 > -t) h0 = -t;
        for (int i = 0; i < N; ++i) ytmp[i] = y[i] + h0 * f[i];
        obg_t b1;
        background_at(tb, t + h0, &b1);
        build_A(tb, p, &L, k, &b1, Mm, e, col);
        matvec(N, Mm, ytmp, tmp);
        for (int i = 0; i < N; ++i) tmp[i] -= f[i];
        double d2 = rms_norm(N, tmp, y, NULL, p->rtol, p->atol) / h0;
        double dm = fmax(d1, d2);
        double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 0.2);
        h = fmin(100.0 * h0, h1);
    }
    double q = 4.0;
    double b1c = (p->pcoeff + p->icoeff + p->dcoeff) / q;
    double b2c = -(p->pcoeff + 2.0 * p->dcoeff) / q;
    double b3c = p->dcoeff / q;
    double Eprev = 1.0, Eprev2 = 1.0;
    const double gam = 0.25;

    while (t < 0.0) {
        if (ns >= p->max_steps) {
            status = O_MAX_STEPS;
            break;
        }
        int last = 0;
        if (fixed) {
            if (na >= n_fixed) {
                status = O_MAX_STEPS;
                break;
            }
            h = fixed[1 + na];
            last = t + h >= 0.0;
        } else if (h >= -t) {
            h = -t;
            last = 1;
        }
        memcpy(K, f, sizeof(double) * N);
        for (int s = 1; s < 6; ++s) {
            double ts = t + RK_c[s] * h;
            if (s == 5) ts = last ? 0.0 : t + h;
            for (int i = 0; i < N; ++i) {
                double acc = y[i];
                for (int j = 0; j < s; ++j) acc += h * RK_A[s][j] * K[j * N + i];
                R[i] = acc;
            }
            obg_t bs;
            background_at(tb, ts, &bs);
            build_A(tb, p, &L, k, &bs, A, e, col);
            for (int i = 0; i < N * N; ++i) Mm[i] = -h * gam * A[i];
            for (int i = 0; i < N; ++i) Mm[i * N + i] += 1.0;
            if (lu_solve(N, Mm, R, LU, piv, res) != 0) {
                status = O_NONFINITE;
                break;
            }
            matvec(N, A, R, K + s * N);
            if (s == 5) memcpy(ynew, R, sizeof(double) * N);
        }
        if (status != O_OK) break;
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) acc += (RK_A[5][j] - RK_bh[j]) * K[j * N + i];
            err[i] = h * acc;
        }
        double E = rms_norm(N, err, y, ynew, p->rtol, p->atol);
        ++ns;
        if (!(E == E) || isinf(E)) {
            status = O_NONFINITE;
            break;
        }
        double fac;
        if (fixed || E <= 1.0) {
            double tn = last ? 0.0 : t + h;
            if (acc_h && na < acc_cap) acc_h[na] = h;
            if (tn >= 0.0) tn = 0.0;
            /* dense output */
            while (jo < n_out && lna_out[jo] <= tn) {
                double hh = tn - t;
                double th = (hh > 0.0) ? (lna_out[jo] - t) / hh : 1.0;
                double h00 = 2 * th * th * th - 3 * th * th + 1, h10 = th * th * th - 2 * th * th + th;
                double h01 = -2 * th * th * th + 3 * th * th, h11 = th * th * th - th * th;
                for (int i = 0; i < N; ++i)
                    ytmp[i] = h00 * y[i] + h10 * hh * f[i] + h01 * ynew[i] + h11 * hh * K[5 * N + i];
                sources_at(tb, p, &L, k, lna_out[jo], ytmp, dyt, &S[jo], &S[n_out + jo], &S[2 * n_out + jo],
                           diag ? diag + 4 * (size_t)jo : NULL);
                if (yout) memcpy(yout + (size_t)jo * N, ytmp, sizeof(double) * N);
                ++jo;
            }
            if (acc_lna && na < acc_cap) acc_lna[na] = tn;
            ++na;
            memcpy(y, ynew, sizeof(double) * N);
            memcpy(f, K + 5 * N, sizeof(double) * N);
            t = tn;
            double Ef = fmax(E, 1e-10);
            fac = 0.9 * pow(Ef, -b1c) * pow(Eprev, -b2c) * pow(Eprev2, -b3c);
            fac = fmin(10.0, fmax(0.2, fac));
            Eprev2 = Eprev;
            Eprev = Ef;
        } else {
            fac = fmin(0.9, fmax(0.2, 0.9 * pow(E, -0.25)));
        }
        h *= fac;
        if (!fixed && t < 0.0 && h < 1e-12) {
            status = O_STEP_UNDERFLOW;
            break;
        }
    }
    *nsteps = ns;
    *naccept = na;
    free(work);
    free(piv);
    return status;
}

/* Derivative of a table-dependent quantity from its values at theta +- eps
   (v1, m1) and, for order 4, at theta +- 2 eps (v2, m2): the central
   difference (v1 - m1) / (2 eps) or the five-point
   (8 (v1 - m1) - (v2 - m2)) / (12 eps). */
static double tdiff(int order, double eps, double v1, double m1, double v2, double m2) {
    if (order == 4) return (8.0 * (v1 - m1) - (v2 - m2)) / (12.0 * eps);
    return (v1 - m1) / (2.0 * eps);
}

/*
 * Forward-mode tangents of one mode along a fixed step sequence (the start
 * fixed[0] and the step sizes fixed[1..n_fixed]): the derivative of the
 * discrete map (initial state, ESDIRK stages, dense output, sources) with
 * respect to nd parameters (section 3: the paper's forward-mode option).
 * Parameter d enters only through the tables: tt[(4 d + m)] for m = 0..3 are
 * the tables at theta_d + eps[d], - eps[d], + 2 eps[d], - 2 eps[d] (the last
 * two read only for order 4), and each table-dependent quantity at a fixed
 * state (the right-hand side, the initial state, the sources) is
 * differentiated by the central (order 2) or five-point (order 4)
 * difference between them (tdiff).  The state's tangent is carried through
 * the stages exactly:
 *   Rdot_s = ydot_n + h sum_{j<s} a_sj Kdot_j,
 *   (I - h gamma A_s) Ydot_s = Rdot_s + h gamma Adot_s Y_s,
 *   Kdot_s = Adot_s Y_s + A_s Ydot_s,   ydot_{n+1} = Ydot_5,
 * and at each output time Sdot = S(ydot) + dS/dtheta at the fixed state (the
 * sources are linear in the state).  S: [3][n_out]; Sd: [nd][3][n_out].
 */
int oracle_perturb_tangent(const otab_t *tb, const otab_t *tt, const double *eps, int nd, int order,
                           const oprec_t *p, double k, int n_out, const double *lna_out, double *S, double *Sd,
                           const double *fixed, int n_fixed) {
    olayout_t L;
    make_layout(p, &L);
    const int N = L.N;
    if (p->lg < 3 || p->ln < 3 || (p->lp != 0 && p->lp < 3) || (p->nq > 0 && p->lq < 3) || p->nq > MAXQ || k <= 0 ||
        nd < 1 || !fixed || (order != 2 && order != 4))
        return O_BAD_INPUT;
    const int nt = order == 4 ? 4 : 2; /* tables per parameter that are read */
    const size_t nn = (size_t)N * N, nv = (size_t)nd * N;
    double *work = (double *)calloc(3 * nn + 22 * (size_t)N + 12 * nv, sizeof(double));
    int *piv = (int *)calloc((size_t)N, sizeof(int));
    double *A = work, *Mm = A + nn, *LU = Mm + nn;
    double *y = LU + nn, *f = y + N, *ynew = f + N, *R = ynew + N, *e = R + N, *col = e + N, *K = col + N;
    double *ytmp = K + 6 * N, *dyt = ytmp + N, *v = dyt + N, *res = v + 4 * N; /* v: 4 N, res: 2 N */
    double *yd = res + 2 * N, *fd = yd + nv, *ynewd = fd + nv, *Rd = ynewd + nv, *Kd = Rd + nv; /* Kd: 6 nv */
    double *ytd = Kd + 6 * nv;
    for (int i = 0; i < 3 * n_out; ++i) S[i] = 0.0;
    for (size_t i = 0; i < (size_t)nd * 3 * n_out; ++i) Sd[i] = 0.0;
    int status = O_OK;
    double t = fixed[0];
    obg_t b, bt[4];
    background_at(tb, t, &b);
    initial_conditions(tb, p, &L, k, &b, y);
    build_A(tb, p, &L, k, &b, A, e, col);
    matvec(N, A, y, f);
    for (int d = 0; d < nd; ++d) {
        for (int m = 0; m < nt; ++m) {
            background_at(&tt[4 * d + m], t, &bt[m]);
            initial_conditions(&tt[4 * d + m], p, &L, k, &bt[m], v + m * N);
        }
        for (int i = 0; i < N; ++i)
            yd[d * N + i] = tdiff(order, eps[d], v[i], v[N + i], v[2 * N + i], v[3 * N + i]);
        for (int m = 0; m < nt; ++m) rhs(&tt[4 * d + m], p, &L, k, &bt[m], y, v + m * N, NULL, NULL);
        matvec(N, A, yd + d * N, fd + d * N);
        for (int i = 0; i < N; ++i)
            fd[d * N + i] += tdiff(order, eps[d], v[i], v[N + i], v[2 * N + i], v[3 * N + i]);
    }
    int jo = 0;
    while (jo < n_out && lna_out[jo] < t) ++jo;
    const double gam = 0.25;
    int na = 0;
    while (t < 0.0) {
        if (na >= n_fixed) {
            status = O_MAX_STEPS;
            break;
        }
        const double h = fixed[1 + na];
        const int last = t + h >= 0.0;
        memcpy(K, f, sizeof(double) * N);
        memcpy(Kd, fd, sizeof(double) * nv);
        for (int s = 1; s < 6; ++s) {
            double ts = t + RK_c[s] * h;
            if (s == 5) ts = last ? 0.0 : t + h;
            for (int i = 0; i < N; ++i) {
                double acc = y[i];
                for (int j = 0; j < s; ++j) acc += h * RK_A[s][j] * K[j * N + i];
                R[i] = acc;
            }
            for (int d = 0; d < nd; ++d)
                for (int i = 0; i < N; ++i) {
                    double acc = yd[d * N + i];
                    for (int j = 0; j < s; ++j) acc += h * RK_A[s][j] * Kd[(size_t)j * nv + d * N + i];
                    Rd[d * N + i] = acc;
                }
            obg_t bs;
            background_at(tb, ts, &bs);
            build_A(tb, p, &L, k, &bs, A, e, col);
            for (size_t i = 0; i < nn; ++i) Mm[i] = -h * gam * A[i];
            for (int i = 0; i < N; ++i) Mm[i * N + i] += 1.0;
            if (lu_solve(N, Mm, R, LU, piv, res) != 0) { /* R becomes Y_s */
                status = O_NONFINITE;
                break;
            }
            matvec(N, A, R, K + s * N);
            for (int d = 0; d < nd; ++d) {
                for (int m = 0; m < nt; ++m) {
                    background_at(&tt[4 * d + m], ts, &bt[m]);
                    rhs(&tt[4 * d + m], p, &L, k, &bt[m], R, v + m * N, NULL, NULL);
                }
                double *Yd = Rd + d * N, *kd = Kd + (size_t)s * nv + d * N;
                for (int i = 0; i < N; ++i) {
                    v[i] = tdiff(order, eps[d], v[i], v[N + i], v[2 * N + i], v[3 * N + i]); /* Adot_s Y_s */
                    Yd[i] += h * gam * v[i];
                }
                lu_resolve(N, Mm, LU, piv, Yd, res);
                matvec(N, A, Yd, kd);
                for (int i = 0; i < N; ++i) kd[i] += v[i];
            }
            if (s == 5) {
                memcpy(ynew, R, sizeof(double) * N);
                memcpy(ynewd, Rd, sizeof(double) * nv);
            }
        }
        if (status != O_OK) break;
        double tn = last ? 0.0 : t + h;
        if (tn >= 0.0) tn = 0.0;
        while (jo < n_out && lna_out[jo] <= tn) {
            const double hh = tn - t;
            const double th = (hh > 0.0) ? (lna_out[jo] - t) / hh : 1.0;
            const double h00 = 2 * th * th * th - 3 * th * th + 1, h10 = th * th * th - 2 * th * th + th;
            const double h01 = -2 * th * th * th + 3 * th * th, h11 = th * th * th - th * th;
            for (int i = 0; i < N; ++i)
                ytmp[i] = h00 * y[i] + h10 * hh * f[i] + h01 * ynew[i] + h11 * hh * K[5 * N + i];
            sources_at(tb, p, &L, k, lna_out[jo], ytmp, dyt, &S[jo], &S[n_out + jo], &S[2 * n_out + jo], NULL);
            for (int d = 0; d < nd; ++d) {
                for (int i = 0; i < N; ++i)
                    ytd[d * N + i] = h00 * yd[d * N + i] + h10 * hh * fd[d * N + i] + h01 * ynewd[d * N + i] +
                                     h11 * hh * Kd[5 * nv + d * N + i];
                double sl[3], st[4][3] = {{0}};
                sources_at(tb, p, &L, k, lna_out[jo], ytd + d * N, dyt, &sl[0], &sl[1], &sl[2], NULL);
                for (int m = 0; m < nt; ++m)
                    sources_at(&tt[4 * d + m], p, &L, k, lna_out[jo], ytmp, dyt, &st[m][0], &st[m][1], &st[m][2],
                               NULL);
                double *o = Sd + (size_t)d * 3 * n_out;
                for (int c = 0; c < 3; ++c)
                    o[c * n_out + jo] = sl[c] + tdiff(order, eps[d], st[0][c], st[1][c], st[2][c], st[3][c]);
            }
            ++jo;
        }
        ++na;
        memcpy(y, ynew, sizeof(double) * N);
        memcpy(f, K + 5 * N, sizeof(double) * N);
        memcpy(yd, ynewd, sizeof(double) * nv);
        memcpy(fd, Kd + 5 * nv, sizeof(double) * nv);
        t = tn;
    }
    free(work);
    free(piv);
    return status;
}

/* Forward-mode tangents of all modes (oracle_perturb_tangent), in parallel
   over k, each mode replaying its own history hist[i][0 .. hn[i]]. */
int oracle_perturb_many_tangent(const otab_t *tb, const otab_t *tt, const double *eps, int nd, int order,
                                const oprec_t *p0, int nk, const double *k, int n_out, const double *lna_out,
                                double *S, double *Sd, int *status, const double *hist, const int *hn, int cap) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = nk - 1; i >= 0; --i)
        status[i] = oracle_perturb_tangent(tb, tt, eps, nd, order, p0, k[i], n_out, lna_out,
                                           S + (size_t)i * 3 * n_out, Sd + (size_t)i * nd * 3 * n_out,
                                           hist + (size_t)i * cap, hn[i]);
    return 0;
}

/* All modes of one cosmology, in parallel over k (each mode is independent
   and writes its own slice, so the result does not depend on the threads). */
int oracle_perturb_many(const otab_t *tb, const oprec_t *p0, int nk, const double *k, const double *lna0,
                        const double *rtol, const double *atol, int n_out, const double *lna_out, double *S,
                        int *status, int *nsteps, int *naccept) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = nk - 1; i >= 0; --i) {
        oprec_t p = *p0;
        p.rtol = rtol[i];
        p.atol = atol[i];
        status[i] = oracle_perturb(tb, &p, k[i], lna0[i], n_out, lna_out, S + (size_t)i * 3 * n_out, NULL, NULL,
                                   &nsteps[i], &naccept[i], NULL, 0, NULL, NULL, NULL, 0);
    }
    return 0;
}

/* All modes with their accepted-step histories hist[nk][cap] (entry 0 the
   start, then every accepted end point; cap >= max_steps + 1), or, with
   replay != 0, replaying those histories (counts hn[nk]) without error control. */
int oracle_perturb_many_hist(const otab_t *tb, const oprec_t *p0, int nk, const double *k, const double *lna0,
                             const double *rtol, const double *atol, int n_out, const double *lna_out, double *S,
                             int *status, int *nsteps, int *naccept, double *hist, int *hn, int cap, int replay) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = nk - 1; i >= 0; --i) {
        oprec_t p = *p0;
        p.rtol = rtol[i];
        p.atol = atol[i];
        double *hi = hist + (size_t)i * cap;
        if (replay) {
            status[i] = oracle_perturb(tb, &p, k[i], hi[0], n_out, lna_out, S + (size_t)i * 3 * n_out, NULL, NULL,
                                       &nsteps[i], &naccept[i], NULL, 0, NULL, NULL, hi, hn[i]);
        } else {
            hi[0] = lna0[i];
            status[i] = oracle_perturb(tb, &p, k[i], lna0[i], n_out, lna_out, S + (size_t)i * 3 * n_out, NULL, NULL,
                                       &nsteps[i], &naccept[i], NULL, cap - 1, NULL, hi + 1, NULL, 0);
            hn[i] = naccept[i] < cap - 1 ? naccept[i] : cap - 1;
        }
    }
    return 0;
}

/* As oracle_perturb_many, plus the matter density contrast Dm[nk][n_out] at
   every output time (zero where S is zero: before the start, after an abort). */
int oracle_perturb_many_dm(const otab_t *tb, const oprec_t *p0, int nk, const double *k, const double *lna0,
                           const double *rtol, const double *atol, int n_out, const double *lna_out, double *S,
                           double *Dm, int *status, int *nsteps, int *naccept) {
    int N = oracle_state_size(p0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = nk - 1; i >= 0; --i) {
        oprec_t p = *p0;
        p.rtol = rtol[i];
        p.atol = atol[i];
        double *Y = (double *)calloc((size_t)n_out * N, sizeof(double));
        status[i] = oracle_perturb(tb, &p, k[i], lna0[i], n_out, lna_out, S + (size_t)i * 3 * n_out, Y, NULL,
                                   &nsteps[i], &naccept[i], NULL, 0, NULL, NULL, NULL, 0);
        for (int j = 0; j < n_out; ++j) {
            /* a state row that the integration never produced is still all zero */
            const double *y = Y + (size_t)j * N;
            int produced = 0;
            for (int r = 0; r < N; ++r)
                if (y[r] != 0.0) produced = 1;
            Dm[(size_t)i * n_out + j] = produced ? oracle_delta_m(tb, &p, lna_out[j], y) : 0.0;
        }
        free(Y);
    }
    return 0;
}

/* The source functions S_T0, S_T1, S_T2 (App. B.4) at ln a = lna from a given
   state y (the oracle's layout), for tests of the transposed source map. */
void oracle_sources_state(const otab_t *tb, const oprec_t *p, double k, double lna, const double *y, double *S) {
    olayout_t L;
    make_layout(p, &L);
    double *dy = (double *)malloc(sizeof(double) * (size_t)L.N);
    sources_at(tb, p, &L, k, lna, y, dy, &S[0], &S[1], &S[2], NULL);
    free(dy);
}

/* y' at (ln a, y) for tests. */
void oracle_rhs(const otab_t *tb, const oprec_t *p, double k, double lna, const double *y, double *dy) {
    olayout_t L;
    make_layout(p, &L);
    obg_t b;
    background_at(tb, lna, &b);
    rhs(tb, p, &L, k, &b, y, dy, NULL, NULL);
}

/* Brute-force classical RK4 from lna0 through the output times, with the
   step bounded by h_max and by c_stab / (largest rate estimate), landing
   exactly on each output time.  Writes the sources (and states) there. */
int oracle_rk4(const otab_t *tb, const oprec_t *p, double k, double lna0, int n_out, const double *lna_out, double *S,
               double *yout, double h_max, double c_stab, long *nsteps) {
    olayout_t L;
    make_layout(p, &L);
    int N = L.N;
    double *w = (double *)calloc((size_t)N * 8, sizeof(double));
    double *y = w, *k1 = y + N, *k2 = k1 + N, *k3 = k2 + N, *k4 = k3 + N, *yt = k4 + N, *dyt = yt + N;
    obg_t b;
    background_at(tb, lna0, &b);
    initial_conditions(tb, p, &L, k, &b, y);
    for (int i = 0; i < 3 * n_out; ++i) S[i] = 0.0;
    double t = lna0;
    long ns = 0;
    for (int jo = 0; jo < n_out; ++jo) {
        double target = lna_out[jo];
        if (target < lna0) continue;
        while (t < target) {
            background_at(tb, t, &b);
            double Rgb = 4.0 * b.rt_g / (3.0 * b.rt_b);
            double lam = (1.0 + Rgb) * p->thom * b.dk / b.Hc + k / b.Hc + (p->lg + 1.0) / (b.Hc * b.tau) + 10.0;
            double h = fmin(h_max, c_stab / lam);
            if (t + h > target) h = target - t;
            obg_t bb;
            rhs(tb, p, &L, k, &b, y, k1, NULL, NULL);
            background_at(tb, t + 0.5 * h, &bb);
            for (int i = 0; i < N; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
            rhs(tb, p, &L, k, &bb, yt, k2, NULL, NULL);
            for (int i = 0; i < N; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
            rhs(tb, p, &L, k, &bb, yt, k3, NULL, NULL);
            background_at(tb, t + h, &bb);
            for (int i = 0; i < N; ++i) yt[i] = y[i] + h * k3[i];
            rhs(tb, p, &L, k, &bb, yt, k4, NULL, NULL);
            for (int i = 0; i < N; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
            t = (t + h >= target) ? target : t + h;
            ++ns;
        }
        sources_at(tb, p, &L, k, target, y, dyt, &S[jo], &S[n_out + jo], &S[2 * n_out + jo], NULL);
        if (yout) memcpy(yout + (size_t)jo * N, y, sizeof(double) * N);
    }
    *nsteps = ns;
    free(w);
    return 0;
}
