/*
 * CPU oracle, part 3: spherical Bessel functions, line-of-sight projection and
 * the k quadrature to C_ell.
 *
 * TEST INFRASTRUCTURE ONLY (see perturb.c).  Shares no code with the library.
 *
 * Bessel functions j_l(x), l = 0..L, in long double by a method chosen to be
 * plainly correct rather than fast:
 *   - l <= x/2: upward recurrence from the closed forms of j_0 and j_1;
 *   - above that: the ratio j_L/j_{L-1} from its continued fraction
 *     (modified Lentz), then downward recurrence to the last upward order
 *     (or to l = 0), normalised against the exact value there.
 * No cut-off is applied: every (l, x) is evaluated.
 *
 * Transfer functions (App. B.4, the four line-of-sight integrals), with the
 * derivatives of j_l written through the recurrence and Bessel's equation:
 *   j'   = j_{l-1} - (l+1) j_l / x
 *   j''  = -2 j'/x + (l(l+1)/x^2 - 1) j_l
 *   Delta_T = sum_j w_j [S_T0 j_l + S_T1 j' + s_pol S_T2 (3 j'' + j_l)/2]
 *   Delta_E = sqrt(3 (l+2)!/(8 (l-2)!)) sum_j w_j sqrt(6) S_T2 j_l / x^2
 * with the x = 0 limits j_l = j' = 0, (3j''+j)/2 = delta_l2/5, j/x^2 = delta_l2/15.
 * C_ell = 4 pi int dk/k P(k) Delta_X Delta_Y (eq. c_ell_def), trapezoid in k on
 * the given grid, P(k) = A_s (k/k_pivot)^(n_s-1) (eq. PK_pivot).
 */
#include <math.h>
#include <stdlib.h>

/* j_0..j_L at x (x >= 0) into out[0..L] */
void oracle_bessel(int L, double xd, long double *out) {
    long double x = xd;
    if (xd == 0.0) {
        out[0] = 1.0L;
        for (int l = 1; l <= L; ++l) out[l] = 0.0L;
        return;
    }
    long double s = sinl(x), c = cosl(x);
    long double j0 = s / x;
    long double j1 = s / (x * x) - c / x;
    int lup = (int)floorl(x / 2.0L);
    if (lup > L) lup = L;
    out[0] = j0;
    if (L >= 1) out[1] = j1;
    for (int l = 1; l < lup; ++l) out[l + 1] = (2.0L * l + 1.0L) / x * out[l] - out[l - 1];
    if (lup >= L) return;
    /* continued fraction for r = j_L / j_{L-1} = 1/(b_L - 1/(b_{L+1} - ...)), b_l = (2l+1)/x */
    const long double tiny = 1e-4000L;
    long double f = tiny, C = f, D = 0.0L;
    for (int m = 0; m < 1000000; ++m) {
        long double bm = (2.0L * (L + m) + 1.0L) / x;
        long double am = (m == 0) ? 1.0L : -1.0L;
        D = bm + am * D;
        if (D == 0.0L) D = tiny;
        C = bm + am / C;
        if (C == 0.0L) C = tiny;
        D = 1.0L / D;
        long double delta = C * D;
        f *= delta;
        if (fabsl(delta - 1.0L) < 1e-19L) break;
    }
    /* downward recurrence with unnormalised start (j_{L-1} = 1, j_L = r) */
    int lstop = lup > 0 ? lup - 1 : 0; /* lowest index we recompute */
    long double *tmp = (long double *)malloc(sizeof(long double) * (L + 1));
    tmp[L] = f;
    tmp[L - 1] = 1.0L;
    for (int l = L - 1; l > lstop; --l) {
        tmp[l - 1] = (2.0L * l + 1.0L) / x * tmp[l] - tmp[l + 1];
        if (fabsl(tmp[l - 1]) > 1e4000L) {
            for (int m = l - 1; m <= L; ++m) tmp[m] *= 1e-4000L;
        }
    }
    /* normalise against an exactly known value */
    long double scale;
    if (lup >= 2) {
        /* match at the larger (in magnitude) of the two last upward values */
        int m = (fabsl(out[lup]) > fabsl(out[lup - 1])) ? lup : lup - 1;
        scale = out[m] / tmp[m];
    } else {
        /* lstop == 0: j_0 or j_1 from the closed forms */
        if (fabsl(j0) > fabsl(j1))
            scale = j0 / tmp[0];
        else
            scale = j1 / tmp[1];
    }
    for (int l = lstop; l <= L; ++l) {
        if (l <= lup && lup >= 2) continue;
        out[l] = tmp[l] * scale;
    }
    free(tmp);
}

/* Delta_T[l][k], Delta_E[l][k] for l = 2..lmax (row l-2), all modes;
   S is [nk][3][ntau]. */
void oracle_los(int nk, const double *k, int ntau, const double *chi, const double *w, const double *S, int lmax,
                double s_pol, int want_E, double *DT, double *DE) {
    int nl = lmax - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int ik = nk - 1; ik >= 0; --ik) {
        long double *jl = (long double *)malloc(sizeof(long double) * (lmax + 2));
        long double *accT = (long double *)calloc(nl, sizeof(long double));
        long double *accE = (long double *)calloc(nl, sizeof(long double));
        const double *S0 = S + (size_t)ik * 3 * ntau, *S1 = S0 + ntau, *S2 = S1 + ntau;
        for (int j = 0; j < ntau; ++j) {
            double x = k[ik] * chi[j];
            oracle_bessel(lmax + 1, x, jl);
            for (int l = 2; l <= lmax; ++l) {
                long double J, Jp, Rt2, Je;
                if (x == 0.0) {
                    J = 0.0L;
                    Jp = 0.0L;
                    Rt2 = (l == 2) ? 0.2L : 0.0L;
                    Je = (l == 2) ? 1.0L / 15.0L : 0.0L;
                } else {
                    long double X = x;
                    J = jl[l];
                    Jp = jl[l - 1] - (l + 1.0L) * J / X;
                    long double Jpp = -2.0L * Jp / X + ((long double)l * (l + 1.0L) / (X * X) - 1.0L) * J;
                    Rt2 = 0.5L * (3.0L * Jpp + J);
                    Je = J / (X * X);
                }
                accT[l - 2] += (long double)w[j] * (S0[j] * J + S1[j] * Jp + s_pol * S2[j] * Rt2);
                if (want_E) accE[l - 2] += (long double)w[j] * sqrtl(6.0L) * S2[j] * Je;
            }
        }
        for (int l = 2; l <= lmax; ++l) {
            DT[(size_t)(l - 2) * nk + ik] = (double)accT[l - 2];
            if (want_E) {
                long double cl = sqrtl(3.0L * (l + 2.0L) * (l + 1.0L) * l * (l - 1.0L) / 8.0L);
                DE[(size_t)(l - 2) * nk + ik] = (double)(cl * accE[l - 2]);
            }
        }
        free(jl);
        free(accT);
        free(accE);
    }
}

/* Transpose of oracle_los: given G_T[l][k], G_E[l][k] (rows l-2), the
   gradient with respect to the sources, gS[k][3][ntau]:
     gS_T0 = w_j sum_l G_T j_l,   gS_T1 = w_j sum_l G_T j_l',
     gS_T2 = w_j sum_l [s_pol G_T (3 j_l'' + j_l)/2 + c_l sqrt(6) G_E j_l/x^2],
   c_l = sqrt(3 (l+2)!/(8 (l-2)!)) (the E part only with want_E). */
void oracle_los_adjoint(int nk, const double *k, int ntau, const double *chi, const double *w, const double *GT,
                        const double *GE, int lmax, double s_pol, int want_E, double *gS) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int ik = nk - 1; ik >= 0; --ik) {
        long double *jl = (long double *)malloc(sizeof(long double) * (lmax + 2));
        double *g0 = gS + (size_t)ik * 3 * ntau, *g1 = g0 + ntau, *g2 = g1 + ntau;
        for (int j = 0; j < ntau; ++j) {
            double x = k[ik] * chi[j];
            oracle_bessel(lmax + 1, x, jl);
            long double a0 = 0, a1 = 0, a2 = 0;
            for (int l = 2; l <= lmax; ++l) {
                long double J, Jp, Rt2, Je;
                if (x == 0.0) {
                    J = 0.0L;
                    Jp = 0.0L;
                    Rt2 = (l == 2) ? 0.2L : 0.0L;
                    Je = (l == 2) ? 1.0L / 15.0L : 0.0L;
                } else {
                    long double X = x;
                    J = jl[l];
                    Jp = jl[l - 1] - (l + 1.0L) * J / X;
                    long double Jpp = -2.0L * Jp / X + ((long double)l * (l + 1.0L) / (X * X) - 1.0L) * J;
                    Rt2 = 0.5L * (3.0L * Jpp + J);
                    Je = J / (X * X);
                }
                long double gt = GT[(size_t)(l - 2) * nk + ik];
                a0 += gt * J;
                a1 += gt * Jp;
                a2 += s_pol * gt * Rt2;
                if (want_E) {
                    long double cl = sqrtl(3.0L * (l + 2.0L) * (l + 1.0L) * l * (l - 1.0L) / 8.0L);
                    a2 += cl * sqrtl(6.0L) * (long double)GE[(size_t)(l - 2) * nk + ik] * Je;
                }
            }
            g0[j] = (double)(w[j] * a0);
            g1[j] = (double)(w[j] * a1);
            g2[j] = (double)(w[j] * a2);
        }
        free(jl);
    }
}

/* Cl[3][lmax+1] (TT, TE, EE; l < 2 zero) from the transfer functions. */
void oracle_cl(int nk, const double *k, int lmax, const double *DT, const double *DE, int want_E, double A_s,
               double n_s, double k_pivot, double *Cl) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < 3 * (lmax + 1); ++i) Cl[i] = 0.0;
    for (int l = 2; l <= lmax; ++l) {
        long double tt = 0, te = 0, ee = 0;
        for (int i = 0; i < nk; ++i) {
            double wk = 0.5 * ((i + 1 < nk ? k[i + 1] : k[i]) - (i > 0 ? k[i - 1] : k[i]));
            double P = A_s * pow(k[i] / k_pivot, n_s - 1.0);
            long double f = (long double)wk * P / k[i];
            double T = DT[(size_t)(l - 2) * nk + i];
            tt += f * T * T;
            if (want_E) {
                double E = DE[(size_t)(l - 2) * nk + i];
                te += f * T * E;
                ee += f * E * E;
            }
        }
        Cl[l] = (double)(4.0L * pi * tt);
        Cl[(lmax + 1) + l] = (double)(4.0L * pi * te);
        Cl[2 * (lmax + 1) + l] = (double)(4.0L * pi * ee);
    }
}
