// Lensing (arXiv 2602.15104, App. B.5).
//
// Lensing potential by Limber's approximation:
//   C_l^psipsi = 8 pi^2 / (l+1/2)^3  int_0^chi_* dchi/chi  P_psi(k = (l+1/2)/chi, tau_0 - chi)
//                                                        ((chi_* - chi)/chi_*)^2,
//   P_psi(k, a) = 9 Omega_m^2 H^4 / (8 pi^2 k) P(k, a),  P(k, a) = 2 pi^2/k^3 P_R(k) delta_m^2,
// so the integrand is (3/2 a^2 rho_m)^2 P_R(k) delta_m(k, tau)^2 / k^4 per unit
// chi, chi.  The host folds the time quadrature (the output-time weights in
// tau), 1/chi, (3/2 a^2 rho_m)^2 and the window ((chi_* - chi)/chi_*)^2 into
// one weight per output time (zero outside 0 < chi < chi_*).  delta_m(k, tau_j)
// at k = (l+1/2)/chi_j comes from the natural cubic spline in k of the
// perturbation grid's values at that output time, and is zero outside the
// grid's k range.
//
// One 256-lane workgroup per (cosmology, l); lanes stride over output times,
// so the loads of delta_m and its spline coefficients at neighbouring times
// are neighbouring addresses.  The sum over times is a fixed-order LDS tree.
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

namespace {

constexpr int BLOCK = 256;
constexpr double PI = 3.141592653589793238462643383;

__global__ void __launch_bounds__(BLOCK) limber_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                       int n_tau, int ell_max, const double *__restrict__ Dm,
                                                       const double *__restrict__ M, double *__restrict__ Clpp) {
    __shared__ double red[BLOCK];
    const int tid = threadIdx.x;
    const int c = blockIdx.x % n_cosmo;
    const int l = blockIdx.x / n_cosmo;
    double *out = Clpp + (size_t)c * (ell_max + 1);
    if (l < 2) {
        if (tid == 0) out[l] = 0.0;
        return;
    }
    const DevTab &tb = tabs[c];
    const double *kg = tb.k;
    const double k_lo = kg[0], k_hi = kg[n_k - 1];
    const double nu = l + 0.5;
    const double *D = Dm + (size_t)c * n_k * n_tau;
    const double *Mc = M + (size_t)c * n_k * n_tau;
    double acc = 0.0;
    for (int j = tid; j < n_tau; j += BLOCK) {
        const double w = tb.lens_w[j];
        if (w == 0.0) continue;
        const double kk = nu / tb.chi_src[j];
        if (!(kk >= k_lo && kk <= k_hi)) continue;
        // interval i with k_i <= kk <= k_{i+1}, i <= n_k - 2
        int lo = 0, hi = n_k - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (kg[mid] <= kk)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int i = lo;
        const double h = kg[i + 1] - kg[i];
        const double A = (kg[i + 1] - kk) / h, B = 1.0 - A;
        const double f0 = D[(size_t)i * n_tau + j], f1 = D[(size_t)(i + 1) * n_tau + j];
        const double m0 = Mc[(size_t)i * n_tau + j], m1 = Mc[(size_t)(i + 1) * n_tau + j];
        const double d = A * f0 + B * f1 + ((A * A * A - A) * m0 + (B * B * B - B) * m1) * h * h / 6.0;
        const double prim = tb.A_s * pow(kk / tb.k_pivot, tb.n_s - 1.0);
        const double k2 = kk * kk;
        acc += w * prim * d * d / (k2 * k2);
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) out[l] = 8.0 * PI * PI / (nu * nu * nu) * red[0];
}

}  // namespace

int launch_limber(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, const double *d_Dm,
                  const double *d_M, double *d_Clpp, void *stream) {
    dim3 grid((unsigned)((long)n_cosmo * (ell_max + 1))), block(BLOCK);
    hipLaunchKernelGGL(limber_kernel, grid, block, 0, (hipStream_t)stream, d_tabs, n_cosmo, n_k, n_tau, ell_max, d_Dm,
                       d_M, d_Clpp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("limber launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}


// ---------------------------------------------------------------------------
// Lensed spectra from full-sky correlation functions over the whole range of
// mu = cos(beta) (Gauss-Legendre nodes), following the correlation-function
// method of Challinor & Lewis (2005) that the paper implements:
//   C_gl(b) = sum_l (2l+1)/(4 pi) l(l+1) C^psi_l d^l_11,  C_gl,2 with d^l_{1,-1},
//   sigma^2 = C_gl(0) - C_gl(b),
// the lensing changes of xi_T, xi_+, xi_-, xi_x at each node from the small-
// deflection X functions (the leading products as X^2 - 1 through expm1), and
// the back transforms C~ - C = 2 pi sum_i w_i xi(mu_i) d^l(mu_i) with d00,
// d22, d2-2 and d20.  Wigner d functions run by the three-term recurrence in
// l from host coefficients (d^{l+1} = (a_l mu - b_l) d^l - g_l d^{l-1}) and
// host start values at l0 = max(|m'|, |m|).
//
// Kernel 1: one thread per (cosmology, node), two passes over l (the
// deflection correlations, then the four correlation changes with thirteen
// recurrences).  Kernel 2: one thread per node and a 256-node block per
// (cosmology, block); per-l partial sums through LDS in batches of six
// multipoles, in a fixed order.  Kernel 3: the blocks' partial sums in a fixed
// order plus the unlensed spectra.
namespace {

constexpr int NPAIR = 13;  // 00 11 1-1 22 2-2 31 3-3 40 4-4 02 3-1 20 -24
__host__ __device__ constexpr int pair_l0(int p) {
    return p == 0 ? 0 : (p <= 2 ? 1 : (p <= 4 ? 2 : (p <= 6 ? 3 : (p <= 8 ? 4 : (p == 9 ? 2 : (p == 10 ? 3 : (p == 11 ? 2 : 4)))))));
}
constexpr int LBB = 6;

struct Rec {
    double prev, cur;
};

// advance pair p from l-1 to l (l > l0) or start it (l == l0)
__device__ inline void rec_to(Rec &r, int p, int l, double mu, const double *__restrict__ coef,
                              const double *__restrict__ start, int i, int n_mu) {
    const int l0 = pair_l0(p);
    if (l < l0) return;
    if (l == l0) {
        r.prev = 0.0;
        r.cur = start[(size_t)p * n_mu + i];
        return;
    }
    const double *cf = coef + ((size_t)(l - 1) * NPAIR + p) * 3;
    const double nx = fma(cf[0], mu, -cf[1]) * r.cur - cf[2] * r.prev;
    r.prev = r.cur;
    r.cur = nx;
}

__global__ void __launch_bounds__(256) lens_xi_kernel(int n_cosmo, int L, int n_mu, const double *__restrict__ Cl,
                                                      const double *__restrict__ Clpp, const double *__restrict__ mu_n,
                                                      const double *__restrict__ coef,
                                                      const double *__restrict__ lfac, const double *__restrict__ start,
                                                      double *__restrict__ xi) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n_mu) return;
    const double mu = mu_n[i];
    const double *Cp = Clpp + (size_t)c * (L + 1);
    const double *T = Cl + (size_t)c * 3 * (L + 1), *X = T + (L + 1), *E = X + (L + 1);
    const double inv4pi = 1.0 / (4.0 * PI);
    // pass 1: deflection correlations
    Rec r11{0.0, 0.0}, r1m1{0.0, 0.0};
    rec_to(r11, 1, 1, mu, coef, start, i, n_mu);
    rec_to(r1m1, 2, 1, mu, coef, start, i, n_mu);
    double Cgl = 0.0, Cgl2 = 0.0, Cgl0 = 0.0;
    for (int l = 2; l <= L; ++l) {
        rec_to(r11, 1, l, mu, coef, start, i, n_mu);
        rec_to(r1m1, 2, l, mu, coef, start, i, n_mu);
        const double f = (2.0 * l + 1.0) * inv4pi * l * (l + 1.0) * Cp[l];
        Cgl = fma(f, r11.cur, Cgl);
        Cgl2 = fma(f, r1m1.cur, Cgl2);
        Cgl0 += f;
    }
    const double s = Cgl0 - Cgl, c2 = Cgl2;
    // X_imn = E0 * exp(k s / 4) * (l-dependent factor): the per-node constants
    const double e220 = exp(2.0 * s / 4.0), e022 = exp(4.0 * s / 4.0), e121 = exp((8.0 / 3.0) * s / 4.0),
                 e132 = exp((20.0 / 3.0) * s / 4.0), e242 = exp(10.0 * s / 4.0);
    // pass 2: the four correlation changes
    Rec r[NPAIR];
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) r[p] = Rec{0.0, 0.0};
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) {
        for (int l = 0; l <= 1; ++l) rec_to(r[p], p, l, mu, coef, start, i, n_mu);
    }
    double xT = 0.0, xP = 0.0, xM = 0.0, xX = 0.0;
    for (int l = 2; l <= L; ++l) {
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) rec_to(r[p], p, l, mu, coef, start, i, n_mu);
        const double d00 = r[0].cur, d11 = r[1].cur, d1m1 = r[2].cur, d22 = r[3].cur, d2m2 = r[4].cur,
                     d31 = r[5].cur, d3m3 = r[6].cur, d40 = r[7].cur, d4m4 = r[8].cur, d02 = r[9].cur,
                     d3m1 = r[10].cur, d20 = r[11].cur, dm24 = r[12].cur;
        const double ll = l * (l + 1.0);
        const double *lf = lfac + (size_t)l * 4;  // sqrt factors of X220, X121, X132, X242
        const double E0 = exp(-ll * s / 4.0);
        const double p000 = -ll / 4.0 * E0;
        const double X220 = lf[0] * E0 * e220, X022 = E0 * e022, p022 = -(ll - 4.0) / 4.0 * X022;
        const double X121 = lf[1] * E0 * e121, X132 = lf[2] * E0 * e132, X242 = lf[3] * E0 * e242;
        const double X112 = X121;
        const double dT = expm1(-ll * s / 2.0), dP = expm1(-(ll - 4.0) * s / 2.0),
                     dX = expm1(-(2.0 * ll - 4.0) * s / 4.0);
        const double pre = (2.0 * l + 1.0) * inv4pi;
        const double cc2 = c2 * c2;
        xT += pre * T[l] *
              (dT * d00 + 8.0 / ll * c2 * p000 * p000 * d1m1 + cc2 * (p000 * p000 * d00 + X220 * X220 * d2m2));
        xP += pre * E[l] * (dP * d22 + 2.0 * c2 * X132 * X121 * d31 + cc2 * (p022 * p022 * d22 + X242 * X220 * d40));
        xM += pre * E[l] *
              (dP * d2m2 + c2 * (X121 * X121 * d1m1 + X132 * X132 * d3m3) +
               0.5 * cc2 * (2.0 * p022 * p022 * d2m2 + X220 * X220 * d00 + X242 * X242 * d4m4));
        xX += pre * X[l] *
              (dX * d02 + c2 * 2.0 * p000 / sqrt(ll) * (X112 * d11 + X132 * d3m1) +
               0.5 * cc2 * ((2.0 * p022 * p000 + X220 * X220) * d20 + X220 * X242 * dm24));
    }
    double *o = xi + (size_t)c * 4 * n_mu;
    o[i] = xT;
    o[n_mu + i] = xP;
    o[2 * n_mu + i] = xM;
    o[3 * n_mu + i] = xX;
}

__global__ void __launch_bounds__(256) lens_back_kernel(int n_cosmo, int n_mu, int lmax, const double *__restrict__ mu_n,
                                                        const double *__restrict__ w_n, const double *__restrict__ coef,
                                                        const double *__restrict__ start, const double *__restrict__ xi,
                                                        double *__restrict__ part) {
    __shared__ double red[4][LBB][256 + 1];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * 256 + tid;
    const int c = blockIdx.y;
    const int nblk = gridDim.x;
    const bool act = i < n_mu;
    const int ii = act ? i : 0;
    const double mu = mu_n[ii];
    const double *x = xi + (size_t)c * 4 * n_mu;
    const double wT = act ? w_n[ii] * x[ii] : 0.0, wP = act ? w_n[ii] * x[n_mu + ii] : 0.0,
                 wM = act ? w_n[ii] * x[2 * n_mu + ii] : 0.0, wX = act ? w_n[ii] * x[3 * n_mu + ii] : 0.0;
    // pairs 00, 22, 2-2, 20 (indices 0, 3, 4, 11)
    Rec a{0.0, 0.0}, b{0.0, 0.0}, m{0.0, 0.0}, x20{0.0, 0.0};
    for (int l = 0; l <= 1; ++l) rec_to(a, 0, l, mu, coef, start, ii, n_mu);
    double *pc = part + ((size_t)c * nblk + blockIdx.x) * 4 * (lmax + 1);
    const int sum_id = tid >> 3, sub = tid & 7;
    for (int lb = 2; lb <= lmax; lb += LBB) {
        const int nb = lmax - lb + 1 < LBB ? lmax - lb + 1 : LBB;
        for (int q = 0; q < nb; ++q) {
            const int l = lb + q;
            rec_to(a, 0, l, mu, coef, start, ii, n_mu);
            rec_to(b, 3, l, mu, coef, start, ii, n_mu);
            rec_to(m, 4, l, mu, coef, start, ii, n_mu);
            rec_to(x20, 11, l, mu, coef, start, ii, n_mu);
            red[0][q][tid] = wT * a.cur;
            red[1][q][tid] = wP * b.cur;
            red[2][q][tid] = wM * m.cur;
            red[3][q][tid] = wX * x20.cur;
        }
        __syncthreads();
        {
            const int v = sum_id / LBB, q = sum_id % LBB;
            const bool valid = v < 4 && q < nb;
            double s = 0.0;
            if (valid)
                for (int r = 0; r < 32; ++r) s += red[v][q][sub + 8 * r];
            s += __shfl_xor(s, 1, 8);
            s += __shfl_xor(s, 2, 8);
            s += __shfl_xor(s, 4, 8);
            if (sub == 0 && valid) pc[(size_t)v * (lmax + 1) + lb + q] = s;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) lens_sum_kernel(int n_cosmo, int L, int lmax, int nblk,
                                                       const double *__restrict__ Cl, const double *__restrict__ part,
                                                       double *__restrict__ Cll) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n_cosmo * (lmax + 1)) return;
    const int c = (int)(t / (lmax + 1)), l = (int)(t % (lmax + 1));
    double *o = Cll + (size_t)c * 4 * (lmax + 1);
    if (l < 2) {
        o[l] = o[(lmax + 1) + l] = o[2 * (lmax + 1) + l] = o[3 * (lmax + 1) + l] = 0.0;
        return;
    }
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int bk = 0; bk < nblk; ++bk) {
        const double *pc = part + ((size_t)c * nblk + bk) * 4 * (lmax + 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) s[v] += pc[(size_t)v * (lmax + 1) + l];
    }
    const double *T = Cl + (size_t)c * 3 * (L + 1), *X = T + (L + 1), *E = X + (L + 1);
    const double tp = 2.0 * PI;
    const double p = tp * s[1], mm = tp * s[2];
    o[l] = T[l] + tp * s[0];
    o[(lmax + 1) + l] = X[l] + tp * s[3];
    o[2 * (lmax + 1) + l] = E[l] + 0.5 * (p + mm);
    o[3 * (lmax + 1) + l] = 0.5 * (p - mm);
}

}  // namespace

int lens_back_blocks(int n_mu) { return (n_mu + 255) / 256; }

int launch_lensed_cl(int n_cosmo, int L, int lmax, int n_mu, const double *d_Cl, const double *d_Clpp,
                     const double *d_mu, const double *d_w, const double *d_coef, const double *d_lfac,
                     const double *d_start, double *d_xi, double *d_part, double *d_Cll, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const int nblk = lens_back_blocks(n_mu);
    hipLaunchKernelGGL(lens_xi_kernel, dim3((unsigned)nblk, (unsigned)n_cosmo), dim3(256), 0, s, n_cosmo, L, n_mu, d_Cl,
                       d_Clpp, d_mu, d_coef, d_lfac, d_start, d_xi);
    hipLaunchKernelGGL(lens_back_kernel, dim3((unsigned)nblk, (unsigned)n_cosmo), dim3(256), 0, s, n_cosmo, n_mu, lmax,
                       d_mu, d_w, d_coef, d_start, d_xi, d_part);
    const long n = (long)n_cosmo * (lmax + 1);
    hipLaunchKernelGGL(lens_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_cosmo, L, lmax, nblk, d_Cl,
                       d_part, d_Cll);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("lensing launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
