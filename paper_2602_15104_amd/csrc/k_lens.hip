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

}  // namespace cmbhip
