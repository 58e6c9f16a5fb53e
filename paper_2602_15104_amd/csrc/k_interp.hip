// Sources on a transfer k-grid (App. A.2, eq. k_transfer_spacing): the
// sources S[c][k][3][n_tau] of the perturbation grid are interpolated in k,
// at every output time and for each of the three types, by natural cubic
// splines, onto the points kt[n_kt] of a finer grid:
//
//   second derivatives M of each (cosmology, type, time) spline from the
//   tridiagonal system  h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
//   = 6 [(f_{i+1} - f_i)/h_i - (f_i - f_{i-1})/h_{i-1}],  M_0 = M_{n-1} = 0,
//   whose elimination factors depend on the k grid only and come from the
//   host; then  S(kt) = A f_i + B f_{i+1} + [(A^3 - A) M_i + (B^3 - B) M_{i+1}] h_i^2/6
//   with A = (k_{i+1} - kt)/h_i, B = 1 - A on the interval i holding kt.
//
// One thread per (cosmology, type, time): consecutive lanes take consecutive
// times, so every load and store of S, M and the result is coalesced (times
// are the fastest index of all three arrays).  The second-derivative kernel
// takes any number of types per mode (3 for the sources, 1 for the matter
// density contrast of the lensing potential).
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

namespace {

constexpr int BLOCK = 256;

// Thomas sweep: sub/diag/sup of the interior rows factored on the host as
// dinv[i] = 1/(pivot_i) and lo[i] = sub_i * dinv[i-1] (rows 1..n-2).
__global__ void __launch_bounds__(BLOCK) spline_m_kernel(const double *__restrict__ S, double *__restrict__ M,
                                                        const double *__restrict__ kg, const double *__restrict__ lo,
                                                        const double *__restrict__ dinv, int n_cosmo, int n_k,
                                                        int nty, int n_tau) {
    const long sys = (long)blockIdx.x * BLOCK + threadIdx.x;
    const long n_sys = (long)n_cosmo * nty * n_tau;
    if (sys >= n_sys) return;
    const int j = (int)(sys % n_tau);
    const int ty = (int)((sys / n_tau) % nty);
    const int c = (int)(sys / ((long)nty * n_tau));
    const size_t st = (size_t)nty * n_tau;  // stride between consecutive k
    const double *f = S + (size_t)c * n_k * st + (size_t)ty * n_tau + j;
    double *m = M + (size_t)c * n_k * st + (size_t)ty * n_tau + j;
    m[0] = 0.0;
    m[(size_t)(n_k - 1) * st] = 0.0;
    if (n_k < 3) return;
    // forward elimination of the right-hand sides
    double f0 = f[0], f1 = f[st];
    double hprev = kg[1] - kg[0];
    double yprev = 0.0;
    for (int i = 1; i < n_k - 1; ++i) {
        const double f2 = f[(size_t)(i + 1) * st];
        const double h = kg[i + 1] - kg[i];
        const double rhs = 6.0 * ((f2 - f1) / h - (f1 - f0) / hprev);
        const double y = rhs - lo[i] * yprev;  // lo[1] = 0
        m[(size_t)i * st] = y;
        yprev = y;
        f0 = f1;
        f1 = f2;
        hprev = h;
    }
    // back substitution: M_i = (y_i - h_i M_{i+1}) / pivot_i
    double mnext = 0.0;
    for (int i = n_k - 2; i >= 1; --i) {
        const double h = kg[i + 1] - kg[i];
        const double v = (m[(size_t)i * st] - h * mnext) * dinv[i];
        m[(size_t)i * st] = v;
        mnext = v;
    }
}

__global__ void __launch_bounds__(BLOCK) spline_eval_kernel(const double *__restrict__ S, const double *__restrict__ M,
                                                           const double *__restrict__ kg,
                                                           const int *__restrict__ seg, const double *__restrict__ kt,
                                                           double *__restrict__ St, int n_cosmo, int n_k, int n_tau,
                                                           int n_kt) {
    const long sys = (long)blockIdx.x * BLOCK + threadIdx.x;
    const long n_sys = (long)n_cosmo * 3 * n_tau;
    if (sys >= n_sys) return;
    const int j = (int)(sys % n_tau);
    const int ty = (int)((sys / n_tau) % 3);
    const int c = (int)(sys / (3L * n_tau));
    const size_t st = (size_t)3 * n_tau;
    const double *f = S + (size_t)c * n_k * st + (size_t)ty * n_tau + j;
    const double *m = M + (size_t)c * n_k * st + (size_t)ty * n_tau + j;
    double *out = St + (size_t)c * n_kt * st + (size_t)ty * n_tau + j;
    for (int q = 0; q < n_kt; ++q) {
        const int i = seg[q];
        const double h = kg[i + 1] - kg[i];
        const double A = (kg[i + 1] - kt[q]) / h, B = 1.0 - A;
        const double v = A * f[(size_t)i * st] + B * f[(size_t)(i + 1) * st] +
                         ((A * A * A - A) * m[(size_t)i * st] + (B * B * B - B) * m[(size_t)(i + 1) * st]) * h * h /
                             6.0;
        out[(size_t)q * st] = v;
    }
}

}  // namespace

int launch_spline_sources(const double *d_S, double *d_M, const double *d_kg, const double *d_lo,
                          const double *d_dinv, const int *d_seg, const double *d_kt, double *d_St, int n_cosmo,
                          int n_k, int n_tau, int n_kt, void *stream) {
    const long n_sys = (long)n_cosmo * 3 * n_tau;
    dim3 grid((unsigned)((n_sys + BLOCK - 1) / BLOCK)), block(BLOCK);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(spline_m_kernel, grid, block, 0, s, d_S, d_M, d_kg, d_lo, d_dinv, n_cosmo, n_k, 3, n_tau);
    hipLaunchKernelGGL(spline_eval_kernel, grid, block, 0, s, d_S, d_M, d_kg, d_seg, d_kt, d_St, n_cosmo, n_k, n_tau,
                       n_kt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("spline launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_spline_m(const double *d_F, double *d_M, const double *d_kg, const double *d_lo, const double *d_dinv,
                    int n_cosmo, int n_k, int nty, int n_tau, void *stream) {
    const long n_sys = (long)n_cosmo * nty * n_tau;
    dim3 grid((unsigned)((n_sys + BLOCK - 1) / BLOCK)), block(BLOCK);
    hipLaunchKernelGGL(spline_m_kernel, grid, block, 0, (hipStream_t)stream, d_F, d_M, d_kg, d_lo, d_dinv, n_cosmo,
                       n_k, nty, n_tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("spline launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
