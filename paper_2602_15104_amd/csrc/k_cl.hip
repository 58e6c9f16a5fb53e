// K3: k quadrature to the angular power spectra (arXiv 2602.15104, eq.
// c_ell_def with the primordial spectrum of eq. PK_pivot):
//   C_l^XY = 4 pi sum_i w_i P(k_i) Delta_X(l,k_i) Delta_Y(l,k_i) / k_i,
// trapezoid weights w_i on the mode grid, XY in {TT, TE, EE}.  One lane per
// (cosmology, l): with Delta[c][type][k][l - 2] the lanes of a wavefront
// read consecutive l of one k (coalesced), and each lane sums over k in
// order, so results are bitwise reproducible.  The k weights w_i P(k_i)/k_i
// of the cosmology are formed once per workgroup in LDS (in chunks of
// CL_KCHUNK modes).  With dlog set, P(k) is weighted by ln(k/k_pivot): the
// derivative of C_l with respect to n_s.
//
// Also the finite-difference combination of spectra for the parameter
// derivatives (central or five-point stencil).
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {
namespace {

constexpr int CL_BLOCK = 256;
constexpr int CL_KCHUNK = 2048;

__global__ void __launch_bounds__(CL_BLOCK) cl_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                      int ell_max, const double *__restrict__ Delta,
                                                      double *__restrict__ Cl, long out_stride, int dlog) {
    __shared__ double wk[CL_KCHUNK];
    const int c = blockIdx.y;
    const int l = blockIdx.x * CL_BLOCK + threadIdx.x;
    const DevTab &tb = tabs[c];
    double *out = Cl + (size_t)c * out_stride;
    const int nl = ell_max - 1;
    const bool on = l >= 2 && l <= ell_max;
    const double *T = Delta + (size_t)c * 2 * n_k * nl + (on ? l - 2 : 0);
    const double *E = T + (size_t)n_k * nl;
    double tt = 0.0, te = 0.0, ee = 0.0;
    for (int k0 = 0; k0 < n_k; k0 += CL_KCHUNK) {
        const int nk = n_k - k0 < CL_KCHUNK ? n_k - k0 : CL_KCHUNK;
        __syncthreads();  // the previous chunk's weights are no longer read
        for (int j = threadIdx.x; j < nk; j += CL_BLOCK) {
            const int i = k0 + j;
            const double ki = tb.k[i];
            const double kl = i > 0 ? tb.k[i - 1] : ki;
            const double kr = i + 1 < n_k ? tb.k[i + 1] : ki;
            double f = 0.5 * (kr - kl) * tb.A_s * pow(ki / tb.k_pivot, tb.n_s - 1.0) / ki;
            if (dlog) f *= log(ki / tb.k_pivot);
            wk[j] = f;
        }
        __syncthreads();
        if (on) {
            const double *Tc = T + (size_t)k0 * nl, *Ec = E + (size_t)k0 * nl;
            for (int j = 0; j < nk; ++j) {
                const double f = wk[j], t = Tc[(size_t)j * nl], e = Ec[(size_t)j * nl];
                tt = fma(f * t, t, tt);
                te = fma(f * t, e, te);
                ee = fma(f * e, e, ee);
            }
        }
    }
    if (l <= ell_max) {
        const double fpi = 4.0 * 3.14159265358979323846;
        out[l] = on ? fpi * tt : 0.0;
        out[(ell_max + 1) + l] = on ? fpi * te : 0.0;
        out[2 * (ell_max + 1) + l] = on ? fpi * ee : 0.0;
    }
}

// J[c][0..3(l+1)) = stencil of C[m][c] (m = +1, -1, +2, -2 steps) / e[c]:
// central (C+1 - C-1)/(2e) or five-point (8 (C+1 - C-1) - (C+2 - C-2))/(12 e)
__global__ void __launch_bounds__(256) fd_kernel(int n_base, int n3, int order, const double *__restrict__ C,
                                                 const double *__restrict__ e, double *__restrict__ J,
                                                 long j_stride) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n_base * n3) return;
    const int c = (int)(t / n3), i = (int)(t % n3);
    const size_t ms = (size_t)n_base * n3;
    const double *p = C + (size_t)c * n3 + i;
    const double d1 = p[0] - p[ms];
    double v;
    if (order == 4) {
        const double d2 = p[2 * ms] - p[3 * ms];
        v = (8.0 * d1 - d2) / (12.0 * e[c]);
    } else {
        v = d1 / (2.0 * e[c]);
    }
    J[(size_t)c * j_stride + i] = v;
}

// base status takes the first failing replay's status of the same mode
__global__ void __launch_bounds__(256) merge_status_kernel(int n_base, int n_k, int n_rep, const int *__restrict__ rep,
                                                           int *__restrict__ st) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n_base * n_k) return;
    if (st[t] != 0) return;
    for (int m = 0; m < n_rep; ++m) {
        const int r = rep[(size_t)m * n_base * n_k + t];
        if (r != 0) {
            st[t] = r;
            return;
        }
    }
}

}  // namespace

int launch_fd(int n_base, int ell_max, int order, const double *d_C, const double *d_e, double *d_J, long j_stride,
              void *stream) {
    const int n3 = 3 * (ell_max + 1);
    const long n = (long)n_base * n3;
    hipLaunchKernelGGL(fd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n_base, n3,
                       order, d_C, d_e, d_J, j_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("fd launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_merge_status(int n_base, int n_k, int n_rep, const int *d_rep, int *d_st, void *stream) {
    const long n = (long)n_base * n_k;
    hipLaunchKernelGGL(merge_status_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       n_base, n_k, n_rep, d_rep, d_st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("status launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_cl_ex(const DevTab *d_tabs, int n_cosmo, int n_k, int ell_max, const double *d_Delta, double *d_Cl,
                 long out_stride, int dlog, void *stream) {
    dim3 grid((unsigned)((ell_max + CL_BLOCK) / CL_BLOCK), (unsigned)n_cosmo), block(CL_BLOCK);
    hipLaunchKernelGGL(cl_kernel, grid, block, 0, (hipStream_t)stream, d_tabs, n_cosmo, n_k, ell_max, d_Delta, d_Cl,
                       out_stride, dlog);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("cl launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_cl(const DevTab *d_tabs, int n_cosmo, int n_k, int ell_max, const double *d_Delta, double *d_Cl,
              void *stream) {
    return launch_cl_ex(d_tabs, n_cosmo, n_k, ell_max, d_Delta, d_Cl, (long)3 * (ell_max + 1), 0, stream);
}

}  // namespace cmbhip
