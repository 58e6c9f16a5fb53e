// K3: k quadrature to the angular power spectra (arXiv 2602.15104, eq.
// c_ell_def with the primordial spectrum of eq. PK_pivot):
//   C_l^XY = 4 pi sum_i w_i P(k_i) Delta_X(l,k_i) Delta_Y(l,k_i) / k_i,
// trapezoid weights w_i on the mode grid, XY in {TT, TE, EE}.  One wavefront
// per (cosmology, l); lanes stride over k and the wavefront sum uses a fixed
// shuffle tree, so results are bitwise reproducible.  With dlog set, P(k) is
// weighted by ln(k/k_pivot): the derivative of C_l with respect to n_s.
//
// Also the finite-difference combination of spectra for the parameter
// derivatives (central or five-point stencil).
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {
namespace {

__global__ void __launch_bounds__(64) cl_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k, int ell_max,
                                                const double *__restrict__ Delta, double *__restrict__ Cl,
                                                long out_stride, int dlog) {
    const int c = blockIdx.y;
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const DevTab &tb = tabs[c];
    double *out = Cl + (size_t)c * out_stride;
    if (l < 2) {
        if (lane < 3) out[lane * (ell_max + 1) + l] = 0.0;
        return;
    }
    const int nl = ell_max - 1;
    const double *T = Delta + (size_t)c * 2 * nl * n_k + (size_t)(l - 2) * n_k;
    const double *E = T + (size_t)nl * n_k;
    double tt = 0.0, te = 0.0, ee = 0.0;
    for (int i = lane; i < n_k; i += 64) {
        double ki = tb.k[i];
        double kl = i > 0 ? tb.k[i - 1] : ki;
        double kr = i + 1 < n_k ? tb.k[i + 1] : ki;
        double f = 0.5 * (kr - kl) * tb.A_s * pow(ki / tb.k_pivot, tb.n_s - 1.0) / ki;
        if (dlog) f *= log(ki / tb.k_pivot);
        double t = T[i], e = E[i];
        tt = fma(f * t, t, tt);
        te = fma(f * t, e, te);
        ee = fma(f * e, e, ee);
    }
    for (int off = 32; off > 0; off >>= 1) {
        tt += __shfl_down(tt, off, 64);
        te += __shfl_down(te, off, 64);
        ee += __shfl_down(ee, off, 64);
    }
    if (lane == 0) {
        const double fpi = 4.0 * 3.14159265358979323846;
        out[l] = fpi * tt;
        out[(ell_max + 1) + l] = fpi * te;
        out[2 * (ell_max + 1) + l] = fpi * ee;
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
    dim3 grid((unsigned)(ell_max + 1), (unsigned)n_cosmo), block(64);
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
    dim3 grid((unsigned)(ell_max + 1), (unsigned)n_cosmo), block(64);
    hipLaunchKernelGGL(cl_kernel, grid, block, 0, (hipStream_t)stream, d_tabs, n_cosmo, n_k, ell_max, d_Delta, d_Cl,
                       (long)3 * (ell_max + 1), 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("cl launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
