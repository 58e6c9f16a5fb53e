// K3: k quadrature to the angular power spectra (arXiv 2602.15104, eq.
// c_ell_def with the primordial spectrum of eq. PK_pivot):
//   C_l^XY = 4 pi sum_i w_i P(k_i) Delta_X(l,k_i) Delta_Y(l,k_i) / k_i,
// trapezoid weights w_i on the mode grid, XY in {TT, TE, EE}.  One wavefront
// per (cosmology, l); lanes stride over k and the wavefront sum uses a fixed
// shuffle tree, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {
namespace {

__global__ void __launch_bounds__(64) cl_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k, int ell_max,
                                                const double *__restrict__ Delta, double *__restrict__ Cl) {
    const int c = blockIdx.y;
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const DevTab &tb = tabs[c];
    double *out = Cl + (size_t)c * 3 * (ell_max + 1);
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

}  // namespace

int launch_cl(const DevTab *d_tabs, int n_cosmo, int n_k, int ell_max, const double *d_Delta, double *d_Cl,
              void *stream) {
    dim3 grid((unsigned)(ell_max + 1), (unsigned)n_cosmo), block(64);
    hipLaunchKernelGGL(cl_kernel, grid, block, 0, (hipStream_t)stream, d_tabs, n_cosmo, n_k, ell_max, d_Delta, d_Cl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("cl launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
