// K2 variant: the line-of-sight projection with the paper's three-region
// spherical Bessel scheme (arXiv 2602.15104, App. B.4, the strategy stated
// below the transfer integrals) in place of the exact recurrence.
//
// For each multipole l >= 1:
//   * j_l(x) = 0 for x <= x_start(l), where x_start is the first x at which
//     j_l reaches 1e-10;
//   * linear interpolation on B3_PTS equally spaced samples of j_l over
//     [x_start(l), x_5(l)], x_5 being the fifth local maximum (positive peak)
//     of j_l;
//   * above x_5 the leading Debye-type form
//       j_l(x) ~ cos(Q(x) - pi/4) / sqrt(x sqrt(x^2 - nu^2)),
//       Q(x) = sqrt(x^2 - nu^2) - nu pi/2 + nu arcsin(nu/x),  nu = l + 1/2.
// The projection needs j_l' and j_l'': j_l' = j_{l-1} - (l+1) j_l / x from
// the scheme's own j_{l-1}, j_l, and j_l'' from Bessel's equation, so
//   (3 j'' + j)/2 = -(3/x) j' + (3 l(l+1)/(2 x^2) - 1) j.
//
// Table build (once per context, for every l up to the largest l_max asked
// for): one thread per l finds x_start by bisection on (0, nu] (j_l rises
// monotonically there) and x_5 by scanning j_l' from nu in steps of 1/4 for
// its fifth sign change from + to -, then bisection; one thread per sample
// evaluates j_l by Miller's downward recurrence.  Every loop has a fixed
// iteration bound.
//
// Projection: one 256-lane workgroup per (cosmology, k), lanes own output
// times as in the recurrence kernel; l runs upwards, each lane evaluating
// j_l at its own x_j and keeping j_{l-1}.  A lane stops one multipole above
// the last l with x_start(l) < x_j (beyond it j_l = j_{l-1} = 0).  Per-l
// partial sums are reduced through LDS in batches of 12 in a fixed order.
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

namespace {

constexpr int BLOCK = 256;
constexpr int LB = 12;
constexpr int PAD = 1;
constexpr double THRESH = 1e-10;
constexpr double PI = 3.141592653589793238462643383;

// j_l(x) and j_{l+1}(x) for x > 0 by Miller's downward recurrence
// J_{L-1} = (2L+1)/x J_L - J_{L+1} from L_s = max(x + 16 x^{1/3} + 24, l + 24),
// normalised by j_0 = sin x / x or j_1, whichever is larger.
__device__ void miller_pair(int l, double x, double &jl, double &jl1) {
    const double ix = 1.0 / x;
    int ls = (int)ceil(x + 16.0 * cbrt(x) + 24.0);
    if (ls < l + 24) ls = l + 24;
    double hi = 0.0, lo = 1e-200, rl = 0.0, rp = 0.0;
    for (int L = ls; L > 0; --L) {
        const double nlo = (2.0 * L + 1.0) * ix * lo - hi;
        hi = lo;
        lo = nlo;
        if (L - 1 == l) {
            rl = lo;
            rp = hi;
        }
        if (fabs(lo) > 1e250) {
            lo *= 1e-250;
            hi *= 1e-250;
            rl *= 1e-250;
            rp *= 1e-250;
        }
    }
    double sx, cx;
    sincos(x, &sx, &cx);
    const double j0 = sx * ix, j1 = (sx * ix - cx) * ix;
    const double sc = (fabs(j0) >= fabs(j1)) ? j0 / lo : j1 / hi;
    jl = rl * sc;
    jl1 = rp * sc;
}

__device__ inline double djl(int l, double x) {
    double j, j1;
    miller_pair(l, x, j, j1);
    return l / x * j - j1;
}

__global__ void __launch_bounds__(64) bessel3_edges_kernel(int l_lo, int l_hi, double *__restrict__ xs,
                                                           double *__restrict__ x5) {
    const int l = l_lo + blockIdx.x * 64 + threadIdx.x;
    if (l > l_hi) return;
    const double nu = l + 0.5;
    // x_start: j_l(x) = THRESH on (0, nu]
    double lo = 0.0, hi = nu;
    for (int it = 0; it < 200 && hi - lo > 4e-16 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        double j, j1;
        miller_pair(l, mid, j, j1);
        if (j > THRESH)
            hi = mid;
        else
            lo = mid;
    }
    xs[l - 1] = hi;
    // x_5: fifth + to - sign change of j_l' beyond nu (the first maximum lies
    // beyond nu); NaN if the bounded scan does not find it
    const int n_scan = 20 * (int)(60.0 + 8.0 * cbrt(nu));
    double xp = nu, dp = djl(l, nu), res = __builtin_nan("");
    int found = 0;
    for (int i = 1; i <= n_scan; ++i) {
        const double xc = nu + 0.25 * i;
        const double dc = djl(l, xc);
        if (dp > 0.0 && dc <= 0.0 && ++found == 5) {
            double a = xp, b = xc;
            for (int it = 0; it < 200 && b - a > 4e-16 * b; ++it) {
                const double m = 0.5 * (a + b);
                if (djl(l, m) > 0.0)
                    a = m;
                else
                    b = m;
            }
            res = 0.5 * (a + b);
            break;
        }
        xp = xc;
        dp = dc;
    }
    x5[l - 1] = res;
}

__global__ void __launch_bounds__(256) bessel3_samples_kernel(int l_lo, const double *__restrict__ xs,
                                                              const double *__restrict__ x5,
                                                              double *__restrict__ tab) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int l = l_lo + blockIdx.y;
    if (i >= B3_PTS) return;
    const double a = xs[l - 1], dx = (x5[l - 1] - a) / (B3_PTS - 1);
    double j, j1;
    miller_pair(l, a + dx * i, j, j1);
    tab[(size_t)(l - 1) * B3_PTS + i] = j;
}

__device__ inline double j3(int l, double x, const double *__restrict__ xs, const double *__restrict__ x5,
                            const double *__restrict__ tab) {
    const double a = xs[l - 1], b = x5[l - 1];
    if (x <= a) return 0.0;
    if (x <= b) {
        const double dx = (b - a) / (B3_PTS - 1);
        const double u = (x - a) / dx;
        int i = (int)floor(u);
        if (i > B3_PTS - 2) i = B3_PTS - 2;
        const double f = u - i;
        const double *t = tab + (size_t)(l - 1) * B3_PTS;
        return (1.0 - f) * t[i] + f * t[i + 1];
    }
    const double nu = l + 0.5;
    const double s = sqrt(x * x - nu * nu);
    return cos(s - nu * (PI / 2) + nu * asin(nu / x) - PI / 4) / sqrt(x * s);
}

template <int M>
__global__ void __launch_bounds__(BLOCK) los3_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k, int n_tau,
                                                     int ell_max, int want_E, double s_pol,
                                                     const double *__restrict__ S, const double *__restrict__ xs,
                                                     const double *__restrict__ x5, const double *__restrict__ tab,
                                                     double *__restrict__ Delta) {
    __shared__ double red[2][LB][BLOCK + PAD];
    __shared__ int s_lstop;
    const int tid = threadIdx.x;
    const int c = blockIdx.x % n_cosmo;
    const int ik = n_k - 1 - (int)(blockIdx.x / n_cosmo);
    const DevTab &tb = tabs[c];
    const double k = tb.k[ik];
    const double *S0 = S + ((size_t)c * n_k + ik) * 3 * n_tau;
    const double *S1 = S0 + n_tau;
    const double *S2 = S1 + n_tau;
    const int nl = ell_max - 1;
    double *DT = Delta + ((size_t)c * 2 * n_k + ik) * nl;  // this mode's rows of Delta[c][type][k][l - 2]
    double *DE = Delta + ((size_t)(c * 2 + 1) * n_k + ik) * nl;

    double cA[M], cB[M], cC[M], cE[M], xx[M], rx[M], jm[M];
    int lstop[M];
    double t2_extra = 0.0, e2_extra = 0.0;  // x = 0 limits (only l = 2)
    int my_stop = 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = tid + m * BLOCK;
        lstop[m] = 1;
        cA[m] = cB[m] = cC[m] = cE[m] = xx[m] = rx[m] = jm[m] = 0.0;
        if (j >= n_tau) continue;
        const double x = k * tb.chi_src[j];
        const double w = tb.w_src[j];
        // read once: nontemporal, as in los_kernel
        const double s0 = __builtin_nontemporal_load(S0 + j), s1 = __builtin_nontemporal_load(S1 + j),
                     s2 = __builtin_nontemporal_load(S2 + j);
        const double p2 = s_pol * s2;
        if (x == 0.0) {
            // j_l = j_l' = 0, (3j''+j)/2 = delta_l2/5, j_l/x^2 = delta_l2/15
            t2_extra += w * p2 * 0.2;
            e2_extra += w * s2 * (2.449489742783178098 / 15.0);
            continue;
        }
        const double ix = 1.0 / x;
        xx[m] = x;
        rx[m] = ix;
        cA[m] = w * (s0 - p2);
        cB[m] = 1.5 * w * p2 * ix * ix;
        cC[m] = w * s1 - 3.0 * w * p2 * ix;
        cE[m] = 2.449489742783178098 * w * s2 * ix * ix;
        jm[m] = j3(1, x, xs, x5, tab);
        // last l with x_start(l) < x (x_start rises with l), then one more
        int lo = 0, hi = ell_max;  // invariant: xs[lo-1] < x (l = lo active), l = hi+1 inactive
        if (xs[0] >= x) {
            hi = 0;
        } else {
            lo = 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (xs[mid - 1] < x)
                    lo = mid;
                else
                    hi = mid - 1;
            }
        }
        const int la = lo + 1 < ell_max ? lo + 1 : ell_max;
        lstop[m] = la;
        my_stop = la > my_stop ? la : my_stop;
    }
    if (tid == 0) s_lstop = 2;
    __syncthreads();
    atomicMax(&s_lstop, my_stop);
    __syncthreads();
    const int ltop = s_lstop;  // >= 2: l = 2 always visited (x = 0 terms)
    for (int l = ltop + 1 + tid; l <= ell_max; l += BLOCK) {
        DT[l - 2] = 0.0;
        DE[l - 2] = 0.0;
    }
    const int sum_id = tid >> 3, sub = tid & 7;
    for (int lb = 2; lb <= ltop; lb += LB) {
        const int nb = ltop - lb + 1 < LB ? ltop - lb + 1 : LB;  // multipoles lb .. lb+nb-1
        for (int i = 0; i < nb; ++i) {
            const int l = lb + i;
            const double fl = (double)l;
            const double q = fl * (fl + 1.0);
            double tacc = 0.0, eacc = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (l <= lstop[m]) {
                    const double j = j3(l, xx[m], xs, x5, tab);
                    const double jp = fma(-(fl + 1.0) * rx[m], j, jm[m]);
                    tacc = fma(j, fma(q, cB[m], cA[m]), fma(jp, cC[m], tacc));
                    eacc = fma(cE[m], j, eacc);
                    jm[m] = j;
                }
            }
            if (l == 2) {
                tacc += t2_extra;
                eacc += e2_extra;
            }
            red[0][i][tid] = tacc;
            red[1][i][tid] = eacc;
        }
        __syncthreads();
        {
            const int v = sum_id / LB, i = sum_id % LB;
            const bool valid = v < 2 && i < nb;
            double a = 0.0;
            if (valid) {
                for (int r = 0; r < BLOCK / 8; ++r) a += red[v][i][sub + 8 * r];
            }
            a += __shfl_xor(a, 1, 8);
            a += __shfl_xor(a, 2, 8);
            a += __shfl_xor(a, 4, 8);
            if (sub == 0 && valid) {
                const int l = lb + i;
                if (v == 0) {
                    DT[l - 2] = a;
                } else {
                    const double cl = sqrt(3.0 * (l + 2.0) * (l + 1.0) * l * (l - 1.0) / 8.0);
                    DE[l - 2] = want_E ? cl * a : 0.0;
                }
            }
        }
        __syncthreads();
    }
}

template <int M>
void launch_m(dim3 grid, hipStream_t s, const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max,
              int want_E, double s_pol, const double *d_S, const double *xs, const double *x5, const double *tab,
              double *d_Delta) {
    hipLaunchKernelGGL(los3_kernel<M>, grid, dim3(BLOCK), 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                       d_S, xs, x5, tab, d_Delta);
}

}  // namespace

int launch_bessel3_build(int l_lo, int l_hi, double *d_xs, double *d_x5, double *d_tab, void *stream) {
    if (l_lo < 1 || l_hi < l_lo) return CMB_OK;
    hipStream_t s = (hipStream_t)stream;
    const int n = l_hi - l_lo + 1;
    hipLaunchKernelGGL(bessel3_edges_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, l_lo, l_hi, d_xs, d_x5);
    hipLaunchKernelGGL(bessel3_samples_kernel, dim3((unsigned)((B3_PTS + 255) / 256), (unsigned)n), dim3(256), 0, s,
                       l_lo, d_xs, d_x5, d_tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("bessel table launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int launch_los3(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E, double s_pol,
                const double *d_S, const double *d_xs, const double *d_x5, const double *d_tab, double *d_Delta,
                void *stream) {
    dim3 grid((unsigned)(n_cosmo * n_k));
    hipStream_t s = (hipStream_t)stream;
    const int M = (n_tau + BLOCK - 1) / BLOCK;
    if (M <= 1)
        launch_m<1>(grid, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S, d_xs, d_x5, d_tab, d_Delta);
    else if (M <= 2)
        launch_m<2>(grid, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S, d_xs, d_x5, d_tab, d_Delta);
    else if (M <= 4)
        launch_m<4>(grid, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S, d_xs, d_x5, d_tab, d_Delta);
    else if (M <= 8)
        launch_m<8>(grid, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S, d_xs, d_x5, d_tab, d_Delta);
    else if (M <= 16)
        launch_m<16>(grid, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S, d_xs, d_x5, d_tab, d_Delta);
    else {
        set_error("n_tau too large for the line-of-sight kernel");
        return CMB_E_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("los3 launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
