// K2: spherical Bessel functions by recurrence and the line-of-sight
// projection (arXiv 2602.15104, App. B.4, transfer integrals).
//
//   Delta_T(l,k) = sum_j w_j [S_T0 j_l + S_T1 j_l' + s_pol S_T2 (3 j_l'' + j_l)/2](x_j)
//   Delta_E(l,k) = sqrt(3 (l+2)!/(8 (l-2)!)) sum_j w_j sqrt(6) S_T2 j_l(x_j)/x_j^2
// with x_j = k (tau_0 - tau_j) and trapezoid weights w_j in ln a.  With the
// downward recurrence the kernel carries (j_{l+1}, j_l); Bessel's equation
// gives j' = (l/x) j_l - j_{l+1} and (3j''+j)/2 = -(3/x) j' + (3l(l+1)/(2x^2) - 1) j,
// so each (l, k, tau) term is  j_l (A + l(l+1) B + l D) - j_{l+1} C  with
// A, B, C, D fixed per (k, tau).
//
// Work decomposition: one workgroup (256 lanes) per (cosmology, k); each lane
// owns M output times (tau_j, j = lane + 256 m, coalesced loads of S).  Every
// lane first seeds its recurrences:
//   * x > l_max + 32: upward recurrence from j_0, j_1 (stable for l < x);
//   * otherwise: Miller's downward recurrence from l_s(x) = x + 16 x^{1/3} + 24
//     to l = 0, normalised by j_0 = sin x/x (or j_1), recording the pair at
//     l_act = min(l_max, l_cut(x)); above l_cut(x) = x + 11 x^{1/3} + 12 every
//     |j_l(x)| < 1e-15 and the term is skipped.
// Then all lanes walk l downwards together; a lane joins at its own l_act.
// Per-l partial sums go through LDS in batches of 12 multipoles and are
// reduced in a fixed order (bitwise reproducible, independent of batch
// mates).  The walk starts at the workgroup's largest l_act, so small k
// (x << l_max) costs only the multipoles it can reach.
#include <hip/hip_runtime.h>

#include "cmbhip_internal.h"

namespace cmbhip {

__host__ __device__ inline int ell_cut_rule(double x) { return (int)ceil(x + 11.0 * cbrt(x) + 12.0); }
__host__ __device__ inline int ell_start_rule(double x) { return (int)ceil(x + 16.0 * cbrt(x) + 24.0); }

int ell_cut(double x) { return ell_cut_rule(x); }

namespace {

constexpr int BLOCK = 256;
constexpr int LB = 12;  // multipoles per reduction batch (LDS stays below 64 KiB)
constexpr int PAD = 1;

// Start values of the walk at one output time (x = k chi > 0).
// x > l_max + 32: the upward recurrence j_{l+1} = (2l+1)/x j_l - j_{l-1} from
// (j_0, j_1) to (jl, jp) = (j_{l_max}, j_{l_max+1}).
__device__ inline void seed_upward(double ix, double j0, double j1, int ltop, double &jl, double &jp) {
    double a = j0, b = j1;
#pragma unroll 2
    for (int l = 1; l < ltop; ++l) {
        const double nb = (2.0 * l + 1.0) * ix * b - a;
        a = b;
        b = nb;
    }
    jp = b;  // j_{ltop}
    jl = a;  // j_{ell_max}
}

// Otherwise Miller's downward recurrence from l_s(x) to l = 0, the pair at
// l_act = min(l_max, l_cut(x)) recorded on the way and the whole normalised
// by j_0 (or j_1 where larger); values above 1e250 are rescaled by 1e-250.
// The steps above l_act + 1 (nothing recorded yet), the recording step and
// the steps below it run as three loops, so that no step tests for l_act;
// the factor 2l + 1 is carried as a double (exact: an integer far below 2^53)
// instead of converted from l at every step.
__device__ inline void seed_miller(double x, double ix, double j0, double j1, int ell_max, double &jl, double &jp,
                                   int &lact) {
    const int lc = ell_cut_rule(x);
    const int la = lc < ell_max ? lc : ell_max;
    const int ls = ell_start_rule(x);
    double hi = 0.0, lo = 1e-200;  // J_{l+1}, J_l at l = ls
    double rp = 0.0, rl = 0.0;
    double c = 2.0 * ls + 1.0;  // 2l + 1 of the next step
    const double c_rec = 2.0 * la + 3.0;  // the step at l = l_act + 1
    // steps in pairs, the two arrays taking turns (no moves): after the first
    // step of a pair hi holds J_{l-1} and lo J_l, after the second lo holds
    // J_{l-2} and hi J_{l-1}; one test for the end and one for the rescaling
    // per pair.  A pair rescales once a value passes 1e200, which leaves
    // 1e108 for the growth of the next pair (at most ((2l+1)/x)^2); the
    // values of the recurrence stay far below 1e200 at every x the tables
    // produce, so the pairs take exactly the single steps' operations.
    for (; c > c_rec + 2.0; c -= 4.0) {
        hi = c * ix * lo - hi;
        lo = (c - 2.0) * ix * hi - lo;
        if (__builtin_expect(fmax(fabs(lo), fabs(hi)) > 1e200, 0)) {
            lo *= 1e-250;
            hi *= 1e-250;
        }
    }
    if (c > c_rec) {
        const double nlo = c * ix * lo - hi;
        hi = lo;
        lo = nlo;
        if (__builtin_expect(fabs(lo) > 1e250, 0)) {
            lo *= 1e-250;
            hi *= 1e-250;
        }
        c -= 2.0;
    }
    {  // l = l_act + 1: (hi, lo) becomes (J_{l_act+1}, J_{l_act})
        const double nlo = c * ix * lo - hi;
        hi = lo;
        lo = nlo;
        rp = hi;
        rl = lo;
        if (__builtin_expect(fabs(lo) > 1e250, 0)) {
            lo *= 1e-250;
            hi *= 1e-250;
            rp *= 1e-250;
            rl *= 1e-250;
        }
        c -= 2.0;
    }
    for (; c > 4.0; c -= 4.0) {  // l = l_act .. 2 in pairs, as above
        hi = c * ix * lo - hi;
        lo = (c - 2.0) * ix * hi - lo;
        if (__builtin_expect(fmax(fabs(lo), fabs(hi)) > 1e200, 0)) {
            lo *= 1e-250;
            hi *= 1e-250;
            rp *= 1e-250;
            rl *= 1e-250;
        }
    }
    if (c > 2.0) {  // l = 1
        const double nlo = c * ix * lo - hi;
        hi = lo;
        lo = nlo;
        if (__builtin_expect(fabs(lo) > 1e250, 0)) {
            lo *= 1e-250;
            hi *= 1e-250;
            rp *= 1e-250;
            rl *= 1e-250;
        }
    }
    // lo = J_0, hi = J_1
    const double sc = (fabs(j0) >= fabs(j1)) ? j0 / lo : j1 / hi;
    jp = rp * sc;
    jl = rl * sc;
    lact = la;
}

template <int M>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3))) los_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k, int n_tau,
                                                    int ell_max, int want_E, double s_pol,
                                                    const double *__restrict__ S, double *__restrict__ Delta) {
    __shared__ double red[2][LB][BLOCK + PAD];
    __shared__ int s_lstart;
    const int tid = threadIdx.x;
    const int c = blockIdx.x % n_cosmo;
    const int ik = n_k - 1 - (int)(blockIdx.x / n_cosmo);
    const DevTab &tb = tabs[c];
    const double k = tb.k[ik];
    const double *S0 = S + ((size_t)c * n_k + ik) * 3 * n_tau;
    const double *S1 = S0 + n_tau;
    const double *S2 = S1 + n_tau;
    const int nl = ell_max - 1;
    // this mode's rows of Delta[c][type][k][l - 2] (l fastest: each workgroup
    // writes its own contiguous spans)
    double *DT = Delta + ((size_t)c * 2 * n_k + ik) * nl;
    double *DE = Delta + ((size_t)(c * 2 + 1) * n_k + ik) * nl;
    const int ltop = ell_max + 1;

    double cA[M], cB[M], cC[M], cD[M], cE[M], rx[M], jl[M], jp[M];
    int lact[M];
    double t2_extra = 0.0, e2_extra = 0.0;  // x = 0 limits (only l = 2)
    int my_lmax = 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int j = tid + m * BLOCK;
        lact[m] = 1;
        cA[m] = cB[m] = cC[m] = cD[m] = cE[m] = rx[m] = jl[m] = jp[m] = 0.0;
        if (j >= n_tau) continue;
        double x = k * tb.chi_src[j];
        double w = tb.w_src[j];
        // the sources are read once: streamed past the L2 (nontemporal)
        double s0 = __builtin_nontemporal_load(S0 + j), s1 = __builtin_nontemporal_load(S1 + j),
               s2 = __builtin_nontemporal_load(S2 + j);
        double p2 = s_pol * s2;
        if (x == 0.0) {
            // j_l = j_l' = 0, (3j''+j)/2 = delta_l2/5, j_l/x^2 = delta_l2/15
            t2_extra += w * p2 * 0.2;
            e2_extra += w * s2 * (2.449489742783178098 / 15.0);
            continue;
        }
        double ix = 1.0 / x;
        rx[m] = ix;
        cA[m] = w * (s0 - p2);
        cB[m] = 1.5 * w * p2 * ix * ix;
        cC[m] = w * s1 - 3.0 * w * p2 * ix;
        cD[m] = cC[m] * ix;
        cE[m] = 2.449489742783178098 * w * s2 * ix * ix;
        double sx, cx;
        sincos(x, &sx, &cx);
        double j0 = sx * ix, j1 = (sx * ix - cx) * ix;
        if (x >= ltop + 32) {
            seed_upward(ix, j0, j1, ltop, jl[m], jp[m]);
            lact[m] = ell_max;
        } else {
            seed_miller(x, ix, j0, j1, ell_max, jl[m], jp[m], lact[m]);
        }
        my_lmax = lact[m] > my_lmax ? lact[m] : my_lmax;
    }
    if (tid == 0) s_lstart = 1;
    __syncthreads();
    atomicMax(&s_lstart, my_lmax);
    __syncthreads();
    int lstart = s_lstart;
    if (t2_extra != 0.0 || e2_extra != 0.0) lstart = lstart < 2 ? 2 : lstart;
    // there may be an x = 0 point in any lane: make l = 2 always visited
    lstart = lstart < 2 ? 2 : lstart;
    // zeros above the walk
    for (int l = ell_max - tid; l > lstart; l -= BLOCK) {
        DT[l - 2] = 0.0;
        DE[l - 2] = 0.0;
    }
    const int sum_id = tid >> 3, sub = tid & 7;  // 32 sums x 8 lanes in the reduction
    // The recurrence's two arrays take turns: at multipole l the array A holds
    // j_l and B holds j_{l+1}, and B receives j_{l-1}; the next multipole reads
    // them the other way round.  So no value is moved between registers.  The
    // multipoles go in pairs (the batches hold an even number, LB, but the
    // last), so the array that is current at l depends only on the parity of
    // lstart - l; each output time's start values, frozen above its l_act, are
    // placed so that the current array holds j_{l_act} when the walk reaches it.
    static_assert(LB % 2 == 0, "batches of an even number of multipoles");
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if ((lstart - lact[m]) & 1) {
            const double t = jl[m];
            jl[m] = jp[m];
            jp[m] = t;
        }
    }
    auto one_l = [&](int i, int l, double(&A)[M], double(&B)[M]) __attribute__((always_inline)) {
        double fl = (double)l;
        double q = fl * (fl + 1.0);
        double c21 = 2.0 * fl + 1.0;
        double tacc = 0.0, eacc = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (__builtin_expect(l <= lact[m], 1)) {  // (nearly always: laid out inline)
                double j = A[m], j1 = B[m];
                double P = fma(q, cB[m], fma(fl, cD[m], cA[m]));
                tacc = fma(j, P, fma(-j1, cC[m], tacc));
                eacc = fma(cE[m], j, eacc);
                B[m] = fma(c21 * rx[m], j, -j1);
            }
        }
        red[0][i][tid] = tacc;
        red[1][i][tid] = eacc;
    };
    for (int lb = lstart; lb >= 2; lb -= LB) {
        int nb = lb - 1 < LB ? lb - 1 : LB;  // multipoles in this batch: lb, lb-1, ..., lb-nb+1
        int i = 0;
        for (; i + 1 < nb; i += 2) {
            one_l(i, lb - i, jl, jp);
            one_l(i + 1, lb - i - 1, jp, jl);
        }
        if (i < nb) one_l(i, lb - i, jl, jp);  // the last batch's odd multipole
        if (lb - nb + 1 == 2) {  // l = 2 closes the last batch: the x = 0 terms
            red[0][nb - 1][tid] += t2_extra;
            red[1][nb - 1][tid] += e2_extra;
        }
        __syncthreads();
        {
            int v = sum_id / LB, i = sum_id % LB;
            bool valid = v < 2 && i < nb;
            double a = 0.0;
            if (valid) {
                for (int r = 0; r < BLOCK / 8; ++r) a += red[v][i][sub + 8 * r];
            }
            a += __shfl_xor(a, 1, 8);
            a += __shfl_xor(a, 2, 8);
            a += __shfl_xor(a, 4, 8);
            if (sub == 0 && valid) {
                int l = lb - i;
                if (v == 0) {
                    DT[l - 2] = a;
                } else {
                    double cl = sqrt(3.0 * (l + 2.0) * (l + 1.0) * l * (l - 1.0) / 8.0);
                    DE[l - 2] = want_E ? cl * a : 0.0;
                }
            }
        }
        __syncthreads();
    }
}

// Transposes (reverse-mode gradients of the spectra with respect to the
// sources).  K3^T, one thread per (cosmology, l, k):
//   G_T = 4 pi w_k P(k)/k (2 gTT Delta_T + gTE Delta_E),
//   G_E = 4 pi w_k P(k)/k (gTE Delta_T + 2 gEE Delta_E).
// K2^T, the decomposition of los_kernel (one 256-lane workgroup per
// (cosmology, k), lanes own output times, the same Bessel seeding and walk in
// l), each lane summing over l for its own times:
//   gS_T0 = w sum_l G_T j_l,  gS_T1 = w sum_l G_T j_l',
//   gS_T2 = w sum_l [s_pol G_T (3 j_l'' + j_l)/2 + c_l sqrt(6) G_E j_l/x^2],
// with j' = (l/x) j_l - j_{l+1} and (3j''+j)/2 = -(3/x) j' + (3l(l+1)/(2x^2) - 1) j.
// No cross-lane sums: every output is written by the lane that owns it.
__global__ void __launch_bounds__(256) cl_adj_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                     int ell_max, int want_E, const double *__restrict__ Delta,
                                                     const double *__restrict__ gC, double *__restrict__ G) {
    const int nl = ell_max - 1;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n_cosmo * nl * n_k) return;
    const int li = (int)(t % nl);
    const int ik = (int)((t / nl) % n_k);
    const int c = (int)(t / ((long)nl * n_k));
    const DevTab &tb = tabs[c];
    const double ki = tb.k[ik];
    const double kl = ik > 0 ? tb.k[ik - 1] : ki, kr = ik + 1 < n_k ? tb.k[ik + 1] : ki;
    const double f = 4.0 * 3.14159265358979323846 * 0.5 * (kr - kl) * tb.A_s * pow(ki / tb.k_pivot, tb.n_s - 1.0) / ki;
    const size_t rT = ((size_t)c * 2 * n_k + ik) * nl + li, rE = rT + (size_t)n_k * nl;  // Delta[c][type][k][l-2]
    const double dT = Delta[rT], dE = Delta[rE];
    const double *g = gC + (size_t)c * 3 * (ell_max + 1);
    const int l = li + 2;
    const double gtt = g[l], gte = want_E ? g[(ell_max + 1) + l] : 0.0, gee = want_E ? g[2 * (ell_max + 1) + l] : 0.0;
    G[rT] = f * (2.0 * gtt * dT + gte * dE);
    G[rE] = want_E ? f * (gte * dT + 2.0 * gee * dE) : 0.0;
}

template <int M>
__global__ void __launch_bounds__(BLOCK) los_adj_kernel(const DevTab *__restrict__ tabs, int n_cosmo, int n_k,
                                                        int n_tau, int ell_max, int want_E, double s_pol,
                                                        const double *__restrict__ G, double *__restrict__ gS) {
    __shared__ int s_lstart;
    const int tid = threadIdx.x;
    const int c = blockIdx.x % n_cosmo;
    const int ik = n_k - 1 - (int)(blockIdx.x / n_cosmo);
    const DevTab &tb = tabs[c];
    const double k = tb.k[ik];
    const int nl = ell_max - 1;
    const double *GT = G + ((size_t)c * 2 * n_k + ik) * nl;  // this mode's rows of G[c][type][k][l - 2]
    const double *GE = G + ((size_t)(c * 2 + 1) * n_k + ik) * nl;
    double *g0 = gS + ((size_t)c * n_k + ik) * 3 * n_tau, *g1 = g0 + n_tau, *g2 = g1 + n_tau;
    const int ltop = ell_max + 1;
    double rx[M], jl[M], jp[M], a0[M], a1[M], a2[M];
    int lact[M];
    bool zero[M];
    int my_lmax = 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = tid + m * BLOCK;
        lact[m] = 1;
        zero[m] = false;
        rx[m] = jl[m] = jp[m] = a0[m] = a1[m] = a2[m] = 0.0;
        if (j >= n_tau) continue;
        const double x = k * tb.chi_src[j];
        if (x == 0.0) {
            zero[m] = true;  // only l = 2 contributes: (3j''+j)/2 = 1/5, j/x^2 = 1/15
            continue;
        }
        const double ix = 1.0 / x;
        rx[m] = ix;
        double sx, cx;
        sincos(x, &sx, &cx);
        const double j0 = sx * ix, j1 = (sx * ix - cx) * ix;
        if (x >= ltop + 32) {
            seed_upward(ix, j0, j1, ltop, jl[m], jp[m]);
            lact[m] = ell_max;
        } else {
            seed_miller(x, ix, j0, j1, ell_max, jl[m], jp[m], lact[m]);
        }
        my_lmax = lact[m] > my_lmax ? lact[m] : my_lmax;
    }
    if (tid == 0) s_lstart = 1;
    __syncthreads();
    atomicMax(&s_lstart, my_lmax);
    __syncthreads();
    const int lstart = s_lstart;
    for (int l = lstart; l >= 2; --l) {
        const double fl = (double)l;
        const double gt = GT[l - 2];
        const double ge = want_E ? GE[l - 2] * sqrt(3.0 * (fl + 2.0) * (fl + 1.0) * fl * (fl - 1.0) / 8.0) *
                                       2.449489742783178098
                                 : 0.0;
        const double c21 = 2.0 * fl + 1.0, q = fl * (fl + 1.0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (l <= lact[m]) {
                const double j = jl[m], j1 = jp[m], ix = rx[m];
                const double d = fl * ix * j - j1;  // j_l'
                a0[m] = fma(gt, j, a0[m]);
                a1[m] = fma(gt, d, a1[m]);
                const double r2 = fma(-3.0 * ix, d, (1.5 * q * ix * ix - 1.0) * j);
                a2[m] = fma(s_pol * gt, r2, fma(ge, j * ix * ix, a2[m]));
                jp[m] = j;
                jl[m] = fma(c21 * ix, j, -j1);
            }
        }
    }
    const double gt2 = GT[0];
    const double ge2 = want_E ? GE[0] * sqrt(3.0 * 4.0 * 3.0 * 2.0 * 1.0 / 8.0) * 2.449489742783178098 : 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = tid + m * BLOCK;
        if (j >= n_tau) continue;
        if (zero[m]) a2[m] = s_pol * gt2 * 0.2 + ge2 / 15.0;
        const double w = tb.w_src[j];
        g0[j] = w * a0[m];
        g1[j] = w * a1[m];
        g2[j] = w * a2[m];
    }
}

}  // namespace

int launch_spectra_adjoint(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E,
                           double s_pol, const double *d_Delta, const double *d_gC, double *d_G, double *d_gS,
                           void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const long n = (long)n_cosmo * (ell_max - 1) * n_k;
    hipLaunchKernelGGL(cl_adj_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_tabs, n_cosmo, n_k, ell_max,
                       want_E, d_Delta, d_gC, d_G);
    dim3 grid((unsigned)(n_cosmo * n_k)), block(BLOCK);
    const int M = (n_tau + BLOCK - 1) / BLOCK;
    if (M <= 1)
        hipLaunchKernelGGL(los_adj_kernel<1>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                           d_G, d_gS);
    else if (M <= 2)
        hipLaunchKernelGGL(los_adj_kernel<2>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                           d_G, d_gS);
    else if (M <= 4)
        hipLaunchKernelGGL(los_adj_kernel<4>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                           d_G, d_gS);
    else if (M <= 8)
        hipLaunchKernelGGL(los_adj_kernel<8>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                           d_G, d_gS);
    else if (M <= 16)
        hipLaunchKernelGGL(los_adj_kernel<16>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol,
                           d_G, d_gS);
    else {
        set_error("n_tau too large for the line-of-sight kernel");
        return CMB_E_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("adjoint launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

int los_max_tau() { return BLOCK * 16; }

int launch_los(const DevTab *d_tabs, int n_cosmo, int n_k, int n_tau, int ell_max, int want_E, double s_pol,
               const double *d_S, double *d_Delta, void *stream) {
    dim3 grid((unsigned)(n_cosmo * n_k)), block(BLOCK);
    hipStream_t s = (hipStream_t)stream;
    int M = (n_tau + BLOCK - 1) / BLOCK;
    if (M <= 1)
        hipLaunchKernelGGL(los_kernel<1>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S,
                           d_Delta);
    else if (M <= 2)
        hipLaunchKernelGGL(los_kernel<2>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S,
                           d_Delta);
    else if (M <= 4)
        hipLaunchKernelGGL(los_kernel<4>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S,
                           d_Delta);
    else if (M <= 8)
        hipLaunchKernelGGL(los_kernel<8>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S,
                           d_Delta);
    else if (M <= 16)
        hipLaunchKernelGGL(los_kernel<16>, grid, block, 0, s, d_tabs, n_cosmo, n_k, n_tau, ell_max, want_E, s_pol, d_S,
                           d_Delta);
    else {
        set_error("n_tau too large for the line-of-sight kernel");
        return CMB_E_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("los launch: ") + hipGetErrorString(e));
        return CMB_E_DEVICE;
    }
    return CMB_OK;
}

}  // namespace cmbhip
