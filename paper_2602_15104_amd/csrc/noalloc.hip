// cmb_solve_noalloc: the whole path (perturbations and sources, projection,
// k quadrature) with every intermediate in a fixed, library-owned device
// array, so that the call allocates nothing.  For callers that cannot
// allocate device memory.
//
// The array `scratch` below is one per device (each device that loads the
// library holds its own copy until the process ends).  In host code its name
// is a host-side stand-in, not a device address: the address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is used on the host (kernel arguments, copies).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "cmbhip_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)CMB_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// the current device's scratch address (taken once per device)
int scratch_of_current(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        cmbhip::set_error("cmb_solve_noalloc: no current HIP device");
        return CMB_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            cmbhip::set_error(std::string("cmb_solve_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return CMB_E_DEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return CMB_OK;
}

// Descriptors travel as kernel arguments (copied at launch), so no host
// buffer has to outlive the call; each launch writes up to kPack of them.
constexpr int kPack = 8;
struct DescPack {
    cmbhip::DevTab d[kPack];
};
static_assert(sizeof(DescPack) <= 3072, "descriptor pack fits the kernel-argument space");

__global__ void put_desc(DescPack p, int n, cmbhip::DevTab *dst) {
    // one lane per double of the packed descriptors (plain vector stores)
    const int nd = n * (int)(sizeof(cmbhip::DevTab) / sizeof(double));
    const double *src = reinterpret_cast<const double *>(p.d);
    double *out = reinterpret_cast<double *>(dst);
    for (int i = threadIdx.x; i < nd; i += blockDim.x) out[i] = src[i];
}
static_assert(sizeof(cmbhip::DevTab) % sizeof(double) == 0, "descriptor is whole doubles");

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t cmb_noalloc_scratch_bytes(void) { return kScratchBytes; }

int cmb_solve_noalloc(const cmb_tables *const *tabs, int n_cosmo, int ell_max, double *d_Cl, int32_t *d_status,
                      int32_t *d_nsteps, void *stream) {
    if (!d_Cl || !d_status) {
        cmbhip::set_error("cmb_solve_noalloc: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        cmbhip::set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    cmbhip::Batch b;
    int rc = cmbhip::check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    if (b.n_tau > cmbhip::los_max_tau()) {
        cmbhip::set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    if (!cmbhip::perturb2_supported(b.prec)) {
        cmbhip::set_error("hierarchy larger than the perturbation kernel holds (320 state rows, 16 momentum nodes)");
        return CMB_E_UNSUPPORTED;
    }
    // layout: descriptors | tables | sources | transfer functions | step counts
    const size_t n = (size_t)n_cosmo;
    size_t off = up256(sizeof(cmbhip::DevTab) * n);
    const size_t o_T = off;
    for (size_t i = 0; i < n; ++i) off += up256(cmbhip::table_doubles(cmbhip::tables_of(tabs[i])) * sizeof(double));
    const size_t o_S = off;
    off += up256(sizeof(double) * n * b.n_k * 3 * b.n_tau);
    const size_t o_D = off;
    off += up256(sizeof(double) * n * 2 * (size_t)(ell_max - 1) * b.n_k);
    const size_t o_N = off;
    off += up256(sizeof(int32_t) * n * b.n_k);
    if (off > kScratchBytes) {
        cmbhip::set_error("cmb_solve_noalloc: tables, sources and transfer functions of this batch exceed the "
                          "library's fixed scratch (cmb_noalloc_scratch_bytes)");
        return CMB_E_NOMEM;
    }
    void *base = nullptr;
    rc = scratch_of_current(&base);
    if (rc) return rc;
    char *sb = static_cast<char *>(base);
    hipStream_t s = (hipStream_t)stream;
    // table arrays: copied from the tables' own host arrays
    DescPack pack;
    size_t to = o_T;
    for (size_t i = 0; i < n; ++i) {
        const cmbhip::Tables &t = cmbhip::tables_of(tabs[i]);
        const double *dp = reinterpret_cast<const double *>(sb + to);
        hipError_t e = hipSuccess;
        cmbhip::describe_table(t, dp, pack.d[i % kPack], [&](const double *src, size_t nd, const double *dst) {
            if (nd && e == hipSuccess)
                e = hipMemcpyAsync(const_cast<double *>(dst), src, nd * sizeof(double), hipMemcpyHostToDevice, s);
        });
        if (e != hipSuccess) {
            cmbhip::set_error(std::string("cmb_solve_noalloc: table copy: ") + hipGetErrorString(e));
            return CMB_E_DEVICE;
        }
        to += up256(cmbhip::table_doubles(t) * sizeof(double));
        const int filled = (int)(i % kPack) + 1;
        if (filled == kPack || i + 1 == n) {
            cmbhip::DevTab *dst = reinterpret_cast<cmbhip::DevTab *>(sb) + (i + 1 - filled);
            hipLaunchKernelGGL(put_desc, dim3(1), dim3(256), 0, s, pack, filled, dst);
            e = hipGetLastError();
            if (e != hipSuccess) {
                cmbhip::set_error(std::string("cmb_solve_noalloc: descriptor launch: ") + hipGetErrorString(e));
                return CMB_E_DEVICE;
            }
        }
    }
    const cmbhip::DevTab *d_tabs = reinterpret_cast<const cmbhip::DevTab *>(sb);
    double *S = reinterpret_cast<double *>(sb + o_S);
    double *D = reinterpret_cast<double *>(sb + o_D);
    int32_t *ns = d_nsteps ? d_nsteps : reinterpret_cast<int32_t *>(sb + o_N);
    rc = cmbhip::launch_perturb2(d_tabs, n_cosmo, b.n_k, b.n_tau, b.prec, S, d_status, ns, nullptr, nullptr, stream);
    if (rc) return rc;
    rc = cmbhip::launch_los(d_tabs, n_cosmo, b.n_k, b.n_tau, ell_max, b.polar, b.s_pol, S, D, stream);
    if (rc) return rc;
    rc = cmbhip::launch_cl(d_tabs, n_cosmo, b.n_k, ell_max, D, d_Cl, stream);
    if (rc == CMB_OK) cmbhip::set_error("");
    return rc;
}

}  // extern "C"
