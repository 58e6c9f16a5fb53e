// C ABI of libcmbhip: argument validation, device contexts, table upload and
// the ordering of the three stages on the caller's HIP stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <memory>
#include <string>
#include <thread>

#include "cmbhip_internal.h"

struct cmb_tables {
    cmbhip::Tables t;
};

namespace cmbhip {

size_t table_doubles(const Tables &t) {
    return t.poly.size() + 2 * t.k.size() + 4 * t.lna_src.size() + 2 * t.q.size();
}

void pack_table(const Tables &t, double *hp, const double *dp, DevTab &x) {
    describe_table(t, dp, x, [&](const double *src, size_t n, const double *dst) {
        if (n) std::memcpy(hp + (dst - dp), src, n * sizeof(double));
    });
}

DevPrec dev_prec(const cmb_prec &p, int nq) {
    DevPrec d{};
    d.lg = p.ell_gamma;
    d.lp = p.ell_pol;
    d.ln = p.ell_nu;
    d.max_steps = p.max_steps;
    d.nq = nq;
    d.lq = nq > 0 ? p.ell_ncdm : 0;
    d.pcoeff = p.pcoeff;
    d.icoeff = p.icoeff;
    d.dcoeff = p.dcoeff;
    d.sw = p.scale_sw;
    d.isw = p.scale_isw;
    d.dop = p.scale_dop;
    d.pol = p.scale_pol;
    d.grav = p.gravity_scale;
    d.thom = p.thomson_scale;
    return d;
}

}  // namespace cmbhip

struct cmb_ctx {
    int device = 0;
    size_t budget = 0;
    // device buffers (grown on demand within the budget)
    void *tab_buf = nullptr;
    size_t tab_cap = 0;
    void *ws_buf = nullptr;
    size_t ws_cap = 0;
    void *s_buf = nullptr;
    size_t s_cap = 0;
    void *d_buf = nullptr;
    size_t d_cap = 0;
    void *st_buf = nullptr;
    size_t st_cap = 0;
    // host staging for uploads (pinned)
    void *h_stage = nullptr;
    size_t h_cap = 0;
    // transfer-grid interpolation: small device arrays and their pinned staging
    void *kt_buf = nullptr;
    size_t kt_cap = 0;
    void *kt_stage = nullptr;
    size_t kt_stage_cap = 0;
    // three-region Bessel table: x_start[L] | x_5[L] | samples[L][B3_PTS], built for l <= b3_lmax
    void *b3_buf = nullptr;
    size_t b3_cap = 0;
    int b3_lmax = 0;
    // lensed spectra: nodes | weights | recurrence coefficients | X factors | start values, for (lens_L, lens_nmu)
    void *lens_buf = nullptr;
    size_t lens_cap = 0;
    int lens_L = 0, lens_nmu = 0;
    // cache key of the resident tables, their device descriptors and a host copy
    std::vector<unsigned long long> resident;
    cmbhip::DevTab *d_tabs = nullptr;
    std::vector<cmbhip::DevTab> h_tabs;
    // completion of the last call's device work and the stream it ran on: a
    // call on another stream waits for it before it touches the buffers above
    hipEvent_t done_ev = nullptr;
    hipStream_t done_stream = nullptr;
    bool done_live = false;
    std::mutex mu;
};

namespace cmbhip {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
static std::atomic<unsigned long long> g_uid{1};
}  // namespace cmbhip

using cmbhip::set_error;

static int herr(hipError_t e, const char *what) {
    if (e == hipSuccess) return CMB_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return CMB_E_DEVICE;
}

extern "C" {

int cmb_abi_version(void) { return CMB_ABI_VERSION; }

const char *cmb_last_error(void) { return cmbhip::g_err.c_str(); }

int cmb_defaults(cmb_cosmo *c, cmb_prec *p) {
    if (!c && !p) {
        set_error("cmb_defaults: both pointers NULL");
        return CMB_E_INVALID;
    }
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (c) {
        // App. A.2 defaults
        c->h = 0.6736;
        c->omega_b = 0.02237;
        c->omega_cdm = 0.120;
        c->A_s = 2.1e-9;
        c->n_s = 0.9649;
        c->tau_reio = 0.05430842;
        c->z_reio = nan;
        c->Delta_z_reio = 0.5;
        c->z_reio_He = 3.5;
        c->Delta_z_reio_He = 0.5;
        c->exp_reio = 1.5;
        c->YHe = 0.245;
        c->TCMB0 = 2.34865418e-4;
        c->Neff = nan;
        c->N_nu_massless = nan;
        c->T_nu_massless = 0.71636856;
        c->N_nu_massive = 0.0;
        c->m_nu_massive = 0.06;
        c->T_nu_massive = 0.71611;
    }
    if (p) {
        p->ell_gamma = 12;
        p->ell_pol = 10;
        p->ell_nu = 17;
        p->n_q = 0;
        p->ell_ncdm = 17;
        p->max_steps = 2048;
        p->n_tab = 8192;
        p->rtol_small = 1e-5;
        p->rtol_large = 1e-4;
        p->atol_small = 1e-10;
        p->atol_large = 1e-6;
        p->k_split = 1e-2;
        p->R_tc = 1.5e-3;
        p->R_large = 7e-2;
        p->k_pivot = 0.05;
        p->pcoeff = 0.25;
        p->icoeff = 0.8;
        p->dcoeff = 0.0;
        p->scale_sw = p->scale_isw = p->scale_dop = p->scale_pol = 1.0;
        p->gravity_scale = p->thomson_scale = 1.0;
    }
    set_error("");
    return CMB_OK;
}

int cmb_tables_build(const cmb_cosmo *c, const cmb_prec *p, const double *k, int n_k, int n_tau, cmb_tables **out) {
    if (!c || !p || !k || !out) {
        set_error("cmb_tables_build: NULL argument");
        return CMB_E_INVALID;
    }
    *out = nullptr;
    cmb_tables *t = new (std::nothrow) cmb_tables;
    if (!t) {
        set_error("out of host memory");
        return CMB_E_INVALID;
    }
    int rc;
    try {
        rc = cmbhip::build_tables(*c, *p, k, n_k, n_tau, t->t);
    } catch (const std::exception &e) {
        set_error(std::string("table build failed: ") + e.what());
        rc = CMB_E_INVALID;
    }
    if (rc != CMB_OK) {
        delete t;
        return rc;
    }
    t->t.uid = cmbhip::g_uid.fetch_add(1);
    *out = t;
    set_error("");
    return CMB_OK;
}

void cmb_tables_destroy(cmb_tables *t) { delete t; }

int cmb_tables_export(const cmb_tables *tt, cmb_table_view *v) {
    if (!tt || !v) {
        set_error("cmb_tables_export: NULL argument");
        return CMB_E_INVALID;
    }
    const cmbhip::Tables &t = tt->t;
    std::memset(v, 0, sizeof(*v));
    v->n_k = (int)t.k.size();
    v->n_tau = (int)t.lna_src.size();
    v->n_tab = t.n_tab;
    v->n_q = (int)t.q.size();
    v->L0 = t.L0;
    v->dlna = t.dl;
    v->tau0 = t.tau0;
    v->z_reio = t.z_reio;
    v->lna_tc = t.lna_tc;
    v->N_massless = t.N_massless;
    v->Neff = t.Neff;
    v->R_nu = t.R_nu;
    v->k = t.k.data();
    v->lna_start = t.lna_start.data();
    v->lna_src = t.lna_src.data();
    v->tau_src = t.tau_src.data();
    v->chi_src = t.chi_src.data();
    v->w_src = t.w_src.data();
    v->tau_star = t.tau_star;
    v->chi_star = t.chi_star;
    v->lens_w = t.lens_w.data();
    v->xe = t.xe.data();
    v->tm = t.tm.data();
    v->ln_dk = t.col[0].data();
    v->kappa = t.col[1].data();
    v->ln_cs2 = t.col[2].data();
    v->ln_tau = t.col[3].data();
    v->M_ln_dk = t.M[0].data();
    v->M_kappa = t.M[1].data();
    v->M_ln_cs2 = t.M[2].data();
    v->M_ln_tau = t.M[3].data();
    v->q = t.q.data();
    v->W = t.W.data();
    v->rt_g0 = t.rt_g0;
    v->rt_ur0 = t.rt_ur0;
    v->rt_c0 = t.rt_c0;
    v->rt_b0 = t.rt_b0;
    v->rt_L = t.rt_L;
    v->pref_ncdm = t.pref_ncdm;
    v->m_over_T = t.m_over_T;
    v->H0 = t.H0;
    return CMB_OK;
}

int cmb_ctx_create(int device, size_t budget, cmb_ctx **out) {
    if (!out) {
        set_error("cmb_ctx_create: NULL out");
        return CMB_E_INVALID;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        set_error("no HIP device available");
        return CMB_E_DEVICE;
    }
    if (device < 0 || device >= n) {
        set_error("device index out of range");
        return CMB_E_INVALID;
    }
    cmb_ctx *c = new (std::nothrow) cmb_ctx;
    if (!c) return CMB_E_INVALID;
    c->device = device;
    c->budget = budget ? budget : (size_t)16 << 30;
    {
        int prev = 0;
        (void)hipGetDevice(&prev);
        e = hipSetDevice(device);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            delete c;
            set_error(std::string("cmb_ctx_create: ") + hipGetErrorString(e));
            return CMB_E_DEVICE;
        }
    }
    *out = c;
    set_error("");
    return CMB_OK;
}

void cmb_ctx_destroy(cmb_ctx *c) {
    if (!c) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (void *p : {c->tab_buf, c->ws_buf, c->s_buf, c->d_buf, c->st_buf, c->kt_buf, c->b3_buf, c->lens_buf})
        hipFree(p);
    if (c->h_stage) hipHostFree(c->h_stage);
    if (c->kt_stage) hipHostFree(c->kt_stage);
    if (c->done_ev) hipEventDestroy(c->done_ev);
    hipSetDevice(prev);
    delete c;
}

}  // extern "C"

namespace {

size_t total_bytes(const cmb_ctx *c) {
    return c->tab_cap + c->ws_cap + c->s_cap + c->d_cap + c->st_cap + c->kt_cap + c->b3_cap + c->lens_cap;
}

int grow(cmb_ctx *c, void **buf, size_t *cap, size_t need, hipStream_t s) {
    if (need <= *cap) return CMB_OK;
    size_t newcap = need + need / 4;
    if (total_bytes(c) - *cap + newcap > c->budget) {
        newcap = need;
        if (total_bytes(c) - *cap + newcap > c->budget) {
            set_error("device memory budget of the context exceeded");
            return CMB_E_NOMEM;
        }
    }
    if (*buf) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
        hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc(buf, newcap);
    if (e != hipSuccess) {
        *buf = nullptr;
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return CMB_E_NOMEM;
    }
    *cap = newcap;
    return CMB_OK;
}

}  // namespace

namespace cmbhip {

int check_batch(const cmb_tables *const *tabs, int n_cosmo, Batch &b) {
    if (!tabs || n_cosmo < 1) {
        set_error("tables array NULL or n_cosmo < 1");
        return CMB_E_INVALID;
    }
    for (int i = 0; i < n_cosmo; ++i)
        if (!tabs[i]) {
            set_error("NULL table in batch");
            return CMB_E_INVALID;
        }
    const cmbhip::Tables &t0 = tabs[0]->t;
    b.n_k = (int)t0.k.size();
    b.n_tau = (int)t0.lna_src.size();
    const cmb_prec &p = t0.prec;
    for (int i = 1; i < n_cosmo; ++i) {
        const cmbhip::Tables &t = tabs[i]->t;
        const cmb_prec &q = t.prec;
        if ((int)t.k.size() != b.n_k || (int)t.lna_src.size() != b.n_tau || q.ell_gamma != p.ell_gamma ||
            q.ell_pol != p.ell_pol || q.ell_nu != p.ell_nu || t.q.size() != t0.q.size() ||
            (!t.q.empty() && q.ell_ncdm != p.ell_ncdm) || q.max_steps != p.max_steps ||
            q.pcoeff != p.pcoeff || q.icoeff != p.icoeff || q.dcoeff != p.dcoeff || q.scale_sw != p.scale_sw ||
            q.scale_isw != p.scale_isw || q.scale_dop != p.scale_dop || q.scale_pol != p.scale_pol ||
            q.gravity_scale != p.gravity_scale || q.thomson_scale != p.thomson_scale) {
            set_error("cosmologies in one call must share n_k, n_tau and the static options");
            return CMB_E_INVALID;
        }
    }
    b.prec = cmbhip::dev_prec(p, (int)t0.q.size());
    b.polar = p.ell_pol > 0;
    b.s_pol = p.scale_pol;
    return CMB_OK;
}

const Tables &tables_of(const cmb_tables *t) { return t->t; }

}  // namespace cmbhip

namespace {

using cmbhip::Batch;
using cmbhip::check_batch;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t table_bytes(const cmbhip::Tables &t) { return align256(cmbhip::table_doubles(t) * sizeof(double)); }

// Upload the batch's tables (skipped when the same tables are resident).
int upload(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, hipStream_t s) {
    std::vector<unsigned long long> key(n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) key[i] = tabs[i]->t.uid;
    if (key == c->resident) return CMB_OK;
    // the cache names no tables until this upload has been queued: a failure
    // below (the buffer regrown, staging reallocated) must not leave it
    // pointing at freed or half-written memory
    c->resident.clear();
    c->d_tabs = nullptr;
    c->h_tabs.clear();
    size_t bytes = align256(sizeof(cmbhip::DevTab) * n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) bytes += table_bytes(tabs[i]->t);
    int rc = grow(c, &c->tab_buf, &c->tab_cap, bytes, s);
    if (rc) return rc;
    if (bytes > c->h_cap) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
        if (c->h_stage) hipHostFree(c->h_stage);
        c->h_stage = nullptr;
        c->h_cap = 0;
        e = hipHostMalloc(&c->h_stage, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return herr(e, "hipHostMalloc");
        c->h_cap = bytes;
    } else {
        // the staging buffer may still be read by a previous upload
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    }
    char *h = (char *)c->h_stage;
    char *d = (char *)c->tab_buf;
    size_t off = align256(sizeof(cmbhip::DevTab) * n_cosmo);
    cmbhip::DevTab *dt = (cmbhip::DevTab *)h;
    for (int i = 0; i < n_cosmo; ++i) {
        const cmbhip::Tables &t = tabs[i]->t;
        cmbhip::pack_table(t, (double *)(h + off), (const double *)(d + off), dt[i]);
        off += table_bytes(t);
    }
    hipError_t e = hipMemcpyAsync(c->tab_buf, c->h_stage, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return herr(e, "hipMemcpyAsync (tables)");
    c->d_tabs = (cmbhip::DevTab *)c->tab_buf;
    c->resident = key;
    c->h_tabs.assign(dt, dt + n_cosmo);
    return CMB_OK;
}

struct DeviceGuard {
    int prev = 0;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (ok) hipSetDevice(prev);
    }
};

// Calls on one context may name different streams, and later calls reuse,
// overwrite or regrow the context's buffers (tables, staging, scratch).  So
// every call first makes its stream wait for the previous call's device work
// (an event recorded at that call's end on its stream), and records the event
// on its own stream when it returns.  Construct after taking the context lock
// with the context's device current; rc != CMB_OK means the wait could not
// be queued.
struct StreamOrder {
    cmb_ctx *c;
    hipStream_t s;
    int rc = CMB_OK;
    StreamOrder(cmb_ctx *c_, void *stream) : c(c_), s((hipStream_t)stream) {
        if (c->done_live && c->done_stream != s) rc = herr(hipStreamWaitEvent(s, c->done_ev, 0), "hipStreamWaitEvent");
    }
    ~StreamOrder() {
        if (rc != CMB_OK) return;
        c->done_live = hipEventRecord(c->done_ev, s) == hipSuccess;
        c->done_stream = s;
    }
};

}  // namespace

extern "C" {

size_t cmb_solve_workspace_bytes(const cmb_tables *const *tabs, int n_cosmo) {
    Batch b;
    if (check_batch(tabs, n_cosmo, b)) return 0;
    size_t bytes = align256(sizeof(cmbhip::DevTab) * n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) bytes += table_bytes(tabs[i]->t);
    bytes += align256(sizeof(int32_t) * (size_t)n_cosmo * b.n_k);  // step counts when the caller passes none
    return bytes;
}

}  // extern "C"

namespace {

int perturb_impl(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                 int32_t *d_nsteps, double *d_Pk, void *stream, double *d_Dm = nullptr) {
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    if (!cmbhip::perturb2_supported(b.prec)) {
        set_error("hierarchy of " + std::to_string(cmbhip::state_rows(b.prec)) +
                  " state rows: the perturbation kernel holds at most 320 (five rows on each of 64 lanes) "
                  "and 16 momentum nodes");
        return CMB_E_UNSUPPORTED;
    }
    int32_t *ns2 = d_nsteps;
    if (!ns2) {
        rc = grow(c, &c->st_buf, &c->st_cap, sizeof(int32_t) * (size_t)n_cosmo * b.n_k, s);
        if (rc) return rc;
        ns2 = (int32_t *)c->st_buf;
    }
    rc = cmbhip::launch_perturb2(c->d_tabs, n_cosmo, b.n_k, b.n_tau, b.prec, d_S, d_status, ns2, d_Pk, d_Dm, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

}  // namespace

extern "C" {

int cmb_perturb(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                int32_t *d_nsteps, void *stream) {
    if (!c || !d_S || !d_status) {
        set_error("cmb_perturb: NULL argument");
        return CMB_E_INVALID;
    }
    return perturb_impl(c, tabs, n_cosmo, d_S, d_status, d_nsteps, nullptr, stream);
}

int cmb_perturb_pk(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                   int32_t *d_nsteps, double *d_Pk, void *stream) {
    if (!c || !d_S || !d_status || !d_Pk) {
        set_error("cmb_perturb_pk: NULL argument");
        return CMB_E_INVALID;
    }
    return perturb_impl(c, tabs, n_cosmo, d_S, d_status, d_nsteps, d_Pk, stream);
}

int cmb_perturb_matter(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                       int32_t *d_nsteps, double *d_Pk, double *d_Dm, void *stream) {
    if (!c || !d_S || !d_status || (!d_Pk && !d_Dm)) {
        set_error("cmb_perturb_matter: NULL argument");
        return CMB_E_INVALID;
    }
    return perturb_impl(c, tabs, n_cosmo, d_S, d_status, d_nsteps, d_Pk, stream, d_Dm);
}

int cmb_los(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S, double *d_Delta,
            void *stream) {
    if (!c || !d_S || !d_Delta) {
        set_error("cmb_los: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    if (b.n_tau > cmbhip::los_max_tau()) {
        set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    rc = upload(c, tabs, n_cosmo, (hipStream_t)stream);
    if (rc) return rc;
    rc = cmbhip::launch_los(c->d_tabs, n_cosmo, b.n_k, b.n_tau, ell_max, b.polar, b.s_pol, d_S, d_Delta, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_cl(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Delta, double *d_Cl,
           void *stream) {
    if (!c || !d_Delta || !d_Cl) {
        set_error("cmb_cl: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    rc = upload(c, tabs, n_cosmo, (hipStream_t)stream);
    if (rc) return rc;
    rc = cmbhip::launch_cl(c->d_tabs, n_cosmo, b.n_k, ell_max, d_Delta, d_Cl, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_solve(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, double *d_S, double *d_Delta,
              double *d_Cl, int32_t *d_status, int32_t *d_nsteps, void *stream) {
    if (!c || !d_Cl || !d_status) {
        set_error("cmb_solve: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!d_S) {
        std::lock_guard<std::mutex> lk(c->mu);
        DeviceGuard g(c->device);
        if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
        StreamOrder so(c, stream);
        if (so.rc) return so.rc;
        rc = grow(c, &c->s_buf, &c->s_cap, sizeof(double) * (size_t)n_cosmo * b.n_k * 3 * b.n_tau, s);
        if (rc) return rc;
        d_S = (double *)c->s_buf;
    }
    if (!d_Delta) {
        std::lock_guard<std::mutex> lk(c->mu);
        DeviceGuard g(c->device);
        if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
        StreamOrder so(c, stream);
        if (so.rc) return so.rc;
        rc = grow(c, &c->d_buf, &c->d_cap, sizeof(double) * (size_t)n_cosmo * 2 * (ell_max - 1) * b.n_k, s);
        if (rc) return rc;
        d_Delta = (double *)c->d_buf;
    }
    rc = cmb_perturb(c, tabs, n_cosmo, d_S, d_status, d_nsteps, stream);
    if (rc) return rc;
    rc = cmb_los(c, tabs, n_cosmo, ell_max, d_S, d_Delta, stream);
    if (rc) return rc;
    return cmb_cl(c, tabs, n_cosmo, ell_max, d_Delta, d_Cl, stream);
}

}  // extern "C"

namespace {

// Transfer k-grid constants: the fiducial values of App. A.2 (k_min_tau0,
// k_max_tau0_over_l_max, tau0_fid, tau_rec_fid, k_transfer_linstep,
// k_transfer_logstep).
constexpr double kMinTau0 = 0.1, kMaxTau0PerL = 1.8, kTau0Fid = 1.418668e4, kTauRecFid = 281.040565;
constexpr double kLinStep = 0.45, kLogStep = 170.0;

}  // namespace

extern "C" {

int cmb_transfer_kgrid(int ell_max, double k_lo, double k_hi, double *k_out, int cap) {
    if (ell_max < 2 || !(k_lo > 0) || !(k_hi > k_lo) || cap < 0 || (cap > 0 && !k_out)) {
        set_error("cmb_transfer_kgrid: ell_max >= 2, 0 < k_lo < k_hi, cap >= 0");
        return -CMB_E_INVALID;
    }
    const double kmin = std::max(kMinTau0 / kTau0Fid, k_lo);
    const double kmax = std::min(kMaxTau0PerL * ell_max / kTau0Fid, k_hi);
    if (!(kmax > kmin)) {
        set_error("cmb_transfer_kgrid: empty range");
        return -CMB_E_INVALID;
    }
    const double kperiod = 2.0 * M_PI / (kTau0Fid - kTauRecFid);
    int n = 0;
    double k = kmin;
    while (k < kmax) {
        if (n < cap) k_out[n] = k;
        ++n;
        k += kperiod * kLinStep * k / (k + kLinStep / kLogStep);
    }
    if (n < cap) k_out[n] = kmax;
    ++n;
    set_error("");
    return n;
}

}  // extern "C"

// Thomas factors of the natural-spline system on the grid kg (interior rows
// 1..n-2): dinv[i] = 1/pivot_i, lo[i] = sub_i / pivot_{i-1}
static void spline_factors(const std::vector<double> &kg, std::vector<double> &lo, std::vector<double> &dinv) {
    const int nk = (int)kg.size();
    lo.assign(nk, 0.0);
    dinv.assign(nk, 0.0);
    for (int i = 1; i < nk - 1; ++i) {
        const double hm = kg[i] - kg[i - 1], hp = kg[i + 1] - kg[i];
        double piv = 2.0 * (hm + hp);
        if (i > 1) {
            lo[i] = hm * dinv[i - 1];
            piv -= lo[i] * hm;  // sub_i = h_{i-1}, sup_{i-1} = h_{i-1}
        }
        dinv[i] = 1.0 / piv;
    }
}

// the context's three-region Bessel table covering l <= ell_max (rebuilt
// whole, on the caller's stream, when a larger l_max is asked for)
static int ensure_bessel3(cmb_ctx *c, int ell_max, hipStream_t s) {
    if (c->b3_lmax >= ell_max) return CMB_OK;
    const size_t need = sizeof(double) * (size_t)ell_max * (2 + cmbhip::B3_PTS);
    c->b3_lmax = 0;
    int rc = grow(c, &c->b3_buf, &c->b3_cap, need, s);
    if (rc) return rc;
    double *xs = (double *)c->b3_buf, *x5 = xs + ell_max, *tab = x5 + ell_max;
    rc = cmbhip::launch_bessel3_build(1, ell_max, xs, x5, tab, s);
    if (rc) return rc;
    std::vector<double> h(2 * (size_t)ell_max);
    hipError_t e = hipMemcpyAsync(h.data(), xs, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return herr(e, "bessel table build");
    for (int l = 1; l <= ell_max; ++l)
        if (!(h[ell_max + l - 1] > h[l - 1]) || (l > 1 && !(h[l - 1] >= h[l - 2]))) {
            set_error("bessel table build: x_start / x_5 search failed at l = " + std::to_string(l));
            return CMB_E_DEVICE;
        }
    c->b3_lmax = ell_max;
    return CMB_OK;
}

// Wigner d^l_{m'm} at l = max(|m'|, |m|) by the explicit sum (long double)
static double wigner_d_start(int mp, int m, double mu) {
    const int l = std::max(std::abs(mp), std::abs(m));
    auto fact = [](int n) {
        long double f = 1.0L;
        for (int i = 2; i <= n; ++i) f *= i;
        return f;
    };
    const long double c2 = (1.0L + mu) / 2.0L, s2 = std::max((1.0L - mu) / 2.0L, 0.0L);
    const long double pre = std::sqrt(fact(l + m) * fact(l - m) * fact(l + mp) * fact(l - mp));
    long double out = 0.0L;
    for (int k = 0; k <= 2 * l; ++k) {
        const int a = l + m - k, b = k, cc = l - k - mp, d = k - m + mp;
        if (a < 0 || b < 0 || cc < 0 || d < 0) continue;
        const long double coef = ((k - m + mp) % 2 ? -1.0L : 1.0L) * pre / (fact(a) * fact(b) * fact(cc) * fact(d));
        // exponents 2l-2k+m-m' and 2k-m+m' are even for every pair used
        out += coef * std::pow(c2, (2 * l - 2 * k + m - mp) / 2) * std::pow(s2, (2 * k - m + mp) / 2);
    }
    return (double)out;
}

// host tables of the lensed-spectrum kernels for (L, n_mu), cached in the context
static int ensure_lens_tables(cmb_ctx *c, int L, int n_mu, hipStream_t s) {
    if (c->lens_L == L && c->lens_nmu == n_mu) return CMB_OK;
    static const int PM[13][2] = {{0, 0}, {1, 1}, {1, -1}, {2, 2}, {2, -2}, {3, 1}, {3, -3},
                                  {4, 0}, {4, -4}, {0, 2}, {3, -1}, {2, 0}, {-2, 4}};
    std::vector<double> mu, w;
    cmbhip::gauss_legendre_nodes(n_mu, mu, w);
    const size_t n_coef = (size_t)(L + 1) * 13 * 3, n_lf = (size_t)(L + 1) * 4, n_st = (size_t)13 * n_mu;
    std::vector<double> h(2 * (size_t)n_mu + n_coef + n_lf + n_st, 0.0);
    double *hmu = h.data(), *hw = hmu + n_mu, *hcoef = hw + n_mu, *hlf = hcoef + n_coef, *hst = hlf + n_lf;
    std::copy(mu.begin(), mu.end(), hmu);
    std::copy(w.begin(), w.end(), hw);
    for (int l = 0; l <= L; ++l) {
        for (int p = 0; p < 13; ++p) {
            const double mp = PM[p][0], m = PM[p][1];
            double *cf = hcoef + ((size_t)l * 13 + p) * 3;
            if (l < std::max(std::abs(PM[p][0]), std::abs(PM[p][1]))) continue;
            if (l == 0) {  // d^1_00 = mu d^0_00
                cf[0] = 1.0;
                continue;
            }
            const double cl = l * std::sqrt(((l + 1.0) * (l + 1.0) - mp * mp) * ((l + 1.0) * (l + 1.0) - m * m));
            cf[0] = (2.0 * l + 1.0) * l * (l + 1.0) / cl;
            cf[1] = (2.0 * l + 1.0) * mp * m / cl;
            cf[2] = (l + 1.0) * std::sqrt(std::max(((double)l * l - mp * mp) * ((double)l * l - m * m), 0.0)) / cl;
        }
        const double x = l;
        hlf[4 * (size_t)l + 0] = 0.25 * std::sqrt(std::max((x + 2) * (x - 1) * x * (x + 1), 0.0));
        hlf[4 * (size_t)l + 1] = -0.5 * std::sqrt(std::max((x + 2) * (x - 1), 0.0));
        hlf[4 * (size_t)l + 2] = -0.5 * std::sqrt(std::max((x + 3) * (x - 2), 0.0));
        hlf[4 * (size_t)l + 3] = 0.25 * std::sqrt(std::max((x + 4) * (x + 3) * (x - 2) * (x - 3), 0.0));
    }
    for (int p = 0; p < 13; ++p)
        for (int i = 0; i < n_mu; ++i) hst[(size_t)p * n_mu + i] = wigner_d_start(PM[p][0], PM[p][1], mu[i]);
    c->lens_L = c->lens_nmu = 0;
    int rc = grow(c, &c->lens_buf, &c->lens_cap, h.size() * sizeof(double), s);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(c->lens_buf, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // h is pageable and goes out of scope
    if (e != hipSuccess) return herr(e, "lensing tables upload");
    c->lens_L = L;
    c->lens_nmu = n_mu;
    return CMB_OK;
}

// DevTab copies (with step-history pointers) and n_extra doubles, staged
// through the context's small buffer; synchronises the stream first (the
// staging may still be read by a previous call)
static int upload_devtabs(cmb_ctx *c, const std::vector<cmbhip::DevTab> &v, const std::vector<double> &extra,
                          hipStream_t s, cmbhip::DevTab **d_tabs, double **d_extra) {
    const size_t o_x = align256(sizeof(cmbhip::DevTab) * v.size());
    const size_t bytes = o_x + align256(sizeof(double) * std::max<size_t>(extra.size(), 1));
    int rc = grow(c, &c->kt_buf, &c->kt_cap, bytes, s);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    if (bytes > c->kt_stage_cap) {
        if (c->kt_stage) hipHostFree(c->kt_stage);
        c->kt_stage = nullptr;
        c->kt_stage_cap = 0;
        e = hipHostMalloc(&c->kt_stage, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return herr(e, "hipHostMalloc");
        c->kt_stage_cap = bytes;
    }
    std::memcpy(c->kt_stage, v.data(), sizeof(cmbhip::DevTab) * v.size());
    if (!extra.empty()) std::memcpy((char *)c->kt_stage + o_x, extra.data(), sizeof(double) * extra.size());
    e = hipMemcpyAsync(c->kt_buf, c->kt_stage, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return herr(e, "hipMemcpyAsync (descriptors)");
    *d_tabs = (cmbhip::DevTab *)c->kt_buf;
    if (d_extra) *d_extra = (double *)((char *)c->kt_buf + o_x);
    return CMB_OK;
}

// trajectory checkpoints of a history launch: every ck_every accepted steps
// into (seg < 0) or, for segment seg, out of ck [n][n_k][ck_cap][1 + 2 N]
struct Ckpt {
    double *ck = nullptr;
    int every = 0, cap = 0, seg = -1;
};

// K1 over tabs with step histories: cosmology i records into (replay = false)
// or replays (replay = true) hist + base[i] n_k cap, hist_n + base[i] n_k
static int perturb_hist(cmb_ctx *c, const cmb_tables *const *tabs, int n, const std::vector<int> &base,
                        double *d_hist, int32_t *d_hist_n, int cap, bool replay, double *d_S, int32_t *d_status,
                        int32_t *d_nsteps, hipStream_t s, const Ckpt &ck = Ckpt()) {
    Batch b;
    int rc = check_batch(tabs, n, b);
    if (rc) return rc;
    if (!cmbhip::perturb2_supported(b.prec)) {
        set_error("hierarchy larger than the perturbation kernel holds (320 state rows, 16 momentum nodes)");
        return CMB_E_UNSUPPORTED;
    }
    if (cap < tabs[0]->t.prec.max_steps + 1) {
        set_error("step history capacity below max_steps + 1");
        return CMB_E_INVALID;
    }
    const size_t ck_rec = ck.ck ? (size_t)ck.cap * (1 + 2 * (size_t)cmbhip::state_rows(b.prec)) : 0;
    if (ck.ck && (ck.every < 1 || ck.cap < (cap - 1) / ck.every + 1 || ck.seg >= ck.cap || (ck.seg >= 0 && !replay) ||
                  (long long)ck.seg * ck.every >= cap)) {
        // (the last condition also keeps seg * every, the segment's first step
        // index in the kernel, inside int)
        set_error("checkpoints: need every >= 1, ck_cap >= (hist_cap - 1) / every + 1, 0 <= seg < ck_cap, "
                  "seg * every < hist_cap, and a segment only from a replay");
        return CMB_E_INVALID;
    }
    rc = upload(c, tabs, n, s);
    if (rc) return rc;
    std::vector<cmbhip::DevTab> v(c->h_tabs);
    for (int i = 0; i < n; ++i) {
        double *h = d_hist + (size_t)base[i] * b.n_k * cap;
        int *hn = d_hist_n + (size_t)base[i] * b.n_k;
        v[i].hist_cap = cap;
        if (ck.ck) {
            double *ci = ck.ck + (size_t)base[i] * b.n_k * ck_rec;
            v[i].ck_every = ck.every;
            v[i].ck_cap = ck.cap;
            if (ck.seg >= 0) {
                v[i].ck_in = ci;
                v[i].ck_seg = ck.seg;
            } else {
                v[i].ck_out = ci;
            }
        }
        if (replay) {
            v[i].hist_in = h;
            v[i].hist_in_n = hn;
        } else {
            v[i].hist_out = h;
            v[i].hist_out_n = hn;
        }
    }
    cmbhip::DevTab *dt = nullptr;
    rc = upload_devtabs(c, v, {}, s, &dt, nullptr);
    if (rc) return rc;
    int32_t *ns = d_nsteps;
    if (!ns) {
        rc = grow(c, &c->st_buf, &c->st_cap, sizeof(int32_t) * (size_t)n * b.n_k, s);
        if (rc) return rc;
        ns = (int32_t *)c->st_buf;
    }
    return cmbhip::launch_perturb2(dt, n, b.n_k, b.n_tau, b.prec, d_S, d_status, ns, nullptr, nullptr, s, true);
}

// trajectory checkpoint spacing of the reverse sweep (accepted steps per segment)
constexpr int kGradEvery = 64;

// Tables at theta_p (1 + mult[m] rel) for the four table parameters p = h,
// omega_b, omega_cdm, tau_reio, one per base cosmology and (p, m), built on
// up to 16 worker threads in parameter order, so that the device can start on
// the parameters already built.  wait(p) blocks until every table of p is
// built and returns the first failing build's code.  The destructor joins the
// workers (the tables live as long as the object).
class PerturbedTables {
  public:
    PerturbedTables(const cmb_tables *const *tabs, int nb, int n_k, int n_tau, double rel, const double *mult, int nm)
        : tabs_(tabs), nb_(nb), nm_(nm), n_k_(n_k), n_tau_(n_tau), rel_(rel), mult_(mult, mult + nm), pert_(4), brc_((size_t)4 * nm * nb, CMB_OK),
          built_(4, 0) {
        for (int p = 0; p < 4; ++p) pert_[p].resize((size_t)nm * nb);
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        try {
            for (unsigned i = 0; i < nth; ++i) th_.emplace_back([this] { work(); });
        } catch (const std::exception &) {
            // no thread could start: build every table here (started workers
            // share the jobs and are joined in the destructor)
            if (th_.empty()) work();
        }
    }
    ~PerturbedTables() {
        for (auto &x : th_) x.join();
    }
    PerturbedTables(const PerturbedTables &) = delete;
    PerturbedTables &operator=(const PerturbedTables &) = delete;

    int wait(int p) {
        std::unique_lock<std::mutex> bl(mu_);
        cv_.wait(bl, [&] { return built_[p] == nm_ * nb_; });
        for (int j = 0; j < nm_ * nb_; ++j)
            if (brc_[(size_t)p * nm_ * nb_ + j] != CMB_OK) return brc_[(size_t)p * nm_ * nb_ + j];
        return CMB_OK;
    }
    const cmb_tables *get(int p, int m, int cb) const { return pert_[p][(size_t)m * nb_ + cb].get(); }
    static double value(const cmb_cosmo &c, int p) {
        return p == 0 ? c.h : p == 1 ? c.omega_b : p == 2 ? c.omega_cdm : c.tau_reio;
    }

  private:
    void work() {
        const size_t n_jobs = (size_t)4 * nm_ * nb_;
        for (size_t q; (q = next_.fetch_add(1)) < n_jobs;) {
            const int p = (int)(q / ((size_t)nm_ * nb_)), j = (int)(q % ((size_t)nm_ * nb_)), m = j / nb_,
                      cb = j % nb_;
            const cmbhip::Tables &t0 = tabs_[cb]->t;
            cmb_cosmo cc = t0.cosmo;
            double *v = p == 0 ? &cc.h : p == 1 ? &cc.omega_b : p == 2 ? &cc.omega_cdm : &cc.tau_reio;
            *v *= 1.0 + mult_[m] * rel_;
            std::unique_ptr<cmb_tables> t(new (std::nothrow) cmb_tables);
            int r = t ? CMB_OK : CMB_E_NOMEM;
            try {
                if (r == CMB_OK) r = cmbhip::build_tables(cc, t0.prec, t0.k.data(), n_k_, n_tau_, t->t);
            } catch (const std::exception &) {
                r = CMB_E_INVALID;
            }
            if (r == CMB_OK) t->t.uid = cmbhip::g_uid.fetch_add(1);
            brc_[(size_t)p * nm_ * nb_ + j] = r;
            pert_[p][j] = std::move(t);
            std::lock_guard<std::mutex> bl(mu_);
            if (++built_[p] == nm_ * nb_) cv_.notify_all();
        }
    }
    const cmb_tables *const *tabs_;
    int nb_, nm_, n_k_, n_tau_;
    double rel_;
    std::vector<double> mult_;
    std::vector<std::vector<std::unique_ptr<cmb_tables>>> pert_;
    std::vector<int> brc_;
    std::vector<int> built_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::atomic<size_t> next_{0};
    std::vector<std::thread> th_;  // last member: joined before the others go
};

extern "C" {

int cmb_perturb_record(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, double *d_S, int32_t *d_status,
                       int32_t *d_nsteps, double *d_hist, int32_t *d_hist_n, int hist_cap, void *stream) {
    if (!c || !d_S || !d_status || !d_hist || !d_hist_n || n_cosmo < 1) {
        set_error("cmb_perturb_record: NULL argument");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    std::vector<int> base(n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) base[i] = i;
    int rc = perturb_hist(c, tabs, n_cosmo, base, d_hist, d_hist_n, hist_cap, false, d_S, d_status, d_nsteps,
                          (hipStream_t)stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_perturb_replay(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, const double *d_hist,
                       const int32_t *d_hist_n, int hist_cap, double *d_S, int32_t *d_status, int32_t *d_nsteps,
                       void *stream) {
    if (!c || !d_S || !d_status || !d_hist || !d_hist_n || n_cosmo < 1) {
        set_error("cmb_perturb_replay: NULL argument");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    std::vector<int> base(n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) base[i] = i;
    int rc = perturb_hist(c, tabs, n_cosmo, base, const_cast<double *>(d_hist), const_cast<int32_t *>(d_hist_n),
                          hist_cap, true, d_S, d_status, d_nsteps, (hipStream_t)stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_perturb_checkpoint(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int replay, double *d_hist,
                           int32_t *d_hist_n, int hist_cap, int every, double *d_ck, int ck_cap, double *d_S,
                           int32_t *d_status, int32_t *d_nsteps, void *stream) {
    if (!c || !d_S || !d_status || !d_hist || !d_hist_n || !d_ck || n_cosmo < 1) {
        set_error("cmb_perturb_checkpoint: NULL argument");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    std::vector<int> base(n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) base[i] = i;
    Ckpt ck;
    ck.ck = d_ck;
    ck.every = every;
    ck.cap = ck_cap;
    int rc = perturb_hist(c, tabs, n_cosmo, base, d_hist, d_hist_n, hist_cap, replay != 0, d_S, d_status, d_nsteps,
                          (hipStream_t)stream, ck);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_perturb_segment(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, const double *d_hist,
                        const int32_t *d_hist_n, int hist_cap, int every, const double *d_ck, int ck_cap, int seg,
                        double *d_S, int32_t *d_status, int32_t *d_nsteps, void *stream) {
    if (!c || !d_S || !d_status || !d_hist || !d_hist_n || !d_ck || n_cosmo < 1) {
        set_error("cmb_perturb_segment: NULL argument");
        return CMB_E_INVALID;
    }
    if (seg < 0) {
        set_error("cmb_perturb_segment: seg < 0");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    std::vector<int> base(n_cosmo);
    for (int i = 0; i < n_cosmo; ++i) base[i] = i;
    Ckpt ck;
    ck.ck = const_cast<double *>(d_ck);
    ck.every = every;
    ck.cap = ck_cap;
    ck.seg = seg;
    int rc = perturb_hist(c, tabs, n_cosmo, base, const_cast<double *>(d_hist), const_cast<int32_t *>(d_hist_n),
                          hist_cap, true, d_S, d_status, d_nsteps, (hipStream_t)stream, ck);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_jacobian(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, double rel, int order,
                 double *d_Cl, double *d_J, int32_t *d_status, void *stream) {
    if (!c || !tabs || !d_Cl || !d_J || !d_status || n_cosmo < 1) {
        set_error("cmb_jacobian: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000 || !(rel > 0.0 && rel <= 0.01) || (order != 2 && order != 4)) {
        set_error("cmb_jacobian: need 2 <= ell_max <= 10000, 0 < rel <= 0.01 and order 2 or 4");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    for (int i = 0; i < n_cosmo; ++i)
        if (!std::isfinite(tabs[i]->t.cosmo.tau_reio) || tabs[i]->t.k != tabs[0]->t.k) {
            set_error("cmb_jacobian: every cosmology needs tau_reio (not z_reio) and the same k grid");
            return CMB_E_INVALID;
        }
    if (b.n_tau > cmbhip::los_max_tau()) {
        set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    const int nb = n_cosmo, nm = order == 4 ? 4 : 2, n_k = b.n_k, n_tau = b.n_tau;
    const double mult[4] = {1.0, -1.0, 2.0, -2.0};
    const int slot[4] = {0, 1, 2, 5};  // h, omega_b, omega_cdm, tau_reio in (h, wb, wc, ln A_s, n_s, tau)
    // perturbed tables on host threads, built in parameter order while the
    // device records the base steps and replays the parameters already built
    // (each replay waits only for its own tables)
    PerturbedTables pt(tabs, nb, n_k, n_tau, rel, mult, nm);
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    const int cap = tabs[0]->t.prec.max_steps + 1;
    const int n3 = 3 * (ell_max + 1), nl = ell_max - 1;
    const size_t n_run = (size_t)nm * nb;  // cosmologies per replay launch
    // workspace: hist | hist_n | replay status | C of the stencil points
    const size_t o_hn = align256(sizeof(double) * (size_t)nb * n_k * cap);
    const size_t o_rs = o_hn + align256(sizeof(int32_t) * (size_t)nb * n_k);
    const size_t o_cp = o_rs + align256(sizeof(int32_t) * n_run * n_k);
    const size_t ws = o_cp + align256(sizeof(double) * n_run * n3);
    rc = grow(c, &c->ws_buf, &c->ws_cap, ws, s);
    if (rc) return rc;
    rc = grow(c, &c->s_buf, &c->s_cap, sizeof(double) * n_run * n_k * 3 * n_tau, s);
    if (rc) return rc;
    rc = grow(c, &c->d_buf, &c->d_cap, sizeof(double) * n_run * 2 * nl * n_k, s);
    if (rc) return rc;
    char *w = (char *)c->ws_buf;
    double *hist = (double *)w, *Cp = (double *)(w + o_cp);
    int32_t *hn = (int32_t *)(w + o_hn), *rst = (int32_t *)(w + o_rs);
    double *S = (double *)c->s_buf, *D = (double *)c->d_buf;
    // base: record, project, C_l; ln A_s slot = C_l, n_s slot = ln-weighted quadrature
    std::vector<int> base(n_run);
    for (size_t j = 0; j < n_run; ++j) base[j] = (int)(j % nb);
    rc = perturb_hist(c, tabs, nb, base, hist, hn, cap, false, S, d_status, nullptr, s);
    if (rc) return rc;
    rc = cmbhip::launch_los(c->d_tabs, nb, n_k, n_tau, ell_max, b.polar, b.s_pol, S, D, s);
    if (rc) return rc;
    rc = cmbhip::launch_cl(c->d_tabs, nb, n_k, ell_max, D, d_Cl, s);
    if (rc) return rc;
    rc = cmbhip::launch_cl_ex(c->d_tabs, nb, n_k, ell_max, D, d_J + 3 * n3, (long)6 * n3, 0, s);
    if (rc) return rc;
    rc = cmbhip::launch_cl_ex(c->d_tabs, nb, n_k, ell_max, D, d_J + 4 * n3, (long)6 * n3, 1, s);
    if (rc) return rc;
    // the four table parameters: replays of the base steps at the stencil points
    for (int p = 0; p < 4; ++p) {
        rc = pt.wait(p);
        if (rc) {
            set_error("cmb_jacobian: a perturbed table build failed");
            hipStreamSynchronize(s);  // launches already queued use tables freed on return
            return rc;
        }
        std::vector<const cmb_tables *> run(n_run);
        for (size_t j = 0; j < n_run; ++j) run[j] = pt.get(p, (int)(j / nb), (int)(j % nb));
        rc = perturb_hist(c, run.data(), (int)n_run, base, hist, hn, cap, true, S, rst, nullptr, s);
        if (rc) return rc;
        rc = cmbhip::launch_los(c->d_tabs, (int)n_run, n_k, n_tau, ell_max, b.polar, b.s_pol, S, D, s);
        if (rc) return rc;
        rc = cmbhip::launch_cl(c->d_tabs, (int)n_run, n_k, ell_max, D, Cp, s);
        if (rc) return rc;
        std::vector<double> e(nb);
        for (int cb = 0; cb < nb; ++cb) {
            e[cb] = rel * PerturbedTables::value(tabs[cb]->t.cosmo, p);
        }
        cmbhip::DevTab *unused = nullptr;
        double *d_e = nullptr;
        rc = upload_devtabs(c, {}, e, s, &unused, &d_e);
        if (rc) return rc;
        rc = cmbhip::launch_fd(nb, ell_max, order, Cp, d_e, d_J + (size_t)slot[p] * n3, (long)6 * n3, s);
        if (rc) return rc;
        rc = cmbhip::launch_merge_status(nb, n_k, nm, rst, d_status, s);
        if (rc) return rc;
    }
    hipError_t e = hipStreamSynchronize(s);  // the perturbed tables are freed on return
    if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    set_error("");
    return CMB_OK;
}

int cmb_gradient(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_gCl, double rel,
                 double *d_Cl, double *d_grad, int32_t *d_status, double *d_dLdy0, void *stream) {
    if (!c || !tabs || !d_gCl || !d_Cl || !d_grad || !d_status || n_cosmo < 1) {
        set_error("cmb_gradient: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000 || !(rel > 0.0 && rel <= 0.01)) {
        set_error("cmb_gradient: need 2 <= ell_max <= 10000 and 0 < rel <= 0.01");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    for (int i = 0; i < n_cosmo; ++i)
        if (!std::isfinite(tabs[i]->t.cosmo.tau_reio)) {
            set_error("cmb_gradient: every cosmology needs tau_reio (not z_reio)");
            return CMB_E_INVALID;
        }
    if (b.n_tau > cmbhip::los_max_tau()) {
        set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    if (!cmbhip::perturb2_supported(b.prec) || !cmbhip::adjoint_supported(b.prec)) {
        set_error("cmb_gradient: the reverse sweep takes massless neutrinos only and a hierarchy of at most 320 rows");
        return CMB_E_UNSUPPORTED;
    }
    const int nb = n_cosmo, n_k = b.n_k, n_tau = b.n_tau, N = cmbhip::state_rows(b.prec);
    const double mult[2] = {1.0, -1.0};
    // the tables at theta_p (1 +- rel) build on host threads while the device
    // records the base run and takes the spectrum side's reverse mode
    PerturbedTables pt(tabs, nb, n_k, n_tau, rel, mult, 2);
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    const int cap = tabs[0]->t.prec.max_steps + 1, every = kGradEvery, ck_cap = (cap - 1) / every + 1;
    const int n3 = 3 * (ell_max + 1), nl = ell_max - 1;
    const size_t nm = (size_t)nb * n_k, nS = nm * 3 * n_tau, nD = (size_t)nb * 2 * nl * n_k;
    const size_t ck_rec = (size_t)ck_cap * (1 + 2 * (size_t)N), tr_rec = (size_t)every * cmbhip::traj_rec(N);
    // workspace: hist | hist_n | checkpoints | trajectories | segment sources |
    // dL/dS | projection adjoint | n_s spectra | perturbed spectra | lambda |
    // per-mode sums | replay status | replay counts
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t o_h = take(sizeof(double) * nm * cap), o_hn = take(sizeof(int32_t) * nm),
                 o_ck = take(sizeof(double) * nm * ck_rec), o_tr = take(sizeof(double) * nm * tr_rec),
                 o_s2 = take(sizeof(double) * nS), o_gs = take(sizeof(double) * nS), o_gw = take(sizeof(double) * nD),
                 o_cn = take(sizeof(double) * (size_t)nb * n3), o_cp = take(sizeof(double) * 8 * (size_t)nb * n3),
                 o_lm = take(sizeof(double) * nm * 2 * N), o_ad = take(sizeof(double) * nm * 4),
                 o_rs = take(sizeof(int32_t) * nm), o_ns = take(sizeof(int32_t) * nm);
    rc = grow(c, &c->ws_buf, &c->ws_cap, off, s);
    if (rc) return rc;
    rc = grow(c, &c->s_buf, &c->s_cap, sizeof(double) * nS, s);
    if (rc) return rc;
    rc = grow(c, &c->d_buf, &c->d_cap, sizeof(double) * nD, s);
    if (rc) return rc;
    char *w = (char *)c->ws_buf;
    double *hist = (double *)(w + o_h), *ck = (double *)(w + o_ck), *traj = (double *)(w + o_tr);
    double *S2 = (double *)(w + o_s2), *gS = (double *)(w + o_gs), *Gw = (double *)(w + o_gw);
    double *Cns = (double *)(w + o_cn), *Cp = (double *)(w + o_cp), *lam = (double *)(w + o_lm);
    double *adj = (double *)(w + o_ad);
    int32_t *hn = (int32_t *)(w + o_hn), *rst = (int32_t *)(w + o_rs), *nsc = (int32_t *)(w + o_ns);
    double *S = (double *)c->s_buf, *D = (double *)c->d_buf;
    // (1) record the base run with trajectory checkpoints, project, C_l, the
    // n_s-weighted quadrature and dL/dS
    rc = upload(c, tabs, nb, s);
    if (rc) return rc;
    {
        std::vector<cmbhip::DevTab> v(c->h_tabs);
        for (int i = 0; i < nb; ++i) {
            v[i].hist_out = hist + (size_t)i * n_k * cap;
            v[i].hist_out_n = hn + (size_t)i * n_k;
            v[i].hist_cap = cap;
            v[i].ck_out = ck + (size_t)i * n_k * ck_rec;
            v[i].ck_every = every;
            v[i].ck_cap = ck_cap;
        }
        cmbhip::DevTab *dt = nullptr;
        rc = upload_devtabs(c, v, {}, s, &dt, nullptr);
        if (rc) return rc;
        rc = cmbhip::launch_perturb2(dt, nb, n_k, n_tau, b.prec, S, d_status, nsc, nullptr, nullptr, s, true);
        if (rc) return rc;
    }
    rc = cmbhip::launch_los(c->d_tabs, nb, n_k, n_tau, ell_max, b.polar, b.s_pol, S, D, s);
    if (rc) return rc;
    rc = cmbhip::launch_cl(c->d_tabs, nb, n_k, ell_max, D, d_Cl, s);
    if (rc) return rc;
    rc = cmbhip::launch_cl_ex(c->d_tabs, nb, n_k, ell_max, D, Cns, (long)n3, 1, s);
    if (rc) return rc;
    rc = cmbhip::launch_spectra_adjoint(c->d_tabs, nb, n_k, n_tau, ell_max, b.polar, b.s_pol, D, d_gCl, Gw, gS, s);
    if (rc) return rc;
    // (2) every table, base and perturbed, resident at once: base at 0 .. nb-1,
    // then set q = 2 p + (0: +rel, 1: -rel) at nb + q nb
    for (int p = 0; p < 4; ++p) {
        rc = pt.wait(p);
        if (rc) {
            set_error("cmb_gradient: a perturbed table build failed");
            hipStreamSynchronize(s);
            return rc;
        }
    }
    std::vector<const cmb_tables *> all((size_t)9 * nb);
    for (int i = 0; i < nb; ++i) all[i] = tabs[i];
    for (int q = 0; q < 8; ++q)
        for (int i = 0; i < nb; ++i) all[(size_t)nb + (size_t)q * nb + i] = pt.get(q >> 1, q & 1, i);
    rc = upload(c, all.data(), 9 * nb, s);
    if (rc) return rc;
    const cmbhip::DevTab *d_base = c->d_tabs, *d_pert = c->d_tabs + nb;
    // (3) the projection's own dependence on the four table parameters: the
    // base sources under each perturbed geometry
    for (int q = 0; q < 8; ++q) {
        rc = cmbhip::launch_los(d_pert + (size_t)q * nb, nb, n_k, n_tau, ell_max, b.polar, b.s_pol, S, D, s);
        if (rc) return rc;
        rc = cmbhip::launch_cl(d_pert + (size_t)q * nb, nb, n_k, ell_max, D, Cp + (size_t)q * nb * n3, s);
        if (rc) return rc;
    }
    // (4) segments: as many as the longest recorded history needs
    std::vector<int32_t> h_hn(nm);
    hipError_t e = hipMemcpyAsync(h_hn.data(), hn, sizeof(int32_t) * nm, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return herr(e, "step counts to host");
    int n_seg = 1;
    for (int32_t x : h_hn) n_seg = std::max(n_seg, (int)((std::max(x, 0) + every - 1) / every));
    std::vector<cmbhip::DevTab> v((size_t)n_seg * nb);
    for (int sg = 0; sg < n_seg; ++sg)
        for (int i = 0; i < nb; ++i) {
            cmbhip::DevTab &x = v[(size_t)sg * nb + i];
            x = c->h_tabs[i];
            x.hist_in = hist + (size_t)i * n_k * cap;
            x.hist_in_n = hn + (size_t)i * n_k;
            x.hist_cap = cap;
            x.ck_in = ck + (size_t)i * n_k * ck_rec;
            x.ck_every = every;
            x.ck_cap = ck_cap;
            x.ck_seg = sg;
            x.traj_out = traj + (size_t)i * n_k * tr_rec;
            x.traj_cap = every;
        }
    std::vector<double> den((size_t)nb * 4);
    for (int i = 0; i < nb; ++i)
        for (int p = 0; p < 4; ++p) den[(size_t)i * 4 + p] = 2.0 * rel * PerturbedTables::value(tabs[i]->t.cosmo, p);
    cmbhip::DevTab *dseg = nullptr;
    double *d_den = nullptr;
    rc = upload_devtabs(c, v, den, s, &dseg, &d_den);
    if (rc) return rc;
    // (5) the reverse sweep, last segment first: replay the segment from its
    // checkpoint writing its step trajectories, then walk them backwards
    for (int sg = n_seg - 1; sg >= 0; --sg) {
        rc = cmbhip::launch_perturb2(dseg + (size_t)sg * nb, nb, n_k, n_tau, b.prec, S2, rst, nsc, nullptr, nullptr, s,
                                     true);
        if (rc) return rc;
        rc = cmbhip::launch_merge_status(nb, n_k, 1, rst, d_status, s);
        if (rc) return rc;
        rc = cmbhip::launch_adjoint_segment(d_base, d_pert, d_den, nb, n_k, n_tau, b.prec, traj, every, hn, sg, every,
                                            gS, lam, adj, sg == n_seg - 1, s);
        if (rc) return rc;
    }
    rc = cmbhip::launch_grad_assemble(nb, n_k, ell_max, d_gCl, d_Cl, Cns, Cp, d_den, adj, d_grad, s);
    if (rc) return rc;
    if (d_dLdy0) {
        e = hipMemcpy2DAsync(d_dLdy0, sizeof(double) * N, lam, sizeof(double) * 2 * N, sizeof(double) * N, nm,
                             hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return herr(e, "dL/dy0 copy");
    }
    e = hipStreamSynchronize(s);  // the descriptors' staging and the perturbed tables go on return
    if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    set_error("");
    return CMB_OK;
}

int cmb_state_rows(const cmb_tables *tab) {
    if (!tab) {
        set_error("cmb_state_rows: NULL table");
        return -CMB_E_INVALID;
    }
    Batch b;
    const cmb_tables *one[1] = {tab};
    int rc = check_batch(one, 1, b);
    if (rc) return -rc;
    set_error("");
    return cmbhip::state_rows(b.prec);
}

int cmb_sources_adjoint(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, const double *d_gS, double *d_gY,
                        void *stream) {
    if (!c || !d_gS || !d_gY) {
        set_error("cmb_sources_adjoint: NULL argument");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    rc = cmbhip::launch_sources_adjoint(c->d_tabs, n_cosmo, b.n_k, b.n_tau, b.prec, d_gS, d_gY, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_spectra_adjoint(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Delta,
                        const double *d_gCl, double *d_gS, void *stream) {
    if (!c || !d_Delta || !d_gCl || !d_gS) {
        set_error("cmb_spectra_adjoint: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    if (b.n_tau > cmbhip::los_max_tau()) {
        set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    rc = grow(c, &c->ws_buf, &c->ws_cap, sizeof(double) * (size_t)n_cosmo * 2 * (ell_max - 1) * b.n_k, s);
    if (rc) return rc;
    rc = cmbhip::launch_spectra_adjoint(c->d_tabs, n_cosmo, b.n_k, b.n_tau, ell_max, b.polar, b.s_pol, d_Delta, d_gCl,
                                        (double *)c->ws_buf, d_gS, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_lensed_cl(cmb_ctx *c, int n_cosmo, int L, const double *d_Cl, const double *d_Clpp, int ell_max, int n_mu,
                  double *d_Cll, void *stream) {
    if (!c || !d_Cl || !d_Clpp || !d_Cll || n_cosmo < 1 || n_cosmo > 65535) {
        set_error("cmb_lensed_cl: NULL argument or n_cosmo outside [1, 65535]");
        return CMB_E_INVALID;
    }
    if (L < 2 || L > 20000 || ell_max < 2 || ell_max > L || n_mu < 2 || n_mu > 200000) {
        set_error("cmb_lensed_cl: need 2 <= ell_max <= L <= 20000 and 2 <= n_mu <= 200000");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_lens_tables(c, L, n_mu, s);
    if (rc) return rc;
    const int nblk = cmbhip::lens_back_blocks(n_mu);
    const size_t n_xi = (size_t)n_cosmo * 4 * n_mu, n_part = (size_t)n_cosmo * nblk * 4 * (ell_max + 1);
    rc = grow(c, &c->ws_buf, &c->ws_cap, sizeof(double) * (n_xi + n_part), s);
    if (rc) return rc;
    const double *mu = (const double *)c->lens_buf, *w = mu + n_mu, *coef = w + n_mu,
                 *lf = coef + (size_t)(L + 1) * 13 * 3, *st = lf + (size_t)(L + 1) * 4;
    double *xi = (double *)c->ws_buf, *part = xi + n_xi;
    rc = cmbhip::launch_lensed_cl(n_cosmo, L, ell_max, n_mu, d_Cl, d_Clpp, mu, w, coef, lf, st, xi, part, d_Cll,
                                  stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_bessel3_table(cmb_ctx *c, int ell_max, double *h_xs, double *h_x5, double *h_tab) {
    if (!c || ell_max < 1 || ell_max > 10000) {
        set_error("cmb_bessel3_table: NULL context or ell_max outside [1, 10000]");
        return CMB_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, nullptr);
    if (so.rc) return so.rc;
    hipStream_t s = nullptr;
    int rc = ensure_bessel3(c, ell_max, s);
    if (rc) return rc;
    const int L = c->b3_lmax;
    const double *xs = (const double *)c->b3_buf, *x5 = xs + L, *tab = x5 + L;
    hipError_t e = hipSuccess;
    if (h_xs) e = hipMemcpy(h_xs, xs, sizeof(double) * ell_max, hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_x5) e = hipMemcpy(h_x5, x5, sizeof(double) * ell_max, hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_tab)
        e = hipMemcpy(h_tab, tab, sizeof(double) * (size_t)ell_max * cmbhip::B3_PTS, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return herr(e, "hipMemcpy (bessel table)");
    set_error("");
    return CMB_OK;
}

int cmb_los_bessel3(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S,
                    double *d_Delta, void *stream) {
    if (!c || !d_S || !d_Delta) {
        set_error("cmb_los_bessel3: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    if (b.n_tau > cmbhip::los_max_tau()) {
        set_error("n_tau above the line-of-sight kernel's limit");
        return CMB_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = ensure_bessel3(c, ell_max, s);
    if (rc) return rc;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    const int L = c->b3_lmax;
    const double *xs = (const double *)c->b3_buf, *x5 = xs + L, *tab = x5 + L;
    rc = cmbhip::launch_los3(c->d_tabs, n_cosmo, b.n_k, b.n_tau, ell_max, b.polar, b.s_pol, d_S, xs, x5, tab, d_Delta,
                             stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_lensing_potential(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_Dm,
                          double *d_Clpp, void *stream) {
    if (!c || !d_Dm || !d_Clpp) {
        set_error("cmb_lensing_potential: NULL argument");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 20000) {
        set_error("ell_max must be in [2, 20000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    const std::vector<double> &kg = tabs[0]->t.k;
    const int nk = b.n_k;
    for (int i = 1; i < n_cosmo; ++i)
        if (tabs[i]->t.k != kg) {
            set_error("cmb_lensing_potential: the cosmologies of one call must share the perturbation k grid");
            return CMB_E_INVALID;
        }
    if (nk < 2) {
        set_error("cmb_lensing_potential: need n_k >= 2");
        return CMB_E_INVALID;
    }
    std::vector<double> lo, dinv;
    spline_factors(kg, lo, dinv);
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    const size_t o_kg = 0, o_lo = align256(sizeof(double) * nk), o_di = o_lo + align256(sizeof(double) * nk);
    const size_t small = o_di + align256(sizeof(double) * nk);
    rc = grow(c, &c->kt_buf, &c->kt_cap, small, s);
    if (rc) return rc;
    rc = grow(c, &c->ws_buf, &c->ws_cap, sizeof(double) * (size_t)n_cosmo * nk * b.n_tau, s);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);  // the staging may still be read by a previous call
    if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    if (small > c->kt_stage_cap) {
        if (c->kt_stage) hipHostFree(c->kt_stage);
        c->kt_stage = nullptr;
        c->kt_stage_cap = 0;
        e = hipHostMalloc(&c->kt_stage, small, hipHostMallocDefault);
        if (e != hipSuccess) return herr(e, "hipHostMalloc");
        c->kt_stage_cap = small;
    }
    char *h = (char *)c->kt_stage;
    char *d = (char *)c->kt_buf;
    std::memcpy(h + o_kg, kg.data(), sizeof(double) * nk);
    std::memcpy(h + o_lo, lo.data(), sizeof(double) * nk);
    std::memcpy(h + o_di, dinv.data(), sizeof(double) * nk);
    e = hipMemcpyAsync(d, h, small, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return herr(e, "hipMemcpyAsync (spline factors)");
    double *M = (double *)c->ws_buf;
    rc = cmbhip::launch_spline_m(d_Dm, M, (const double *)(d + o_kg), (const double *)(d + o_lo),
                                 (const double *)(d + o_di), n_cosmo, nk, 1, b.n_tau, stream);
    if (rc) return rc;
    rc = cmbhip::launch_limber(c->d_tabs, n_cosmo, nk, b.n_tau, ell_max, d_Dm, M, d_Clpp, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

int cmb_spectra_on_grid(cmb_ctx *c, const cmb_tables *const *tabs, int n_cosmo, int ell_max, const double *d_S,
                        const double *kt, int n_kt, double *d_St, double *d_Delta, double *d_Cl, void *stream) {
    if (!c || !d_S || !kt || !d_St || !d_Delta || !d_Cl || n_kt < 2) {
        set_error("cmb_spectra_on_grid: NULL argument or n_kt < 2");
        return CMB_E_INVALID;
    }
    if (ell_max < 2 || ell_max > 10000) {
        set_error("ell_max must be in [2, 10000]");
        return CMB_E_INVALID;
    }
    Batch b;
    int rc = check_batch(tabs, n_cosmo, b);
    if (rc) return rc;
    const std::vector<double> &kg = tabs[0]->t.k;
    const int nk = b.n_k;
    for (int i = 1; i < n_cosmo; ++i)
        if (tabs[i]->t.k != kg) {
            set_error("cmb_spectra_on_grid: the cosmologies of one call must share the perturbation k grid");
            return CMB_E_INVALID;
        }
    if (nk < 2 || b.n_tau > cmbhip::los_max_tau()) {
        set_error("cmb_spectra_on_grid: need n_k >= 2 and n_tau within the projection kernel's limit");
        return CMB_E_INVALID;
    }
    for (int q = 0; q < n_kt; ++q)
        if (!(kt[q] >= kg.front() && kt[q] <= kg.back()) || (q > 0 && !(kt[q] > kt[q - 1]))) {
            set_error("cmb_spectra_on_grid: kt must increase strictly inside the perturbation k range");
            return CMB_E_INVALID;
        }
    // spline factors of the k grid (interior rows 1..nk-2) and the interval of every kt
    std::vector<double> lo, dinv;
    spline_factors(kg, lo, dinv);
    std::vector<int> seg(n_kt);
    for (int q = 0, i = 0; q < n_kt; ++q) {
        while (i < nk - 2 && kt[q] > kg[i + 1]) ++i;
        seg[q] = i;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (!g.ok) return herr(hipErrorInvalidDevice, "hipSetDevice");
    StreamOrder so(c, stream);
    if (so.rc) return so.rc;
    hipStream_t s = (hipStream_t)stream;
    rc = upload(c, tabs, n_cosmo, s);
    if (rc) return rc;
    // small arrays: DevTab copies on kt | kg | lo | dinv | kt | seg
    const size_t o_tabs = 0;
    const size_t o_kg = align256(sizeof(cmbhip::DevTab) * n_cosmo);
    const size_t o_lo = o_kg + align256(sizeof(double) * nk);
    const size_t o_di = o_lo + align256(sizeof(double) * nk);
    const size_t o_kt = o_di + align256(sizeof(double) * nk);
    const size_t o_seg = o_kt + align256(sizeof(double) * n_kt);
    const size_t small = o_seg + align256(sizeof(int) * n_kt);
    rc = grow(c, &c->kt_buf, &c->kt_cap, small, s);
    if (rc) return rc;
    const size_t need_m = sizeof(double) * (size_t)n_cosmo * nk * 3 * b.n_tau;
    rc = grow(c, &c->ws_buf, &c->ws_cap, need_m, s);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);  // the staging may still be read by a previous call
    if (e != hipSuccess) return herr(e, "hipStreamSynchronize");
    if (small > c->kt_stage_cap) {
        if (c->kt_stage) hipHostFree(c->kt_stage);
        c->kt_stage = nullptr;
        c->kt_stage_cap = 0;
        e = hipHostMalloc(&c->kt_stage, small, hipHostMallocDefault);
        if (e != hipSuccess) return herr(e, "hipHostMalloc");
        c->kt_stage_cap = small;
    }
    char *h = (char *)c->kt_stage;
    char *d = (char *)c->kt_buf;
    cmbhip::DevTab *ht = (cmbhip::DevTab *)(h + o_tabs);
    for (int i = 0; i < n_cosmo; ++i) {
        ht[i] = c->h_tabs[i];
        ht[i].k = (const double *)(d + o_kt);
        ht[i].n_k = n_kt;
    }
    std::memcpy(h + o_kg, kg.data(), sizeof(double) * nk);
    std::memcpy(h + o_lo, lo.data(), sizeof(double) * nk);
    std::memcpy(h + o_di, dinv.data(), sizeof(double) * nk);
    std::memcpy(h + o_kt, kt, sizeof(double) * n_kt);
    std::memcpy(h + o_seg, seg.data(), sizeof(int) * n_kt);
    e = hipMemcpyAsync(d, h, small, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return herr(e, "hipMemcpyAsync (transfer grid)");
    rc = cmbhip::launch_spline_sources(d_S, (double *)c->ws_buf, (const double *)(d + o_kg),
                                       (const double *)(d + o_lo), (const double *)(d + o_di),
                                       (const int *)(d + o_seg), (const double *)(d + o_kt), d_St, n_cosmo, nk,
                                       b.n_tau, n_kt, stream);
    if (rc) return rc;
    const cmbhip::DevTab *dt = (const cmbhip::DevTab *)(d + o_tabs);
    rc = cmbhip::launch_los(dt, n_cosmo, n_kt, b.n_tau, ell_max, b.polar, b.s_pol, d_St, d_Delta, stream);
    if (rc) return rc;
    rc = cmbhip::launch_cl(dt, n_cosmo, n_kt, ell_max, d_Delta, d_Cl, stream);
    if (rc == CMB_OK) set_error("");
    return rc;
}

}  // extern "C"
