// Continuous-batching runtime for independent spectrum requests (the serving
// side of the hot path: host tables of App. A.2/B.1/B.2, then the device path
// of App. B.3-B.4 per request).
//
//   submit -> worker pool builds the host tables -> ready queue
//   scheduler thread: admits ready requests while their device footprint fits
//     the arena, packs their tables and a work list of all their (request, k)
//     modes (largest k first), launches the perturbation kernel once over the
//     list, then each request's projection and k quadrature, copies the
//     spectra back and queues a host callback -- on one of n_streams streams,
//     so a new batch starts while the previous one is still finishing its
//     longest modes;
//   host callback (runtime thread, no HIP calls) marks the batch complete;
//   the scheduler releases its arena blocks and wakes the waiters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "cmbhip_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over one device arena: offsets in 256-byte granules,
// free blocks kept by offset and merged with their neighbours on release.
class Arena {
  public:
    void reset(size_t cap) {
        free_.clear();
        cap_ = cap & ~(size_t)255;
        if (cap_) free_[0] = cap_;
        used_ = 0;
    }
    bool alloc(size_t n, size_t &off) {
        n = up256(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = up256(n ? n : 1);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    const std::map<size_t, size_t> &free_blocks() const { return free_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0;
};

struct Req {
    uint64_t id = 0;
    cmb_cosmo c{};
    cmb_prec p{};
    std::vector<double> k;
    int n_tau = 0, ell_max = 0;
    cmbhip::Tables T;
    int rc = CMB_OK;
    // device block: tables | S | Delta | Cl | status | nsteps
    size_t off = 0, bytes = 0, o_S = 0, o_D = 0, o_Cl = 0, o_st = 0, o_ns = 0;
    std::vector<double> Cl;
    std::vector<int32_t> status;
    double t_submit = 0, t_ready = 0, t_launch = 0, t_done = 0;
    int batch_size = 0;
    bool ready = false, done = false;
};

struct Slot;

struct Batch {
    cmb_server *srv = nullptr;
    Slot *slot = nullptr;
    std::vector<Req *> reqs;
    size_t off = 0, bytes = 0;  // arena block of the DevTab array and the work list
    std::atomic<bool> complete{false};
    double t_done = 0;
};

// one stream with its pinned staging buffers; holds at most one batch
struct Slot {
    hipStream_t stream = nullptr;
    char *up = nullptr, *down = nullptr;
    size_t up_cap = 0, down_cap = 0;
    std::unique_ptr<Batch> batch;
};

}  // namespace

struct cmb_server {
    int device = 0;
    int max_batch = 64;
    Clock::time_point t0;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::vector<std::thread> workers;
    std::thread sched;
    std::mutex mu;
    std::condition_variable cv_work, cv_sched, cv_done;
    std::deque<Req *> to_build, ready;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_id = 1;
    bool stop = false;        // workers: finish the build queue, then exit
    bool stop_sched = false;  // scheduler: set after the workers joined; drain, then exit
    bool have_prec = false, massive = false;
    cmb_prec prec{};
    cmbhip::DevPrec dprec{};
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

bool same_hierarchy(const cmb_prec &a, const cmb_prec &b, bool massive) {
    return a.ell_gamma == b.ell_gamma && a.ell_pol == b.ell_pol && a.ell_nu == b.ell_nu && a.max_steps == b.max_steps &&
           (!massive || (a.n_q == b.n_q && a.ell_ncdm == b.ell_ncdm)) && a.pcoeff == b.pcoeff &&
           a.icoeff == b.icoeff && a.dcoeff == b.dcoeff && a.scale_sw == b.scale_sw && a.scale_isw == b.scale_isw &&
           a.scale_dop == b.scale_dop && a.scale_pol == b.scale_pol && a.gravity_scale == b.gravity_scale &&
           a.thomson_scale == b.thomson_scale;
}

void worker_main(cmb_server *s) {
    for (;;) {
        Req *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->to_build.empty(); });
            if (s->to_build.empty()) return;
            r = s->to_build.front();
            s->to_build.pop_front();
        }
        const int rc = cmbhip::build_tables(r->c, r->p, r->k.data(), (int)r->k.size(), r->n_tau, r->T);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->t_ready = s->now();
            if (rc != CMB_OK) {
                r->rc = rc;
                r->done = true;
                r->t_done = r->t_ready;
                s->cv_done.notify_all();
            } else {
                r->ready = true;
                s->ready.push_back(r);
                s->cv_sched.notify_one();
            }
        }
    }
}

// device bytes of one request
void layout(Req &r) {
    const size_t nk = r.k.size(), nt = (size_t)r.n_tau, L = (size_t)r.ell_max;
    size_t o = up256(cmbhip::table_doubles(r.T) * sizeof(double));
    r.o_S = o;
    o += up256(nk * 3 * nt * sizeof(double));
    r.o_D = o;
    o += up256(2 * (L - 1) * nk * sizeof(double));
    r.o_Cl = o;
    o += up256(3 * (L + 1) * sizeof(double));
    r.o_st = o;
    o += up256(nk * sizeof(int32_t));
    r.o_ns = o;
    o += up256(nk * sizeof(int32_t));
    r.bytes = o;
}

void on_batch_done(void *arg) {
    Batch *b = static_cast<Batch *>(arg);
    cmb_server *s = b->srv;
    std::lock_guard<std::mutex> lk(s->mu);
    b->t_done = s->now();
    b->complete.store(true);
    s->cv_sched.notify_one();
}

int grow_pinned(char **buf, size_t *cap, size_t need) {
    if (need <= *cap) return CMB_OK;
    if (*buf) (void)hipHostFree(*buf);
    *buf = nullptr;
    *cap = 0;
    size_t n = std::max(need, (size_t)1 << 20);
    if (hipHostMalloc((void **)buf, n, hipHostMallocDefault) != hipSuccess) {
        *buf = nullptr;
        return CMB_E_NOMEM;
    }
    *cap = n;
    return CMB_OK;
}

// Pack and launch one batch on a free slot (scheduler thread, device current).
int launch_batch(cmb_server *s, Slot &slot, Batch &b) {
    const int nb = (int)b.reqs.size();
    // work list: every mode of every request, largest k first
    std::vector<cmbhip::WorkItem> items;
    for (int i = 0; i < nb; ++i)
        for (int ik = 0; ik < (int)b.reqs[i]->k.size(); ++ik) items.push_back({i, ik});
    std::stable_sort(items.begin(), items.end(), [&](const cmbhip::WorkItem &x, const cmbhip::WorkItem &y) {
        return b.reqs[x.c]->k[x.ik] > b.reqs[y.c]->k[y.ik];
    });
    const size_t head = up256(sizeof(cmbhip::DevTab) * nb) + up256(sizeof(cmbhip::WorkItem) * items.size());
    size_t up = head, down = 0;
    for (Req *r : b.reqs) {
        up += up256(cmbhip::table_doubles(r->T) * sizeof(double));
        down += up256(3 * (r->ell_max + 1) * sizeof(double)) + up256(r->k.size() * sizeof(int32_t));
    }
    if (grow_pinned(&slot.up, &slot.up_cap, up) || grow_pinned(&slot.down, &slot.down_cap, down)) {
        cmbhip::set_error("server: pinned staging allocation failed");
        return CMB_E_NOMEM;
    }
    char *dbatch = s->arena_base + b.off;
    cmbhip::DevTab *hdt = reinterpret_cast<cmbhip::DevTab *>(slot.up);
    const cmbhip::DevTab *ddt = reinterpret_cast<const cmbhip::DevTab *>(dbatch);
    std::memcpy(slot.up + up256(sizeof(cmbhip::DevTab) * nb), items.data(), sizeof(cmbhip::WorkItem) * items.size());
    const cmbhip::WorkItem *ditems =
        reinterpret_cast<const cmbhip::WorkItem *>(dbatch + up256(sizeof(cmbhip::DevTab) * nb));
    size_t uo = head;
    std::vector<size_t> up_off(nb);
    for (int i = 0; i < nb; ++i) {
        Req *r = b.reqs[i];
        char *dr = s->arena_base + r->off;
        up_off[i] = uo;
        cmbhip::pack_table(r->T, reinterpret_cast<double *>(slot.up + uo), reinterpret_cast<const double *>(dr),
                           hdt[i]);
        hdt[i].S = reinterpret_cast<double *>(dr + r->o_S);
        hdt[i].status = reinterpret_cast<int *>(dr + r->o_st);
        hdt[i].nsteps = reinterpret_cast<int *>(dr + r->o_ns);
        uo += up256(cmbhip::table_doubles(r->T) * sizeof(double));
    }
    hipStream_t st = slot.stream;
    auto check = [&](hipError_t e, const char *what) {
        if (e != hipSuccess) {
            cmbhip::set_error(std::string("server: ") + what + ": " + hipGetErrorString(e));
            return CMB_E_DEVICE;
        }
        return CMB_OK;
    };
    int rc = check(hipMemcpyAsync(dbatch, slot.up, head, hipMemcpyHostToDevice, st), "upload work list");
    for (int i = 0; i < nb && rc == CMB_OK; ++i)
        rc = check(hipMemcpyAsync(s->arena_base + b.reqs[i]->off, slot.up + up_off[i],
                                  cmbhip::table_doubles(b.reqs[i]->T) * sizeof(double), hipMemcpyHostToDevice, st),
                   "upload tables");
    if (rc) return rc;
    rc = cmbhip::launch_perturb2_items(ddt, ditems, (int)items.size(), s->dprec, st);
    if (rc) return rc;
    const int polar = s->prec.ell_pol > 0;
    size_t dof = 0;
    for (int i = 0; i < nb && rc == CMB_OK; ++i) {
        Req *r = b.reqs[i];
        char *dr = s->arena_base + r->off;
        const int nk = (int)r->k.size();
        rc = cmbhip::launch_los(ddt + i, 1, nk, r->n_tau, r->ell_max, polar, s->prec.scale_pol,
                                reinterpret_cast<const double *>(dr + r->o_S), reinterpret_cast<double *>(dr + r->o_D),
                                st);
        if (rc) break;
        rc = cmbhip::launch_cl(ddt + i, 1, nk, r->ell_max, reinterpret_cast<const double *>(dr + r->o_D),
                               reinterpret_cast<double *>(dr + r->o_Cl), st);
        if (rc) break;
        const size_t ncl = 3 * (r->ell_max + 1) * sizeof(double);
        rc = check(hipMemcpyAsync(slot.down + dof, dr + r->o_Cl, ncl, hipMemcpyDeviceToHost, st), "copy spectra");
        dof += up256(ncl);
        if (rc) break;
        rc = check(hipMemcpyAsync(slot.down + dof, dr + r->o_st, nk * sizeof(int32_t), hipMemcpyDeviceToHost, st),
                   "copy status");
        dof += up256(nk * sizeof(int32_t));
    }
    if (rc) return rc;
    return check(hipLaunchHostFunc(st, on_batch_done, &b), "host callback");
}

// Collect a finished batch (scheduler thread, lock held).
void retire(cmb_server *s, Slot &slot) {
    Batch &b = *slot.batch;
    size_t dof = 0;
    for (Req *r : b.reqs) {
        const size_t ncl = 3 * (r->ell_max + 1);
        r->Cl.assign(reinterpret_cast<double *>(slot.down + dof), reinterpret_cast<double *>(slot.down + dof) + ncl);
        dof += up256(ncl * sizeof(double));
        const int32_t *hs = reinterpret_cast<int32_t *>(slot.down + dof);
        r->status.assign(hs, hs + r->k.size());
        dof += up256(r->k.size() * sizeof(int32_t));
        r->t_done = b.t_done;
        r->done = true;
        s->arena.release(r->off, r->bytes);
    }
    s->arena.release(b.off, b.bytes);
    slot.batch.reset();
    s->cv_done.notify_all();
}

void fail_batch(cmb_server *s, Slot &slot, int rc) {
    Batch &b = *slot.batch;
    for (Req *r : b.reqs) {
        r->rc = rc;
        r->done = true;
        r->t_done = s->now();
        s->arena.release(r->off, r->bytes);
    }
    s->arena.release(b.off, b.bytes);
    slot.batch.reset();
    s->cv_done.notify_all();
}

void sched_main(cmb_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto free_slot = [&]() -> Slot * {
            for (auto &sl : s->slots)
                if (!sl.batch) return &sl;
            return nullptr;
        };
        auto completed = [&]() {
            for (auto &sl : s->slots)
                if (sl.batch && sl.batch->complete.load()) return true;
            return false;
        };
        auto busy = [&]() {
            for (auto &sl : s->slots)
                if (sl.batch) return true;
            return false;
        };
        s->cv_sched.wait(lk, [&] {
            return completed() || (!s->ready.empty() && free_slot()) || (s->stop_sched && !busy());
        });
        for (auto &sl : s->slots)
            if (sl.batch && sl.batch->complete.load()) {
                // the callback ran after the stream's copies; its last HIP
                // error (if any) belongs to this stream
                hipError_t e = hipStreamQuery(sl.stream);
                if (e != hipSuccess && e != hipErrorNotReady) {
                    cmbhip::set_error(std::string("server: stream error: ") + hipGetErrorString(e));
                    fail_batch(s, sl, CMB_E_DEVICE);
                } else {
                    retire(s, sl);
                }
            }
        if (s->stop_sched && !busy() && s->ready.empty()) return;
        Slot *sl = free_slot();
        if (!sl || s->ready.empty()) continue;
        // admit requests (in arrival order) while they fit
        auto b = std::make_unique<Batch>();
        b->srv = s;
        b->slot = sl;
        while (!s->ready.empty() && (int)b->reqs.size() < s->max_batch) {
            Req *r = s->ready.front();
            layout(*r);
            if (!s->arena.alloc(r->bytes, r->off)) break;
            b->reqs.push_back(r);
            s->ready.pop_front();
        }
        if (b->reqs.empty()) {
            if (!busy()) {  // cannot fit even on an idle device
                Req *r = s->ready.front();
                s->ready.pop_front();
                r->rc = CMB_E_NOMEM;
                r->done = true;
                r->t_done = s->now();
                s->cv_done.notify_all();
            }
            continue;  // wait for a batch to retire
        }
        size_t nitems = 0;
        for (Req *r : b->reqs) nitems += r->k.size();
        b->bytes = up256(sizeof(cmbhip::DevTab) * b->reqs.size()) + up256(sizeof(cmbhip::WorkItem) * nitems);
        if (!s->arena.alloc(b->bytes, b->off)) {
            for (Req *r : b->reqs) {
                s->arena.release(r->off, r->bytes);
                s->ready.push_front(r);
            }
            std::reverse(s->ready.begin(), s->ready.begin() + b->reqs.size());
            if (!busy()) {
                Req *r = s->ready.front();
                s->ready.pop_front();
                r->rc = CMB_E_NOMEM;
                r->done = true;
                r->t_done = s->now();
                s->cv_done.notify_all();
            }
            continue;
        }
        const double tl = s->now();
        for (Req *r : b->reqs) {
            r->t_launch = tl;
            r->batch_size = (int)b->reqs.size();
        }
        sl->batch = std::move(b);
        lk.unlock();
        const int rc = launch_batch(s, *sl, *sl->batch);
        lk.lock();
        if (rc != CMB_OK) {
            (void)hipStreamSynchronize(sl->stream);
            fail_batch(s, *sl, rc);
        }
    }
}

}  // namespace

extern "C" {

int cmb_server_create(int device, const cmb_server_opts *opts, cmb_server **out) {
    if (!out) {
        cmbhip::set_error("cmb_server_create: NULL out");
        return CMB_E_INVALID;
    }
    *out = nullptr;
    cmb_server_opts o{};
    if (opts) o = *opts;
    const int nw = o.n_workers > 0 ? o.n_workers : 4;
    const int ns = o.n_streams > 0 ? o.n_streams : 2;
    const int mb = o.max_batch > 0 ? o.max_batch : 64;
    const size_t budget = o.hbm_budget_bytes ? o.hbm_budget_bytes : ((size_t)8 << 30);
    if (nw > 64 || ns > 4 || budget < ((size_t)64 << 20)) {
        cmbhip::set_error("cmb_server_create: n_workers <= 64, n_streams <= 4, budget >= 64 MiB");
        return CMB_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        cmbhip::set_error("cmb_server_create: no such HIP device");
        return CMB_E_DEVICE;
    }
    auto s = std::make_unique<cmb_server>();
    s->device = device;
    s->max_batch = mb;
    s->t0 = Clock::now();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    if (hipMalloc((void **)&s->arena_base, budget) != hipSuccess) {
        (void)hipSetDevice(prev);
        cmbhip::set_error("cmb_server_create: arena allocation failed");
        return CMB_E_NOMEM;
    }
    s->arena.reset(budget);
    s->slots.resize(ns);
    for (auto &sl : s->slots)
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            for (auto &x : s->slots)
                if (x.stream) (void)hipStreamDestroy(x.stream);
            (void)hipFree(s->arena_base);
            (void)hipSetDevice(prev);
            cmbhip::set_error("cmb_server_create: stream creation failed");
            return CMB_E_DEVICE;
        }
    (void)hipSetDevice(prev);
    cmb_server *raw = s.release();
    try {
        for (int i = 0; i < nw; ++i) raw->workers.emplace_back(worker_main, raw);
        raw->sched = std::thread(sched_main, raw);
    } catch (const std::exception &) {
        cmb_server_destroy(raw);  // stops and joins whatever started, frees the device resources
        cmbhip::set_error("cmb_server_create: thread creation failed");
        return CMB_E_NOMEM;
    }
    *out = raw;
    cmbhip::set_error("");
    return CMB_OK;
}

int cmb_server_submit(cmb_server *s, const cmb_cosmo *c, const cmb_prec *p, const double *k, int n_k, int n_tau,
                      int ell_max, uint64_t *ticket) {
    if (!s || !c || !p || !k || !ticket || n_k < 1 || n_tau < 3 || n_tau > cmbhip::los_max_tau() || ell_max < 2 ||
        ell_max > 10000) {
        cmbhip::set_error("cmb_server_submit: NULL argument or size out of range");
        return CMB_E_INVALID;
    }
    auto r = std::make_unique<Req>();
    r->c = *c;
    r->p = *p;
    r->k.assign(k, k + n_k);
    r->n_tau = n_tau;
    r->ell_max = ell_max;
    const bool massive = c->N_nu_massive > 0;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->have_prec) {
        s->prec = *p;
        s->massive = massive;
        s->dprec = cmbhip::dev_prec(*p, massive ? p->n_q : 0);
        if (!cmbhip::perturb2_supported(s->dprec)) {
            cmbhip::set_error("cmb_server_submit: hierarchy too large for the perturbation kernel");
            return CMB_E_UNSUPPORTED;
        }
        s->have_prec = true;
    } else if (massive != s->massive || !same_hierarchy(*p, s->prec, massive)) {
        cmbhip::set_error("cmb_server_submit: hierarchy options differ from the server's first request");
        return CMB_E_INVALID;
    }
    r->id = s->next_id++;
    r->t_submit = s->now();
    *ticket = r->id;
    s->to_build.push_back(r.get());
    s->reqs[r->id] = std::move(r);
    s->cv_work.notify_one();
    cmbhip::set_error("");
    return CMB_OK;
}

int cmb_server_wait(cmb_server *s, uint64_t ticket, double timeout_s, double *Cl, int32_t *status,
                    cmb_request_times *times) {
    if (!s || !Cl) {
        cmbhip::set_error("cmb_server_wait: NULL argument");
        return CMB_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        cmbhip::set_error("cmb_server_wait: unknown ticket");
        return CMB_E_INVALID;
    }
    Req *r = it->second.get();
    auto pred = [&] { return r->done; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return -1;
    const int rc = r->rc;
    if (rc == CMB_OK) {
        std::memcpy(Cl, r->Cl.data(), r->Cl.size() * sizeof(double));
        if (status) std::memcpy(status, r->status.data(), r->status.size() * sizeof(int32_t));
    }
    if (times) {
        times->submit = r->t_submit;
        times->tables_ready = r->t_ready;
        times->launched = r->t_launch;
        times->done = r->t_done;
        times->batch_size = r->batch_size;
    }
    s->reqs.erase(it);
    return rc;
}

void cmb_server_destroy(cmb_server *s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    for (auto &w : s->workers) w.join();  // every submitted request is now built or failed
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->stop_sched = true;
        s->cv_sched.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto &sl : s->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.up) (void)hipHostFree(sl.up);
        if (sl.down) (void)hipHostFree(sl.down);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    (void)hipSetDevice(prev);
    delete s;
}

int cmb_server_selftest_arena(unsigned seed, int n_ops) {
    Arena a;
    const size_t cap = (size_t)1 << 24;
    a.reset(cap);
    std::mt19937_64 rng(seed);
    std::vector<std::pair<size_t, size_t>> live;  // (offset, rounded size)
    for (int op = 0; op < n_ops; ++op) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t n = 1 + rng() % (cap / 16);
            size_t off;
            if (a.alloc(n, off)) {
                const size_t m = up256(n);
                if (off % 256 || off + m > cap) return 1;
                for (auto &l : live)
                    if (off < l.first + l.second && l.first < off + m) return 2;  // overlap
                live.push_back({off, m});
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].first, live[i].second);
            live.erase(live.begin() + i);
        }
        size_t u = 0;
        for (auto &l : live) u += l.second;
        if (u != a.used()) return 3;
        size_t f = 0;
        for (auto &b : a.free_blocks()) f += b.second;
        if (f + u != cap) return 4;
    }
    for (auto &l : live) a.release(l.first, l.second);
    if (a.used() != 0 || a.free_blocks().size() != 1 || a.free_blocks().begin()->second != cap) return 5;
    return 0;
}

}  // extern "C"
