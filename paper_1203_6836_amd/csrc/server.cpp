// Continuous-batching server of SP2 solves.
//
// Requests (H on the host, any size) are queued by sp2_server_submit.  A
// scheduler thread admits them into device "slots" whenever a slot is free
// and the request's footprint fits in the device arena (one allocation of
// hbm_budget_bytes made at creation, carved by a first-fit allocator), runs
// H is uploaded on a copy stream; once it has landed, the per-system start
// kernels (H check, bounds, X_0, first branch) run on the compute stream and
// the system joins the group, which advances every started system by
// iters_per_tick SP2 products per tick with grouped launches (encode,
// product, control) that cover all tiles of all systems in the group.  The
// launches are captured once in a hipGraph and replayed every tick; only the
// device-side work description changes between ticks.  After each tick the
// control states are read back; finished systems leave the group (D and the
// charges are formed on the compute stream and copied to the request's
// pinned host buffers on the copy stream), and waiting requests are admitted
// in their place, so new work joins systems that are mid-solve and no tick
// waits for a host transfer.  A completion thread waits for each download
// and then frees the request's arena block and wakes its waiter.  Each request's result depends only on its own H
// (tiling, reductions and branch decisions are per system), so it is the same
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sp2qmd.h"
#include "sp2_internal.h"
#include "split_internal.h"

using namespace sp2;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over one device allocation (offsets, 256-byte aligned).
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(char* b, size_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t* off) {
        n = align_up(n, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n, 256);
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
};

// Device footprint of one request and its layout inside its arena block.
struct Layout {
    size_t H, X, digits, scale, part, chk, D, q, total;
};
Layout layout_for(int N, int slices) {
    const size_t ld = align_up((size_t)N, kTile);
    const size_t nt = ld / kTile;
    Layout L;
    size_t o = 0;
    L.H = o;      o = align_up(o + (size_t)N * N * 8, 256);
    L.X = o;      o = align_up(o + 2 * ld * ld * 8, 256);
    L.digits = o; o = align_up(o + (size_t)slices * ld * ld, 256);
    L.scale = o;  o = align_up(o + ld * 8, 256);
    L.part = o;   o = align_up(o + std::max<size_t>(nt * (nt + 1) / 2, ld / 4) * 3 * 8, 256);
    L.chk = o;    o = align_up(o + 2 * (size_t)kCheckGrid * 8, 256);
    L.D = o;      o = align_up(o + (size_t)N * N * 8, 256);
    L.q = o;      o = align_up(o + (size_t)(N / 4 + 1) * 8, 256);
    L.total = o;
    return L;
}

// Pinned host buffers recycled across requests (size classes of 1 MiB), so a
// steady stream of submits does not pay a pinned allocation each time.
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void*> free_;
    static size_t cls(size_t n) { return align_up(std::max<size_t>(n, 1), (size_t)1 << 20); }
    void* get(size_t n) {
        const size_t c = cls(n);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free_.find(c);
            if (it != free_.end()) {
                void* p = it->second;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p, size_t n) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        free_.emplace(cls(n), p);
    }
    void clear() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : free_) (void)hipHostFree(kv.second);
        free_.clear();
    }
};

struct Request {
    uint64_t ticket = 0;
    int N = 0, n_occ = 0;
    double* H = nullptr;   // pinned host
    double* D = nullptr;   // pinned host (result)
    double* q = nullptr;   // pinned host (result)
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = 0;        // sp2_status of the solve
    bool done = false;
    size_t off = 0;        // arena block
    Layout L{};
    int slot = -1;
    bool started = false;  // start kernels issued: part of the group
    hipEvent_t ev_up = nullptr;    // H landed on the device / D formed (compute stream)
    hipEvent_t ev_down = nullptr;  // D and q landed in host memory
    sp2_stats stats{};
};

}  // namespace

struct sp2_server {
    sp2_ctx* ctx = nullptr;
    int device = 0;
    sp2_server_options opt{};
    hipStream_t stream = nullptr;       // kernels
    hipStream_t copy = nullptr;         // host <-> device transfers of requests
    char* arena_mem = nullptr;
    Arena arena;
    GroupDesc* g_dev = nullptr;
    GroupDesc* g_host = nullptr;   // pinned
    State* st_dev = nullptr;       // kMaxGroup control states
    State* st_host = nullptr;      // pinned
    hipGraphExec_t graph = nullptr;
    hipEvent_t ev_tick = nullptr;       // end of a tick's state read-back
    PinnedPool pinned;
    std::vector<Request*> slots;
    std::vector<Request*> uploading;    // admitted, H in flight (worker thread only)
    std::thread worker, completer;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_down;
    std::deque<Request*> queue;
    std::deque<Request*> downloading;   // results in flight, in order of issue (under mu)
    bool worker_done = false;
    std::map<uint64_t, Request*> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string err;
    // statistics
    std::vector<double> lat_ms;
    double first_submit = -1, last_done = -1;
    long completed = 0, ticks = 0;
    double busy_s = 0;

    void loop();
    void complete_loop();
    bool admit_locked(std::vector<Request*>& fresh);
    sp2_status begin_upload(Request* r);
    sp2_status start_system(Request* r);
    sp2_status retire(std::vector<Request*>& finished);
    void finish_locked(Request* r, double t);
    void build_group();
};

static bool fits_int8(int N) { return N >= 2 && N <= 65536; }

void sp2_server::build_group() {
    GroupDesc& g = *g_host;
    int n = 0, toff = 0, roff = 0;
    for (int s = 0; s < (int)slots.size(); ++s) {
        Request* r = slots[s];
        if (!r || !r->started) continue;
        const int ld = (int)align_up((size_t)r->N, kTile);
        const int nt = ld / kTile;
        char* b = arena.base + r->off;
        SysView& v = g.sys[n];
        v.buf0 = reinterpret_cast<double*>(b + r->L.X);
        v.buf1 = v.buf0 + (size_t)ld * ld;
        v.digits = reinterpret_cast<int8_t*>(b + r->L.digits);
        v.scale = reinterpret_cast<double*>(b + r->L.scale);
        v.part = reinterpret_cast<double*>(b + r->L.part);
        v.st = st_dev + s;
        v.ld = ld;
        v.ctrl.n_occ = (double)r->n_occ;
        v.ctrl.idem_tol = opt.idem_tol;
        v.ctrl.stall_tol = 1e-2;
        v.ctrl.stall_ratio = 0.5;   // int8 products: the floor rule of direct int8 solves
        v.ctrl.max_iter = opt.max_iter;
        v.ctrl.fp64_head = 0;
        v.ctrl.fp32_tail = 0;
        v.ctrl.mixed = 1;
        v.ctrl.total_blocks = 0.0;
        g.tile_off[n] = toff;
        g.row_off[n] = roff;
        toff += nt * (nt + 1) / 2;
        roff += ld / 4;
        ++n;
    }
    g.tile_off[n] = toff;
    g.row_off[n] = roff;
    g.nsys = n;
    g.total_tiles = toff;
    g.total_rowq = roff;
}

bool sp2_server::admit_locked(std::vector<Request*>& fresh) {
    bool any = false;
    while (!queue.empty()) {
        int free_slot = -1;
        for (int s = 0; s < (int)slots.size(); ++s)
            if (!slots[s]) { free_slot = s; break; }
        if (free_slot < 0) break;
        Request* r = queue.front();
        size_t off = 0;
        if (!arena.alloc(r->L.total, &off)) break;   // wait for memory to free up (FIFO)
        queue.pop_front();
        r->off = off;
        r->slot = free_slot;
        r->t_admit = now_s();
        slots[free_slot] = r;
        fresh.push_back(r);
        any = true;
    }
    return any;
}

// Copy H to the request's arena block on the copy stream; ev_up marks its
// arrival.
sp2_status sp2_server::begin_upload(Request* r) {
    const unsigned flags = hipEventDisableTiming | hipEventBlockingSync;
    if (hipEventCreateWithFlags(&r->ev_up, flags) != hipSuccess ||
        hipEventCreateWithFlags(&r->ev_down, flags) != hipSuccess)
        return SP2_EDEVICE;
    double* H = reinterpret_cast<double*>(arena.base + r->off + r->L.H);
    if (hipMemcpyAsync(H, r->H, (size_t)r->N * r->N * 8, hipMemcpyHostToDevice, copy) != hipSuccess ||
        hipEventRecord(r->ev_up, copy) != hipSuccess)
        return SP2_EDEVICE;
    return SP2_OK;
}

// Per-system start kernels (H check, bounds, X_0, first branch) on the
// compute stream, once H has landed.
sp2_status sp2_server::start_system(Request* r) {
    const int N = r->N;
    const int ld = (int)align_up((size_t)N, kTile);
    char* b = arena.base + r->off;
    double* H = reinterpret_cast<double*>(b + r->L.H);
    double* X0 = reinterpret_cast<double*>(b + r->L.X);
    double* part = reinterpret_cast<double*>(b + r->L.part);
    State* st = st_dev + r->slot;
    CtrlArgs a{};
    a.n_occ = (double)r->n_occ;
    a.idem_tol = opt.idem_tol;
    a.stall_tol = 1e-2;
    a.stall_ratio = 0.5;
    a.max_iter = opt.max_iter;
    a.fp64_head = 0;
    a.mixed = 1;
    double* chk = reinterpret_cast<double*>(b + r->L.chk);
    int ns = 0, nchk = 0;
    if (launch_check_h(H, N, chk, &nchk, stream) != hipSuccess) return SP2_EDEVICE;
    if (launch_gershgorin(H, N, part, &ns, stream) != hipSuccess) return SP2_EDEVICE;
    if (launch_bounds(part, ns, chk, nchk, st, stream) != hipSuccess) return SP2_EDEVICE;
    if (launch_init(H, N, ld, X0, st, part, &ns, stream) != hipSuccess) return SP2_EDEVICE;
    if (launch_ctrl_init(part, ns, st, a, stream) != hipSuccess) return SP2_EDEVICE;
    return SP2_OK;
}

// Finished systems leave the group: statistics from the control state; for a
// solved system D and the charges are formed on the compute stream and
// copied out on the copy stream after it (ev_up, then ev_down), and the
// completion thread finishes the request; a failed one finishes at once.
sp2_status sp2_server::retire(std::vector<Request*>& finished) {
    sp2_status rc = SP2_OK;
    std::vector<Request*> failed;
    for (Request* r : finished) {
        const int N = r->N;
        const int ld = (int)align_up((size_t)N, kTile);
        char* b = arena.base + r->off;
        double* X0 = reinterpret_cast<double*>(b + r->L.X);
        double* D = reinterpret_cast<double*>(b + r->L.D);
        double* q = reinterpret_cast<double*>(b + r->L.q);
        const State& h = st_host[r->slot];
        sp2_stats& st = r->stats;
        std::memset(&st, 0, sizeof(st));
        st.iterations = h.iter;
        st.status = h.done - 1;   // 0 converged, 1 stalled, 2 max_iter, 3 gap, 4 invalid H
        st.fp64_products = h.fp64_products;
        st.head_switch = h.head_switch;
        st.eps_min = h.eps_min;
        st.eps_max = h.eps_max;
        st.idem_err = h.iter > 0 ? h.idem[h.iter - 1] : 0.0;
        st.trace = h.t1;
        st.branch_bits[0] = h.bits[0];
        st.branch_bits[1] = h.bits[1];
        for (int k = 0; k < kMaxIter && k < 128; ++k) st.idem_hist[k] = (float)h.idem[k];
        if (r->status == SP2_OK)
            r->status = h.done == 3 ? SP2_ENOCONV : (h.done == 4 ? SP2_EGAP : (h.done == 5 ? SP2_EINVAL : SP2_OK));
        bool issued = false;
        if (r->status == SP2_OK && (h.done == 1 || h.done == 2)) {
            issued = launch_finalize(X0, X0 + (size_t)ld * ld, ld, N, D, st_dev + r->slot, stream) == hipSuccess &&
                     (N % 4 != 0 || launch_mulliken(D, N / 4, 4.0, q, stream) == hipSuccess) &&
                     hipEventRecord(r->ev_up, stream) == hipSuccess &&
                     hipStreamWaitEvent(copy, r->ev_up, 0) == hipSuccess &&
                     hipMemcpyAsync(r->D, D, (size_t)N * N * 8, hipMemcpyDeviceToHost, copy) == hipSuccess &&
                     (N % 4 != 0 ||
                      hipMemcpyAsync(r->q, q, (size_t)(N / 4) * 8, hipMemcpyDeviceToHost, copy) == hipSuccess) &&
                     hipEventRecord(r->ev_down, copy) == hipSuccess;
            if (!issued) {
                r->status = SP2_EDEVICE;
                rc = SP2_EDEVICE;
            }
        }
        if (!issued) failed.push_back(r);
    }
    const double t = now_s();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Request* r : finished) {
            slots[r->slot] = nullptr;
            r->slot = -1;
        }
        for (Request* r : finished)
            if (std::find(failed.begin(), failed.end(), r) == failed.end()) downloading.push_back(r);
        for (Request* r : failed) finish_locked(r, t);
    }
    cv_down.notify_all();
    cv_done.notify_all();
    return rc;
}

// Under mu: the request's arena block is free again and its waiter may go.
void sp2_server::finish_locked(Request* r, double t) {
    arena.release(r->off, r->L.total);
    r->t_done = t;
    r->stats.ms = (t - r->t_submit) * 1e3;
    r->done = true;
    lat_ms.push_back((t - r->t_submit) * 1e3);
    last_done = t;
    ++completed;
}

// Completion thread: waits for the downloads in the order they were issued.
void sp2_server::complete_loop() {
    (void)hipSetDevice(device);
    for (;;) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_down.wait(lk, [this] { return !downloading.empty() || worker_done; });
            if (downloading.empty()) return;   // the worker has stopped and nothing is in flight
            r = downloading.front();
        }
        const bool ok = hipEventSynchronize(r->ev_down) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(mu);
            downloading.pop_front();
            if (!ok) r->status = SP2_EDEVICE;
            finish_locked(r, now_s());
        }
        cv_done.notify_all();
        cv_work.notify_all();   // freed arena space may admit a queued request
    }
}

void sp2_server::loop() {
    (void)hipSetDevice(device);
    bool group_dirty = true;
    for (;;) {
        std::vector<Request*> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                admit_locked(fresh);
                bool busy = !fresh.empty() || !uploading.empty();
                for (Request* r : slots) busy = busy || r != nullptr;
                if (busy) break;
                if (stop) {
                    worker_done = true;
                    lk.unlock();
                    cv_down.notify_all();
                    return;
                }
                cv_work.wait_for(lk, std::chrono::milliseconds(50));
            }
        }
        const double t0 = now_s();
        sp2_status rc = SP2_OK;
        for (Request* r : fresh) {
            uploading.push_back(r);
            if (rc == SP2_OK) rc = begin_upload(r);
        }
        // systems whose H has landed start and join the group
        for (auto it = uploading.begin(); rc == SP2_OK && it != uploading.end();) {
            const hipError_t e = hipEventQuery((*it)->ev_up);
            if (e == hipErrorNotReady) {
                ++it;
                continue;
            }
            if (e != hipSuccess || (rc = start_system(*it)) != SP2_OK) {
                rc = rc == SP2_OK ? SP2_EDEVICE : rc;
                break;
            }
            (*it)->started = true;
            group_dirty = true;
            it = uploading.erase(it);
        }
        bool any_started = false;
        for (Request* r : slots) any_started = any_started || (r && r->started);
        std::vector<Request*> finished;
        if (rc == SP2_OK && any_started) {
            if (group_dirty) {
                build_group();
                if (hipMemcpyAsync(g_dev, g_host, sizeof(GroupDesc), hipMemcpyHostToDevice, stream) != hipSuccess)
                    rc = SP2_EDEVICE;
                group_dirty = false;
            }
            if (rc == SP2_OK && hipGraphLaunch(graph, stream) != hipSuccess) rc = SP2_EDEVICE;
            if (rc == SP2_OK &&
                hipMemcpyAsync(st_host, st_dev, sizeof(State) * slots.size(), hipMemcpyDeviceToHost, stream) !=
                    hipSuccess)
                rc = SP2_EDEVICE;
            // the worker waits for the tick by polling (a blocking wait wakes up
            // late and leaves the GPU idle until the next tick is launched)
            if (rc == SP2_OK && hipEventRecord(ev_tick, stream) != hipSuccess) rc = SP2_EDEVICE;
            while (rc == SP2_OK) {
                const hipError_t e = hipEventQuery(ev_tick);
                if (e == hipSuccess) break;
                if (e != hipErrorNotReady) rc = SP2_EDEVICE;
            }
            ++ticks;
        } else if (rc == SP2_OK) {
            // only uploads in flight: wait for the oldest
            if (!uploading.empty() && hipEventSynchronize(uploading.front()->ev_up) != hipSuccess) rc = SP2_EDEVICE;
        }
        for (Request* r : slots)
            if (r && r->started && (rc != SP2_OK || st_host[r->slot].done)) finished.push_back(r);
        if (rc != SP2_OK) {
            // a device error ends every request the worker holds
            for (Request* r : slots)
                if (r && !r->started) finished.push_back(r);
            uploading.clear();
            (void)hipStreamSynchronize(copy);   // no transfer may still target a block about to be freed
            std::lock_guard<std::mutex> lk(mu);
            err = "device error in the serving loop";
            for (Request* r : finished) r->status = rc;
        }
        if (!finished.empty()) {
            if (retire(finished) != SP2_OK) {
                std::lock_guard<std::mutex> lk(mu);
                err = "device error while retiring requests";
            }
            group_dirty = true;
        }
        busy_s += now_s() - t0;
    }
}

extern "C" {

void sp2_server_options_default(sp2_server_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget_bytes = (uint64_t)8 << 30;
    o->max_slots = 32;
    o->slices = 5;
    o->max_iter = 100;
    o->idem_tol = 1e-10;
    o->iters_per_tick = 8;
}

sp2_status sp2_server_create(sp2_ctx* ctx, const sp2_server_options* opt, sp2_server** out) {
    if (!ctx || !out) return SP2_EINVAL;
    *out = nullptr;
    sp2_server_options o;
    if (opt) o = *opt;
    else sp2_server_options_default(&o);
    if (o.levels == 0) o.levels = o.slices;
    if (!(o.levels == o.slices || (o.levels == o.slices + 1 && o.slices <= 5))) return SP2_EINVAL;
    if (o.max_slots < 1 || o.max_slots > kMaxGroup || o.slices < 2 || o.slices > kMaxSlices ||
        o.hbm_budget_bytes < ((uint64_t)1 << 20) || o.max_iter < 1 || o.max_iter > kMaxIter ||
        !(o.idem_tol > 0) || o.iters_per_tick < 1 || o.iters_per_tick > 16)
        return SP2_EINVAL;
    const int dev = sp2_ctx_device_of(ctx);
    if (hipSetDevice(dev) != hipSuccess) return SP2_EDEVICE;
    sp2_server* s = new sp2_server();
    s->ctx = ctx;
    s->device = dev;
    s->opt = o;
    s->slots.assign(o.max_slots, nullptr);
    bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->ev_tick, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->arena_mem, o.hbm_budget_bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->g_dev, sizeof(GroupDesc)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->g_host, sizeof(GroupDesc), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->st_dev, sizeof(State) * kMaxGroup) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->st_host, sizeof(State) * kMaxGroup, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        sp2_server_destroy(s);
        return SP2_ENOMEM;
    }
    s->arena.init(s->arena_mem, o.hbm_budget_bytes);
    std::memset(s->g_host, 0, sizeof(GroupDesc));
    // capture one tick: iters_per_tick x (grouped encode, product, control)
    ok = hipMemcpy(s->g_dev, s->g_host, sizeof(GroupDesc), hipMemcpyHostToDevice) == hipSuccess;
    // make the lazily set kernel attributes happen outside the capture
    ok = ok && launch_int8x_grouped(o.slices, o.levels, s->g_dev, 256, s->stream) == hipSuccess;
    ok = ok && launch_ctrl_step_grouped(s->g_dev, s->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(s->stream) == hipSuccess;
    hipGraph_t g = nullptr;
    ok = ok && hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (int k = 0; k < o.iters_per_tick && ok; ++k) {
            ok = launch_int8x_grouped(o.slices, o.levels, s->g_dev, 256, s->stream) == hipSuccess;
            ok = ok && launch_ctrl_step_grouped(s->g_dev, s->stream) == hipSuccess;
        }
        ok = (hipStreamEndCapture(s->stream, &g) == hipSuccess) && ok;
    }
    ok = ok && hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        sp2_server_destroy(s);
        return SP2_EDEVICE;
    }
    s->worker = std::thread([s] { s->loop(); });
    s->completer = std::thread([s] { s->complete_loop(); });
    *out = s;
    return SP2_OK;
}

sp2_status sp2_server_submit(sp2_server* s, int N, const double* H_host, int n_occ, uint64_t* ticket) {
    if (!s || !H_host || !ticket) return SP2_EINVAL;
    if (!fits_int8(N) || n_occ <= 0 || n_occ >= N) return SP2_EINVAL;
    const double t_call = now_s();
    Layout L = layout_for(N, s->opt.slices);
    if (L.total > s->opt.hbm_budget_bytes) return SP2_EBUDGET;
    Request* r = new Request();
    r->N = N;
    r->n_occ = n_occ;
    r->L = L;
    r->H = (double*)s->pinned.get((size_t)N * N * 8);
    r->D = (double*)s->pinned.get((size_t)N * N * 8);
    r->q = (double*)s->pinned.get((size_t)(N / 4 + 1) * 8);
    if (!r->H || !r->D || !r->q) {
        s->pinned.put(r->H, (size_t)N * N * 8);
        s->pinned.put(r->D, (size_t)N * N * 8);
        s->pinned.put(r->q, (size_t)(N / 4 + 1) * 8);
        delete r;
        return SP2_ENOMEM;
    }
    std::memcpy(r->H, H_host, (size_t)N * N * 8);
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = t_call;
    if (s->first_submit < 0) s->first_submit = r->t_submit;
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return SP2_OK;
}

sp2_status sp2_server_wait(sp2_server* s, uint64_t ticket, double timeout_s, double* D_out, double* q_out,
                           sp2_stats* stats) {
    if (!s) return SP2_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return SP2_EINVAL;
    Request* r = it->second;
    const auto pred = [r] { return r->done; };
    if (timeout_s < 0) s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return SP2_ETIMEOUT;
    if (stats) *stats = r->stats;
    const int status = r->status;
    s->reqs.erase(it);
    lk.unlock();
    // the request is finished and no longer known to the server: copy the
    // results out without holding the lock the scheduler needs every tick
    if (status == SP2_OK) {
        if (D_out) std::memcpy(D_out, r->D, (size_t)r->N * r->N * 8);
        if (q_out && r->N % 4 == 0) std::memcpy(q_out, r->q, (size_t)(r->N / 4) * 8);
    }
    if (r->ev_up) (void)hipEventDestroy(r->ev_up);
    if (r->ev_down) (void)hipEventDestroy(r->ev_down);
    s->pinned.put(r->H, (size_t)r->N * r->N * 8);
    s->pinned.put(r->D, (size_t)r->N * r->N * 8);
    s->pinned.put(r->q, (size_t)(r->N / 4 + 1) * 8);
    delete r;
    return (sp2_status)status;
}

sp2_status sp2_server_report(sp2_server* s, double* p50_ms, double* p99_ms, double* solves_per_s) {
    if (!s) return SP2_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat_ms;
    if (v.empty()) {
        if (p50_ms) *p50_ms = 0;
        if (p99_ms) *p99_ms = 0;
        if (solves_per_s) *solves_per_s = 0;
        return SP2_OK;
    }
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        const double idx = p * (v.size() - 1);
        const size_t lo = (size_t)idx, hi = std::min(lo + 1, v.size() - 1);
        return v[lo] + (idx - lo) * (v[hi] - v[lo]);
    };
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (solves_per_s) {
        const double span = s->last_done - s->first_submit;
        *solves_per_s = span > 0 ? s->completed / span : 0.0;
    }
    return SP2_OK;
}

void sp2_server_destroy(sp2_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->worker_done = true;   // also when the worker never ran
    }
    s->cv_down.notify_all();
    if (s->completer.joinable()) s->completer.join();
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (auto& kv : s->reqs) {
        Request* r = kv.second;
        if (r->ev_up) (void)hipEventDestroy(r->ev_up);
        if (r->ev_down) (void)hipEventDestroy(r->ev_down);
        s->pinned.put(r->H, (size_t)r->N * r->N * 8);
        s->pinned.put(r->D, (size_t)r->N * r->N * 8);
        s->pinned.put(r->q, (size_t)(r->N / 4 + 1) * 8);
        delete r;
    }
    s->pinned.clear();
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->g_dev) (void)hipFree(s->g_dev);
    if (s->g_host) (void)hipHostFree(s->g_host);
    if (s->st_dev) (void)hipFree(s->st_dev);
    if (s->st_host) (void)hipHostFree(s->st_host);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->ev_tick) (void)hipEventDestroy(s->ev_tick);
    delete s;
}

}  // extern "C"
