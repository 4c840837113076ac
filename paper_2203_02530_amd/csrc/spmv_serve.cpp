// Serving engine: resident matrices, HBM-budget admission and continuous
// batching of y = A x requests.
//
// A worker thread runs the loop
//   retire:  batches whose completion event has fired release their request
//            buffers and report their requests as done;
//   admit:   queued requests (FIFO) move onto the device while the budget
//            (resident matrices + request buffers in use) and the in-flight
//            limit allow; buffers come from a first-fit arena;
//   launch:  all admitted requests not yet running, up to max_batch, become
//            one batch on a free batch slot: x copies, one grouped
//            stream-CSR launch over all their tiles, y copies, an event.
// Up to max_epochs batches are on the device at once, each on its own
// stream, so requests that arrive while others run are launched without
// waiting for them (continuous batching, not a queue in front of one
// executor).  mode 1 (plain) sets max_batch = max_epochs = max_inflight = 1.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "spmv_internal.h"

namespace spmv {
namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

int64_t al256(int64_t v) { return (v + 255) & ~int64_t(255); }

// First-fit allocator over [0, cap) with coalescing of free neighbours.
struct Arena {
    std::map<int64_t, int64_t> free_;   // offset -> size
    int64_t cap = 0, used = 0, peak = 0;

    void init(int64_t c)
    {
        cap = c;
        used = peak = 0;
        free_.clear();
        if (c > 0) free_[0] = c;
    }
    int64_t alloc(int64_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, rem = it->second - n;
            free_.erase(it);
            if (rem) free_[off + n] = rem;
            used += n;
            peak = std::max(peak, used);
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        used -= n;
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

struct Req {
    int64_t tag = 0;
    int32_t mat = 0;
    const double *xh = nullptr;
    double *yh = nullptr;
    double t_arrival = 0, t_done = 0;
    int64_t off = -1, bytes = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    ServeDev *d_desc = nullptr;   // device: descriptors then prefix
    int32_t *d_pref = nullptr;
    char *h_stage = nullptr;      // pinned: same layout as the device copy
    std::vector<int64_t> reqs;
    bool busy = false;
};

}  // namespace
}  // namespace spmv

using namespace spmv;

struct spmv_server {
    spmv_server_opts_t o{};
    int device = 0;
    std::vector<spmv_plan *> mats;
    int64_t resident = 0;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    size_t stage_bytes = 0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> reqs;                 // all requests, by id (stable)
    std::deque<int64_t> pending;          // ids not yet admitted
    std::vector<std::pair<int64_t, double>> done;  // (tag, latency) not yet polled
    int64_t submitted = 0, completed = 0, batches = 0, batched_reqs = 0;

    // worker-only state
    std::vector<int64_t> admitted;
    int32_t inflight = 0, peak_inflight = 0;

    std::thread worker;
    std::atomic<bool> stop{false}, started{false};
    int worker_error = SPMV_OK;
    std::string worker_msg;
};

namespace {

int64_t req_bytes(const spmv_server *s, int32_t mat)
{
    return 2 * al256(std::max<int64_t>(s->mats[size_t(mat)]->share.n_loc, 1) * 8);
}

// `rq` holds copies of the batch's requests, taken under the lock (the
// request deque grows concurrently with submissions).
int launch_batch(spmv_server *s, Slot &sl, const std::vector<int64_t> &ids,
                 const std::vector<Req> &rq)
{
    const int n = int(ids.size());
    auto *desc = reinterpret_cast<ServeDev *>(sl.h_stage);
    auto *pref = reinterpret_cast<int32_t *>(sl.h_stage + al256(int64_t(s->o.max_batch) *
                                                                 int64_t(sizeof(ServeDev))));
    pref[0] = 0;
    for (int i = 0; i < n; ++i) {
        const Req &r = rq[size_t(i)];
        const spmv_plan *p = s->mats[size_t(r.mat)];
        const int64_t nl = p->share.n_loc;
        double *x = reinterpret_cast<double *>(s->arena_base + r.off);
        ServeDev &d = desc[i];
        d.tile_row = p->d_tile_row[0];
        d.tile_k = p->d_tile_k[0];
        d.rp = p->dL_ptr;
        d.col = p->dL_col;
        d.val = p->dL_val;
        d.x = x;
        d.y = reinterpret_cast<double *>(reinterpret_cast<char *>(x) + al256(std::max<int64_t>(nl, 1) * 8));
        d.nnz_alloc = uint32_t(p->share.L_col.size() + kEntryPad);
        d.n = uint32_t(nl);
        d.lanes = p->cfg[0].lanes;
        d.n_tiles = int32_t(p->cfg[0].tile_row.size()) - 1;
        pref[i + 1] = pref[i] + d.n_tiles;
    }
    // A small batch passes its descriptors in the kernel arguments; a larger one
    // copies them to the slot's device buffer ahead of the launch.
    const bool inline_desc = n <= kServeInline;
    if (!inline_desc)
        SPMV_HIP(hipMemcpyAsync(sl.d_desc, sl.h_stage, s->stage_bytes, hipMemcpyHostToDevice, sl.st));
    for (int i = 0; i < n; ++i) {
        const Req &r = rq[size_t(i)];
        const int64_t nl = s->mats[size_t(r.mat)]->share.n_loc;
        if (nl)
            SPMV_HIP(hipMemcpyAsync(const_cast<double *>(desc[i].x), r.xh, size_t(nl) * 8,
                                    hipMemcpyHostToDevice, sl.st));
    }
    if (inline_desc) {
        ServeInline a{};
        for (int i = 0; i < n; ++i) a.d[i] = desc[i];
        for (int i = 0; i <= n; ++i) a.pref[i] = pref[i];
        a.n_req = n;
        SPMV_HIP(launch_serve_inline(s->o.chunk, 2, a, sl.st));
    } else {
        SPMV_HIP(launch_serve(s->o.chunk, 2, sl.d_desc, sl.d_pref, n, pref[n], sl.st));
    }
    for (int i = 0; i < n; ++i) {
        const Req &r = rq[size_t(i)];
        const int64_t nl = s->mats[size_t(r.mat)]->share.n_loc;
        if (nl)
            SPMV_HIP(hipMemcpyAsync(r.yh, desc[i].y, size_t(nl) * 8, hipMemcpyDeviceToHost, sl.st));
    }
    SPMV_HIP(hipEventRecord(sl.ev, sl.st));
    sl.reqs = ids;
    sl.busy = true;
    return SPMV_OK;
}

void worker_loop(spmv_server *s)
{
    (void)hipSetDevice(s->device);
    auto idle_since = Clock::now();
    while (true) {
        bool did = false;
        // retire finished batches
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            const double t = now_s();
            std::lock_guard<std::mutex> lk(s->mu);
            if (q != hipSuccess && s->worker_error == SPMV_OK) {
                s->worker_error = SPMV_EHIP;
                s->worker_msg = std::string("batch event: ") + hipGetErrorString(q);
            }
            for (int64_t id : sl.reqs) {
                Req &r = s->reqs[size_t(id)];
                r.t_done = t;
                s->arena.release(r.off, r.bytes);
                s->done.emplace_back(r.tag, t - r.t_arrival);
                ++s->completed;
            }
            s->inflight -= int32_t(sl.reqs.size());
            sl.reqs.clear();
            sl.busy = false;
            did = true;
        }
        // admit and launch
        std::vector<int64_t> batch;
        std::vector<Req> batch_reqs;
        Slot *free_slot = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            // after a device error nothing more is admitted: the caller sees
            // the error from drain/submit, and destroy must not wait for
            // requests that can no longer complete
            while (!s->worker_error && !s->pending.empty() &&
                   s->inflight + int32_t(s->admitted.size()) < s->o.max_inflight) {
                Req &r = s->reqs[size_t(s->pending.front())];
                if (s->resident + s->arena.used + r.bytes > s->o.budget_bytes) break;
                const int64_t off = s->arena.alloc(r.bytes);
                if (off < 0) break;
                r.off = off;
                s->admitted.push_back(s->pending.front());
                s->pending.pop_front();
                did = true;
            }
            for (Slot &sl : s->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            if (free_slot && !s->admitted.empty() && !s->worker_error) {
                const size_t k = std::min<size_t>(s->admitted.size(), size_t(s->o.max_batch));
                batch.assign(s->admitted.begin(), s->admitted.begin() + long(k));
                for (int64_t id : batch) batch_reqs.push_back(s->reqs[size_t(id)]);
                s->admitted.erase(s->admitted.begin(), s->admitted.begin() + long(k));
                s->inflight += int32_t(k);
                s->peak_inflight = std::max(s->peak_inflight, s->inflight);
                ++s->batches;
                s->batched_reqs += int64_t(k);
            }
        }
        if (!batch.empty()) {
            const int rc = launch_batch(s, *free_slot, batch, batch_reqs);
            if (rc != SPMV_OK) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->worker_error = rc;
                s->worker_msg = spmv_last_error();
            }
            did = true;
        }
        if (did) {
            s->cv.notify_all();
            idle_since = Clock::now();
            continue;
        }
        bool busy = false;
        for (const Slot &sl : s->slots) busy |= sl.busy;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && (s->worker_error || (s->pending.empty() && s->admitted.empty())))
            break;
        if (busy || !s->pending.empty() || Clock::now() - idle_since < std::chrono::milliseconds(2)) {
            lk.unlock();
            std::this_thread::yield();   // keep completion latency low while work is around
        } else {
            s->cv.wait_for(lk, std::chrono::microseconds(200));
        }
    }
}

int submit_at(spmv_server *s, int32_t matrix, const double *x, double *y, int64_t tag,
              double t_arrival)
{
    if (matrix < 0 || matrix >= int32_t(s->mats.size()))
        return set_error(SPMV_EINVAL, "unknown matrix id");
    const int64_t n = s->mats[size_t(matrix)]->share.n_loc;
    if (n > 0 && (!x || !y)) return set_error(SPMV_EINVAL, "x or y is NULL");
    const int64_t need = req_bytes(s, matrix);
    if (s->resident + need > s->o.budget_bytes || need > s->arena.cap)
        return set_error(SPMV_EBUDGET, "request can never fit the budget");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->worker_error) return set_error(s->worker_error, s->worker_msg);
        Req r;
        r.tag = tag;
        r.mat = matrix;
        r.xh = x;
        r.yh = y;
        r.t_arrival = t_arrival;
        r.bytes = need;
        s->reqs.push_back(r);
        s->pending.push_back(int64_t(s->reqs.size()) - 1);
        ++s->submitted;
    }
    s->cv.notify_all();
    return SPMV_OK;
}

void server_release(spmv_server *s)
{
    for (Slot &sl : s->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    for (spmv_plan *p : s->mats) spmv_plan_destroy(p);
    delete s;
}

}  // namespace

extern "C" int spmv_server_create(const spmv_server_opts_t *opts, spmv_server_t **out)
{
    if (!out) return set_error(SPMV_EINVAL, "out is NULL");
    *out = nullptr;
    spmv_server_opts_t o{};
    if (opts) o = *opts;
    if (o.budget_bytes < 0 || o.max_inflight < 0 || o.max_epochs < 0 || o.max_batch < 0 ||
        o.mode < 0 || o.mode > 1 || (o.chunk != 0 && o.chunk != 4 && o.chunk != 8 && o.chunk != 16))
        return set_error(SPMV_EINVAL, "server option out of range");
    if (!o.budget_bytes) o.budget_bytes = int64_t(64) << 30;
    if (!o.max_inflight) o.max_inflight = 256;
    if (!o.max_epochs) o.max_epochs = 4;
    if (!o.max_batch) o.max_batch = 64;
    if (!o.chunk) o.chunk = 8;
    if (o.mode == 1) o.max_inflight = o.max_epochs = o.max_batch = 1;
    auto *s = new (std::nothrow) spmv_server();
    if (!s) return set_error(SPMV_ENOMEM, "server allocation");
    s->o = o;
    const hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "hipGetDevice");
    }
    *out = s;
    return SPMV_OK;
}

extern "C" int spmv_server_add_matrix(spmv_server_t *s, const spmv_csr_t *csr, int32_t *id)
{
    if (!s || !csr || !id) return set_error(SPMV_EINVAL, "NULL argument");
    if (s->started) return set_error(SPMV_ESTATE, "matrices must be added before start");
    spmv_tune_t t{};
    t.kernel_local = SPMV_KERNEL_STREAM;
    t.kernel_remote = SPMV_KERNEL_STREAM;
    t.chunk_local = s->o.chunk;
    t.chunk_remote = s->o.chunk;
    t.width = 2;
    t.form = 1;   // the serving kernel walks packed tiles
    // budget check before allocating: matrix + room for one request on it
    spmv_tune_t th = t;
    th.flags = SPMV_F_HOST_ONLY;
    spmv_plan_t *probe = nullptr;
    if (int rc = spmv_plan_create_ex(csr, 1, 0, nullptr, 0, nullptr, 1, &th, &probe)) return rc;
    const Share &S = probe->share;
    const int64_t est = 4 * int64_t(S.L_ptr.size()) + 12 * (int64_t(S.L_col.size()) + kEntryPad) +
                        8 * int64_t(probe->cfg[0].tile_row.size()) +
                        2 * al256(std::max<int64_t>(S.n_loc, 1) * 8);
    spmv_plan_destroy(probe);
    if (s->resident + est > s->o.budget_bytes)
        return set_error(SPMV_EBUDGET, "matrix does not fit the budget");
    spmv_plan_t *p = nullptr;
    if (int rc = spmv_plan_create_ex(csr, 1, 0, nullptr, 0, nullptr, 1, &t, &p)) return rc;
    s->mats.push_back(p);
    s->resident += int64_t(p->arena_bytes);
    *id = int32_t(s->mats.size()) - 1;
    return SPMV_OK;
}

extern "C" int spmv_server_start(spmv_server_t *s)
{
    if (!s) return set_error(SPMV_EINVAL, "server is NULL");
    if (s->started) return set_error(SPMV_ESTATE, "already started");
    if (s->mats.empty()) return set_error(SPMV_ESTATE, "no matrices");
    int64_t largest = 0;
    for (size_t m = 0; m < s->mats.size(); ++m) largest = std::max(largest, req_bytes(s, int32_t(m)));
    const int64_t room = s->o.budget_bytes - s->resident;
    if (room < largest) return set_error(SPMV_EBUDGET, "no room for a request on the largest matrix");
    const int64_t cap = std::min(room, largest * int64_t(s->o.max_inflight));
    SPMV_HIP(hipSetDevice(s->device));
    SPMV_HIP(hipMalloc((void **)&s->arena_base, size_t(cap)));
    s->arena.init(cap);
    s->stage_bytes = size_t(al256(int64_t(s->o.max_batch) * int64_t(sizeof(ServeDev))) +
                            al256(int64_t(s->o.max_batch + 1) * 4));
    s->slots.resize(size_t(s->o.max_epochs));
    for (Slot &sl : s->slots) {
        SPMV_HIP(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
        SPMV_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
        SPMV_HIP(hipHostMalloc((void **)&sl.h_stage, s->stage_bytes, hipHostMallocDefault));
        void *d = nullptr;
        SPMV_HIP(hipMalloc(&d, s->stage_bytes));
        sl.d_desc = static_cast<ServeDev *>(d);
        sl.d_pref = reinterpret_cast<int32_t *>(static_cast<char *>(d) +
                                                al256(int64_t(s->o.max_batch) * int64_t(sizeof(ServeDev))));
    }
    s->resident += int64_t(s->o.max_epochs) * int64_t(s->stage_bytes);
    s->started = true;
    s->worker = std::thread(worker_loop, s);
    return SPMV_OK;
}

extern "C" int spmv_server_submit(spmv_server_t *s, int32_t matrix, const double *x, double *y,
                                  int64_t tag)
{
    if (!s) return set_error(SPMV_EINVAL, "server is NULL");
    if (!s->started) return set_error(SPMV_ESTATE, "server not started");
    return submit_at(s, matrix, x, y, tag, now_s());
}

extern "C" int spmv_server_poll(spmv_server_t *s, int64_t *tags, double *lat, int32_t cap,
                                int32_t *n)
{
    if (!s || !n || (cap > 0 && (!tags || !lat))) return set_error(SPMV_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const int32_t k = int32_t(std::min<size_t>(size_t(std::max(cap, 0)), s->done.size()));
    for (int32_t i = 0; i < k; ++i) {
        tags[i] = s->done[size_t(i)].first;
        lat[i] = s->done[size_t(i)].second;
    }
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    if (s->worker_error) return set_error(s->worker_error, s->worker_msg);
    return SPMV_OK;
}

extern "C" int spmv_server_drain(spmv_server_t *s)
{
    if (!s) return set_error(SPMV_EINVAL, "server is NULL");
    if (!s->started) return SPMV_OK;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->completed == s->submitted || s->worker_error; });
    if (s->worker_error) return set_error(s->worker_error, s->worker_msg);
    return SPMV_OK;
}

extern "C" int spmv_server_run_trace(spmv_server_t *s, int64_t n, const int32_t *matrix,
                                     const double *arrival, const double *const *x,
                                     double *const *y, double *lat, double *wall)
{
    if (!s || n < 0 || (n > 0 && (!matrix || !arrival || !x || !y || !lat)))
        return set_error(SPMV_EINVAL, "bad argument to spmv_server_run_trace");
    if (!s->started) return set_error(SPMV_ESTATE, "server not started");
    if (int rc = spmv_server_drain(s)) return rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->done.clear();
    }
    const size_t first = s->reqs.size();
    const double t0 = now_s() + 1e-3;
    for (int64_t i = 0; i < n; ++i) {
        const double ta = t0 + arrival[i];
        while (now_s() < ta) {
        }
        if (int rc = submit_at(s, matrix[i], x[i], y[i], i, ta)) return rc;
    }
    if (int rc = spmv_server_drain(s)) return rc;
    double last = t0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int64_t i = 0; i < n; ++i) {
            const Req &r = s->reqs[first + size_t(i)];
            lat[i] = r.t_done - r.t_arrival;
            last = std::max(last, r.t_done);
        }
        s->done.clear();
    }
    if (wall) *wall = n > 0 ? last - (t0 + arrival[0]) : 0.0;
    return SPMV_OK;
}

extern "C" int spmv_server_stats(spmv_server_t *s, spmv_server_stats_t *st)
{
    if (!s || !st) return set_error(SPMV_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->batches = s->batches;
    st->resident_bytes = s->resident;
    st->peak_inflight_bytes = s->arena.peak;
    st->arena_bytes = s->arena.cap;
    st->peak_inflight = s->peak_inflight;
    st->n_matrices = int32_t(s->mats.size());
    st->mean_batch = s->batches ? double(s->batched_reqs) / double(s->batches) : 0.0;
    return SPMV_OK;
}

extern "C" int spmv_server_destroy(spmv_server_t *s)
{
    if (!s) return SPMV_OK;
    if (s->started) {
        (void)spmv_server_drain(s);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        if (s->worker.joinable()) s->worker.join();
        (void)hipDeviceSynchronize();
    }
    server_release(s);
    return SPMV_OK;
}
