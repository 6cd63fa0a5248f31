// cf_server.hip -- continuous-batching serving loop over a filter set
// (include/cf_server.h).
//
// One scheduler thread owns `depth` batch slots, each with a HIP stream of
// its own and a scratch lane of the filter set.  Whenever a slot is free it
// takes pending requests in arrival order that fit the batch and keep
// per-filter arrival order (see cf_server.h), copies the request table to
// the device, and enqueues on the slot's stream: a gather kernel that lays
// the requests' keys out as one mixed batch, the filter set's batch
// kernels, and a scatter kernel that writes each request's results back,
// then records the slot's event.  Batches in different slots run at the
// same time on the device; a batch waits (by event, on the device) only for
// the in-flight batches that touch one of its filters, which keeps each
// filter's arrival order.  A slot retires as soon as its event completes,
// so new requests are admitted while earlier batches are still running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cf.h"
#include "cf_error.hpp"
#include "cf_server.h"
#include "cf_set.h"
#include "cf_set_internal.hpp"

using cferr::fail;

namespace cfv {

constexpr int kBlock = 256;
constexpr uint32_t kMaxDepth = 8;

struct Req {
    uint64_t id = 0;
    uint32_t fid = 0, op = 0;
    const uint64_t *keys = nullptr;
    uint64_t n = 0;
    uint8_t *results = nullptr;
    uint64_t t_submit = 0, t_start = 0, t_done = 0, batch = 0;
    int32_t status = CF_OK;
    bool submitted = false;
    bool done = false;
};

// Device-side request table entry; `off` is the request's first operation
// in the batch, entries sorted by `off`.
struct Entry {
    const uint64_t *keys;
    uint8_t *results;
    uint64_t off;
    uint32_t fid;
    uint32_t op;
};

__device__ __forceinline__ uint32_t find_entry(const Entry *tab, uint32_t nreq, uint64_t j) {
    uint32_t lo = 0, hi = nreq;  // last entry with off <= j
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tab[mid].off <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void gather_kernel(const Entry *__restrict__ tab, uint32_t nreq,
                                                        uint64_t total, uint8_t *__restrict__ ops,
                                                        uint32_t *__restrict__ fids,
                                                        uint64_t *__restrict__ keys) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < total; j += stride) {
        const Entry &e = tab[find_entry(tab, nreq, j)];
        ops[j] = uint8_t(e.op);
        fids[j] = e.fid;
        keys[j] = e.keys[j - e.off];
    }
}

__global__ __launch_bounds__(kBlock) void scatter_kernel(const Entry *__restrict__ tab, uint32_t nreq,
                                                         uint64_t total,
                                                         const uint8_t *__restrict__ res) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < total; j += stride) {
        const Entry &e = tab[find_entry(tab, nreq, j)];
        e.results[j - e.off] = res[j];
    }
}

__global__ __launch_bounds__(kBlock) void fill_kernel(uint8_t *__restrict__ p, uint64_t n,
                                                      uint8_t v) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < n; j += stride) p[j] = v;
}

int grid_for(uint64_t n) {
    const uint64_t g = (n + kBlock - 1) / kBlock;
    return int(g < 4096 ? (g ? g : 1) : 4096);
}

struct Slot {
    uint8_t *d_ops = nullptr;
    uint32_t *d_fids = nullptr;
    uint64_t *d_keys = nullptr;
    uint8_t *d_res = nullptr;
    Entry *h_tab = nullptr;  // pinned
    Entry *d_tab = nullptr;
    hipStream_t stream = nullptr;  // the slot's own stream (default priority)
    hipEvent_t done = nullptr;
    std::vector<Req *> reqs;
    uint64_t seq = 0;
};

// The set's scratch lane of slot k: lanes 1.., so lane 0 stays with callers
// of the set's own entry points.
uint32_t lane_of(int k) { return uint32_t(k) + 1; }

int phase_of(uint32_t op) { return op == CF_OP_QUERY ? 0 : (op == CF_OP_DELETE ? 1 : 2); }

enum : uint8_t { kWaiting = 0, kResident = 1, kReleased = 2 };

}  // namespace cfv

struct cf_server {
    cf_server_config cfg{};
    int device = 0;
    uint32_t nfilters = 0;
    std::vector<cf_params> params;
    std::vector<uint64_t> tbytes;
    std::vector<uint8_t> state;
    uint64_t resident_bytes = 0;
    uint32_t resident_count = 0;
    cf_set *set = nullptr;
    hipStream_t stream = nullptr;  // for completing failed requests
    std::vector<cfv::Slot> slots;
    std::deque<int> inflight;
    std::vector<int> free_slots;
    // per filter: the slot and batch sequence number of the last batch that
    // touched it (scheduler thread only)
    std::vector<int> last_slot;
    std::vector<uint64_t> last_seq;
    // form_batch's per-filter marks (scheduler thread only)
    std::vector<int8_t> fb_maxph;
    std::vector<uint8_t> fb_blocked;
    std::vector<uint32_t> fb_touched;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<cfv::Req *> pending;
    std::vector<std::unique_ptr<cfv::Req>> reqs;
    std::deque<uint32_t> release_q;
    std::vector<uint8_t> released_ack;
    int replay_active = 0;
    bool stop = false;
    uint64_t batch_seq = 0;
    cf_server_stats stats{};
    std::chrono::steady_clock::time_point t0;
    std::thread sched;
    std::vector<std::thread> clients;

    uint64_t now() const {
        return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                            std::chrono::steady_clock::now() - t0)
                            .count());
    }
};

namespace cfv {

// Admit waiting filters, in declaration order, while they fit the budget.
// Called with the lock held and no batch in flight.
void admit(cf_server *s) {
    for (uint32_t f = 0; f < s->nfilters; ++f) {
        if (s->state[f] != kWaiting) continue;
        if (s->cfg.hbm_budget && s->resident_bytes + s->tbytes[f] > s->cfg.hbm_budget) break;
        if (cf_set_attach(s->set, f) != CF_OK) break;
        s->state[f] = kResident;
        s->resident_bytes += s->tbytes[f];
        s->resident_count++;
    }
}

// Complete a request that will not run (released filter or shutdown).
void fail_request(cf_server *s, Req *r) {
    if (r->n) {
        fill_kernel<<<grid_for(r->n), kBlock, 0, s->stream>>>(r->results, r->n, 0xFF);
        (void)hipStreamSynchronize(s->stream);
    }
    r->status = CF_EINVAL;
    r->t_start = r->t_done = s->now();
    r->done = true;
}

// Retire in-flight slot inflight[pos] (its event has completed).  Lock held.
void retire_at(cf_server *s, size_t pos) {
    const int k = s->inflight[pos];
    Slot &sl = s->slots[k];
    const uint64_t t = s->now();
    for (Req *r : sl.reqs) {
        r->t_done = t;
        r->done = true;
        s->stats.requests++;
        s->stats.operations += r->n;
    }
    sl.reqs.clear();
    s->free_slots.push_back(k);
    s->inflight.erase(s->inflight.begin() + long(pos));
    s->cv_done.notify_all();
}

// Retire every in-flight slot whose batch has completed; true if any did.
// Lock held.
bool retire_done(cf_server *s) {
    bool any = false;
    for (size_t pos = 0; pos < s->inflight.size();) {
        if (hipEventQuery(s->slots[s->inflight[pos]].done) == hipSuccess) {
            retire_at(s, pos);
            any = true;
        } else {
            ++pos;
        }
    }
    return any;
}

// Wait for every in-flight slot and retire it.  Lock held (released while
// waiting).
void retire_all(cf_server *s, std::unique_lock<std::mutex> &lk) {
    while (!s->inflight.empty()) {
        const int k = s->inflight.front();
        lk.unlock();
        (void)hipEventSynchronize(s->slots[k].done);
        lk.lock();
        retire_done(s);
    }
}

// Pick the requests of the next batch (lock held).  Returns them in arrival
// order and removes them from `pending`.  The scan stops once the batch is
// full (so one launch per request costs one step, however many requests are
// pending); the per-filter marks live in the server and are reset for the
// filters this call touched.
std::vector<Req *> form_batch(cf_server *s) {
    std::vector<Req *> take;
    // Batched mode takes whole batches only once direct_below requests are
    // pending; below that, one request per slot (cf_server.h, Modes).
    const bool batched =
        s->cfg.mode == CF_SERVE_BATCHED && s->pending.size() >= s->cfg.direct_below;
    // with a long backlog every request joins batches (capacity first)
    const bool backlog = s->pending.size() >= 4ull * s->cfg.direct_below;
    uint64_t ops_left = s->cfg.max_batch;
    uint32_t slots_left = batched ? s->cfg.max_requests : 1;
    std::vector<int8_t> &maxph = s->fb_maxph;     // latest phase taken per filter, -1: none
    std::vector<uint8_t> &blocked = s->fb_blocked;  // a held request precedes: take none
    std::vector<uint32_t> &touched = s->fb_touched;
    touched.clear();
    auto block = [&](uint32_t f) {
        if (!blocked[f]) {
            blocked[f] = 1;
            touched.push_back(f);
        }
    };
    std::deque<Req *> keep;
    auto it = s->pending.begin();
    for (; it != s->pending.end() && slots_left > 0 && ops_left > 0; ++it) {
        Req *r = *it;
        const uint32_t f = r->fid;
        if (s->state[f] == kReleased) {
            fail_request(s, r);
            s->cv_done.notify_all();
            continue;
        }
        if (s->state[f] != kResident || blocked[f]) {
            block(f);
            keep.push_back(r);
            continue;
        }
        const int ph = phase_of(r->op);
        // a request of solo_above keys or more runs alone while the backlog is
        // short: taken by itself when it comes first, otherwise left for a
        // slot of its own (and its filter's later requests with it)
        const bool solo = batched && !backlog && r->n >= s->cfg.solo_above;
        if (maxph[f] > ph || r->n > ops_left || (solo && !take.empty())) {
            block(f);
            keep.push_back(r);
            continue;
        }
        if (solo) {
            take.push_back(r);
            ++it;
            break;
        }
        if (maxph[f] < 0) touched.push_back(f);
        maxph[f] = int8_t(ph);
        ops_left -= r->n;
        slots_left--;
        take.push_back(r);
    }
    keep.insert(keep.end(), it, s->pending.end());
    s->pending.swap(keep);
    for (uint32_t f : touched) {
        maxph[f] = -1;
        blocked[f] = 0;
    }
    return take;
}

// Enqueue one batch on the device (lock not held; scheduler thread).
cf_status launch(cf_server *s, int slot_idx, std::vector<Req *> &take) {
    Slot &sl = s->slots[slot_idx];
    const uint64_t t = s->now();
    sl.seq = s->batch_seq++;
    for (Req *r : take) {
        r->t_start = t;
        r->batch = sl.seq;
    }
    cf_status st = CF_OK;
    // Per-filter order across slots: wait for the last batch that touched
    // one of this batch's filters, if it is still the batch in its slot (a
    // slot reused since then held a later batch, and its event says nothing
    // about this filter; the older batch has completed).
    std::vector<int> after;
    for (Req *r : take) {
        const int j = s->last_slot[r->fid];
        if (j >= 0 && j != slot_idx && s->slots[j].seq == s->last_seq[r->fid] &&
            std::find(after.begin(), after.end(), j) == after.end())
            after.push_back(j);
        s->last_slot[r->fid] = slot_idx;
        s->last_seq[r->fid] = sl.seq;
    }
    for (int j : after)
        if (hipStreamWaitEvent(sl.stream, s->slots[j].done, 0) != hipSuccess) {
            st = fail(CF_EDEVICE, "ordering wait failed");
            break;
        }
    if (st != CF_OK) {
        // nothing else runs on this slot
    } else if (s->cfg.mode == CF_SERVE_PER_REQUEST || take.size() < s->cfg.direct_below) {
        // Arrival order is an order the batch semantics allow (form_batch).
        for (Req *r : take) {
            st = cfs::apply_lane(s->set, lane_of(slot_idx), r->fid, r->op, r->keys, r->n,
                                 r->results, sl.stream);
            if (st != CF_OK) break;
        }
    } else {
        uint64_t off = 0;
        for (size_t k = 0; k < take.size(); ++k) {
            sl.h_tab[k] = Entry{take[k]->keys, take[k]->results, off, take[k]->fid, take[k]->op};
            off += take[k]->n;
        }
        const uint32_t nreq = uint32_t(take.size());
        if (hipMemcpyAsync(sl.d_tab, sl.h_tab, nreq * sizeof(Entry), hipMemcpyHostToDevice,
                           sl.stream) != hipSuccess) {
            st = fail(CF_EDEVICE, "request table copy failed");
        } else {
            gather_kernel<<<grid_for(off), kBlock, 0, sl.stream>>>(sl.d_tab, nreq, off, sl.d_ops,
                                                                   sl.d_fids, sl.d_keys);
            st = cfs::execute_lane(s->set, lane_of(slot_idx), sl.d_ops, sl.d_fids, sl.d_keys,
                                   off, sl.d_res, sl.stream);
            if (st == CF_OK)
                scatter_kernel<<<grid_for(off), kBlock, 0, sl.stream>>>(sl.d_tab, nreq, off,
                                                                        sl.d_res);
        }
    }
    if (st == CF_OK && hipGetLastError() != hipSuccess) st = fail(CF_EDEVICE, "batch launch failed");
    // Every path records the slot's event and hands the requests to the slot,
    // so they retire (and their waiters wake) even when the batch failed; a
    // failed batch's requests carry its status and their results are undefined.
    (void)hipEventRecord(sl.done, sl.stream);
    if (st != CF_OK)
        for (Req *r : take) r->status = st;
    sl.reqs = take;
    return st;
}

bool has_work(cf_server *s) {
    for (Req *r : s->pending)
        if (s->state[r->fid] != kWaiting) return true;
    return false;
}

void process_releases(cf_server *s, std::unique_lock<std::mutex> &lk) {
    std::deque<uint32_t> later;
    while (!s->release_q.empty()) {
        const uint32_t f = s->release_q.front();
        s->release_q.pop_front();
        bool busy = false;
        for (Req *r : s->pending)
            if (r->fid == f) busy = true;
        for (int k : s->inflight)
            for (Req *r : s->slots[k].reqs)
                if (r->fid == f) busy = true;
        if (busy && s->state[f] == kResident) {
            later.push_back(f);
            continue;
        }
        retire_all(s, lk);
        if (s->state[f] == kResident) {
            (void)cf_set_detach(s->set, f);
            s->resident_bytes -= s->tbytes[f];
            s->resident_count--;
        }
        s->state[f] = kReleased;
        s->released_ack[f] = 1;
        admit(s);
        s->cv_done.notify_all();
    }
    s->release_q.swap(later);
}

void scheduler(cf_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (!s->release_q.empty()) process_releases(s, lk);
        bool progress = retire_done(s);
        if (s->stop) {
            retire_all(s, lk);
            for (Req *r : s->pending) fail_request(s, r);
            s->pending.clear();
            s->cv_done.notify_all();
            return;
        }
        if (!s->free_slots.empty() && has_work(s)) {
            std::vector<Req *> take = form_batch(s);
            if (!take.empty()) {
                const int k = s->free_slots.back();
                s->free_slots.pop_back();
                s->inflight.push_back(k);
                lk.unlock();
                (void)launch(s, k, take);
                lk.lock();
                s->stats.batches++;
                progress = true;
            }
        }
        if (progress) continue;
        if (!s->inflight.empty()) {
            // Something is on the device: poll it, but let new requests in.
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

void free_slots_mem(cf_server *s) {
    for (Slot &sl : s->slots) {
        if (sl.d_ops) (void)hipFree(sl.d_ops);
        if (sl.d_fids) (void)hipFree(sl.d_fids);
        if (sl.d_keys) (void)hipFree(sl.d_keys);
        if (sl.d_res) (void)hipFree(sl.d_res);
        if (sl.d_tab) (void)hipFree(sl.d_tab);
        if (sl.h_tab) (void)hipHostFree(sl.h_tab);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    s->slots.clear();
}

}  // namespace cfv

extern "C" {

cf_status cf_server_create(const cf_params *params, uint32_t nfilters,
                           const cf_server_config *cfg, cf_server **out) {
    if (!out || !cfg || !params) return fail(CF_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->mode > CF_SERVE_PER_REQUEST || cfg->depth < 1 || cfg->depth > cfv::kMaxDepth ||
        cfg->max_requests < 1 || cfg->max_requests > 65536 || cfg->max_batch == 0)
        return fail(CF_EINVAL, "bad server config");
    cf_server *s = new (std::nothrow) cf_server();
    if (!s) return fail(CF_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    if (s->cfg.direct_below == 0) s->cfg.direct_below = 16;
    if (s->cfg.solo_above == 0) s->cfg.solo_above = 1u << 16;
    s->nfilters = nfilters;
    s->params.assign(params, params + nfilters);
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(CF_EDEVICE, "no current HIP device");
    }
    // When every table fits the budget, every filter is admitted at once, so
    // the set is created with its tables (in one allocation, which serves
    // batches faster than one per table); otherwise tables are allocated as
    // filters are admitted.
    uint64_t all_tables = 0;
    for (uint32_t f = 0; f < nfilters; ++f) all_tables += cf_table_bytes(&params[f]);
    const bool all_fit = cfg->hbm_budget == 0 || all_tables <= cfg->hbm_budget;
    cf_status st = cf_set_create(params, nfilters, cfg->max_batch,
                                 all_fit ? 0u : uint32_t(CF_SET_DEFER_TABLES), &s->set);
    if (st != CF_OK) {
        delete s;
        return st;
    }
    s->tbytes.resize(nfilters);
    for (uint32_t f = 0; f < nfilters; ++f) s->tbytes[f] = cf_table_bytes(&params[f]);
    s->state.assign(nfilters, cfv::kWaiting);
    s->released_ack.assign(nfilters, 0);
    s->last_slot.assign(nfilters, -1);
    s->last_seq.assign(nfilters, 0);
    s->fb_maxph.assign(nfilters, -1);
    s->fb_blocked.assign(nfilters, 0);
    bool okall = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
                 cfs::reserve_lanes(s->set, cfg->depth + 1) == CF_OK;
    s->slots.resize(cfg->depth);
    const bool batched = cfg->mode == CF_SERVE_BATCHED;
    for (uint32_t k = 0; okall && k < cfg->depth; ++k) {
        cfv::Slot &sl = s->slots[k];
        okall = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
                hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        if (okall && batched)
            okall = hipMalloc(&sl.d_ops, cfg->max_batch) == hipSuccess &&
                    hipMalloc(&sl.d_fids, cfg->max_batch * 4) == hipSuccess &&
                    hipMalloc(&sl.d_keys, cfg->max_batch * 8) == hipSuccess &&
                    hipMalloc(&sl.d_res, cfg->max_batch) == hipSuccess &&
                    hipMalloc(&sl.d_tab, cfg->max_requests * sizeof(cfv::Entry)) == hipSuccess &&
                    hipHostMalloc(&sl.h_tab, cfg->max_requests * sizeof(cfv::Entry)) == hipSuccess;
        s->free_slots.push_back(int(k));
    }
    if (!okall) {
        (void)hipGetLastError();
        cfv::free_slots_mem(s);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        cf_set_destroy(s->set);
        delete s;
        return fail(CF_ENOMEM, "cannot allocate the server's batch slots");
    }
    cfv::admit(s);
    s->sched = std::thread(cfv::scheduler, s);
    *out = s;
    return CF_OK;
}

cf_status cf_server_destroy(cf_server *s) {
    if (!s) return CF_OK;
    for (std::thread &t : s->clients)
        if (t.joinable()) t.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->sched.joinable()) s->sched.join();
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    cfv::free_slots_mem(s);
    (void)hipStreamDestroy(s->stream);
    cf_set_destroy(s->set);
    delete s;
    return CF_OK;
}

static cf_status check_request(cf_server *s, uint32_t fid, uint32_t op, const uint64_t *keys,
                               uint64_t n, const uint8_t *results) {
    if (fid >= s->nfilters || op > CF_OP_INSERT) return fail(CF_EINVAL, "bad filter or kind");
    if (n > s->cfg.max_batch) return fail(CF_EINVAL, "request larger than max_batch");
    if (n && (!keys || !results)) return fail(CF_EINVAL, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return fail(CF_EINVAL, "keys not 8-byte aligned");
    return CF_OK;
}

cf_status cf_server_submit(cf_server *s, uint32_t fid, uint32_t op, const uint64_t *keys,
                           uint64_t n, uint8_t *results, uint64_t *id_out) {
    if (!s || !id_out) return fail(CF_EINVAL, "NULL argument");
    cf_status st = check_request(s, fid, op, keys, n, results);
    if (st != CF_OK) return st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(CF_EINVAL, "server is stopping");
        auto r = std::make_unique<cfv::Req>();
        r->id = s->reqs.size();
        r->fid = fid;
        r->op = op;
        r->keys = keys;
        r->n = n;
        r->results = results;
        r->t_submit = s->now();
        r->submitted = true;
        if (n == 0) {
            r->t_start = r->t_done = r->t_submit;
            r->done = true;
            s->stats.requests++;
        } else {
            s->pending.push_back(r.get());
        }
        *id_out = r->id;
        s->reqs.push_back(std::move(r));
    }
    s->cv_sched.notify_one();
    return CF_OK;
}

cf_status cf_server_wait(cf_server *s, uint64_t id, cf_request_info *info) {
    if (!s) return fail(CF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    if (id >= s->reqs.size()) return fail(CF_EINVAL, "unknown request id");
    cfv::Req *r = s->reqs[id].get();
    s->cv_done.wait(lk, [&] { return r->done; });
    if (info)
        *info = cf_request_info{r->id, r->t_submit, r->t_start, r->t_done, r->batch, r->status, 0};
    return CF_OK;
}

cf_status cf_server_drain(cf_server *s) {
    if (!s) return fail(CF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] {
        if (s->replay_active) return false;
        for (cfv::Req *r : s->pending)
            if (s->state[r->fid] != cfv::kWaiting) return false;
        return s->inflight.empty();
    });
    return CF_OK;
}

cf_status cf_server_release(cf_server *s, uint32_t fid) {
    if (!s || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->state[fid] == cfv::kReleased) return CF_OK;
    s->release_q.push_back(fid);
    s->cv_sched.notify_all();
    s->cv_done.wait(lk, [&] { return s->released_ack[fid] != 0; });
    return CF_OK;
}

cf_status cf_server_resident(cf_server *s, uint32_t fid, int *out) {
    if (!s || !out || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->state[fid] == cfv::kResident ? 1 : 0;
    return CF_OK;
}

cf_status cf_server_stats_get(cf_server *s, cf_server_stats *out) {
    if (!s || !out) return fail(CF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    uint64_t held = 0;
    for (cfv::Req *r : s->pending)
        if (s->state[r->fid] == cfv::kWaiting) held++;
    out->held = held;
    out->resident_bytes = s->resident_bytes;
    out->resident = s->resident_count;
    return CF_OK;
}

cf_set *cf_server_set(cf_server *s) { return s ? s->set : nullptr; }

cf_status cf_server_replay(cf_server *s, uint64_t count, const uint64_t *arrival_ns,
                           const uint32_t *fids, const uint32_t *ops, const uint64_t *key_off,
                           const uint64_t *n, const uint64_t *d_keys, uint8_t *d_results,
                           uint64_t *first_id_out) {
    if (!s || !first_id_out || (count && (!arrival_ns || !fids || !ops || !key_off || !n ||
                                          !d_keys || !d_results)))
        return fail(CF_EINVAL, "NULL argument");
    for (uint64_t k = 0; k < count; ++k) {
        cf_status st = check_request(s, fids[k], ops[k], d_keys + key_off[k], n[k],
                                     d_results + key_off[k]);
        if (st != CF_OK) return st;
    }
    std::vector<cfv::Req *> trace;
    std::vector<uint64_t> when(arrival_ns, arrival_ns + count);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(CF_EINVAL, "server is stopping");
        *first_id_out = s->reqs.size();
        for (uint64_t k = 0; k < count; ++k) {
            auto r = std::make_unique<cfv::Req>();
            r->id = s->reqs.size();
            r->fid = fids[k];
            r->op = ops[k];
            r->keys = d_keys + key_off[k];
            r->n = n[k];
            r->results = d_results + key_off[k];
            trace.push_back(r.get());
            s->reqs.push_back(std::move(r));
        }
        s->replay_active++;
        // under the lock: replays may be started from several threads
        s->clients.emplace_back([s, trace, when]() {
            const uint64_t base = s->now();
            for (size_t k = 0; k < trace.size(); ++k) {
                const uint64_t due = base + when[k];
                // sleep through long gaps, spin the last stretch for timing
                for (uint64_t t = s->now(); t < due; t = s->now()) {
                    if (due - t > 200000)
                        std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
                }
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    cfv::Req *r = trace[k];
                    r->t_submit = due;  // latency counts from the trace's arrival time
                    r->submitted = true;
                    if (r->n == 0) {
                        r->t_start = r->t_done = r->t_submit;
                        r->done = true;
                        s->stats.requests++;
                        s->cv_done.notify_all();
                    } else {
                        s->pending.push_back(r);
                    }
                }
                s->cv_sched.notify_one();
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->replay_active--;
            s->cv_done.notify_all();
        });
    }
    return CF_OK;
}

}  // extern "C"
