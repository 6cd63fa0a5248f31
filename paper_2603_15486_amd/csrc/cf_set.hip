// cf_set.hip -- many filters on one device driven by mixed batches
// (include/cf_set.h).
//
// A batch of n (kind, filter, key) operations runs as one partition launch
// and then, per class (f, b, hash, placement) present in the set, a query, a
// delete and an insert launch, in that phase order.  The partition kernel
// cuts the batch into chunks of `chunk` operations, one per block, and sorts
// each chunk in LDS by bin = (kind, class); every later launch uses the same
// grid and block b works on the bin it owns in chunk b.  So no launch needs a
// global atomic to find its work, each launch runs fully unrolled code for
// one bucket geometry, and the phase order gives each filter the batch
// semantics of cf_set.h: queries see the state before the batch (they never
// overlap a write, as Sec. 4.4 requires), then deletes, then inserts.
// Per-filter occupancy deltas are tallied in LDS and added once per block
// (Sec. 4.3's hierarchical count, per filter).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "cf.h"
#include "cf_error.hpp"
#include "cf_kernels.hpp"
#include "cf_launch.hpp"
#include "cf_set.h"
#include "cf_set_internal.hpp"
#include "cf_set_kernels.hpp"
namespace cfs {

// ------------------------------------------------------------- partition

__global__ __launch_bounds__(kBlock) void partition_kernel(Batch bt, const uint8_t *__restrict__ cls,
                                                           uint32_t nfilters, uint32_t ncls,
                                                           uint32_t chunk, Scratch sc) {
    __shared__ uint32_t hist[kMaxBins + 1];
    __shared__ uint32_t base[kMaxBins + 1];
    const uint32_t nb = 3 * ncls;  // bin nb collects invalid operations
    const uint64_t n = batch_n(bt);
    const uint64_t lo = uint64_t(blockIdx.x) * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    for (uint32_t j = threadIdx.x; j <= nb; j += kBlock) hist[j] = 0;
    __syncthreads();
    auto bin_of = [&](uint64_t i) -> uint32_t {
        const uint32_t op = bt.ops[i], fid = bt.fids[i];
        if (op > 2u || fid >= nfilters) return nb;
        const uint32_t c = cls[fid];
        return c < ncls ? op * ncls + c : nb;  // 0xFF: filter detached
    };
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&hist[bin_of(i)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t j = 0; j <= nb; ++j) {
            base[j] = s;
            s += hist[j];
        }
    }
    __syncthreads();
    uint32_t *off = sc.binoff + uint64_t(blockIdx.x) * (nb + 1);
    for (uint32_t j = threadIdx.x; j <= nb; j += kBlock) {
        off[j] = base[j];
        hist[j] = base[j];  // becomes the scatter cursor
    }
    __syncthreads();
    uint32_t *seg = sc.sorted + lo;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        const uint32_t bin = bin_of(i);
        const uint32_t pos = atomicAdd(&hist[bin], 1u);
        seg[pos] = uint32_t(i);
        if (bin == nb) bt.results[i] = 0xFF;
    }
}

// -------------------------------------------------------------- counters

__global__ void set_totals_kernel(const SetFilter *__restrict__ filters, uint32_t nfilters,
                                  unsigned long long *__restrict__ out, int which) {
    const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfilters) return;
    const Counters *c = filters[f].ctr;
    if (which == 0) {
        unsigned long long s = 0;
        for (int k = 0; k < cfk::kStripes; ++k) s += c->count[k].v;
        out[f] = s;
    } else {
        out[f] = c->failures;
    }
}

bool pick(uint32_t f, uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out) {
    switch (f) {
        case 8:
            return pick_class_f8(b, hash, placement, out) &&
                   pick_class_insert_f8(b, hash, placement, out);
        case 16:
            return pick_class_f16(b, hash, placement, out) &&
                   pick_class_insert_f16(b, hash, placement, out);
        case 32:
            return pick_class_f32(b, hash, placement, out) &&
                   pick_class_insert_f32(b, hash, placement, out);
        default: return false;
    }
}

using cferr::fail;

cf_status check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return CF_OK;
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

cf_status validate_one(const cf_params &p, uint32_t idx) {
    char who[32];
    snprintf(who, sizeof(who), "filter %u", idx);
    return cfl::check_params(p, who);
}

uint64_t tbytes(const cf_params &p) {
    return ((p.num_buckets * uint64_t(p.slots_per_bucket) * p.fp_bits + 63) / 64) * 8;
}

struct Layout {
    std::vector<uint64_t> lost_off;
    uint64_t tables = 0, lost_entries = 0;
    uint64_t sorted_entries = 0, queue_entries = 0, binoff_entries = 0;
};

// Slack of the eviction queue beyond max_batch: single-filter inserts
// (cf_set_apply) round each of up to kApplyGrid blocks up to whole strides.
constexpr uint64_t kApplyGrid = 4096;

Layout layout_of(const cf_params *params, uint32_t nf, uint64_t max_batch) {
    Layout L;
    L.lost_off.resize(nf);
    for (uint32_t i = 0; i < nf; ++i) {
        L.tables += tbytes(params[i]);
        L.lost_off[i] = L.lost_entries;
        L.lost_entries += params[i].lost_capacity ? params[i].lost_capacity : kDefaultSetLost;
    }
    L.sorted_entries = max_batch + kMaxChunk;
    L.queue_entries = max_batch + kApplyGrid * kBlock;
    L.binoff_entries = ((max_batch + kMinChunk - 1) / kMinChunk + 1) * (kMaxBins + 1);
    return L;
}

uint64_t fixed_bytes(const Layout &L, uint32_t nf) {
    return uint64_t(nf) * (sizeof(Counters) + sizeof(SetFilter) + 1 + 8) +
           L.lost_entries * (8 + 4) + (L.sorted_entries + L.queue_entries) * 4 +
           L.binoff_entries * 4;
}

struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) switched = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

}  // namespace cfs

struct cf_set {
    int device = 0;
    uint32_t nfilters = 0;
    uint64_t max_batch = 0;
    uint32_t chunk = cfs::kDefaultChunk;
    uint32_t streams = 0;  // 0: one stream per class, at most kDefaultStreams
    int apply_grid = 4096;
    std::vector<cf_params> params;
    cfs::Layout layout;
    std::vector<uint32_t> cls_of;                // class per filter
    std::vector<cfs::ClassLaunch> classes;       // batched kernels per class
    std::vector<cfl::Launchers> single;          // single-filter kernels per filter
    std::vector<void *> tables;                  // nullptr while detached
    std::vector<cfs::SetFilter> hdesc;           // host copy of the descriptors
    cfs::SetFilter *d_filters = nullptr;
    uint8_t *d_cls = nullptr;
    cfk::Counters *d_ctr = nullptr;
    unsigned long long *d_lost_bucket = nullptr;
    uint32_t *d_lost_tag = nullptr;
    unsigned long long *d_totals = nullptr;
    cfs::Scratch sc{};
    std::vector<hipStream_t> side;  // streams 1.. of the class chains
    hipEvent_t fork = nullptr;      // recorded on the caller's stream
    std::vector<hipEvent_t> join;   // one per side stream
};

uint32_t cfs::filter_count(const cf_set *s) { return s ? s->nfilters : 0; }

struct cf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace cfs {

int grid_of(const cf_set *s, uint64_t n) { return int((n + s->chunk - 1) / s->chunk); }

uint32_t streams_of(const cf_set *s) {
    const uint32_t ncls = uint32_t(s->classes.size());
    const uint32_t want = s->streams ? s->streams : kDefaultStreams;
    const uint32_t l = std::min(want, ncls);
    return std::min<uint32_t>(l, uint32_t(s->side.size()) + 1);
}

// Partition, then per class its query, delete and insert launches in that
// order.  The phase order only binds operations on one filter and every
// filter belongs to exactly one class, so chains of different classes may
// overlap: with L streams, class c runs on stream c mod L, stream 0 being
// the caller's and the others side streams that wait for the partition
// and are waited for at the end.  Concurrent insert launches keep apart in
// the eviction queue because each uses the slice of its own bin.
cf_status enqueue(cf_set *s, const Batch &bt, int grid, hipStream_t st) {
    const uint32_t ncls = uint32_t(s->classes.size());
    const uint32_t nb = 3 * ncls;
    partition_kernel<<<grid, kBlock, 0, st>>>(bt, s->d_cls, s->nfilters, ncls, s->chunk, s->sc);
    cf_status r = check_launch("set partition");
    if (r != CF_OK) return r;
    uint32_t L = streams_of(s);
    if (L > 1 && hipEventRecord(s->fork, st) != hipSuccess) {
        (void)hipGetLastError();
        L = 1;  // no fork recorded: every chain on the caller's stream
    }
    uint32_t forked = 1;  // streams that waited on the fork (and so must be joined)
    for (; forked < L; ++forked)
        if (hipStreamWaitEvent(s->side[forked - 1], s->fork, 0) != hipSuccess) {
            r = fail(CF_EDEVICE, "set: side stream wait failed");
            break;
        }
    for (uint32_t c = 0; r == CF_OK && c < ncls; ++c) {
        const uint32_t l = c % L;
        hipStream_t cs = l ? s->side[l - 1] : st;
        const ClassLaunch &k = s->classes[c];
        k.query(bt, s->d_filters, s->chunk, nb, c, s->sc, grid, cs);
        if ((r = check_launch("set query")) != CF_OK) break;
        k.del(bt, s->d_filters, s->nfilters, s->chunk, nb, ncls + c, s->sc, grid, cs);
        if ((r = check_launch("set delete")) != CF_OK) break;
        k.ins(bt, s->d_filters, s->nfilters, s->chunk, nb, 2 * ncls + c, s->sc, grid, cs);
        r = check_launch("set insert");
    }
    // Join every forked stream back, also after an error, so the caller's
    // stream (or a capture in progress) is never left with a dangling fork.
    for (uint32_t l = 1; l < forked; ++l)
        if ((hipEventRecord(s->join[l - 1], s->side[l - 1]) != hipSuccess ||
             hipStreamWaitEvent(st, s->join[l - 1], 0) != hipSuccess) &&
            r == CF_OK)
            r = fail(CF_EDEVICE, "set: joining side stream %u failed", l);
    return r;
}

// Upload filter fid's descriptor and class entry (synchronous copies).
bool upload(cf_set *s, uint32_t fid) {
    const uint8_t c = s->tables[fid] ? uint8_t(s->cls_of[fid]) : uint8_t(0xFF);
    return hipMemcpy(s->d_filters + fid, &s->hdesc[fid], sizeof(SetFilter),
                     hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->d_cls + fid, &c, 1, hipMemcpyHostToDevice) == hipSuccess;
}

cf_status attach_table(cf_set *s, uint32_t fid) {
    if (s->tables[fid]) return CF_OK;
    const uint64_t nb = tbytes(s->params[fid]);
    void *t = nullptr;
    if (hipMalloc(&t, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_ENOMEM, "filter %u: cannot allocate a %llu-byte table", fid,
                    (unsigned long long)nb);
    }
    if (hipMemset(t, 0, nb) != hipSuccess ||
        hipMemset(s->d_ctr + fid, 0, sizeof(Counters)) != hipSuccess) {
        (void)hipFree(t);
        return fail(CF_EDEVICE, "filter %u: clearing the table failed", fid);
    }
    s->tables[fid] = t;
    s->hdesc[fid].table = t;
    return CF_OK;
}

void free_all(cf_set *s) {
    for (void *&t : s->tables)
        if (t) {
            (void)hipFree(t);
            t = nullptr;
        }
    void *ptrs[] = {s->d_filters,   s->d_cls,      s->d_ctr,    s->d_lost_bucket,
                    s->d_lost_tag,  s->d_totals,   s->sc.sorted, s->sc.queue,
                    s->sc.binoff};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipStream_t t : s->side) (void)hipStreamDestroy(t);
    for (hipEvent_t e : s->join) (void)hipEventDestroy(e);
    if (s->fork) (void)hipEventDestroy(s->fork);
    s->side.clear();
    s->join.clear();
    s->fork = nullptr;
}

// Side streams and events for up to kMaxStreams streams in all.
bool make_streams(cf_set *s) {
    const uint32_t nside = std::min<uint32_t>(uint32_t(s->classes.size()), kMaxStreams) - 1;
    if (nside == 0) return true;
    if (hipEventCreateWithFlags(&s->fork, hipEventDisableTiming) != hipSuccess) return false;
    for (uint32_t i = 0; i < nside; ++i) {
        hipStream_t t = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) return false;
        s->side.push_back(t);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
        s->join.push_back(e);
    }
    return true;
}

}  // namespace cfs

using cferr::fail;

extern "C" {

uint64_t cf_set_bytes(const cf_params *params, uint32_t nfilters, uint64_t max_batch) {
    if (!params || nfilters == 0 || nfilters > cfs::kMaxFilters) return 0;
    for (uint32_t i = 0; i < nfilters; ++i)
        if (cfs::validate_one(params[i], i) != CF_OK) return 0;
    const cfs::Layout L = cfs::layout_of(params, nfilters, max_batch);
    return cfs::fixed_bytes(L, nfilters) + L.tables;
}

cf_status cf_set_create(const cf_params *params, uint32_t nfilters, uint64_t max_batch,
                        uint32_t flags, cf_set **out) {
    if (!out) return fail(CF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || nfilters == 0 || nfilters > cfs::kMaxFilters)
        return fail(CF_EINVAL, "need 1..%u filters", cfs::kMaxFilters);
    if (max_batch == 0 || max_batch > (1ull << 31))
        return fail(CF_EINVAL, "max_batch must be in [1, 2^31]");
    if (flags & ~uint32_t(CF_SET_DEFER_TABLES)) return fail(CF_EINVAL, "unknown flags");
    for (uint32_t i = 0; i < nfilters; ++i) {
        cf_status st = cfs::validate_one(params[i], i);
        if (st != CF_OK) return st;
    }
    cf_set *s = new (std::nothrow) cf_set();
    if (!s) return fail(CF_ENOMEM, "host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(CF_EDEVICE, "no current HIP device");
    }
    s->nfilters = nfilters;
    s->max_batch = max_batch;
    s->params.assign(params, params + nfilters);
    s->layout = cfs::layout_of(params, nfilters, max_batch);
    s->tables.assign(nfilters, nullptr);
    s->single.resize(nfilters);
    std::vector<uint32_t> keys;
    s->cls_of.resize(nfilters);
    for (uint32_t i = 0; i < nfilters; ++i) {
        cfl::pick_launchers(params[i], s->single[i]);
        const uint32_t key = (params[i].fp_bits << 16) | (params[i].slots_per_bucket << 4) |
                             (params[i].placement << 2) | params[i].hash;
        auto it = std::find(keys.begin(), keys.end(), key);
        if (it == keys.end()) {
            if (keys.size() == cfs::kMaxClasses) {
                delete s;
                return fail(CF_EUNSUPPORTED,
                            "more than %u distinct (f, b, hash, placement) in one set",
                            cfs::kMaxClasses);
            }
            keys.push_back(key);
            cfs::ClassLaunch cl;
            cfs::pick(params[i].fp_bits, params[i].slots_per_bucket, params[i].hash,
                      params[i].placement, cl);
            s->classes.push_back(cl);
            it = keys.end() - 1;
        }
        s->cls_of[i] = uint32_t(it - keys.begin());
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) ==
            hipSuccess &&
        cus > 0)
        s->apply_grid = int(std::min<uint64_t>(uint64_t(cus) * 16, cfs::kApplyGrid));
    const cfs::Layout &L = s->layout;
    bool okall =
        hipMalloc(&s->d_filters, nfilters * sizeof(cfs::SetFilter)) == hipSuccess &&
        hipMalloc(&s->d_cls, nfilters) == hipSuccess &&
        hipMalloc(&s->d_ctr, nfilters * sizeof(cfk::Counters)) == hipSuccess &&
        hipMalloc(&s->d_lost_bucket, L.lost_entries * sizeof(unsigned long long)) == hipSuccess &&
        hipMalloc(&s->d_lost_tag, L.lost_entries * sizeof(uint32_t)) == hipSuccess &&
        hipMalloc(&s->d_totals, nfilters * sizeof(unsigned long long)) == hipSuccess &&
        hipMalloc(&s->sc.sorted, L.sorted_entries * 4) == hipSuccess &&
        hipMalloc(&s->sc.queue, L.queue_entries * 4) == hipSuccess &&
        hipMalloc(&s->sc.binoff, L.binoff_entries * 4) == hipSuccess;
    cf_status st = okall ? CF_OK : fail(CF_ENOMEM, "cannot allocate the set's fixed part");
    if (st == CF_OK && !cfs::make_streams(s)) st = fail(CF_EDEVICE, "cannot create the set's streams");
    if (st == CF_OK) {
        s->hdesc.resize(nfilters);
        for (uint32_t i = 0; i < nfilters; ++i) {
            const cf_params &p = params[i];
            cfs::SetFilter &h = s->hdesc[i];
            h.table = nullptr;
            h.ctr = s->d_ctr + i;
            h.lost_bucket = s->d_lost_bucket + L.lost_off[i];
            h.lost_tag = s->d_lost_tag + L.lost_off[i];
            h.lost_cap = p.lost_capacity ? p.lost_capacity : cfs::kDefaultSetLost;
            h.seed = p.seed;
            h.place = cfl::make_place(p);
            h.max_evict = p.max_evict;
            h.evict = p.evict;
            h.cls = s->cls_of[i];
        }
        if (hipMemset(s->d_ctr, 0, nfilters * sizeof(cfk::Counters)) != hipSuccess)
            st = fail(CF_EDEVICE, "clearing counters failed");
        for (uint32_t i = 0; st == CF_OK && !(flags & CF_SET_DEFER_TABLES) && i < nfilters; ++i)
            st = cfs::attach_table(s, i);
        std::vector<uint8_t> hc(nfilters);
        for (uint32_t i = 0; i < nfilters; ++i)
            hc[i] = s->tables[i] ? uint8_t(s->cls_of[i]) : uint8_t(0xFF);
        if (st == CF_OK &&
            (hipMemcpy(s->d_filters, s->hdesc.data(), nfilters * sizeof(cfs::SetFilter),
                       hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(s->d_cls, hc.data(), nfilters, hipMemcpyHostToDevice) != hipSuccess ||
             hipDeviceSynchronize() != hipSuccess))
            st = fail(CF_EDEVICE, "uploading filter descriptors failed");
    }
    if (st != CF_OK) {
        (void)hipGetLastError();
        cfs::free_all(s);
        delete s;
        return st;
    }
    *out = s;
    return CF_OK;
}

cf_status cf_set_destroy(cf_set *s) {
    if (!s) return CF_OK;
    cfs::DeviceGuard g(s->device);
    (void)hipDeviceSynchronize();
    cfs::free_all(s);
    delete s;
    return CF_OK;
}

cf_status cf_set_attach(cf_set *s, uint32_t fid) {
    if (!s || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    cfs::DeviceGuard g(s->device);
    if (s->tables[fid]) return CF_OK;
    if (hipDeviceSynchronize() != hipSuccess) return fail(CF_EDEVICE, "synchronise failed");
    cf_status st = cfs::attach_table(s, fid);
    if (st != CF_OK) return st;
    if (!cfs::upload(s, fid)) return fail(CF_EDEVICE, "descriptor upload failed");
    return CF_OK;
}

cf_status cf_set_detach(cf_set *s, uint32_t fid) {
    if (!s || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    cfs::DeviceGuard g(s->device);
    if (!s->tables[fid]) return CF_OK;
    if (hipDeviceSynchronize() != hipSuccess) return fail(CF_EDEVICE, "synchronise failed");
    (void)hipFree(s->tables[fid]);
    s->tables[fid] = nullptr;
    s->hdesc[fid].table = nullptr;
    if (!cfs::upload(s, fid)) return fail(CF_EDEVICE, "descriptor upload failed");
    return CF_OK;
}

cf_status cf_set_attached(const cf_set *s, uint32_t fid, int *out) {
    if (!s || !out || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    *out = s->tables[fid] ? 1 : 0;
    return CF_OK;
}

cf_status cf_set_execute(cf_set *s, const uint8_t *ops, const uint32_t *fids, const uint64_t *keys,
                         uint64_t n, uint8_t *results, void *stream) {
    if (!s) return fail(CF_EINVAL, "set is NULL");
    if (n == 0) return CF_OK;
    if (n > s->max_batch)
        return fail(CF_EINVAL, "batch of %llu exceeds max_batch %llu", (unsigned long long)n,
                    (unsigned long long)s->max_batch);
    if (!ops || !fids || !keys || !results) return fail(CF_EINVAL, "NULL batch buffer");
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return fail(CF_EINVAL, "keys not 8-byte aligned");
    cfs::DeviceGuard g(s->device);
    const cfs::Batch bt{ops, fids, keys, results, n, nullptr, s->max_batch};
    return cfs::enqueue(s, bt, cfs::grid_of(s, n), static_cast<hipStream_t>(stream));
}

cf_status cf_set_apply(cf_set *s, uint32_t fid, uint32_t op, const uint64_t *keys, uint64_t n,
                       uint8_t *results, void *stream) {
    if (!s || fid >= s->nfilters || op > CF_OP_INSERT) return fail(CF_EINVAL, "bad argument");
    if (n == 0) return CF_OK;
    if (n > s->max_batch) return fail(CF_EINVAL, "n exceeds max_batch");
    if (!keys || !results) return fail(CF_EINVAL, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return fail(CF_EINVAL, "keys not 8-byte aligned");
    if (!s->tables[fid]) return fail(CF_EINVAL, "filter %u is detached", fid);
    cfs::DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const cfl::Launchers &L = s->single[fid];
    const cfs::SetFilter &h = s->hdesc[fid];
    const uint64_t want = (n + cfk::kBlock - 1) / cfk::kBlock;
    const int grid = int(want < uint64_t(s->apply_grid) ? want : uint64_t(s->apply_grid));
    if (op == CF_OP_QUERY) {
        L.query(h.table, h.place, keys, n, results, grid, st);
    } else if (op == CF_OP_DELETE) {
        L.del(h.table, h.place, keys, n, results, h.ctr, grid, st);
    } else {
        const uint64_t seg = cfl::insert_segment(n, grid);
        const cfk::LostLog log{h.lost_bucket, h.lost_tag, h.lost_cap};
        L.ins(h.table, h.place, keys, n, results, nullptr, h.ctr, s->sc.queue, seg, log,
              h.max_evict, h.seed, grid, st);
    }
    return cfs::check_launch("set apply");
}

cf_status cf_set_graph_create(cf_set *s, const uint8_t *ops, const uint32_t *fids,
                              const uint64_t *keys, const uint64_t *d_n, uint8_t *results,
                              cf_graph **out) {
    if (!s || !out || !ops || !fids || !keys || !d_n || !results)
        return fail(CF_EINVAL, "NULL argument");
    *out = nullptr;
    cfs::DeviceGuard g(s->device);
    cf_graph *gr = new (std::nothrow) cf_graph();
    if (!gr) return fail(CF_ENOMEM, "host allocation failed");
    gr->device = s->device;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        delete gr;
        return fail(CF_EDEVICE, "stream creation failed");
    }
    const cfs::Batch bt{ops, fids, keys, results, 0, d_n, s->max_batch};
    cf_status r = CF_OK;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        r = fail(CF_EDEVICE, "begin capture failed");
    } else {
        r = cfs::enqueue(s, bt, cfs::grid_of(s, s->max_batch), st);
        const hipError_t e = hipStreamEndCapture(st, &gr->graph);
        if (r == CF_OK && e != hipSuccess)
            r = fail(CF_EDEVICE, "end capture: %s", hipGetErrorString(e));
        if (r == CF_OK && hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) !=
                              hipSuccess)
            r = fail(CF_EDEVICE, "graph instantiation failed");
    }
    (void)hipStreamDestroy(st);
    if (r != CF_OK) {
        cf_graph_destroy(gr);
        return r;
    }
    *out = gr;
    return CF_OK;
}

cf_status cf_graph_launch(cf_graph *gr, void *stream) {
    if (!gr || !gr->exec) return fail(CF_EINVAL, "graph is NULL");
    cfs::DeviceGuard g(gr->device);
    const hipError_t e = hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(CF_EDEVICE, "graph launch: %s", hipGetErrorString(e));
    return CF_OK;
}

cf_status cf_graph_destroy(cf_graph *gr) {
    if (!gr) return CF_OK;
    cfs::DeviceGuard g(gr->device);
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return CF_OK;
}

static cf_status totals(cf_set *s, uint64_t *out, void *stream, int which) {
    if (!s || !out) return fail(CF_EINVAL, "NULL argument");
    cfs::DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    cfs::set_totals_kernel<<<(s->nfilters + 255) / 256, 256, 0, st>>>(s->d_filters, s->nfilters,
                                                                      s->d_totals, which);
    cf_status r = cfs::check_launch("set totals");
    if (r != CF_OK) return r;
    if (hipMemcpyAsync(out, s->d_totals, s->nfilters * sizeof(uint64_t), hipMemcpyDefault, st) !=
        hipSuccess)
        return fail(CF_EDEVICE, "totals copy failed");
    return CF_OK;
}

cf_status cf_set_counts(cf_set *s, uint64_t *out, void *stream) { return totals(s, out, stream, 0); }

cf_status cf_set_failures(cf_set *s, uint64_t *out, void *stream) {
    return totals(s, out, stream, 1);
}

cf_status cf_set_export(cf_set *s, uint32_t fid, void *dst, uint64_t nbytes, void *stream) {
    if (!s || !dst || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    if (nbytes != cfs::tbytes(s->params[fid])) return fail(CF_EINVAL, "nbytes != table bytes");
    if (!s->tables[fid]) return fail(CF_EINVAL, "filter %u is detached", fid);
    cfs::DeviceGuard g(s->device);
    if (hipMemcpyAsync(dst, s->tables[fid], nbytes, hipMemcpyDefault,
                       static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(CF_EDEVICE, "export copy failed");
    return CF_OK;
}

cf_status cf_set_import(cf_set *s, uint32_t fid, const void *src, uint64_t nbytes, void *stream) {
    if (!s || !src || fid >= s->nfilters) return fail(CF_EINVAL, "bad argument");
    if (nbytes != cfs::tbytes(s->params[fid])) return fail(CF_EINVAL, "nbytes != table bytes");
    if (!s->tables[fid]) return fail(CF_EINVAL, "filter %u is detached", fid);
    cfs::DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *table = s->tables[fid];
    if (hipMemcpyAsync(table, src, nbytes, hipMemcpyDefault, st) != hipSuccess)
        return fail(CF_EDEVICE, "import copy failed");
    cfk::clear_counters_kernel<<<1, 64, 0, st>>>(s->d_ctr + fid);
    cf_status r = cfs::check_launch("set import (clear)");
    if (r != CF_OK) return r;
    const cfs::ClassLaunch &cl = s->classes[s->cls_of[fid]];
    const uint64_t nw = s->params[fid].num_buckets * cl.words_per_bucket;
    const uint64_t want = (nw + cfk::kBlock - 1) / cfk::kBlock;
    cl.recount(table, nw, s->d_ctr + fid, int(want < 4096 ? (want ? want : 1) : 4096), st);
    return cfs::check_launch("set import (recount)");
}

cf_status cf_set_lost(cf_set *s, uint32_t fid, uint64_t *buckets, uint32_t *tags, uint64_t cap,
                      uint64_t *n_out) {
    if (!s || !n_out || fid >= s->nfilters || (cap && (!buckets || !tags)))
        return fail(CF_EINVAL, "bad argument");
    cfs::DeviceGuard g(s->device);
    if (hipDeviceSynchronize() != hipSuccess) return fail(CF_EDEVICE, "synchronise failed");
    unsigned long long total = 0;
    if (hipMemcpy(&total, &s->d_ctr[fid].failures, sizeof(total), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return fail(CF_EDEVICE, "failure count copy failed");
    const uint64_t lcap =
        s->params[fid].lost_capacity ? s->params[fid].lost_capacity : cfs::kDefaultSetLost;
    uint64_t n = total < lcap ? total : lcap;
    if (n > cap) n = cap;
    const uint64_t off = s->layout.lost_off[fid];
    if (n && (hipMemcpy(buckets, s->d_lost_bucket + off, n * 8, hipMemcpyDeviceToHost) !=
                  hipSuccess ||
              hipMemcpy(tags, s->d_lost_tag + off, n * 4, hipMemcpyDeviceToHost) != hipSuccess))
        return fail(CF_EDEVICE, "lost log copy failed");
    *n_out = n;
    return CF_OK;
}

cf_status cf_set_get_shape(const cf_set *s, cf_set_shape *out) {
    if (!s || !out) return fail(CF_EINVAL, "NULL argument");
    *out = cf_set_shape{s->chunk, s->streams, {0, 0}};
    return CF_OK;
}

cf_status cf_set_set_shape(cf_set *s, const cf_set_shape *shape) {
    if (!s || !shape) return fail(CF_EINVAL, "NULL argument");
    const uint32_t c = shape->chunk ? shape->chunk : cfs::kDefaultChunk;
    if (c < cfs::kMinChunk || c > cfs::kMaxChunk || (c % 64))
        return fail(CF_EINVAL, "chunk must be a multiple of 64 in [64, 4096]");
    if (shape->streams > cfs::kMaxStreams) return fail(CF_EINVAL, "streams must be in [0, 8]");
    if (shape->reserved[0] || shape->reserved[1]) return fail(CF_EINVAL, "reserved must be 0");
    s->chunk = c;
    s->streams = shape->streams;
    return CF_OK;
}

}  // extern "C"
