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
#include <map>
#include <mutex>
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
#include "cf_set_persist.hpp"
namespace cfs {

// ------------------------------------------------------------- partition

__global__ __launch_bounds__(kBlock) void partition_kernel(Batch bt, const uint8_t *__restrict__ cls,
                                                           uint32_t nfilters, uint32_t ncls,
                                                           uint32_t chunk, Scratch sc) {
    __shared__ uint32_t hist[kMaxBins + 1];
    __shared__ uint32_t base[kMaxBins + 1];
    partition_chunk<kBlock>(bt, batch_n(bt), cls, nfilters, ncls, chunk, blockIdx.x, sc, hist,
                            base);
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

// A table's share of the set's arena: its bytes rounded up to 256.
uint64_t arena_span(const cf_params &p) { return (tbytes(p) + 255) & ~uint64_t(255); }

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
        L.tables += arena_span(params[i]);
        L.lost_off[i] = L.lost_entries;
        L.lost_entries += params[i].lost_capacity ? params[i].lost_capacity : kDefaultSetLost;
    }
    L.sorted_entries = max_batch + kMaxChunk;
    L.queue_entries = max_batch + kApplyGrid * kBlock;
    L.binoff_entries = ((max_batch + kMinChunk - 1) / kMinChunk + 1) * (kMaxBins + 1);
    return L;
}

uint64_t fixed_bytes(const Layout &L, uint32_t nf) {
    return sizeof(PersistCtl) + uint64_t(nf) * (sizeof(Counters) + sizeof(SetFilter) + 1 + 8) +
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
    // A set created with its tables holds them all in one allocation, the
    // arena (filter i at arena_off[i]); a detached filter's place is kept
    // for its next attach.  Without an arena each table is its own.
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    std::vector<uint64_t> arena_off;
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
    // persistent form (cf_set_persist.hpp)
    bool persist_ok = false;        // all filters share f, hash and placement
    cfs::PersistLaunch persist;
    cfs::ClassB class_b{};
    int persist_fit[2] = {0, 0};    // resident blocks per CU, per block size
    int cus = 0;
    uint64_t barrier_ticks = 0;     // bound on a barrier wait, wall-clock ticks
    cfs::PersistCtl *d_ctl = nullptr;
    uint32_t persistent = 0, pblock = 256, pblocks_per_cu = 0;
    uint32_t wave_bfs = 0;  // breadth-first search one wave per key
    // one launch per phase over every class (cf_set_persist.hpp); available
    // exactly when the persistent form is
    cfs::PhaseLaunch phase;
    uint32_t fused = 0;
    std::vector<cfs::Scratch> lanes;  // scratch lanes 1.. (lane 0 is sc)
};

uint32_t cfs::filter_count(const cf_set *s) { return s ? s->nfilters : 0; }



namespace cfs {
// The persistent kernel's arguments, kept alive with a graph that launches it.
struct PersistArgs {
    Batch b;
    const SetFilter *filters;
    const uint8_t *cls;
    ClassB cb;
    uint32_t nfilters, ncls, chunk;
    Scratch sc;
    PersistCtl *ctl;
    uint64_t limit;
    uint32_t wave_bfs;
    void *ptrs[11];
};
}  // namespace cfs

struct cf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    cfs::PersistArgs *pargs = nullptr;  // persistent form only
};

namespace cfs {

int grid_of(const cf_set *s, uint64_t n) { return int((n + s->chunk - 1) / s->chunk); }

uint32_t streams_of(const cf_set *s) {
    const uint32_t ncls = uint32_t(s->classes.size());
    const uint32_t want = s->streams ? s->streams : kDefaultStreams;
    const uint32_t l = std::min(want, ncls);
    return std::min<uint32_t>(l, uint32_t(s->side.size()) + 1);
}

// The persistent form's launch configuration: the kernel for the shape's
// block size, and the grid (blocks per compute unit x compute units).
struct PersistCfg {
    const void *kern;
    int block;
    int grid;
};

PersistCfg persist_cfg(const cf_set *s) {
    const int k = s->pblock == 512 ? 1 : 0;
    // set_shape stored the measured count when the shape asked for "as many
    // as fit" (0)
    return PersistCfg{s->persist.kern[k], kPersistBlocks[k], int(s->pblocks_per_cu) * s->cus};
}

// One cooperative launch for the whole batch (cf_set_persist.hpp).
cf_status enqueue_persistent(cf_set *s, const Batch &bt, hipStream_t st) {
    const PersistCfg pc = persist_cfg(s);
    Batch b = bt;
    const SetFilter *filters = s->d_filters;
    const uint8_t *cls = s->d_cls;
    ClassB cb = s->class_b;
    uint32_t nfilters = s->nfilters, ncls = uint32_t(s->classes.size()), chunk = s->chunk;
    Scratch sc = s->sc;
    PersistCtl *ctl = s->d_ctl;
    uint64_t limit = s->barrier_ticks;
    uint32_t wave_bfs = s->wave_bfs;
    void *args[] = {&b, &filters, &cls, &cb, &nfilters, &ncls, &chunk, &sc, &ctl, &limit,
                    &wave_bfs};
    const hipError_t e = hipLaunchCooperativeKernel(pc.kern, dim3(pc.grid), dim3(pc.block), args,
                                                    0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_EDEVICE, "set: persistent launch of %d x %d: %s", pc.grid, pc.block,
                    hipGetErrorString(e));
    }
    return CF_OK;
}

// Partition, then per class its query, delete and insert launches in that
// order.  The phase order only binds operations on one filter and every
// filter belongs to exactly one class, so chains of different classes may
// overlap: with L streams, class c runs on stream c mod L, stream 0 being
// the caller's and the others side streams that wait for the partition
// and are waited for at the end.  Concurrent insert launches keep apart in
// the eviction queue because each uses the slice of its own bin.
// The class-kernel form on scratch `sc`, with at most max_streams streams.
cf_status enqueue_classes(cf_set *s, const Batch &bt, int grid, hipStream_t st, const Scratch &sc,
                          uint32_t max_streams) {
    const uint32_t ncls = uint32_t(s->classes.size());
    const uint32_t nb = 3 * ncls;
    partition_kernel<<<grid, kBlock, 0, st>>>(bt, s->d_cls, s->nfilters, ncls, s->chunk, sc);
    cf_status r = check_launch("set partition");
    if (r != CF_OK) return r;
    uint32_t L = std::min(streams_of(s), max_streams);
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
        k.query(bt, s->d_filters, s->chunk, nb, c, sc, grid, cs);
        if ((r = check_launch("set query")) != CF_OK) break;
        k.del(bt, s->d_filters, s->nfilters, s->chunk, nb, ncls + c, sc, grid, cs);
        if ((r = check_launch("set delete")) != CF_OK) break;
        k.ins(bt, s->d_filters, s->nfilters, s->chunk, nb, 2 * ncls + c, sc, s->wave_bfs, grid,
              cs);
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

// Blocks per compute unit that are resident at once, measured: the
// occupancy the runtime reports from the kernel's resources can exceed what
// the device places together (measured for the 8-bit-fingerprint kernel at
// 256 threads: 7 reported, 6 resident).  An empty persistent batch (barriers
// only, each wait bounded by 50 ms) runs with the reported count and then
// one fewer at a time until its barriers complete.  Kept per kernel for the
// process.  0 if none completes.
int verified_fit(cf_set *s, int k) {
    static std::mutex mu;
    static std::map<const void *, int> known;
    const void *kern = s->persist.kern[k];
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find(kern);
        if (it != known.end()) return it->second;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    int fit = 0;
    for (int per = s->persist_fit[k]; per >= 1 && fit == 0; --per) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemset(s->d_ctl, 0, sizeof(PersistCtl)) != hipSuccess)
            break;
        Batch b{nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0};
        const SetFilter *filters = s->d_filters;
        const uint8_t *cls = s->d_cls;
        ClassB cb = s->class_b;
        uint32_t nfilters = s->nfilters, ncls = uint32_t(s->classes.size()), chunk = kMinChunk;
        Scratch sc = s->sc;
        PersistCtl *ctl = s->d_ctl;
        uint64_t limit = uint64_t(khz) * 50;  // 50 ms
        uint32_t wave_bfs = 0;
        void *args[] = {&b, &filters, &cls, &cb, &nfilters, &ncls, &chunk, &sc, &ctl, &limit,
                        &wave_bfs};
        unsigned int err = 1;
        if (hipLaunchCooperativeKernel(kern, dim3(per * s->cus), dim3(kPersistBlocks[k]), args, 0,
                                       nullptr) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(&err, &s->d_ctl->error.v, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            err = 1;
        }
        if (err == 0) fit = per;
    }
    (void)hipMemset(s->d_ctl, 0, sizeof(PersistCtl));
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(mu);
    known[kern] = fit;
    return fit;
}

// The phase form on scratch `sc`: the partition, then one launch per phase
// covering every class (grid x classes blocks), all on `st`.
cf_status enqueue_phases(cf_set *s, const Batch &bt, int grid, hipStream_t st, const Scratch &sc) {
    const uint32_t ncls = uint32_t(s->classes.size());
    partition_kernel<<<grid, kBlock, 0, st>>>(bt, s->d_cls, s->nfilters, ncls, s->chunk, sc);
    cf_status r = check_launch("set partition");
    if (r != CF_OK) return r;
    const int pgrid = grid * int(ncls);
    s->phase.query(bt, s->d_filters, s->class_b, ncls, s->chunk, sc, pgrid, st);
    if ((r = check_launch("set query phase")) != CF_OK) return r;
    s->phase.del(bt, s->d_filters, s->class_b, s->nfilters, ncls, s->chunk, sc, pgrid, st);
    if ((r = check_launch("set delete phase")) != CF_OK) return r;
    s->phase.ins(bt, s->d_filters, s->class_b, s->nfilters, ncls, s->chunk, sc, s->wave_bfs,
                 pgrid, st);
    return check_launch("set insert phase");
}

// A batch in the set's current shape, on the set's own scratch.
cf_status enqueue(cf_set *s, const Batch &bt, int grid, hipStream_t st) {
    if (s->persistent) return enqueue_persistent(s, bt, st);
    if (s->fused) return enqueue_phases(s, bt, grid, st, s->sc);
    return enqueue_classes(s, bt, grid, st, s->sc, kMaxStreams);
}

// The persistent form's graph: one kernel node, marked cooperative (a
// captured cooperative launch), with its arguments owned by the graph.
cf_status persist_graph(cf_set *s, const Batch &bt, cf_graph *gr) {
    const PersistCfg pc = persist_cfg(s);
    PersistArgs *a = new (std::nothrow) PersistArgs{bt,
                                                    s->d_filters,
                                                    s->d_cls,
                                                    s->class_b,
                                                    s->nfilters,
                                                    uint32_t(s->classes.size()),
                                                    s->chunk,
                                                    s->sc,
                                                    s->d_ctl,
                                                    s->barrier_ticks,
                                                    s->wave_bfs,
                                                    {}};
    if (!a) return fail(CF_ENOMEM, "host allocation failed");
    gr->pargs = a;
    void *ptrs[11] = {&a->b,     &a->filters, &a->cls, &a->cb,    &a->nfilters, &a->ncls,
                      &a->chunk, &a->sc,      &a->ctl, &a->limit, &a->wave_bfs};
    std::copy(ptrs, ptrs + 11, a->ptrs);
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(pc.kern);
    kp.gridDim = dim3(pc.grid);
    kp.blockDim = dim3(pc.block);
    kp.sharedMemBytes = 0;
    kp.kernelParams = a->ptrs;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    hipKernelNodeAttrValue coop{};
    coop.cooperative = 1;
    hipError_t e = hipGraphCreate(&gr->graph, 0);
    if (e == hipSuccess) e = hipGraphAddKernelNode(&node, gr->graph, nullptr, 0, &kp);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_EDEVICE, "set: persistent graph node: %s", hipGetErrorString(e));
    }
    e = hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &coop);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_EUNSUPPORTED, "set: cooperative graph node refused: %s",
                    hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_EDEVICE, "set: persistent graph instantiation: %s", hipGetErrorString(e));
    }
    return CF_OK;
}

// Upload filter fid's descriptor and class entry (synchronous copies).
bool upload(cf_set *s, uint32_t fid) {
    const uint8_t c = s->tables[fid] ? uint8_t(s->cls_of[fid]) : uint8_t(0xFF);
    return hipMemcpy(s->d_filters + fid, &s->hdesc[fid], sizeof(SetFilter),
                     hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->d_cls + fid, &c, 1, hipMemcpyHostToDevice) == hipSuccess;
}

bool in_arena(const cf_set *s, const void *t) {
    const char *c = static_cast<const char *>(t);
    return s->arena && c >= s->arena && c < s->arena + s->arena_bytes;
}

cf_status attach_table(cf_set *s, uint32_t fid) {
    if (s->tables[fid]) return CF_OK;
    const uint64_t nb = tbytes(s->params[fid]);
    void *t = nullptr;
    if (s->arena) {
        t = s->arena + s->arena_off[fid];
    } else if (hipMalloc(&t, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CF_ENOMEM, "filter %u: cannot allocate a %llu-byte table", fid,
                    (unsigned long long)nb);
    }
    if (hipMemset(t, 0, nb) != hipSuccess ||
        hipMemset(s->d_ctr + fid, 0, sizeof(Counters)) != hipSuccess) {
        if (!in_arena(s, t)) (void)hipFree(t);
        return fail(CF_EDEVICE, "filter %u: clearing the table failed", fid);
    }
    s->tables[fid] = t;
    s->hdesc[fid].table = t;
    return CF_OK;
}

void free_all(cf_set *s) {
    for (void *&t : s->tables)
        if (t) {
            if (!in_arena(s, t)) (void)hipFree(t);
            t = nullptr;
        }
    if (s->arena) (void)hipFree(s->arena);
    s->arena = nullptr;
    s->arena_bytes = 0;
    void *ptrs[] = {s->d_filters,   s->d_cls,      s->d_ctr,    s->d_lost_bucket,
                    s->d_lost_tag,  s->d_totals,   s->sc.sorted, s->sc.queue,
                    s->sc.binoff,   s->d_ctl};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (const Scratch &l : s->lanes) {
        if (l.sorted) (void)hipFree(l.sorted);
        if (l.queue) (void)hipFree(l.queue);
        if (l.binoff) (void)hipFree(l.binoff);
    }
    s->lanes.clear();
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

uint32_t cfs::lane_count(const cf_set *s) { return s ? 1 + uint32_t(s->lanes.size()) : 0; }

cf_status cfs::reserve_lanes(cf_set *s, uint32_t n) {
    if (!s || n == 0 || n > 64) return cferr::fail(CF_EINVAL, "lanes must be in [1, 64]");
    DeviceGuard g(s->device);
    while (lane_count(s) < n) {
        Scratch l{};
        const Layout &L = s->layout;
        const bool ok = hipMalloc(&l.sorted, L.sorted_entries * 4) == hipSuccess &&
                        hipMalloc(&l.queue, L.queue_entries * 4) == hipSuccess &&
                        hipMalloc(&l.binoff, L.binoff_entries * 4) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            if (l.sorted) (void)hipFree(l.sorted);
            if (l.queue) (void)hipFree(l.queue);
            if (l.binoff) (void)hipFree(l.binoff);
            return cferr::fail(CF_ENOMEM, "cannot allocate a scratch lane");
        }
        s->lanes.push_back(l);
    }
    return CF_OK;
}

static const cfs::Scratch &lane_of(const cf_set *s, uint32_t lane) {
    return lane == 0 ? s->sc : s->lanes[lane - 1];
}

cf_status cfs::execute_lane(cf_set *s, uint32_t lane, const uint8_t *ops, const uint32_t *fids,
                            const uint64_t *keys, uint64_t n, uint8_t *results, hipStream_t st) {
    if (!s || lane >= lane_count(s)) return cferr::fail(CF_EINVAL, "bad set or lane");
    if (n == 0) return CF_OK;
    if (n > s->max_batch)
        return cferr::fail(CF_EINVAL, "batch of %llu exceeds max_batch %llu",
                           (unsigned long long)n, (unsigned long long)s->max_batch);
    if (!ops || !fids || !keys || !results) return cferr::fail(CF_EINVAL, "NULL batch buffer");
    if (reinterpret_cast<uintptr_t>(keys) & 7u)
        return cferr::fail(CF_EINVAL, "keys not 8-byte aligned");
    DeviceGuard g(s->device);
    const Batch bt{ops, fids, keys, results, n, nullptr, s->max_batch};
    if (s->fused) return enqueue_phases(s, bt, grid_of(s, n), st, lane_of(s, lane));
    return enqueue_classes(s, bt, grid_of(s, n), st, lane_of(s, lane), 1);
}

cf_status cfs::apply_lane(cf_set *s, uint32_t lane, uint32_t fid, uint32_t op,
                          const uint64_t *keys, uint64_t n, uint8_t *results, hipStream_t st) {
    using cferr::fail;
    if (!s || fid >= s->nfilters || op > CF_OP_INSERT || lane >= lane_count(s))
        return fail(CF_EINVAL, "bad argument");
    if (n == 0) return CF_OK;
    if (n > s->max_batch) return fail(CF_EINVAL, "n exceeds max_batch");
    if (!keys || !results) return fail(CF_EINVAL, "NULL buffer");
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return fail(CF_EINVAL, "keys not 8-byte aligned");
    if (!s->tables[fid]) return fail(CF_EINVAL, "filter %u is detached", fid);
    DeviceGuard g(s->device);
    const cfl::Launchers &L = s->single[fid];
    const SetFilter &h = s->hdesc[fid];
    const uint64_t want = (n + cfk::kBlock - 1) / cfk::kBlock;
    const int grid = int(want < uint64_t(s->apply_grid) ? want : uint64_t(s->apply_grid));
    if (op == CF_OP_QUERY) {
        L.query(h.table, h.place, keys, n, results, grid, st);
    } else if (op == CF_OP_DELETE) {
        L.del(h.table, h.place, keys, n, results, h.ctr, grid, st);
    } else {
        const uint64_t seg = cfl::insert_segment(n, grid);
        const cfk::LostLog log{h.lost_bucket, h.lost_tag, h.lost_cap};
        L.ins(h.table, h.place, keys, n, results, nullptr, h.ctr, lane_of(s, lane).queue, seg,
              log, h.max_evict, h.seed, grid, st);
    }
    return check_launch("set apply");
}

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
    s->cus = cus > 0 ? cus : 256;
    // The persistent form: every filter shares f, hash and placement; each
    // class then differs only in b.
    s->persist_ok = true;
    for (uint32_t i = 0; i < nfilters; ++i) {
        const cf_params &p = params[i], &q = params[0];
        if (p.fp_bits != q.fp_bits || p.hash != q.hash || p.placement != q.placement)
            s->persist_ok = false;
        s->class_b.b[s->cls_of[i]] = uint8_t(p.slots_per_bucket);
    }
    if (s->persist_ok) {
        const uint32_t f = params[0].fp_bits, h = params[0].hash, pl = params[0].placement;
        uint32_t bm = 0;  // the largest bucket of the set picks the kernels' b range
        for (uint32_t i = 0; i < nfilters; ++i) bm = std::max(bm, params[i].slots_per_bucket);
        s->persist_ok = f == 8    ? cfs::pick_persist_f8(h, pl, bm, s->persist) &&
                                     cfs::pick_phase_f8(h, pl, bm, s->phase) &&
                                     cfs::pick_phase_insert_f8(h, pl, bm, s->phase)
                        : f == 16 ? cfs::pick_persist_f16(h, pl, bm, s->persist) &&
                                     cfs::pick_phase_f16(h, pl, bm, s->phase) &&
                                     cfs::pick_phase_insert_f16(h, pl, bm, s->phase)
                                  : cfs::pick_persist_f32(h, pl, bm, s->persist) &&
                                     cfs::pick_phase_f32(h, pl, bm, s->phase) &&
                                     cfs::pick_phase_insert_f32(h, pl, bm, s->phase);
    }
    for (int k = 0; s->persist_ok && k < 2; ++k) {
        int fit = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, s->persist.kern[k],
                                                         cfs::kPersistBlocks[k], 0) != hipSuccess) {
            (void)hipGetLastError();
            fit = 0;
        }
        s->persist_fit[k] = fit;
    }
    {
        int khz = 0;  // the constant-rate wall clock of wall_clock64()
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) !=
                hipSuccess ||
            khz <= 0)
            khz = 100000;
        uint64_t us = 10000000;
        if (const char *env = getenv("CF_SET_BARRIER_US")) us = strtoull(env, nullptr, 10);
        s->barrier_ticks = us * uint64_t(khz) / 1000;
    }
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
        hipMalloc(&s->sc.binoff, L.binoff_entries * 4) == hipSuccess &&
        hipMalloc(&s->d_ctl, sizeof(cfs::PersistCtl)) == hipSuccess;
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
        if (hipMemset(s->d_ctr, 0, nfilters * sizeof(cfk::Counters)) != hipSuccess ||
            hipMemset(s->d_ctl, 0, sizeof(cfs::PersistCtl)) != hipSuccess)
            st = fail(CF_EDEVICE, "clearing counters failed");
        if (st == CF_OK && !(flags & CF_SET_DEFER_TABLES)) {
            // every table in one allocation: measured 2-5% faster per mixed
            // batch than one allocation per table (256 filters, 3.8 GiB)
            s->arena_off.resize(nfilters);
            uint64_t off = 0;
            for (uint32_t i = 0; i < nfilters; ++i) {
                s->arena_off[i] = off;
                off += cfs::arena_span(params[i]);
            }
            void *a = nullptr;
            if (hipMalloc(&a, off) == hipSuccess) {
                s->arena = static_cast<char *>(a);
                s->arena_bytes = off;
            } else {
                (void)hipGetLastError();  // no block that large: one allocation per table
            }
        }
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
    if (!cfs::in_arena(s, s->tables[fid])) (void)hipFree(s->tables[fid]);
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
    return cfs::apply_lane(s, 0, fid, op, keys, n, results, static_cast<hipStream_t>(stream));
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
    if (s->persistent) {
        (void)hipStreamDestroy(st);
        r = cfs::persist_graph(s, bt, gr);
        if (r != CF_OK) {
            cf_graph_destroy(gr);
            return r;
        }
        *out = gr;
        return CF_OK;
    }
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
    delete gr->pargs;
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
    *out = cf_set_shape{s->chunk, s->streams, s->persistent, s->pblock, s->pblocks_per_cu,
                        s->wave_bfs, s->fused};
    return CF_OK;
}

uint32_t cf_set_persistent_capacity(cf_set *s, uint32_t block) {
    if (!s || !s->persist_ok) return 0;
    const int k = (block == 0 || block == 256) ? 0 : (block == 512 ? 1 : -1);
    if (k < 0 || s->persist_fit[k] <= 0) return 0;
    cfs::DeviceGuard g(s->device);
    return uint32_t(cfs::verified_fit(s, k));
}

cf_status cf_set_status(cf_set *s, uint32_t *error_out) {
    if (!s || !error_out) return fail(CF_EINVAL, "NULL argument");
    cfs::DeviceGuard g(s->device);
    unsigned int e = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&e, &s->d_ctl->error.v, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CF_EDEVICE, "reading the persistent control block failed");
    *error_out = e;
    return CF_OK;
}

cf_status cf_set_phase_ticks(cf_set *s, uint64_t ticks[4], uint64_t *ticks_per_s) {
    if (!s || !ticks) return fail(CF_EINVAL, "NULL argument");
    if (!s->persist_ok) return fail(CF_EUNSUPPORTED, "the set cannot run the persistent form");
    cfs::DeviceGuard g(s->device);
    unsigned long long t[4] = {0, 0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(t, s->d_ctl->stamp.t, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(CF_EDEVICE, "reading the persistent control block failed");
    for (int k = 0; k < 4; ++k) ticks[k] = t[k];
    if (ticks_per_s) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess ||
            khz <= 0)
            khz = 100000;
        *ticks_per_s = uint64_t(khz) * 1000;
    }
    return CF_OK;
}

cf_status cf_set_set_shape(cf_set *s, const cf_set_shape *shape) {
    if (!s || !shape) return fail(CF_EINVAL, "NULL argument");
    const uint32_t c = shape->chunk ? shape->chunk : cfs::kDefaultChunk;
    if (c < cfs::kMinChunk || c > cfs::kMaxChunk || (c % 64))
        return fail(CF_EINVAL, "chunk must be a multiple of 64 in [64, 4096]");
    if (shape->streams > cfs::kMaxStreams) return fail(CF_EINVAL, "streams must be in [0, 8]");
    if (shape->wave_bfs > 1) return fail(CF_EINVAL, "wave_bfs must be 0 or 1");
    if (shape->persistent > 1) return fail(CF_EINVAL, "persistent must be 0 or 1");
    if (shape->fused > 1) return fail(CF_EINVAL, "fused must be 0 or 1");
    if (shape->fused && shape->persistent)
        return fail(CF_EINVAL, "fused applies to the class-kernel form (persistent = 0)");
    if (shape->fused && !s->persist_ok)
        return fail(CF_EUNSUPPORTED,
                    "one launch per phase needs every filter to share f, hash and placement");
    const uint32_t blk = shape->block ? shape->block : 256;
    if (blk != 256 && blk != 512) return fail(CF_EINVAL, "block must be 256 or 512");
    if (shape->persistent) {
        if (!s->persist_ok)
            return fail(CF_EUNSUPPORTED,
                        "the persistent form needs every filter to share f, hash and placement");
        const uint32_t fit = cf_set_persistent_capacity(s, blk);
        if (fit == 0) return fail(CF_EUNSUPPORTED, "no block of %u threads fits a compute unit", blk);
        if (shape->blocks_per_cu > fit)
            return fail(CF_EINVAL, "at most %u blocks of %u threads fit a compute unit", fit, blk);
    }
    cfs::DeviceGuard g(s->device);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemset(s->d_ctl, 0, sizeof(cfs::PersistCtl)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return fail(CF_EDEVICE, "clearing the persistent control block failed");
    s->chunk = c;
    s->streams = shape->streams;
    s->persistent = shape->persistent;
    s->pblock = blk;
    s->pblocks_per_cu = shape->blocks_per_cu;
    s->wave_bfs = shape->wave_bfs;
    s->fused = shape->fused;
    if (shape->persistent && shape->blocks_per_cu == 0)
        s->pblocks_per_cu = cf_set_persistent_capacity(s, blk);
    return CF_OK;
}

}  // extern "C"
