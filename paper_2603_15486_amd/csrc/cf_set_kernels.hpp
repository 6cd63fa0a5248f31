// cf_set_kernels.hpp -- device side of filter sets (include/cf_set.h):
// the descriptor of each filter, the batch and scratch layout, and the
// per-class query, delete and insert kernels with their host launchers.
// Included by cf_set.hip and by the cf_set_inst_f*.hip translation units,
// each of which instantiates one fingerprint width.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "cf.h"
#include "cf_kernels.hpp"

namespace cfs {

using cfk::Counters;
using cfk::Derived;
using cfk::kBlock;

constexpr uint32_t kMaxChunk = 4096;
constexpr uint32_t kMinChunk = 64;
constexpr uint32_t kDefaultChunk = 2048;
constexpr uint32_t kMaxClasses = 16;
constexpr uint32_t kMaxBins = 3 * kMaxClasses;
constexpr uint32_t kLdsFilters = 4096;  // per-filter count deltas in LDS up to this many
constexpr uint32_t kMaxFilters = 65536;
constexpr uint64_t kDefaultSetLost = 4096;
constexpr uint32_t kDefaultStreams = 4;  // class chains in flight by default
constexpr uint32_t kMaxStreams = 8;

struct SetFilter {
    void *table;
    Counters *ctr;
    unsigned long long *lost_bucket;
    uint32_t *lost_tag;
    unsigned long long lost_cap;
    uint64_t seed;
    cfk::Place place;
    uint32_t max_evict;
    uint32_t evict;
    uint32_t cls;
};

struct Batch {
    const uint8_t *ops;
    const uint32_t *fids;
    const uint64_t *keys;
    uint8_t *results;
    uint64_t n;
    const uint64_t *d_n;  // when set, the operation count is read from here,
    uint64_t cap;         // clamped to the set's max_batch
};

struct Scratch {
    uint32_t *sorted;  // per block: its chunk's operation indices grouped by bin
    uint32_t *binoff;  // per block: nbins + 1 bin starts within its chunk
    uint32_t *queue;   // per block: keys deferred to the eviction pass, each bin
                       // in the slice [b0, b1) of its own range
};

__device__ __forceinline__ uint64_t batch_n(const Batch &bt) {
    if (!bt.d_n) return bt.n;
    const uint64_t n = *bt.d_n;
    return n < bt.cap ? n : bt.cap;
}

// Range [b0, b1) of bin `bin` in this block's chunk.
__device__ __forceinline__ void bin_range(const Scratch &sc, uint32_t nb, uint32_t bin,
                                          uint32_t &b0, uint32_t &b1) {
    const uint32_t *off = sc.binoff + uint64_t(blockIdx.x) * (nb + 1);
    b0 = off[bin];
    b1 = off[bin + 1];
}

// Per-filter count deltas: LDS tally flushed once per block, or direct
// atomics for sets larger than the LDS table.
struct Tally {
    int *lds;
    uint32_t nfilters;
    __device__ __forceinline__ void init() {
        if (nfilters <= kLdsFilters)
            for (uint32_t f = threadIdx.x; f < nfilters; f += kBlock) lds[f] = 0;
        __syncthreads();
    }
    __device__ __forceinline__ void add(const SetFilter &F, uint32_t fid, int v) {
        if (nfilters <= kLdsFilters)
            atomicAdd(&lds[fid], v);
        else
            atomicAdd(&F.ctr->count[blockIdx.x % cfk::kStripes].v,
                      (unsigned long long)(long long)v);
    }
    __device__ __forceinline__ void flush(const SetFilter *filters) {
        __syncthreads();
        if (nfilters <= kLdsFilters)
            for (uint32_t f = threadIdx.x; f < nfilters; f += kBlock)
                if (lds[f])
                    atomicAdd(&filters[f].ctr->count[blockIdx.x % cfk::kStripes].v,
                              (unsigned long long)(long long)lds[f]);
    }
};

// ------------------------------------------------------------------ query

template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_query_kernel(Batch bt,
                                                           const SetFilter *__restrict__ filters,
                                                           uint32_t chunk, uint32_t nb,
                                                           uint32_t bin, Scratch sc) {
    using W = typename G::W;
    uint32_t b0, b1;
    bin_range(sc, nb, bin, b0, b1);
    const uint32_t *seg = sc.sorted + uint64_t(blockIdx.x) * chunk;
    for (uint32_t p = b0 + threadIdx.x; p < b1; p += kBlock) {
        const uint32_t i = seg[p];
        const SetFilter &F = filters[bt.fids[i]];
        const W *table = static_cast<const W *>(F.table);
        const Derived d = cfk::derive<G, HASH, POL>(bt.keys[i], F.place);
        cfk::Bucket<G> bk;
        cfk::load_bucket<G>(table, d.i1, bk);
        bool hit = bk.contains(d.t1);
        if (!hit) {
            cfk::load_bucket<G>(table, d.i2, bk);
            hit = bk.contains(d.t2);
        }
        bt.results[i] = uint8_t(hit);
    }
}

// ----------------------------------------------------------------- delete

template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_delete_kernel(Batch bt,
                                                            const SetFilter *__restrict__ filters,
                                                            uint32_t nfilters, uint32_t chunk,
                                                            uint32_t nb, uint32_t bin, Scratch sc) {
    using W = typename G::W;
    __shared__ int lds[kLdsFilters];
    Tally tally{lds, nfilters};
    tally.init();
    uint32_t b0, b1;
    bin_range(sc, nb, bin, b0, b1);
    const uint32_t *seg = sc.sorted + uint64_t(blockIdx.x) * chunk;
    for (uint32_t p = b0 + threadIdx.x; p < b1; p += kBlock) {
        const uint32_t i = seg[p];
        const uint32_t fid = bt.fids[i];
        const SetFilter &F = filters[fid];
        W *table = static_cast<W *>(F.table);
        const Derived d = cfk::derive<G, HASH, POL>(bt.keys[i], F.place);
        cfk::Bucket<G> bk;
        cfk::load_bucket<G>(table, d.i1, bk);
        bool done = cfk::try_remove<G>(table, d.i1, d.t1, bk);
        if (!done) {
            cfk::load_bucket<G>(table, d.i2, bk);
            done = cfk::try_remove<G>(table, d.i2, d.t2, bk);
        }
        if (done) tally.add(F, fid, -1);
        bt.results[i] = uint8_t(done);
    }
    tally.flush(filters);
}

// ----------------------------------------------------------------- insert

// Candidates whose other buckets the set's breadth-first search loads at
// once: as many as 128 bytes of buckets hold, at most b/2.  A set kernel
// has a few operations per thread, so a launch lasts as long as its longest
// eviction chain, and each level of the chain costs one dependent load per
// candidate group; the single-filter kernel, with many keys per thread and
// bound by memory throughput, probes one candidate at a time.
template <class G>
constexpr int probe_width() {
    constexpr int bytes = G::B * G::F / 8;
    constexpr int fit = bytes >= 128 ? 1 : 128 / bytes;
    return fit < G::B / 2 ? fit : G::B / 2;
}

// The single-filter insert_kernel's two passes, per operation on its own
// filter: direct attempts first, keys with two full buckets deferred to the
// block's queue segment and searched afterwards with the filter's policy.
template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_insert_kernel(Batch bt,
                                                            const SetFilter *__restrict__ filters,
                                                            uint32_t nfilters, uint32_t chunk,
                                                            uint32_t nb, uint32_t bin, Scratch sc) {
    using W = typename G::W;
    __shared__ int lds[kLdsFilters];
    __shared__ uint32_t s_qn;
    Tally tally{lds, nfilters};
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();  // s_qn = 0 before any wave adds to it
    tally.init();
    uint32_t b0, b1;
    bin_range(sc, nb, bin, b0, b1);
    const uint32_t *seg = sc.sorted + uint64_t(blockIdx.x) * chunk;
    uint32_t *myq = sc.queue + uint64_t(blockIdx.x) * chunk + b0;
    const uint32_t qcap = b1 - b0;  // the bin's slice of the queue
    const int lane = threadIdx.x & 63;
    // The loop bound is uniform across the block so the ballot below always
    // sees whole waves.
    for (uint32_t p0 = b0; p0 < b1; p0 += kBlock) {
        const uint32_t p = p0 + threadIdx.x;
        bool need_evict = false;
        if (p < b1) {
            const uint32_t i = seg[p];
            const uint32_t fid = bt.fids[i];
            const SetFilter &F = filters[fid];
            W *table = static_cast<W *>(F.table);
            const Derived d = cfk::derive<G, HASH, POL>(bt.keys[i], F.place);
            cfk::Bucket<G> bk;
            cfk::load_bucket<G>(table, d.i1, bk);
            bool done = cfk::try_insert<G>(table, d.i1, d.t1, bk) >= 0;
            if (!done) {
                cfk::load_bucket<G>(table, d.i2, bk);
                done = cfk::try_insert<G>(table, d.i2, d.t2, bk) >= 0;
            }
            if (done) {
                tally.add(F, fid, 1);
                bt.results[i] = 1;
            }
            need_evict = !done;
        }
        const uint64_t need = __ballot(need_evict);
        if (need) {
            const int leader = __builtin_ctzll(need);
            uint32_t qb = 0;
            if (lane == leader) qb = atomicAdd(&s_qn, uint32_t(__popcll(need)));
            qb = __shfl(qb, leader, 64);
            const uint32_t pos = qb + uint32_t(__popcll(need & ((1ull << lane) - 1ull)));
            if (need_evict && pos < qcap) myq[pos] = p;
        }
    }
    __syncthreads();
    const uint32_t qn = s_qn < qcap ? s_qn : qcap;
    for (uint32_t q = threadIdx.x; q < qn; q += kBlock) {
        const uint32_t i = seg[myq[q]];
        const uint32_t fid = bt.fids[i];
        const SetFilter &F = filters[fid];
        W *table = static_cast<W *>(F.table);
        const uint64_t key = bt.keys[i];
        const Derived d = cfk::derive<G, HASH, POL>(key, F.place);
        const uint64_t rs = key ^ F.seed;
        const bool second = (cfk::splitmix_at(rs, 0) & 1) != 0;
        const uint32_t cur = second ? d.i2 : d.i1;
        const uint32_t tag = second ? d.t2 : d.t1;
        uint32_t k = 0, lb = 0, lt = 0;
        const bool done =
            F.evict == CF_EVICT_DFS
                ? cfk::evict_dfs<G, HASH, POL>(table, F.place, rs, cur, tag, F.max_evict, k, lb, lt)
                : cfk::evict_bfs<G, HASH, POL, probe_width<G>()>(table, F.place, rs, cur, tag,
                                                                F.max_evict, k, lb, lt);
        if (done) {
            tally.add(F, fid, 1);
        } else {
            const unsigned long long slot = atomicAdd(&F.ctr->failures, 1ull);
            if (slot < F.lost_cap) {
                F.lost_bucket[slot] = lb;
                F.lost_tag[slot] = lt;
            }
        }
        bt.results[i] = uint8_t(done);
    }
    tally.flush(filters);
}

// ------------------------------------------------------ per-class launchers

struct ClassLaunch {
    void (*query)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, Scratch, int, hipStream_t);
    void (*del)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, uint32_t, Scratch, int,
                hipStream_t);
    void (*ins)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, uint32_t, Scratch, int,
                hipStream_t);
    void (*recount)(const void *table, uint64_t nwords, Counters *ctr, int grid, hipStream_t s);
    uint64_t words_per_bucket;
};

template <int F, int B, int HASH, int POL>
struct SetInstQD {
    using G = cfk::Geom<F, B>;
    static void query(Batch bt, const SetFilter *fl, uint32_t chunk, uint32_t nb, uint32_t bin,
                      Scratch sc, int grid, hipStream_t s) {
        set_query_kernel<G, HASH, POL><<<grid, kBlock, 0, s>>>(bt, fl, chunk, nb, bin, sc);
    }
    static void del(Batch bt, const SetFilter *fl, uint32_t nf, uint32_t chunk, uint32_t nb,
                    uint32_t bin, Scratch sc, int grid, hipStream_t s) {
        set_delete_kernel<G, HASH, POL><<<grid, kBlock, 0, s>>>(bt, fl, nf, chunk, nb, bin, sc);
    }
    static void recount(const void *t, uint64_t nw, Counters *c, int grid, hipStream_t s) {
        cfk::recount_kernel<G><<<grid, kBlock, 0, s>>>(static_cast<const typename G::W *>(t), nw, c);
    }
    static void fill(ClassLaunch &L) {
        L.query = &query;
        L.del = &del;
        L.recount = &recount;
        L.words_per_bucket = uint64_t(G::WPB);
    }
};

template <int F, int B, int HASH, int POL>
struct SetInstI {
    using G = cfk::Geom<F, B>;
    static void ins(Batch bt, const SetFilter *fl, uint32_t nf, uint32_t chunk, uint32_t nb,
                    uint32_t bin, Scratch sc, int grid, hipStream_t s) {
        set_insert_kernel<G, HASH, POL><<<grid, kBlock, 0, s>>>(bt, fl, nf, chunk, nb, bin, sc);
    }
    static void fill(ClassLaunch &L) { L.ins = &ins; }
};

// Fills the query/delete/recount part (INSERT = false) or the insert part
// (INSERT = true) of L; false if b is unsupported.
template <int F, bool INSERT>
bool pick_class_b(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &L) {
    auto one = [&](auto bconst) {
        constexpr int B = decltype(bconst)::value;
        const bool off = placement == CF_PLACE_OFFSET;
        if constexpr (INSERT) {
            if (hash == 0) off ? SetInstI<F, B, 0, 1>::fill(L) : SetInstI<F, B, 0, 0>::fill(L);
            else off ? SetInstI<F, B, 1, 1>::fill(L) : SetInstI<F, B, 1, 0>::fill(L);
        } else {
            if (hash == 0) off ? SetInstQD<F, B, 0, 1>::fill(L) : SetInstQD<F, B, 0, 0>::fill(L);
            else off ? SetInstQD<F, B, 1, 1>::fill(L) : SetInstQD<F, B, 1, 0>::fill(L);
        }
        return true;
    };
    switch (b) {
        case 4: return one(std::integral_constant<int, 4>{});
        case 8: return one(std::integral_constant<int, 8>{});
        case 16: return one(std::integral_constant<int, 16>{});
        case 32: return one(std::integral_constant<int, 32>{});
        default: return false;
    }
}

// Class launchers for 8-, 16- and 32-bit fingerprints: query, delete and
// recount (cf_set_inst_f*.hip) and insert (cf_set_insi_f*.hip, built at -O1).
bool pick_class_f8(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);
bool pick_class_f16(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);
bool pick_class_f32(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);
bool pick_class_insert_f8(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);
bool pick_class_insert_f16(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);
bool pick_class_insert_f32(uint32_t b, uint32_t hash, uint32_t placement, ClassLaunch &out);

}  // namespace cfs
