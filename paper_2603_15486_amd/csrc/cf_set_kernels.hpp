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

// Batch scratch, laid out per chunk of `chunk` operations (chunk c covers
// operations [c * chunk, (c + 1) * chunk)).
struct Scratch {
    uint32_t *sorted;  // per chunk: its operation indices grouped by bin
    uint32_t *binoff;  // per chunk: nbins + 1 bin starts within the chunk
    uint32_t *queue;   // per chunk: keys deferred to the eviction pass, each bin
                       // in the slice [b0, b1) of its own range
};

__device__ __forceinline__ uint64_t batch_n(const Batch &bt) {
    if (!bt.d_n) return bt.n;
    const uint64_t n = *bt.d_n;
    return n < bt.cap ? n : bt.cap;
}

// Sort chunk `cid` of the batch by bin = (kind, class) with a block of BT
// threads: count in LDS, store the bin starts at binoff[cid * (nb + 1) ..]
// and the operations' indices bin by bin at sorted[cid * chunk ..].  Invalid
// kinds and ids, and detached filters (class 0xFF), go to bin nb with result
// 0xFF.  No global atomics; each operation's kind and filter id are read
// twice (count, then place), its key never.  hist and base: LDS arrays of
// kMaxBins + 1 entries.
template <int BT>
__device__ __forceinline__ void partition_chunk(const Batch &bt, uint64_t n,
                                                const uint8_t *__restrict__ cls,
                                                uint32_t nfilters, uint32_t ncls, uint32_t chunk,
                                                uint64_t cid, const Scratch &sc, uint32_t *hist,
                                                uint32_t *base) {
    const uint32_t nb = 3 * ncls;  // bin nb collects invalid operations
    const uint64_t lo = cid * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    for (uint32_t j = threadIdx.x; j <= nb; j += BT) hist[j] = 0;
    __syncthreads();
    auto bin_of = [&](uint64_t i) -> uint32_t {
        const uint32_t op = bt.ops[i], fid = bt.fids[i];
        if (op > 2u || fid >= nfilters) return nb;
        const uint32_t c = cls[fid];
        return c < ncls ? op * ncls + c : nb;  // 0xFF: filter detached
    };
    for (uint64_t i = lo + threadIdx.x; i < hi; i += BT) atomicAdd(&hist[bin_of(i)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t j = 0; j <= nb; ++j) {
            base[j] = acc;
            acc += hist[j];
        }
    }
    __syncthreads();
    uint32_t *off = sc.binoff + cid * (nb + 1);
    for (uint32_t j = threadIdx.x; j <= nb; j += BT) {
        off[j] = base[j];
        hist[j] = base[j];  // becomes the scatter cursor
    }
    __syncthreads();
    uint32_t *seg = sc.sorted + lo;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += BT) {
        const uint32_t bin = bin_of(i);
        const uint32_t pos = atomicAdd(&hist[bin], 1u);
        seg[pos] = uint32_t(i);
        if (bin == nb) bt.results[i] = 0xFF;
    }
    __syncthreads();  // hist and base are free again
}

// Range [b0, b1) of bin `bin` in chunk `cid`.
__device__ __forceinline__ void bin_range(const Scratch &sc, uint32_t nb, uint64_t cid, uint32_t bin,
                                          uint32_t &b0, uint32_t &b1) {
    const uint32_t *off = sc.binoff + cid * (nb + 1);
    b0 = off[bin];
    b1 = off[bin + 1];
}

// Per-filter count deltas: LDS tally flushed once per block, or direct
// atomics for sets larger than the LDS table.  BT = threads per block.
template <int BT>
struct Tally {
    int *lds;
    uint32_t nfilters;
    __device__ __forceinline__ void init() {
        if (nfilters <= kLdsFilters)
            for (uint32_t f = threadIdx.x; f < nfilters; f += BT) lds[f] = 0;
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
            for (uint32_t f = threadIdx.x; f < nfilters; f += BT)
                if (lds[f])
                    atomicAdd(&filters[f].ctr->count[blockIdx.x % cfk::kStripes].v,
                              (unsigned long long)(long long)lds[f]);
    }
};

// The per-bin work of the three phases, for the operations seg[b0 .. b1) of
// one chunk (seg = the chunk's sorted operation indices), done by one block
// of BT threads.  The class kernels below run one bin per block; the
// persistent kernel (cf_set_persist.hpp) runs every bin of its chunks.

// Alg. 2: probe i1, and i2 only when i1 misses.
template <class G, int HASH, int POL, int BT>
__device__ __forceinline__ void query_bin(const Batch &bt, const SetFilter *__restrict__ filters,
                                          const uint32_t *seg, uint32_t b0, uint32_t b1) {
    using W = typename G::W;
    for (uint32_t p = b0 + threadIdx.x; p < b1; p += BT) {
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

// Alg. 3: remove one copy from i1, else from i2.
template <class G, int HASH, int POL, int BT>
__device__ __forceinline__ void delete_bin(const Batch &bt, const SetFilter *__restrict__ filters,
                                           const uint32_t *seg, uint32_t b0, uint32_t b1,
                                           Tally<BT> &tally) {
    using W = typename G::W;
    for (uint32_t p = b0 + threadIdx.x; p < b1; p += BT) {
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
}

// The set's breadth-first search loads each level's candidates' other
// buckets together (cfk::probe_width): a set kernel has a few operations per
// thread, so a launch lasts as long as its longest eviction chain, and each
// level of the chain costs one dependent load per candidate group.
using cfk::probe_width;

// Sec. 4.6.1's breadth-first search for one key by a whole wave (wave64):
// at each level lane j < b/2 probes candidate j's other bucket, a ballot
// picks the lowest candidate whose other bucket has an empty slot, and that
// lane moves it (the displacement-first move of cfk::evict_bfs); failing
// that, lane 0 displaces the last candidate and carries it.  The choice is
// the one the candidate-by-candidate search makes on an unchanged table, so
// one key per launch reproduces the oracle.  A level costs one dependent
// probe however many candidates there are.  Every lane of the wave calls it
// with the same arguments and gets the same result.
template <class G, int HASH, int POL>
__device__ bool evict_bfs_wave(typename G::W *table, const cfk::Place &pl, uint64_t rs,
                               uint32_t cur, uint32_t tag, uint32_t max_evict, uint32_t &kicks,
                               uint32_t &lost_bucket, uint32_t &lost_tag) {
    constexpr int HALF = G::B / 2;
    const int lane = threadIdx.x & 63;
    for (uint32_t n = 1; n <= max_evict; ++n) {
        cfk::Bucket<G> cb;
        cfk::load_bucket<G>(table, cur, cb);
        if (cb.has_empty()) {  // the same words in every lane
            int ok = 0;
            if (lane == 0) ok = cfk::try_insert<G>(table, cur, tag, cb) >= 0;
            if (__shfl(ok, 0)) return true;
            cfk::load_bucket<G>(table, cur, cb);  // it filled meanwhile: fresh words everywhere
        }
        const int r0 = int(cfk::splitmix_at(rs, n) % uint64_t(G::B));
        bool fits = false;
        uint32_t c = 0, moved = 0, a = 0;
        cfk::Bucket<G> ab;
        if (lane < HALF) {
            c = cb.slot((r0 + lane) % G::B);
            moved = c;
            a = cfk::move_tag<G, HASH, POL>(cur, moved, pl);
            if (c != 0 && a != cur) {
                cfk::load_bucket<G>(table, a, ab);
                fits = ab.has_empty();
            }
        }
        uint64_t cand = __ballot(fits);
        int outcome = 0;  // 1: stored, 2: carried on from the candidate's bucket
        while (cand && outcome == 0) {
            const int j = __builtin_ctzll(cand);
            cand &= cand - 1;
            int res = 0;
            uint32_t ncur = 0, ntag = 0;
            if (lane == j && cfk::replace_slot_if<G>(table, cur, (r0 + j) % G::B, c, tag, cb)) {
                if (cfk::try_insert<G>(table, a, moved, ab) >= 0) {
                    res = 1;
                } else {  // `a` filled up meanwhile: carry the candidate from there
                    res = 2;
                    ncur = a;
                    ntag = moved;
                }
            }
            res = __shfl(res, j);
            if (res) {
                ++kicks;
                outcome = res;
                cur = res == 2 ? __shfl(ncur, j) : cur;
                tag = res == 2 ? __shfl(ntag, j) : tag;
            }
        }
        if (outcome == 1) return true;
        if (outcome == 2) continue;
        // no candidate moved: displace the last one and carry it
        uint32_t ev = 0;
        int ins = 0;
        if (lane == 0) {
            ev = cfk::swap_slot<G>(table, cur, (r0 + HALF - 1) % G::B, tag, cb);
            if (ev != 0) {
                uint32_t t2 = ev;
                const uint32_t c2 = cfk::move_tag<G, HASH, POL>(cur, t2, pl);
                cfk::Bucket<G> nb;
                cfk::load_bucket<G>(table, c2, nb);
                ins = cfk::try_insert<G>(table, c2, t2, nb) >= 0;
            }
        }
        ev = __shfl(ev, 0);
        ins = __shfl(ins, 0);
        ++kicks;
        if (ev == 0) return true;
        tag = ev;
        cur = cfk::move_tag<G, HASH, POL>(cur, tag, pl);
        if (ins) return true;
    }
    lost_bucket = cur;
    lost_tag = tag;
    return false;
}

// The single-filter insert_kernel's two passes, per operation on its own
// filter: direct attempts first, keys with two full buckets deferred to the
// bin's queue slice myq[0 .. b1 - b0) and searched afterwards with the
// filter's policy: the random walk one lane per key; the breadth-first
// search one lane per key with grouped probes (wave_bfs = 0) or one wave per
// key (wave_bfs = 1, evict_bfs_wave; the queued keys are dealt to the
// block's waves in turn).  s_qn is an LDS counter of the block; every thread
// of the block calls this (it has block barriers).
template <class G, int HASH, int POL, int BT>
__device__ __forceinline__ void insert_bin(const Batch &bt, const SetFilter *__restrict__ filters,
                                           const uint32_t *seg, uint32_t b0, uint32_t b1,
                                           uint32_t *myq, uint32_t *s_qn, Tally<BT> &tally,
                                           uint32_t wave_bfs) {
    using W = typename G::W;
    if (threadIdx.x == 0) *s_qn = 0;
    __syncthreads();  // s_qn = 0 before any wave adds to it
    const uint32_t qcap = b1 - b0;  // the bin's slice of the queue
    const int lane = threadIdx.x & 63;
    // The loop bound is uniform across the block so the ballot below always
    // sees whole waves.
    for (uint32_t p0 = b0; p0 < b1; p0 += BT) {
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
            if (lane == leader) qb = atomicAdd(s_qn, uint32_t(__popcll(need)));
            qb = __shfl(qb, leader, 64);
            const uint32_t pos = qb + uint32_t(__popcll(need & ((1ull << lane) - 1ull)));
            if (need_evict && pos < qcap) myq[pos] = p;
        }
    }
    __syncthreads();
    const uint32_t qn = *s_qn < qcap ? *s_qn : qcap;
    // the outcome of one queued key's search
    auto finish = [&](const SetFilter &F, uint32_t fid, uint32_t i, bool done, uint32_t lb,
                      uint32_t lt) {
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
    };
    if (!wave_bfs) {
        for (uint32_t q = threadIdx.x; q < qn; q += BT) {
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
                    ? cfk::evict_dfs<G, HASH, POL>(table, F.place, rs, cur, tag, F.max_evict, k,
                                                   lb, lt)
                    : cfk::evict_bfs<G, HASH, POL, probe_width<G>()>(table, F.place, rs, cur, tag,
                                                                    F.max_evict, k, lb, lt);
            finish(F, fid, i, done, lb, lt);
        }
    } else {
        constexpr uint32_t NW = BT / 64;
        const uint32_t wave = threadIdx.x >> 6;
        // wave w takes queued keys w, w + NW, w + 2 NW, ...: 64 of them at a
        // time, one per lane, then searches them one after another
        for (uint32_t base = 0; wave + NW * base < qn; base += 64) {  // uniform per wave
            const uint32_t q = wave + NW * (base + uint32_t(lane));
            const bool have = q < qn;
            uint32_t i = 0, fid = 0;
            bool walk = false;
            if (have) {
                i = seg[myq[q]];
                fid = bt.fids[i];
                walk = filters[fid].evict == CF_EVICT_DFS;
            }
            if (walk) {  // the random walk stays one lane per key
                const SetFilter &F = filters[fid];
                W *table = static_cast<W *>(F.table);
                const uint64_t key = bt.keys[i];
                const Derived d = cfk::derive<G, HASH, POL>(key, F.place);
                const uint64_t rs = key ^ F.seed;
                const bool second = (cfk::splitmix_at(rs, 0) & 1) != 0;
                uint32_t k = 0, lb = 0, lt = 0;
                const bool done = cfk::evict_dfs<G, HASH, POL>(
                    table, F.place, rs, second ? d.i2 : d.i1, second ? d.t2 : d.t1, F.max_evict,
                    k, lb, lt);
                finish(F, fid, i, done, lb, lt);
            }
            uint64_t todo = __ballot(have && !walk);
            while (todo) {  // uniform: one key at a time, the whole wave on it
                const int l = __builtin_ctzll(todo);
                todo &= todo - 1;
                const uint32_t il = __shfl(i, l), fl = __shfl(fid, l);
                const SetFilter &F = filters[fl];
                W *table = static_cast<W *>(F.table);
                const uint64_t key = bt.keys[il];
                const Derived d = cfk::derive<G, HASH, POL>(key, F.place);
                const uint64_t rs = key ^ F.seed;
                const bool second = (cfk::splitmix_at(rs, 0) & 1) != 0;
                uint32_t k = 0, lb = 0, lt = 0;
                const bool done = evict_bfs_wave<G, HASH, POL>(
                    table, F.place, rs, second ? d.i2 : d.i1, second ? d.t2 : d.t1, F.max_evict,
                    k, lb, lt);
                if (lane == 0) finish(F, fl, il, done, lb, lt);
            }
        }
    }
    __syncthreads();  // the queue slice and s_qn are free again
}

// ------------------------------------------------------- class kernels
// One launch per (phase, class): block b works on bin `bin` of chunk b.

template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_query_kernel(Batch bt,
                                                           const SetFilter *__restrict__ filters,
                                                           uint32_t chunk, uint32_t nb,
                                                           uint32_t bin, Scratch sc) {
    uint32_t b0, b1;
    bin_range(sc, nb, blockIdx.x, bin, b0, b1);
    query_bin<G, HASH, POL, kBlock>(bt, filters, sc.sorted + uint64_t(blockIdx.x) * chunk, b0, b1);
}

template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_delete_kernel(Batch bt,
                                                            const SetFilter *__restrict__ filters,
                                                            uint32_t nfilters, uint32_t chunk,
                                                            uint32_t nb, uint32_t bin, Scratch sc) {
    __shared__ int lds[kLdsFilters];
    Tally<kBlock> tally{lds, nfilters};
    tally.init();
    uint32_t b0, b1;
    bin_range(sc, nb, blockIdx.x, bin, b0, b1);
    delete_bin<G, HASH, POL, kBlock>(bt, filters, sc.sorted + uint64_t(blockIdx.x) * chunk, b0,
                                     b1, tally);
    tally.flush(filters);
}

template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void set_insert_kernel(Batch bt,
                                                            const SetFilter *__restrict__ filters,
                                                            uint32_t nfilters, uint32_t chunk,
                                                            uint32_t nb, uint32_t bin, Scratch sc,
                                                            uint32_t wave_bfs) {
    __shared__ int lds[kLdsFilters];
    __shared__ uint32_t s_qn;
    Tally<kBlock> tally{lds, nfilters};
    tally.init();
    uint32_t b0, b1;
    bin_range(sc, nb, blockIdx.x, bin, b0, b1);
    const uint64_t base = uint64_t(blockIdx.x) * chunk;
    insert_bin<G, HASH, POL, kBlock>(bt, filters, sc.sorted + base, b0, b1, sc.queue + base + b0,
                                     &s_qn, tally, wave_bfs);
    tally.flush(filters);
}

// ------------------------------------------------------ per-class launchers

struct ClassLaunch {
    void (*query)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, Scratch, int, hipStream_t);
    void (*del)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, uint32_t, Scratch, int,
                hipStream_t);
    void (*ins)(Batch, const SetFilter *, uint32_t, uint32_t, uint32_t, uint32_t, Scratch,
                uint32_t, int, hipStream_t);
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
                    uint32_t bin, Scratch sc, uint32_t wave_bfs, int grid, hipStream_t s) {
        set_insert_kernel<G, HASH, POL>
            <<<grid, kBlock, 0, s>>>(bt, fl, nf, chunk, nb, bin, sc, wave_bfs);
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
