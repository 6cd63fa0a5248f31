// cf_kernels.hpp -- gfx950 kernels of the cuckoo filter.
//
// One lane per key, wave64, grid-stride loops over any grid; the host picks
// the launch shape (one key per thread for queries and deletes up to a cap,
// a smaller grid with several keys per thread for inserts).  Occupancy
// counts follow Sec. 4.3's hierarchy: wave shuffle, LDS, one atomic per
// block.  Insertion defers the eviction search of keys whose two buckets
// are full to a second pass of the same block (see insert_kernel).
#pragma once

#include "cf_device.hpp"

namespace cfk {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kStripes = 32;  // occupancy counter stripes, one 128-byte line each

// Device-side counters.  The occupancy count is striped over kStripes
// separate lines: blocks add to stripe (blockIdx mod kStripes), so the one
// atomic per block of Sec. 4.3's hierarchical tally never piles up on a
// single address (device-scope atomics execute at the memory side on this
// part and same-address ones serialise).  The failure counter doubles as the
// cursor of the dropped-tag log; failures are rare.
struct alignas(128) Stripe {
    unsigned long long v;
    unsigned long long pad[15];
};

struct Counters {
    Stripe count[kStripes];
    unsigned long long failures;
    unsigned long long total;  // sum of the stripes, written by sum_counts_kernel
};

struct LostLog {
    unsigned long long *bucket;
    uint32_t *tag;
    unsigned long long cap;
};

// Sum v over the block and add it to the block's count stripe with one
// atomic.  Every thread of the block must call it.
__device__ __forceinline__ void block_add(Counters *ctr, unsigned long long v) {
    __shared__ unsigned long long part[kWaves];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) s += part[k];
        if (s) atomicAdd(&ctr->count[blockIdx.x % kStripes].v, s);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ query

// Alg. 2: probe i1, and i2 only when i1 misses.
template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void query_kernel(const typename G::W *__restrict__ table,
                                                       Place pl,
                                                       const uint64_t *__restrict__ keys,
                                                       uint64_t n, uint8_t *__restrict__ found) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t key = __builtin_nontemporal_load(keys + i);
        const Derived d = derive<G, HASH, POL>(key, pl);
        Bucket<G> bk;
        load_bucket<G>(table, d.i1, bk);
        bool hit = bk.contains(d.t1);
        if (!hit) {
            load_bucket<G>(table, d.i2, bk);
            hit = bk.contains(d.t2);
        }
        __builtin_nontemporal_store(uint8_t(hit), found + i);
    }
}

// ----------------------------------------------------------------- delete

// Alg. 3: remove one copy from i1, else from i2; the occupancy count drops
// by the block's number of successes.
template <class G, int HASH, int POL>
__global__ __launch_bounds__(kBlock) void delete_kernel(typename G::W *__restrict__ table,
                                                        Place pl,
                                                        const uint64_t *__restrict__ keys,
                                                        uint64_t n, uint8_t *__restrict__ ok,
                                                        Counters *ctr) {
    unsigned long long removed = 0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t key = __builtin_nontemporal_load(keys + i);
        const Derived d = derive<G, HASH, POL>(key, pl);
        Bucket<G> bk;
        load_bucket<G>(table, d.i1, bk);
        bool done = try_remove<G>(table, d.i1, d.t1, bk);
        if (!done) {
            load_bucket<G>(table, d.i2, bk);
            done = try_remove<G>(table, d.i2, d.t2, bk);
        }
        removed += done;
        if (ok) ok[i] = uint8_t(done);
    }
    // count -= removed, as the two's-complement addition of -removed
    block_add(ctr, 0ull - removed);
}

// --------------------------------------------------- insert: eviction search

// Candidates whose other buckets a grouped breadth-first search loads at
// once: as many as 128 bytes of buckets hold, at most b/2.
template <class G>
constexpr int probe_width() {
    constexpr int bytes = G::B * G::F / 8;
    constexpr int fit = bytes >= 128 ? 1 : 128 / bytes;
    return fit < G::B / 2 ? fit : G::B / 2;
}

// Sec. 4.6.1 breadth-first heuristic.  At each level the candidates are the
// b/2 slots of the current bucket starting at a random slot; the first whose
// fingerprint has an empty slot in its other bucket is moved there and the
// carried fingerprint takes its place.  Failing that, the last candidate is
// displaced and carried to its other bucket.  The move is done displacement
// first: the carried fingerprint replaces the candidate with a CAS that only
// succeeds while the slot still holds the candidate, then the candidate is
// inserted into its other bucket.  If that bucket filled up in the meantime
// the candidate is simply carried on, as after a displacement.  `tag` is
// always the carried fingerprint as it is written in `cur` (the choice bit
// of the offset policy flips with every move).
// The insert kernels that use it are compiled at -O1: built at -O2 or -O3
// they lost fingerprints under heavy contention (one-launch fills of a
// 2^20-slot table), a loss that appears with the backend's Early Machine
// LICM run over the kernel and goes away without it; see the one-launch
// contention tests.
//
// PW (probe width) candidates have their other buckets loaded together, then
// the first of them (in candidate order) with an empty slot is moved, so the
// choice is the one a candidate-by-candidate probe makes on an unchanged
// table; only the number of dependent loads per level drops, from b/2 to
// b/(2 PW), at the price of loading a group's buckets whole.  PW = 1 is the
// candidate-by-candidate probe, which the single-filter insert kernel uses
// on large tables, where it is bound by memory requests and whole groups
// only add reads; tables of a few MiB measured faster with probe_width (the
// launchers choose by table size).
template <class G, int HASH, int POL, int PW = 1>
__device__ __forceinline__ bool evict_bfs(typename G::W *table, const Place &pl, uint64_t rs, uint32_t cur,
                          uint32_t tag, uint32_t max_evict, uint32_t &kicks,
                          uint32_t &lost_bucket, uint32_t &lost_tag) {
    constexpr int HALF = G::B / 2;
    static_assert(PW >= 1 && HALF % PW == 0, "probe width must divide b/2");
    for (uint32_t n = 1; n <= max_evict; ++n) {
        Bucket<G> cb;
        load_bucket<G>(table, cur, cb);
        if (cb.has_empty() && try_insert<G>(table, cur, tag, cb) >= 0) return true;
        const int r0 = int(splitmix_at(rs, n) % uint64_t(G::B));
        bool carried = false;
        if constexpr (PW > 1) {
            for (int j0 = 0; j0 < HALF && !carried; j0 += PW) {
                // the group's other buckets, loaded together; only a bit per
                // candidate (its other bucket has an empty slot) is kept
                uint32_t ok = 0, cv[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    cv[q] = cb.slot((r0 + j0 + q) % G::B);
                    uint32_t moved = cv[q];
                    const uint32_t a = move_tag<G, HASH, POL>(cur, moved, pl);
                    if (cv[q] != 0 && a != cur) {
                        Bucket<G> ab;
                        load_bucket<G>(table, a, ab);
                        if (ab.has_empty()) ok |= 1u << q;
                    }
                }
                // then, in candidate order, the move of the first that takes it
                // (the probed value: the move happens only while the slot holds it)
                while (ok && !carried) {
                    const int q = __builtin_ctz(ok);
                    ok &= ok - 1u;
                    const int s = (r0 + j0 + q) % G::B;
                    uint32_t c = 0;
#pragma unroll
                    for (int k = 0; k < PW; ++k) c = k == q ? cv[k] : c;
                    uint32_t moved = c;
                    const uint32_t a = move_tag<G, HASH, POL>(cur, moved, pl);
                    if (!replace_slot_if<G>(table, cur, s, c, tag, cb)) continue;
                    ++kicks;
                    Bucket<G> ab;
                    load_bucket<G>(table, a, ab);
                    if (try_insert<G>(table, a, moved, ab) >= 0) return true;
                    tag = moved;  // `a` filled up meanwhile: carry the candidate from there
                    cur = a;
                    carried = true;
                }
            }
        }
        for (int j = 0; PW == 1 && j < HALF && !carried; ++j) {
            const int s = (r0 + j) % G::B;
            const uint32_t c = cb.slot(s);
            if (c == 0) continue;
            uint32_t moved = c;
            const uint32_t a = move_tag<G, HASH, POL>(cur, moved, pl);
            if (a == cur) continue;
            Bucket<G> ab;
            load_bucket<G>(table, a, ab);
            if (!ab.has_empty()) continue;
            if (!replace_slot_if<G>(table, cur, s, c, tag, cb)) continue;
            ++kicks;
            if (try_insert<G>(table, a, moved, ab) >= 0) return true;
            tag = moved;  // `a` filled up meanwhile: carry the candidate from there
            cur = a;
            carried = true;
        }
        if (carried) continue;
        const int s_last = (r0 + HALF - 1) % G::B;
        const uint32_t ev = swap_slot<G>(table, cur, s_last, tag, cb);
        ++kicks;
        if (ev == 0) return true;
        tag = ev;
        cur = move_tag<G, HASH, POL>(cur, tag, pl);
        Bucket<G> nb;
        load_bucket<G>(table, cur, nb);
        if (try_insert<G>(table, cur, tag, nb) >= 0) return true;
    }
    lost_bucket = cur;
    lost_tag = tag;
    return false;
}

// Alg. 1 eviction chain: displace a random slot, carry the displaced
// fingerprint to its other bucket, try there.
template <class G, int HASH, int POL>
__device__ __forceinline__ bool evict_dfs(typename G::W *table, const Place &pl, uint64_t rs, uint32_t cur,
                          uint32_t tag, uint32_t max_evict, uint32_t &kicks,
                          uint32_t &lost_bucket, uint32_t &lost_tag) {
    for (uint32_t n = 1; n <= max_evict; ++n) {
        const int s = int(splitmix_at(rs, n) % uint64_t(G::B));
        Bucket<G> cb;
        load_bucket<G>(table, cur, cb);
        const uint32_t ev = swap_slot<G>(table, cur, s, tag, cb);
        ++kicks;
        if (ev == 0) return true;
        tag = ev;
        cur = move_tag<G, HASH, POL>(cur, tag, pl);
        Bucket<G> nb;
        load_bucket<G>(table, cur, nb);
        if (try_insert<G>(table, cur, tag, nb) >= 0) return true;
    }
    lost_bucket = cur;
    lost_tag = tag;
    return false;
}

// ------------------------------------------------------------------ insert

// One launch per batch, in two passes per block.
//  1. Direct pass (Alg. 1 phase 1) over the block's grid-stride share of the
//     keys.  Keys whose two buckets are full go to the block's own segment of
//     the eviction queue, queue[blockIdx * seg ...], through a wave-aggregated
//     LDS counter: no global atomic is involved in the hand-off.
//  2. Eviction pass (BFS of Sec. 4.6.1 or the random walk of Alg. 1) over
//     that segment.
// Within an insert launch slots only ever go from EMPTY to full (evictions
// replace a fingerprint in place), so a queued key's two buckets are still
// full when its eviction starts: this is one legal interleaving of the
// paper's concurrent insert.  Deferring evictions keeps the common path's
// wave64 lanes free of eviction-chain divergence, and blocks in different
// passes overlap the read-heavy direct work with the atomic-heavy evictions.
template <class G, int HASH, int EVICT, int POL, int PW = 1>
__global__ __launch_bounds__(kBlock) void insert_kernel(
    typename G::W *__restrict__ table, Place pl, const uint64_t *__restrict__ keys,
    uint64_t n, uint8_t *__restrict__ ok, uint32_t *__restrict__ kicks, Counters *ctr,
    uint32_t *__restrict__ queue, uint64_t seg, LostLog log, uint32_t max_evict,
    uint64_t seed) {
    __shared__ uint32_t s_qn;
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();
    uint32_t *myq = queue + uint64_t(blockIdx.x) * seg;
    unsigned long long placed = 0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    const int lane = threadIdx.x & 63;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t key = __builtin_nontemporal_load(keys + i);
        const Derived d = derive<G, HASH, POL>(key, pl);
        Bucket<G> bk;
        load_bucket<G>(table, d.i1, bk);
        bool done = try_insert<G>(table, d.i1, d.t1, bk) >= 0;
        if (!done) {
            load_bucket<G>(table, d.i2, bk);
            done = try_insert<G>(table, d.i2, d.t2, bk) >= 0;
        }
        placed += done;
        if (ok) ok[i] = uint8_t(done);
        if (kicks) kicks[i] = 0;
        const uint64_t need = __ballot(!done);
        if (need) {
            const int leader = __builtin_ctzll(need);
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&s_qn, uint32_t(__popcll(need)));
            base = __shfl(base, leader, 64);
            const uint32_t pos = base + uint32_t(__popcll(need & ((1ull << lane) - 1ull)));
            if (!done && pos < seg) myq[pos] = uint32_t(i);
        }
    }
    __syncthreads();
    const uint32_t qn = s_qn < seg ? s_qn : uint32_t(seg);
    for (uint32_t q = threadIdx.x; q < qn; q += kBlock) {
        const uint32_t idx = myq[q];
        const uint64_t key = keys[idx];
        const Derived d = derive<G, HASH, POL>(key, pl);
        const uint64_t rs = key ^ seed;
        const bool second = (splitmix_at(rs, 0) & 1) != 0;
        const uint32_t cur = second ? d.i2 : d.i1;
        const uint32_t tag = second ? d.t2 : d.t1;
        uint32_t k = 0, lb = 0, lt = 0;
        bool done;
        if constexpr (EVICT == 1)
            done = evict_dfs<G, HASH, POL>(table, pl, rs, cur, tag, max_evict, k, lb, lt);
        else
            done = evict_bfs<G, HASH, POL, PW>(table, pl, rs, cur, tag, max_evict, k, lb, lt);
        placed += done;
        if (!done) {
            const unsigned long long slot = atomicAdd(&ctr->failures, 1ull);
            if (slot < log.cap) {
                log.bucket[slot] = lb;
                log.tag[slot] = lt;
            }
        }
        if (ok) ok[idx] = uint8_t(done);
        if (kicks) kicks[idx] = k;
    }
    block_add(ctr, placed);
}

// ------------------------------------------------------------- utilities

// Occupancy recount after an import: non-empty slots over the whole table.
template <class G>
__global__ __launch_bounds__(kBlock) void recount_kernel(const typename G::W *__restrict__ table,
                                                         uint64_t nwords, Counters *ctr) {
    using W = typename G::W;
    constexpr W HI = lane_repeat<W, G::F>(W(1)) << (G::F - 1);
    unsigned long long c = 0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < nwords; i += stride) {
        const W nz = ~zero_lanes<W, G::F>(table[i]) & HI;
        if constexpr (sizeof(W) == 8) c += __popcll(nz);
        else c += __popc(nz);
    }
    block_add(ctr, c);
}

static __global__ void clear_counters_kernel(Counters *ctr) {
    const int t = threadIdx.x;
    if (t < kStripes) ctr->count[t].v = 0;
    if (t == 0) {
        ctr->failures = 0;
        ctr->total = 0;
    }
}

// total = sum of the count stripes (one wave).
static __global__ void sum_counts_kernel(Counters *ctr) {
    unsigned long long v = threadIdx.x < kStripes ? ctr->count[threadIdx.x].v : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (threadIdx.x == 0) ctr->total = v;
}

static __global__ __launch_bounds__(kBlock) void zero_words_kernel(uint64_t *__restrict__ p, uint64_t n) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0;
}

}  // namespace cfk
