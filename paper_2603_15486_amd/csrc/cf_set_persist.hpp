// cf_set_persist.hpp -- the persistent form of a filter set's mixed batch:
// one cooperative launch runs the whole batch (partition, queries, deletes,
// inserts) with grid-wide barriers between the phases, instead of a
// partition launch and one launch per (phase, class).
//
// The phases and their order are those of cf_set.h's batch semantics: every
// query sees its filter as it was before the batch (Sec. 4.4: a query must
// not overlap a write), then all deletes run, then all inserts (inserts and
// deletes never overlap, which the delete's fetch-AND relies on).  Within a
// phase each block takes chunks c = blockIdx, blockIdx + grid, ... and runs
// every bin of that phase in the chunk, dispatching on the bin's bucket size
// b at run time; the per-bin work is the class kernels' own (query_bin,
// delete_bin, insert_bin).  A set qualifies when all its filters share the
// fingerprint width, hash and placement (any mix of b).
//
// Grid barrier.  Every block must be resident at once, which the cooperative
// launch guarantees (it refuses a grid that cannot be).  The blocks are split
// into kBarrierGroups groups (block k in group k mod kBarrierGroups), each
// with an arrival counter and a generation word on lines of their own:
// device-scope atomics on one address are performed one after another at
// the memory side, so a single counter for a grid of a thousand blocks would
// cost a thousand serialised round trips per barrier, and a thousand blocks
// polling one word queue on one memory channel.  Each block's thread 0
// publishes the block's writes (agent-scope release) and adds one to its
// group's counter; the last of a group resets it and adds one to the top
// counter; the last group's last block resets that and advances every
// group's generation (release).  The others poll their group's generation
// (agent-scope acquire), sleeping about a microsecond between polls.  The
// wait is bounded: past `limit` ticks of the constant-rate wall clock, or
// once another block has given up, the block marks the control block's
// error word and leaves the kernel without touching the batch again.  A block
// never enters a phase unless the barrier before it completed, so an
// abandoned batch does no out-of-order work; a marked error also makes later
// launches return at once until the host clears the control block
// (cf_set_set_shape).
#pragma once

#include "cf_set_kernels.hpp"

namespace cfs {

// Control block of the persistent path, one per set; each word on its own
// 128-byte line.  Zeroed at creation and when the host clears an error.
constexpr uint32_t kBarrierGroups = 32;

struct alignas(128) CtlWord {
    unsigned int v;
    unsigned int pad[31];
};

// Wall-clock ticks of the last batch: [0] when block 0 started, [k] when
// barrier k (k = 1, 2, 3: after the partition, the queries, the deletes)
// completed; written by block 0 and by each barrier's releaser.
struct alignas(128) CtlStamps {
    unsigned long long t[4];
    unsigned long long pad[12];
};

struct PersistCtl {
    CtlWord top;                        // groups arrived at the current barrier
    CtlWord error;                      // 1 once a barrier wait gave up
    CtlWord arrive[kBarrierGroups];     // blocks of each group arrived
    CtlWord gen[kBarrierGroups];        // barriers completed, per group
    CtlStamps stamp;
};

// Bucket size b of each class of the set (all classes share f, hash and
// placement on this path).
struct ClassB {
    uint8_t b[kMaxClasses];
};

__device__ __forceinline__ unsigned int ld_relaxed(const unsigned int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned int add_relaxed(unsigned int *p) {
    return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(unsigned int *p, unsigned int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The grid barrier described above.  Returns false if the block must leave
// (this or another block gave up).  Every thread of the block calls it; `gen`
// is the block's count of completed barriers (the same in every thread).
// Ordering is by fences around relaxed atomics: an agent-scope release fence
// writes the L2's dirty lines back and an acquire fence invalidates the
// L2's lines that other agents' caches may have changed, so they are issued
// once per arrival and once after the wait, never per poll (an acquiring
// poll would invalidate the L2 of every waiting block's compute unit again
// and again, under the blocks of that L2 still working).  Each arrival is a
// release fence then a relaxed add; the group's last and the last group
// acquire what came before them (the adds form one release sequence per
// counter) and release it on; the waiters acquire after their poll sees the
// generation move.
__device__ __forceinline__ bool grid_sync(PersistCtl *ctl, unsigned int &gen, uint64_t limit,
                                          int stamp) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t ngroups = gridDim.x < kBarrierGroups ? gridDim.x : kBarrierGroups;
        const uint32_t g = blockIdx.x % kBarrierGroups;
        const uint32_t members = (gridDim.x - g + kBarrierGroups - 1) / kBarrierGroups;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this block's writes first
        bool released = false;
        if (add_relaxed(&ctl->arrive[g].v) == members - 1) {  // the group's last
            // reset for the next barrier, then acquire the group and release
            // it (with the reset) to the top counter
            st_relaxed(&ctl->arrive[g].v, 0u);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if (add_relaxed(&ctl->top.v) == ngroups - 1) {  // the last group: release all
                st_relaxed(&ctl->top.v, 0u);
                ctl->stamp.t[stamp] = wall_clock64();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                for (uint32_t k = 0; k < ngroups; ++k) st_relaxed(&ctl->gen[k].v, gen + 1);
                released = true;
            }
        }
        if (!released) {
            // A poll is a device-coherent load served past the L2; a waiting
            // block sleeps about a microsecond between polls and looks at the
            // error word only every 16th time.
            const uint64_t t0 = wall_clock64();
            uint32_t polls = 0;
            while (ld_relaxed(&ctl->gen[g].v) == gen) {
                if (wall_clock64() - t0 > limit ||
                    ((++polls & 15u) == 0 && ld_relaxed(&ctl->error.v))) {
                    st_relaxed(&ctl->error.v, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(32);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other blocks' writes
        s_ok = ok;
    }
    __syncthreads();
    gen += 1;
    return s_ok != 0;
}

// Run fn(Geom<F, b>{}) for the bucket sizes the library compiles, up to
// BMAX slots.  A kernel holds the code of every bucket size it may meet and
// takes the registers of the largest: the 32-slot insert path alone limits
// a kernel to 4 waves per SIMD, so sets whose buckets have at most 16 slots
// get kernels without it (BMAX = 16).
template <int F, int BMAX, class Fn>
__device__ __forceinline__ void with_b(uint32_t b, Fn &&fn) {
    switch (b) {
        case 4: fn(cfk::Geom<F, 4>{}); break;
        case 8: fn(cfk::Geom<F, 8>{}); break;
        case 16: fn(cfk::Geom<F, 16>{}); break;
        case 32:
            if constexpr (BMAX >= 32) fn(cfk::Geom<F, 32>{});
            break;
        default: break;
    }
}

template <int F, int HASH, int POL, int BT, int BMAX>
__global__ __launch_bounds__(BT) void persist_kernel(Batch bt, const SetFilter *__restrict__ filters,
                                                     const uint8_t *__restrict__ cls, ClassB cb,
                                                     uint32_t nfilters, uint32_t ncls,
                                                     uint32_t chunk, Scratch sc, PersistCtl *ctl,
                                                     uint64_t limit, uint32_t wave_bfs) {
    __shared__ uint32_t hist[kMaxBins + 1];
    __shared__ uint32_t base[kMaxBins + 1];
    __shared__ int lds[kLdsFilters];
    __shared__ uint32_t s_qn;
    __shared__ unsigned int s_gen;
    __shared__ int s_err;
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) ctl->stamp.t[0] = wall_clock64();
        s_err = int(ld_relaxed(&ctl->error.v));
        s_gen = ld_relaxed(&ctl->gen[blockIdx.x % kBarrierGroups].v);
    }
    __syncthreads();
    if (s_err) return;  // an earlier batch was abandoned: nothing runs until cleared
    unsigned int gen = s_gen;
    const uint32_t nb = 3 * ncls;
    const uint64_t n = batch_n(bt);
    const uint64_t nchunks = (n + chunk - 1) / chunk;
    Tally<BT> tally{lds, nfilters};

    // phase 0: sort every chunk by (kind, class)
    for (uint64_t cid = blockIdx.x; cid < nchunks; cid += gridDim.x)
        partition_chunk<BT>(bt, n, cls, nfilters, ncls, chunk, cid, sc, hist, base);
    if (!grid_sync(ctl, gen, limit, 1)) return;

    // phase 1: queries (Alg. 2)
    for (uint64_t cid = blockIdx.x; cid < nchunks; cid += gridDim.x) {
        const uint32_t *seg = sc.sorted + cid * chunk;
        for (uint32_t c = 0; c < ncls; ++c) {
            uint32_t b0, b1;
            bin_range(sc, nb, cid, c, b0, b1);
            if (b0 < b1)
                with_b<F, BMAX>(cb.b[c], [&](auto g) {
                    query_bin<decltype(g), HASH, POL, BT>(bt, filters, seg, b0, b1);
                });
        }
    }
    if (!grid_sync(ctl, gen, limit, 2)) return;

    // phase 2: deletes (Alg. 3)
    tally.init();
    for (uint64_t cid = blockIdx.x; cid < nchunks; cid += gridDim.x) {
        const uint32_t *seg = sc.sorted + cid * chunk;
        for (uint32_t c = 0; c < ncls; ++c) {
            uint32_t b0, b1;
            bin_range(sc, nb, cid, ncls + c, b0, b1);
            if (b0 < b1)
                with_b<F, BMAX>(cb.b[c], [&](auto g) {
                    delete_bin<decltype(g), HASH, POL, BT>(bt, filters, seg, b0, b1, tally);
                });
        }
    }
    tally.flush(filters);
    if (!grid_sync(ctl, gen, limit, 3)) return;

    // phase 3: inserts (Alg. 1 with the eviction search of Sec. 4.6.1)
    tally.init();
    for (uint64_t cid = blockIdx.x; cid < nchunks; cid += gridDim.x) {
        const uint64_t at = cid * chunk;
        for (uint32_t c = 0; c < ncls; ++c) {
            uint32_t b0, b1;
            bin_range(sc, nb, cid, 2 * ncls + c, b0, b1);
            if (b0 < b1)  // uniform across the block: insert_bin has block barriers
                with_b<F, BMAX>(cb.b[c], [&](auto g) {
                    insert_bin<decltype(g), HASH, POL, BT>(bt, filters, sc.sorted + at, b0, b1,
                                                           sc.queue + at + b0, &s_qn, tally,
                                                           wave_bfs);
                });
        }
    }
    tally.flush(filters);
}

// ------------------------------------------------ one launch per phase
// The class-kernel form with the classes of each phase fused into one
// launch: grid = chunks x classes, block k working on bin (phase, k mod
// ncls) of chunk k / ncls with that class's b chosen at run time (with_b).
// The queries of every class run side by side in one launch, then every
// delete, then every insert, all on the caller's stream: no side streams,
// and a captured batch is a straight chain of four kernels (partition and
// three phases).  Same qualification as the persistent form (one f, hash and
// placement, any mix of b).  Bins beyond the batch's chunks are empty (the
// partition writes empty offsets for them), and a block with an empty bin
// returns at once, before any barrier.

template <int F, int HASH, int POL, int BMAX>
__global__ __launch_bounds__(kBlock) void phase_query_kernel(Batch bt,
                                                             const SetFilter *__restrict__ filters,
                                                             ClassB cb, uint32_t ncls,
                                                             uint32_t chunk, Scratch sc) {
    const uint64_t cid = blockIdx.x / ncls;
    const uint32_t c = blockIdx.x % ncls;
    uint32_t b0, b1;
    bin_range(sc, 3 * ncls, cid, c, b0, b1);
    if (b0 >= b1) return;
    const uint32_t *seg = sc.sorted + cid * chunk;
    with_b<F, BMAX>(cb.b[c], [&](auto g) {
        query_bin<decltype(g), HASH, POL, kBlock>(bt, filters, seg, b0, b1);
    });
}

template <int F, int HASH, int POL, int BMAX>
__global__ __launch_bounds__(kBlock) void phase_delete_kernel(Batch bt,
                                                              const SetFilter *__restrict__ filters,
                                                              ClassB cb, uint32_t nfilters,
                                                              uint32_t ncls, uint32_t chunk,
                                                              Scratch sc) {
    __shared__ int lds[kLdsFilters];
    const uint64_t cid = blockIdx.x / ncls;
    const uint32_t c = blockIdx.x % ncls;
    uint32_t b0, b1;
    bin_range(sc, 3 * ncls, cid, ncls + c, b0, b1);
    if (b0 >= b1) return;  // the same in every thread of the block
    Tally<kBlock> tally{lds, nfilters};
    tally.init();
    const uint32_t *seg = sc.sorted + cid * chunk;
    with_b<F, BMAX>(cb.b[c], [&](auto g) {
        delete_bin<decltype(g), HASH, POL, kBlock>(bt, filters, seg, b0, b1, tally);
    });
    tally.flush(filters);
}

template <int F, int HASH, int POL, int BMAX>
__global__ __launch_bounds__(kBlock) void phase_insert_kernel(Batch bt,
                                                              const SetFilter *__restrict__ filters,
                                                              ClassB cb, uint32_t nfilters,
                                                              uint32_t ncls, uint32_t chunk,
                                                              Scratch sc, uint32_t wave_bfs) {
    __shared__ int lds[kLdsFilters];
    __shared__ uint32_t s_qn;
    const uint64_t cid = blockIdx.x / ncls;
    const uint32_t c = blockIdx.x % ncls;
    uint32_t b0, b1;
    bin_range(sc, 3 * ncls, cid, 2 * ncls + c, b0, b1);
    if (b0 >= b1) return;  // the same in every thread of the block
    Tally<kBlock> tally{lds, nfilters};
    tally.init();
    const uint64_t at = cid * chunk;
    with_b<F, BMAX>(cb.b[c], [&](auto g) {
        insert_bin<decltype(g), HASH, POL, kBlock>(bt, filters, sc.sorted + at, b0, b1,
                                                   sc.queue + at + b0, &s_qn, tally, wave_bfs);
    });
    tally.flush(filters);
}

// Host launchers of the three phase kernels for one (f, hash, placement).
// grid = chunks x classes.
struct PhaseLaunch {
    void (*query)(Batch, const SetFilter *, ClassB, uint32_t ncls, uint32_t chunk, Scratch,
                  int grid, hipStream_t) = nullptr;
    void (*del)(Batch, const SetFilter *, ClassB, uint32_t nfilters, uint32_t ncls,
                uint32_t chunk, Scratch, int grid, hipStream_t) = nullptr;
    void (*ins)(Batch, const SetFilter *, ClassB, uint32_t nfilters, uint32_t ncls,
                uint32_t chunk, Scratch, uint32_t wave_bfs, int grid, hipStream_t) = nullptr;
};

template <int F, int HASH, int POL, int BMAX>
struct PhaseInst {
    static void query(Batch bt, const SetFilter *fl, ClassB cb, uint32_t ncls, uint32_t chunk,
                      Scratch sc, int grid, hipStream_t s) {
        phase_query_kernel<F, HASH, POL, BMAX><<<grid, kBlock, 0, s>>>(bt, fl, cb, ncls, chunk, sc);
    }
    static void del(Batch bt, const SetFilter *fl, ClassB cb, uint32_t nf, uint32_t ncls,
                    uint32_t chunk, Scratch sc, int grid, hipStream_t s) {
        phase_delete_kernel<F, HASH, POL, BMAX><<<grid, kBlock, 0, s>>>(bt, fl, cb, nf, ncls, chunk, sc);
    }
    static void ins(Batch bt, const SetFilter *fl, ClassB cb, uint32_t nf, uint32_t ncls,
                    uint32_t chunk, Scratch sc, uint32_t wave_bfs, int grid, hipStream_t s) {
        phase_insert_kernel<F, HASH, POL, BMAX>
            <<<grid, kBlock, 0, s>>>(bt, fl, cb, nf, ncls, chunk, sc, wave_bfs);
    }
};

// Fills the query and delete launchers (INSERT = false) or the insert
// launcher (INSERT = true) of L for sets whose buckets have at most bmax
// slots; false for an unknown hash or placement.
template <int F, bool INSERT, int BMAX>
bool pick_phase_fb(uint32_t hash, uint32_t placement, PhaseLaunch &L) {
    if (hash > 1 || placement > 1) return false;
    auto fill = [&](auto inst) {
        using I = decltype(inst);
        if constexpr (INSERT) {
            L.ins = &I::ins;
        } else {
            L.query = &I::query;
            L.del = &I::del;
        }
    };
    if (hash == 0)
        placement ? fill(PhaseInst<F, 0, 1, BMAX>{}) : fill(PhaseInst<F, 0, 0, BMAX>{});
    else
        placement ? fill(PhaseInst<F, 1, 1, BMAX>{}) : fill(PhaseInst<F, 1, 0, BMAX>{});
    return true;
}

template <int F, bool INSERT>
bool pick_phase_f(uint32_t hash, uint32_t placement, uint32_t bmax, PhaseLaunch &L) {
    return bmax <= 16 ? pick_phase_fb<F, INSERT, 16>(hash, placement, L)
                      : pick_phase_fb<F, INSERT, 32>(hash, placement, L);
}

// Per fingerprint width: query and delete in cf_set_inst_f*.hip, insert in
// cf_set_persist_insi_f*.hip (built at -O1).
bool pick_phase_f8(uint32_t hash, uint32_t placement, uint32_t bmax, PhaseLaunch &out);
bool pick_phase_f16(uint32_t hash, uint32_t placement, uint32_t bmax, PhaseLaunch &out);
bool pick_phase_f32(uint32_t hash, uint32_t placement, uint32_t bmax, PhaseLaunch &out);
bool pick_phase_insert_f8(uint32_t hash, uint32_t placement, uint32_t bmax,
                          PhaseLaunch &out);
bool pick_phase_insert_f16(uint32_t hash, uint32_t placement, uint32_t bmax,
                          PhaseLaunch &out);
bool pick_phase_insert_f32(uint32_t hash, uint32_t placement, uint32_t bmax,
                          PhaseLaunch &out);

// Host side: the kernel for the set's (f, hash, placement) at each block size.
constexpr int kPersistBlocks[2] = {256, 512};

struct PersistLaunch {
    const void *kern[2] = {nullptr, nullptr};  // block of kPersistBlocks[k] threads
};

template <int F, int HASH, int POL, int BMAX>
void fill_persist(PersistLaunch &L) {
    L.kern[0] = reinterpret_cast<const void *>(&persist_kernel<F, HASH, POL, 256, BMAX>);
    L.kern[1] = reinterpret_cast<const void *>(&persist_kernel<F, HASH, POL, 512, BMAX>);
}

template <int F, int BMAX>
bool pick_persist_fb(uint32_t hash, uint32_t placement, PersistLaunch &L) {
    if (hash > 1 || placement > 1) return false;
    if (hash == 0) placement ? fill_persist<F, 0, 1, BMAX>(L) : fill_persist<F, 0, 0, BMAX>(L);
    else placement ? fill_persist<F, 1, 1, BMAX>(L) : fill_persist<F, 1, 0, BMAX>(L);
    return true;
}

// The kernels for a set whose buckets have at most bmax slots.
template <int F>
bool pick_persist_f(uint32_t hash, uint32_t placement, uint32_t bmax, PersistLaunch &L) {
    return bmax <= 16 ? pick_persist_fb<F, 16>(hash, placement, L)
                      : pick_persist_fb<F, 32>(hash, placement, L);
}

// Per fingerprint width, in cf_set_persist_insi_f*.hip (built at -O1 like
// every unit with insert code).
bool pick_persist_f8(uint32_t hash, uint32_t placement, uint32_t bmax, PersistLaunch &out);
bool pick_persist_f16(uint32_t hash, uint32_t placement, uint32_t bmax, PersistLaunch &out);
bool pick_persist_f32(uint32_t hash, uint32_t placement, uint32_t bmax, PersistLaunch &out);

}  // namespace cfs
