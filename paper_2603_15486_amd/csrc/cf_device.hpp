// cf_device.hpp -- device-side building blocks of the gfx950 cuckoo filter:
// bucket geometry, SWAR lane masks, the two hash functions, the eviction
// random stream, and the per-bucket primitives of Alg. 1-3 (TryInsert, Find,
// TryRemove) and of the eviction policies (slot swap).
//
// Everything here is compiled for one (f, b) geometry at a time through the
// Geom template so that loops over a bucket's words unroll and the bucket
// stays in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace cfk {

// ---------------------------------------------------------------- geometry

// Bucket geometry (Sec. 4.2, Fig. 2).  Slots are packed f bits apart from the
// low end of little-endian words; bucket j holds global slots [j*b, (j+1)*b).
// A bucket of 32 bits (b = 4, f = 8) is handled as one 32-bit word: in memory
// this is exactly the low or high half of the 64-bit word the paper's layout
// would use, but it lets each bucket be updated with its own 32-bit CAS.
template <int F_, int B_>
struct Geom {
    static constexpr int F = F_;
    static constexpr int B = B_;
    using W = typename std::conditional<(F_ * B_ < 64), uint32_t, uint64_t>::type;
    static constexpr int WBITS = 8 * sizeof(W);
    static constexpr int TPW = WBITS / F;  // tags per word
    static constexpr int WPB = B / TPW;    // words per bucket
    static constexpr uint32_t FMASK = (F == 32) ? 0xffffffffu : ((1u << F) - 1u);
    static_assert(F * B >= 32, "buckets smaller than 32 bits are not supported");
    static_assert(WPB >= 1 && TPW * WPB == B, "bucket must be whole words");
};

// Repeat `v` in every f-bit lane of a word.
template <typename W, int F>
__host__ __device__ constexpr W lane_repeat(W v) {
    W r = 0;
    for (int i = 0; i < int(8 * sizeof(W)) / F; ++i) r |= v << (i * F);
    return r;
}

// Exact per-lane zero test: bit (k*F + F-1) is set iff lane k of w is 0.
// (The low F-1 bits of a lane plus 2^(F-1)-1 carry into the lane's top bit
// iff they are non-zero and never carry out of the lane; OR-ing w adds the
// lane's own top bit.)
template <typename W, int F>
__device__ __forceinline__ W zero_lanes(W w) {
    constexpr W HI = lane_repeat<W, F>(W(1)) << (F - 1);
    constexpr W LO7 = ~HI;
    return ~(((w & LO7) + LO7) | w) & HI;
}

template <typename W, int F>
__device__ __forceinline__ W match_lanes(W w, uint32_t tag) {
    return zero_lanes<W, F>(w ^ (W(tag) * lane_repeat<W, F>(W(1))));
}

template <typename W>
__device__ __forceinline__ int lowest_bit(W x) {
    if constexpr (sizeof(W) == 8) return __builtin_ctzll(x);
    else return __builtin_ctz(x);
}

// ------------------------------------------------------------------ hashes

// MurmurHash3's 64-bit finalizer.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int r) {
    return (x << r) | (x >> (64 - r));
}

// xxHash64 of the 8-byte little-endian encoding of x, seed 0 (the
// specification's path for inputs shorter than 32 bytes with one 8-byte lane).
__device__ __forceinline__ uint64_t xxh64_8(uint64_t x) {
    constexpr uint64_t P1 = 0x9E3779B185EBCA87ull, P2 = 0xC2B2AE3D27D4EB4Full,
                       P3 = 0x165667B19E3779F9ull, P4 = 0x85EBCA77C2B2AE63ull,
                       P5 = 0x27D4EB2F165667C5ull;
    uint64_t h = P5 + 8u;
    h ^= rotl64(x * P2, 31) * P1;
    h = rotl64(h, 27) * P1 + P4;
    h ^= h >> 33;
    h *= P2;
    h ^= h >> 29;
    h *= P3;
    h ^= h >> 32;
    return h;
}

template <int HASH>
__device__ __forceinline__ uint64_t hash64(uint64_t x) {
    if constexpr (HASH == 1) return xxh64_8(x);
    else return fmix64(x);
}

// Output k of the SplitMix64 stream that starts at state s.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t s, uint64_t k) {
    uint64_t z = s + (k + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// --------------------------------------------------------- derived values

// Bucket placement, as the kernels need it at run time.  POL selects the
// policy at compile time: 0 = XOR (Eq. (3), m a power of two), 1 = offset
// with a choice bit (Sec. 4.6.2, any m in [1, 2^32)).
struct Place {
    uint32_t mmask;  // XOR: m - 1
    uint32_t m;      // offset: bucket count
    uint32_t m1;     // offset: m - 1
    uint32_t pad;
    uint64_t mdiv;   // offset: fastmod constant of m
    uint64_t m1div;  // offset: fastmod constant of m - 1 (m >= 2)
};

// a mod d for 32-bit a and d >= 1, with M = floor((2^64 - 1) / d) + 1
// (Lemire, Kaser and Kurz, "Faster remainder by direct computation", 2019):
// the low 64 bits of M * a hold the fraction a / d, and multiplying them by
// d keeps the remainder in the high 64 bits.  Exact for every 32-bit a, d.
__host__ __device__ constexpr uint64_t fastmod_constant(uint32_t d) {
    return ~0ull / d + 1;
}
__device__ __forceinline__ uint32_t fastmod(uint32_t a, uint64_t M, uint32_t d) {
    return uint32_t(__umul64hi(M * a, uint64_t(d)));
}

struct Derived {
    uint32_t t1;  // the tag as written in i1
    uint32_t t2;  // the tag as written in i2 (= t1 under XOR)
    uint32_t i1;
    uint32_t i2;
};

// offset(v) of Sec. 4.6.2: 1 + (lower 32 bits of H(v)) mod (m - 1), so that
// i2 != i1; 0 for a single bucket.
template <int HASH>
__device__ __forceinline__ uint32_t offset_of(uint32_t v, const Place &pl) {
    if (pl.m < 2) return 0;
    return 1u + fastmod(uint32_t(hash64<HASH>(uint64_t(v))), pl.m1div, pl.m1);
}

// (j + d) mod m and (j - d) mod m for j < m, d <= m - 1, without overflow.
__device__ __forceinline__ uint32_t add_mod(uint32_t j, uint32_t d, uint32_t m) {
    return j >= m - d ? j - (m - d) : j + d;
}
__device__ __forceinline__ uint32_t sub_mod(uint32_t j, uint32_t d, uint32_t m) {
    return j >= d ? j - d : j + (m - d);
}

// Eqs. (1)-(3) with the split of Sec. 4.3 step 1: upper 32 hash bits give
// the fingerprint, lower 32 bits the primary bucket.  Under XOR, i2 =
// i1 ^ (H(fp) mod m) and the tag is fp in both buckets; under the offset
// policy the fingerprint v has f - 1 bits, i2 = (i1 + offset(v)) mod m and
// the tag in i2 carries the choice bit (the slot's top bit).
template <class G, int HASH, int POL>
__device__ __forceinline__ Derived derive(uint64_t key, const Place &pl) {
    const uint64_t h = hash64<HASH>(key);
    Derived d;
    if constexpr (POL == 1) {
        constexpr uint32_t CB = 1u << (G::F - 1);
        uint32_t v = uint32_t(h >> 32) & (CB - 1u);
        v = v ? v : 1u;
        d.t1 = v;
        d.t2 = v | CB;
        d.i1 = fastmod(uint32_t(h), pl.mdiv, pl.m);
        d.i2 = add_mod(d.i1, offset_of<HASH>(v, pl), pl.m);
    } else {
        uint32_t fp = uint32_t(h >> 32) & G::FMASK;
        fp = fp ? fp : 1u;
        d.t1 = d.t2 = fp;
        d.i1 = uint32_t(h) & pl.mmask;
        d.i2 = d.i1 ^ (uint32_t(hash64<HASH>(uint64_t(fp))) & pl.mmask);
    }
    return d;
}

// The bucket a tag stored in j moves to, with `tag` rewritten as it is
// stored there: XOR leaves it; the offset policy flips the choice bit and
// goes forward from the primary bucket or back from the alternate one.
template <class G, int HASH, int POL>
__device__ __forceinline__ uint32_t move_tag(uint32_t j, uint32_t &tag, const Place &pl) {
    if constexpr (POL == 1) {
        constexpr uint32_t CB = 1u << (G::F - 1);
        const uint32_t off = offset_of<HASH>(tag & ~CB, pl);
        const bool in_alt = (tag & CB) != 0;
        tag ^= CB;
        return in_alt ? sub_mod(j, off, pl.m) : add_mod(j, off, pl.m);
    } else {
        return j ^ (uint32_t(hash64<HASH>(uint64_t(tag))) & pl.mmask);
    }
}

// -------------------------------------------------------- bucket registers

// A bucket's words held in registers.  Dynamic word indices are resolved by
// select chains so the array never spills to scratch memory.
template <class G>
struct Bucket {
    using W = typename G::W;
    W w[G::WPB];

    // Masked OR over the words rather than a select chain: the compiler turns
    // a select chain back into a dynamically indexed (scratch) array.
    __device__ __forceinline__ W get(int idx) const {
        W r = 0;
#pragma unroll
        for (int k = 0; k < G::WPB; ++k) r |= w[k] & (W(0) - W(idx == k));
        return r;
    }
    __device__ __forceinline__ void set(int idx, W v) {
#pragma unroll
        for (int k = 0; k < G::WPB; ++k) {
            const W m = W(0) - W(idx == k);
            w[k] = (w[k] & ~m) | (v & m);
        }
    }
    __device__ __forceinline__ uint32_t slot(int s) const {
        const W word = get(s / G::TPW);
        return uint32_t(word >> ((s % G::TPW) * G::F)) & G::FMASK;
    }
    // Bit k set iff word k has an empty lane.
    __device__ __forceinline__ uint32_t words_with_empty() const {
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < G::WPB; ++k)
            m |= (zero_lanes<W, G::F>(w[k]) != 0 ? 1u : 0u) << k;
        return m;
    }
    __device__ __forceinline__ bool has_empty() const {
        W acc = 0;
#pragma unroll
        for (int k = 0; k < G::WPB; ++k) acc |= zero_lanes<W, G::F>(w[k]);
        return acc != 0;
    }
    __device__ __forceinline__ bool contains(uint32_t tag) const {
        W acc = 0;
#pragma unroll
        for (int k = 0; k < G::WPB; ++k) acc |= match_lanes<W, G::F>(w[k], tag);
        return acc != 0;
    }
};

// Load bucket j's words with the widest loads the geometry allows
// (16-byte vector loads for buckets of two or more 64-bit words).
template <class G>
__device__ __forceinline__ void load_bucket(const typename G::W *table, uint32_t j,
                                            Bucket<G> &bk) {
    using W = typename G::W;
    const W *p = table + uint64_t(j) * G::WPB;
    if constexpr (sizeof(W) == 8 && G::WPB >= 2) {
        const ulonglong2 *v = reinterpret_cast<const ulonglong2 *>(p);
#pragma unroll
        for (int k = 0; k < G::WPB / 2; ++k) {
            ulonglong2 t = v[k];
            bk.w[2 * k] = t.x;
            bk.w[2 * k + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < G::WPB; ++k) bk.w[k] = p[k];
    }
}

// Word index at which the scan of a bucket for `tag` starts (Alg. 1/3:
// (tag mod b) / tagsPerWord), and the rotation of a per-word bit set into
// scan order.
template <class G>
__device__ __forceinline__ int scan_start(uint32_t tag) {
    return int((tag % uint32_t(G::B)) / uint32_t(G::TPW));
}

template <class G>
__device__ __forceinline__ int first_in_scan(uint32_t word_bits, int start) {
    constexpr uint32_t ALL = (G::WPB >= 32) ? 0xffffffffu : ((1u << G::WPB) - 1u);
    const uint32_t rot = ((word_bits >> start) | (word_bits << ((G::WPB - start) & 31))) & ALL;
    const int k = __builtin_ctz(rot);
    return (start + k) & (G::WPB - 1);
}

template <typename W>
__device__ __forceinline__ W cas_word(W *addr, W expected, W desired) {
    return atomicCAS(addr, expected, desired);
}

// Alg. 1 TryInsert on a bucket whose words are in `bk` (possibly stale):
// the first empty slot in scan order is claimed with a CAS; a failed CAS
// returns the word's current value, which replaces the stale copy before
// the search continues.  Returns the slot index, or -1 if the bucket is full.
template <class G>
__device__ __forceinline__ int try_insert(typename G::W *table, uint32_t j, uint32_t tag,
                                          Bucket<G> &bk) {
    using W = typename G::W;
    W *base = table + uint64_t(j) * G::WPB;
    const int start = scan_start<G>(tag);
    while (true) {
        const uint32_t have = bk.words_with_empty();
        if (have == 0) return -1;
        const int idx = first_in_scan<G>(have, start);
        const W w = bk.get(idx);
        const int lane = lowest_bit(zero_lanes<W, G::F>(w)) / G::F;
        const W desired = w | (W(tag) << (lane * G::F));
        const W old = cas_word(base + idx, w, desired);
        if (old == w) {
            bk.set(idx, desired);
            return idx * G::TPW + lane;
        }
        bk.set(idx, old);
    }
}

// Alg. 3 TryRemove: clear the first slot holding `tag` in scan order.  Alg. 3
// clears it with a CAS of the whole word, which fails (and costs another
// round trip) whenever any other slot of the word changed since the read.
// Deletes never run concurrently with inserts on a table (one operation kind
// per launch), so during a delete a slot can only go from a tag to empty:
// clearing just this slot with a fetch-AND either removes `tag` or changes
// nothing, and the word it returns says which.  The slots cleared are the
// same as with the CAS: for each key, the first match in scan order that no
// other delete took.
template <class G>
__device__ __forceinline__ bool try_remove(typename G::W *table, uint32_t j, uint32_t tag,
                                           Bucket<G> &bk) {
    using W = typename G::W;
    W *base = table + uint64_t(j) * G::WPB;
    const int start = scan_start<G>(tag);
    while (true) {
        uint32_t have = 0;
#pragma unroll
        for (int k = 0; k < G::WPB; ++k)
            have |= (match_lanes<W, G::F>(bk.w[k], tag) != 0 ? 1u : 0u) << k;
        if (have == 0) return false;
        const int idx = first_in_scan<G>(have, start);
        const W w = bk.get(idx);
        const int sh = (lowest_bit(match_lanes<W, G::F>(w, tag)) / G::F) * G::F;
        const W slot = W(G::FMASK) << sh;
        const W old = atomicAnd(base + idx, W(~slot));
        bk.set(idx, old & ~slot);
        if ((old & slot) == (W(tag) << sh)) return true;
    }
}

// Put `tag` into slot s of bucket j, but only while the slot still holds
// `expect` (BFS relocation, Sec. 4.6.1).  Returns true on success.
template <class G>
__device__ __forceinline__ bool replace_slot_if(typename G::W *table, uint32_t j, int s,
                                                uint32_t expect, uint32_t tag, Bucket<G> &bk) {
    using W = typename G::W;
    const int idx = s / G::TPW;
    const int sh = (s % G::TPW) * G::F;
    W *addr = table + uint64_t(j) * G::WPB + idx;
    W w = bk.get(idx);
    while ((uint32_t(w >> sh) & G::FMASK) == expect) {
        const W desired = (w & ~(W(G::FMASK) << sh)) | (W(tag) << sh);
        const W old = cas_word(addr, w, desired);
        if (old == w) {
            bk.set(idx, desired);
            return true;
        }
        w = old;
    }
    bk.set(idx, w);
    return false;
}

// Swap `tag` into slot s of bucket j whatever it holds (the eviction step of
// Alg. 1); returns the value displaced.
template <class G>
__device__ __forceinline__ uint32_t swap_slot(typename G::W *table, uint32_t j, int s,
                                              uint32_t tag, Bucket<G> &bk) {
    using W = typename G::W;
    const int idx = s / G::TPW;
    const int sh = (s % G::TPW) * G::F;
    W *addr = table + uint64_t(j) * G::WPB + idx;
    W w = bk.get(idx);
    while (true) {
        const W desired = (w & ~(W(G::FMASK) << sh)) | (W(tag) << sh);
        const W old = cas_word(addr, w, desired);
        if (old == w) {
            bk.set(idx, desired);
            return uint32_t(w >> sh) & G::FMASK;
        }
        w = old;
    }
}

}  // namespace cfk
