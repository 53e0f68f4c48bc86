// device.hpp -- gfx950 device primitives shared by the partition kernels.
//
// Wave64 building blocks (ballot / mbcnt ranks, DPP reductions), the
// predicates p of `cs = map p xs` (Section 2.1), the tile loader, the in-tile
// rank computation, and the decoupled look-back over tile descriptors that
// turns per-tile true counts into exclusive prefixes (the `scan (+) 0 flagsT`
// of partition2, Section 2.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ixp {

constexpr int kWave = 64;

// ---------------------------------------------------------------- wave ops --

__device__ __forceinline__ uint64_t ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// Number of set bits of `m` in lanes strictly below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ int lane_id() { return static_cast<int>(rank_below(~0ull)); }

// DPP row_ror:k control code (rotate right by k inside each 16-lane row).
template <int K>
__device__ __forceinline__ uint32_t dpp_row_ror(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        0, static_cast<int>(v), 0x120 + K, 0xF, 0xF, false));
}

// Sum of a 32-bit value over the 64 lanes, returned wave-uniform.  Four DPP
// rotate-and-add steps give every lane its row's sum; the four row sums are
// then read from lanes 0, 16, 32 and 48.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += dpp_row_ror<8>(v);
    v += dpp_row_ror<4>(v);
    v += dpp_row_ror<2>(v);
    v += dpp_row_ror<1>(v);
    const int iv = static_cast<int>(v);
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(iv, 0)) +
           static_cast<uint32_t>(__builtin_amdgcn_readlane(iv, 16)) +
           static_cast<uint32_t>(__builtin_amdgcn_readlane(iv, 32)) +
           static_cast<uint32_t>(__builtin_amdgcn_readlane(iv, 48));
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), lane));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), lane));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// ---------------------------------------------------------------- predicates --
// Keys travel as raw 32-bit words; each predicate interprets them.

// x mod d == r with the floor modulus, for int32 x and 1 <= d < 2^32.
// |x| mod d uses the direct-remainder method of Lemire, Kaser and Kurz
// ("Faster Remainder by Direct Computation", 2019): with M = floor((2^64-1)/d)+1,
// a mod d = high64((M * a mod 2^64) * d), exact for all 32-bit a and d.
struct PredModEq {
    static constexpr bool kUsesFlags = false;
    uint64_t M;
    uint32_t d;
    int64_t r;
    __device__ __forceinline__ bool operator()(uint32_t bits, uint8_t) const {
        const int32_t x = static_cast<int32_t>(bits);
        const uint32_t a = x < 0 ? 0u - bits : bits;   // |x|, 2^31 for INT_MIN
        const uint32_t m = static_cast<uint32_t>(__umul64hi(M * a, d));
        const uint32_t fm = (x < 0 && m != 0) ? d - m : m;
        return static_cast<int64_t>(fm) == r;
    }
};

// x < s in IEEE single precision (NaN compares false).
struct PredLt {
    static constexpr bool kUsesFlags = false;
    float s;
    __device__ __forceinline__ bool operator()(uint32_t bits, uint8_t) const {
        return __uint_as_float(bits) < s;
    }
};

// A caller-supplied flag array (partition2L's csL): true where the byte != 0.
struct PredFlags {
    static constexpr bool kUsesFlags = true;
    const uint8_t *flags;
    __device__ __forceinline__ bool operator()(uint32_t, uint8_t f) const { return f != 0; }
};

// ---------------------------------------------------------- tile descriptors --
// One 64-bit word per tile: status in bits 63..62, value in bits 61..0.
//   0 = nothing published yet, 1 = the tile's own count (aggregate),
//   2 = inclusive prefix (count of all earlier tiles of the scan plus its own).
constexpr uint64_t kStA = 1ull << 62;
constexpr uint64_t kStP = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t desc_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void desc_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Error word in the workspace: 1 = a look-back wait gave up (device error),
// 2 = invalid segment shape.
constexpr int32_t kErrSpin = 1;
constexpr int32_t kErrShape = 2;

__device__ __forceinline__ void set_error(int32_t *err, int32_t code) {
    __hip_atomic_fetch_or(err, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bound on the number of consecutive look-back polls that find an unpublished
// predecessor.  Predecessors always run (tile numbers are handed out in launch
// order), so the bound only guarantees that every wave exits.
constexpr uint32_t kSpinLimit = 1u << 22;

// Decoupled look-back, executed by one full wave: the exclusive prefix of tile
// `t` over the tiles [first, t) of the same scan.  Each step reads the 64
// nearest unread predecessors at once (lane i reads tile j - i), waits while
// any of them up to the nearest inclusive prefix is unpublished, and sums the
// window with a DPP reduction.  Aggregates are below 2^32; an inclusive prefix
// may be any 62-bit value and is added separately.  Tiles before `first`
// behave as an inclusive prefix of 0.
__device__ __forceinline__ int64_t lookback(const uint64_t *desc, int64_t t,
                                            int64_t first, int32_t *err) {
    const int lane = lane_id();
    int64_t excl = 0;
    int64_t j = t - 1;
    uint32_t spins = 0;
    while (j >= first) {
        const int64_t i = j - lane;
        const uint64_t d = i >= first ? desc_load(desc + i) : kStP;
        const uint32_t st = static_cast<uint32_t>(d >> 62);
        const uint64_t mX = ballot(st == 0);
        const uint64_t mP = ballot(st == 2);
        const uint64_t upto = mP ? (((mP & (~mP + 1)) << 1) - 1) : ~0ull;
        if (mX & upto) {
            if (++spins > kSpinLimit) {
                if (lane == 0) set_error(err, kErrSpin);
                return excl;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        const int firstP = mP ? __builtin_ctzll(mP) : kWave;
        const bool in = (upto >> lane) & 1ull;
        const uint32_t small = (in && lane != firstP) ? static_cast<uint32_t>(d & kValMask) : 0u;
        excl += wave_sum_u32(small);
        if (mP) {
            excl += static_cast<int64_t>(readlane_u64(d & kValMask, firstP));
            break;
        }
        j -= kWave;
    }
    return excl;
}

// ----------------------------------------------------------------- the tile --
// A tile is BLOCK threads x ROWS rows x VEC consecutive elements.  Wave w owns
// the contiguous run [base + w*ROWS*64*VEC, +ROWS*64*VEC); inside it row r,
// lane l holds elements base + w*ROWS*64*VEC + r*64*VEC + l*VEC + q, q < VEC.
// Only positions in [lo, hi) are valid; invalid ones are never stored.
template <int BLOCK, int ROWS, int VEC>
struct Tile {
    static constexpr int kWaves = BLOCK / kWave;
    static constexpr int kPerWave = ROWS * kWave * VEC;
    static constexpr int kSize = BLOCK * ROWS * VEC;
    static_assert(BLOCK % kWave == 0 && BLOCK <= 1024, "block");
    static_assert(VEC == 1 || VEC == 4, "vec");
    static_assert(ROWS * VEC <= 32, "flag bits");

    uint32_t key[ROWS][VEC];
    uint32_t rank[ROWS][VEC];   // exclusive rank among the tile's trues
    uint32_t fbits = 0;         // bit r*VEC+q: element is valid and true
    uint32_t vbits = 0;         // bit r*VEC+q: element is valid
    uint32_t wave_total = 0;    // trues of this wave (uniform)

    __device__ static __forceinline__ int64_t pos(int64_t base, int wave, int r, int lane, int q) {
        return base + static_cast<int64_t>(wave) * kPerWave + r * (kWave * VEC) + lane * VEC + q;
    }

    // Loads keys (if need_keys) and flag bytes (for a flag predicate) of the
    // valid positions and evaluates the predicate.  Groups of VEC elements
    // that lie fully inside [0, n) and are VEC-aligned use one vector load.
    template <class Pred>
    __device__ __forceinline__ void load(const uint32_t *keys, int64_t n, int64_t base,
                                         int64_t lo, int64_t hi, const Pred &pred,
                                         bool need_keys, int wave, int lane) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int64_t p0 = pos(base, wave, r, lane, 0);
            uint32_t kv[VEC];
            uint8_t fv[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) { kv[q] = 0; fv[q] = 0; }
            const bool any = p0 + VEC > lo && p0 < hi;
            const bool full = p0 >= lo && p0 + VEC <= hi;
            if (any) {
                if (VEC == 4 && full) {
                    if (need_keys) {
                        const uint4 v = *reinterpret_cast<const uint4 *>(keys + p0);
                        kv[0] = v.x; kv[1 % VEC] = v.y; kv[2 % VEC] = v.z; kv[3 % VEC] = v.w;
                    }
                    if constexpr (Pred::kUsesFlags) {
                        const uint32_t w = *reinterpret_cast<const uint32_t *>(pred.flags + p0);
#pragma unroll
                        for (int q = 0; q < VEC; ++q) fv[q] = static_cast<uint8_t>(w >> (8 * q));
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const int64_t p = p0 + q;
                        if (p >= lo && p < hi) {
                            if (need_keys) kv[q] = keys[p];
                            if constexpr (Pred::kUsesFlags) fv[q] = pred.flags[p];
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const int64_t p = p0 + q;
                const bool valid = p >= lo && p < hi;
                key[r][q] = kv[q];
                const bool f = valid && pred(kv[q], fv[q]);
                vbits |= static_cast<uint32_t>(valid) << (r * VEC + q);
                fbits |= static_cast<uint32_t>(f) << (r * VEC + q);
            }
        }
        (void)n;
    }

    __device__ __forceinline__ bool flag(int r, int q) const { return (fbits >> (r * VEC + q)) & 1u; }
    __device__ __forceinline__ bool valid(int r, int q) const { return (vbits >> (r * VEC + q)) & 1u; }

    // Ranks of the trues inside this wave's run, from one ballot per
    // (row, q): the rank of element (r, lane, q) counts the trues of earlier
    // rows, of lower lanes in row r, and of q' < q in its own lane.
    __device__ __forceinline__ void wave_ranks() {
        uint32_t acc = 0;   // uniform
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            uint32_t below = 0, row_total = 0, mine = 0;
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const uint64_t m = ballot(flag(r, q));
                below += rank_below(m);
                row_total += static_cast<uint32_t>(__builtin_popcountll(m));
            }
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                rank[r][q] = acc + below + mine;
                mine += flag(r, q) ? 1u : 0u;
            }
            acc += row_total;
        }
        wave_total = acc;
    }

    // Count of trues in this wave's run (uniform), without ranks.
    __device__ __forceinline__ uint32_t wave_count() const {
        uint32_t acc = 0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int q = 0; q < VEC; ++q)
                acc += static_cast<uint32_t>(__builtin_popcountll(ballot(flag(r, q))));
        return acc;
    }

    // Combines the waves: returns the tile's true count and adds each wave's
    // exclusive offset to its ranks.  `wtot` is LDS of kWaves words.  Starts
    // and ends with a barrier-separated exchange.
    __device__ __forceinline__ uint32_t block_ranks(uint32_t *wtot, int wave, int lane) {
        if (lane == 0) wtot[wave] = wave_total;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = wtot[w];
            before += w < wave ? v : 0u;
            total += v;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int q = 0; q < VEC; ++q) rank[r][q] += before;
        return total;
    }
};

// Stores one VEC group of indices: a vector store when the whole group is
// valid (and so VEC-aligned), else element by element.
template <int VEC, class Idx>
__device__ __forceinline__ void store_idx_group(Idx *out, int64_t p0, const Idx (&v)[VEC],
                                                uint32_t valid_mask) {
    if (VEC == 4 && valid_mask == 0xFu) {
        if constexpr (sizeof(Idx) == 4) {
            uint4 w;
            w.x = static_cast<uint32_t>(v[0]); w.y = static_cast<uint32_t>(v[1 % VEC]);
            w.z = static_cast<uint32_t>(v[2 % VEC]); w.w = static_cast<uint32_t>(v[3 % VEC]);
            *reinterpret_cast<uint4 *>(out + p0) = w;
        } else {
            ulonglong2 a, b;
            a.x = static_cast<uint64_t>(v[0]); a.y = static_cast<uint64_t>(v[1 % VEC]);
            b.x = static_cast<uint64_t>(v[2 % VEC]); b.y = static_cast<uint64_t>(v[3 % VEC]);
            reinterpret_cast<ulonglong2 *>(out + p0)[0] = a;
            reinterpret_cast<ulonglong2 *>(out + p0)[1] = b;
        }
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
            if ((valid_mask >> q) & 1u) out[p0 + q] = v[q];
    }
}

}  // namespace ixp
