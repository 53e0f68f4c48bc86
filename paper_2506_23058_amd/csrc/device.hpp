// device.hpp -- gfx950 device primitives shared by the partition kernels.
//
// Wave64 building blocks (ballot / mbcnt ranks, DPP reductions), the
// predicates p that partition2 maps over the elements (Section 2.1), the
// tile loader, the in-tile rank computation, and the decoupled look-back over
// tile descriptors that turns per-tile true counts into exclusive prefixes
// (partition2's scan of the true flags, Section 2.1).
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

// Index of this thread's wave inside the workgroup, as a wave-uniform value.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

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

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), lane));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), lane));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Tile of workgroup b among nt tiles in an XCD-aware order.  The hardware
// deals workgroups round-robin to the 8 XCDs; this gives each XCD one
// contiguous range of tiles (the first nt - 8 (per - 1) XCDs take `per`
// tiles, the others per - 1), so neighbouring tiles' output runs and the
// partial cache lines between them meet in one L2.  A bijection of [0, nt).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nt) {
    const int64_t per = (nt + 7) / 8;
    const int64_t x = b % 8, k = b / 8;
    const int64_t full = nt - (per - 1) * 8;   // XCDs that take `per` tiles
    return x < full ? x * per + k : full * per + (x - full) * (per - 1) + k;
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
    // the predicate of row k (this one does not depend on the row)
    __device__ __forceinline__ PredModEq at_row(int64_t) const { return *this; }
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
    __device__ __forceinline__ PredLt at_row(int64_t) const { return *this; }
    __device__ __forceinline__ bool operator()(uint32_t bits, uint8_t) const {
        return __uint_as_float(bits) < s;
    }
};

// A caller-supplied flag array (partition2L's csL): true where the byte != 0.
struct PredFlags {
    static constexpr bool kUsesFlags = true;
    const uint8_t *flags;
    __device__ __forceinline__ PredFlags at_row(int64_t) const { return *this; }
    __device__ __forceinline__ bool operator()(uint32_t, uint8_t f) const { return f != 0; }
};

// Predicates of the row number k (segmented calls): at_row(k) fixes k and
// returns a predicate of the key alone.
// x < row_s[k] in IEEE single precision.
struct PredLtRow {
    static constexpr bool kUsesFlags = false;
    const float *row_s;
    float s;
    __device__ __forceinline__ PredLtRow at_row(int64_t k) const { return PredLtRow{row_s, row_s[k]}; }
    __device__ __forceinline__ bool operator()(uint32_t bits, uint8_t) const {
        return __uint_as_float(bits) < s;
    }
};

// x mod d == k mod d, floor moduli (k >= 0, so k mod d is the remainder).
struct PredModRow {
    static constexpr bool kUsesFlags = false;
    PredModEq eq;
    __device__ __forceinline__ PredModRow at_row(int64_t k) const {
        PredModRow p = *this;
        p.eq.r = static_cast<int64_t>(static_cast<uint64_t>(k) % eq.d);
        return p;
    }
    __device__ __forceinline__ bool operator()(uint32_t bits, uint8_t f) const { return eq(bits, f); }
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
// `t` over the tiles [first, t) of the same scan.  Each round reads the
// 64*LOADS nearest unread predecessors at once (lane i, load u reads tile
// j - 64u - i), then walks the 64-wide windows in order: a window is summed
// with a DPP reduction when every tile up to its nearest inclusive prefix has
// published; at an unpublished one the walk re-reads from there (with a short
// sleep).  Aggregates are below 2^32; an inclusive prefix may be any 62-bit
// value and is added separately.  With WIDE = false a window's aggregates
// must also sum below 2^32 (64 tiles of at most 2^26 each); WIDE sums the low
// and high 16-bit halves apart, so 64 aggregates of up to 2^32 - 1 add without
// wrapping.  Tiles before `first` behave as an inclusive prefix of 0.
template <int LOADS = 4, bool WIDE = false>
__device__ __forceinline__ int64_t lookback(const uint64_t *desc, int64_t t,
                                            int64_t first, int32_t *err) {
    const int lane = lane_id();
    int64_t excl = 0;
    int64_t j = t - 1;
    uint32_t spins = 0;
    while (j >= first) {
        uint64_t d[LOADS];
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            const int64_t i = j - u * kWave - lane;
            d[u] = i >= first ? desc_load(desc + i) : kStP;
        }
        bool done = false, stalled = false;
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            if (done || stalled) continue;
            const uint32_t st = static_cast<uint32_t>(d[u] >> 62);
            const uint64_t mX = ballot(st == 0);
            const uint64_t mP = ballot(st == 2);
            const uint64_t upto = mP ? (((mP & (~mP + 1)) << 1) - 1) : ~0ull;
            if (mX & upto) {
                stalled = true;
                continue;
            }
            const int firstP = mP ? __builtin_ctzll(mP) : kWave;
            const bool in = (upto >> lane) & 1ull;
            const uint32_t small = (in && lane != firstP) ? static_cast<uint32_t>(d[u] & kValMask) : 0u;
            if constexpr (WIDE) {
                excl += static_cast<int64_t>(wave_sum_u32(small & 0xFFFFu)) +
                        (static_cast<int64_t>(wave_sum_u32(small >> 16)) << 16);
            } else {
                excl += wave_sum_u32(small);
            }
            if (mP) {
                excl += static_cast<int64_t>(readlane_u64(d[u] & kValMask, firstP));
                done = true;
            } else {
                j -= kWave;
            }
        }
        if (done) break;
        if (stalled) {
            if (++spins > kSpinLimit) {
                if (lane == 0) set_error(err, kErrSpin);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// ------------------------------------------------------------ streaming loads --
// Input keys and flags are read exactly once: nontemporal loads keep them from
// displacing reusable lines in the caches.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int VEC>
__device__ __forceinline__ void load_group(const uint32_t *p, uint32_t (&out)[VEC]) {
    if constexpr (VEC == 4) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        out[0] = __builtin_nontemporal_load(p);
    }
}

template <int VEC>
__device__ __forceinline__ void load_flags(const uint8_t *p, uint8_t (&out)[VEC]) {
    if constexpr (VEC == 4) {
        const uint32_t w = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p));
#pragma unroll
        for (int q = 0; q < VEC; ++q) out[q] = static_cast<uint8_t>(w >> (8 * q));
    } else {
        out[0] = *p;
    }
}

// Outputs are written once and not read again by the kernel: stores may be
// marked nontemporal (streamed past the caches).
#ifndef IXP_NT_STORES
#define IXP_NT_STORES 1
#endif

template <class T>
__device__ __forceinline__ void stream_store(T *p, T v) {
#if IXP_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// ----------------------------------------------------------------- the tile --
// A tile is BLOCK threads x ROWS rows x VEC consecutive elements.  Wave w owns
// the contiguous run [base + w*ROWS*64*VEC, +ROWS*64*VEC); inside it row r,
// lane l holds elements base + w*ROWS*64*VEC + r*64*VEC + l*VEC + q, q < VEC.
// Only positions in [lo, hi) are valid; invalid ones are never stored.
// Bits holds one flag bit per element of a thread; a 32-bit word (enough for
// ROWS * VEC <= 32) keeps the flag arithmetic in single registers.
template <int BLOCK, int ROWS, int VEC, class Bits = uint64_t>
struct Tile {
    static constexpr int kWaves = BLOCK / kWave;
    static constexpr int kPerWave = ROWS * kWave * VEC;
    static constexpr int kSize = BLOCK * ROWS * VEC;
    static_assert(BLOCK % kWave == 0 && BLOCK <= 1024, "block");
    static_assert(VEC == 1 || VEC == 4, "vec");
    static_assert(ROWS * VEC <= 8 * static_cast<int>(sizeof(Bits)), "flag bits");

    uint32_t key[ROWS][VEC];
    uint32_t rank[ROWS][VEC];   // exclusive rank among the tile's trues
    Bits fbits = 0;             // bit r*VEC+q: element is valid and true
    Bits vbits = 0;             // bit r*VEC+q: element is valid
    uint32_t wave_total = 0;    // trues of this wave (uniform)

    __device__ static __forceinline__ int64_t pos(int64_t base, int wave, int r, int lane, int q) {
        return base + static_cast<int64_t>(wave) * kPerWave + r * (kWave * VEC) + lane * VEC + q;
    }

    // Loads keys (if need_keys) and flag bytes (for a flag predicate) of the
    // valid positions and evaluates the predicate.
    //
    // Three paths, chosen per tile (wave-uniform): a full tile issues one
    // unconditional nontemporal vector load per row from one base address; a
    // partial tile (except one holding the array's incomplete last vector
    // group) does the same, but rows that miss [lo, hi) re-read the group
    // containing lo instead (a cache hit), so the loads still form one
    // branch-free batch; the tile holding the incomplete last group uses
    // element-wise guarded loads.
    template <class Pred>
    __device__ __forceinline__ void load(const uint32_t *keys, int64_t n, int64_t base,
                                         int64_t lo, int64_t hi, const Pred &pred,
                                         bool need_keys, int wave, int lane) {
        const bool tail = VEC > 1 && (n & (VEC - 1)) != 0 && hi > (n & ~static_cast<int64_t>(VEC - 1));
        uint32_t kv[ROWS][VEC];
        uint8_t fv[ROWS][VEC];
        if (base >= lo && base + kSize <= hi) {
            // whole tile valid: plain strided addresses (immediate offsets)
            const uint32_t *kp = keys + pos(base, wave, 0, lane, 0);
            const uint8_t *fp = nullptr;
            if constexpr (Pred::kUsesFlags) fp = pred.flags + pos(base, wave, 0, lane, 0);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                if (need_keys) load_group(kp + r * (kWave * VEC), kv[r]);
                else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) kv[r][q] = 0;
                }
                if constexpr (Pred::kUsesFlags) load_flags(fp + r * (kWave * VEC), fv[r]);
                else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) fv[r][q] = 0;
                }
            }
        } else if (!tail) {
            const int64_t park = lo & ~static_cast<int64_t>(VEC - 1);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t p0 = pos(base, wave, r, lane, 0);
                const bool live = p0 + VEC > lo && p0 < hi;
                const int64_t src = live ? p0 : park;
                if (need_keys) load_group(keys + src, kv[r]);
                else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) kv[r][q] = 0;
                }
                if constexpr (Pred::kUsesFlags) load_flags(pred.flags + src, fv[r]);
                else {
#pragma unroll
                    for (int q = 0; q < VEC; ++q) fv[r][q] = 0;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t p0 = pos(base, wave, r, lane, 0);
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const int64_t p = p0 + q;
                    const bool ok = p >= lo && p < hi;
                    kv[r][q] = (need_keys && ok) ? keys[p] : 0u;
                    if constexpr (Pred::kUsesFlags) fv[r][q] = ok ? pred.flags[p] : 0;
                    else fv[r][q] = 0;
                }
            }
        }
        // validity from 32-bit offsets relative to lo (a tile spans < 2^31)
        const int32_t l0 = static_cast<int32_t>(base - lo) + wave * kPerWave + lane * VEC;
        const uint32_t span = static_cast<uint32_t>(hi - lo);
        // The words are built by shifting in one bit per element, last
        // element first: a per-element mask constant would hold a register of
        // its own (a select with a literal has no encoding here), and every
        // predicate is plain arithmetic, so no branch guards it.
#pragma unroll
        for (int k = ROWS * VEC - 1; k >= 0; --k) {
            const int r = k / VEC, q = k % VEC;
            const int32_t l = l0 + r * (kWave * VEC) + q;
            const bool valid = static_cast<uint32_t>(l) < span;
            key[r][q] = kv[r][q];
            const bool f = valid & pred(kv[r][q], fv[r][q]);
            vbits = (vbits << 1) | static_cast<Bits>(valid);
            fbits = (fbits << 1) | static_cast<Bits>(f);
        }
        (void)n;
    }

    // True when this wave's run of the tile meets [lo, hi) (wave-uniform).
    __device__ static __forceinline__ bool wave_live(int64_t base, int64_t lo, int64_t hi, int wave) {
        const int64_t w0 = base + static_cast<int64_t>(wave) * kPerWave;
        return w0 < hi && w0 + kPerWave > lo;
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
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    if (VEC == 1) {
        if (valid_mask & 1u) stream_store(out + p0, v[0]);
    } else if (valid_mask == 0xFu) {
        if constexpr (sizeof(Idx) == 4) {
            u32x4 w;
            w.x = static_cast<uint32_t>(v[0]); w.y = static_cast<uint32_t>(v[1 % VEC]);
            w.z = static_cast<uint32_t>(v[2 % VEC]); w.w = static_cast<uint32_t>(v[3 % VEC]);
            stream_store(reinterpret_cast<u32x4 *>(out + p0), w);
        } else {
            u64x2 a, b;
            a.x = static_cast<uint64_t>(v[0]); a.y = static_cast<uint64_t>(v[1 % VEC]);
            b.x = static_cast<uint64_t>(v[2 % VEC]); b.y = static_cast<uint64_t>(v[3 % VEC]);
            stream_store(reinterpret_cast<u64x2 *>(out + p0), a);
            stream_store(reinterpret_cast<u64x2 *>(out + p0) + 1, b);
        }
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q)
            if ((valid_mask >> q) & 1u) stream_store(out + p0 + q, v[q]);
    }
}

// Writes the run stage[src, src+len) to out[g, g+len): a head of up to three
// elements up to the next 16-byte boundary of out + g, 16-byte stores for the
// aligned body, then the tail.
template <int BLOCK>
__device__ __forceinline__ void write_run(const uint32_t *stage, uint32_t src, uint32_t len, int64_t g,
                                          uint32_t *out, int64_t n, int tid) {
    if (len == 0) return;
    // elements until out + g reaches a 16-byte boundary (out is 4-byte aligned)
    const uint32_t mis = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(out + g) >> 2) & 3);
    const uint32_t to16 = (4 - mis) & 3;
    const uint32_t head = to16 < len ? to16 : len;
    const uint32_t groups = (len - head) / 4;
    const uint32_t tail = len - head - 4 * groups;
    for (uint32_t j = tid; j < groups; j += BLOCK) {
        const uint32_t s = src + head + 4 * j;
        u32x4 v;
        v.x = stage[s]; v.y = stage[s + 1]; v.z = stage[s + 2]; v.w = stage[s + 3];
        const int64_t d = g + head + 4 * static_cast<int64_t>(j);
        if (d + 4 <= n) stream_store(reinterpret_cast<u32x4 *>(out + d), v);
    }
    if (static_cast<uint32_t>(tid) < head && g + tid < n) stream_store(out + g + tid, stage[src + tid]);
    if (static_cast<uint32_t>(tid) < tail) {
        const uint32_t k = head + 4 * groups + tid;
        if (g + k < n) stream_store(out + g + k, stage[src + k]);
    }
}

}  // namespace ixp
