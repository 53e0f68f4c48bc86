// flatv.hip -- v-way stable partition on gfx950 (FiltPart with v pairwise
// exclusive predicates, Section 2.3; partition3 of Section 6 is v = 3).
//
// Element i has a class c(i) in [0, v); class 0 comes first, then class 1,
// and so on, each class in input order:
//   idx[i] = B_{c(i)} + (number of earlier elements of class c(i)),
//   B_c = N_0 + ... + N_{c-1},   N_c = size of class c.
// It is partition2 with v - 1 counters instead of one.  Three kernels, as for
// partition2:
//   count   -- one wave per contiguous run of tiles: per-class counts by
//              ballot + popcount, each tile's per-class prefix inside its run
//              and the run totals;
//   scan    -- one workgroup: exclusive scan of the run totals of every
//              class but the last, and the class sizes N_c;
//   scatter -- one workgroup per tile: per-class in-tile ranks from one
//              ballot per class and (row, quad), indices in input order, keys
//              staged in LDS class by class and written as v contiguous runs.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr int kVBlockThreads = 256;   // scatter tile: 256 threads x 4 rows x 4
constexpr int kVRows = 4;
constexpr int64_t kVCountWaves = 8192;
constexpr size_t kVHeader = 256;

// ------------------------------------------------------------------ classes --
// floor-mod(key, v) of an int32 key (the direct-remainder method of Lemire,
// Kaser and Kurz, as for the modulus predicate).
struct ClassMod {
    static constexpr bool kUsesBytes = false;
    uint64_t M;
    uint32_t d;
    __device__ __forceinline__ uint32_t operator()(uint32_t bits, uint8_t) const {
        const int32_t x = static_cast<int32_t>(bits);
        const uint32_t a = x < 0 ? 0u - bits : bits;
        const uint32_t m = static_cast<uint32_t>(__umul64hi(M * a, d));
        return (x < 0 && m != 0) ? d - m : m;
    }
};

// f32 thresholds s0 <= s1 <= s2: class h for s_{h-1} <= x < s_h, the last
// class for x >= s_{v-2} and for NaN (which no earlier predicate takes).
template <int V>
struct ClassThresh {
    static constexpr bool kUsesBytes = false;
    float s0, s1, s2;
    __device__ __forceinline__ uint32_t operator()(uint32_t bits, uint8_t) const {
        const float x = __uint_as_float(bits);
        if (x < s0) return 0;
        if (V > 2 && x < s1) return 1;
        if (V > 3 && x < s2) return 2;
        return V - 1;
    }
};

// A caller byte per element; values past the last class count as the last.
template <int V>
struct ClassBytes {
    static constexpr bool kUsesBytes = true;
    const uint8_t *cls;
    __device__ __forceinline__ uint32_t operator()(uint32_t, uint8_t b) const {
        return b < V - 1 ? b : V - 1;
    }
};

// a[c] for a class c < V, as a[0] plus the steps a[k] - a[k-1] of every
// k <= c.  Compares and adds only: a chain of selects on c == k is turned by
// the compiler into an indexed load from a per-lane scratch copy of a[].
template <int V, class T>
struct Picker {
    T a0;
    T step[V - 1];
    __device__ __forceinline__ explicit Picker(const T (&a)[V]) : a0(a[0]) {
#pragma unroll
        for (int k = 1; k < V; ++k) step[k - 1] = a[k] - a[k - 1];
    }
    __device__ __forceinline__ T operator()(uint32_t c) const {
        T r = a0;
#pragma unroll
        for (int k = 1; k < V; ++k) r += c >= static_cast<uint32_t>(k) ? step[k - 1] : T{0};
        return r;
    }
};

// --------------------------------------------------------------------- tile --
// Same element layout as the partition2 tile (wave w owns a contiguous run,
// row r, lane l, quad q); the class of each element is kept as two bit planes.
template <int BLOCK, int ROWS, int V>
struct TileV {
    static constexpr int kWaves = BLOCK / kWave;
    static constexpr int kPerWave = ROWS * kWave * 4;
    static constexpr int kSize = BLOCK * ROWS * 4;
    static_assert(ROWS * 4 <= 32, "class bit planes");

    uint32_t key[ROWS][4];
    uint32_t rank[ROWS][4];   // rank among the tile's elements of the same class
    uint32_t c0 = 0, c1 = 0, vbits = 0;
    uint64_t wtotal = 0;   // packed per-class counts of this wave's run

    __device__ static __forceinline__ int64_t pos(int64_t base, int wave, int r, int lane) {
        return base + static_cast<int64_t>(wave) * kPerWave + r * (kWave * 4) + lane * 4;
    }
    __device__ __forceinline__ uint32_t cls(int r, int q) const {
        const int i = r * 4 + q;
        return ((c0 >> i) & 1u) | (((c1 >> i) & 1u) << 1);
    }
    __device__ __forceinline__ bool valid(int r, int q) const { return (vbits >> (r * 4 + q)) & 1u; }

    // Keys (if need_keys) and class bytes (for byte classes) of [lo, hi):
    // one unconditional 16-byte load per row for whole tiles, parked loads
    // for partial tiles, guarded element loads where the array's last group
    // is incomplete.
    template <class Cls>
    __device__ __forceinline__ void load(const uint32_t *keys, int64_t n, int64_t base, int64_t lo, int64_t hi,
                                         const Cls &cl, bool need_keys, int wave, int lane) {
        const bool tail = (n & 3) != 0 && hi > (n & ~int64_t{3});
        uint32_t kv[ROWS][4];
        uint8_t bv[ROWS][4];
        if (!tail) {
            const bool whole = base >= lo && base + kSize <= hi;
            const int64_t park = lo & ~int64_t{3};
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t p0 = pos(base, wave, r, lane);
                const bool live = whole || (p0 + 4 > lo && p0 < hi);
                const int64_t src = live ? p0 : park;
                uint32_t k4[4];
                if (need_keys) load_group<4>(keys + src, k4);
                else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) k4[q] = 0;
                }
                uint8_t b4[4] = {0, 0, 0, 0};
                if constexpr (Cls::kUsesBytes) load_flags<4>(cl.cls + src, b4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    kv[r][q] = k4[q];
                    bv[r][q] = b4[q];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t p0 = pos(base, wave, r, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t p = p0 + q;
                    const bool ok = p >= lo && p < hi;
                    kv[r][q] = (need_keys && ok) ? keys[p] : 0u;
                    if constexpr (Cls::kUsesBytes) bv[r][q] = ok ? cl.cls[p] : 0;
                    else bv[r][q] = 0;
                }
            }
        }
        const int32_t l0 = static_cast<int32_t>(base - lo) + wave * kPerWave + lane * 4;
        const uint32_t span = static_cast<uint32_t>(hi - lo);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t l = l0 + r * (kWave * 4) + q;
                const bool ok = static_cast<uint32_t>(l) < span;
                key[r][q] = kv[r][q];
                const uint32_t c = ok ? cl(kv[r][q], bv[r][q]) : 0u;
                const int i = r * 4 + q;
                vbits |= static_cast<uint32_t>(ok) << i;
                c0 |= (c & 1u) << i;
                c1 |= ((c >> 1) & 1u) << i;
            }
        }
    }

    // One-hot counters packed 16 bits per class in a 64-bit word (a class
    // holds at most 4096 elements of a tile, so no field overflows).
    __device__ __forceinline__ uint64_t onehot(int r, int q) const {
        return valid(r, q) ? (1ull << (16 * cls(r, q))) : 0ull;
    }
    __device__ static __forceinline__ uint32_t field(uint64_t x, uint32_t c) {
        return static_cast<uint32_t>(x >> (16 * c)) & 0xFFFFu;
    }

    // Per-class counts of this wave's valid elements (uniform), packed.
    __device__ __forceinline__ uint64_t wave_counts() const {
        uint64_t x = 0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) x += onehot(r, q);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
        return x;
    }

    // Ranks inside this wave's run.  Per row, the counts of every class but
    // the last are packed 9 bits each into 32 bits (a row of a wave holds at
    // most 256 elements) and scanned over the lanes with shuffles; the rank
    // of a last-class element is its position minus the earlier elements of
    // the other classes (the valid elements of a run form a prefix).
    __device__ static __forceinline__ uint32_t onehot9(uint32_t c, bool ok) {
        return (ok && c < static_cast<uint32_t>(V - 1)) ? (1u << (9 * c)) : 0u;
    }
    __device__ __forceinline__ void wave_ranks(int lane) {
        uint64_t acc = 0;   // packed 16-bit counts of the earlier rows (uniform)
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            uint32_t mine = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) mine += onehot9(cls(r, q), valid(r, q));
            uint32_t inc = mine;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t o = __shfl_up(inc, off, kWave);
                if (lane >= off) inc += o;
            }
            uint32_t run = inc - mine;
            const uint32_t pos0 = static_cast<uint32_t>(r * kWave * 4 + lane * 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t c = cls(r, q);
                uint32_t others = 0;   // earlier elements of the classes before the last
#pragma unroll
                for (int k = 0; k < V - 1; ++k) others += field(acc, k) + ((run >> (9 * k)) & 0x1FFu);
                const uint32_t mine_c = c < static_cast<uint32_t>(V - 1)
                                            ? field(acc, c) + ((run >> (9 * c)) & 0x1FFu)
                                            : pos0 + q - others;
                rank[r][q] = mine_c;
                run += onehot9(c, valid(r, q));
            }
            const uint32_t row = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(inc), kWave - 1));
#pragma unroll
            for (int k = 0; k < V - 1; ++k) acc += static_cast<uint64_t>((row >> (9 * k)) & 0x1FFu) << (16 * k);
        }
        // the last class of the run: valid elements minus the others
        uint32_t nvalid = static_cast<uint32_t>(__builtin_popcount(vbits));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nvalid += __shfl_xor(nvalid, off, kWave);
        uint32_t others = 0;
#pragma unroll
        for (int k = 0; k < V - 1; ++k) others += field(acc, k);
        wtotal = acc + (static_cast<uint64_t>(nvalid - others) << (16 * (V - 1)));
    }

    // Adds each wave's per-class offset to its ranks; returns the tile's
    // packed class sizes.
    __device__ __forceinline__ uint64_t block_ranks(uint64_t *wt, int wave, int lane) {
        if (lane == 0) wt[wave] = wtotal;
        __syncthreads();
        uint64_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint64_t x = wt[w];
            before += w < wave ? x : 0ull;
            tot += x;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) rank[r][q] += field(before, cls(r, q));
        return tot;
    }
};

struct VArgs {
    const uint32_t *keys;
    int64_t n;
    uint32_t *out_keys;
    void *out_idx;
    int64_t *counts;          // [v] class sizes (output)
    uint64_t *desc;           // [num_tiles][4] per-class prefix of the tile inside its run
    int64_t *wsum;            // [3][kVCountWaves] run totals, then run prefixes
    int64_t num_tiles;
    int64_t tiles_per_wave;
    int32_t need_keys;
};

template <int V, class Cls>
__global__ __launch_bounds__(256) void flatv_count_kernel(VArgs a, Cls cl) {
    constexpr int kTile = kVBlockThreads * kVRows * 4;
    using WT = TileV<kWave, 8, V>;   // one wave, 2048 elements: 8 vector loads in flight per lane
    constexpr int kChunks = kTile / WT::kSize;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = static_cast<int64_t>(blockIdx.x) * (256 / kWave) + wave_id();
    const int64_t t0 = w * a.tiles_per_wave;
    const int64_t t1 = t0 + a.tiles_per_wave < a.num_tiles ? t0 + a.tiles_per_wave : a.num_tiles;
    uint64_t run[V - 1];
#pragma unroll
    for (int k = 0; k < V - 1; ++k) run[k] = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t lo = t * kTile;
        const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;
        uint64_t cnt = 0;   // packed per-class counts of the tile
        for (int c = 0; c < kChunks; ++c) {
            WT chunk;
            chunk.load(a.keys, a.n, lo + c * WT::kSize, lo, hi, cl, !Cls::kUsesBytes, 0, lane);
            cnt += chunk.wave_counts();
        }
        if (lane < V - 1) {
            uint64_t mine = run[0];
#pragma unroll
            for (int k = 1; k < V - 1; ++k) mine = lane == k ? run[k] : mine;
            a.desc[t * 4 + lane] = mine;
        }
#pragma unroll
        for (int k = 0; k < V - 1; ++k) run[k] += WT::field(cnt, k);
    }
    if (lane < V - 1 && w < kVCountWaves) {
        uint64_t mine = run[0];
#pragma unroll
        for (int k = 1; k < V - 1; ++k) mine = lane == k ? run[k] : mine;
        a.wsum[lane * kVCountWaves + w] = static_cast<int64_t>(mine);
    }
}

// One workgroup: for every class but the last, the run totals become
// exclusive prefixes (8 entries per thread, wave shuffles, LDS across waves);
// the class sizes go to counts[0..v).
template <int V>
__global__ __launch_bounds__(1024) void flatv_scan_kernel(int64_t *wsum, int64_t nw, int64_t n, int64_t *counts) {
    constexpr int kPer = 8;
    static_assert(kPer * 1024 >= kVCountWaves, "scan capacity");
    __shared__ int64_t wtot[16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
    int64_t rest = n;
    for (int k = 0; k < V - 1; ++k) {
        int64_t *ws = wsum + k * kVCountWaves;
        int64_t v[kPer];
        int64_t run = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int64_t i = static_cast<int64_t>(tid) * kPer + j;
            v[j] = i < nw ? ws[i] : 0;
            run += v[j];
        }
        int64_t inc = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        int64_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int64_t x = wtot[w];
            before += w < wave ? x : 0;
            total += x;
        }
        __syncthreads();   // wtot is reused by the next class
        int64_t acc = before + inc - run;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int64_t i = static_cast<int64_t>(tid) * kPer + j;
            if (i < nw) ws[i] = acc;
            acc += v[j];
        }
        if (tid == 0) counts[k] = total;
        rest -= total;
    }
    if (tid == 0) counts[V - 1] = rest;
}

template <int V, class Cls, class Idx>
__global__ __launch_bounds__(kVBlockThreads) void flatv_scatter_kernel(VArgs a, Cls cl) {
    using T = TileV<kVBlockThreads, kVRows, V>;
    constexpr int kTile = T::kSize;
    __shared__ uint32_t stage[kTile];
    __shared__ uint64_t wt[T::kWaves];

    const int tid = threadIdx.x;
    const int wave = wave_id();
    const int lane = tid & (kWave - 1);
    const int64_t t = blockIdx.x;   // (the XCD-aware order of the 2-way scatter measured 1 % slower here)
    const int64_t lo = t * kTile;
    const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;

    // destination of the tile's first element of each class:
    // B_c (classes before c) + elements of class c before the tile
    int64_t dst[V];
    {
        int64_t before_tile = 0, base = 0;
#pragma unroll
        for (int k = 0; k < V - 1; ++k) {
            const int64_t e = static_cast<int64_t>(a.desc[t * 4 + k]) +
                              a.wsum[k * kVCountWaves + t / a.tiles_per_wave];
            dst[k] = base + e;
            before_tile += e;
            base += a.counts[k];
        }
        dst[V - 1] = base + (lo - before_tile);
    }

    T tile;
    tile.load(a.keys, a.n, lo, lo, hi, cl, a.need_keys != 0, wave, lane);
    tile.wave_ranks(lane);
    const uint64_t ptot = tile.block_ranks(wt, wave, lane);
    uint32_t tot[V], sbase[V];   // class sizes and stage offsets inside the tile
#pragma unroll
    for (int k = 0; k < V; ++k) {
        tot[k] = T::field(ptot, k);
        sbase[k] = k == 0 ? 0u : sbase[k - 1] + tot[k - 1];
    }

    Idx *out_idx = static_cast<Idx *>(a.out_idx);
    const Picker<V, int64_t> dst_of(dst);
    const Picker<V, uint32_t> sbase_of(sbase);
#pragma unroll
    for (int r = 0; r < kVRows; ++r) {
        const int64_t p0 = T::pos(lo, wave, r, lane);
        Idx v[4];
        uint32_t vm = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = tile.cls(r, q);
            const bool ok = tile.valid(r, q);
            vm |= static_cast<uint32_t>(ok) << q;
            v[q] = static_cast<Idx>(dst_of(c) + tile.rank[r][q]);
            if (a.out_keys && ok) stage[sbase_of(c) + tile.rank[r][q]] = tile.key[r][q];
        }
        if (out_idx && vm) store_idx_group<4, Idx>(out_idx, p0, v, vm);
    }
    if (a.out_keys) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < V; ++k) write_run<kVBlockThreads>(stage, sbase[k], tot[k], dst[k], a.out_keys, a.n, tid);
    }
}

template <int V, class Cls>
int launch_v(VArgs a, const Cls &cl, int idx_t, hipStream_t st) {
    constexpr int64_t kTile = kVBlockThreads * kVRows * 4;
    a.num_tiles = ceil_div(a.n, kTile);
    const int64_t nt = a.num_tiles;
    int64_t nw = 0;
    if (nt > 0) {
        a.tiles_per_wave = ceil_div(nt, kVCountWaves);
        nw = ceil_div(nt, a.tiles_per_wave);
        IXP_LAUNCH("flatv_count", (flatv_count_kernel<V, Cls>), dim3(static_cast<uint32_t>(ceil_div(nw, 4))),
                   dim3(256), 0, st, a, cl);
    }
    IXP_LAUNCH("flatv_scan", flatv_scan_kernel<V>, dim3(1), dim3(1024), 0, st, a.wsum, nw, a.n, a.counts);
    if (nt == 0) return launch_status();
    if (idx_t == IXP_I32)
        IXP_LAUNCH("flatv_scatter", (flatv_scatter_kernel<V, Cls, int32_t>), dim3(static_cast<uint32_t>(nt)),
                   dim3(kVBlockThreads), 0, st, a, cl);
    else
        IXP_LAUNCH("flatv_scatter", (flatv_scatter_kernel<V, Cls, int64_t>), dim3(static_cast<uint32_t>(nt)),
                   dim3(kVBlockThreads), 0, st, a, cl);
    return launch_status();
}

template <int V>
int dispatch_v(const VArgs &a, const ixp_classes &c, int idx_t, hipStream_t st) {
    switch (c.kind) {
    case IXP_CLASS_MOD: {
        ClassMod cl{~0ull / static_cast<uint32_t>(V) + 1, static_cast<uint32_t>(V)};
        return launch_v<V>(a, cl, idx_t, st);
    }
    case IXP_CLASS_THRESH: {
        ClassThresh<V> cl{c.s[0], c.s[1], c.s[2]};
        return launch_v<V>(a, cl, idx_t, st);
    }
    default: {
        ClassBytes<V> cl{c.classes};
        return launch_v<V>(a, cl, idx_t, st);
    }
    }
}

}  // namespace
}  // namespace ixp

using namespace ixp;

extern "C" size_t ixp_partition_v_workspace(int64_t n) {
    if (n < 0) return 0;
    const int64_t nt = ceil_div(n, static_cast<int64_t>(kVBlockThreads) * kVRows * 4);
    return kVHeader + 3 * kVCountWaves * sizeof(int64_t) + static_cast<size_t>(nt) * 4 * sizeof(uint64_t);
}

extern "C" int ixp_partition_v(const void *keys, int32_t key_t, int64_t n, const ixp_classes *cls,
                               void *out_keys, void *out_idx, int32_t idx_t, int64_t *d_counts, void *ws,
                               size_t ws_bytes, void *stream) {
    if (n < 0 || !cls || !d_counts) return IXP_EINVAL;
    const int v = cls->v;
    if (v < 2 || v > 4) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (idx_t == IXP_I32 && n > 0x7FFFFFFFll) return IXP_EINVAL;
    switch (cls->kind) {
    case IXP_CLASS_MOD:
        if (key_t != IXP_I32) return IXP_EINVAL;
        break;
    case IXP_CLASS_THRESH:
        if (key_t != IXP_F32) return IXP_EINVAL;
        for (int h = 1; h < v - 1; ++h)
            if (!(cls->s[h - 1] <= cls->s[h])) return IXP_EINVAL;
        break;
    case IXP_CLASS_BYTES:
        if (key_t != IXP_I32 && key_t != IXP_F32) return IXP_EINVAL;
        if (n > 0 && !cls->classes) return IXP_EINVAL;
        break;
    default:
        return IXP_EINVAL;
    }
    const bool need_keys = cls->kind != IXP_CLASS_BYTES || out_keys != nullptr;
    if (n > 0 && need_keys && !keys) return IXP_EINVAL;
    if (!ws || ws_bytes < ixp_partition_v_workspace(n)) return IXP_EWORKSPACE;
    const size_t isz = idx_t == IXP_I32 ? 4 : 8;
    if (!aligned(keys, 16) || !aligned(out_keys, 4) || !aligned(out_idx, 4 * isz) || !aligned(d_counts, 8) ||
        !aligned(ws, 8) || !aligned(cls->classes, 4))
        return IXP_EINVAL;
    char *w = static_cast<char *>(ws);
    VArgs a;
    a.keys = static_cast<const uint32_t *>(keys);
    a.n = n;
    a.out_keys = static_cast<uint32_t *>(out_keys);
    a.out_idx = out_idx;
    a.counts = d_counts;
    a.wsum = reinterpret_cast<int64_t *>(w + kVHeader);
    a.desc = reinterpret_cast<uint64_t *>(w + kVHeader + 3 * kVCountWaves * sizeof(int64_t));
    a.num_tiles = 0;
    a.tiles_per_wave = 1;
    a.need_keys = need_keys ? 1 : 0;
    hipStream_t st = as_stream(stream);
    switch (v) {
    case 2: return dispatch_v<2>(a, *cls, idx_t, st);
    case 3: return dispatch_v<3>(a, *cls, idx_t, st);
    default: return dispatch_v<4>(a, *cls, idx_t, st);
    }
}
