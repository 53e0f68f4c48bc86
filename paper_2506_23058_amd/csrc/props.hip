// props.hip -- run-time checkers of the array properties of Section 2.3
// (figure "Array Properties"): Range, Monotonic, Inj, Bij and FiltPart.
//
// Range / Monotonic / Inj / Bij share one streaming pass over X (16-byte
// nontemporal loads).  Every failing index is reduced to the least one with a
// wave minimum and one atomicMin per wave, so verdicts do not depend on
// scheduling.  Inj and Bij insert every in-Rcd value into a bitmap over the
// restricted co-domain with atomicOr; a bit found already set only says that
// its value repeats, not which occurrence is the first, so values seen twice
// are marked in a second bitmap.  Only when some value repeats, two more passes
// run: the first records, for every repeated value, its least index
// (atomicMin into a per-value table that only repeated values ever touch), the
// second reports the least index that is not such a first occurrence -- the
// earliest second occurrence.  Without repeats those passes exit at once.
//
// FiltPart checks the outputs of a flat partition: the split point against
// the number of trues, Bij of the indices (as above), the class order, the
// values moved, and stability (indices strictly increasing inside each class,
// InvFiltPart item 3), the latter with a per-class running maximum carried
// from tile to tile by an exclusive max-scan over tiles.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr uint64_t kNone = 0x7FFFFFFFFFFFFFFFull;
constexpr int kPropsBlock = 256;

// Device-side state at the start of the workspace.
struct PropsState {
    unsigned long long fv_range, fv_mono, fv_img, fv_inj;   // least failing index, kNone if none
    unsigned long long in_count;                            // entries inside Rcd
    unsigned long long missing;                             // least value of Img not attained
    unsigned int dup_found;
    unsigned int pad0;
    // FiltPart
    unsigned long long fp_fv;          // least index failing bits 1..4
    unsigned long long fp_true;        // number of trues
    unsigned int fp_bits;              // OR of failing sub-check bits (2..16)
    unsigned int pad1;
};
constexpr size_t kPropsHeader = 256;
static_assert(sizeof(PropsState) <= kPropsHeader, "props header");

struct PropsArgs {
    const void *x;
    int32_t x64;          // 1: int64 elements, 0: int32
    int64_t n;
    uint32_t mask;
    int64_t lo, hi, ilo, ihi;
    int32_t mono_op;
    PropsState *st;
    uint32_t *seen;       // bitmap over [lo, hi)
    uint32_t *dup;        // repeated values
    uint32_t *first;      // least index of each repeated value (n < 2^32) or...
    unsigned long long *first64;   // ... 64-bit when n >= 2^32
    int64_t width;        // hi - lo when a bitmap is in use
    // Bucketed Inj/Bij (see props_place_kernel): values of Rcd grouped in
    // buckets of 2^kBucketShift consecutive values.
    int32_t bucketed;
    int32_t nbuckets;
    unsigned long long *bucket_total;   // [nbuckets]
    unsigned long long *bucket_start;   // [nbuckets]
    unsigned long long *wg_base;        // [gridDim of pass 1][nbuckets]
    uint32_t *records;                  // [entries inside Rcd] value - lo - bucket base (20 bits)
    // FiltPart
    const uint32_t *fp_src;
    const uint32_t *fp_dst;
    const int64_t *fp_split;
    int32_t fp_mode;
    int64_t *fp_tmax;     // per tile, two classes: max index value seen (kNoZ if none)
    int64_t fp_tiles;
};

__device__ __forceinline__ int64_t load_x(const void *x, int32_t x64, int64_t i) {
    return x64 ? static_cast<const int64_t *>(x)[i] : static_cast<int64_t>(static_cast<const int32_t *>(x)[i]);
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ bool mono_ok(int64_t a, int64_t b, int op) {
    switch (op) {
    case IXP_MONO_LE: return a <= b;
    case IXP_MONO_LT: return a < b;
    case IXP_MONO_GE: return a >= b;
    default: return a > b;
    }
}

__global__ void props_init_kernel(PropsState *st, uint32_t *seen, uint32_t *dup, int64_t words,
                                  unsigned long long *zero2, int64_t nzero2) {
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < nzero2; i += static_cast<int64_t>(gridDim.x) * blockDim.x) zero2[i] = 0;
    if (i0 == 0 && st) {
        st->fv_range = st->fv_mono = st->fv_img = st->fv_inj = kNone;
        st->in_count = 0;
        st->missing = kNone;
        st->dup_found = 0;
        st->fp_fv = kNone;
        st->fp_true = 0;
        st->fp_bits = 0;
    }
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    const int64_t w4 = words / 4;
    for (int64_t i = i0; i < w4; i += stride) {
        __builtin_nontemporal_store(v4{0, 0, 0, 0}, reinterpret_cast<v4 *>(seen) + i);
        __builtin_nontemporal_store(v4{0, 0, 0, 0}, reinterpret_cast<v4 *>(dup) + i);
    }
    for (int64_t i = w4 * 4 + i0; i < words; i += stride) {
        seen[i] = 0;
        dup[i] = 0;
    }
}

// Inserts v (inside [lo, hi)) into the seen bitmap; a repeat marks it in the
// dup bitmap and resets its first-index slot.
__device__ __forceinline__ void insert_value(const PropsArgs &a, int64_t v, bool *dup_seen) {
    const uint64_t o = static_cast<uint64_t>(v - a.lo);
    const uint32_t bit = 1u << (o & 31);
    const uint32_t old = atomicOr(a.seen + (o >> 5), bit);
    if (old & bit) {
        atomicOr(a.dup + (o >> 5), bit);
        if (a.first64) a.first64[o] = ~0ull;
        else a.first[o] = ~0u;
        *dup_seen = true;
    }
}

// Monotonic comparison with the operator decoded once: LE a<=b, LT a<b,
// GE b<=a, GT b<a.
struct MonoCmp {
    bool swap, strict;
    __device__ __forceinline__ bool ok(int64_t a, int64_t b) const {
        const int64_t l = swap ? b : a, r = swap ? a : b;
        return strict ? l < r : l <= r;
    }
};

// Pass 1: Range, Monotonic, the Img part of Bij, the in-Rcd count and the
// bitmap insertions of Inj / Bij, for every element.  Each thread takes
// 16-byte groups (2 int64 or 4 int32); a group's left neighbour for the
// monotonic check comes from the previous lane (consecutive lanes hold
// consecutive groups), lane 0 loads it.
constexpr int kBucketShift = 20;              // 2^20 values: a 128 KiB LDS bitmap
constexpr int kMaxBuckets = 4096;

__device__ __forceinline__ void note_value(const PropsArgs &a, int64_t v, bool *dup_seen,
                                           uint32_t *hist) {
    if (a.bucketed) atomicAdd(hist + ((v - a.lo) >> kBucketShift), 1u);
    else insert_value(a, v, dup_seen);
}

template <bool X64, int UNROLL>
__global__ __launch_bounds__(kPropsBlock) void props_pass1_kernel(PropsArgs a) {
    constexpr int kPer = X64 ? 2 : 4;
    extern __shared__ uint32_t hist[];   // nbuckets counters when bucketed
    if (a.bucketed) {
        for (int b = threadIdx.x; b < a.nbuckets; b += blockDim.x) hist[b] = 0;
        __syncthreads();
    }
    const bool want_range = a.mask & IXP_RANGE;
    const bool want_mono = a.mask & IXP_MONO;
    const bool want_set = a.mask & (IXP_INJ | IXP_BIJ);
    const bool want_img = a.mask & IXP_BIJ;
    const MonoCmp cmp{a.mono_op == IXP_MONO_GE || a.mono_op == IXP_MONO_GT,
                      a.mono_op == IXP_MONO_LT || a.mono_op == IXP_MONO_GT};
    const int lane = threadIdx.x & 63;
    unsigned long long c_range = kNone, c_mono = kNone, c_img = kNone, cnt = 0;
    bool dup_seen = false;
    const int64_t groups = a.n / kPer;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    // every lane of a wave runs the same number of iterations (shuffles below)
    const int64_t wave_g0 = g0 - lane;
    for (int64_t gb = g0; wave_g0 + (gb - g0) < groups; gb += UNROLL * stride) {
        v4 raw[UNROLL];
        int64_t gi[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            gi[u] = gb + u * stride;
            raw[u] = gi[u] < groups
                         ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi[u])
                         : v4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            int64_t val[kPer];
            if constexpr (X64) {
                val[0] = static_cast<int64_t>((static_cast<uint64_t>(raw[u].y) << 32) | raw[u].x);
                val[1 % kPer] = static_cast<int64_t>((static_cast<uint64_t>(raw[u].w) << 32) | raw[u].z);
            } else {
                val[0] = static_cast<int32_t>(raw[u].x);
                val[1 % kPer] = static_cast<int32_t>(raw[u].y);
                val[2 % kPer] = static_cast<int32_t>(raw[u].z);
                val[3 % kPer] = static_cast<int32_t>(raw[u].w);
            }
            const bool live = gi[u] < groups;
            const int64_t p0 = gi[u] * kPer;
            int64_t prev = 0;
            if (want_mono) {
                prev = __shfl_up(val[kPer - 1], 1, 64);
                if (lane == 0 && live && p0 > 0) prev = load_x(a.x, X64 ? 1 : 0, p0 - 1);
            }
            if (!live) continue;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int64_t i = p0 + q;
                const int64_t v = val[q];
                if (want_range && !(a.lo <= v && v < a.hi) && static_cast<unsigned long long>(i) < c_range)
                    c_range = i;
                if (want_mono && i > 0 && !cmp.ok(prev, v) && static_cast<unsigned long long>(i) < c_mono)
                    c_mono = i;
                prev = v;
                if (want_set && a.lo <= v && v < a.hi) {
                    ++cnt;
                    if (want_img && !(a.ilo <= v && v < a.ihi) && static_cast<unsigned long long>(i) < c_img)
                        c_img = i;
                    note_value(a, v, &dup_seen, hist);
                }
            }
        }
    }
    // the last n % kPer elements: thread 0 of block 0
    if (g0 == 0) {
        for (int64_t i = groups * kPer; i < a.n; ++i) {
            const int64_t v = load_x(a.x, X64 ? 1 : 0, i);
            if (want_range && !(a.lo <= v && v < a.hi) && static_cast<unsigned long long>(i) < c_range)
                c_range = i;
            if (want_mono && i > 0 && !cmp.ok(load_x(a.x, X64 ? 1 : 0, i - 1), v) &&
                static_cast<unsigned long long>(i) < c_mono)
                c_mono = i;
            if (want_set && a.lo <= v && v < a.hi) {
                ++cnt;
                if (want_img && !(a.ilo <= v && v < a.ihi) && static_cast<unsigned long long>(i) < c_img)
                    c_img = i;
                note_value(a, v, &dup_seen, hist);
            }
        }
    }
    if (a.bucketed) {
        // reserve this workgroup's range inside every bucket it fills
        __syncthreads();
        for (int b = threadIdx.x; b < a.nbuckets; b += blockDim.x) {
            const uint32_t c = hist[b];
            a.wg_base[static_cast<int64_t>(blockIdx.x) * a.nbuckets + b] =
                c ? atomicAdd(a.bucket_total + b, static_cast<unsigned long long>(c)) : 0ull;
        }
    }
    c_range = wave_min_u64(c_range);
    c_mono = wave_min_u64(c_mono);
    c_img = wave_min_u64(c_img);
    cnt = wave_sum_u64(cnt);
    const bool any_dup = ballot(dup_seen) != 0;
    if (lane == 0) {
        if (c_range != kNone) atomicMin(&a.st->fv_range, c_range);
        if (c_mono != kNone) atomicMin(&a.st->fv_mono, c_mono);
        if (c_img != kNone) atomicMin(&a.st->fv_img, c_img);
        if (cnt) atomicAdd(&a.st->in_count, cnt);
        if (any_dup) atomicOr(&a.st->dup_found, 1u);
    }
}

// Bucketed Inj/Bij.  Random device-scope atomics on a bitmap in HBM run far
// below the memory bandwidth, so the values inside Rcd are first grouped by
// bucket (2^20 consecutive values each): pass 1 counts them per workgroup and
// reserves each workgroup's range in each bucket; props_place writes one
// 8-byte record (index << 20 | offset in bucket) per value into its bucket;
// props_check gives each bucket one workgroup, whose 128 KiB LDS bitmap
// finds the repeated values with LDS atomics and, for Bij, the least value of
// Img left unset.  Repeats are then located exactly by props_first/second.
__global__ __launch_bounds__(1024) void props_bucket_scan_kernel(PropsArgs a) {
    __shared__ unsigned long long lds[16];
    constexpr int kPer = kMaxBuckets / 1024;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    unsigned long long v[kPer], run = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int b = tid * kPer + k;
        v[k] = b < a.nbuckets ? a.bucket_total[b] : 0ull;
        run += v[k];
    }
    unsigned long long inc = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    unsigned long long before = 0;
    for (int w = 0; w < wave; ++w) before += lds[w];
    unsigned long long acc = before + inc - run;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int b = tid * kPer + k;
        if (b < a.nbuckets) a.bucket_start[b] = acc;
        acc += v[k];
    }
}

// Placement works in rounds of UNROLL groups per thread (the same elements
// per workgroup as pass 1).  A round's records are first grouped by bucket in
// LDS (a local counting sort: LDS atomics give ranks, a scan of the round's
// bucket counts gives offsets), then written bucket run by bucket run, so
// global stores form contiguous runs instead of scattered 8-byte writes.
template <bool X64, int UNROLL>
__global__ __launch_bounds__(kPropsBlock) void props_place_kernel(PropsArgs a) {
    constexpr int kPer = X64 ? 2 : 4;
    constexpr int kRound = kPropsBlock * UNROLL * kPer;   // records per round at most
    static_assert(kRound <= (1 << 14), "rank field");
    extern __shared__ unsigned long long base[];          // [nb] global write position
    const int nb = a.nbuckets;
    uint32_t *rhist = reinterpret_cast<uint32_t *>(base + nb);   // [nb] round counts
    uint32_t *roff = rhist + nb;                                 // [nb] round offsets
    uint32_t *stage = roff + nb;                                 // [kRound] staged records
    uint16_t *sbkt = reinterpret_cast<uint16_t *>(stage + kRound);
    __shared__ uint32_t wsum[kPropsBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    for (int b = tid; b < nb; b += kPropsBlock) {
        base[b] = a.bucket_start[b] + a.wg_base[static_cast<int64_t>(blockIdx.x) * nb + b];
        rhist[b] = 0;
    }
    __syncthreads();
    const int64_t groups = a.n / kPer;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
    const int64_t wg_g0 = static_cast<int64_t>(blockIdx.x) * blockDim.x;   // workgroup-uniform
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    constexpr uint32_t kOut = ~0u;   // not inside Rcd
    for (int64_t rb = 0; wg_g0 + rb < groups; rb += UNROLL * stride) {
        uint32_t rec[UNROLL * kPer];    // offset inside the bucket
        uint32_t meta[UNROLL * kPer];   // bucket << 14 | rank inside the round, or kOut
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t gi = g0 + rb + u * stride;
            v4 raw = gi < groups ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi)
                                 : v4{0, 0, 0, 0};
            int64_t val[kPer];
            if constexpr (X64) {
                val[0] = static_cast<int64_t>((static_cast<uint64_t>(raw.y) << 32) | raw.x);
                val[1 % kPer] = static_cast<int64_t>((static_cast<uint64_t>(raw.w) << 32) | raw.z);
            } else {
                val[0] = static_cast<int32_t>(raw.x);
                val[1 % kPer] = static_cast<int32_t>(raw.y);
                val[2 % kPer] = static_cast<int32_t>(raw.z);
                val[3 % kPer] = static_cast<int32_t>(raw.w);
            }
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int k = u * kPer + q;
                const int64_t v = val[q];
                const bool in = gi < groups && a.lo <= v && v < a.hi;
                const uint64_t o = static_cast<uint64_t>(v - a.lo);
                const uint32_t bk = static_cast<uint32_t>(o >> kBucketShift);
                rec[k] = static_cast<uint32_t>(o & ((1ull << kBucketShift) - 1));
                meta[k] = in ? (bk << 14) | atomicAdd(rhist + bk, 1u) : kOut;
            }
        }
        __syncthreads();
        // exclusive scan of the round's bucket counts (threads own buckets
        // b = tid, tid + 256, ...; a sequential pass per thread suffices for
        // nb <= 4096 after a block scan of the per-thread sums)
        uint32_t mysum = 0;
        for (int b = tid; b < nb; b += kPropsBlock) mysum += rhist[b];
        uint32_t inc = mysum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t before = inc - mysum;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        // thread tid lays out its buckets tid, tid + 256, ... after its
        // exclusive prefix; any bucket order inside a round works, since the
        // write pass reads each slot's bucket back
        for (int b = tid; b < nb; b += kPropsBlock) {
            roff[b] = before;
            before += rhist[b];
        }
        __syncthreads();
        uint32_t round_total = 0;
        for (int w = 0; w < kPropsBlock / 64; ++w) round_total += wsum[w];
#pragma unroll
        for (int k = 0; k < UNROLL * kPer; ++k) {
            if (meta[k] != kOut) {
                const uint32_t bk = meta[k] >> 14;
                const uint32_t slot = roff[bk] + (meta[k] & ((1u << 14) - 1));
                stage[slot] = rec[k];
                sbkt[slot] = static_cast<uint16_t>(bk);
            }
        }
        __syncthreads();
        for (uint32_t sl = tid; sl < round_total; sl += kPropsBlock) {
            const int b = sbkt[sl];
            __builtin_nontemporal_store(stage[sl], a.records + base[b] + (sl - roff[b]));
        }
        __syncthreads();
        for (int b = tid; b < nb; b += kPropsBlock) {
            base[b] += rhist[b];
            rhist[b] = 0;
        }
        __syncthreads();
    }
    // the last n % kPer elements: thread 0 of block 0, directly
    if (g0 == 0) {
        for (int64_t i = groups * kPer; i < a.n; ++i) {
            const int64_t v = load_x(a.x, X64 ? 1 : 0, i);
            if (!(a.lo <= v && v < a.hi)) continue;
            const uint64_t o = static_cast<uint64_t>(v - a.lo);
            const int b = static_cast<int>(o >> kBucketShift);
            a.records[base[b]] = static_cast<uint32_t>(o & ((1ull << kBucketShift) - 1));
            base[b] += 1;
        }
    }
}

// Records placed per workgroup and round: 32 per bucket for 256 buckets.
constexpr int kPlaceRound = 8192;

constexpr int kCheckThreads = 1024;
constexpr int kBucketWords = (1 << kBucketShift) / 32;

__global__ __launch_bounds__(kCheckThreads) void props_check_kernel(PropsArgs a) {
    __shared__ uint32_t bits[kBucketWords];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    for (int w = tid; w < kBucketWords; w += kCheckThreads) bits[w] = 0;
    __syncthreads();
    const unsigned long long r0 = a.bucket_start[b], r1 = r0 + a.bucket_total[b];
    bool dup_seen = false;
    for (unsigned long long r = r0 + tid; r < r1; r += kCheckThreads) {
        const uint32_t off = __builtin_nontemporal_load(a.records + r);
        const uint32_t bit = 1u << (off & 31);
        const uint32_t old = atomicOr(bits + (off >> 5), bit);
        if (old & bit) {
            const uint64_t o = (static_cast<uint64_t>(b) << kBucketShift) + off;   // value - lo
            atomicOr(a.dup + (o >> 5), 1u << (o & 31));
            if (a.first64) a.first64[o] = ~0ull;
            else a.first[o] = ~0u;
            dup_seen = true;
        }
    }
    const bool any_dup = ballot(dup_seen) != 0;
    if ((tid & 63) == 0 && any_dup) atomicOr(&a.st->dup_found, 1u);
    if (!(a.mask & IXP_BIJ)) return;
    __syncthreads();
    // least value of Img inside this bucket whose bit is clear
    const int64_t v0 = a.lo + (static_cast<int64_t>(b) << kBucketShift);
    const int64_t lo_b = a.ilo > v0 ? a.ilo - v0 : 0;
    const int64_t hi_b = a.ihi - v0 < (int64_t{1} << kBucketShift) ? a.ihi - v0 : (int64_t{1} << kBucketShift);
    unsigned long long c = kNone;
    if (lo_b < hi_b) {
        for (int64_t w = (lo_b >> 5) + tid; w <= ((hi_b - 1) >> 5); w += kCheckThreads) {
            uint32_t clear = ~bits[w];
            const int64_t wb = w << 5;
            if (wb < lo_b) clear &= ~0u << (lo_b - wb);
            if (wb + 32 > hi_b) clear &= (hi_b - wb) >= 32 ? ~0u : ((1u << (hi_b - wb)) - 1u);
            if (clear) {
                const unsigned long long v = static_cast<unsigned long long>(v0 + wb + __builtin_ctz(clear));
                if (v < c) c = v;
            }
        }
    }
    c = wave_min_u64(c);
    if ((tid & 63) == 0 && c != kNone) atomicMin(&a.st->missing, c);
}

// Value inserted by the Inj / Bij bitmap for element i, or false.
__device__ __forceinline__ bool inserted_value(const PropsArgs &a, int64_t i, int64_t *v_out) {
    const int64_t v = load_x(a.x, a.x64, i);
    *v_out = v;
    return a.lo <= v && v < a.hi;
}

__device__ __forceinline__ bool is_dup(const PropsArgs &a, int64_t v) {
    const uint64_t o = static_cast<uint64_t>(v - a.lo);
    return (a.dup[o >> 5] >> (o & 31)) & 1u;
}

// Pass 2 (only when a value repeats): least index of every repeated value.
__global__ __launch_bounds__(kPropsBlock) void props_first_kernel(PropsArgs a) {
    if (a.st->dup_found == 0) return;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        int64_t v;
        if (!inserted_value(a, i, &v) || !is_dup(a, v)) continue;
        const uint64_t o = static_cast<uint64_t>(v - a.lo);
        if (a.first64) atomicMin(a.first64 + o, static_cast<unsigned long long>(i));
        else atomicMin(a.first + o, static_cast<uint32_t>(i));
    }
}

// Pass 3 (only when a value repeats): least index that is not the first
// occurrence of its value.
__global__ __launch_bounds__(kPropsBlock) void props_second_kernel(PropsArgs a, unsigned long long *target) {
    if (a.st->dup_found == 0) return;
    unsigned long long c = kNone;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        int64_t v;
        if (!inserted_value(a, i, &v) || !is_dup(a, v)) continue;
        const uint64_t o = static_cast<uint64_t>(v - a.lo);
        const uint64_t f = a.first64 ? a.first64[o] : static_cast<uint64_t>(a.first[o]);
        if (static_cast<uint64_t>(i) != f && static_cast<unsigned long long>(i) < c) c = i;
    }
    c = wave_min_u64(c);
    if ((threadIdx.x & 63) == 0 && c != kNone) atomicMin(target, c);
}

// Bij failing only on the count: least value of Img whose bit is clear.
__global__ __launch_bounds__(kPropsBlock) void props_missing_kernel(PropsArgs a) {
    if (a.bucketed) return;
    PropsState *st = a.st;
    const unsigned long long inj = st->fv_inj, img = st->fv_img;
    if (inj != kNone || img != kNone) return;
    if (static_cast<int64_t>(st->in_count) == a.ihi - a.ilo) return;
    const int64_t b0 = a.ilo - a.lo, b1 = a.ihi - a.lo;   // bit range inside the bitmap
    unsigned long long c = kNone;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t w = (b0 >> 5) + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
         w <= ((b1 - 1) >> 5); w += stride) {
        uint32_t clear = ~a.seen[w];
        const int64_t wb = w << 5;
        if (wb < b0) clear &= ~0u << (b0 - wb);
        if (wb + 32 > b1) clear &= (b1 - wb) >= 32 ? ~0u : ((1u << (b1 - wb)) - 1u);
        if (clear) {
            const unsigned long long v = static_cast<unsigned long long>(wb + __builtin_ctz(clear) + a.lo);
            if (v < c) c = v;
        }
    }
    c = wave_min_u64(c);
    if ((threadIdx.x & 63) == 0 && c != kNone) atomicMin(&st->missing, c);
}

// ---------------------------------------------------------------- FiltPart --
// One wave per tile of 64 x 64 elements, one element per lane per row.
constexpr int kFpRows = 64;
constexpr int64_t kNoZ = INT64_MIN;   // no earlier kept element of the class
constexpr int64_t kFpTile = kFpRows * kWave;

struct FpElem {
    bool c;        // predicate
    bool kept;     // takes part (partition: all; filter: trues)
    int cls;       // class for the stability check
    int64_t z;
};

template <class Pred>
__device__ __forceinline__ FpElem fp_elem(const PropsArgs &a, const Pred &pred, int64_t i) {
    FpElem e;
    uint32_t key = 0;
    uint8_t fl = 0;
    if constexpr (Pred::kUsesFlags) fl = pred.flags[i];
    else key = a.fp_src[i];
    e.c = pred(key, fl);
    e.kept = a.fp_mode == IXP_MODE_PARTITION || e.c;
    e.cls = a.fp_mode == IXP_MODE_PARTITION ? (e.c ? 1 : 0) : 1;
    e.z = load_x(a.x, a.x64, i);
    return e;
}

// Tile maxima of the index values per class (for the carried running max;
// kNoZ when the tile has no kept element of the class) and the number of
// trues.
template <class Pred>
__global__ __launch_bounds__(kPropsBlock) void fp_tile_max_kernel(PropsArgs a, Pred pred) {
    const int lane = threadIdx.x & 63;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * (kPropsBlock / 64) + wave_id();
    if (t >= a.fp_tiles) return;
    int64_t m0 = kNoZ, m1 = kNoZ;
    unsigned long long nt = 0;
    for (int r = 0; r < kFpRows; ++r) {
        const int64_t i = t * kFpTile + static_cast<int64_t>(r) * kWave + lane;
        if (i >= a.n) break;
        const FpElem e = fp_elem(a, pred, i);
        nt += e.c ? 1 : 0;
        if (!e.kept) continue;
        if (e.cls == 0) m0 = e.z > m0 ? e.z : m0;
        else m1 = e.z > m1 ? e.z : m1;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o0 = __shfl_xor(m0, off, 64), o1 = __shfl_xor(m1, off, 64);
        m0 = o0 > m0 ? o0 : m0;
        m1 = o1 > m1 ? o1 : m1;
    }
    nt = wave_sum_u64(nt);
    if (lane == 0) {
        a.fp_tmax[2 * t] = m0;
        a.fp_tmax[2 * t + 1] = m1;
        if (nt) atomicAdd(&a.st->fp_true, nt);
    }
}

// Exclusive running max over tiles, per class (one workgroup, chunks of 1024).
__global__ __launch_bounds__(1024) void fp_tile_scan_kernel(PropsArgs a) {
    __shared__ int64_t buf[2][2][1024];
    int64_t carry0 = kNoZ, carry1 = kNoZ;
    for (int64_t c0 = 0; c0 < a.fp_tiles; c0 += 1024) {
        const int64_t t = c0 + threadIdx.x;
        int64_t v0 = t < a.fp_tiles ? a.fp_tmax[2 * t] : kNoZ;
        int64_t v1 = t < a.fp_tiles ? a.fp_tmax[2 * t + 1] : kNoZ;
        int cur = 0;
        buf[cur][0][threadIdx.x] = v0;
        buf[cur][1][threadIdx.x] = v1;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t x0 = buf[cur][0][threadIdx.x], x1 = buf[cur][1][threadIdx.x];
            if (static_cast<int>(threadIdx.x) >= off) {
                const int64_t y0 = buf[cur][0][threadIdx.x - off], y1 = buf[cur][1][threadIdx.x - off];
                x0 = y0 > x0 ? y0 : x0;
                x1 = y1 > x1 ? y1 : x1;
            }
            buf[cur ^ 1][0][threadIdx.x] = x0;
            buf[cur ^ 1][1][threadIdx.x] = x1;
            cur ^= 1;
            __syncthreads();
        }
        // exclusive = inclusive of the previous thread, combined with the carry
        int64_t e0 = threadIdx.x > 0 ? buf[cur][0][threadIdx.x - 1] : kNoZ;
        int64_t e1 = threadIdx.x > 0 ? buf[cur][1][threadIdx.x - 1] : kNoZ;
        e0 = carry0 > e0 ? carry0 : e0;
        e1 = carry1 > e1 ? carry1 : e1;
        const int64_t last0 = buf[cur][0][1023], last1 = buf[cur][1][1023];
        __syncthreads();
        if (t < a.fp_tiles) {
            a.fp_tmax[2 * t] = e0;
            a.fp_tmax[2 * t + 1] = e1;
        }
        carry0 = last0 > carry0 ? last0 : carry0;
        carry1 = last1 > carry1 ? last1 : carry1;
    }
}

// Per element: Bij range part and bitmap insertion (bit 2), class order
// (bit 4), stability against the running max (bit 8), values (bit 16).
template <class Pred>
__global__ __launch_bounds__(kPropsBlock) void fp_check_kernel(PropsArgs a, Pred pred) {
    const int lane = threadIdx.x & 63;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * (kPropsBlock / 64) + wave_id();
    if (t >= a.fp_tiles) return;
    const int64_t split = *a.fp_split;
    const int64_t ylen = a.fp_mode == IXP_MODE_PARTITION ? a.n : split;
    int64_t run0 = a.fp_tmax[2 * t], run1 = a.fp_tmax[2 * t + 1];
    unsigned long long cand = kNone;
    uint32_t bits = 0;
    bool dup_seen = false;
    for (int r = 0; r < kFpRows; ++r) {
        const int64_t i = t * kFpTile + static_cast<int64_t>(r) * kWave + lane;
        const bool live = i < a.n;
        FpElem e{false, false, 0, 0};
        if (live) e = fp_elem(a, pred, i);
        uint32_t bad = 0;
        if (live) {
            if (a.fp_mode == IXP_MODE_PARTITION) {
                if (!(0 <= e.z && e.z < a.n)) bad |= 2;
                else insert_value(a, e.z, &dup_seen);
                if ((e.z < split) != e.c) bad |= 4;
            } else if (e.c) {
                if (!(0 <= e.z && e.z < split) || e.z >= a.n) bad |= 2;
                else insert_value(a, e.z, &dup_seen);
            } else if (0 <= e.z && e.z < split) {
                bad |= 2;
            }
            if (e.kept && 0 <= e.z && e.z < ylen && e.z < a.n && a.fp_dst[e.z] != a.fp_src[i]) bad |= 16;
        }
        // running max of earlier kept elements of the same class: an
        // inclusive max-scan over the lanes of this row, per class
        const int64_t mine0 = live && e.kept && e.cls == 0 ? e.z : kNoZ;
        const int64_t mine1 = live && e.kept && e.cls == 1 ? e.z : kNoZ;
        int64_t s0 = mine0, s1 = mine1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t o0 = __shfl_up(s0, off, 64), o1 = __shfl_up(s1, off, 64);
            if (lane >= off) {
                s0 = o0 > s0 ? o0 : s0;
                s1 = o1 > s1 ? o1 : s1;
            }
        }
        int64_t ex0 = __shfl_up(s0, 1, 64), ex1 = __shfl_up(s1, 1, 64);
        if (lane == 0) { ex0 = kNoZ; ex1 = kNoZ; }
        ex0 = run0 > ex0 ? run0 : ex0;
        ex1 = run1 > ex1 ? run1 : ex1;
        if (live && e.kept) {
            const int64_t before = e.cls == 0 ? ex0 : ex1;
            if (before != kNoZ && !(e.z > before)) bad |= 8;
        }
        const int64_t r0 = __shfl(s0, 63, 64), r1 = __shfl(s1, 63, 64);
        run0 = r0 > run0 ? r0 : run0;
        run1 = r1 > run1 ? r1 : run1;
        if (bad) {
            bits |= bad;
            if (static_cast<unsigned long long>(i) < cand) cand = i;
        }
    }
    cand = wave_min_u64(cand);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) bits |= __shfl_xor(bits, off, 64);
    const bool any_dup = ballot(dup_seen) != 0;
    if (lane == 0) {
        if (cand != kNone) atomicMin(&a.st->fp_fv, cand);
        if (bits) atomicOr(&a.st->fp_bits, bits);
        if (any_dup) atomicOr(&a.st->dup_found, 1u);
    }
}

// FiltPart's repeats: value inserted for element i, if any (same rule as
// fp_check_kernel).
template <class Pred>
__global__ __launch_bounds__(kPropsBlock) void fp_first_kernel(PropsArgs a, Pred pred, int pass,
                                                               unsigned long long *target) {
    if (a.st->dup_found == 0) return;
    const int64_t split = *a.fp_split;
    unsigned long long c = kNone;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const FpElem e = fp_elem(a, pred, i);
        const bool ins = a.fp_mode == IXP_MODE_PARTITION ? (0 <= e.z && e.z < a.n)
                                                         : (e.c && 0 <= e.z && e.z < split && e.z < a.n);
        if (!ins || !is_dup(a, e.z)) continue;
        const uint64_t o = static_cast<uint64_t>(e.z - a.lo);
        if (pass == 0) {
            if (a.first64) atomicMin(a.first64 + o, static_cast<unsigned long long>(i));
            else atomicMin(a.first + o, static_cast<uint32_t>(i));
        } else {
            const uint64_t f = a.first64 ? a.first64[o] : static_cast<uint64_t>(a.first[o]);
            if (static_cast<uint64_t>(i) != f && static_cast<unsigned long long>(i) < c) c = i;
        }
    }
    if (pass == 1) {
        c = wave_min_u64(c);
        if ((threadIdx.x & 63) == 0 && c != kNone) {
            atomicMin(target, c);
            atomicOr(&a.st->fp_bits, 2u);
        }
    }
}

// Writes the five verdicts.
__global__ void props_finalize_kernel(PropsArgs a, ixp_verdict *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const PropsState *st = a.st;
    for (int b = 0; b < 5; ++b) {
        out[b].holds = 1;
        out[b].reserved = 0;
        out[b].first_violation = -1;
        out[b].aux = 0;
    }
    auto fail = [&](int b, int64_t fv, int64_t aux) {
        out[b].holds = 0;
        out[b].first_violation = fv;
        out[b].aux = aux;
    };
    if ((a.mask & IXP_RANGE) && st->fv_range != kNone)
        fail(0, st->fv_range, load_x(a.x, a.x64, st->fv_range));
    if ((a.mask & IXP_MONO) && st->fv_mono != kNone) fail(1, st->fv_mono, 0);
    if ((a.mask & IXP_INJ) && st->fv_inj != kNone)
        fail(2, st->fv_inj, load_x(a.x, a.x64, st->fv_inj));
    if (a.mask & IXP_BIJ) {
        const unsigned long long f = st->fv_inj < st->fv_img ? st->fv_inj : st->fv_img;
        if (f != kNone) fail(3, f, load_x(a.x, a.x64, f));
        else if (static_cast<int64_t>(st->in_count) != a.ihi - a.ilo) fail(3, a.n, st->missing);
    }
    if (a.mask & IXP_FILTPART) {
        uint32_t bits = st->fp_bits;
        if (static_cast<int64_t>(st->fp_true) != *a.fp_split) bits |= 1u;
        if (bits) fail(4, st->fp_fv != kNone ? static_cast<int64_t>(st->fp_fv) : a.n, bits);
    }
}

template <class Pred>
int launch_filtpart(PropsArgs a, const Pred &pred, hipStream_t st, int grid) {
    const uint32_t tb = static_cast<uint32_t>(ceil_div(a.fp_tiles, kPropsBlock / 64));
    if (a.fp_tiles > 0) {
        IXP_LAUNCH("fp_tile_max", (fp_tile_max_kernel<Pred>), dim3(tb), dim3(kPropsBlock), 0, st, a, pred);
        IXP_LAUNCH("fp_tile_scan", fp_tile_scan_kernel, dim3(1), dim3(1024), 0, st, a);
        IXP_LAUNCH("fp_check", (fp_check_kernel<Pred>), dim3(tb), dim3(kPropsBlock), 0, st, a, pred);
        IXP_LAUNCH("fp_first", (fp_first_kernel<Pred>), dim3(grid), dim3(kPropsBlock), 0, st, a, pred, 0,
                   &a.st->fp_fv);
        IXP_LAUNCH("fp_second", (fp_first_kernel<Pred>), dim3(grid), dim3(kPropsBlock), 0, st, a, pred, 1,
                   &a.st->fp_fv);
    }
    return launch_status();
}

}  // namespace
}  // namespace ixp

using namespace ixp;

namespace {
constexpr int kPass1Grid = 2048;   // fixed, so the workspace size does not depend on the device

// Inj/Bij take the bucketed path when Rcd spans at most kMaxBuckets buckets
// and the array is large enough for the extra passes to pay.
int buckets_for(int64_t n, uint32_t mask, const ixp_prop_args *a) {
    if (!(mask & (IXP_INJ | IXP_BIJ)) || !a) return 0;
    const int64_t w = a->hi - a->lo;
    if (w <= 0 || n < (int64_t{1} << 16) || n >= (int64_t{1} << 43)) return 0;
    const int64_t b = (w + (int64_t{1} << kBucketShift) - 1) >> kBucketShift;
    return b <= kMaxBuckets ? static_cast<int>(b) : 0;
}

size_t bucket_bytes(int64_t n, int nb) {
    if (!nb) return 0;
    return round_up(static_cast<size_t>(nb) * 8, 256) * 2 +
           round_up(static_cast<size_t>(kPass1Grid) * nb * 8, 256) +
           round_up(static_cast<size_t>(n) * 4, 256);
}

int64_t rcd_width(int64_t n, uint32_t mask, const ixp_prop_args *a) {
    int64_t w = 0;
    if ((mask & (IXP_INJ | IXP_BIJ)) && a) w = a->hi - a->lo;
    if (mask & IXP_FILTPART) w = w > n ? w : n;
    return w;
}
}  // namespace

extern "C" size_t ixp_check_props_workspace(int64_t n, uint32_t mask, const ixp_prop_args *a) {
    if (n < 0) return 0;
    if ((mask & (IXP_INJ | IXP_BIJ | IXP_FILTPART)) && !a) return 0;
    if ((mask & (IXP_INJ | IXP_BIJ)) && (a->hi < a->lo || a->hi - a->lo > (int64_t{1} << 36))) return 0;
    const int64_t w = rcd_width(n, mask, a);
    const size_t words = static_cast<size_t>((w + 127) / 128 * 4);   // multiple of 4 words
    const size_t first_bytes = static_cast<size_t>(w) * (n >= (int64_t{1} << 32) ? 8 : 4);
    const int64_t tiles = (mask & IXP_FILTPART) ? ceil_div(n, kFpTile) : 0;
    return kPropsHeader + 2 * round_up(words * 4, 256) + round_up(first_bytes, 256) +
           round_up(static_cast<size_t>(tiles) * 16, 256) + bucket_bytes(n, buckets_for(n, mask, a));
}

extern "C" int ixp_check_props(const void *x, int32_t x_t, int64_t n, uint32_t mask,
                               const ixp_prop_args *args, ixp_verdict *d_out, void *ws,
                               size_t ws_bytes, void *stream) {
    if (n < 0 || !d_out || (mask & ~31u)) return IXP_EINVAL;
    if (x_t != IXP_I32 && x_t != IXP_I64) return IXP_EINVAL;
    if (n > 0 && !x) return IXP_EINVAL;
    const size_t esz = x_t == IXP_I64 ? 8 : 4;
    if (!aligned(x, 16) || !aligned(d_out, 8) || !aligned(ws, 256)) return IXP_EINVAL;
    if ((mask & ~static_cast<uint32_t>(IXP_MONO)) && !args) return IXP_EINVAL;
    ixp_prop_args dflt{};
    const ixp_prop_args *pa = args ? args : &dflt;
    if (mask & (IXP_INJ | IXP_BIJ)) {
        if (pa->hi < pa->lo || pa->hi - pa->lo > (int64_t{1} << 36)) return IXP_EINVAL;
    }
    if (mask & IXP_BIJ) {
        if (pa->img_lo > pa->img_hi || pa->img_lo < pa->lo || pa->img_hi > pa->hi) return IXP_EINVAL;
    }
    if ((mask & IXP_MONO) && (pa->mono_op < 0 || pa->mono_op > 3)) return IXP_EINVAL;
    HostPred hp{};
    if (mask & IXP_FILTPART) {
        if (pa->fp_mode != IXP_MODE_PARTITION && pa->fp_mode != IXP_MODE_FILTER) return IXP_EINVAL;
        if (!pa->fp_split || !pa->fp_dst || (n > 0 && !pa->fp_src && pa->fp_pred.kind != IXP_PRED_FLAGS))
            return IXP_EINVAL;
        int rc = check_pred(&pa->fp_pred, pa->fp_key_t, &hp, n);
        if (rc != IXP_OK) return rc;
        if (is_row_pred(hp.kind)) return IXP_EINVAL;
        if (!pa->fp_src) return IXP_EINVAL;
        if (!aligned(pa->fp_src, 4) || !aligned(pa->fp_dst, 4) || !aligned(pa->fp_split, 8)) return IXP_EINVAL;
    }
    if (!ws || ws_bytes < ixp_check_props_workspace(n, mask, pa)) return IXP_EWORKSPACE;
    (void)esz;

    hipStream_t st = as_stream(stream);
    const int64_t w = rcd_width(n, mask, pa);
    const int64_t words = (w + 127) / 128 * 4;
    char *p = static_cast<char *>(ws);
    PropsArgs a{};
    a.x = x;
    a.x64 = x_t == IXP_I64 ? 1 : 0;
    a.n = n;
    a.mask = mask;
    a.lo = (mask & (IXP_INJ | IXP_BIJ)) ? pa->lo : 0;
    a.hi = (mask & (IXP_INJ | IXP_BIJ)) ? pa->hi : 0;
    a.ilo = pa->img_lo;
    a.ihi = pa->img_hi;
    a.mono_op = pa->mono_op;
    a.st = reinterpret_cast<PropsState *>(p);
    a.seen = reinterpret_cast<uint32_t *>(p + kPropsHeader);
    a.dup = reinterpret_cast<uint32_t *>(p + kPropsHeader + round_up(words * 4, 256));
    char *fp = p + kPropsHeader + 2 * round_up(words * 4, 256);
    if (n >= (int64_t{1} << 32)) {
        a.first64 = reinterpret_cast<unsigned long long *>(fp);
        a.first = nullptr;
    } else {
        a.first = reinterpret_cast<uint32_t *>(fp);
        a.first64 = nullptr;
    }
    a.width = w;
    const size_t first_bytes = static_cast<size_t>(w) * (n >= (int64_t{1} << 32) ? 8 : 4);
    a.fp_tmax = reinterpret_cast<int64_t *>(fp + round_up(first_bytes, 256));
    a.fp_tiles = (mask & IXP_FILTPART) ? ceil_div(n, kFpTile) : 0;
    a.nbuckets = buckets_for(n, mask, pa);
    a.bucketed = a.nbuckets > 0 ? 1 : 0;
    if (a.bucketed) {
        char *bp = reinterpret_cast<char *>(a.fp_tmax) + round_up(static_cast<size_t>(a.fp_tiles) * 16, 256);
        const size_t bb = round_up(static_cast<size_t>(a.nbuckets) * 8, 256);
        a.bucket_total = reinterpret_cast<unsigned long long *>(bp);
        a.bucket_start = reinterpret_cast<unsigned long long *>(bp + bb);
        a.wg_base = reinterpret_cast<unsigned long long *>(bp + 2 * bb);
        a.records = reinterpret_cast<uint32_t *>(
            bp + 2 * bb + round_up(static_cast<size_t>(kPass1Grid) * a.nbuckets * 8, 256));
    }
    a.fp_src = static_cast<const uint32_t *>(pa->fp_src);
    a.fp_dst = static_cast<const uint32_t *>(pa->fp_dst);
    a.fp_split = pa->fp_split;
    a.fp_mode = pa->fp_mode;

    const int grid = kPass1Grid;
    const int64_t iwords = words > 0 ? words : 1;
    const uint32_t iblocks = static_cast<uint32_t>(ceil_div(iwords / 4 + 1, 256) < 4096 ? ceil_div(iwords / 4 + 1, 256) : 4096);
    IXP_LAUNCH("props_init", props_init_kernel, dim3(iblocks), dim3(256), 0, st, a.st, a.seen, a.dup, words,
               a.bucket_total, a.bucketed ? static_cast<int64_t>(a.nbuckets) : int64_t{0});
    if (launch_status() != IXP_OK) return IXP_EHIP;

    const uint32_t main_mask = mask & (IXP_RANGE | IXP_MONO | IXP_INJ | IXP_BIJ);
    if (main_mask && n > 0) {
        PropsArgs b = a;
        b.mask = main_mask;
        const size_t hist_lds = b.bucketed ? static_cast<size_t>(b.nbuckets) * 4 : 0;
        if (b.x64)
            IXP_LAUNCH("props_pass1", (props_pass1_kernel<true, 4>), dim3(grid), dim3(kPropsBlock), hist_lds, st, b);
        else
            IXP_LAUNCH("props_pass1", (props_pass1_kernel<false, 4>), dim3(grid), dim3(kPropsBlock), hist_lds, st, b);
        if (b.bucketed) {
            IXP_LAUNCH("props_bucket_scan", props_bucket_scan_kernel, dim3(1), dim3(1024), 0, st, b);
            // base[nb] + round counts/offsets [2 nb] + staged records (4 B) and bucket ids (2 B)
            const size_t place_lds = static_cast<size_t>(b.nbuckets) * 16 + static_cast<size_t>(kPlaceRound) * 6;
            if (b.x64)
                IXP_LAUNCH("props_place", (props_place_kernel<true, kPlaceRound / (kPropsBlock * 2)>), dim3(grid),
                           dim3(kPropsBlock), place_lds, st, b);
            else
                IXP_LAUNCH("props_place", (props_place_kernel<false, kPlaceRound / (kPropsBlock * 4)>), dim3(grid),
                           dim3(kPropsBlock), place_lds, st, b);
            IXP_LAUNCH("props_check", props_check_kernel, dim3(b.nbuckets), dim3(kCheckThreads), 0, st, b);
        }
        if (main_mask & (IXP_INJ | IXP_BIJ)) {
            IXP_LAUNCH("props_first", props_first_kernel, dim3(grid), dim3(kPropsBlock), 0, st, b);
            IXP_LAUNCH("props_second", props_second_kernel, dim3(grid), dim3(kPropsBlock), 0, st, b,
                       &a.st->fv_inj);
        }
        if (main_mask & IXP_BIJ)
            IXP_LAUNCH("props_missing", props_missing_kernel, dim3(grid), dim3(kPropsBlock), 0, st, b);
        if (launch_status() != IXP_OK) return IXP_EHIP;
    } else if ((main_mask & IXP_BIJ) && n == 0) {
        IXP_LAUNCH("props_missing", props_missing_kernel, dim3(grid), dim3(kPropsBlock), 0, st, a);
    }
    if (mask & IXP_FILTPART) {
        // FiltPart's bijection check uses its own bitmap over [0, n): the
        // Inj/Bij passes above are done with it.
        PropsArgs f = a;
        f.lo = 0;
        f.hi = n;
        if (main_mask & (IXP_INJ | IXP_BIJ)) {
            IXP_LAUNCH("props_init_fp", props_init_kernel, dim3(iblocks), dim3(256), 0, st,
                       static_cast<PropsState *>(nullptr), a.seen, a.dup, words,
                       static_cast<unsigned long long *>(nullptr), int64_t{0});
        }
        int rc = IXP_OK;
        switch (hp.kind) {
        case IXP_PRED_MOD_EQ: rc = launch_filtpart(f, PredModEq{hp.M, hp.d, hp.r}, st, grid); break;
        case IXP_PRED_LT: rc = launch_filtpart(f, PredLt{hp.s}, st, grid); break;
        default: rc = launch_filtpart(f, PredFlags{hp.flags}, st, grid); break;
        }
        if (rc != IXP_OK) return rc;
    }
    IXP_LAUNCH("props_finalize", props_finalize_kernel, dim3(1), dim3(64), 0, st, a, d_out);
    return launch_status();
}
