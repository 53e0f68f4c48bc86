// props.hip -- run-time checkers of the array properties of Section 2.3
// (figure "Array Properties"): Range, Monotonic, Inj, Bij and FiltPart.
//
// Range / Monotonic / Inj / Bij share one streaming pass over X (16-byte
// nontemporal loads).  Every failing index is reduced to the least one with a
// wave minimum and an atomicMin, so verdicts do not depend on scheduling.
//
// Inj and Bij need to know which in-Rcd values occur more than once.  For
// large arrays whose Rcd spans at most 4096 buckets of 2^20 values, the pass
// over X also groups each workgroup's chunk of in-Rcd values by bucket in LDS
// and writes the chunk's values bucket by bucket into its own region, with a
// per-chunk table of where each bucket starts (no global histogram is
// needed); then one workgroup per bucket reads that bucket's runs from every
// chunk into a 128 KiB LDS bitmap.  Smaller arrays insert into a bitmap over
// Rcd in global memory directly.  A bit found already set says that its value
// repeats, not which occurrence is the first, so each repeated value is
// listed once (a second bitmap marks it).  One more streaming pass then looks
// every in-Rcd value up in an LDS hash table of the listed values and keeps,
// per listed value, the least index seen; an arrival that displaces an
// earlier least index, or finds one already there, proposes the larger of
// the two, and the least proposal is the earliest second occurrence.  When
// more values repeat than the list holds, two global passes over a per-value
// first-index table locate it instead.
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
constexpr int kBucketShift = 20;              // 2^20 values: a 128 KiB LDS bitmap
constexpr int kMaxBuckets = 4096;
constexpr int kChunk = 16384;                 // elements per props_scan workgroup
constexpr int kScanThreads = 512;             // two workgroups per CU (64 KiB of LDS each)
constexpr int kRepCap = 2048;                 // repeated values one rescan can locate
constexpr int kRepSlots = 4 * kRepCap;        // hash table slots: load factor <= 1/4
constexpr uint64_t kEmptySlot = ~0ull;

// Device-side state at the start of the workspace.
struct PropsState {
    unsigned long long fv_range, fv_mono, fv_img, fv_inj;   // least failing index, kNone if none
    unsigned long long in_count;                            // entries inside Rcd
    unsigned long long missing;                             // least value of Img not attained, minus img_lo
    unsigned int dup_found;
    unsigned int nrep;                 // repeated values listed (may exceed the list)
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
    // Chunked Inj/Bij (props_scan / props_check): values of Rcd grouped in
    // buckets of 2^kBucketShift consecutive values.
    int32_t bucketed;
    int32_t nbuckets;
    int64_t nchunks;
    uint16_t *ctab;       // [(nbuckets + 1) * nchunks]: bucket starts per chunk; last row: chunk totals
    uint32_t *records;    // [nchunks * kChunk]: value - lo - bucket base (20 bits)
    // Repeated values (Inj's first-violation search)
    uint64_t *rep;        // [kRepCap] value - lo of each repeated value
    unsigned long long *rep_min;   // [kRepCap] least index seen per listed value
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
                                  unsigned long long *rep_min) {
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (rep_min)
        for (int64_t i = i0; i < kRepCap; i += static_cast<int64_t>(gridDim.x) * blockDim.x) rep_min[i] = kNone;
    if (i0 == 0 && st) {
        st->fv_range = st->fv_mono = st->fv_img = st->fv_inj = kNone;
        st->in_count = 0;
        st->missing = kNone;
        st->dup_found = 0;
        st->nrep = 0;
        st->fp_fv = kNone;
        st->fp_true = 0;
        st->fp_bits = 0;
    }
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    const int64_t w4 = words / 4;
    for (int64_t i = i0; i < w4; i += stride) {
        if (seen) __builtin_nontemporal_store(v4{0, 0, 0, 0}, reinterpret_cast<v4 *>(seen) + i);
        __builtin_nontemporal_store(v4{0, 0, 0, 0}, reinterpret_cast<v4 *>(dup) + i);
    }
    for (int64_t i = w4 * 4 + i0; i < words; i += stride) {
        if (seen) seen[i] = 0;
        dup[i] = 0;
    }
}

// A value found already set in the seen bitmap (o = value - lo): mark it in
// the dup bitmap, list it the first time, and reset its first-index slot for
// the global fallback passes.
__device__ __forceinline__ void note_repeat(const PropsArgs &a, uint64_t o, bool list) {
    const uint32_t bit = 1u << (o & 31);
    const uint32_t old = atomicOr(a.dup + (o >> 5), bit);
    if (list && !(old & bit)) {
        const uint32_t k = atomicAdd(&a.st->nrep, 1u);
        if (k < kRepCap) a.rep[k] = o;
    }
    if (a.first64) a.first64[o] = ~0ull;
    else a.first[o] = ~0u;
}

// Inserts v (inside [lo, hi)) into the seen bitmap; a repeat is noted.
template <bool LIST>
__device__ __forceinline__ void insert_value(const PropsArgs &a, int64_t v, bool *dup_seen) {
    const uint64_t o = static_cast<uint64_t>(v - a.lo);
    const uint32_t bit = 1u << (o & 31);
    const uint32_t old = atomicOr(a.seen + (o >> 5), bit);
    if (old & bit) {
        note_repeat(a, o, LIST);
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

// Pass 1 (arrays without the chunked path): Range, Monotonic, the Img part of
// Bij, the in-Rcd count and the bitmap insertions of Inj / Bij, for every
// element.  Each thread takes 16-byte groups (2 int64 or 4 int32); a group's
// left neighbour for the monotonic check comes from the previous lane
// (consecutive lanes hold consecutive groups), lane 0 loads it.
template <bool X64, int UNROLL>
__global__ __launch_bounds__(kPropsBlock) void props_pass1_kernel(PropsArgs a) {
    constexpr int kPer = X64 ? 2 : 4;
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
        int64_t gi[UNROLL], left[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            gi[u] = gb + u * stride;
            raw[u] = gi[u] < groups
                         ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi[u])
                         : v4{0, 0, 0, 0};
        }
        // lane 0's left neighbours, loaded beside the groups rather than
        // one dependent load per group
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            left[u] = want_mono && lane == 0 && gi[u] < groups && gi[u] > 0
                          ? load_x(a.x, X64 ? 1 : 0, gi[u] * kPer - 1)
                          : 0;
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
                if (lane == 0) prev = left[u];
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
                    insert_value<true>(a, v, &dup_seen);
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
                insert_value<true>(a, v, &dup_seen);
            }
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

// Chunked Inj/Bij.  Random device-scope atomics on a bitmap in HBM run far
// below the memory bandwidth, so the in-Rcd values are routed to one
// workgroup per bucket of 2^20 values, whose bitmap sits in LDS.
//
// props_scan: workgroup c owns elements [c kChunk, (c+1) kChunk) (chunks in
// an XCD-aware order).  Besides Range / Monotonic / Img it ranks every in-Rcd
// value inside its bucket with an LDS atomic, scans the chunk's bucket
// counts, stages the values in bucket order in LDS and writes them as one
// contiguous run to the chunk's own region of `records`; ctab row b, column
// c receives the start of bucket b inside the chunk (row nbuckets: the
// chunk's in-Rcd total).  The values are written once and read once.
template <bool X64>
__global__ __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4)))
void props_scan_kernel(PropsArgs a) {
    constexpr int kPer = X64 ? 2 : 4;                       // elements per 16-byte group
    constexpr int kGroups = kChunk / kPer / kScanThreads;   // groups per thread
    constexpr int kElems = kGroups * kPer;
    constexpr uint32_t kOut = ~0u;
    __shared__ uint32_t stage[kChunk];
    __shared__ uint32_t wtot[kScanThreads / kWave];
    __shared__ unsigned long long wmin[3][kScanThreads / kWave];
    __shared__ int64_t wlast[kGroups][kScanThreads / kWave];   // Monotonic's left neighbours
    __shared__ int64_t wfirst;
    extern __shared__ uint32_t bstart[];                    // [nbuckets + 1]
    const int nb = a.nbuckets;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const int64_t c = xcd_tile(blockIdx.x, a.nchunks);
    for (int b = tid; b <= nb; b += kScanThreads) bstart[b] = 0;
    __syncthreads();
    const bool want_range = a.mask & IXP_RANGE;
    const bool want_mono = a.mask & IXP_MONO;
    const bool want_img = a.mask & IXP_BIJ;
    const MonoCmp cmp{a.mono_op == IXP_MONO_GE || a.mono_op == IXP_MONO_GT,
                      a.mono_op == IXP_MONO_LT || a.mono_op == IXP_MONO_GT};
    const int64_t e0 = c * kChunk;
    const int64_t e1 = a.n < e0 + kChunk ? a.n : e0 + kChunk;
    const int64_t g_lo = e0 / kPer, g_hi = e1 / kPer;       // whole groups of the chunk
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    v4 raw[kGroups];
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
        const int64_t gi = g_lo + tid + u * kScanThreads;
        raw[u] = gi < g_hi ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi)
                           : v4{0, 0, 0, 0};
    }
    unsigned long long c_range = kNone, c_mono = kNone, c_img = kNone;
    if (want_mono) {
        // the last element of every wave's group u, for the lane 0 of the
        // next wave (thread 0's group u follows thread kScanThreads-1's
        // group u-1); thread 0's first left neighbour comes from memory
        if (lane == kWave - 1) {
#pragma unroll
            for (int u = 0; u < kGroups; ++u)
                wlast[u][wave] = X64 ? static_cast<int64_t>((static_cast<uint64_t>(raw[u].w) << 32) | raw[u].z)
                                     : static_cast<int64_t>(static_cast<int32_t>(raw[u].w));
        }
        if (tid == 0 && e0 > 0) wfirst = load_x(a.x, X64 ? 1 : 0, e0 - 1);
        __syncthreads();
    }
    uint32_t off[kElems], meta[kElems];   // offset in bucket; bucket << 16 | rank, or kOut
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
        const int64_t gi = g_lo + tid + u * kScanThreads;
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
        const bool live = gi < g_hi;
        const int64_t p0 = gi * kPer;
        int64_t prev = 0;
        if (want_mono) {
            // consecutive lanes hold consecutive groups
            prev = __shfl_up(val[kPer - 1], 1, 64);
            if (lane == 0)
                prev = wave > 0 ? wlast[u][wave - 1] : u > 0 ? wlast[u - 1][kScanThreads / kWave - 1] : wfirst;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int k = u * kPer + q;
            const int64_t i = p0 + q;
            const int64_t v = val[q];
            meta[k] = kOut;
            off[k] = 0;
            if (!live) continue;
            if (want_range && !(a.lo <= v && v < a.hi) && static_cast<unsigned long long>(i) < c_range)
                c_range = i;
            if (want_mono && i > 0 && !cmp.ok(prev, v) && static_cast<unsigned long long>(i) < c_mono)
                c_mono = i;
            prev = v;
            if (a.lo <= v && v < a.hi) {
                if (want_img && !(a.ilo <= v && v < a.ihi) && static_cast<unsigned long long>(i) < c_img)
                    c_img = i;
                const uint64_t o = static_cast<uint64_t>(v - a.lo);
                const uint32_t bk = static_cast<uint32_t>(o >> kBucketShift);
                off[k] = static_cast<uint32_t>(o & ((1u << kBucketShift) - 1));
                meta[k] = (bk << 16) | atomicAdd(bstart + bk, 1u);
            }
        }
    }
    // the chunk's last n % kPer elements (only in the chunk holding the end
    // of the array): thread 0, one at a time
    uint32_t toff[3] = {0, 0, 0}, tmeta[3] = {kOut, kOut, kOut};
    if (tid == 0) {
        for (int64_t i = g_hi * kPer; i < e1; ++i) {
            const int j = static_cast<int>(i - g_hi * kPer);
            const int64_t v = load_x(a.x, X64 ? 1 : 0, i);
            if (want_range && !(a.lo <= v && v < a.hi) && static_cast<unsigned long long>(i) < c_range)
                c_range = i;
            if (want_mono && i > 0 && !cmp.ok(load_x(a.x, X64 ? 1 : 0, i - 1), v) &&
                static_cast<unsigned long long>(i) < c_mono)
                c_mono = i;
            if (a.lo <= v && v < a.hi) {
                if (want_img && !(a.ilo <= v && v < a.ihi) && static_cast<unsigned long long>(i) < c_img)
                    c_img = i;
                const uint64_t o = static_cast<uint64_t>(v - a.lo);
                const uint32_t bk = static_cast<uint32_t>(o >> kBucketShift);
                toff[j] = static_cast<uint32_t>(o & ((1u << kBucketShift) - 1));
                tmeta[j] = (bk << 16) | atomicAdd(bstart + bk, 1u);
            }
        }
    }
    __syncthreads();
    // exclusive scan of the nb + 1 bucket counts (the last is 0, so it
    // becomes the chunk's total): thread t owns `per` consecutive entries
    {
        const int per = (nb + 1 + kScanThreads - 1) / kScanThreads;
        const int b0 = tid * per;
        uint32_t mine = 0;
        for (int j = 0; j < per; ++j)
            if (b0 + j <= nb) mine += bstart[b0 + j];
        uint32_t inc = mine;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == kWave - 1) wtot[wave] = inc;
        __syncthreads();
        uint32_t run = inc - mine;
        for (int w = 0; w < wave; ++w) run += wtot[w];
        for (int j = 0; j < per; ++j) {
            if (b0 + j <= nb) {
                const uint32_t cnt = bstart[b0 + j];
                bstart[b0 + j] = run;
                run += cnt;
            }
        }
    }
    __syncthreads();
    for (int b = tid; b <= nb; b += kScanThreads)
        a.ctab[static_cast<int64_t>(b) * a.nchunks + c] = static_cast<uint16_t>(bstart[b]);
#pragma unroll
    for (int k = 0; k < kElems; ++k)
        if (meta[k] != kOut) stage[bstart[meta[k] >> 16] + (meta[k] & 0xFFFFu)] = off[k];
    if (tid == 0) {
        for (int j = 0; j < 3; ++j)
            if (tmeta[j] != kOut) stage[bstart[tmeta[j] >> 16] + (tmeta[j] & 0xFFFFu)] = toff[j];
    }
    __syncthreads();
    const uint32_t total = bstart[nb];
    uint32_t *dst = a.records + c * kChunk;
    for (uint32_t j = tid; j < total / 4; j += kScanThreads) {
        const v4 w{stage[4 * j], stage[4 * j + 1], stage[4 * j + 2], stage[4 * j + 3]};
        __builtin_nontemporal_store(w, reinterpret_cast<v4 *>(dst) + j);
    }
    for (uint32_t j = total / 4 * 4 + tid; j < total; j += kScanThreads) dst[j] = stage[j];
    // least failing indices: one atomicMin per workgroup, and none when the
    // target already holds a smaller index (a permutation fails Monotonic
    // almost everywhere, and same-address atomics serialise)
    c_range = wave_min_u64(c_range);
    c_mono = wave_min_u64(c_mono);
    c_img = wave_min_u64(c_img);
    if (lane == 0) {
        wmin[0][wave] = c_range;
        wmin[1][wave] = c_mono;
        wmin[2][wave] = c_img;
    }
    __syncthreads();
    if (tid < 3) {
        unsigned long long m = kNone;
        for (int w = 0; w < kScanThreads / kWave; ++w) m = wmin[tid][w] < m ? wmin[tid][w] : m;
        unsigned long long *t = tid == 0 ? &a.st->fv_range : tid == 1 ? &a.st->fv_mono : &a.st->fv_img;
        if (m != kNone && m < __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(t, m);
    }
}

// props_check: workgroup b sets the bits of bucket b's values in a 128 KiB
// LDS bitmap.  The bucket's records are one run per chunk; a wave takes 16
// chunks at a time, 4 lanes per chunk, and reads each run as the aligned
// 16-byte quads that cover it (records of neighbouring buckets in the edge
// quads are skipped), each lane up to kCheckDepth quads per pass, all loads
// issued before the bits are set, and the next chunks' run bounds fetched
// while the current ones are read.  Plain loads: the quads of one run are
// spread over several lanes and passes, so its cache lines are met more than
// once.  A bit found set lists its value as repeated.  For Bij it also finds
// the least value of Img inside the bucket whose bit is clear; the
// workgroup of the last bucket adds up the chunks' in-Rcd totals.
constexpr int kCheckThreads = 1024;
constexpr int kBucketWords = (1 << kBucketShift) / 32;
constexpr int kCheckLanes = 4;
constexpr int kCheckDepth = 8;

__global__ __launch_bounds__(kCheckThreads) void props_check_kernel(PropsArgs a) {
    __shared__ uint32_t bits[kBucketWords];
    __shared__ unsigned long long wsum[kCheckThreads / kWave];
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    for (int w = tid; w < kBucketWords; w += kCheckThreads) bits[w] = 0;
    __syncthreads();
    const int64_t nc = a.nchunks;
    const uint16_t *rs = a.ctab + static_cast<int64_t>(b) * nc;
    const uint16_t *re = rs + nc;
    const int sub = lane / kCheckLanes, sl = lane % kCheckLanes;
    constexpr int kChunksPerWave = kWave / kCheckLanes;
    constexpr int kStride = (kCheckThreads / kWave) * kChunksPerWave;
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    bool dup_seen = false;
    unsigned long long tot = 0;
    // Sets the bits of the records at positions [s, e) of quads q, q + 4, ...
    // (one lane's share of a pass) whose values are in r.
    auto set_bits = [&](const v4 (&r)[kCheckDepth], uint32_t q0, uint32_t s, uint32_t e) {
#pragma unroll
        for (int d = 0; d < kCheckDepth; ++d) {
            const uint32_t q = q0 + sl + d * kCheckLanes;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t p = 4 * q + j;
                if (p < s || p >= e) continue;
                const uint32_t off = r[d][j];
                const uint32_t bit = 1u << (off & 31);
                const uint32_t old = atomicOr(bits + (off >> 5), bit);
                if (old & bit) {
                    note_repeat(a, (static_cast<uint64_t>(b) << kBucketShift) + off, true);
                    dup_seen = true;
                }
            }
        }
    };
    auto load_pass = [&](v4 (&r)[kCheckDepth], int64_t c, uint32_t q0, uint32_t e) {
        const v4 *rq = reinterpret_cast<const v4 *>(a.records + c * kChunk);
        const uint32_t q_hi = (e + 3) >> 2;
#pragma unroll
        for (int d = 0; d < kCheckDepth; ++d) {
            const uint32_t q = q0 + sl + d * kCheckLanes;
            r[d] = q < q_hi ? rq[q] : v4{0, 0, 0, 0};
        }
    };
    // Software pipeline over this wave's chunk batches: the first pass of
    // batch k + 1 is loaded while batch k's bits are set; the run bounds of
    // batch k + 2 are loaded meanwhile.  Runs longer than one pass (rare
    // with many buckets) take their further passes in place.
    constexpr uint32_t kPassQuads = kCheckLanes * kCheckDepth;
    int64_t c = static_cast<int64_t>(wave) * kChunksPerWave + sub;
    uint32_t s = c < nc ? rs[c] : 0u, e = c < nc ? re[c] : 0u;
    int64_t c1 = c + kStride;
    uint32_t s1 = c1 < nc ? rs[c1] : 0u, e1 = c1 < nc ? re[c1] : 0u;
    v4 cur[kCheckDepth], nxt[kCheckDepth];
    load_pass(cur, c, s >> 2, e);
    while (c - sub < nc) {   // wave-uniform
        const int64_t c2 = c1 + kStride;
        const uint32_t s2 = c2 < nc ? rs[c2] : 0u, e2 = c2 < nc ? re[c2] : 0u;
        load_pass(nxt, c1, s1 >> 2, e1);
        if (sl == 0 && c < nc) tot += e;
        set_bits(cur, s >> 2, s, e);
        for (uint32_t q0 = (s >> 2) + kPassQuads; q0 < ((e + 3) >> 2); q0 += kPassQuads) {
            load_pass(cur, c, q0, e);
            set_bits(cur, q0, s, e);
        }
#pragma unroll
        for (int d = 0; d < kCheckDepth; ++d) cur[d] = nxt[d];
        c = c1;
        s = s1;
        e = e1;
        c1 = c2;
        s1 = s2;
        e1 = e2;
    }
    const bool any_dup = ballot(dup_seen) != 0;
    if (lane == 0 && any_dup) atomicOr(&a.st->dup_found, 1u);
    if (b == a.nbuckets - 1) {
        // re is the totals row for the last bucket
        tot = wave_sum_u64(tot);
        if (lane == 0) wsum[wave] = tot;
        __syncthreads();
        if (tid == 0) {
            unsigned long long all = 0;
            for (int w = 0; w < kCheckThreads / kWave; ++w) all += wsum[w];
            a.st->in_count = all;
        }
    }
    if (!(a.mask & IXP_BIJ)) return;
    __syncthreads();
    // least value of Img inside this bucket whose bit is clear
    const int64_t v0 = a.lo + (static_cast<int64_t>(b) << kBucketShift);
    const int64_t lo_b = a.ilo > v0 ? a.ilo - v0 : 0;
    const int64_t hi_b = a.ihi - v0 < (int64_t{1} << kBucketShift) ? a.ihi - v0 : (int64_t{1} << kBucketShift);
    unsigned long long cm = kNone;
    if (lo_b < hi_b) {
        for (int64_t w = (lo_b >> 5) + tid; w <= ((hi_b - 1) >> 5); w += kCheckThreads) {
            uint32_t clear = ~bits[w];
            const int64_t wb = w << 5;
            if (wb < lo_b) clear &= ~0u << (lo_b - wb);
            if (wb + 32 > hi_b) clear &= (hi_b - wb) >= 32 ? ~0u : ((1u << (hi_b - wb)) - 1u);
            if (clear) {
                // offset from img_lo: values may be negative
                const unsigned long long v =
                    static_cast<unsigned long long>(v0 + wb + __builtin_ctz(clear) - a.ilo);
                if (v < cm) cm = v;
            }
        }
    }
    cm = wave_min_u64(cm);
    if (lane == 0 && cm != kNone) atomicMin(&a.st->missing, cm);
}

// ------------------------------------------- locating the first repeat --
__device__ __forceinline__ uint32_t rep_hash(uint64_t o, int log2_slots) {
    return static_cast<uint32_t>((o * 0x9E3779B97F4A7C15ull) >> (64 - log2_slots));
}

// Streams X once more (only when some value repeats and the list held every
// repeated value).  Each workgroup first builds an LDS hash table of the
// listed values (entry: value - lo << 12 | position in the list; the layout
// depends on the insertion order, the positions do not).  Each in-Rcd value
// is looked up; for a listed value at index i, m = atomicMin(least index of
// its list position, i) returns the previous least index, and when there
// was one, the larger of m and i is at least the value's second occurrence,
// with equality for the arrival that meets the least two.  The least such
// proposal over all values is Inj's first violation.
constexpr int kRescanThreads = 1024;   // two workgroups per CU (LDS, and at most 64 VGPRs)
constexpr int kRepPosBits = 12;
static_assert(kRepCap <= (1 << kRepPosBits), "list position field");

template <bool X64, int UNROLL>
__global__ __launch_bounds__(kRescanThreads) __attribute__((amdgpu_waves_per_eu(8)))
void props_rescan_kernel(PropsArgs a) {
    constexpr int kPer = X64 ? 2 : 4;
    __shared__ unsigned long long tab[kRepSlots];
    const uint32_t nrep = a.st->nrep;
    if (nrep == 0 || nrep > static_cast<uint32_t>(kRepCap)) return;
    uint32_t tsz = 64;
    while (tsz < 4 * nrep) tsz <<= 1;
    const int lg = __builtin_ctz(tsz);
    for (uint32_t s = threadIdx.x; s < tsz; s += blockDim.x) tab[s] = kEmptySlot;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nrep; k += blockDim.x) {
        const uint64_t o = a.rep[k];
        uint32_t h = rep_hash(o, lg);
        while (atomicCAS(tab + h, static_cast<unsigned long long>(kEmptySlot),
                         static_cast<unsigned long long>((o << kRepPosBits) | k)) != kEmptySlot)
            h = (h + 1) & (tsz - 1);
    }
    __syncthreads();
    unsigned long long cand = kNone;
    // a listed value at index i: propose its second occurrence
    auto found = [&](int64_t i, uint32_t k) {
        const unsigned long long m = atomicMin(a.rep_min + k, static_cast<unsigned long long>(i));
        if (m != kNone) {
            const unsigned long long p = m > static_cast<unsigned long long>(i) ? m : i;
            if (p < cand) cand = p;
        }
    };
    // the slot of o starting at h whose entry t was already read, or none
    auto probe = [&](int64_t i, uint64_t o, uint32_t h, unsigned long long t) {
        while (t != kEmptySlot) {
            if ((t >> kRepPosBits) == o) {
                found(i, static_cast<uint32_t>(t & ((1u << kRepPosBits) - 1)));
                return;
            }
            h = (h + 1) & (tsz - 1);
            t = tab[h];
        }
    };
    constexpr int K = UNROLL * kPer;
    const int64_t groups = a.n / kPer;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    // the next iteration's groups are loaded while this one's are looked up
    v4 raw[UNROLL], nxt[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int64_t gi = g0 + u * stride;
        raw[u] = gi < groups ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi) : v4{0, 0, 0, 0};
    }
    for (int64_t gb = g0; gb < groups; gb += UNROLL * stride) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t gi = gb + (UNROLL + u) * stride;
            nxt[u] = gi < groups ? __builtin_nontemporal_load(reinterpret_cast<const v4 *>(a.x) + gi)
                                 : v4{0, 0, 0, 0};
        }
        // every first probe is read before any is examined
        uint64_t o[K];
        uint32_t h[K];
        unsigned long long t[K];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const bool live = gb + u * stride < groups;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int k = u * kPer + q;
                int64_t v;
                if constexpr (X64)
                    v = static_cast<int64_t>((static_cast<uint64_t>(raw[u][2 * q + 1]) << 32) | raw[u][2 * q]);
                else
                    v = static_cast<int32_t>(raw[u][q]);
                const bool in = live && a.lo <= v && v < a.hi;
                o[k] = static_cast<uint64_t>(v - a.lo);
                h[k] = rep_hash(o[k], lg);
                t[k] = in ? tab[h[k]] : kEmptySlot;
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int k = u * kPer + q;
                if (t[k] != kEmptySlot) probe((gb + u * stride) * kPer + q, o[k], h[k], t[k]);
            }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) raw[u] = nxt[u];
    }
    if (g0 == 0) {
        for (int64_t i = groups * kPer; i < a.n; ++i) {
            const int64_t v = load_x(a.x, X64 ? 1 : 0, i);
            if (!(a.lo <= v && v < a.hi)) continue;
            const uint64_t ov = static_cast<uint64_t>(v - a.lo);
            const uint32_t hv = rep_hash(ov, lg);
            probe(i, ov, hv, tab[hv]);
        }
    }
    cand = wave_min_u64(cand);
    if ((threadIdx.x & 63) == 0 && cand != kNone) atomicMin(&a.st->fv_inj, cand);
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

// Fallback when more values repeat than the list holds.  Pass 2: least index
// of every repeated value.
__global__ __launch_bounds__(kPropsBlock) void props_first_kernel(PropsArgs a) {
    if (a.st->nrep <= static_cast<uint32_t>(kRepCap)) return;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        int64_t v;
        if (!inserted_value(a, i, &v) || !is_dup(a, v)) continue;
        const uint64_t o = static_cast<uint64_t>(v - a.lo);
        if (a.first64) atomicMin(a.first64 + o, static_cast<unsigned long long>(i));
        else atomicMin(a.first + o, static_cast<uint32_t>(i));
    }
}

// Fallback pass 3: least index that is not the first occurrence of its value.
__global__ __launch_bounds__(kPropsBlock) void props_second_kernel(PropsArgs a, unsigned long long *target) {
    if (a.st->nrep <= static_cast<uint32_t>(kRepCap)) return;
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
            // offset from img_lo: values may be negative
            const unsigned long long v = static_cast<unsigned long long>(wb + __builtin_ctz(clear) + a.lo - a.ilo);
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
                else insert_value<false>(a, e.z, &dup_seen);
                if ((e.z < split) != e.c) bad |= 4;
            } else if (e.c) {
                if (!(0 <= e.z && e.z < split) || e.z >= a.n) bad |= 2;
                else insert_value<false>(a, e.z, &dup_seen);
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
        else if (static_cast<int64_t>(st->in_count) != a.ihi - a.ilo)
            fail(3, a.n, a.ilo + static_cast<int64_t>(st->missing));
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
constexpr int kRescanGrid = 512;

// Inj/Bij take the chunked path when Rcd spans at most kMaxBuckets buckets
// and the array is large enough for the extra pass to pay.
int buckets_for(int64_t n, uint32_t mask, const ixp_prop_args *a) {
    if (!(mask & (IXP_INJ | IXP_BIJ)) || !a) return 0;
    const int64_t w = a->hi - a->lo;
    if (w <= 0 || n < (int64_t{1} << 16) || n >= (int64_t{1} << 43)) return 0;
    const int64_t b = (w + (int64_t{1} << kBucketShift) - 1) >> kBucketShift;
    // one workgroup reads each bucket: with more than 2^22 values per bucket
    // on average the global bitmap is faster
    if (n > (b << 22)) return 0;
    return b <= kMaxBuckets ? static_cast<int>(b) : 0;
}

int64_t chunks_for(int64_t n) { return ceil_div(n, kChunk); }

// Chunked path: the chunks' records and the bucket-start table.
size_t bucket_bytes(int64_t n, int nb) {
    if (!nb) return 0;
    const int64_t nc = chunks_for(n);
    return round_up(static_cast<size_t>(nc) * kChunk * 4, 256) +
           round_up(static_cast<size_t>(nb + 1) * nc * 2, 256);
}

// The repeated-value list, its hash table and each slot's least index.
constexpr size_t kRepBytes = 2 * static_cast<size_t>(kRepCap) * 8;

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
           round_up(static_cast<size_t>(tiles) * 16, 256) + kRepBytes +
           bucket_bytes(n, buckets_for(n, mask, a));
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
    char *rp = reinterpret_cast<char *>(a.fp_tmax) + round_up(static_cast<size_t>(a.fp_tiles) * 16, 256);
    a.rep = reinterpret_cast<uint64_t *>(rp);
    a.rep_min = reinterpret_cast<unsigned long long *>(a.rep + kRepCap);
    if (a.bucketed) {
        char *bp = rp + kRepBytes;
        a.nchunks = chunks_for(n);
        a.records = reinterpret_cast<uint32_t *>(bp);
        a.ctab = reinterpret_cast<uint16_t *>(bp + round_up(static_cast<size_t>(a.nchunks) * kChunk * 4, 256));
    }
    a.fp_src = static_cast<const uint32_t *>(pa->fp_src);
    a.fp_dst = static_cast<const uint32_t *>(pa->fp_dst);
    a.fp_split = pa->fp_split;
    a.fp_mode = pa->fp_mode;

    const int grid = kPass1Grid;
    const int64_t iwords = words > 0 ? words : 1;
    const uint32_t iblocks = static_cast<uint32_t>(ceil_div(iwords / 4 + 1, 256) < 4096 ? ceil_div(iwords / 4 + 1, 256) : 4096);
    // the chunked path reads no seen bitmap: only the dup bitmap is cleared
    IXP_LAUNCH("props_init", props_init_kernel, dim3(iblocks), dim3(256), 0, st, a.st,
               a.bucketed ? static_cast<uint32_t *>(nullptr) : a.seen, a.dup, words, a.rep_min);
    if (launch_status() != IXP_OK) return IXP_EHIP;

    const uint32_t main_mask = mask & (IXP_RANGE | IXP_MONO | IXP_INJ | IXP_BIJ);
    if (main_mask && n > 0) {
        PropsArgs b = a;
        b.mask = main_mask;
        if (b.bucketed) {
            const size_t scan_lds = static_cast<size_t>(b.nbuckets + 1) * 4;   // bucket counts
            if (b.x64)
                IXP_LAUNCH("props_scan", props_scan_kernel<true>, dim3(static_cast<uint32_t>(b.nchunks)),
                           dim3(kScanThreads), scan_lds, st, b);
            else
                IXP_LAUNCH("props_scan", props_scan_kernel<false>, dim3(static_cast<uint32_t>(b.nchunks)),
                           dim3(kScanThreads), scan_lds, st, b);
            IXP_LAUNCH("props_check", props_check_kernel, dim3(b.nbuckets), dim3(kCheckThreads), 0, st, b);
        } else if (b.x64) {
            IXP_LAUNCH("props_pass1", (props_pass1_kernel<true, 4>), dim3(grid), dim3(kPropsBlock), 0, st, b);
        } else {
            IXP_LAUNCH("props_pass1", (props_pass1_kernel<false, 4>), dim3(grid), dim3(kPropsBlock), 0, st, b);
        }
        if (main_mask & (IXP_INJ | IXP_BIJ)) {
            if (b.x64)
                IXP_LAUNCH("props_rescan", (props_rescan_kernel<true, 2>), dim3(kRescanGrid), dim3(kRescanThreads),
                           0, st, b);
            else
                IXP_LAUNCH("props_rescan", (props_rescan_kernel<false, 1>), dim3(kRescanGrid), dim3(kRescanThreads),
                           0, st, b);
            IXP_LAUNCH("props_first", props_first_kernel, dim3(grid), dim3(kPropsBlock), 0, st, b);
            IXP_LAUNCH("props_second", props_second_kernel, dim3(grid), dim3(kPropsBlock), 0, st, b,
                       &a.st->fv_inj);
        }
        if ((main_mask & IXP_BIJ) && !b.bucketed)   // props_check finds it on the chunked path
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
                       static_cast<unsigned long long *>(nullptr));
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
