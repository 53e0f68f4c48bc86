// flat.hip -- flat stable partition (partition2) and filter on gfx950.
//
// partition2 (Section 2.1, figure "Running Examples") evaluates the
// predicate on every element, counts trues and falses with two inclusive
// scans, sends a true to its true count minus one and a false to the number
// of trues plus its false count minus one, and scatters the elements there.
// Here the two scans collapse into one exclusive count of trues E(i), since
// #falses before i = i - E(i); the index map becomes
//   idx[i] = c_i ? E(i) : T + i - E(i)            (T = num_true)
// which is the closed form of `indices` the paper derives (Section 2.3).
// Filter keeps only the trues: idx[i] = c_i ? E(i) : -1.
//
// Partition (three kernels on the caller's stream).  The falses cannot be
// placed before T is known, so a counting pass comes first; it yields every
// tile's true count, which makes a look-back unnecessary:
//   count     -- one wave per tile (nontemporal vector loads, ballot +
//                popcount), writes the tile's count;
//   tile_scan -- one workgroup: exclusive scan of the tile counts (DPP wave
//                scans), writes each tile's prefix, T and clears the error word;
//   scatter   -- one workgroup per tile: flags by ballot, in-tile ranks by
//                mbcnt, the tile prefix by one load; indices written in input
//                order with vector stores, keys staged in LDS in output order
//                and written as the tile's two contiguous runs.
// Up to 1024 tiles (n <= 2^22) skip the tile scan: one workgroup counts each
// tile (a wave per 1024 elements), and each scatter workgroup adds up the tile
// counts before its tile and in total itself.
// Filter (single pass, two kernels):
//   init      -- clears the tile descriptors, ticket and error word;
//   scan      -- tiles taken in ticket order; each publishes its count, finds
//                its prefix by decoupled look-back over the descriptors,
//                publishes its inclusive prefix, then writes as above.  The
//                last tile writes T.
#include <atomic>
#include <mutex>

#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr size_t kWsHeader = 256;   // ticket (u32), error word (i32), padding

// Tile geometry.  Partition: 256 threads x 4 rows x 4 = 4096 elements per
// tile (the count kernel uses the same tiles).  Filter: 1024 x 4 x 4 = 16384:
// every filter tile takes one ticket from a single counter, whose atomics
// serialise (~10 ns each), and its look-back must reach a published inclusive
// prefix in one round, so fewer, larger tiles go faster.  Unaligned buffers
// use one-element groups (VEC = 1).
#ifndef IXP_FLAT_PART_BLOCK
#define IXP_FLAT_PART_BLOCK 256
#endif
#ifndef IXP_FLAT_PART_ROWS
#define IXP_FLAT_PART_ROWS 4
#endif
#ifndef IXP_FLAT_FILT_BLOCK
#define IXP_FLAT_FILT_BLOCK 1024
#endif
#ifndef IXP_VEC_RUNS
#define IXP_VEC_RUNS 1
#endif
#ifndef IXP_XCD_MAP
#define IXP_XCD_MAP 1
#endif
// rows of 64 x 4 elements a counting wave loads at once
#ifndef IXP_COUNT_ROWS
#define IXP_COUNT_ROWS 16
#endif

template <int MODE, int VEC>
struct FlatCfg {
    static constexpr int kBlock = MODE == IXP_MODE_PARTITION ? IXP_FLAT_PART_BLOCK : IXP_FLAT_FILT_BLOCK;
    static constexpr int kRows = VEC == 4 ? (MODE == IXP_MODE_PARTITION ? IXP_FLAT_PART_ROWS : 4)
                                          : 16 * (MODE == IXP_MODE_PARTITION ? IXP_FLAT_PART_ROWS : 4) / 4;
    using T = Tile<kBlock, kRows, VEC>;
    static constexpr int kTile = T::kSize;
};

struct FlatArgs {
    const uint32_t *keys;
    int64_t n;
    uint32_t *out_keys;
    void *out_idx;
    int64_t *split;
    uint64_t *desc;
    uint32_t *ticket;
    int32_t *err;
    int64_t num_tiles;
    int64_t *wsum;            // partition: per counting wave total, then prefix
    int64_t tiles_per_wave;   // partition: tiles owned by one counting wave
    int32_t need_keys;
};

// A partition of at most this many tiles skips the one-workgroup tile scan:
// one workgroup counts each tile (a wave per kSmallChunk elements), and every
// scatter workgroup adds up the tile counts itself (4 words per thread) and
// tile 0 writes T.
constexpr int64_t kSmallTiles = 1024;
constexpr int64_t kSmallChunk = 1024;

// Counting waves per partition call (fixed, so the workspace size does not
// depend on the device).
constexpr int64_t kCountWaves = 8192;

// Resident partition-scatter workgroups per CU.  Fewer tiles in flight means
// fewer interleaved output streams (an index run and two key runs per tile):
// measured on 2^28 f32, 3 per CU takes 548 us where the 7 that registers and
// LDS allow take 584 us (2 per CU: 565 us, 4: 581 us).
constexpr int kScatterWgsPerCu = 3;

__global__ void flat_init_kernel(uint32_t *ticket, int32_t *err, uint64_t *desc, int64_t num_desc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        *ticket = 0;
        *err = 0;
    }
    for (int64_t j = i; j < num_desc; j += static_cast<int64_t>(gridDim.x) * blockDim.x)
        desc[j] = 0;
}

// Counting: wave w owns the contiguous tiles [w*k, w*k + k) (k =
// tiles_per_wave).  It counts them in order, a whole 4096-element tile at a
// time (16 vector loads in flight per lane), writes
// each tile's exclusive prefix inside the run to desc[t] and the run total to
// wsum[w].
template <int VEC, class Pred>
__global__ __launch_bounds__(256) void flat_count_kernel(FlatArgs a, Pred pred) {
    constexpr int kTile = FlatCfg<IXP_MODE_PARTITION, VEC>::kTile;
    using WT = Tile<kWave, (VEC == 4 ? IXP_COUNT_ROWS : 16), VEC>;
    constexpr int kChunks = kTile / WT::kSize;
    static_assert(kChunks * WT::kSize == kTile, "count chunks");
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t w = static_cast<int64_t>(blockIdx.x) * (256 / kWave) + wave_id();
    const int64_t t0 = w * a.tiles_per_wave;
    const int64_t t1 = t0 + a.tiles_per_wave < a.num_tiles ? t0 + a.tiles_per_wave : a.num_tiles;
    uint64_t run = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t lo = t * kTile;
        const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;
        uint32_t cnt = 0;
        for (int c = 0; c < kChunks; ++c) {
            WT chunk;
            chunk.load(a.keys, a.n, lo + c * WT::kSize, lo, hi, pred, !Pred::kUsesFlags, 0, lane);
            cnt += chunk.wave_count();
        }
        if (lane == 0) a.desc[t] = run;
        run += cnt;
    }
    if (lane == 0 && w < kCountWaves) a.wsum[w] = static_cast<int64_t>(run);
}

// Small partitions: workgroup t counts tile t, one wave per kSmallChunk
// elements, and writes the tile's count to wsum[t].
template <int VEC, class Pred>
__global__ __launch_bounds__(256) void flat_count_small_kernel(FlatArgs a, Pred pred) {
    using WT = Tile<kWave, kSmallChunk / (kWave * VEC), VEC>;
    constexpr int kTile = FlatCfg<IXP_MODE_PARTITION, VEC>::kTile;
    static_assert(WT::kSize == kSmallChunk && kTile == 4 * kSmallChunk, "one chunk per wave");
    __shared__ uint32_t wc[4];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = wave_id();
    const int64_t t = blockIdx.x;
    const int64_t tlo = t * kTile;
    const int64_t thi = tlo + kTile < a.n ? tlo + kTile : a.n;
    const int64_t lo = tlo + static_cast<int64_t>(wave) * kSmallChunk;
    uint32_t cnt = 0;
    if (lo < thi) {   // wave-uniform
        // [lo, thi) bounds the valid positions; the chunk itself covers
        // [lo, lo + kSmallChunk).  (Passing min(thi, lo + kSmallChunk) here
        // made hipcc select the bound on a stale SCC after a VCC compare.)
        WT chunk;
        chunk.load(a.keys, a.n, lo, lo, thi, pred, !Pred::kUsesFlags, 0, lane);
        cnt = chunk.wave_count();
    }
    if (lane == 0) wc[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) a.wsum[t] = static_cast<int64_t>(wc[0]) + wc[1] + wc[2] + wc[3];
}

// One workgroup of 1024 threads turns wsum[0..nw) (nw <= 8 * 1024) from run
// totals into exclusive prefixes, in place, and writes T.  Thread i holds the
// 8 consecutive entries [8i, 8i+8) in registers; the thread sums are scanned
// inside each wave with shuffles and across the 16 waves through LDS.
__global__ __launch_bounds__(1024) void flat_tile_scan_kernel(int64_t *wsum, int64_t nw,
                                                              int64_t *split, int32_t *err) {
    constexpr int kPer = 8;
    static_assert(kPer * 1024 >= kCountWaves, "scan capacity");
    __shared__ int64_t wtot[16];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = wave_id();
    int64_t v[kPer];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = static_cast<int64_t>(tid) * kPer + k;
        v[k] = i < nw ? wsum[i] : 0;
        run += v[k];
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
    int64_t acc = before + inc - run;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = static_cast<int64_t>(tid) * kPer + k;
        if (i < nw) wsum[i] = acc;
        acc += v[k];
    }
    if (tid == 0) {
        *split = total;
        *err = 0;
    }
}

// Partition paths (PATH):
//   0  the tile prefix and T come from the counting kernel and the tile scan;
//   1  at most kSmallTiles tiles, counted by flat_count_small (one
//      workgroup per tile, one wave per 1024 elements): every workgroup adds
//      up the tile counts before its own and in total itself, and tile 0
//      writes T.
template <int VEC, class Pred, int MODE, class Idx, int PATH = 0>
__global__ __launch_bounds__((FlatCfg<MODE, VEC>::kBlock)) void flat_scan_kernel(FlatArgs a, Pred pred) {
    using Cfg = FlatCfg<MODE, VEC>;
    using T = typename Cfg::T;
    constexpr int kTile = T::kSize;
    constexpr int kRows = Cfg::kRows;
    constexpr int kBlock = Cfg::kBlock;
    static_assert(PATH == 0 || MODE == IXP_MODE_PARTITION, "small paths are partitions");
    __shared__ uint32_t stage[kTile];
    __shared__ uint32_t wtot[T::kWaves];
    __shared__ int64_t sh[2];
    __shared__ int64_t sh_small[PATH > 0 ? T::kWaves : 1][2];

    const int tid = threadIdx.x;
    const int wave = wave_id();
    const int lane = tid & (kWave - 1);
    int64_t t;
    if (MODE == IXP_MODE_PARTITION) {
#if IXP_XCD_MAP
        t = PATH > 0 ? blockIdx.x : xcd_tile(blockIdx.x, a.num_tiles);
#else
        t = blockIdx.x;
#endif
    } else {
        if (tid == 0) sh[0] = atomicAdd(a.ticket, 1u);
        __syncthreads();
        t = sh[0];
    }
    const int64_t lo = t * kTile;
    const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;
    // path 0: the tile prefix and T are ready before the kernel starts
    int64_t excl = 0, total = 0;
    if (MODE == IXP_MODE_PARTITION && PATH == 0) {
        excl = static_cast<int64_t>(a.desc[t]) + a.wsum[t / a.tiles_per_wave];
        total = *a.split;
    }

    // small path: wsum[j] is tile j's count; each thread's share of the
    // counts is loaded before the tile, so the two loads overlap
    constexpr int kPer = PATH > 0 ? (kSmallTiles + kBlock - 1) / kBlock : 1;
    int64_t cnt[kPer];
    if constexpr (PATH > 0) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t j = static_cast<int64_t>(tid) * kPer + k;
            cnt[k] = j < a.num_tiles ? a.wsum[j] : 0;
        }
    }

    T tile;
    tile.load(a.keys, a.n, lo, lo, hi, pred, a.need_keys != 0, wave, lane);
    tile.wave_ranks();
    if constexpr (PATH > 0) {
        int64_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t j = static_cast<int64_t>(tid) * kPer + k;
            all += cnt[k];
            before += j < t ? cnt[k] : 0;
        }
        before = wave_sum_i64(before);
        all = wave_sum_i64(all);
        if (lane == 0) {
            sh_small[wave][0] = before;
            sh_small[wave][1] = all;
        }
    }
    // (its barrier also publishes sh_small)
    const uint32_t tcount = tile.block_ranks(wtot, wave, lane);

    if constexpr (PATH > 0) {
        for (int w = 0; w < T::kWaves; ++w) {
            excl += sh_small[w][0];
            total += sh_small[w][1];
        }
        if (t == 0 && tid == 0) {
            *a.split = total;
            *a.err = 0;
        }
    }

    if (MODE == IXP_MODE_FILTER) {
        if (tid == 0 && t > 0) desc_store(a.desc + t, kStA | tcount);
        if (wave == 0) {
            const int64_t e = t == 0 ? 0 : lookback<4>(a.desc, t, 0, a.err);
            if (lane == 0) {
                desc_store(a.desc + t, kStP | static_cast<uint64_t>(e + tcount));
                sh[1] = e;
                if (t == a.num_tiles - 1) *a.split = e + tcount;
            }
        }
        __syncthreads();
        excl = sh[1];
    }
    const int64_t false_base = total + (lo - excl);   // T + #falses before the tile

    Idx *out_idx = static_cast<Idx *>(a.out_idx);
    const bool full = hi - lo == kTile;   // wave-uniform
    const int32_t l0 = wave * T::kPerWave + lane * VEC;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t p0 = T::pos(lo, wave, r, lane, 0);
        Idx v[VEC];
        uint32_t vm = 0;
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const uint32_t rt = tile.rank[r][q];
            const uint32_t rf = static_cast<uint32_t>(l0 + r * (kWave * VEC) + q) - rt;
            const bool f = tile.flag(r, q);
            const bool ok = tile.valid(r, q);
            vm |= static_cast<uint32_t>(ok) << q;
            if (MODE == IXP_MODE_PARTITION)
                v[q] = static_cast<Idx>(f ? excl + rt : false_base + rf);
            else
                v[q] = static_cast<Idx>(f ? excl + rt : -1);
            if (a.out_keys && ok && (MODE == IXP_MODE_PARTITION || f))
                stage[f ? rt : tcount + rf] = tile.key[r][q];
        }
        if (out_idx) {
            if (full) store_idx_group<VEC, Idx>(out_idx, p0, v, (1u << VEC) - 1);
            else if (vm) store_idx_group<VEC, Idx>(out_idx, p0, v, vm);
        }
    }
    if (a.out_keys) {
        __syncthreads();
        const int64_t nvalid = hi - lo;
#if IXP_VEC_RUNS
        write_run<kBlock>(stage, 0, tcount, excl, a.out_keys, a.n, tid);
        if (MODE == IXP_MODE_PARTITION)
            write_run<kBlock>(stage, tcount, static_cast<uint32_t>(nvalid) - tcount, false_base, a.out_keys, a.n, tid);
#else
        const int64_t nout = MODE == IXP_MODE_PARTITION ? nvalid : static_cast<int64_t>(tcount);
        for (int64_t s = tid; s < nout; s += kBlock) {
            const int64_t dst = s < tcount ? excl + s : false_base + (s - tcount);
            if (dst < a.n) stream_store(a.out_keys + dst, stage[s]);
        }
#endif
    }
}

template <int VEC, class Pred>
int launch_flat(FlatArgs a, const Pred &pred, int mode, int idx_t, hipStream_t st) {
    const int64_t n = a.n;
    if (mode == IXP_MODE_PARTITION) {
        using Cfg = FlatCfg<IXP_MODE_PARTITION, VEC>;
        a.num_tiles = ceil_div(n, Cfg::kTile);
        const int64_t nt = a.num_tiles;
        int64_t nw = 0;
        const bool small = nt > 0 && nt <= kSmallTiles;
        if (small) {
            IXP_LAUNCH("flat_count", (flat_count_small_kernel<VEC, Pred>), dim3(static_cast<uint32_t>(nt)),
                       dim3(256), 0, st, a, pred);
        } else if (nt > 0) {
            a.tiles_per_wave = ceil_div(nt, kCountWaves);
            nw = ceil_div(nt, a.tiles_per_wave);
            IXP_LAUNCH("flat_count", (flat_count_kernel<VEC, Pred>),
                       dim3(static_cast<uint32_t>(ceil_div(nw, 4))), dim3(256), 0, st, a, pred);
        }
        if (!small)
            IXP_LAUNCH("flat_tile_scan", flat_tile_scan_kernel, dim3(1), dim3(1024), 0, st, a.wsum, nw,
                       a.split, a.err);
        if (nt == 0) return launch_status();
        // at most kScatterWgsPerCu scatter workgroups per CU (LDS reserved at launch)
        const size_t cap = VEC == 4 ? lds_for_wgs_per_cu(kScatterWgsPerCu, Cfg::kTile * 4 + 256) : 0;
        if (small) {
            if (idx_t == IXP_I32)
                IXP_LAUNCH("flat_scatter_partition",
                           (flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int32_t, 1>),
                           dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), 0, st, a, pred);
            else
                IXP_LAUNCH("flat_scatter_partition",
                           (flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int64_t, 1>),
                           dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), 0, st, a, pred);
        } else if (idx_t == IXP_I32) {
            IXP_LAUNCH("flat_scatter_partition", (flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int32_t>),
                       dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), cap, st, a, pred);
        } else {
            IXP_LAUNCH("flat_scatter_partition", (flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int64_t>),
                       dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), cap, st, a, pred);
        }
    } else {
        using Cfg = FlatCfg<IXP_MODE_FILTER, VEC>;
        a.num_tiles = ceil_div(n, Cfg::kTile);
        const int64_t nt = a.num_tiles;
        const int64_t iblocks = nt > 0 ? (ceil_div(nt, 256) < 1024 ? ceil_div(nt, 256) : 1024) : 1;
        IXP_LAUNCH("flat_init", flat_init_kernel, dim3(static_cast<uint32_t>(iblocks)), dim3(256), 0, st,
                   a.ticket, a.err, a.desc, nt);
        if (nt == 0) {
            // T = 0: let the tile scan of zero tiles write it
            IXP_LAUNCH("flat_tile_scan", flat_tile_scan_kernel, dim3(1), dim3(1024), 0, st, a.wsum,
                       int64_t{0}, a.split, a.err);
            return launch_status();
        }
        if (idx_t == IXP_I32)
            IXP_LAUNCH("flat_scan_filter", (flat_scan_kernel<VEC, Pred, IXP_MODE_FILTER, int32_t>),
                       dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), 0, st, a, pred);
        else
            IXP_LAUNCH("flat_scan_filter", (flat_scan_kernel<VEC, Pred, IXP_MODE_FILTER, int64_t>),
                       dim3(static_cast<uint32_t>(nt)), dim3(Cfg::kBlock), 0, st, a, pred);
    }
    return launch_status();
}

template <int VEC>
int dispatch_pred(const FlatArgs &a, const HostPred &hp, int mode, int idx_t, hipStream_t st) {
    switch (hp.kind) {
    case IXP_PRED_MOD_EQ: {
        PredModEq p{hp.M, hp.d, hp.r};
        return launch_flat<VEC>(a, p, mode, idx_t, st);
    }
    case IXP_PRED_LT: {
        PredLt p{hp.s};
        return launch_flat<VEC>(a, p, mode, idx_t, st);
    }
    default: {
        PredFlags p{hp.flags};
        return launch_flat<VEC>(a, p, mode, idx_t, st);
    }
    }
}

}  // namespace

}  // namespace ixp

using namespace ixp;

// The workspace holds one descriptor per tile of the smallest tile size in use.
extern "C" size_t ixp_partition_workspace(int64_t n) {
    if (n < 0) return 0;
    const int64_t nt = ceil_div(n, FlatCfg<IXP_MODE_PARTITION, 1>::kTile);
    return kWsHeader + kCountWaves * sizeof(int64_t) +
           round_up(static_cast<size_t>(nt) * sizeof(uint64_t), 256);
}

namespace {

// The body of ixp_partition over a workspace `ws` of `ws_bytes` bytes (the
// caller's, or the static scratch of ixp_partition_noalloc).
int partition_impl(const void *keys, int32_t key_t, int64_t n, const ixp_pred *pred,
                   int32_t mode, void *out_keys, void *out_idx, int32_t idx_t,
                   int64_t *d_split, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || !d_split) return IXP_EINVAL;
    if (mode != IXP_MODE_PARTITION && mode != IXP_MODE_FILTER) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (idx_t == IXP_I32 && n > 0x7FFFFFFFll) return IXP_EINVAL;
    if (key_t != IXP_I32 && key_t != IXP_F32) return key_t == IXP_I64 ? IXP_EUNSUPPORTED : IXP_EINVAL;
    HostPred hp;
    int rc = check_pred(pred, key_t, &hp, n);
    if (rc != IXP_OK) return rc;
    if (is_row_pred(hp.kind)) return IXP_EINVAL;   // a flat array has no rows
    const bool need_keys = hp.kind != IXP_PRED_FLAGS || out_keys != nullptr;
    if (n > 0 && need_keys && !keys) return IXP_EINVAL;
    if (!ws || ws_bytes < ixp_partition_workspace(n)) return IXP_EWORKSPACE;
    const size_t isz = idx_t == IXP_I32 ? 4 : 8;
    if (!aligned(keys, 4) || !aligned(out_keys, 4) || !aligned(out_idx, isz) ||
        !aligned(d_split, 8) || !aligned(ws, 8))
        return IXP_EINVAL;

    hipStream_t st = as_stream(stream);
    char *w = static_cast<char *>(ws);
    FlatArgs a;
    a.keys = static_cast<const uint32_t *>(keys);
    a.n = n;
    a.out_keys = static_cast<uint32_t *>(out_keys);
    a.out_idx = out_idx;
    a.split = d_split;
    a.ticket = reinterpret_cast<uint32_t *>(w);
    a.err = reinterpret_cast<int32_t *>(w + 4);
    a.wsum = reinterpret_cast<int64_t *>(w + kWsHeader);
    a.desc = reinterpret_cast<uint64_t *>(w + kWsHeader + kCountWaves * sizeof(int64_t));
    a.num_tiles = 0;
    a.tiles_per_wave = 1;
    a.need_keys = need_keys ? 1 : 0;

    const bool vec4 = aligned(keys, 16) && aligned(out_idx, 16) &&
                      (hp.kind != IXP_PRED_FLAGS || aligned(hp.flags, 4));
    return vec4 ? dispatch_pred<4>(a, hp, mode, idx_t, st) : dispatch_pred<1>(a, hp, mode, idx_t, st);
}

// Static scratch of ixp_partition_noalloc: one copy per device, allocated when
// the code object is loaded and kept until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it only names the symbol);
// it passes the device address hipGetSymbolAddress returns for the current
// device.  Every kernel of the flat path clears, before use, the header words
// and descriptors it reads, so nothing left by an earlier call is consumed.
static __device__ __align__(256) unsigned char scratch[IXP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return IXP_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return IXP_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IXP_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return IXP_OK;
}

}  // namespace

extern "C" int ixp_partition(const void *keys, int32_t key_t, int64_t n, const ixp_pred *pred,
                             int32_t mode, void *out_keys, void *out_idx, int32_t idx_t,
                             int64_t *d_split, void *ws, size_t ws_bytes, void *stream) {
    return partition_impl(keys, key_t, n, pred, mode, out_keys, out_idx, idx_t, d_split, ws,
                          ws_bytes, stream);
}

extern "C" int ixp_partition_noalloc(const void *keys, int32_t key_t, int64_t n,
                                     const ixp_pred *pred, int32_t mode, void *out_keys,
                                     void *out_idx, int32_t idx_t, int64_t *d_split,
                                     void *stream) {
    if (n < 0) return IXP_EINVAL;
    if (ixp_partition_workspace(n) > IXP_NOALLOC_SCRATCH_BYTES) return IXP_ETOOLARGE;
    void *ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc != IXP_OK) return rc;
    return partition_impl(keys, key_t, n, pred, mode, out_keys, out_idx, idx_t, d_split, ws,
                          IXP_NOALLOC_SCRATCH_BYTES, stream);
}
