// sgmscan.hip -- sgmSum (Section 2.1, figure "Running Examples", right): the
// inclusive scan of int64 values under the lifted operator
//   (fx, vx) (+) (fy, vy) = (fx || fy, fy ? vy : vx + vy),
// i.e. a running sum that restarts at every flagged position.
//
// Reduce, scan, rescan over C <= 8192 chunks of whole 8192-element tiles:
//   reduce -- the aggregate of a chunk is (some flag, sum of the values from
//             its last flag on, that element included): one workgroup per
//             chunk finds the last flag from the flag bytes, then sums only
//             the values from there;
//   scan   -- one workgroup: exclusive scan of the C aggregates under the
//             lifted operator (8 per thread, wave shuffles, LDS);
//   rescan -- one workgroup per chunk: its tiles in order, each loaded through
//             LDS (coalesced), 8 consecutive elements per thread, waves
//             combined with shuffles and LDS, starting from the chunk's prefix.
// No inter-workgroup waiting; the values from each chunk's last flag on are
// read twice, everything else once.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr int kSgThreads = 1024;
constexpr int kSgPer = 8;
constexpr int64_t kSgTile = kSgThreads * kSgPer;
constexpr int64_t kSgMaxChunks = 8192;

struct Pair {
    bool f;
    int64_t v;
};

__device__ __forceinline__ Pair combine(Pair x, Pair y) { return Pair{x.f || y.f, y.f ? y.v : x.v + y.v}; }

struct SgArgs {
    const uint8_t *flags;
    const int64_t *xs;
    int64_t *out;
    int64_t n;
    int64_t chunk;      // elements per chunk, a multiple of kSgTile
    int64_t chunks;
    int64_t *agg_v;     // [chunks] aggregate value, then exclusive prefix value
    int32_t *agg_f;     // [chunks] aggregate flag
};

// Block-wide reductions of 1024 threads through LDS.
__device__ __forceinline__ int64_t block_max_1024(int64_t x, int64_t *lds16) {
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(x, off, kWave);
        x = o > x ? o : x;
    }
    if ((threadIdx.x & 63) == 0) lds16[threadIdx.x >> 6] = x;
    __syncthreads();
    int64_t r = lds16[0];
    for (int w = 1; w < 16; ++w) r = lds16[w] > r ? lds16[w] : r;
    __syncthreads();
    return r;
}
__device__ __forceinline__ int64_t block_sum_1024(int64_t x, int64_t *lds16) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    if ((threadIdx.x & 63) == 0) lds16[threadIdx.x >> 6] = x;
    __syncthreads();
    int64_t r = 0;
    for (int w = 0; w < 16; ++w) r += lds16[w];
    __syncthreads();
    return r;
}

// The 8 flags of a thread's 8 consecutive elements, as one 8-byte load when
// the flag array is 8-byte aligned and the group lies inside [0, len).
__device__ __forceinline__ uint64_t flag_group(const uint8_t *f, int64_t p, int64_t len, bool vec) {
    if (vec && p + 8 <= len) return *reinterpret_cast<const uint64_t *>(f + p);
    uint64_t x = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (p + k < len) x |= static_cast<uint64_t>(f[p + k]) << (8 * k);
    return x;
}

__global__ __launch_bounds__(kSgThreads) void sg_reduce_kernel(SgArgs a) {
    __shared__ int64_t lds[16];
    const int64_t c = blockIdx.x;
    const int64_t lo = c * a.chunk;
    const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
    // last flagged position of the chunk (lo - 1 if none), from 8 flag bytes per thread and step
    int64_t last = lo - 1;
    const bool fvec = (reinterpret_cast<uintptr_t>(a.flags) & 7) == 0;
    for (int64_t p = static_cast<int64_t>(threadIdx.x) * 8; lo + p < hi; p += kSgThreads * 8) {
        const uint64_t fg = flag_group(a.flags + lo, p, hi - lo, fvec);
        if (fg) last = lo + p + (63 - __builtin_clzll(fg)) / 8;
    }
    last = block_max_1024(last, lds);
    // a flagged element restarts the sum with its own value
    const int64_t start = last >= lo ? last : lo;
    int64_t s = 0;
    for (int64_t p = start + threadIdx.x; p < hi; p += kSgThreads) s += a.xs[p];
    s = block_sum_1024(s, lds);
    if (threadIdx.x == 0) {
        a.agg_v[c] = s;
        a.agg_f[c] = last >= lo ? 1 : 0;
    }
}

// One workgroup: aggregates -> exclusive prefixes (in place, values only).
__global__ __launch_bounds__(1024) void sg_chunk_scan_kernel(SgArgs a) {
    constexpr int kPer = 8;
    static_assert(kPer * 1024 >= kSgMaxChunks, "scan capacity");
    __shared__ int64_t wv[16];
    __shared__ int32_t wf[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    Pair e[kPer];
    Pair run{false, 0};
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = static_cast<int64_t>(tid) * kPer + k;
        e[k] = i < a.chunks ? Pair{a.agg_f[i] != 0, a.agg_v[i]} : Pair{false, 0};
        run = combine(run, e[k]);
    }
    Pair inc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        Pair o;
        o.f = __shfl_up(static_cast<int>(inc.f), off, kWave) != 0;
        o.v = __shfl_up(inc.v, off, kWave);
        if (lane >= off) inc = combine(o, inc);
    }
    Pair before{__shfl_up(static_cast<int>(inc.f), 1, kWave) != 0, __shfl_up(inc.v, 1, kWave)};
    if (lane == 0) before = Pair{false, 0};
    if (lane == kWave - 1) {
        wv[wave] = inc.v;
        wf[wave] = inc.f ? 1 : 0;
    }
    __syncthreads();
    Pair acc{false, 0};
    for (int w = 0; w < wave; ++w) acc = combine(acc, Pair{wf[w] != 0, wv[w]});
    acc = combine(acc, before);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = static_cast<int64_t>(tid) * kPer + k;
        if (i < a.chunks) a.agg_v[i] = acc.v;   // a flag only matters for later elements
        acc = combine(acc, e[k]);
    }
}

__global__ __launch_bounds__(kSgThreads) void sg_rescan_kernel(SgArgs a) {
    static_assert(kSgPer == 8, "one 8-byte flag group per thread");
    __shared__ int64_t sv[kSgTile];
    __shared__ int64_t wv[kSgThreads / kWave];
    __shared__ int32_t wf[kSgThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    const int64_t c = blockIdx.x;
    const int64_t lo_c = c * a.chunk;
    const int64_t hi_c = lo_c + a.chunk < a.n ? lo_c + a.chunk : a.n;
    int64_t carry = a.agg_v[c];   // value before the chunk (a flag inside the chunk resets it)
    const bool fvec = (reinterpret_cast<uintptr_t>(a.flags) & 7) == 0;
    for (int64_t lo = lo_c; lo < hi_c; lo += kSgTile) {
        const int64_t len = hi_c - lo < kSgTile ? hi_c - lo : kSgTile;
        const uint64_t fg = flag_group(a.flags + lo, static_cast<int64_t>(tid) * kSgPer, len, fvec);
#pragma unroll
        for (int k = 0; k < kSgPer; ++k) {
            const int l = k * kSgThreads + tid;
            sv[l] = l < len ? __builtin_nontemporal_load(a.xs + lo + l) : 0;
        }
        __syncthreads();
        Pair run{false, 0};
        Pair el[kSgPer];
#pragma unroll
        for (int k = 0; k < kSgPer; ++k) {
            const int l = tid * kSgPer + k;
            run = combine(run, Pair{((fg >> (8 * k)) & 0xFFu) != 0, sv[l]});
            el[k] = run;
        }
        Pair inc = run;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            Pair o;
            o.f = __shfl_up(static_cast<int>(inc.f), off, kWave) != 0;
            o.v = __shfl_up(inc.v, off, kWave);
            if (lane >= off) inc = combine(o, inc);
        }
        Pair before_lane{__shfl_up(static_cast<int>(inc.f), 1, kWave) != 0, __shfl_up(inc.v, 1, kWave)};
        if (lane == 0) before_lane = Pair{false, 0};
        if (lane == kWave - 1) {
            wv[wave] = inc.v;
            wf[wave] = inc.f ? 1 : 0;
        }
        __syncthreads();
        Pair before_wave{false, 0}, tile{false, 0};
#pragma unroll
        for (int w = 0; w < kSgThreads / kWave; ++w) {
            const Pair x{wf[w] != 0, wv[w]};
            if (w < wave) before_wave = combine(before_wave, x);
            tile = combine(tile, x);
        }
        const Pair prefix = combine(Pair{false, carry}, combine(before_wave, before_lane));
#pragma unroll
        for (int k = 0; k < kSgPer; ++k) sv[tid * kSgPer + k] = combine(prefix, el[k]).v;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSgPer; ++k) {
            const int l = k * kSgThreads + tid;
            if (l < len) stream_store(a.out + lo + l, sv[l]);
        }
        carry = combine(Pair{false, carry}, tile).v;
        __syncthreads();   // LDS reused by the next tile
    }
}

// Chunks of whole tiles, at most kSgMaxChunks of them.
void sg_geometry(int64_t n, int64_t *chunk, int64_t *chunks) {
    const int64_t tiles = ceil_div(n, kSgTile);
    const int64_t per = ceil_div(tiles, kSgMaxChunks);
    *chunk = per * kSgTile;
    *chunks = ceil_div(n, *chunk);
}

}  // namespace
}  // namespace ixp

using namespace ixp;

extern "C" size_t ixp_sgm_sum_workspace(int64_t n) {
    if (n < 0) return 0;
    int64_t chunk = 0, chunks = 0;
    sg_geometry(n > 0 ? n : 1, &chunk, &chunks);
    return round_up(static_cast<size_t>(chunks) * 8, 256) + static_cast<size_t>(chunks) * 4;
}

extern "C" int ixp_sgm_sum(const uint8_t *d_flags, const int64_t *d_xs, int64_t n, int64_t *d_out, void *ws,
                           size_t ws_bytes, void *stream) {
    if (n < 0 || (n > 0 && (!d_flags || !d_xs || !d_out))) return IXP_EINVAL;
    if (!aligned(d_xs, 8) || !aligned(d_out, 8) || !aligned(ws, 8)) return IXP_EINVAL;
    if (!ws || ws_bytes < ixp_sgm_sum_workspace(n)) return IXP_EWORKSPACE;
    if (n == 0) return IXP_OK;
    SgArgs a;
    a.flags = d_flags;
    a.xs = d_xs;
    a.out = d_out;
    a.n = n;
    sg_geometry(n, &a.chunk, &a.chunks);
    a.agg_v = static_cast<int64_t *>(ws);
    a.agg_f = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + round_up(static_cast<size_t>(a.chunks) * 8, 256));
    hipStream_t st = as_stream(stream);
    const dim3 grid(static_cast<uint32_t>(a.chunks));
    IXP_LAUNCH("sgm_reduce", sg_reduce_kernel, grid, dim3(kSgThreads), 0, st, a);
    IXP_LAUNCH("sgm_chunk_scan", sg_chunk_scan_kernel, dim3(1), dim3(1024), 0, st, a);
    IXP_LAUNCH("sgm_rescan", sg_rescan_kernel, grid, dim3(kSgThreads), 0, st, a);
    return launch_status();
}
