// sgmscan.hip -- sgmSum (Section 2.1, figure "Running Examples", right): the
// inclusive scan of int64 values under the lifted operator
//   (fx, vx) (+) (fy, vy) = (fx || fy, fy ? vy : vx + vy),
// i.e. a running sum that restarts at every flagged position.
//
// Single pass over tiles of 8192 elements taken in ticket order.  A tile
// holding a flag knows its inclusive value (the sum after its last flag)
// without its predecessors, so it publishes it as an inclusive prefix at once;
// the look-back of a later tile therefore stops at the nearest flagged tile or
// published prefix.  Values are int64 of any sign, so each descriptor is a
// status word plus separate values, published value first, status second;
// the aggregate and the inclusive value of a tile have separate slots, so a
// reader that saw one status reads the value written for it.
// Inside a tile: loads and stores go through LDS so that global accesses are
// coalesced, each thread scans 8 consecutive elements, waves combine their
// threads with shuffles and the workgroup combines its waves in LDS.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr int kSgThreads = 1024;
constexpr int kSgPer = 8;
constexpr int kSgTile = kSgThreads * kSgPer;
constexpr size_t kSgHeader = 256;   // ticket u32 @0, error i32 @4
constexpr uint32_t kSgA = 1, kSgP = 2;

struct SgArgs {
    const uint8_t *flags;
    const int64_t *xs;
    int64_t *out;
    int64_t n;
    int64_t num_tiles;
    uint32_t *ticket;
    int32_t *err;
    uint32_t *status;   // [num_tiles] 0, aggregate published, or inclusive published
    int64_t *agg;       // [num_tiles] written once, before status A
    int64_t *incl;      // [num_tiles] written once, before status P
};

struct Pair {
    bool f;
    int64_t v;
};

__device__ __forceinline__ Pair combine(Pair x, Pair y) { return Pair{x.f || y.f, y.f ? y.v : x.v + y.v}; }

__global__ void sg_init_kernel(SgArgs a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        *a.ticket = 0;
        *a.err = 0;
    }
    for (int64_t j = i; j < a.num_tiles; j += static_cast<int64_t>(gridDim.x) * blockDim.x) a.status[j] = 0;
}

__device__ __forceinline__ void publish(SgArgs &a, int64_t t, uint32_t st, int64_t v) {
    (st == kSgP ? a.incl : a.agg)[t] = v;
    __threadfence();
    __hip_atomic_store(a.status + t, st, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the values of tiles [j, t) back to the nearest inclusive prefix
// (whose value is included), by one wave, 64 predecessors per round.
__device__ __forceinline__ int64_t sg_lookback(const SgArgs &a, int64_t t, int lane) {
    int64_t excl = 0;
    int64_t j = t - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        const int64_t i = j - lane;
        const uint32_t st = i >= 0 ? __hip_atomic_load(a.status + i, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                                   : kSgP;
        const uint64_t mP = ballot(st == kSgP);
        // tiles from this lane up to the nearest inclusive prefix (lanes 0..firstP)
        const int firstP = mP ? __builtin_ctzll(mP) : kWave;
        const uint64_t upto = firstP < kWave ? ((2ull << firstP) - 1) : ~0ull;
        if (ballot(st == 0) & upto) {
            if (++spins > kSpinLimit) {
                if (lane == 0) set_error(a.err, kErrSpin);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        int64_t v = 0;
        if (((upto >> lane) & 1ull) && i >= 0) v = st == kSgP ? a.incl[i] : a.agg[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        excl += v;
        if (mP) break;
        j -= kWave;
    }
    return excl;
}

__global__ __launch_bounds__(kSgThreads) void sg_scan_kernel(SgArgs a) {
    __shared__ int64_t sv[kSgTile];
    __shared__ uint8_t sf[kSgTile];
    __shared__ int64_t wv[kSgThreads / kWave];
    __shared__ int32_t wf[kSgThreads / kWave];
    __shared__ int64_t sh[2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id();
    if (tid == 0) sh[0] = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t t = sh[0];
    const int64_t lo = t * kSgTile;
    const int64_t len = a.n - lo < kSgTile ? a.n - lo : kSgTile;
    // coalesced loads into LDS (positions past the end hold a neutral element)
#pragma unroll
    for (int k = 0; k < kSgPer; ++k) {
        const int l = k * kSgThreads + tid;
        sv[l] = l < len ? a.xs[lo + l] : 0;
        sf[l] = l < len ? a.flags[lo + l] : 0;
    }
    __syncthreads();
    // each thread: an inclusive scan of its 8 consecutive elements
    Pair run{false, 0};
    Pair el[kSgPer];
#pragma unroll
    for (int k = 0; k < kSgPer; ++k) {
        const int l = tid * kSgPer + k;
        run = combine(run, Pair{sf[l] != 0, sv[l]});
        el[k] = run;
    }
    // exclusive scan of the thread aggregates across the wave
    Pair inc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        Pair o;
        o.f = __shfl_up(static_cast<int>(inc.f), off, kWave) != 0;
        o.v = __shfl_up(inc.v, off, kWave);
        if (lane >= off) inc = combine(o, inc);
    }
    Pair before_lane;
    before_lane.f = __shfl_up(static_cast<int>(inc.f), 1, kWave) != 0;
    before_lane.v = __shfl_up(inc.v, 1, kWave);
    if (lane == 0) before_lane = Pair{false, 0};
    if (lane == kWave - 1) {
        wv[wave] = inc.v;
        wf[wave] = inc.f ? 1 : 0;
    }
    __syncthreads();
    // waves before this one, and the tile's aggregate
    Pair before_wave{false, 0}, tile{false, 0};
#pragma unroll
    for (int w = 0; w < kSgThreads / kWave; ++w) {
        const Pair x{wf[w] != 0, wv[w]};
        if (w < wave) before_wave = combine(before_wave, x);
        tile = combine(tile, x);
    }
    // the tile's prefix from its predecessors
    if (wave == 0) {
        int64_t excl = 0;
        if (tile.f) {
            if (lane == 0) publish(a, t, kSgP, tile.v);
        } else {
            if (lane == 0 && t > 0) publish(a, t, kSgA, tile.v);
        }
        if (t > 0) excl = sg_lookback(a, t, lane);
        if (lane == 0) {
            if (!tile.f) publish(a, t, kSgP, excl + tile.v);
            sh[1] = excl;
        }
    }
    __syncthreads();
    const Pair prefix = combine(Pair{false, sh[1]}, combine(before_wave, before_lane));
#pragma unroll
    for (int k = 0; k < kSgPer; ++k) sv[tid * kSgPer + k] = combine(prefix, el[k]).v;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSgPer; ++k) {
        const int l = k * kSgThreads + tid;
        if (l < len) stream_store(a.out + lo + l, sv[l]);
    }
}

}  // namespace
}  // namespace ixp

using namespace ixp;

extern "C" size_t ixp_sgm_sum_workspace(int64_t n) {
    if (n < 0) return 0;
    const int64_t nt = ceil_div(n, kSgTile);
    return kSgHeader + round_up(static_cast<size_t>(nt) * 4, 256) + 2 * round_up(static_cast<size_t>(nt) * 8, 256);
}

extern "C" int ixp_sgm_sum(const uint8_t *d_flags, const int64_t *d_xs, int64_t n, int64_t *d_out, void *ws,
                           size_t ws_bytes, void *stream) {
    if (n < 0 || (n > 0 && (!d_flags || !d_xs || !d_out))) return IXP_EINVAL;
    if (!aligned(d_xs, 8) || !aligned(d_out, 8) || !aligned(ws, 8)) return IXP_EINVAL;
    if (!ws || ws_bytes < ixp_sgm_sum_workspace(n)) return IXP_EWORKSPACE;
    if (n == 0) return IXP_OK;
    char *w = static_cast<char *>(ws);
    SgArgs a;
    a.flags = d_flags;
    a.xs = d_xs;
    a.out = d_out;
    a.n = n;
    a.num_tiles = ceil_div(n, kSgTile);
    a.ticket = reinterpret_cast<uint32_t *>(w);
    a.err = reinterpret_cast<int32_t *>(w + 4);
    a.status = reinterpret_cast<uint32_t *>(w + kSgHeader);
    a.agg = reinterpret_cast<int64_t *>(w + kSgHeader + round_up(static_cast<size_t>(a.num_tiles) * 4, 256));
    a.incl = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(a.agg) +
                                         round_up(static_cast<size_t>(a.num_tiles) * 8, 256));
    hipStream_t st = as_stream(stream);
    const int64_t ib = ceil_div(a.num_tiles, 256) < 1024 ? ceil_div(a.num_tiles, 256) : 1024;
    IXP_LAUNCH("sgm_init", sg_init_kernel, dim3(static_cast<uint32_t>(ib)), dim3(256), 0, st, a);
    IXP_LAUNCH("sgm_scan", sg_scan_kernel, dim3(static_cast<uint32_t>(a.num_tiles)), dim3(kSgThreads), 0, st, a);
    return launch_status();
}
