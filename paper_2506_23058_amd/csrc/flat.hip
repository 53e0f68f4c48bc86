// flat.hip -- flat stable partition (partition2) and filter on gfx950.
//
// partition2 (Section 2.1, figure "Running Examples") computes
//   cs = map p xs; indicesT = scan (+) 0 flagsT; num_true = last of indicesT;
//   indicesF = num_true + scan (+) 0 flagsF; indices = c ? t-1 : f-1;
//   ys = scatter zeros indices xs.
// Here the two scans collapse into one exclusive count of trues E(i), since
// #falses before i = i - E(i); the index map becomes
//   idx[i] = c_i ? E(i) : T + i - E(i)            (T = num_true)
// which is the closed form of `indices` the paper derives (Section 2.3).
//
// Kernels, all on the caller's stream:
//   init   -- zeroes the tile ticket, error word and split (and, for filter,
//             the tile descriptors);
//   count  -- (partition only) one wave per tile counts its trues, publishes
//             the count as the tile's aggregate and adds it to T.  The stable
//             order of the falses needs T before any false is placed;
//   scan   -- one workgroup per tile, tiles taken in ticket order: flags by
//             ballot, in-tile ranks by mbcnt, tile prefix by decoupled
//             look-back, indices written in input order (vector stores),
//             keys staged in LDS in output order and written as the tile's
//             two contiguous runs.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

constexpr int kFlatBlock = 256;
constexpr size_t kWsHeader = 256;   // ticket (u32), error word (i32), padding

template <int VEC>
struct FlatCfg {
    static constexpr int kBlock = kFlatBlock;
    static constexpr int kRows = VEC == 4 ? 4 : 16;
    using T = Tile<kBlock, kRows, VEC>;
    static constexpr int kTile = T::kSize;   // 4096 for both widths
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
    int32_t need_keys;
};

__global__ void flat_init_kernel(uint32_t *ticket, int32_t *err, int64_t *split,
                                 uint64_t *desc, int64_t num_desc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        *ticket = 0;
        *err = 0;
        *split = 0;
    }
    for (int64_t j = i; j < num_desc; j += static_cast<int64_t>(gridDim.x) * blockDim.x)
        desc[j] = 0;
}

// One wave counts one tile (same tile bounds as the scan kernel) and
// publishes the count as that tile's aggregate; each wave adds its running
// total to T once at the end.
template <int VEC, class Pred>
__global__ __launch_bounds__(kFlatBlock) void flat_count_kernel(FlatArgs a, Pred pred) {
    constexpr int kTile = FlatCfg<VEC>::kTile;
    constexpr int kSteps = kTile / (kWave * VEC);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    uint64_t mine = 0;
    for (int64_t t = wave0; t < a.num_tiles; t += nwaves) {
        const int64_t lo = t * kTile;
        const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int64_t p0 = lo + static_cast<int64_t>(k) * (kWave * VEC) + lane * VEC;
            uint32_t kv[VEC];
            uint8_t fv[VEC];
#pragma unroll
            for (int q = 0; q < VEC; ++q) { kv[q] = 0; fv[q] = 0; }
            if (VEC == 4 && p0 + VEC <= hi) {
                if (!Pred::kUsesFlags) {
                    const uint4 v = *reinterpret_cast<const uint4 *>(a.keys + p0);
                    kv[0] = v.x; kv[1 % VEC] = v.y; kv[2 % VEC] = v.z; kv[3 % VEC] = v.w;
                } else if constexpr (Pred::kUsesFlags) {
                    const uint32_t w = *reinterpret_cast<const uint32_t *>(pred.flags + p0);
#pragma unroll
                    for (int q = 0; q < VEC; ++q) fv[q] = static_cast<uint8_t>(w >> (8 * q));
                }
            } else {
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    if (p0 + q < hi) {
                        if constexpr (Pred::kUsesFlags) fv[q] = pred.flags[p0 + q];
                        else kv[q] = a.keys[p0 + q];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < VEC; ++q) {
                const bool f = p0 + q < hi && pred(kv[q], fv[q]);
                cnt += static_cast<uint32_t>(__builtin_popcountll(ballot(f)));
            }
        }
        if (lane == 0) desc_store(a.desc + t, kStA | cnt);
        mine += cnt;
    }
    if (lane == 0 && mine)
        atomicAdd(reinterpret_cast<unsigned long long *>(a.split),
                  static_cast<unsigned long long>(mine));
}

template <int VEC, class Pred, int MODE, class Idx>
__global__ __launch_bounds__(kFlatBlock) void flat_scan_kernel(FlatArgs a, Pred pred) {
    using T = typename FlatCfg<VEC>::T;
    constexpr int kTile = T::kSize;
    constexpr int kRows = FlatCfg<VEC>::kRows;
    __shared__ uint32_t stage[kTile];
    __shared__ uint32_t wtot[T::kWaves];
    __shared__ int64_t sh[2];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & (kWave - 1);
    if (tid == 0) sh[0] = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t t = sh[0];
    const int64_t lo = t * kTile;
    const int64_t hi = lo + kTile < a.n ? lo + kTile : a.n;

    T tile;
    tile.load(a.keys, a.n, lo, lo, hi, pred, a.need_keys != 0, wave, lane);
    tile.wave_ranks();
    const uint32_t tcount = tile.block_ranks(wtot, wave, lane);

    if (MODE == IXP_MODE_FILTER && tid == 0 && t > 0) desc_store(a.desc + t, kStA | tcount);
    if (wave == 0) {
        const int64_t excl = t == 0 ? 0 : lookback(a.desc, t, 0, a.err);
        if (lane == 0) {
            desc_store(a.desc + t, kStP | static_cast<uint64_t>(excl + tcount));
            sh[1] = excl;
            if (MODE == IXP_MODE_FILTER && t == a.num_tiles - 1) *a.split = excl + tcount;
        }
    }
    __syncthreads();
    const int64_t excl = sh[1];
    const int64_t total = MODE == IXP_MODE_PARTITION ? __hip_atomic_load(a.split, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    const int64_t false_base = total + (lo - excl);   // T + #falses before the tile

    Idx *out_idx = static_cast<Idx *>(a.out_idx);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t p0 = T::pos(lo, wave, r, lane, 0);
        Idx v[VEC];
        uint32_t vm = 0;
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const uint32_t rt = tile.rank[r][q];
            const uint32_t rf = static_cast<uint32_t>(p0 + q - lo) - rt;
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
        if (out_idx && vm) store_idx_group<VEC, Idx>(out_idx, p0, v, vm);
    }
    if (a.out_keys) {
        __syncthreads();
        const int64_t nvalid = hi - lo;
        const int64_t nout = MODE == IXP_MODE_PARTITION ? nvalid : static_cast<int64_t>(tcount);
        for (int64_t s = tid; s < nout; s += kFlatBlock) {
            const int64_t dst = s < tcount ? excl + s : false_base + (s - tcount);
            if (dst < a.n) a.out_keys[dst] = stage[s];
        }
    }
}

template <int VEC, class Pred>
int launch_flat(const FlatArgs &a, const Pred &pred, int mode, int idx_t, hipStream_t st) {
    const int64_t nt = a.num_tiles;
    if (mode == IXP_MODE_PARTITION) {
        const int64_t cap = static_cast<int64_t>(device_cus()) * 8;
        const int64_t waves_per_block = kFlatBlock / kWave;
        const int64_t blocks = ceil_div(nt, waves_per_block) < cap ? ceil_div(nt, waves_per_block) : cap;
        hipLaunchKernelGGL((flat_count_kernel<VEC, Pred>), dim3(static_cast<uint32_t>(blocks)),
                           dim3(kFlatBlock), 0, st, a, pred);
        if (launch_status() != IXP_OK) return IXP_EHIP;
        if (idx_t == IXP_I32)
            hipLaunchKernelGGL((flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int32_t>),
                               dim3(static_cast<uint32_t>(nt)), dim3(kFlatBlock), 0, st, a, pred);
        else
            hipLaunchKernelGGL((flat_scan_kernel<VEC, Pred, IXP_MODE_PARTITION, int64_t>),
                               dim3(static_cast<uint32_t>(nt)), dim3(kFlatBlock), 0, st, a, pred);
    } else {
        if (idx_t == IXP_I32)
            hipLaunchKernelGGL((flat_scan_kernel<VEC, Pred, IXP_MODE_FILTER, int32_t>),
                               dim3(static_cast<uint32_t>(nt)), dim3(kFlatBlock), 0, st, a, pred);
        else
            hipLaunchKernelGGL((flat_scan_kernel<VEC, Pred, IXP_MODE_FILTER, int64_t>),
                               dim3(static_cast<uint32_t>(nt)), dim3(kFlatBlock), 0, st, a, pred);
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

int64_t flat_tile_size() { return FlatCfg<4>::kTile; }

}  // namespace ixp

using namespace ixp;

extern "C" size_t ixp_partition_workspace(int64_t n) {
    if (n < 0) return 0;
    const int64_t nt = ceil_div(n, FlatCfg<4>::kTile);
    return kWsHeader + round_up(static_cast<size_t>(nt) * sizeof(uint64_t), 256);
}

extern "C" int ixp_partition(const void *keys, int32_t key_t, int64_t n, const ixp_pred *pred,
                             int32_t mode, void *out_keys, void *out_idx, int32_t idx_t,
                             int64_t *d_split, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || !d_split) return IXP_EINVAL;
    if (mode != IXP_MODE_PARTITION && mode != IXP_MODE_FILTER) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (idx_t == IXP_I32 && n > 0x7FFFFFFFll) return IXP_EINVAL;
    if (key_t != IXP_I32 && key_t != IXP_F32) return key_t == IXP_I64 ? IXP_EUNSUPPORTED : IXP_EINVAL;
    HostPred hp;
    int rc = check_pred(pred, key_t, &hp);
    if (rc != IXP_OK) return rc;
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
    a.desc = reinterpret_cast<uint64_t *>(w + kWsHeader);
    a.num_tiles = ceil_div(n, FlatCfg<4>::kTile);
    a.need_keys = need_keys ? 1 : 0;

    const int64_t ndesc = mode == IXP_MODE_FILTER ? a.num_tiles : 0;
    const int64_t iblocks = ndesc > 0 ? (ceil_div(ndesc, 256) < 1024 ? ceil_div(ndesc, 256) : 1024) : 1;
    hipLaunchKernelGGL(flat_init_kernel, dim3(static_cast<uint32_t>(iblocks)), dim3(256), 0, st,
                       a.ticket, a.err, a.split, a.desc, ndesc);
    if (launch_status() != IXP_OK) return IXP_EHIP;
    if (n == 0) return IXP_OK;

    const bool vec4 = aligned(keys, 16) && aligned(out_idx, 16) &&
                      (hp.kind != IXP_PRED_FLAGS || aligned(hp.flags, 4));
    return vec4 ? dispatch_pred<4>(a, hp, mode, idx_t, st) : dispatch_pred<1>(a, hp, mode, idx_t, st);
}
