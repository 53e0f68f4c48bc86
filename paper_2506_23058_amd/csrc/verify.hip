// verify.hip -- reduce-by-index with min and the dynamically verified scatter
// of the evaluation (Section 6, table "tab:eval", right: the Base variant of
// partition2 checks at run time that its scatter writes no location twice,
// with a reduce-by-index of atomic minima; Static drops the check and +Opt
// also drops the zero initialisation of the scattered array).  The same
// reduce-by-index (`hist` with min) computes H in get_smallest_pairs.
//
// These kernels are the comparison point for the statically verified path:
// random-access atomics on a table as large as the output, one extra pass
// over the indices and the values, and an output that must be zeroed first.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int kVBlock = 256;

int vgrid(int64_t work) {
    const int64_t cap = static_cast<int64_t>(device_cus()) * 32;
    const int64_t need = ceil_div(work > 0 ? work : 1, kVBlock);
    return static_cast<int>(need < cap ? need : cap);
}

// Zeroes `bytes` bytes at p: 16-byte stores over the aligned body, byte
// stores for the unaligned head and the tail.
__device__ __forceinline__ void zero_bytes(uint8_t *p, int64_t bytes, int64_t gtid, int64_t gstride) {
    const int64_t head = static_cast<int64_t>((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15);
    const int64_t h = head < bytes ? head : bytes;
    const int64_t body = (bytes - h) / 16;
    v4u *q = reinterpret_cast<v4u *>(p + h);
    const v4u z = {0u, 0u, 0u, 0u};
    for (int64_t u = gtid; u < body; u += gstride) stream_store(q + u, z);
    const int64_t tail0 = h + body * 16;
    if (gtid < h) p[gtid] = 0;
    if (gtid < bytes - tail0) p[tail0 + gtid] = 0;
}

__global__ __launch_bounds__(kVBlock) void zero_kernel(uint8_t *p, int64_t bytes) {
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    zero_bytes(p, bytes, static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x, gstride);
}

__global__ __launch_bounds__(kVBlock) void fill_i64_kernel(int64_t *p, int64_t n, int64_t v) {
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x; i < n; i += gstride) p[i] = v;
}

// dst[idx[i]] = min(dst[idx[i]], vals[i]) for in-bounds idx[i] (vals NULL: i).
template <class Idx>
__global__ __launch_bounds__(kVBlock) void hist_min_kernel(int64_t *dst, int64_t n_dst, const Idx *idx,
                                                           const int64_t *vals, int64_t m) {
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x; i < m; i += gstride) {
        const int64_t d = static_cast<int64_t>(idx[i]);
        if (0 <= d && d < n_dst) {
            const int64_t v = vals ? vals[i] : i;
            atomicMin(reinterpret_cast<long long *>(dst + d), static_cast<long long>(v));
        }
    }
}

// flags[k] = (0 <= idx[k] < n_hist) && hist[idx[k]] == vals[k]: the keep
// flags of get_smallest_pairs (an entry whose value is the minimum recorded
// at its endpoint).  Four entries per thread, their flags leave as one
// 32-bit store.
template <class Idx>
__global__ __launch_bounds__(kVBlock) void match_min_kernel(uint8_t *flags, const int64_t *hist, int64_t n_hist,
                                                            const Idx *idx, const int64_t *vals, int64_t m) {
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    const int64_t groups = (m + 3) / 4;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x; g < groups; g += gstride) {
        uint32_t w = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = 4 * g + q;
            if (k < m) {
                const int64_t d = static_cast<int64_t>(idx[k]);
                const bool keep = 0 <= d && d < n_hist && hist[d] == vals[k];
                w |= static_cast<uint32_t>(keep) << (8 * q);
            }
        }
        if (4 * g + 4 <= m) stream_store(reinterpret_cast<uint32_t *>(flags + 4 * g), w);
        else
            for (int q = 0; 4 * g + q < m; ++q) flags[4 * g + q] = static_cast<uint8_t>(w >> (8 * q));
    }
}

struct CheckState {
    unsigned long long first;   // least unsafe write, or ~0
};

// Step 1 of the checked scatter: zero the destination, set every location's
// least writer to m, clear the state.
__global__ __launch_bounds__(kVBlock) void checked_init_kernel(uint8_t *dst, int64_t dst_bytes, int64_t *win,
                                                               int64_t n_dst, int64_t m, CheckState *st) {
    const int64_t gtid = static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x;
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    zero_bytes(dst, dst_bytes, gtid, gstride);
    for (int64_t v = gtid; v < n_dst; v += gstride) win[v] = m;
    if (gtid == 0) st->first = ~0ull;
}

// Step 3: a write is safe when it is the least writer of its location; safe
// writes store their value, the least unsafe index is kept (one atomic per
// wave that saw one).
template <class Idx, class Elem>
__global__ __launch_bounds__(kVBlock) void checked_scatter_kernel(Elem *dst, int64_t n_dst, const Idx *idx,
                                                                  const Elem *vals, int64_t m,
                                                                  const int64_t *win, CheckState *st) {
    const int64_t gstride = static_cast<int64_t>(gridDim.x) * kVBlock;
    unsigned long long bad = ~0ull;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kVBlock + threadIdx.x; i < m; i += gstride) {
        const int64_t d = static_cast<int64_t>(idx[i]);
        if (0 <= d && d < n_dst) {
            if (win[d] == i) dst[d] = vals[i];
            else if (static_cast<unsigned long long>(i) < bad) bad = static_cast<unsigned long long>(i);
        }
    }
    if (ballot(bad != ~0ull)) {
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(bad, off, kWave);
            if (o < bad) bad = o;
        }
        if ((threadIdx.x & (kWave - 1)) == 0) atomicMin(&st->first, bad);
    }
}

template <class Idx>
__global__ void checked_finalize_kernel(const CheckState *st, const Idx *idx, ixp_verdict *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long f = st->first;
    ixp_verdict v;
    v.reserved = 0;
    if (f == ~0ull) {
        v.holds = 1;
        v.first_violation = -1;
        v.aux = 0;
    } else {
        v.holds = 0;
        v.first_violation = static_cast<int64_t>(f);
        v.aux = static_cast<int64_t>(idx[f]);
    }
    *out = v;
}

template <class Idx, class Elem>
int launch_checked(void *dst, int64_t n_dst, const void *idx, const void *vals, int64_t m,
                   ixp_verdict *d_out, int64_t *win, CheckState *st, hipStream_t s) {
    const int64_t eb = static_cast<int64_t>(sizeof(Elem));
    IXP_LAUNCH("checked_init", checked_init_kernel, dim3(vgrid(n_dst * eb / 16 + n_dst)), dim3(kVBlock), 0, s,
               static_cast<uint8_t *>(dst), n_dst * eb, win, n_dst, m, st);
    IXP_LAUNCH("checked_hist_min", hist_min_kernel<Idx>, dim3(vgrid(m)), dim3(kVBlock), 0, s, win, n_dst,
               static_cast<const Idx *>(idx), static_cast<const int64_t *>(nullptr), m);
    IXP_LAUNCH("checked_scatter", (checked_scatter_kernel<Idx, Elem>), dim3(vgrid(m)), dim3(kVBlock), 0, s,
               static_cast<Elem *>(dst), n_dst, static_cast<const Idx *>(idx), static_cast<const Elem *>(vals),
               m, static_cast<const int64_t *>(win), st);
    IXP_LAUNCH("checked_finalize", checked_finalize_kernel<Idx>, dim3(1), dim3(64), 0, s,
               static_cast<const CheckState *>(st), static_cast<const Idx *>(idx), d_out);
    return launch_status();
}

constexpr size_t kCheckedHeader = 256;

}  // namespace
}  // namespace ixp

using namespace ixp;

extern "C" int ixp_zero(void *d, size_t bytes, void *stream) {
    if (bytes > 0 && !d) return IXP_EINVAL;
    if (bytes == 0) return IXP_OK;
    const int64_t b = static_cast<int64_t>(bytes);
    IXP_LAUNCH("zero", zero_kernel, dim3(vgrid(b / 16 + 1)), dim3(kVBlock), 0, as_stream(stream),
               static_cast<uint8_t *>(d), b);
    return launch_status();
}

extern "C" int ixp_hist_min(int64_t *d_dst, int64_t n_dst, int64_t neutral, const void *idx, int32_t idx_t,
                            const int64_t *vals, int64_t m, void *stream) {
    if (n_dst < 0 || m < 0 || (n_dst > 0 && !d_dst) || (m > 0 && !idx)) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (!aligned(d_dst, 8) || !aligned(vals, 8) || !aligned(idx, idx_t == IXP_I32 ? 4 : 8)) return IXP_EINVAL;
    hipStream_t s = as_stream(stream);
    if (n_dst > 0)
        IXP_LAUNCH("hist_min_fill", fill_i64_kernel, dim3(vgrid(n_dst)), dim3(kVBlock), 0, s, d_dst, n_dst,
                   neutral);
    if (m > 0 && n_dst > 0) {
        if (idx_t == IXP_I32)
            IXP_LAUNCH("hist_min", hist_min_kernel<int32_t>, dim3(vgrid(m)), dim3(kVBlock), 0, s, d_dst, n_dst,
                       static_cast<const int32_t *>(idx), vals, m);
        else
            IXP_LAUNCH("hist_min", hist_min_kernel<int64_t>, dim3(vgrid(m)), dim3(kVBlock), 0, s, d_dst, n_dst,
                       static_cast<const int64_t *>(idx), vals, m);
    }
    return launch_status();
}

extern "C" int ixp_match_min(uint8_t *d_flags, const int64_t *d_hist, int64_t n_hist, const void *idx,
                             int32_t idx_t, const int64_t *vals, int64_t m, void *stream) {
    if (n_hist < 0 || m < 0 || (m > 0 && (!d_flags || !idx || !vals)) || (n_hist > 0 && !d_hist))
        return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (!aligned(d_flags, 4) || !aligned(d_hist, 8) || !aligned(vals, 8) ||
        !aligned(idx, idx_t == IXP_I32 ? 4 : 8))
        return IXP_EINVAL;
    if (m == 0) return IXP_OK;
    hipStream_t s = as_stream(stream);
    const int grid = vgrid((m + 3) / 4);
    if (idx_t == IXP_I32)
        IXP_LAUNCH("match_min", match_min_kernel<int32_t>, dim3(grid), dim3(kVBlock), 0, s, d_flags, d_hist, n_hist,
                   static_cast<const int32_t *>(idx), vals, m);
    else
        IXP_LAUNCH("match_min", match_min_kernel<int64_t>, dim3(grid), dim3(kVBlock), 0, s, d_flags, d_hist, n_hist,
                   static_cast<const int64_t *>(idx), vals, m);
    return launch_status();
}

extern "C" size_t ixp_scatter_checked_workspace(int64_t n_dst) {
    if (n_dst < 0) return 0;
    return kCheckedHeader + static_cast<size_t>(n_dst > 0 ? n_dst : 1) * sizeof(int64_t);
}

extern "C" int ixp_scatter_checked(void *dst, int64_t n_dst, const void *idx, int32_t idx_t, const void *vals,
                                   int64_t m, int64_t elem_bytes, ixp_verdict *d_out, void *ws,
                                   size_t ws_bytes, void *stream) {
    if (n_dst < 0 || m < 0 || !d_out) return IXP_EINVAL;
    if (elem_bytes != 4 && elem_bytes != 8) return IXP_EUNSUPPORTED;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if ((n_dst > 0 && !dst) || (m > 0 && (!idx || !vals))) return IXP_EINVAL;
    if (!aligned(dst, elem_bytes) || !aligned(vals, elem_bytes) || !aligned(idx, idx_t == IXP_I32 ? 4 : 8) ||
        !aligned(d_out, 8))
        return IXP_EINVAL;
    if (!ws || ws_bytes < ixp_scatter_checked_workspace(n_dst) || !aligned(ws, 256)) return IXP_EWORKSPACE;
    CheckState *st = static_cast<CheckState *>(ws);
    int64_t *win = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + kCheckedHeader);
    hipStream_t s = as_stream(stream);
    if (idx_t == IXP_I32)
        return elem_bytes == 4 ? launch_checked<int32_t, uint32_t>(dst, n_dst, idx, vals, m, d_out, win, st, s)
                               : launch_checked<int32_t, uint64_t>(dst, n_dst, idx, vals, m, d_out, win, st, s);
    return elem_bytes == 4 ? launch_checked<int64_t, uint32_t>(dst, n_dst, idx, vals, m, d_out, win, st, s)
                           : launch_checked<int64_t, uint64_t>(dst, n_dst, idx, vals, m, d_out, win, st, s);
}
