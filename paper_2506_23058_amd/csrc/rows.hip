// rows.hip -- scatter of rows by an injective index array (Section 2.1:
// scatter dst is vs, restricted to index arrays with Inj, so no two rows race
// and no atomics are needed) and its inverse, a gather of rows.  Together they
// are the forward and backward of the differentiable partition: a bijective
// index array (Bij, Section 2.3) makes the scatter invertible by the gather.
//
// Rows are moved as raw bytes in 16-byte units when the row size and the
// buffers allow it (else 4-byte units); consecutive lanes move consecutive
// units of a row, so each row is read and written as one contiguous run.
#include "device.hpp"
#include "host.hpp"

namespace ixp {
namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <class Unit, class Idx>
__global__ __launch_bounds__(256) void scatter_rows_kernel(Unit *dst, int64_t n_dst, const Idx *idx,
                                                           const Unit *vals, int64_t m, int64_t upr,
                                                           int shift) {
    const int64_t total = m * upr;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < total; u += stride) {
        const int64_t row = shift >= 0 ? (u >> shift) : u / upr;   // units per row: 2^shift
        const int64_t c = u - row * upr;
        const int64_t d = static_cast<int64_t>(idx[row]);
        const Unit v = __builtin_nontemporal_load(vals + u);
        if (0 <= d && d < n_dst) stream_store(dst + d * upr + c, v);
    }
}

template <class Unit, class Idx>
__global__ __launch_bounds__(256) void gather_rows_kernel(Unit *dst, const Unit *src, int64_t n_src,
                                                          const Idx *idx, int64_t m, int64_t upr,
                                                          int shift, int32_t *err) {
    const int64_t total = m * upr;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    bool bad = false;
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < total; u += stride) {
        const int64_t row = shift >= 0 ? (u >> shift) : u / upr;   // units per row: 2^shift
        const int64_t c = u - row * upr;
        const int64_t s = static_cast<int64_t>(idx[row]);
        Unit v{};
        if (0 <= s && s < n_src) v = src[s * upr + c];
        else bad = true;
        stream_store(dst + u, v);
    }
    if (err && ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(err, 1);
}

// log2 of a power of two, else -1.
int pow2_shift(int64_t v) {
    int s = 0;
    while ((int64_t{1} << s) < v) ++s;
    return (int64_t{1} << s) == v ? s : -1;
}

int grid_for(int64_t units) {
    const int64_t cap = static_cast<int64_t>(device_cus()) * 16;
    const int64_t want = ceil_div(units, 256);
    return static_cast<int>(want < cap ? (want > 0 ? want : 1) : cap);
}

}  // namespace
}  // namespace ixp

using namespace ixp;

extern "C" int ixp_scatter_inj(void *dst, int64_t n_dst, const void *idx, int32_t idx_t,
                               const void *vals, int64_t m, int64_t row_bytes, void *stream) {
    if (n_dst < 0 || m < 0 || row_bytes <= 0 || row_bytes % 4) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (m > 0 && (!idx || !vals || !dst)) return IXP_EINVAL;
    if (m == 0) return IXP_OK;
    if (!aligned(dst, 4) || !aligned(vals, 4) || !aligned(idx, idx_t == IXP_I32 ? 4 : 8)) return IXP_EINVAL;
    hipStream_t st = as_stream(stream);
    const bool v16 = row_bytes % 16 == 0 && aligned(dst, 16) && aligned(vals, 16);
    const int64_t upr = v16 ? row_bytes / 16 : row_bytes / 4;
    const int grid = grid_for(m * upr);
    if (v16) {
        if (idx_t == IXP_I32)
            IXP_LAUNCH("scatter_rows", (scatter_rows_kernel<v4u, int32_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<v4u *>(dst), n_dst, static_cast<const int32_t *>(idx),
                       static_cast<const v4u *>(vals), m, upr, pow2_shift(upr));
        else
            IXP_LAUNCH("scatter_rows", (scatter_rows_kernel<v4u, int64_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<v4u *>(dst), n_dst, static_cast<const int64_t *>(idx),
                       static_cast<const v4u *>(vals), m, upr, pow2_shift(upr));
    } else {
        if (idx_t == IXP_I32)
            IXP_LAUNCH("scatter_rows", (scatter_rows_kernel<uint32_t, int32_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<uint32_t *>(dst), n_dst, static_cast<const int32_t *>(idx),
                       static_cast<const uint32_t *>(vals), m, upr, pow2_shift(upr));
        else
            IXP_LAUNCH("scatter_rows", (scatter_rows_kernel<uint32_t, int64_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<uint32_t *>(dst), n_dst, static_cast<const int64_t *>(idx),
                       static_cast<const uint32_t *>(vals), m, upr, pow2_shift(upr));
    }
    return launch_status();
}

extern "C" int ixp_gather(void *dst, const void *src, int64_t n_src, const void *idx, int32_t idx_t,
                          int64_t m, int64_t row_bytes, int32_t *d_err, void *stream) {
    if (n_src < 0 || m < 0 || row_bytes <= 0 || row_bytes % 4) return IXP_EINVAL;
    if (idx_t != IXP_I32 && idx_t != IXP_I64) return IXP_EINVAL;
    if (m > 0 && (!idx || !dst || (n_src > 0 && !src))) return IXP_EINVAL;
    if (m == 0) return IXP_OK;
    if (!aligned(dst, 4) || !aligned(src, 4) || !aligned(idx, idx_t == IXP_I32 ? 4 : 8) ||
        !aligned(d_err, 4))
        return IXP_EINVAL;
    hipStream_t st = as_stream(stream);
    const bool v16 = row_bytes % 16 == 0 && aligned(dst, 16) && aligned(src, 16);
    const int64_t upr = v16 ? row_bytes / 16 : row_bytes / 4;
    const int grid = grid_for(m * upr);
    if (v16) {
        if (idx_t == IXP_I32)
            IXP_LAUNCH("gather_rows", (gather_rows_kernel<v4u, int32_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<v4u *>(dst), static_cast<const v4u *>(src), n_src,
                       static_cast<const int32_t *>(idx), m, upr, pow2_shift(upr), d_err);
        else
            IXP_LAUNCH("gather_rows", (gather_rows_kernel<v4u, int64_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<v4u *>(dst), static_cast<const v4u *>(src), n_src,
                       static_cast<const int64_t *>(idx), m, upr, pow2_shift(upr), d_err);
    } else {
        if (idx_t == IXP_I32)
            IXP_LAUNCH("gather_rows", (gather_rows_kernel<uint32_t, int32_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<uint32_t *>(dst), static_cast<const uint32_t *>(src), n_src,
                       static_cast<const int32_t *>(idx), m, upr, pow2_shift(upr), d_err);
        else
            IXP_LAUNCH("gather_rows", (gather_rows_kernel<uint32_t, int64_t>), dim3(grid), dim3(256), 0, st,
                       static_cast<uint32_t *>(dst), static_cast<const uint32_t *>(src), n_src,
                       static_cast<const int64_t *>(idx), m, upr, pow2_shift(upr), d_err);
    }
    return launch_status();
}
