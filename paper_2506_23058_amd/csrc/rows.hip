// rows.hip -- scatter of rows by an injective index array (Section 2.1:
// scatter dst is vs, restricted to index arrays with Inj, so no two rows race
// and no atomics are needed) and its inverse, a gather of rows.  Together they
// are the forward and backward of the differentiable partition: a bijective
// index array (Bij, Section 2.3) makes the scatter invertible by the gather.
//
// Rows are moved as raw bytes in 16-byte units when the row size and the
// buffers allow it (else 4-byte units); consecutive lanes move consecutive
// units of a row, so each row is read and written as one contiguous run.
// The gather of rows of 1..16 units takes one wave per 64 rows (index loads
// shared by shuffle, every unit load of a step in flight at once); other
// gathers and every scatter take one thread per unit.
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

// Gather of rows of UPR 16-byte units (UPR a power of two, at most 16), 64
// rows per wave and step: lane l loads the index of row r0 + l (one coalesced
// load for the wave), the row indices reach the lanes that move the rows'
// units by shuffle, and each lane then issues all of its UPR unit loads
// before any store, so no load waits on an index load.  Consecutive lanes
// move consecutive units, so each row is one contiguous run on both sides;
// the next step's indices are loaded while this step's units move.  (The
// same shape for the scatter measured slower than one thread per unit,
// whose index load does not delay its data load.)
template <int UPR, class Idx>
__global__ __launch_bounds__(256) void gather_rows_wave_kernel(v4u *dst, const v4u *src, int64_t n_src,
                                                               const Idx *idx, int64_t m, int32_t *err) {
    constexpr int kRowsPerPass = kWave / UPR;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (256 / kWave);
    int64_t r0 = (static_cast<int64_t>(blockIdx.x) * (256 / kWave) + wave_id()) * kWave;
    int64_t s = r0 + lane < m ? static_cast<int64_t>(idx[r0 + lane]) : 0;
    bool bad = false;
    for (; r0 < m; r0 += nw * kWave) {
        const int64_t rn = r0 + nw * kWave;
        const int64_t sn = rn + lane < m ? static_cast<int64_t>(idx[rn + lane]) : 0;
        v4u v[UPR];
#pragma unroll
        for (int j = 0; j < UPR; ++j) {
            const int64_t row = r0 + j * kRowsPerPass + lane / UPR;
            const int64_t t = __shfl(s, j * kRowsPerPass + lane / UPR, 64);
            const bool ok = 0 <= t && t < n_src;
            bad |= row < m && !ok;
            v[j] = row < m && ok ? __builtin_nontemporal_load(src + t * UPR + lane % UPR) : v4u{0, 0, 0, 0};
        }
#pragma unroll
        for (int j = 0; j < UPR; ++j) {
            const int64_t row = r0 + j * kRowsPerPass + lane / UPR;
            if (row < m) stream_store(dst + row * UPR + lane % UPR, v[j]);
        }
        s = sn;
    }
    if (err && ballot(bad) != 0 && lane == 0) atomicOr(err, 1);
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

bool wave_rows_ok(int64_t upr) { return upr == 1 || upr == 2 || upr == 4 || upr == 8 || upr == 16; }

// One wave per 64 rows and step; as many waves as 16 workgroups of 256 per CU.
int wave_grid(int64_t m) {
    const int64_t cap = static_cast<int64_t>(device_cus()) * 16;
    const int64_t want = ceil_div(m, 256);
    return static_cast<int>(want < cap ? (want > 0 ? want : 1) : cap);
}

template <int UPR>
int gather_wave_upr(void *dst, const void *src, int64_t n_src, const void *idx, int32_t idx_t, int64_t m,
                    int32_t *err, hipStream_t st) {
    const int grid = wave_grid(m);
    if (idx_t == IXP_I32)
        IXP_LAUNCH("gather_rows", (gather_rows_wave_kernel<UPR, int32_t>), dim3(grid), dim3(256), 0, st,
                   static_cast<v4u *>(dst), static_cast<const v4u *>(src), n_src,
                   static_cast<const int32_t *>(idx), m, err);
    else
        IXP_LAUNCH("gather_rows", (gather_rows_wave_kernel<UPR, int64_t>), dim3(grid), dim3(256), 0, st,
                   static_cast<v4u *>(dst), static_cast<const v4u *>(src), n_src,
                   static_cast<const int64_t *>(idx), m, err);
    return launch_status();
}

int launch_gather_wave(void *dst, const void *src, int64_t n_src, const void *idx, int32_t idx_t, int64_t m,
                       int64_t upr, int32_t *err, hipStream_t st) {
    switch (upr) {
    case 1: return gather_wave_upr<1>(dst, src, n_src, idx, idx_t, m, err, st);
    case 2: return gather_wave_upr<2>(dst, src, n_src, idx, idx_t, m, err, st);
    case 4: return gather_wave_upr<4>(dst, src, n_src, idx, idx_t, m, err, st);
    case 8: return gather_wave_upr<8>(dst, src, n_src, idx, idx_t, m, err, st);
    default: return gather_wave_upr<16>(dst, src, n_src, idx, idx_t, m, err, st);
    }
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
    if (v16 && wave_rows_ok(upr)) return launch_gather_wave(dst, src, n_src, idx, idx_t, m, upr, d_err, st);
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
