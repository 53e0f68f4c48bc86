// host.hpp -- host-side helpers shared by the C-ABI entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ixpart.h"

namespace ixp {

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void *p, uintptr_t a) {
    return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline size_t round_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

// Launch status of the kernel just enqueued.
inline int launch_status() {
    return hipGetLastError() == hipSuccess ? IXP_OK : IXP_EHIP;
}

// Validated, device-ready form of ixp_pred.
struct HostPred {
    int kind;
    uint64_t M;     // MOD_EQ: ceil(2^64 / d) mod 2^64
    uint32_t d;
    int64_t r;
    float s;
    const uint8_t *flags;
    const float *row_s;
};

// `n` elements are tested: a flag or row array may be NULL only when n == 0.
// Row predicates are accepted here; calls without rows reject them.
inline int check_pred(const ixp_pred *p, int32_t key_t, HostPred *out, int64_t n) {
    if (!p) return IXP_EINVAL;
    out->kind = p->kind;
    out->flags = p->flags;
    out->s = p->s;
    out->r = p->r;
    out->d = 1;
    out->M = 0;
    out->row_s = p->row_s;
    switch (p->kind) {
    case IXP_PRED_MOD_ROW:
    case IXP_PRED_MOD_EQ:
        if (key_t != IXP_I32) return key_t == IXP_I64 ? IXP_EUNSUPPORTED : IXP_EINVAL;
        if (p->d < 1 || p->d > 0xFFFFFFFFll) return IXP_EINVAL;
        out->d = static_cast<uint32_t>(p->d);
        out->M = ~0ull / out->d + 1;
        return IXP_OK;
    case IXP_PRED_LT:
        return key_t == IXP_F32 ? IXP_OK : IXP_EINVAL;
    case IXP_PRED_LT_ROW:
        if (key_t != IXP_F32) return IXP_EINVAL;
        return (p->row_s || n == 0) ? IXP_OK : IXP_EINVAL;
    case IXP_PRED_FLAGS:
        if (key_t != IXP_I32 && key_t != IXP_F32) return IXP_EINVAL;
        return (p->flags || n == 0) ? IXP_OK : IXP_EINVAL;
    default:
        return IXP_EINVAL;
    }
}

inline bool is_row_pred(int kind) { return kind == IXP_PRED_LT_ROW || kind == IXP_PRED_MOD_ROW; }

// Number of compute units of the current device, cached per device.
int device_cus();

// Dynamic LDS bytes to request at launch so that at most `wgs` workgroups of a
// kernel with `static_lds` bytes of static LDS fit on one CU (an occupancy
// cap), from the current device's LDS per CU; 0 when it cannot be applied.
size_t lds_for_wgs_per_cu(int wgs, size_t static_lds);

// Kernel timing: while profiling is enabled, a ProfScope records a HIP event
// on `st` at construction and another at destruction, around one launch.
bool profiling();
struct ProfScope {
    ProfScope(const char *name, hipStream_t st);
    ~ProfScope();
    const char *name_;
    hipStream_t st_;
    void *ev0_ = nullptr;
};

}  // namespace ixp

// Enqueues a kernel, timed when profiling is on.
#define IXP_LAUNCH(name, kernel, grid, block, shmem, stream, ...)              \
    do {                                                                      \
        ::ixp::ProfScope ixp_prof_scope_(name, stream);                       \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);  \
    } while (0)
