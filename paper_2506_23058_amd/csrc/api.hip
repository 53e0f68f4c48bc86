// api.hip -- status strings, device queries and error read-back.
#include <mutex>

#include "host.hpp"

namespace ixp {

int device_cus() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return IXP_EHIP;
    if (dev < 64) {
        std::lock_guard<std::mutex> lock(mu);
        if (cached[dev] > 0) return cached[dev];
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return IXP_EHIP;
    if (dev < 64) {
        std::lock_guard<std::mutex> lock(mu);
        cached[dev] = cus;
    }
    return cus;
}

}  // namespace ixp

extern "C" const char *ixp_status_str(int status) {
    switch (status) {
    case IXP_OK: return "ok";
    case IXP_EINVAL: return "invalid argument";
    case IXP_ENOMEM: return "out of host memory";
    case IXP_EHIP: return "HIP runtime error";
    case IXP_EUNSUPPORTED: return "unsupported";
    case IXP_EWORKSPACE: return "workspace missing or too small";
    case IXP_EDEVICE: return "device-side error";
    default: return "unknown status";
    }
}

extern "C" int ixp_device_cus(void) { return ixp::device_cus(); }

// Every workspace starts with the same 256-byte header: a u32 ticket at
// offset 0 and the i32 error word at offset 4.
extern "C" int ixp_read_error(const void *ws, void *stream) {
    if (!ws) return IXP_EWORKSPACE;
    if (hipStreamSynchronize(ixp::as_stream(stream)) != hipSuccess) return IXP_EHIP;
    int32_t err = 0;
    const char *p = static_cast<const char *>(ws) + 4;
    if (hipMemcpy(&err, p, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return IXP_EHIP;
    if (err == 0) return IXP_OK;
    const int32_t zero = 0;
    if (hipMemcpy(const_cast<char *>(p), &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        return IXP_EHIP;
    return (err & 2) ? IXP_EINVAL : IXP_EDEVICE;
}
