// api.hip -- status strings, device queries and error read-back.
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

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

namespace {
std::atomic<int> g_prof{0};
std::mutex g_prof_mu;
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return true;
    return cs != hipStreamCaptureStatusNone;
}
}  // namespace

bool profiling() { return g_prof.load(std::memory_order_relaxed) != 0; }

ProfScope::ProfScope(const char *name, hipStream_t st) : name_(name), st_(st) {
    if (!profiling() || capturing(st)) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, st) == hipSuccess) ev0_ = e;
}

ProfScope::~ProfScope() {
    if (!ev0_) return;
    hipEvent_t e = take_event();
    if (!e || hipEventRecord(e, st_) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_recs.push_back({name_, static_cast<hipEvent_t>(ev0_), e});
}

}  // namespace ixp

extern "C" int ixp_profile_enable(int on) {
    ixp::g_prof.store(on ? 1 : 0);
    return IXP_OK;
}

extern "C" int ixp_profile_read(ixp_kernel_stat *out, int max, int *count) {
    using namespace ixp;
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        recs.swap(g_recs);
    }
    std::map<std::string, std::pair<int64_t, double>> acc;
    std::vector<std::string> order;
    int rc = IXP_OK;
    for (const ProfRec &r : recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            rc = IXP_EHIP;
        auto it = acc.find(r.name);
        if (it == acc.end()) {
            order.push_back(r.name);
            it = acc.emplace(r.name, std::make_pair(int64_t{0}, 0.0)).first;
        }
        it->second.first += 1;
        it->second.second += ms;
    }
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        for (const ProfRec &r : recs) {
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
    }
    int k = 0;
    for (const std::string &nm : order) {
        if (out && k < max) {
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, nm.c_str(), sizeof(out[k].name) - 1);
            out[k].launches = acc[nm].first;
            out[k].total_ms = acc[nm].second;
        }
        ++k;
    }
    if (count) *count = k;
    return rc;
}

extern "C" const char *ixp_status_str(int status) {
    switch (status) {
    case IXP_OK: return "ok";
    case IXP_EINVAL: return "invalid argument";
    case IXP_ENOMEM: return "out of host memory";
    case IXP_EHIP: return "HIP runtime error";
    case IXP_EUNSUPPORTED: return "unsupported";
    case IXP_EWORKSPACE: return "workspace missing or too small";
    case IXP_EDEVICE: return "device-side error";
    case IXP_ETOOLARGE: return "size exceeds the fixed capacity of the static scratch";
    default: return "unknown status";
    }
}

namespace ixp {
size_t lds_for_wgs_per_cu(int wgs, size_t static_lds) {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (wgs < 1 || hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    int lds = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (dev < 64) lds = cached[dev];
    }
    if (lds <= 0) {
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            lds <= 0)
            return 0;
        std::lock_guard<std::mutex> lock(mu);
        if (dev < 64) cached[dev] = lds;
    }
    // per-workgroup total in (lds / (wgs + 1), lds / wgs], on a 2 KiB boundary
    const size_t per_wg = (static_cast<size_t>(lds) / static_cast<size_t>(wgs)) & ~static_cast<size_t>(2047);
    if (per_wg * static_cast<size_t>(wgs + 1) <= static_cast<size_t>(lds) || per_wg <= static_lds) return 0;
    return per_wg - static_lds;
}
}  // namespace ixp

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
