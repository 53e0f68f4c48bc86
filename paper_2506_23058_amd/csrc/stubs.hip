// Entry points not implemented yet.
#include "host.hpp"
extern "C" {
int ixp_scatter_inj(void *, int64_t, const void *, int32_t, const void *, int64_t, int64_t, void *) { return IXP_EUNSUPPORTED; }
int ixp_gather(void *, const void *, int64_t, const void *, int32_t, int64_t, int64_t, int32_t *, void *) { return IXP_EUNSUPPORTED; }
}
