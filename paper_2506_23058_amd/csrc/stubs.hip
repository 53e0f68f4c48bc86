// Entry points not implemented yet.
#include "host.hpp"
extern "C" {
int ixp_scatter_inj(void *, int64_t, const void *, int32_t, const void *, int64_t, int64_t, void *) { return IXP_EUNSUPPORTED; }
int ixp_gather(void *, const void *, int64_t, const void *, int32_t, int64_t, int64_t, int32_t *, void *) { return IXP_EUNSUPPORTED; }
size_t ixp_check_props_workspace(int64_t, uint32_t, const ixp_prop_args *) { return 0; }
int ixp_check_props(const void *, int32_t, int64_t, uint32_t, const ixp_prop_args *, ixp_verdict *, void *, size_t, void *) { return IXP_EUNSUPPORTED; }
}
