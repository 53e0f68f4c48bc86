// Entry points not implemented yet.
#include "host.hpp"
extern "C" {
size_t ixp_segmented_workspace(int64_t, int64_t, const ixp_tuning *) { return 0; }
int ixp_segmented_partition(const void *, int32_t, int64_t, const int64_t *, int64_t, const ixp_pred *, int32_t, void *, void *, int32_t, int64_t *, uint8_t *, const ixp_tuning *, void *, size_t, void *) { return IXP_EUNSUPPORTED; }
int ixp_tune_segmented(const void *, int32_t, int64_t, const int64_t *, int64_t, const ixp_pred *, int32_t, void *, void *, int32_t, int64_t *, uint8_t *, void *, size_t, int32_t, ixp_tuning *, float *, void *) { return IXP_EUNSUPPORTED; }
int ixp_segmented_graph_create(ixp_graph *, const void *, int32_t, int64_t, const int64_t *, int64_t, const ixp_pred *, int32_t, void *, void *, int32_t, int64_t *, uint8_t *, const ixp_tuning *, void *, size_t) { return IXP_EUNSUPPORTED; }
int ixp_graph_launch(ixp_graph, void *) { return IXP_EUNSUPPORTED; }
int ixp_graph_destroy(ixp_graph) { return IXP_EUNSUPPORTED; }
int ixp_scatter_inj(void *, int64_t, const void *, int32_t, const void *, int64_t, int64_t, void *) { return IXP_EUNSUPPORTED; }
int ixp_gather(void *, const void *, int64_t, const void *, int32_t, int64_t, int64_t, int32_t *, void *) { return IXP_EUNSUPPORTED; }
size_t ixp_check_props_workspace(int64_t, uint32_t, const ixp_prop_args *) { return 0; }
int ixp_check_props(const void *, int32_t, int64_t, uint32_t, const ixp_prop_args *, ixp_verdict *, void *, size_t, void *) { return IXP_EUNSUPPORTED; }
}
