"""MI355X (gfx950) filter-partition library: stable partition / filter, flat
and segmented, property checkers and a differentiable partition, as HIP
kernels behind the C ABI of include/ixpart.h."""
from ._lib import (MODE_FILTER, MODE_PARTITION, PRED_FLAGS, PRED_LT, PRED_MOD_EQ,  # noqa: F401
                   RANGE, MONO, INJ, BIJ, FILTPART, CLASS_MOD, CLASS_THRESH, CLASS_BYTES, MONO_LE, MONO_LT, MONO_GE, MONO_GT,
                   IxpError, lib)
from .ops import (Classes, FiltPartArgs, partition_v, autotuned_tiling, PartitionScatter, Pred, SegmentedGraph, check_props,  # noqa: F401
                  gather, get_smallest_pairs, hist_min, match_min, mk_ii, mk_sgm_descr, sgm_sum, shape_tools_error, partition, partition_scatter, profile_enable, profile_read,
                  read_error, scatter_checked, SmallestPairs, scatter_inj, segmented_error, segmented_partition,
                  tune_segmented, verdicts, workspace, zero_)
