"""The C ABI library loads and exports every entry point include/ixpart.h
declares; host-side argument checks and workspace queries (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ixpart.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ixp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ixp_partition", "ixp_segmented_partition", "ixp_scatter_inj",
                     "ixp_gather", "ixp_check_props"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2506_23058_amd._lib as L
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the Python binding covers every one of them
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_host_side_validation_without_gpu():
    import paper_2506_23058_amd._lib as L
    lib = L.lib()
    assert lib.ixp_status_str(L.IXP_EINVAL) == b"invalid argument"
    assert lib.ixp_partition_workspace(-1) == 0
    assert lib.ixp_partition_workspace(1 << 28) > 8 * ((1 << 28) // 4096)
    p = L.ixp_pred()
    p.kind = L.PRED_MOD_EQ
    p.d = 0          # invalid divisor: rejected on the host, nothing enqueued
    split = ctypes.c_int64(0)
    rc = lib.ixp_partition(None, L.I32, 10, ctypes.byref(p), 0, None, None, L.I64,
                           ctypes.addressof(split), None, 0, None)
    assert rc == L.IXP_EINVAL
    rc = lib.ixp_partition(None, L.I32, -5, ctypes.byref(p), 0, None, None, L.I64,
                           ctypes.addressof(split), None, 0, None)
    assert rc == L.IXP_EINVAL
    p.d = 2
    rc = lib.ixp_partition(None, L.I64, 10, ctypes.byref(p), 0, None, None, L.I64,
                           ctypes.addressof(split), None, 0, None)
    assert rc == L.IXP_EUNSUPPORTED
    assert lib.ixp_segmented_workspace(1000, 10, None) > 0
    t = L.ixp_tuning()
    t.block, t.rows = 300, 4
    assert lib.ixp_segmented_workspace(1000, 10, ctypes.byref(t)) == 0
    t.block, t.rows = 256, 4
    for sync, ok in ((L.ROW_SYNC_AUTO, True), (L.ROW_SYNC_COUNT, True), (L.ROW_SYNC_NOWAIT, True),
                     (L.ROW_SYNC_WAIT, True), (4, False), (-1, False)):
        t.row_sync = sync
        assert (lib.ixp_segmented_workspace(1000, 10, ctypes.byref(t)) > 0) == ok
    a = L.ixp_prop_args()
    a.lo, a.hi = 0, 1 << 28
    assert lib.ixp_check_props_workspace(1 << 28, 4, ctypes.byref(a)) >= (1 << 28) // 8
    # the allocation-free partition: its capacity, checked before anything else
    assert lib.ixp_partition_workspace(L.NOALLOC_MAX_N) <= L.NOALLOC_SCRATCH_BYTES
    assert lib.ixp_partition_workspace(L.NOALLOC_MAX_N + 1) > L.NOALLOC_SCRATCH_BYTES
    rc = lib.ixp_partition_noalloc(None, L.F32, L.NOALLOC_MAX_N + 1, ctypes.byref(p), 0, None,
                                   None, L.I64, ctypes.addressof(split), None)
    assert rc == L.IXP_ETOOLARGE
    assert lib.ixp_partition_noalloc(None, L.F32, -1, ctypes.byref(p), 0, None, None, L.I64,
                                     ctypes.addressof(split), None) == L.IXP_EINVAL
    assert lib.ixp_scatter_inj(None, 10, None, L.I64, None, 5, 6, None) == L.IXP_EINVAL
    assert lib.ixp_gather(None, None, 10, None, L.I32, 5, 16, None, None) == L.IXP_EINVAL


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    import importlib
    import paper_2506_23058_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()
    importlib.reload(L)


def test_new_entry_points_validate_on_the_host():
    """Argument errors of the entry points added for the evaluation's
    comparison and the next-stage programs are caught before any launch."""
    import paper_2506_23058_amd._lib as L
    lib = L.lib()
    # reduce-by-index, checked scatter, zero fill, keep flags
    assert lib.ixp_hist_min(None, -1, 0, None, L.I64, None, 0, None) == L.IXP_EINVAL
    assert lib.ixp_hist_min(None, 4, 0, None, 7, None, 0, None) == L.IXP_EINVAL
    assert lib.ixp_scatter_checked_workspace(-1) == 0
    assert lib.ixp_scatter_checked_workspace(1000) >= 8000
    assert lib.ixp_scatter_checked(None, 10, None, L.I64, None, 5, 3, None, None, 0, None) == L.IXP_EINVAL
    verdict = ctypes.create_string_buffer(64)   # host memory: the call must fail before using it
    assert lib.ixp_scatter_checked(None, 10, None, L.I64, None, 0, 16, verdict, None, 0, None) == L.IXP_EUNSUPPORTED
    assert lib.ixp_zero(None, 16, None) == L.IXP_EINVAL
    assert lib.ixp_zero(None, 0, None) == L.IXP_OK
    assert lib.ixp_match_min(None, None, 4, None, L.I64, None, 3, None) == L.IXP_EINVAL
    # v-way partition: class count, unsorted thresholds, key type
    assert lib.ixp_partition_v_workspace(-1) == 0
    # structs of the handle's own argument types (an earlier test reloads the module)
    c = lib.ixp_partition_v.argtypes[3]._type_()
    c.kind, c.v = L.CLASS_THRESH, 5
    cnt = ctypes.c_int64(0)
    ws = ctypes.create_string_buffer(1 << 16)
    args = (ctypes.byref(c), None, None, L.I32, ctypes.addressof(cnt), ws, len(ws), None)
    assert lib.ixp_partition_v(None, L.F32, 0, *args) == L.IXP_EINVAL         # v > 4
    c.v, c.s[0], c.s[1] = 3, 0.5, 0.2
    assert lib.ixp_partition_v(None, L.F32, 0, *args) == L.IXP_EINVAL         # thresholds not sorted
    c.kind, c.v = L.CLASS_MOD, 3
    assert lib.ixp_partition_v(None, L.F32, 0, *args) == L.IXP_EINVAL         # modulus needs int32 keys
    # segment tools and sgmSum
    assert lib.ixp_mk_ii_workspace(-1, 3) == 0
    assert lib.ixp_mk_ii(None, 3, 10, None, L.I32, None, 0, None) == L.IXP_EINVAL
    assert lib.ixp_mk_ii(None, 0, 0, None, 9, None, 0, None) == L.IXP_EINVAL
    assert lib.ixp_mk_sgm_descr(None, 2, 5, None, None, None, 0, None) == L.IXP_EINVAL
    assert lib.ixp_sgm_sum_workspace(-1) == 0
    assert lib.ixp_sgm_sum(None, None, 10, None, None, 0, None) == L.IXP_EINVAL
    # row predicates are rejected by calls without rows
    p = lib.ixp_partition.argtypes[3]._type_()
    p.kind = L.PRED_LT_ROW
    split = ctypes.c_int64(0)
    rc = lib.ixp_partition(None, L.F32, 0, ctypes.byref(p), 0, None, None, L.I64,
                           ctypes.addressof(split), ws, len(ws), None)
    assert rc == L.IXP_EINVAL
