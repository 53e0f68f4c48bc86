"""GPU parity of the segmented partition (partition2L / filter_seg) with the
CPU oracle, bit-exact: keys, indices, per-row split points and the segment
descriptor bytes."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


def _preds(kind, **kw):
    if kind == "mod":
        return P.Pred.mod_eq(kw["d"], kw["r"]), O.Pred.mod_eq(kw["d"], kw["r"])
    if kind == "lt":
        return P.Pred.lt(kw["s"]), O.Pred.lt(kw["s"])
    flags = kw["flags"]
    return P.Pred.from_flags(torch.from_numpy(flags).to(DEV)), O.Pred.from_flags(flags)


def run_both(keys, shape, kind="mod", mode=0, idx_dtype=torch.int32, tune=None, **kw):
    if not kw:
        kw = {"d": 3, "r": 0}
    gp, op = _preds(kind, **kw)
    print(f"[seg] n={len(keys)} m={len(shape)} pred={kind} mode={mode} tune={tune}", flush=True)
    kt = torch.from_numpy(keys).to(DEV)
    st = torch.from_numpy(np.asarray(shape, dtype=np.int64)).to(DEV)
    ok, oi, ss, fl = P.segmented_partition(kt, st, gp, mode=mode, idx_dtype=idx_dtype, tune=tune)
    torch.cuda.synchronize()
    assert P.segmented_error() == 0
    ys, idx, seg, flags = O.partition2L(keys, np.asarray(shape, dtype=np.int64), op, mode)
    gi = oi.cpu().numpy().astype(np.int64)
    assert np.array_equal(gi, idx), f"idx differs first at {np.argmax(gi != idx)}"
    assert np.array_equal(ss.cpu().numpy(), seg)
    assert np.array_equal(fl.cpu().numpy(), flags)
    nout = len(keys) if mode == P.MODE_PARTITION else int(seg.sum())
    gk = ok.cpu().numpy()[:nout]
    assert np.array_equal(gk.view(np.uint32), ys[:nout].view(np.uint32))
    return gk, gi, ss.cpu().numpy()


def test_paper_shape_example():
    # the jagged shape of the paper's mkSgmDescr / mkII example
    shape = [0, 2, 1, 0, 3]
    keys = np.array([3, 4, 9, 5, 6, 7], dtype=np.int32)
    gk, gi, ss = run_both(keys, shape)
    # row 1 = [3,4] -> trues (x%3==0) first: [3,4]; row 2 = [9]; row 4 = [5,6,7] -> [6,5,7]
    assert gk.tolist() == [3, 4, 9, 6, 5, 7]
    assert ss.tolist() == [0, 1, 1, 0, 1]


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
def test_random_shapes_with_empty_rows(mode, idx_dtype):
    for seed, (m, med, sig, empty) in enumerate([(1, 3, 0, 0), (17, 4, 2, 0.3), (300, 8, 2, 0.2),
                                                 (2000, 6, 1.5, 0.5), (40, 13, 1.5, 0.1)]):
        shape = W.segment_sizes(m, 200 + seed, median_log2=med, sigma_log2=sig, empty_frac=empty)
        keys = W.int_keys(int(shape.sum()), 300 + seed)
        run_both(keys, shape, mode=mode, idx_dtype=idx_dtype)


@pytest.mark.parametrize("tune", [(256, 2), (256, 4), (256, 8), (512, 2), (512, 4), (512, 8),
                                  (1024, 2), (1024, 4), (512, 4, 1), (256, 2, 64)])
def test_every_tiling_matches(tune):
    shape = W.segment_sizes(400, 11, median_log2=11, sigma_log2=2.0, empty_frac=0.1)
    keys = W.int_keys(int(shape.sum()), 12)
    run_both(keys, shape, tune=tune)
    run_both(keys, shape, mode=1, tune=tune)


def test_rows_spanning_many_items_and_unaligned_starts():
    shape = np.array([1, 3, 70_001, 2, 5, 0, 130_003, 1, 0, 4097, 4095, 16385], dtype=np.int64)
    keys = W.int_keys(int(shape.sum()), 5)
    run_both(keys, shape)
    run_both(keys, shape, mode=1)
    f = W.f32_uniform(int(shape.sum()), 6)
    run_both(f, shape, kind="lt", s=0.3)
    flags = (W.int_keys(int(shape.sum()), 7) % 5 == 0).astype(np.uint8)
    run_both(keys, shape, kind="flags", flags=flags)


def test_degenerate_shapes():
    run_both(np.zeros(0, np.int32), [])
    run_both(np.zeros(0, np.int32), [0, 0, 0])
    run_both(np.arange(7, dtype=np.int32), [7])
    run_both(np.arange(9, dtype=np.int32), [0, 0, 9, 0])
    # n not a multiple of 4 at the array end
    keys = W.int_keys(10_007, 3)
    run_both(keys, [5000, 5007])


def test_invalid_shape_reported_on_device_and_outputs_untouched():
    keys = torch.arange(10, dtype=torch.int32, device=DEV)
    out_idx = torch.full((10,), 77, dtype=torch.int32, device=DEV)
    for bad in ([5, -1, 6], [3, 3], [4, 4, 4]):
        shape = torch.tensor(bad, dtype=torch.int64, device=DEV)
        P.segmented_partition(keys, shape, P.Pred.mod_eq(2, 0), out_idx=out_idx)
        assert P.segmented_error() == P._lib.IXP_EINVAL
        assert (out_idx == 77).all()
    assert P.segmented_error() == 0


def test_config_segmented_full_compare():
    """10^4 rows, log-normal sizes (median 2^12, sigma 1.5 in log2), int32 keys,
    key % 3 == 0, with the descriptor flag array."""
    shape = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
    keys = W.int_keys(int(shape.sum()), W.SEG_KEYS_SEED)
    run_both(keys, shape)
    run_both(keys, shape, tune=(256, 4, 64, 2))   # every sibling counted by the waiter
    shape_e = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED, empty_frac=0.1)
    run_both(keys[: int(shape_e.sum())].copy(), shape_e, mode=0)


def _items(shape, tile):
    o = np.concatenate([[0], np.cumsum(shape)])[:-1]
    return np.where(shape > 0, ((o & 3) + shape + tile - 1) // tile, 0)


@pytest.mark.parametrize("mode,tune", [(0, (256, 4, 64, 1)), (0, (256, 2, 64, 1)),
                                       (1, None), (1, (256, 2, 64, 0)), (1, (1024, 4, 0, 0))])
def test_config_segmented_counted_items_lookback(mode, tune):
    """The 10^4-row workload with the counting pass: row sync COUNT counts
    every item of a multi-item row, filter mode every item.  Every case counts
    more than 8192 items (11,331 to 39,318), so the item scan chains two to
    five 8192-count chunks by decoupled look-back."""
    shape = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
    keys = W.int_keys(int(shape.sum()), W.SEG_KEYS_SEED)
    tile = (tune[0] * tune[1] * 4) if tune else 4096
    it = _items(shape, tile)
    counted = int(it.sum()) if mode == 1 else int(it[it > 1].sum())
    assert counted > 8192, counted
    run_both(keys, shape, mode=mode, tune=tune)


def test_graph_replays_match_eager():
    shape = W.segment_sizes(500, 21, median_log2=10, sigma_log2=1.5, empty_frac=0.1)
    n = int(shape.sum())
    k1 = torch.from_numpy(W.int_keys(n, 22)).to(DEV)
    st = torch.from_numpy(shape).to(DEV)
    g = P.SegmentedGraph(k1, st, P.Pred.mod_eq(3, 0))
    for rep in range(4):
        # refill the captured input in place, then replay
        g.keys.copy_(torch.from_numpy(W.int_keys(n, 30 + rep)).to(DEV))
        ok, oi, ss, fl = [t.clone() for t in g.launch()]
        torch.cuda.synchronize()
        ek, ei, es, ef = P.segmented_partition(g.keys, st, P.Pred.mod_eq(3, 0))
        torch.cuda.synchronize()
        assert torch.equal(ok, ek) and torch.equal(oi, ei)
        assert torch.equal(ss, es) and torch.equal(fl, ef)
        assert g.error() == 0
    g.close()


def test_autotuner_returns_a_valid_tiling():
    shape = W.segment_sizes(1000, 41, median_log2=10, sigma_log2=1.5)
    keys = W.int_keys(int(shape.sum()), 42)
    kt = torch.from_numpy(keys).to(DEV)
    st = torch.from_numpy(shape).to(DEV)
    best, ms = P.tune_segmented(kt, st, P.Pred.mod_eq(3, 0), reps=2)
    assert best[0] in (256, 512, 1024) and best[1] in (2, 4, 8) and ms > 0
    assert best[3] in (P._lib.ROW_SYNC_COUNT, P._lib.ROW_SYNC_WAIT)
    run_both(keys, shape, tune=best)


@pytest.mark.parametrize("tune", [(256, 2), (512, 2), (512, 4), (1024, 4)])
def test_many_rows_per_tile_with_empty_rows(tune):
    """Rows of 0-3 elements: a tile holds hundreds of rows, with empty rows
    between them."""
    shape = np.random.default_rng(77).integers(0, 4, 200_000).astype(np.int64)
    keys = W.int_keys(int(shape.sum()), 78)
    run_both(keys, shape, tune=tune)


@pytest.mark.parametrize("tune", [(256, 2), (512, 2), (512, 4), (1024, 4)])
def test_rows_on_tile_boundaries(tune):
    """Row starts and ends exactly on tile boundaries (tiles of 2048 to 16384
    elements), rows filling whole tiles, and empty rows at a boundary."""
    shape = np.array([4096, 8192, 2048, 2048, 4096 * 3, 1, 4095, 0, 4096, 0, 0, 16384, 2048, 0],
                     dtype=np.int64)
    keys = W.int_keys(int(shape.sum()), 79)
    run_both(keys, shape, tune=tune)
    run_both(keys, shape, tune=tune, kind="flags",
             flags=(W.int_keys(int(shape.sum()), 80) % 3 == 0).astype(np.uint8))


@pytest.mark.parametrize("row_sync", [0, 1, 2, 3])
@pytest.mark.parametrize("geom", [(256, 2, 0), (256, 2, 64), (1024, 4, 0)])
def test_row_sync_modes(row_sync, geom):
    """Rows of 2..256 items learn T_k inside the main kernel (WAIT, 3), from
    the counting pass (COUNT, 1), by counting every sibling not yet published
    (NOWAIT, 2: the fallback of WAIT made the rule), or by the grid's choice
    (AUTO, 0).  With 2048-element tiles,
    rows of 64/65 and 128/129 items straddle the 64-wide chunks of the
    exchange, and rows of 256/257 items the limit between the exchange and
    the counting pass."""
    t = 2048
    shape = np.array([3, 64 * t - 3, 64 * t, 1, 64 * t + 1, 2, t + 1, 0, 65 * t, 7, 2 * t,
                      128 * t, 128 * t + 3, 256 * t - 4, 256 * t + 2, 257 * t,
                      63 * t + 5, 5, 3 * t - 1], dtype=np.int64)
    o = np.concatenate([[0], np.cumsum(shape)])[:-1]
    items = np.where(shape > 0, ((o & 3) + shape + t - 1) // t, 0)
    assert {64, 65, 128, 129, 256, 257} <= set(items.tolist())
    keys = W.int_keys(int(shape.sum()), 91)
    tune = geom + (row_sync,)
    run_both(keys, shape, tune=tune)
    run_both(keys, shape, mode=1, tune=tune)
    run_both(W.f32_uniform(int(shape.sum()), 92), shape, kind="lt", s=0.6, tune=tune)
    flags = (W.int_keys(int(shape.sum()), 93) % 7 == 0).astype(np.uint8)
    run_both(keys, shape, kind="flags", flags=flags, tune=tune)
    mix = W.segment_sizes(700, 94, median_log2=13, sigma_log2=1.5, empty_frac=0.1)
    run_both(W.int_keys(int(mix.sum()), 95), mix, tune=tune)


def test_rows_of_millions_of_elements_among_small_rows():
    """Rows spanning hundreds of tiles next to rows of a few elements."""
    shape = np.array([5, 3_000_001, 7, 0, 70_000, 2_500_000, 1], dtype=np.int64)
    keys = W.int_keys(int(shape.sum()), 81)
    run_both(keys, shape)
    run_both(keys, shape, tune=(1024, 4))
    run_both(keys, shape, tune=(256, 2, 0, 2))
    run_both(keys, shape, mode=1)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tune", [None, (256, 2), (1024, 4), (256, 2, 0, 2), (512, 4, 0, 1)])
def test_predicates_of_the_row_number(mode, tune):
    """partition2L with predicates of the row number k: x < s[k] (per-row
    thresholds) and x mod 3 == k mod 3, against the row-predicate oracle."""
    shape = W.segment_sizes(3000, 111, median_log2=9, sigma_log2=2.0, empty_frac=0.15)
    n = int(shape.sum())
    g = np.random.default_rng(112)
    s_rows = g.random(len(shape)).astype(np.float32)
    xf = W.f32_uniform(n, 113)
    xi = W.int_keys(n, 114) - (1 << 30)
    st = torch.from_numpy(shape).to(DEV)
    for pred, x, kind in ((P.Pred.lt_rows(torch.from_numpy(s_rows).to(DEV)), xf, O.ROW_LT),
                          (P.Pred.mod_rows(3), xi, O.ROW_MOD)):
        print(f"[seg-rows] n={n} kind={kind} mode={mode} tune={tune}", flush=True)
        ok, oi, ss, fl = P.segmented_partition(torch.from_numpy(x).to(DEV), st, pred, mode=mode, tune=tune)
        torch.cuda.synchronize()
        assert P.segmented_error() == 0
        ys, idx, seg, flags = O.partition2L_rows(x, shape, kind, 3, s_rows, mode)
        assert np.array_equal(oi.cpu().numpy().astype(np.int64), idx)
        assert np.array_equal(ss.cpu().numpy(), seg) and np.array_equal(fl.cpu().numpy(), flags)
        nout = n if mode == 0 else int(seg.sum())
        assert np.array_equal(ok.cpu().numpy()[:nout].view(np.uint32), ys[:nout].view(np.uint32))


def test_row_predicates_rejected_without_rows():
    x = torch.zeros(16, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        P.partition(x, P.Pred.lt_rows(torch.zeros(1, device=DEV)))


def test_filter_seg_counts_beyond_2e32():
    """filter_seg of 2^32 + 2^28 all-true flags in three rows, tiles of 16384:
    34 chunks of 8192 item counts, each chunk holding 2^27 trues, so the
    item scan's look-back windows sum past 2^32.  With every flag set the
    row counts are the row sizes, and the rows that span chunk boundaries see
    any wrapped window sum."""
    n = (1 << 32) + (1 << 28)
    a = (1 << 31) + 3
    shape = torch.tensor([a, n - a - 7, 7], dtype=torch.int64, device=DEV)
    flags = torch.ones(n, dtype=torch.uint8, device=DEV)
    seg = torch.full((3,), -1, dtype=torch.int64, device=DEV)
    t = P._lib.ixp_tuning()
    t.block, t.rows, t.wgs_per_cu, t.row_sync = 1024, 4, 0, 0
    ws = torch.empty(P._lib.lib().ixp_segmented_workspace(n, 3, ctypes.byref(t)), dtype=torch.uint8,
                     device=DEV)
    pc = P.Pred.from_flags(flags).c()
    print(f"[seg-2^32] n={n} ws={ws.numel()}", flush=True)
    rc = P._lib.lib().ixp_segmented_partition(
        None, P._lib.I32, n, shape.data_ptr(), 3, ctypes.byref(pc), P.MODE_FILTER, None, None,
        P._lib.I64, seg.data_ptr(), None, ctypes.byref(t), ws.data_ptr(), ws.numel(),
        torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    assert P._lib.lib().ixp_read_error(ws.data_ptr(), torch.cuda.current_stream().cuda_stream) == 0
    assert seg.cpu().tolist() == shape.cpu().tolist()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tune", [(256, 4, 64, 3), (256, 8, 64, 3), (512, 2, 0, 1)])
def test_any_subset_of_outputs_through_the_c_abi(mode, tune):
    """Every output of the C ABI may be NULL.  Each subset is produced on its
    own and compared with the oracle: keys only, indices only, descriptor
    bytes only, split points only, and indices of a flag predicate with no
    key array at all.  Rows of 0 to ~3 tiles, so single-item rows, exchanging
    multi-item rows and empty rows all occur."""
    g = np.random.default_rng(11 + mode)
    shape = g.integers(0, 3 * 4096, 900).astype(np.int64)
    shape[g.integers(0, 900, 120)] = 0
    shape[::97] = 1
    n = int(shape.sum())
    keys = W.int_keys(n, 12)
    flags = (g.random(n) < 0.4).astype(np.uint8)
    lib = P._lib.lib()
    t = P._lib.ixp_tuning()
    t.block, t.rows, t.wgs_per_cu, t.row_sync = tune
    m = len(shape)
    ws = torch.empty(lib.ixp_segmented_workspace(n, m, ctypes.byref(t)), dtype=torch.uint8, device=DEV)
    kt = torch.from_numpy(keys).to(DEV)
    st = torch.from_numpy(shape).to(DEV)
    stream = torch.cuda.current_stream().cuda_stream
    for kind in ("mod", "flags"):
        gp, op = _preds(kind, d=3, r=1, flags=flags)
        pc = gp.c()
        ys, idx, seg, fl = O.partition2L(keys, shape, op, mode)
        nout = n if mode == P.MODE_PARTITION else int(seg.sum())
        for want in ("keys", "idx", "flags", "split", "idx_no_keys"):
            if want == "idx_no_keys" and kind != "flags":
                continue
            print(f"[seg-subset] mode={mode} tune={tune} pred={kind} out={want}", flush=True)
            ok = torch.full((n,), 0x7F7F7F7F, dtype=torch.int32, device=DEV) if want == "keys" else None
            oi = torch.full((n,), -7, dtype=torch.int64, device=DEV) if want.startswith("idx") else None
            of = torch.full((n,), 9, dtype=torch.uint8, device=DEV) if want == "flags" else None
            osp = torch.full((m,), -5, dtype=torch.int64, device=DEV) if want == "split" else None
            src = None if want == "idx_no_keys" else kt.data_ptr()
            rc = lib.ixp_segmented_partition(
                src, P._lib.I32, n, st.data_ptr(), m, ctypes.byref(pc), mode,
                ok.data_ptr() if ok is not None else None, oi.data_ptr() if oi is not None else None,
                P._lib.I64, osp.data_ptr() if osp is not None else None,
                of.data_ptr() if of is not None else None, ctypes.byref(t), ws.data_ptr(), ws.numel(), stream)
            assert rc == 0
            assert lib.ixp_read_error(ws.data_ptr(), stream) == 0
            if ok is not None:
                got = ok.cpu().numpy()
                assert np.array_equal(got[:nout].view(np.uint32), ys[:nout].view(np.uint32))
                assert (got[nout:] == 0x7F7F7F7F).all()
            if oi is not None:
                assert np.array_equal(oi.cpu().numpy(), idx)
            if of is not None:
                assert np.array_equal(of.cpu().numpy(), fl)
            if osp is not None:
                assert np.array_equal(osp.cpu().numpy(), seg)


@pytest.mark.parametrize("tune", [None, (256, 8, 64, 3), (512, 2, 64, 1)])
def test_item_starts_on_and_off_the_cache_line(tune):
    """A row's first item starts on the 128-byte line of its first element
    only when that adds no item.  Rows one group short of a tile (their line
    start would spill into a second item), rows of a whole tile behind an
    odd offset, and rows that span several items with every start offset
    mod 32: both choices and every offset occur, in both modes."""
    tile = 4096 if tune is None else tune[0] * tune[1] * 4
    parts = [np.array([3]), np.full(40, tile - 4), np.array([2]), np.full(40, tile),
             np.full(32, 2 * tile + 5), np.arange(1, 33) * 97]
    shape = np.concatenate(parts).astype(np.int64)
    keys = W.int_keys(int(shape.sum()), 23)
    for mode in (0, 1):
        run_both(keys, shape, mode=mode, tune=tune)
