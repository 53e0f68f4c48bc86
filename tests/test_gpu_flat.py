"""GPU parity of the flat partition / filter against the CPU oracle (bit-exact).

Every case runs the HIP path through the C ABI and the oracle on the same
seeded input, and compares output keys, indices and the split point exactly.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


def _preds(kind, keys_np, **kw):
    if kind == "mod":
        return P.Pred.mod_eq(kw["d"], kw["r"]), O.Pred.mod_eq(kw["d"], kw["r"])
    if kind == "lt":
        return P.Pred.lt(kw["s"]), O.Pred.lt(kw["s"])
    flags = kw["flags"]
    return (P.Pred.from_flags(torch.from_numpy(flags).to(DEV)),
            O.Pred.from_flags(flags))


def run_both(keys_np, kind, mode, idx_dtype=torch.int64, keys_t=None, **kw):
    gp, op = _preds(kind, keys_np, **kw)
    kt = torch.from_numpy(keys_np).to(DEV) if keys_t is None else keys_t
    print(f"[flat] n={len(keys_np)} pred={kind} mode={mode} idx={idx_dtype}", flush=True)
    ok, oi, sp = P.partition(kt, gp, mode=mode, idx_dtype=idx_dtype)
    torch.cuda.synchronize()
    ys, idx, t = O.partition2(keys_np, op, mode)
    T = int(sp.item())
    assert T == t
    gi = oi.cpu().numpy().astype(np.int64)
    assert np.array_equal(gi, idx), f"first idx mismatch at {np.argmax(gi != idx)}"
    gk = ok.cpu().numpy()
    n_out = len(keys_np) if mode == P.MODE_PARTITION else t
    assert np.array_equal(gk[:n_out].view(np.uint32), ys[:n_out].view(np.uint32))
    return gk, gi, T


def test_paper_demo_on_gpu():
    xs = np.array([5, 4, 2, 8, 7, 3], dtype=np.float32)
    gk, gi, T = run_both(xs, "lt", P.MODE_PARTITION, s=5.0)
    assert gi.tolist() == [3, 0, 1, 4, 5, 2] and T == 3
    assert gk.tolist() == [4, 2, 3, 5, 8, 7]


EDGE_N = [0, 1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097, 8191, 12289,
          (1 << 20) + 17]


@pytest.mark.parametrize("n", EDGE_N)
@pytest.mark.parametrize("mode", [0, 1])
def test_edge_sizes_random(n, mode):
    keys = W.int_keys(n, 100 + n)
    run_both(keys, "mod", mode, torch.int64, d=2, r=0)
    run_both(keys, "mod", mode, torch.int32, d=3, r=1)


@pytest.mark.parametrize("pattern", ["all_true", "all_false", "alternating", "blocks"])
@pytest.mark.parametrize("n", [1, 4097, 100_003])
def test_flag_patterns(pattern, n):
    i = np.arange(n)
    flags = {"all_true": np.ones(n), "all_false": np.zeros(n),
             "alternating": i % 2, "blocks": (i // 5000) % 2}[pattern].astype(np.uint8)
    keys = W.int_keys(n, 7)
    for mode in (0, 1):
        run_both(keys, "flags", mode, torch.int32, flags=flags)


def test_predicate_edge_values():
    keys = np.array([-7, -6, -1, 0, 1, 5, 2**31 - 1, -2**31] * 700, dtype=np.int32)
    for d, r in [(2, 0), (3, 1), (3, 2), (7, 6), (1, 0), (2**32 - 1, 5), (2**31, 2**31 - 1)]:
        run_both(keys, "mod", 0, torch.int64, d=d, r=r)
    f = np.array([0.0, -0.0, 0.5, 0.49999997, np.nan, -np.inf, np.inf, 1e-40] * 700,
                 dtype=np.float32)
    for s in (0.5, 0.0, 1e-40, -np.inf):
        run_both(f, "lt", 0, torch.int32, s=s)
        run_both(f, "lt", 1, torch.int32, s=s)


def test_unaligned_views_take_scalar_path():
    base = W.int_keys(50_001, 8)
    t = torch.from_numpy(base).to(DEV)
    for off in (1, 2, 3):
        view = t[off:]
        assert view.data_ptr() % 16 != 0
        run_both(base[off:], "mod", 0, torch.int64, keys_t=view, d=2, r=0)


def test_indices_only_and_keys_only():
    keys = W.int_keys(70_000, 9)
    kt = torch.from_numpy(keys).to(DEV)
    _, idx, t = O.partition2(keys, O.Pred.mod_eq(2, 0))
    ok, oi, sp = P.partition(kt, P.Pred.mod_eq(2, 0), want_keys=False)
    assert ok is None and np.array_equal(oi.cpu().numpy(), idx)
    ok, oi, sp = P.partition(kt, P.Pred.mod_eq(2, 0), want_idx=False)
    ys, _, _ = O.partition2(keys, O.Pred.mod_eq(2, 0))
    assert oi is None and np.array_equal(ok.cpu().numpy(), ys) and sp.item() == t


def test_invalid_arguments_rejected():
    kt = torch.zeros(10, dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError):
        P.partition(kt, P.Pred.mod_eq(0, 0))          # d must be >= 1
    with pytest.raises(ValueError):
        P.partition(kt, P.Pred.lt(0.5))               # LT needs f32 keys
    with pytest.raises(ValueError):
        P.partition(kt, P.Pred.mod_eq(2, 0), mode=7)


@pytest.mark.parametrize("n", [1023, 1024, 1025, 2047, 3 * 1024 + 3, (1 << 20) - 1, 1 << 20,
                               (1 << 20) + 1, (1 << 22) - 1, 1 << 22, (1 << 22) + 1])
@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
def test_sizes_at_the_small_path_bounds(n, idx_dtype):
    """One wave per 1024-element tile up to 2^20 keys, 4096-element tiles
    counted per tile up to 2^22, the counting pass above: every side of both
    bounds, with a key predicate and with a flag predicate."""
    keys = W.int_keys(n, 17)
    run_both(keys, "mod", P.MODE_PARTITION, idx_dtype, d=3, r=2)
    flags = (np.random.default_rng(n).random(n) < 0.3).astype(np.uint8)
    run_both(keys, "flags", P.MODE_PARTITION, idx_dtype, flags=flags)


def test_flag_predicate_without_keys_small():
    """A flag predicate needs no key array when no keys are written."""
    n = 300_001
    flags = (np.random.default_rng(3).random(n) < 0.6).astype(np.uint8)
    _, idx, t = O.partition2(np.zeros(n, dtype=np.int32), O.Pred.from_flags(flags))
    ft = torch.from_numpy(flags).to(DEV)
    oi = torch.empty(n, dtype=torch.int64, device=DEV)
    sp = torch.empty(1, dtype=torch.int64, device=DEV)
    lib = P._lib.lib()
    ws = torch.empty(lib.ixp_partition_workspace(n), dtype=torch.uint8, device=DEV)
    pc = P.Pred.from_flags(ft).c()
    import ctypes
    rc = lib.ixp_partition(None, P._lib.I32, n, ctypes.byref(pc), P.MODE_PARTITION, None, oi.data_ptr(),
                           P._lib.I64, sp.data_ptr(), ws.data_ptr(), ws.numel(),
                           torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    assert int(sp.item()) == t and np.array_equal(oi.cpu().numpy(), idx)


def test_config_flat_small_int64_indices():
    """n = 2^20 int32 keys uniform in [0, 2^31), key % 2 == 0, int64 indices."""
    keys = W.int_keys(W.FLAT_SMALL_N, W.FLAT_SMALL_SEED)
    run_both(keys, "mod", P.MODE_PARTITION, torch.int64, d=2, r=0)


@pytest.mark.parametrize("s", W.FLAT_LARGE_SELECTIVITIES)
def test_config_flat_large_full_compare(s):
    """n = 2^28 f32 uniform in [0,1), x < s, int32 positions: partition and
    filter, compared element by element with the oracle."""
    x = _large_input()
    run_both(x, "lt", P.MODE_PARTITION, torch.int32, s=s)
    run_both(x, "lt", P.MODE_FILTER, torch.int32, s=s)


_LARGE = {}


def _large_input():
    if "x" not in _LARGE:
        _LARGE["x"] = W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)
    return _LARGE["x"]


def test_deterministic_repeat():
    keys = W.int_keys(3_000_001, 13)
    kt = torch.from_numpy(keys).to(DEV)
    a = P.partition(kt, P.Pred.mod_eq(3, 0))
    b = P.partition(kt, P.Pred.mod_eq(3, 0))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def test_unaligned_output_keys():
    """Output keys 4-byte but not 16-byte aligned: the run writer's head and
    tail handle the misalignment."""
    keys = W.int_keys(100_001, 14)
    kt = torch.from_numpy(keys).to(DEV)
    ys, idx, t = O.partition2(keys, O.Pred.mod_eq(2, 0))
    big = torch.zeros(len(keys) + 4, dtype=torch.int32, device=DEV)
    for off in (1, 2, 3):
        out = big[off:off + len(keys)]
        assert out.data_ptr() % 16 != 0
        P.partition(kt, P.Pred.mod_eq(2, 0), out_keys=out)
        assert np.array_equal(out.cpu().numpy(), ys)


@pytest.mark.parametrize("mode", [0, 1])
def test_captured_graph_replays_match_eager(mode):
    """The flat call enqueues only kernels (the partition scatter with LDS
    reserved at launch), so it can be captured into a HIP graph: every replay,
    with the input refilled in place and eager work in between, matches an
    eager call on the same input."""
    n = 3 * 4096 * 7 + 123
    x = torch.from_numpy(W.f32_uniform(n, 70)).to(DEV)
    ok = torch.empty_like(x)
    oi = torch.empty(n, dtype=torch.int32, device=DEV)
    sp = torch.empty(1, dtype=torch.int64, device=DEV)
    pred = P.Pred.lt(0.4)
    P.partition(x, pred, mode, torch.int32, out_keys=ok, out_idx=oi, split=sp)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.partition(x, pred, mode, torch.int32, out_keys=ok, out_idx=oi, split=sp)
    for rep in range(4):
        print(f"[graph] mode={mode} replay={rep}", flush=True)
        x.copy_(torch.from_numpy(W.f32_uniform(n, 71 + rep)).to(DEV))
        g.replay()
        torch.cuda.synchronize()
        got = (ok.clone(), oi.clone(), sp.clone())
        ek, ei, es = P.partition(x, pred, mode, torch.int32)
        torch.cuda.synchronize()
        nout = n if mode == 0 else int(es.item())
        assert torch.equal(got[2], es)
        assert torch.equal(got[1], ei)
        assert torch.equal(got[0][:nout], ek[:nout])
    del g
