"""ixp_partition_noalloc (the entry point for callers that cannot allocate)
against ixp_partition on the same inputs, through the C ABI: outputs must be
identical bit for bit.  Two calls in a row share the device's static scratch,
the second on a smaller input, in both modes and with both index widths."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd._lib as L  # noqa: E402

DEV = "cuda:0"


def _pred_lt(s):
    p = L.ixp_pred()
    p.kind, p.s = L.PRED_LT, s
    return p


def _pred_mod(d, r):
    p = L.ixp_pred()
    p.kind, p.d, p.r = L.PRED_MOD_EQ, d, r
    return p


def _call(noalloc, x, key_t, pred, mode, idx_dtype):
    n = x.numel()
    lib = L.lib()
    out_k = torch.full_like(x, 0x7F7F7F7F if x.dtype == torch.int32 else float("nan"))
    out_i = torch.full((n,), -7, dtype=idx_dtype, device=DEV)
    split = torch.full((1,), -9, dtype=torch.int64, device=DEV)
    idx_t = L.I32 if idx_dtype == torch.int32 else L.I64
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        rc = lib.ixp_partition_noalloc(x.data_ptr(), key_t, n, ctypes.byref(pred), mode,
                                       out_k.data_ptr(), out_i.data_ptr(), idx_t,
                                       split.data_ptr(), stream)
    else:
        ws = torch.empty(max(lib.ixp_partition_workspace(n), 1), dtype=torch.uint8, device=DEV)
        rc = lib.ixp_partition(x.data_ptr(), key_t, n, ctypes.byref(pred), mode, out_k.data_ptr(),
                               out_i.data_ptr(), idx_t, split.data_ptr(), ws.data_ptr(), ws.numel(),
                               stream)
    assert rc == L.IXP_OK, rc
    torch.cuda.synchronize()
    return out_k, out_i, split


def _same(a, b, n_keys):
    ka, ia, sa = a
    kb, ib, sb = b
    assert int(sa.item()) == int(sb.item())
    assert torch.equal(ia, ib)
    ka32, kb32 = ka.view(torch.int32), kb.view(torch.int32)
    assert torch.equal(ka32[:n_keys], kb32[:n_keys])


@pytest.mark.parametrize("mode", [L.MODE_PARTITION, L.MODE_FILTER])
@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
def test_noalloc_matches_workspace_call_twice(mode, idx_dtype):
    for n, seed in (((1 << 24) + 4099, 31), (70_001, 32)):
        print(f"[noalloc] f32 n={n} mode={mode} idx={idx_dtype}", flush=True)
        x = torch.from_numpy(W.f32_uniform(n, seed)).to(DEV)
        p = _pred_lt(0.37)
        a = _call(True, x, L.F32, p, mode, idx_dtype)
        b = _call(False, x, L.F32, p, mode, idx_dtype)
        n_keys = n if mode == L.MODE_PARTITION else int(b[2].item())
        _same(a, b, n_keys)


def test_noalloc_int_keys_unaligned_view_and_empty():
    """int32 keys under key % 3 == 1, a view starting one element in (the
    one-element load path), then an empty input (writes T = 0)."""
    base = torch.from_numpy(W.int_keys((1 << 20) + 9, 33)).to(DEV)
    for x in (base, base[1:]):
        print(f"[noalloc] int32 n={x.numel()} ptr%16={x.data_ptr() % 16}", flush=True)
        p = _pred_mod(3, 1)
        a = _call(True, x, L.I32, p, L.MODE_PARTITION, torch.int64)
        b = _call(False, x, L.I32, p, L.MODE_PARTITION, torch.int64)
        _same(a, b, x.numel())
    e = torch.empty(0, dtype=torch.int32, device=DEV)
    _, _, s = _call(True, e, L.I32, _pred_mod(3, 1), L.MODE_PARTITION, torch.int64)
    assert int(s.item()) == 0


def test_noalloc_rejects_sizes_beyond_the_scratch():
    lib = L.lib()
    split = torch.empty(1, dtype=torch.int64, device=DEV)
    p = _pred_lt(0.5)
    assert lib.ixp_partition_workspace(L.NOALLOC_MAX_N) <= L.NOALLOC_SCRATCH_BYTES
    rc = lib.ixp_partition_noalloc(None, L.F32, L.NOALLOC_MAX_N + 1, ctypes.byref(p), 0, None,
                                   None, L.I64, split.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert rc == L.IXP_ETOOLARGE
