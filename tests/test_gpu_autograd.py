"""Row scatter / gather and the differentiable partition on the GPU.

Forward rows are compared bit for bit with the oracle's scatter and gradients
bit for bit with the oracle's gather (every gradient entry is one copied value,
so no rounding enters); torch's index_select gradient agrees in value; finite
differences in float64 check the linear map itself.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("cols,dtype", [(16, torch.float32), (3, torch.float32), (8, torch.float64),
                                        (1, torch.int32), (4, torch.float32), (8, torch.float32),
                                        (32, torch.float32), (64, torch.float32), (128, torch.float32)])
@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
def test_scatter_and_gather_rows_match_oracle(cols, dtype, idx_dtype):
    n = 100_003
    g = np.random.default_rng(5)
    perm = g.permutation(n)
    idx = perm.copy()
    idx[::97] = -1
    idx[1::101] = n + 3
    vals = g.standard_normal((n, cols)).astype(torch.empty(0, dtype=dtype).numpy().dtype)
    print(f"[rows] cols={cols} dtype={dtype} idx={idx_dtype}", flush=True)
    dst = torch.zeros((n, cols), dtype=dtype, device=DEV)
    P.scatter_inj(dst, torch.from_numpy(idx).to(DEV).to(idx_dtype), torch.from_numpy(vals).to(DEV))
    ref = O.scatter(np.zeros_like(vals), idx, vals)
    assert np.array_equal(dst.cpu().numpy().view(np.uint8), ref.view(np.uint8))
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    got = P.gather(dst, torch.from_numpy(perm).to(DEV).to(idx_dtype), err)
    assert np.array_equal(got.cpu().numpy().view(np.uint8), O.gather(ref, perm).view(np.uint8))
    assert err.item() == 0
    got = P.gather(dst, torch.tensor([0, n, -2, 5], device=DEV).to(idx_dtype), err)
    assert err.item() == 1
    assert (got[1] == 0).all() and (got[2] == 0).all()
    assert torch.equal(got[0], dst[0]) and torch.equal(got[3], dst[5])


def _forward_backward(n, seeds=W.AUTOGRAD_SEEDS, cols=W.AUTOGRAD_ROW, mode=P.MODE_PARTITION):
    keys = W.int_keys(n, seeds[0])
    payload = W.f32_normal((n, cols), seeds[1])
    gy = W.f32_normal((n, cols), seeds[2])
    kt = torch.from_numpy(keys).to(DEV)
    pt = torch.from_numpy(payload).to(DEV).requires_grad_(True)
    y, ok, idx, split = P.partition_scatter(kt, pt, P.Pred.mod_eq(2, 0), mode)
    y.backward(torch.from_numpy(gy).to(DEV))
    torch.cuda.synchronize()
    return keys, payload, gy, y.detach(), idx, split, pt.grad


@pytest.mark.parametrize("n", [1, 4097, 1 << 16, W.AUTOGRAD_N])
def test_partition_scatter_forward_and_gradient_exact(n):
    print(f"[autograd] n={n}", flush=True)
    keys, payload, gy, y, idx, split, grad = _forward_backward(n)
    _, oidx, t = O.partition2(keys, O.Pred.mod_eq(2, 0))
    assert int(split.item()) == t
    assert np.array_equal(idx.cpu().numpy(), oidx)
    yref = O.scatter(np.zeros_like(payload), oidx, payload)
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yref.view(np.uint32))
    # the gradient of row i is the upstream gradient at its destination:
    # bit for bit the oracle's gather of gy by the oracle's indices
    assert np.array_equal(grad.cpu().numpy().view(np.uint32), O.gather(gy, oidx).view(np.uint32))
    # torch reference: y = payload[inv] with inv the inverse permutation; its
    # gradient accumulates gy into zeros through inv (one contribution per
    # row), which equals ours in value -- only a -0.0 in gy comes back +0.0
    inv = torch.empty(n, dtype=torch.int64, device=DEV)
    inv[idx.long()] = torch.arange(n, device=DEV)
    pr = torch.from_numpy(payload).to(DEV).requires_grad_(True)
    yr = pr.index_select(0, inv)
    assert torch.equal(yr.detach(), y)
    yr.backward(torch.from_numpy(gy).to(DEV))
    assert torch.equal(pr.grad, grad)
    differ = pr.grad.view(torch.int32) != grad.view(torch.int32)
    assert (grad[differ] == 0).all()


@pytest.mark.parametrize("n", [1 << 16, W.AUTOGRAD_N])
def test_finite_differences_float64(n):
    """L = sum(w * y) in float64, at 2^16 rows and at the workload's 2^24.  The
    map is a permutation of rows, so central differences reproduce <grad, dv>
    up to float64 summation error, where dv is the perturbation actually
    applied after rounding to f32."""
    print(f"[fd] n={n}", flush=True)
    cols = W.AUTOGRAD_ROW
    keys = torch.from_numpy(W.int_keys(n, 43)).to(DEV)
    p = torch.from_numpy(W.f32_normal((n, cols), 44)).to(DEV)
    w = torch.from_numpy(W.f32_normal((n, cols), 45)).to(DEV).double()
    pred = P.Pred.mod_eq(2, 0)
    pg = p.clone().requires_grad_(True)
    y, *_ = P.partition_scatter(keys, pg, pred)
    (y.double() * w).sum().backward()
    g = pg.grad.double()
    eps = 1e-3
    for k in range(8):
        v = torch.from_numpy(W.f32_normal((n, cols), 100 + k)).to(DEV)
        pp, pm = p + eps * v, p - eps * v
        lp = (P.partition_scatter(keys, pp, pred)[0].double() * w).sum()
        lm = (P.partition_scatter(keys, pm, pred)[0].double() * w).sum()
        fd = (lp - lm) / (2 * eps)
        dv = (pp.double() - pm.double()) / (2 * eps)
        an = (g * dv).sum()
        assert abs(fd.item() - an.item()) <= 1e-9 * (abs(an.item()) + (g.abs() * dv.abs()).sum().item())


def test_gradcheck_float64_small():
    keys = torch.from_numpy(W.int_keys(37, 47)).to(DEV)
    p = torch.randn(37, 3, dtype=torch.float64, device=DEV, requires_grad=True)
    pred = P.Pred.mod_eq(3, 0)
    assert torch.autograd.gradcheck(lambda x: P.partition_scatter(keys, x, pred)[0], (p,))
    assert torch.autograd.gradcheck(lambda x: P.partition_scatter(keys, x, pred, P.MODE_FILTER)[0], (p,))


def test_filter_mode_gradient_zero_for_dropped_rows():
    keys, payload, gy, y, idx, split, grad = _forward_backward(50_001, mode=P.MODE_FILTER)
    c = keys % 2 == 0
    t = int(c.sum())
    assert int(split.item()) == t
    assert np.array_equal(y.cpu().numpy()[:t], payload[c])
    assert (y.cpu().numpy()[t:] == 0).all()
    gnp = grad.cpu().numpy()
    assert (gnp[~c] == 0).all()
    assert np.array_equal(gnp[c], gy[:t])
