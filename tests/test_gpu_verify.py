"""Reduce-by-index with min, the dynamically verified scatter and the zero
fill on the GPU, bit-exact against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
@pytest.mark.parametrize("n_dst,m", [(0, 10), (1, 0), (7, 1000), (100_003, 300_007), (1 << 20, 1 << 16)])
def test_hist_min_matches_oracle(n_dst, m, idx_dtype):
    g = np.random.default_rng(n_dst + m)
    idx = g.integers(-2, n_dst + 2, m)
    vals = g.integers(-10**15, 10**15, m)
    print(f"[hist] n_dst={n_dst} m={m} idx={idx_dtype}", flush=True)
    it = torch.from_numpy(idx).to(DEV).to(idx_dtype)
    got = P.hist_min(n_dst, 2**62, it, torch.from_numpy(vals).to(DEV))
    assert np.array_equal(got.cpu().numpy(), O.hist_min(n_dst, 2**62, idx, vals))
    got = P.hist_min(n_dst, m, it)
    assert np.array_equal(got.cpu().numpy(), O.hist_min(n_dst, m, idx))


def _checked(n_dst, idx, vals, idx_dtype=torch.int64):
    print(f"[checked] n_dst={n_dst} m={len(idx)} dtype={vals.dtype} idx={idx_dtype}", flush=True)
    dst, v = P.scatter_checked(n_dst, torch.from_numpy(idx).to(DEV).to(idx_dtype),
                               torch.from_numpy(vals).to(DEV))
    ref, rv = O.scatter_checked(n_dst, idx, vals)
    assert tuple(int(x) for x in v.cpu()) == rv
    assert np.array_equal(dst.cpu().numpy().view(np.uint8), ref.view(np.uint8))
    return rv


@pytest.mark.parametrize("idx_dtype", [torch.int32, torch.int64])
def test_checked_scatter_injective_and_out_of_bounds(idx_dtype):
    n = 1_000_003
    idx = np.random.default_rng(3).permutation(n)
    idx[::101] = -1
    idx[7::103] = n + 5
    assert _checked(n, idx, W.f32_uniform(n, 4), idx_dtype) == (1, -1, 0)
    assert _checked(n, idx, W.int_keys(n, 5).astype(np.int64), idx_dtype) == (1, -1, 0)


@pytest.mark.parametrize("k", [1, 10, 1000])
def test_checked_scatter_planted_repeats(k):
    n = 1 << 20
    g = np.random.default_rng(70 + k)
    idx = g.permutation(n)
    pos = g.choice(n, size=2 * k, replace=False)
    idx[pos[:k]] = idx[pos[k:]]           # k positions copy another's location
    v = _checked(n, idx, W.f32_uniform(n, 8))
    assert v[0] == 0 and v == O.check_inj(idx, 0, n)


def test_checked_scatter_many_writers_per_location():
    g = np.random.default_rng(11)
    for n_dst, m in [(1, 5000), (17, 100_000), (4096, 1 << 20)]:
        idx = g.integers(0, n_dst, m)
        _checked(n_dst, idx, W.f32_normal(m, 12))
        _checked(n_dst, idx, g.integers(0, 2**62, m))


@pytest.mark.parametrize("nbytes,off", [(0, 0), (1, 0), (15, 3), (16, 0), (1000, 1), (1 << 22, 0),
                                        ((1 << 22) + 7, 5)])
def test_zero_fill_exact_range(nbytes, off):
    buf = torch.full((nbytes + 64,), 0xAB, dtype=torch.uint8, device=DEV)
    P.zero_(buf[off:off + nbytes])
    h = buf.cpu().numpy()
    assert (h[off:off + nbytes] == 0).all()
    assert (h[:off] == 0xAB).all() and (h[off + nbytes:] == 0xAB).all()
