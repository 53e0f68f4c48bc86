"""mkII and mkSgmDescr (Section 2.1 segment helpers) as device outputs,
bit-exact against the CPU oracle (itself pinned to the paper's worked
examples)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


def _both(shape):
    shape = np.asarray(shape, dtype=np.int64)
    n = int(shape.sum())
    print(f"[shape-tools] m={len(shape)} n={n}", flush=True)
    st = torch.from_numpy(shape).to(DEV)
    xs = np.arange(1, len(shape) + 1, dtype=np.int64) * 7 - 3
    for dt in (torch.int32, torch.int64):
        ii = P.mk_ii(st, n, dt)
        assert np.array_equal(ii.cpu().numpy().astype(np.int64), O.mk_ii(shape))
    d = P.mk_sgm_descr(st, torch.from_numpy(xs).to(DEV), n)
    assert np.array_equal(d.cpu().numpy(), O.mk_sgm_descr(shape, xs))
    assert P.shape_tools_error() == 0


def test_paper_example_shape():
    _both([0, 2, 1, 0, 3])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_shapes(seed):
    for m, med, sig, empty in [(1, 3, 0, 0), (500, 4, 2, 0.4), (10_000, 12, 1.5, 0.1), (3000, 1, 1, 0.5)]:
        _both(W.segment_sizes(m, 300 + seed, median_log2=med, sigma_log2=sig, empty_frac=empty))


@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_outputs_not_16_byte_aligned(offset):
    """Outputs starting 1..3 elements past a 16-byte boundary take the
    element-wise stores; the aligned case takes 16-byte groups."""
    shape = W.segment_sizes(700, 77, median_log2=8, sigma_log2=2.0, empty_frac=0.2)
    n = int(shape.sum())
    st = torch.from_numpy(shape).to(DEV)
    xs = np.arange(len(shape), dtype=np.int64) * 5 + 1
    print(f"[shape-tools] offset={offset} n={n}", flush=True)
    for dt in (torch.int32, torch.int64):
        buf = torch.full((n + 8,), -9, dtype=dt, device=DEV)
        ii = P.mk_ii(st, n, dt, out=buf[offset:offset + n])
        assert np.array_equal(ii.cpu().numpy().astype(np.int64), O.mk_ii(shape))
        assert (buf[:offset] == -9).all() and (buf[offset + n:] == -9).all()
    buf = torch.full((n + 8,), -9, dtype=torch.int64, device=DEV)
    d = P.mk_sgm_descr(st, torch.from_numpy(xs).to(DEV), n, out=buf[offset:offset + n])
    assert np.array_equal(d.cpu().numpy(), O.mk_sgm_descr(shape, xs))
    assert (buf[:offset] == -9).all() and (buf[offset + n:] == -9).all()


def test_degenerate_and_bad_shapes():
    _both([])
    _both([0, 0])
    _both([70_001, 0, 130_003])
    st = torch.tensor([3, -1, 4], dtype=torch.int64, device=DEV)
    out = P.mk_ii(st, 6)
    assert P.shape_tools_error() == P._lib.IXP_EINVAL


@pytest.mark.parametrize("n", [0, 1, 7, 8191, 8192, 8193, 100_003, (1 << 22) + 5])
@pytest.mark.parametrize("density", [0.0, 1e-5, 0.01, 0.5, 1.0])
def test_sgm_sum_matches_oracle(n, density):
    g = np.random.default_rng(n + int(density * 1000))
    flags = (g.random(n) < density).astype(np.uint8)
    xs = g.integers(-2**40, 2**40, n)
    print(f"[sgm_sum] n={n} density={density}", flush=True)
    got = P.sgm_sum(torch.from_numpy(flags).to(DEV), torch.from_numpy(xs).to(DEV))
    assert np.array_equal(got.cpu().numpy(), O.sgm_sum(flags, xs))


@pytest.mark.parametrize("offset", [0, 1, 3, 7])
def test_sgm_sum_flags_not_8_byte_aligned(offset):
    """Flag arrays starting 1..7 bytes past an 8-byte boundary are read byte
    by byte, aligned ones 8 bytes per thread; both over several chunks and a
    ragged last tile."""
    n = 3 * 8192 * 5 + 1234
    g = np.random.default_rng(900 + offset)
    flags = (g.random(n) < 3e-4).astype(np.uint8)
    flags[8191] = 1   # last element of a tile
    xs = g.integers(-2**40, 2**40, n)
    print(f"[sgm_sum] offset={offset} n={n}", flush=True)
    buf = torch.zeros(n + 16, dtype=torch.uint8, device=DEV)
    buf[offset:offset + n] = torch.from_numpy(flags).to(DEV)
    got = P.sgm_sum(buf[offset:offset + n], torch.from_numpy(xs).to(DEV))
    assert np.array_equal(got.cpu().numpy(), O.sgm_sum(flags, xs))


def test_sgm_sum_builds_mk_ii():
    """mkII as the paper builds it: sgmSum over the segment descriptor of the
    row numbers (row k at o_k, 0 elsewhere; flags where it is nonzero)."""
    shape = W.segment_sizes(5000, 120, median_log2=8, sigma_log2=2.0, empty_frac=0.2)
    n = int(shape.sum())
    st = torch.from_numpy(shape).to(DEV)
    rows = torch.arange(1, len(shape) + 1, dtype=torch.int64, device=DEV)   # k + 1
    descr = P.mk_sgm_descr(st, rows, n)
    vals = torch.where(descr > 0, descr - 1, torch.zeros_like(descr))
    ii = P.sgm_sum((descr > 0).to(torch.uint8), vals)
    assert torch.equal(ii, P.mk_ii(st, n)) and np.array_equal(ii.cpu().numpy(), O.mk_ii(shape))


def test_sgm_sum_chunks_of_several_tiles():
    """Above 8192 * 8192 elements a chunk holds several tiles, rescanned in
    order with a carried prefix."""
    n = (1 << 26) + 12_345
    g = np.random.default_rng(121)
    flags = (g.random(n) < 2e-6).astype(np.uint8)     # long stretches without a flag
    xs = g.integers(-2**30, 2**30, n)
    print(f"[sgm_sum] n={n} multi-tile chunks", flush=True)
    got = P.sgm_sum(torch.from_numpy(flags).to(DEV), torch.from_numpy(xs).to(DEV))
    assert np.array_equal(got.cpu().numpy(), O.sgm_sum(flags, xs))
