"""get_smallest_pairs (Section 6, maximal matching) on the GPU, bit-exact
against the CPU oracle; the outputs pass the device Inj checker."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"


def _run(n_verts, n_es, es, is_):
    print(f"[pairs] n_verts={n_verts} m={len(es)}", flush=True)
    eo, io = P.get_smallest_pairs(n_verts, n_es, torch.from_numpy(es).to(DEV), torch.from_numpy(is_).to(DEV))
    re, ri = O.get_smallest_pairs(n_verts, n_es, es, is_)
    assert np.array_equal(eo.cpu().numpy(), re) and np.array_equal(io.cpu().numpy(), ri)
    return eo, io


@pytest.mark.parametrize("n_verts,m", [(1, 1), (1, 1000), (7, 5), (1000, 3), (5000, 100_003),
                                       (1 << 20, 1 << 22)])
def test_pairs_match_oracle(n_verts, m):
    g = np.random.default_rng(n_verts * 7 + m)
    es = g.integers(0, n_verts, m)
    is_ = g.permutation(2 * m)[:m]
    eo, io = _run(n_verts, 2 * m, es, is_)
    v = P.verdicts(P.check_props(eo, P.INJ, lo=0, hi=n_verts))
    assert v[2][0] == 1   # Inj is bit 2
    v = P.verdicts(P.check_props(io, P.INJ, lo=0, hi=2 * m))
    assert v[2][0] == 1   # Inj is bit 2


def test_pairs_edge_cases():
    _run(4, 10, np.zeros(0, np.int64), np.zeros(0, np.int64))
    _run(0, 10, np.array([0, 1], np.int64), np.array([3, 4], np.int64))   # no vertices: nothing kept
    _run(3, 10, np.array([5, -1, 2, 2, 9], np.int64), np.array([0, 1, 7, 2, 3], np.int64))
    g = np.random.default_rng(5)
    es = np.where(g.random(10_001) < 0.1, -3, g.integers(0, 100, 10_001))   # out-of-range endpoints
    _run(100, 20_002, es, g.permutation(20_002)[:10_001])
