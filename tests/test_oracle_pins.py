"""Pins of the CPU oracle to things other than itself (CPU only).

Each test fixes the oracle against a value the paper prints, a closed form the
paper states, a library routine (Python's stable ``sorted``, numpy), brute force
over tiny inputs, or a fault planted at a known index.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W
from conftest import load_golden


def _ints(tokens):
    return [int(t) for t in tokens]


def _bools(tokens):
    return [t == "T" for t in tokens]


# ---------------------------------------------------------------- goldens ---

def test_partition2_paper_demo():
    g = load_golden("partition2_demo.txt")
    xs = np.array(_ints(g["xs"]), dtype=np.float32)
    cs = O.map_pred(xs, O.Pred.lt(5))
    assert cs.tolist() == _bools(g["cs"])
    ys, idx, t = O.partition2(xs, O.Pred.lt(5))
    assert t == int(g["num_true"][0])
    assert idx.tolist() == _ints(g["indices"])
    assert ys.astype(int).tolist() == _ints(g["ys"])
    # The same through a caller flag array (partition2L's csL form).
    ys2, idx2, t2 = O.partition2(xs, O.Pred.from_flags(cs))
    assert (idx2 == idx).all() and (ys2 == ys).all() and t2 == t


def test_segment_helpers_paper_examples():
    g = load_golden("segment_helpers.txt")
    shape = np.array(_ints(g["shape"]))
    xs = np.array(_ints(g["xs"]))
    assert O.mk_sgm_descr(shape, xs).tolist() == _ints(g["mkSgmDescr"])
    assert O.mk_ii(shape).tolist() == _ints(g["mkII"])
    # sgmSum on the printed intermediate arrays gives the printed II.
    sct = np.array(_ints(g["mkII.sct_vs"]))
    flags = np.array(_bools(g["mkII.flags"]), dtype=np.uint8)
    assert O.sgm_sum(flags, sct).tolist() == _ints(g["mkII"])


# ------------------------------------------------------- brute force / lib ---

def _stable_reference(n, c):
    """Stable partition by Python's (stable) sort on the key 'not c'."""
    order = sorted(range(n), key=lambda i: not c[i])
    idx = [0] * n
    for pos, i in enumerate(order):
        idx[i] = pos
    return order, idx


@pytest.mark.parametrize("n", range(0, 15))
def test_partition2_all_flag_patterns(n):
    xs = np.arange(100, 100 + n, dtype=np.int32)
    for bits in itertools.product([0, 1], repeat=n):
        c = np.array(bits, dtype=np.uint8)
        ys, idx, t = O.partition2(xs, O.Pred.from_flags(c))
        order, ref_idx = _stable_reference(n, bits)
        assert t == sum(bits)
        assert idx.tolist() == ref_idx
        assert ys.tolist() == [int(xs[i]) for i in order]
        # filter: kept elements in order, dropped get -1
        fy, fidx, ft = O.partition2(xs, O.Pred.from_flags(c), O.MODE_FILTER)
        assert ft == sum(bits)
        assert fy.tolist() == [int(xs[i]) for i in range(n) if bits[i]]
        assert fidx.tolist() == [ref_idx[i] if bits[i] else -1 for i in range(n)]


def test_partition2_closed_form_index_function():
    """Section 2.3: indices[i] = -1 + sum_{j<=i} cs[j] if cs[i], else
    i + sum_{j>i} cs[j]; evaluated by an independent quadratic loop."""
    g = np.random.default_rng(7)
    for n in (1, 2, 17, 300):
        keys = g.integers(-1000, 1000, n).astype(np.int32)
        p = O.Pred.mod_eq(3, 1)
        cs = [((int(k) % 3) == 1) for k in keys]   # Python % is floor-mod
        _, idx, _ = O.partition2(keys, p)
        for i in range(n):
            if cs[i]:
                expect = -1 + sum(1 for j in range(i + 1) if cs[j])
            else:
                expect = i + sum(1 for j in range(i + 1, n) if cs[j])
            assert idx[i] == expect


def test_partition2_invariants_large():
    keys = W.int_keys(200_003, 11)
    ys, idx, t = O.partition2(keys, O.Pred.mod_eq(2, 0))
    c = keys % 2 == 0
    assert t == int(c.sum())
    assert (np.sort(idx) == np.arange(len(keys))).all()          # Bij onto [0,n)
    assert ((idx < t) == c).all()                                # trues first
    assert (np.diff(idx[c]) > 0).all() and (np.diff(idx[~c]) > 0).all()  # stable
    assert (ys[idx] == keys).all()
    # numpy's stable argsort on the class key reproduces the output
    order = np.argsort(~c, kind="stable")
    assert (ys == keys[order]).all()


def test_predicates_against_python_and_numpy():
    keys = np.array([-7, -6, -1, 0, 1, 5, 2**31 - 1, -2**31], dtype=np.int32)
    for d, r in [(2, 0), (3, 1), (3, 2), (7, 6), (1, 0)]:
        cs = O.map_pred(keys, O.Pred.mod_eq(d, r))
        assert cs.tolist() == [int(k) % d == r for k in keys]
    k64 = np.array([-(2**62), 2**62 + 3, -5], dtype=np.int64)
    assert O.map_pred(k64, O.Pred.mod_eq(5, 0)).tolist() == [int(k) % 5 == 0 for k in k64]
    f = np.array([0.0, -0.0, 0.5, 0.49999997, np.nan, -np.inf, np.inf, 1e-40],
                 dtype=np.float32)
    for s in (0.5, 0.0, 1e-40):
        assert (O.map_pred(f, O.Pred.lt(s)) == (f < np.float32(s))).all()


def test_filter_mode_matches_numpy_compress():
    x = W.f32_uniform(100_000, 12)
    for s in W.FLAT_LARGE_SELECTIVITIES:
        ys, idx, t = O.partition2(x, O.Pred.lt(s), O.MODE_FILTER)
        c = x < np.float32(s)
        assert t == int(c.sum())
        assert (ys == x[c]).all()
        assert (idx[c] == np.arange(t)).all() and (idx[~c] == -1).all()


# --------------------------------------------------------------- segmented ---

def _segments(shape):
    off = np.concatenate([[0], np.cumsum(shape)]).astype(np.int64)
    return off


def test_partition2L_closed_form():
    """Section 6: for row k with offset o_k, a true at i goes to
    o_k + #trues in [o_k, i), a false to i + #trues in (i, o_k + s_k)."""
    g = np.random.default_rng(5)
    shape = np.array([0, 3, 1, 0, 0, 7, 2, 0, 12, 1], dtype=np.int64)
    n = int(shape.sum())
    keys = g.integers(0, 100, n).astype(np.int32)
    _, idx, seg, _ = O.partition2L(keys, shape, O.Pred.mod_eq(3, 0))
    off = _segments(shape)
    cs = [int(k) % 3 == 0 for k in keys]
    for k in range(len(shape)):
        lo, hi = off[k], off[k + 1]
        assert seg[k] == sum(cs[lo:hi])
        for i in range(lo, hi):
            if cs[i]:
                expect = lo + sum(cs[lo:i])
            else:
                expect = i + sum(cs[i + 1:hi])
            assert idx[i] == expect


def test_partition2L_rowwise_stable_sort_and_descriptor():
    shape = W.segment_sizes(300, 3, median_log2=6, sigma_log2=1.5, empty_frac=0.2)
    n = int(shape.sum())
    keys = W.int_keys(n, 30)
    ys, idx, seg, flags = O.partition2L(keys, shape, O.Pred.mod_eq(3, 0))
    off = _segments(shape)
    c = keys % 3 == 0
    for k in range(len(shape)):
        lo, hi = off[k], off[k + 1]
        order = lo + np.argsort(~c[lo:hi], kind="stable")
        assert (ys[lo:hi] == keys[order]).all()
        assert seg[k] == int(c[lo:hi].sum())
    # flag array: 1 exactly at the starts of the non-empty rows
    expect = np.zeros(n, dtype=np.uint8)
    expect[off[:-1][shape > 0]] = 1
    assert (flags == expect).all()
    # the segment number of every element, by numpy searchsorted
    ii = np.searchsorted(off, np.arange(n), side="right") - 1
    assert (O.mk_ii(shape) == ii).all()


def test_partition2L_single_row_is_flat_and_filter_seg():
    keys = W.int_keys(5000, 31)
    p = O.Pred.mod_eq(3, 0)
    ys, idx, seg, flags = O.partition2L(keys, np.array([5000]), p)
    fys, fidx, ft = O.partition2(keys, p)
    assert (ys == fys).all() and (idx == fidx).all() and seg[0] == ft
    # filter_seg: kept elements of every row, packed row after row
    shape = np.array([10, 0, 4990], dtype=np.int64)
    ys, idx, seg, _ = O.partition2L(keys, shape, p, O.MODE_FILTER)
    c = keys % 3 == 0
    assert (ys == keys[c]).all()
    assert (idx[c] == np.arange(int(c.sum()))).all() and (idx[~c] == -1).all()
    assert seg.tolist() == [int(c[:10].sum()), 0, int(c[10:].sum())]


def test_partition2L_rejects_bad_shapes():
    keys = np.zeros(4, np.int32)
    with pytest.raises(ValueError):
        O.partition2L(keys, np.array([2, -1, 3]), O.Pred.mod_eq(2, 0))
    with pytest.raises(ValueError):
        O.partition2L(keys, np.array([2, 1]), O.Pred.mod_eq(2, 0))


def test_sgm_sum_brute_force():
    g = np.random.default_rng(9)
    for n in (0, 1, 5, 64, 257):
        flags = (g.random(n) < 0.2).astype(np.uint8)
        xs = g.integers(-50, 50, n)
        out = O.sgm_sum(flags, xs)
        for i in range(n):
            start = max([j for j in range(i + 1) if flags[j]], default=0)
            assert out[i] == int(xs[start:i + 1].sum())


# ---------------------------------------------------------- scatter/gather ---

def test_scatter_gather_match_numpy():
    g = np.random.default_rng(3)
    n = 1000
    perm = g.permutation(n)
    idx = perm.copy()
    idx[::7] = -3          # out of bounds, ignored
    idx[1::11] = n + 5     # out of bounds, ignored
    vals = g.standard_normal((n, 16)).astype(np.float32)
    dst = np.zeros((n, 16), np.float32)
    out = O.scatter(dst, idx, vals)
    ref = dst.copy()
    ok = (idx >= 0) & (idx < n)
    ref[idx[ok]] = vals[ok]
    assert (out.view(np.uint32) == ref.view(np.uint32)).all()
    back = O.gather(out, perm)
    assert (back == out[perm]).all()
    with pytest.raises(ValueError):
        O.gather(out, np.array([0, n]))


# -------------------------------------------------------------- properties ---

def _brute_inj(X, lo, hi):
    for i in range(len(X)):
        if lo <= X[i] < hi and any(X[j] == X[i] for j in range(i)):
            return (0, i, int(X[i]))
    return (1, -1, 0)


def test_checkers_brute_force_small():
    g = np.random.default_rng(21)
    for trial in range(300):
        n = int(g.integers(0, 40))
        X = g.integers(-3, 12, n).astype(np.int64)
        lo, hi = sorted(g.integers(-4, 14, 2).tolist())
        # Range
        bad = [i for i in range(n) if not (lo <= X[i] < hi)]
        assert O.check_range(X, lo, hi) == ((0, bad[0], int(X[bad[0]])) if bad else (1, -1, 0))
        # Monotonic, all pairs
        for op, f in enumerate([lambda a, b: a <= b, lambda a, b: a < b,
                                lambda a, b: a >= b, lambda a, b: a > b]):
            fails = [j for j in range(n) if any(not f(X[i], X[j]) for i in range(j))]
            assert O.check_mono(X, op) == ((0, fails[0], 0) if fails else (1, -1, 0))
        # Inj
        assert O.check_inj(X, lo, hi) == _brute_inj(X, lo, hi)
        # Bij with Img inside Rcd
        ilo = int(g.integers(lo, hi + 1))
        ihi = int(g.integers(ilo, hi + 1))
        inr = [i for i in range(n) if lo <= X[i] < hi]
        exp = (1, -1, 0)
        for i in inr:
            if any(X[j] == X[i] for j in inr if j < i) or not (ilo <= X[i] < ihi):
                exp = (0, i, int(X[i]))
                break
        if exp[0] == 1 and len(inr) != ihi - ilo:
            present = set(int(X[i]) for i in inr)
            exp = (0, n, min(v for v in range(ilo, ihi) if v not in present))
        assert O.check_bij(X, lo, hi, ilo, ihi) == exp


def test_bij_permutation_matches_library_and_planted_faults():
    n = 1 << 16
    perm = W.permutation(n, 50)
    assert O.check_bij(perm, 0, n, 0, n) == (1, -1, 0)
    assert O.check_inj(perm, 0, n) == (1, -1, 0)
    assert O.check_range(perm, 0, n) == (1, -1, 0)
    # a duplicate planted at p copying the entry at s: first violation max(p, s)
    for p, s in [(10, 5000), (6000, 3), (n - 1, 0)]:
        y = perm.copy()
        y[p] = perm[s]
        assert O.check_inj(y, 0, n) == (0, max(p, s), int(perm[s]))
        assert O.check_bij(y, 0, n, 0, n) == (0, max(p, s), int(perm[s]))
        assert O.check_range(y, 0, n)[0] == 1
    # an out-of-range entry: Range fails there, Inj ignores it, Bij misses a value
    y = perm.copy()
    y[123] = n + 7
    assert O.check_range(y, 0, n) == (0, 123, n + 7)
    assert O.check_inj(y, 0, n) == (1, -1, 0)
    assert O.check_bij(y, 0, n, 0, n) == (0, n, int(perm[123]))
    y[77] = -1
    assert O.check_range(y, 0, n) == (0, 77, -1)


def test_mono_sorted_and_swaps():
    x = W.sorted_keys(1 << 16, 51)
    assert O.check_mono(x, O.MONO_LE) == (1, -1, 0)
    y = W.adjacent_swaps(x, 3, 61)
    bad = np.nonzero(np.diff(y) < 0)[0]
    assert O.check_mono(y, O.MONO_LE) == (0, int(bad[0]) + 1, 0)
    assert O.check_mono(x[::-1].copy(), O.MONO_GE) == (1, -1, 0)


def test_filtpart_holds_on_outputs_and_planted_faults():
    keys = W.int_keys(4096, 70)
    p = O.Pred.mod_eq(2, 0)
    ys, idx, t = O.partition2(keys, p)
    assert O.check_filtpart(keys, p, O.MODE_PARTITION, ys, idx, t) == (1, -1, 0)
    # wrong split only
    v = O.check_filtpart(keys, p, O.MODE_PARTITION, ys, idx, t + 1)
    assert v[0] == 0 and v[2] & 1
    # swapping the destinations of the 10th and 20th trues: the true right
    # after the 10th now has a smaller destination, the first stability break
    tr = np.nonzero(keys % 2 == 0)[0]
    z = idx.copy()
    a, b = tr[10], tr[20]
    z[a], z[b] = z[b], z[a]
    y2 = O.scatter(np.zeros_like(ys), z, keys)
    v = O.check_filtpart(keys, p, O.MODE_PARTITION, y2, z, t)
    assert v == (0, int(tr[11]), 8)
    # a duplicated destination: Bij fails at the later copy
    z = idx.copy()
    z[500] = z[100]
    v = O.check_filtpart(keys, p, O.MODE_PARTITION, ys, z, t)
    assert v[0] == 0 and v[1] == 500 and v[2] & 2
    # a corrupted output value
    y3 = ys.copy()
    y3[idx[999]] ^= 1
    assert O.check_filtpart(keys, p, O.MODE_PARTITION, y3, idx, t) == (0, 999, 16)
    # filter mode
    fy, fidx, ft = O.partition2(keys, p, O.MODE_FILTER)
    assert O.check_filtpart(keys, p, O.MODE_FILTER, fy, fidx, ft) == (1, -1, 0)
    z = fidx.copy()
    drop = np.nonzero(keys % 2 != 0)[0][3]
    z[drop] = 0
    v = O.check_filtpart(keys, p, O.MODE_FILTER, fy, z, ft)
    assert v[0] == 0 and v[2] & 2


# ------------------------------------------- reduce-by-index, checked scatter ---

def test_hist_min_matches_numpy_minimum_at():
    """hist min against numpy's unbuffered reduce-by-index (ufunc.at), with
    out-of-bounds and negative indices dropped as the definition says."""
    g = np.random.default_rng(90)
    for n_dst, m in [(0, 5), (1, 0), (7, 40), (1000, 5000), (5000, 1000)]:
        idx = g.integers(-3, n_dst + 3, m)
        vals = g.integers(-10**12, 10**12, m)
        neutral = 2**62
        ref = np.full(n_dst, neutral, dtype=np.int64)
        keep = (idx >= 0) & (idx < n_dst)
        np.minimum.at(ref, idx[keep], vals[keep])
        assert np.array_equal(O.hist_min(n_dst, neutral, idx, vals), ref)
        # iota values: the least writer of each location
        ref = np.full(n_dst, m, dtype=np.int64)
        np.minimum.at(ref, idx[keep], np.arange(m)[keep])
        assert np.array_equal(O.hist_min(n_dst, m, idx), ref)


def test_scatter_checked_injective_equals_scatter():
    """With injective indices the verified scatter is the plain scatter into
    zeros and the verdict holds; out-of-bounds writes are dropped."""
    g = np.random.default_rng(91)
    n = 10_000
    idx = g.permutation(n)
    idx[::37] = -1
    idx[5::41] = n + 2
    vals = W.f32_normal(n, 92)
    dst, v = O.scatter_checked(n, idx, vals)
    assert v == (1, -1, 0)
    assert np.array_equal(dst.view(np.uint32), O.scatter(np.zeros(n, np.float32), idx, vals).view(np.uint32))


def test_scatter_checked_planted_repeats():
    """A repeated location: the verdict fails at the planted second write,
    agrees with the Inj checker over [0, n), and the least writer's value is
    the one stored."""
    g = np.random.default_rng(93)
    n = 5_000
    idx = g.permutation(n)
    p, s = 4_000, 1_234          # position p copies the index of s < p
    idx[p] = idx[s]
    vals = np.arange(n, dtype=np.int64) * 3 + 1
    dst, v = O.scatter_checked(n, idx, vals)
    assert v == (0, p, int(idx[s]))
    assert v == O.check_inj(idx, 0, n)
    assert dst[idx[s]] == vals[s]
    # the location that lost its writer stays zero
    lost = int(np.setdiff1d(np.arange(n), idx)[0])
    assert dst[lost] == 0
    # brute force on a tiny case: every location gets the least writer
    for trial in range(50):
        m = int(g.integers(0, 12))
        k = int(g.integers(1, 8))
        idx = g.integers(-1, k + 1, m)
        vals = g.integers(1, 100, m)
        dst, v = O.scatter_checked(k, idx, vals)
        for loc in range(k):
            writers = [i for i in range(m) if idx[i] == loc]
            assert dst[loc] == (vals[min(writers)] if writers else 0)
        bad = [i for i in range(m) if 0 <= idx[i] < k and any(idx[j] == idx[i] for j in range(i))]
        assert v == ((0, bad[0], int(idx[bad[0]])) if bad else (1, -1, 0))


def test_get_smallest_pairs_against_groupby_min():
    """The kept pairs are, per endpoint, the least edge id (pandas group-by
    minimum), listed in input order; both outputs are injective."""
    import pandas as pd
    g = np.random.default_rng(95)
    for n_verts, m in [(1, 10), (50, 40), (1000, 20_000), (100_000, 50_000)]:
        es = g.integers(0, n_verts, m)
        is_ = g.permutation(4 * m)[:m]            # injective edge ids
        eo, io = O.get_smallest_pairs(n_verts, 4 * m, es, is_)
        mins = pd.DataFrame({"e": es, "i": is_}).groupby("e")["i"].min()
        keep = is_ == mins.reindex(es).to_numpy()
        assert np.array_equal(eo, es[keep]) and np.array_equal(io, is_[keep])
        assert len(eo) == len(mins) == len(np.unique(eo))
        assert O.check_inj(eo, 0, n_verts)[0] == 1 and O.check_inj(io, 0, 4 * m)[0] == 1
    # endpoints outside [0, n_verts) are never kept; no edges, no pairs
    eo, io = O.get_smallest_pairs(3, 10, np.array([5, -1, 2]), np.array([0, 1, 2]))
    assert eo.tolist() == [2] and io.tolist() == [2]
    eo, io = O.get_smallest_pairs(3, 10, np.zeros(0, np.int64), np.zeros(0, np.int64))
    assert len(eo) == 0


# ------------------------------------------------------------ v-way partition ---

def _classes_ref(kind, v, xs=None, s=None, cls=None):
    if kind == O.CLASS_MOD:
        return np.mod(xs.astype(np.int64), v)
    if kind == O.CLASS_THRESH:
        c = np.full(len(xs), v - 1)
        for h in reversed(range(v - 1)):
            lo = -np.inf if h == 0 else s[h - 1]
            c = np.where((xs >= lo) & (xs < s[h]), h, c)
        return c
    return np.minimum(cls, v - 1)


def test_partition_v_is_stable_sort_by_class():
    """The v-way partition is the stable sort by class (numpy argsort with a
    stable kind, Python's sorted on tiny inputs); counts are bincount."""
    g = np.random.default_rng(96)
    for v in (2, 3, 4):
        for n in (0, 1, 17, 10_000):
            xs = W.int_keys(n, 97 + n).astype(np.int32) - (1 << 30)
            xf = g.random(n, dtype=np.float32)
            xf[::13] = np.nan
            s = np.sort(g.random(3)).astype(np.float32)
            cls = g.integers(0, 6, n).astype(np.uint8)
            for kind, x in ((O.CLASS_MOD, xs), (O.CLASS_THRESH, xf), (O.CLASS_BYTES, xs)):
                c = _classes_ref(kind, v, x, s, cls)
                ys, idx, counts = O.partition_v(x, v, kind, tuple(s), cls)
                order = np.argsort(c, kind="stable")
                assert np.array_equal(ys.view(np.uint32), x[order].view(np.uint32))
                inv = np.empty(n, dtype=np.int64)
                inv[order] = np.arange(n)
                assert np.array_equal(idx, inv)
                assert np.array_equal(counts, np.bincount(c, minlength=v)[:v])
                if n <= 17:
                    assert list(order) == sorted(range(n), key=lambda i: c[i])


def test_partition_v_two_classes_is_partition2():
    xs = W.int_keys(5000, 98)
    ys, idx, counts = O.partition_v(xs, 2, O.CLASS_MOD)
    ys2, idx2, t = O.partition2(xs, O.Pred.mod_eq(2, 0))
    assert np.array_equal(ys, ys2) and np.array_equal(idx, idx2) and counts[0] == t
    xf = W.f32_uniform(5000, 99)
    ys, idx, counts = O.partition_v(xf, 2, O.CLASS_THRESH, (0.3,))
    ys2, idx2, t = O.partition2(xf, O.Pred.lt(0.3))
    assert np.array_equal(ys, ys2) and np.array_equal(idx, idx2) and counts[0] == t


def test_partition_v_rejects_unsorted_thresholds():
    with pytest.raises(ValueError):
        O.partition_v(np.zeros(4, np.float32), 3, O.CLASS_THRESH, (0.5, 0.2))


# --------------------------------------- predicates of the row number (partition2L) ---

def test_partition2L_row_predicates_against_numpy():
    """Each row partitioned by its own predicate: numpy stable argsort of the
    negated flags, row by row; equal thresholds reduce to partition2L."""
    g = np.random.default_rng(101)
    shape = W.segment_sizes(60, 102, median_log2=6, sigma_log2=1.5, empty_frac=0.2)
    n = int(shape.sum())
    xf = g.random(n, dtype=np.float32)
    s_rows = g.random(len(shape)).astype(np.float32)
    xi = W.int_keys(n, 103) - (1 << 30)
    off = np.concatenate([[0], np.cumsum(shape)])
    for mode in (O.MODE_PARTITION, O.MODE_FILTER):
        for kind, x in ((O.ROW_LT, xf), (O.ROW_MOD, xi)):
            ys, idx, seg, fl = O.partition2L_rows(x, shape, kind, 3, s_rows, mode)
            exp_idx = np.full(n, -1, dtype=np.int64)
            kept_before = 0
            exp_ys = []
            for k in range(len(shape)):
                row = x[off[k]:off[k + 1]]
                c = row < s_rows[k] if kind == O.ROW_LT else np.mod(row.astype(np.int64), 3) == k % 3
                order = np.argsort(~c, kind="stable")
                if mode == O.MODE_PARTITION:
                    exp_idx[off[k] + order] = off[k] + np.arange(len(row))
                    exp_ys.append(row[order])
                else:
                    kept = np.flatnonzero(c)
                    exp_idx[off[k] + kept] = kept_before + np.arange(len(kept))
                    exp_ys.append(row[kept])
                    kept_before += len(kept)
                assert seg[k] == c.sum()
            assert np.array_equal(idx, exp_idx)
            assert np.array_equal(ys.view(np.uint32), np.concatenate(exp_ys).view(np.uint32))
    same = np.full(len(shape), 0.4, dtype=np.float32)
    a = O.partition2L_rows(xf, shape, O.ROW_LT, s_rows=same)
    b = O.partition2L(xf, shape, O.Pred.lt(0.4))
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
