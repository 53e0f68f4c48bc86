"""GPU property checkers against the CPU oracle: verdicts, first-violation
indices and aux values must be identical."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_2506_23058_amd as P  # noqa: E402

DEV = "cuda:0"
ALL4 = P.RANGE | P.MONO | P.INJ | P.BIJ


def oracle_verdicts(X, mask, lo, hi, ilo, ihi, op):
    X = np.asarray(X, dtype=np.int64)
    v = [(1, -1, 0)] * 5
    if mask & P.RANGE:
        v[0] = O.check_range(X, lo, hi)
    if mask & P.MONO:
        v[1] = O.check_mono(X, op)
    if mask & P.INJ:
        v[2] = O.check_inj(X, lo, hi)
    if mask & P.BIJ:
        v[3] = O.check_bij(X, lo, hi, ilo, ihi)
    return v


def both(X, mask=ALL4, lo=0, hi=None, ilo=None, ihi=None, op=P.MONO_LE, dtype=np.int64):
    X = np.asarray(X, dtype=dtype)
    n = len(X)
    hi = n if hi is None else hi
    ilo = lo if ilo is None else ilo
    ihi = hi if ihi is None else ihi
    print(f"[props] n={n} mask={mask} lo={lo} hi={hi} img=[{ilo},{ihi}) op={op} {X.dtype}", flush=True)
    g = P.verdicts(P.check_props(torch.from_numpy(X).to(DEV), mask, lo, hi, ilo, ihi, op))
    o = oracle_verdicts(X, mask, lo, hi, ilo, ihi, op)
    assert g[:4] == o[:4], (g, o)
    return g


def test_small_random_against_oracle():
    g = np.random.default_rng(123)
    for trial in range(60):
        n = int(g.integers(0, 3000))
        X = g.integers(-20, 600, n)
        lo, hi = sorted(g.integers(-30, 700, 2).tolist())
        ilo = int(g.integers(lo, hi + 1))
        ihi = int(g.integers(ilo, hi + 1))
        for dt in (np.int64, np.int32):
            both(X, ALL4, lo, hi, ilo, ihi, int(g.integers(0, 4)), dtype=dt)


def test_sorted_and_permutations_hold():
    n = (1 << 20) + 3
    perm = W.permutation(n, 50)
    v = both(perm)
    assert v[3] == (1, -1, 0) and v[2] == (1, -1, 0) and v[0] == (1, -1, 0)
    s = W.sorted_keys(n, 51)
    v = both(s, P.MONO, op=P.MONO_LE)
    assert v[1] == (1, -1, 0)
    both(s[::-1].copy(), P.MONO, op=P.MONO_GE)
    both(np.arange(n), P.MONO, op=P.MONO_LT)


@pytest.mark.parametrize("k", [1, 10, 100, 1000])
@pytest.mark.parametrize("kind", ["dup", "oob", "mixed"])
def test_planted_faults(k, kind):
    n = 1 << 20
    perm = W.permutation(n, 50)
    both(W.inject_faults(perm, k, 52 + k, kind))
    s = W.sorted_keys(n, 51)
    both(W.adjacent_swaps(s, k, 60 + k), P.MONO)


def test_bij_count_failure_reports_missing_value():
    n = 100_000
    perm = W.permutation(n, 3)
    x = perm.copy()
    x[777] = -5                     # out of Rcd: ignored by Inj, missing for Bij
    v = both(x)
    assert v[3] == (0, n, int(perm[777]))
    # Img strictly inside Rcd
    both(perm, P.BIJ, 0, n, 10, n - 10)
    both(np.arange(50), P.BIJ, 0, 100, 0, 100)
    # negative missing values (the least missing value is reduced as an
    # offset from img_lo), global-bitmap path and chunked path
    assert both(np.array([-3, -1, -4]), P.BIJ, -5, 0, -5, 0)[3] == (0, 3, -5)
    both(W.permutation(1 << 17, 4) - (1 << 17) - 2, P.BIJ, -(1 << 17) - 2, 0, -(1 << 17) - 2, 0)


def test_empty_and_tiny():
    for X in ([], [5], [3, 3], [1, 0], [0, 1, 2]):
        both(np.array(X, dtype=np.int64), ALL4, 0, 4, 0, 3)
        both(np.array(X, dtype=np.int64), ALL4, 0, 4, 0, 3, op=P.MONO_GT)


def test_values_repeated_many_times():
    """300 values each written to 4 more positions (5 occurrences each) of a
    permutation with a ragged length: the single rescan must still find the
    earliest second occurrence, whatever order the occurrences arrive in."""
    g = np.random.default_rng(7)
    for n in ((1 << 20) + 5, 3 * 32768 + 1):
        x = W.permutation(n, 8)
        src = g.choice(n, 300, replace=False)
        for s_ in src:
            x[g.choice(n, 4, replace=False)] = x[s_]
        both(x)
        both(x.astype(np.int32), dtype=np.int32)


@pytest.mark.parametrize("n,k", [(1 << 20, 5000), (50_000, 3000)])
def test_more_repeats_than_the_list_holds(n, k):
    """More than 2048 repeated values: the two global fallback passes locate
    the first violation (chunked path at 2^20, bitmap path below 2^16)."""
    perm = W.permutation(n, 9)
    both(W.inject_faults(perm, k, 99, "dup"))


def test_chunked_path_int32_and_offset_rcd():
    """Arrays of at least 2^16 take the chunked path: int32 elements, an Rcd
    with a negative base whose width is not a multiple of the 2^20-value
    bucket, Img strictly inside, and a chunk tail of n % 4 elements."""
    g = np.random.default_rng(11)
    n = 200_003
    x = g.integers(-100, 300_000, n)
    both(x, ALL4, -50, 290_000, -10, 280_000, P.MONO_LE, dtype=np.int32)
    lo = -12_345
    perm = W.permutation(3_000_001, 12)[:n] + lo
    both(perm, ALL4, lo, lo + 3_000_001, lo + 5, lo + 3_000_001)
    p2 = W.permutation(n, 13)
    both(p2, ALL4, -7, n + 1_000_000, -7, n + 1_000_000, dtype=np.int32)


def test_chunked_path_4096_buckets():
    """Rcd = [0, 2^32): 4096 buckets, values spread over all of them, a few
    planted repeats; Bij fails on the count and reports the least missing."""
    g = np.random.default_rng(14)
    n = 1 << 20
    x = g.choice(1 << 32, n, replace=False).astype(np.int64)
    both(x, P.RANGE | P.INJ | P.BIJ, 0, 1 << 32)
    x[g.choice(n, 10, replace=False)] = x[g.choice(n, 10, replace=False)]
    both(x, P.RANGE | P.INJ | P.BIJ, 0, 1 << 32)


@pytest.fixture(scope="module")
def perm_2e28():
    return W.permutation(W.PROPS_N, W.PROPS_PERM_SEED)


def test_config_props_full_size(perm_2e28):
    """int64 n = 2^28: a permutation (Bij) and a sorted array (Mono)."""
    v = both(perm_2e28)
    assert v[3][0] == 1
    s = W.sorted_keys(W.PROPS_N, W.PROPS_SORTED_SEED)
    assert both(s, P.MONO)[1][0] == 1
    both(W.adjacent_swaps(s, 10, 70), P.MONO)


@pytest.mark.parametrize("k", [1, 10, 100, 1000])
def test_config_props_full_size_faults(perm_2e28, k):
    """The 2^28 permutation with k planted duplicates / out-of-range values."""
    both(W.inject_faults(perm_2e28, k, 52 + k, "mixed"))


# ------------------------------------------------------------------ FiltPart

def _fp_both(keys, opred, gpred, mode, ys, z, split, idx_dtype=np.int64):
    kt = torch.from_numpy(keys).to(DEV)
    yfull = np.zeros(len(keys), keys.dtype)      # output keys have n entries
    yfull[: len(ys)] = ys
    yt = torch.from_numpy(yfull).to(DEV)
    zt = torch.from_numpy(np.asarray(z, dtype=idx_dtype)).to(DEV)
    st = torch.tensor([split], dtype=torch.int64, device=DEV)
    g = P.verdicts(P.check_props(zt, P.FILTPART, fp=P.FiltPartArgs(kt, yt, gpred, st, mode)))[4]
    full_y = np.zeros(len(keys), keys.dtype)
    full_y[: len(ys)] = ys
    o = O.check_filtpart(keys, opred, mode, full_y, np.asarray(z, dtype=np.int64), split)
    assert g == o, (g, o)
    return g


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("idx_dtype", [np.int64, np.int32])
def test_filtpart_on_partition_outputs_and_planted_faults(mode, idx_dtype):
    n = 300_007
    keys = W.int_keys(n, 90)
    op, gp = O.Pred.mod_eq(3, 1), P.Pred.mod_eq(3, 1)
    ys, idx, t = O.partition2(keys, op, mode)
    assert _fp_both(keys, op, gp, mode, ys, idx, t, idx_dtype) == (1, -1, 0)
    assert _fp_both(keys, op, gp, mode, ys, idx, t + 1, idx_dtype)[2] & 1
    c = keys % 3 == 1
    tr = np.nonzero(c)[0]
    fa = np.nonzero(~c)[0]
    # swap the destinations of two kept elements
    z = idx.copy()
    z[tr[100]], z[tr[5000]] = z[tr[5000]], z[tr[100]]
    _fp_both(keys, op, gp, mode, ys, z, t, idx_dtype)
    # duplicate destination
    z = idx.copy()
    z[tr[20000]] = z[tr[10]]
    _fp_both(keys, op, gp, mode, ys, z, t, idx_dtype)
    # out-of-range / negative destinations
    z = idx.copy()
    z[tr[3]] = n + 5
    z[fa[7]] = -9 if mode == 0 else 0
    _fp_both(keys, op, gp, mode, ys, z, t, idx_dtype)
    # corrupted output value
    y2 = ys.copy()
    y2[idx[tr[1234]]] ^= 8
    _fp_both(keys, op, gp, mode, y2, idx, t, idx_dtype)
    # class order broken in partition mode: a false sent before the split
    if mode == 0:
        z = idx.copy()
        z[fa[50]], z[tr[60]] = z[tr[60]], z[fa[50]]
        _fp_both(keys, op, gp, mode, ys, z, t, idx_dtype)


def test_filtpart_checks_gpu_partition_output():
    x = W.f32_uniform(5_000_000, 91)
    gp = P.Pred.lt(0.37)
    xt = torch.from_numpy(x).to(DEV)
    for mode in (0, 1):
        ok, oi, sp = P.partition(xt, gp, mode=mode, idx_dtype=torch.int32)
        v = P.verdicts(P.check_props(oi, P.FILTPART, fp=P.FiltPartArgs(xt, ok, gp, sp, mode)))
        assert v[4] == (1, -1, 0)


def test_bucketed_and_fallback_paths():
    """Arrays of 2^16 or more entries whose Rcd spans at most 4096 buckets of
    2^20 values take the bucketed Inj/Bij path; wider co-domains fall back to
    the global bitmap.  Both must give the oracle's verdicts."""
    g = np.random.default_rng(77)
    n = 200_003
    # int32 values, bucketed, with repeats and values outside Rcd
    x = g.integers(-1000, 3 * n, n).astype(np.int32)
    both(x, ALL4, 0, 3 * n, 5, 3 * n - 5, dtype=np.int32)
    # a permutation with its Rcd shifted: Img is a strict sub-range
    p = W.permutation(n, 78) + 10_000_000
    both(p, ALL4, 10_000_000, 10_000_000 + n, 10_000_000, 10_000_000 + n)
    both(p, P.INJ | P.BIJ, 9_000_000, 12_000_000, 10_000_000, 10_000_000 + n)
    # fewer than 2^16 entries: the global-bitmap path
    y = g.integers(0, 1 << 26, (1 << 16) - 1)
    y[500] = y[77]
    both(y, ALL4, 0, 1 << 26, 0, 1 << 26)
    # a co-domain of 2^33 values spans more than 4096 buckets: global bitmap
    y = g.integers(0, 1 << 33, 1 << 16)
    y[900] = y[800]
    both(y, P.INJ | P.RANGE, 0, 1 << 33)
    # more than 2^22 entries per 2^20-value bucket on average: global bitmap
    w = g.integers(0, 1 << 20, (1 << 23) + 5)
    both(w, ALL4, 0, 1 << 20, 0, 1 << 20)
    # a bucket boundary: values just around multiples of 2^20
    z = (np.arange(n) // 7) * (1 << 20) + (np.arange(n) % 7) - 3
    both(z, P.INJ | P.RANGE, -3, int(z.max()) + 1)
