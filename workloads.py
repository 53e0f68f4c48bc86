"""Seeded synthetic inputs for the filter-partition path.

This module only draws random numbers (numpy ``Generator(PCG64(seed))``); it
holds none of the method's arithmetic.  The oracle and the HIP library are fed
the same arrays from here, and neither imports the other.

The shapes follow the workloads of the paper's evaluation (Section 6: arrays of
random floats of 50M-200M elements for partition2; jagged arrays with possibly
empty rows for partition2L).  No dataset is used anywhere: every array is drawn
here from a fixed seed.
"""
import numpy as np

# Workload definitions (sizes and seeds).
FLAT_SMALL_N = 1 << 20          # int32 keys uniform in [0, 2^31), key % 2 == 0
FLAT_SMALL_SEED = 1
FLAT_LARGE_N = 1 << 28          # f32 uniform in [0, 1), x < s
FLAT_LARGE_SEED = 2
FLAT_LARGE_SELECTIVITIES = (0.01, 0.5, 0.99)
SEG_M = 10_000                  # log-normal row sizes, median 2^12, sigma 1.5 (log2)
SEG_SIZES_SEED = 3
SEG_KEYS_SEED = 30
AUTOGRAD_N = 1 << 24            # int32 keys, payload f32 [n, 16] ~ N(0, 1)
AUTOGRAD_ROW = 16
AUTOGRAD_SEEDS = (40, 41, 42)   # keys, payload, upstream gradient
VERIFY_NS = (50_000_000, 100_000_000, 200_000_000)   # f32 uniform in [0, 1), x < 0.5
VERIFY_SEED = 20
VERIFY_S = 0.5
PAIRS_VERTS = 1 << 24           # get_smallest_pairs: endpoints uniform in [0, 2^24)
PAIRS_M = 1 << 26               # entries; ids are a permutation of [0, 2^26)
PAIRS_SEEDS = (21, 22)          # endpoints, ids
PROPS_N = 1 << 28               # int64 index arrays
PROPS_PERM_SEED = 50
PROPS_SORTED_SEED = 51


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def int_keys(n: int, seed: int, dtype=np.int32) -> np.ndarray:
    """Uniform integers in [0, 2^31)."""
    return rng(seed).integers(0, 1 << 31, size=n, dtype=dtype)


def f32_uniform(n: int, seed: int) -> np.ndarray:
    """Uniform f32 in [0, 1)."""
    return rng(seed).random(n, dtype=np.float32)


def segment_sizes(m: int, seed: int, median_log2: float = 12.0,
                  sigma_log2: float = 1.5, empty_frac: float = 0.0) -> np.ndarray:
    """Row sizes max(1, round(2^(median_log2 + sigma_log2 * z))), z ~ N(0,1).

    The spread is read in log2 units (a natural-log sigma of 1.5 would put the
    expected total near 1.26e8 for 10^4 rows, far from the stated ~6.7e7).  With
    ``empty_frac`` > 0 that fraction of rows (chosen by the same generator) is
    set to size 0, to exercise empty rows.
    """
    g = rng(seed)
    z = g.standard_normal(m)
    sizes = np.maximum(1, np.rint(np.exp2(median_log2 + sigma_log2 * z))).astype(np.int64)
    if empty_frac > 0:
        empty = g.random(m) < empty_frac
        sizes[empty] = 0
    return sizes


def f32_normal(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(shape, dtype=np.float32)


def permutation(n: int, seed: int) -> np.ndarray:
    return rng(seed).permutation(n).astype(np.int64)


def sorted_keys(n: int, seed: int, high: int = 1 << 40) -> np.ndarray:
    a = rng(seed).integers(0, high, size=n, dtype=np.int64)
    a.sort()
    return a


def inject_faults(x: np.ndarray, k: int, seed: int, kind: str = "mixed") -> np.ndarray:
    """Copy of ``x`` with ``k`` entries overwritten at distinct random positions.

    kind "dup": the entry becomes a copy of another (random) entry;
    kind "oob": the entry becomes a value in [n, 2n) or a negative value;
    kind "mixed": each fault is a dup or an oob with equal odds.
    """
    g = rng(seed)
    y = x.copy()
    n = len(x)
    pos = g.choice(n, size=k, replace=False)
    kinds = {"dup": np.zeros(k, bool), "oob": np.ones(k, bool)}.get(kind)
    if kinds is None:
        kinds = g.random(k) < 0.5
    src = g.integers(0, n, size=k)
    hi = g.integers(n, 2 * n, size=k)
    neg = -g.integers(1, n + 1, size=k)
    use_neg = g.random(k) < 0.5
    for j in range(k):
        if kinds[j]:
            y[pos[j]] = neg[j] if use_neg[j] else hi[j]
        else:
            s = int(src[j])
            if s == pos[j]:
                s = (s + 1) % n
            y[pos[j]] = x[s]
    return y


def adjacent_swaps(x: np.ndarray, k: int, seed: int) -> np.ndarray:
    """Copy of a sorted array with ``k`` swaps of unequal neighbours."""
    g = rng(seed)
    y = x.copy()
    n = len(x)
    done = 0
    while done < k:
        i = int(g.integers(0, n - 1))
        if y[i] != y[i + 1]:
            y[i], y[i + 1] = y[i + 1], y[i]
            done += 1
    return y


def graph_entries(n_verts: int, m: int, seeds=(21, 22)):
    """Edge entries of a random graph: endpoints uniform in [0, n_verts)
    (Poisson degrees) and injective ids, a random permutation of [0, m)."""
    e = np.random.Generator(np.random.PCG64(seeds[0])).integers(0, n_verts, m, dtype=np.int64)
    i = np.random.Generator(np.random.PCG64(seeds[1])).permutation(m).astype(np.int64)
    return e, i
