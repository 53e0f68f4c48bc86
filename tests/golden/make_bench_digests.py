#!/usr/bin/env python3
"""Writes ``tests/golden/bench_digests.json``: SHA-256 digests of the oracle's
outputs on every workload that ``bench.py`` times, and the oracle's verdicts
on its property-checking arrays.

Only the oracle and the seeded input generators are called here.  The bench
hashes the device outputs of the launches it times and compares them with
these digests, so every timed configuration is also checked bit for bit
against the oracle at its full size, without the bench importing it.

Layout conventions (the same bytes the library writes):
  * keys as their own dtype, little-endian, n entries (filter: the first T);
  * indices as the width the bench requests (int32, or int64 for the small
    flat workload; filter writes -1 for every false);
  * split points, class sizes and per-row splits as int64.

Run:  python tests/golden/make_bench_digests.py   (about a minute, ~12 GiB RAM)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "bench_digests.json")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes()).hexdigest()


def verdict(v):
    return [int(v[0]), int(v[1]), int(v[2])]


def main():
    t0 = time.time()
    d = {"generator": "tests/golden/make_bench_digests.py", "hash": "sha256"}

    x = W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)
    flat, filt = {}, {}
    for s in W.FLAT_LARGE_SELECTIVITIES:
        ys, idx, t = O.partition2(x, O.Pred.lt(s))
        flat[str(s)] = {"keys": sha(ys), "idx_i32": sha(idx.astype(np.int32)), "split": int(t)}
        ys, idx, t = O.partition2(x, O.Pred.lt(s), O.MODE_FILTER)
        filt[str(s)] = {"keys": sha(ys), "idx_i32": sha(idx.astype(np.int32)), "split": int(t)}
        print(f"flat s={s} done ({time.time() - t0:.0f} s)", flush=True)
    d["flat_2e28_f32"] = flat
    d["filter_2e28_f32"] = filt
    ys, idx, cnt = O.partition_v(x, 3, O.CLASS_THRESH, (1 / 3, 2 / 3, 0.0))
    d["partition3_2e28_f32"] = {"keys": sha(ys), "idx_i32": sha(idx.astype(np.int32)),
                                "counts": [int(c) for c in cnt]}
    del x, ys, idx
    print(f"partition3 done ({time.time() - t0:.0f} s)", flush=True)

    ks = W.int_keys(W.FLAT_SMALL_N, W.FLAT_SMALL_SEED)
    ys, idx, t = O.partition2(ks, O.Pred.mod_eq(2, 0))
    d["flat_2e20_i32"] = {"keys": sha(ys), "idx_i64": sha(idx), "split": int(t)}

    shape = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
    keys = W.int_keys(int(shape.sum()), W.SEG_KEYS_SEED)
    ys, idx, seg, flags = O.partition2L(keys, shape, O.Pred.mod_eq(3, 0))
    d["segmented_1e4_rows"] = {"keys": sha(ys), "idx_i32": sha(idx.astype(np.int32)),
                               "seg_split": sha(seg), "flags": sha(flags)}
    del keys, ys, idx, seg, flags
    print(f"segmented done ({time.time() - t0:.0f} s)", flush=True)

    n, cols = W.AUTOGRAD_N, W.AUTOGRAD_ROW
    ak = W.int_keys(n, W.AUTOGRAD_SEEDS[0])
    _, idx, _ = O.partition2(ak, O.Pred.mod_eq(2, 0))
    p = W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[1])
    y = O.scatter(np.zeros_like(p), idx, p)
    del p
    gy = W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[2])
    gp = O.gather(gy, idx)
    d["fwd_bwd_2e24x16"] = {"y": sha(y), "grad_payload": sha(gp)}
    del y, gy, gp, idx
    print(f"fwd+bwd done ({time.time() - t0:.0f} s)", flush=True)

    ver = {}
    for nv in W.VERIFY_NS:
        xv = W.f32_uniform(nv, W.VERIFY_SEED)
        ys, _, t = O.partition2(xv, O.Pred.lt(W.VERIFY_S))
        ver[f"{nv // 1_000_000}M"] = {"keys": sha(ys), "split": int(t)}
    d["verify_partition2"] = ver
    del xv, ys
    print(f"verify done ({time.time() - t0:.0f} s)", flush=True)

    n = W.PROPS_N
    perm = W.permutation(n, W.PROPS_PERM_SEED)
    props = {"perm": {"range": verdict(O.check_range(perm, 0, n)),
                      "inj": verdict(O.check_inj(perm, 0, n)),
                      "bij": verdict(O.check_bij(perm, 0, n, 0, n))}}
    bad = W.inject_faults(perm, 1000, 1052, "mixed")
    del perm
    props["faulty_1000_mixed"] = {"range": verdict(O.check_range(bad, 0, n)),
                                  "mono": verdict(O.check_mono(bad, O.MONO_LE)),
                                  "inj": verdict(O.check_inj(bad, 0, n)),
                                  "bij": verdict(O.check_bij(bad, 0, n, 0, n))}
    del bad
    srt = W.sorted_keys(n, W.PROPS_SORTED_SEED)
    props["sorted"] = {"mono": verdict(O.check_mono(srt, O.MONO_LE))}
    d["check_props_2e28_i64"] = props
    print(f"props done ({time.time() - t0:.0f} s)", flush=True)

    with open(OUT, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
