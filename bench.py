#!/usr/bin/env python3
"""Throughput of the filter-partition hot path on one MI355X.

Headline workload: stable partition (partition2) of n = 2^28 f32 values drawn
uniform in [0,1), predicate x < s, for the three selectivities
s in {0.01, 0.5, 0.99}, writing int32 positions, the partitioned values and the
split point.  One step = one partition per selectivity (3 * 2^28 elements),
inputs resident in HBM.  value = partitioned elements per second over the timed
steps (GElem/s).

The JSON line also carries
  roofline      -- the dominant kernel (the scan-scatter kernel) against the
                   8 TB/s HBM peak: algorithmic bytes per launch / its average
                   duration, timed with HIP events on its own stream during the
                   timed steps;
  cpu_baseline  -- the sequential C oracle timed on a bounded sample of the
                   same workload, on the host;
  sections      -- the other workloads (filter mode, small flat, segmented,
                   fwd+bwd, property checks), each timed on its own.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


# Sources each profiled kernel is compiled from: a counter reading in
# profiles/counters.json stays valid while the hash of these is unchanged.
KERNEL_SOURCES = {
    "flat_count": ("flat.hip", "device.hpp", "host.hpp"),
    "flat_scatter_partition": ("flat.hip", "device.hpp", "host.hpp"),
    "flat_scan_filter": ("flat.hip", "device.hpp", "host.hpp"),
    "seg_main_partition": ("segmented.hip", "device.hpp", "host.hpp"),
    "scatter_rows": ("rows.hip", "device.hpp", "host.hpp"),
    "gather_rows": ("rows.hip", "device.hpp", "host.hpp"),
    "props_scan": ("props.hip", "device.hpp", "host.hpp"),
    "props_check": ("props.hip", "device.hpp", "host.hpp"),
    "props_rescan": ("props.hip", "device.hpp", "host.hpp"),
}

DIGESTS = os.path.join(ROOT, "tests", "golden", "bench_digests.json")


def sources_hash(files):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2506_23058_amd", "csrc")
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, elements: int):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated
    against a plain copy) from the committed rocprofv3 counter summary, or
    None when it is absent, taken on another workload, or the kernel's
    sources changed since."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as f:
        c = json.load(f)
    k = c.get("kernels", {}).get(kernel)
    if not k or k.get("elements") != elements:
        return None
    if k.get("sources_hash") != sources_hash(KERNEL_SOURCES[kernel]):
        return None
    return k.get("hbm_bytes_per_launch")


def _golden():
    with open(DIGESTS) as f:
        return json.load(f)


def _sha(t) -> str:
    """SHA-256 of a tensor's bytes (copied to the host)."""
    import numpy as np
    a = t.detach().contiguous().cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(a).reshape(-1).view(np.uint8)).hexdigest()


def _verify(what: str, got: dict, want: dict):
    """Every field of `got` must equal the oracle's stored value."""
    bad = {k: (v, want.get(k)) for k, v in got.items() if want.get(k) != v}
    if bad:
        raise AssertionError(f"{what}: device outputs differ from the oracle's: {sorted(bad)}")
    return True


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sections", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="headline steps only (for profiler runs)")
    ap.add_argument("--with-copy", action="store_true",
                    help="also run one plain device copy of the input (counter calibration)")
    ap.add_argument("--profile", default=None,
                    choices=["flat", "filter", "flat_small", "segmented", "fwd_bwd", "props", "props_faulty"],
                    help="run only this workload's launches, once untimed and --steps times, "
                         "for rocprofv3 kernel traces and counters; prints one line")
    ap.add_argument("--section", default=None,
                    help="run only this section (segmented, autograd, props, verify, pairs, "
                         "partition3, shape_tools) and print it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path is single-device; see the sharding notes in DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_23058_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    if args.profile:
        profile_run(args, torch, np, P, W, dev)
        return
    if args.section:
        fn = {"segmented": section_segmented, "autograd": section_autograd,
              "props": section_props, "verify": section_verify, "pairs": section_pairs,
              "partition3": section_partition3, "shape_tools": section_shape_tools}[args.section]
        print(json.dumps({args.section: fn(args, torch, np, P, W, dev)}))
        return
    n = W.FLAT_LARGE_N
    sels = W.FLAT_LARGE_SELECTIVITIES
    x = torch.from_numpy(W.f32_uniform(n, W.FLAT_LARGE_SEED)).to(dev)
    out_keys = torch.empty_like(x)
    out_idx = torch.empty(n, dtype=torch.int32, device=dev)
    split = torch.empty(1, dtype=torch.int64, device=dev)
    preds = [P.Pred.lt(s) for s in sels]

    def step():
        for p in preds:
            P.partition(x, p, P.MODE_PARTITION, torch.int32, out_keys=out_keys,
                        out_idx=out_idx, split=split)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    P.profile_read()
    P.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    P.profile_enable(False)
    prof = P.profile_read()

    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in prof.items()}
    scan = kern.get("flat_scatter_partition", {"avg_ms": float("nan")})
    count = kern.get("flat_count", {"avg_ms": float("nan")})
    scan_alg = n * (4 + 4 + 4)            # read keys, write idx, write keys
    count_alg = n * 4                     # read keys
    achieved = scan_alg / (scan["avg_ms"] * 1e-3) / 1e9
    for k, alg in (("flat_scatter_partition", scan_alg), ("flat_count", count_alg)):
        if k in kern:
            kern[k]["alg_bytes_per_launch"] = alg
            kern[k]["alg_GBps"] = alg / (kern[k]["avg_ms"] * 1e-3) / 1e9
    traffic = _traffic("flat_scatter_partition", n)
    # whole partition: count + tile scan + scatter, per selectivity
    per_part_s = dt / len(sels)
    verified = None
    if not args.only_headline:
        # the outputs of the launch configuration timed above, once per
        # selectivity, against the oracle's digests
        gold = _golden()["flat_2e28_f32"]
        for s, p in zip(sels, preds):
            P.partition(x, p, P.MODE_PARTITION, torch.int32, out_keys=out_keys, out_idx=out_idx,
                        split=split)
            _verify(f"flat partition s={s}", {"keys": _sha(out_keys), "idx_i32": _sha(out_idx),
                                              "split": int(split.item())}, gold[str(s)])
        verified = True
    out = {
        "metric": "partitioned GElem/s + % HBM peak (flat, segmented, fwd+bwd) on 1 MI355X",
        "value": len(sels) * n / dt / 1e9,
        "unit": "GElem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "flat stable partition2, n=2^28 f32 uniform[0,1), x<s for "
                               "s in {0.01,0.5,0.99} (one partition each per step), int32 "
                               "positions + partitioned values + split",
                   "n": n, "selectivities": list(sels), "idx_dtype": "int32"},
        "roofline": {"bound": "hbm", "kernel": "flat_scatter_partition",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": scan_alg,
                     # the whole partition (count, tile scan and scatter) on
                     # its 12 algorithmic bytes per element
                     "frac_whole_op": scan_alg / per_part_s / 1e9 / HBM_PEAK_GBPS},
        # 12 B/element: read keys, write positions, write keys
        "whole_step_alg_GBps": len(sels) * scan_alg / dt / 1e9,
        # 16 B/element: the above plus the counting pass's re-read of the keys
        "whole_step_design_GBps": len(sels) * (scan_alg + count_alg) / dt / 1e9,
        "verified_against_oracle": verified,
        "kernels": kern,
    }

    if args.with_copy:
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del y
    if not args.only_headline and not args.no_sections:
        out["sections"] = sections(args, torch, np, P, W, dev, x, out_keys, out_idx, split)

    if not args.only_headline and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, np)
    print(json.dumps(out))


def _prof(P):
    return {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)} for k, v in P.profile_read().items()}


def sections(args, torch, np, P, W, dev, x, out_keys, out_idx, split):
    res = {}
    n = x.numel()
    steps = max(3, args.steps // 2)
    # copy kernel: achievable HBM bandwidth reference (read n*4 + write n*4)
    y = torch.empty_like(x)
    t = timed(lambda: y.copy_(x), steps, 2, torch)
    res["copy_reference"] = {"bytes": 2 * 4 * n, "ms": t * 1e3, "GBps": 8 * n / t / 1e9}
    del y
    # filter mode (single pass with decoupled look-back) on the same input
    gold = _golden()
    fl = {}
    for s in W.FLAT_LARGE_SELECTIVITIES:
        p = P.Pred.lt(s)
        P.profile_read()
        P.profile_enable(True)
        t = timed(lambda: P.partition(x, p, P.MODE_FILTER, torch.int32, out_keys=out_keys,
                                      out_idx=out_idx, split=split), steps, 2, torch)
        P.profile_enable(False)
        k = _prof(P).get("flat_scan_filter", {})
        T = int(split.item())
        alg = n * 4 + n * 4 + T * 4
        r = {"ms": t * 1e3, "GElem_s": n / t / 1e9, "alg_GBps": alg / t / 1e9,
             "frac_of_8TBps": alg / t / 8e12, "alg_bytes": alg}
        if k:
            r["kernel_avg_ms"] = k["avg_ms"]
            r["traffic"] = _traffic("flat_scan_filter", n) if s == 0.5 else None
        r["verified_against_oracle"] = _verify(
            f"filter s={s}", {"keys": _sha(out_keys[:T]), "idx_i32": _sha(out_idx), "split": T},
            gold["filter_2e28_f32"][str(s)])
        fl[str(s)] = r
    res["flat_filter_2^28_f32"] = fl
    # small flat config: n = 2^20 int32 keys, key % 2 == 0, int64 indices
    ks = torch.from_numpy(W.int_keys(W.FLAT_SMALL_N, W.FLAT_SMALL_SEED)).to(dev)
    p = P.Pred.mod_eq(2, 0)
    oks = torch.empty_like(ks)
    ois = torch.empty(ks.numel(), dtype=torch.int64, device=dev)
    t = timed(lambda: P.partition(ks, p, P.MODE_PARTITION, torch.int64, out_keys=oks,
                                  out_idx=ois, split=split), steps * 10, 5, torch)
    res["flat_partition_2^20_int32_int64idx"] = {
        "ms": t * 1e3, "GElem_s": ks.numel() / t / 1e9, "alg_GBps": ks.numel() * 16 / t / 1e9,
        "verified_against_oracle": _verify(
            "flat 2^20", {"keys": _sha(oks), "idx_i64": _sha(ois), "split": int(split.item())},
            gold["flat_2e20_i32"])}
    del ks, oks, ois
    res["segmented_10^4_rows"] = section_segmented(args, torch, np, P, W, dev)
    res["fwd_bwd_2^24x16"] = section_autograd(args, torch, np, P, W, dev)
    res["check_props_2^28_int64"] = section_props(args, torch, np, P, W, dev)
    res["scatter_verification_partition2"] = section_verify(args, torch, np, P, W, dev)
    res["get_smallest_pairs"] = section_pairs(args, torch, np, P, W, dev)
    res["partition3_2^28_f32"] = section_partition3(args, torch, np, P, W, dev, x)
    res["shape_tools"] = section_shape_tools(args, torch, np, P, W, dev)
    return res


def section_segmented(args, torch, np, P, W, dev):
    """10^4 rows, log-normal sizes (median 2^12, sigma 1.5 in log2), int32 keys,
    key % 3 == 0; int32 indices, int64 per-row splits, u8 descriptor."""
    shape_np = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
    n = int(shape_np.sum())
    keys = torch.from_numpy(W.int_keys(n, W.SEG_KEYS_SEED)).to(dev)
    shape = torch.from_numpy(shape_np).to(dev)
    pred = P.Pred.mod_eq(3, 0)
    tiling, tune_ms, cached = P.autotuned_tiling(keys, shape, pred)
    g = P.SegmentedGraph(keys, shape, pred, tune=tiling)
    steps = max(5, args.steps)
    t_graph = timed(g.launch, steps, 2, torch)
    t_eager = timed(lambda: P.segmented_partition(keys, shape, pred, tune=tiling,
                                                  out_keys=g.out_keys, out_idx=g.out_idx,
                                                  seg_split=g.seg_split, flags=g.flags),
                    steps, 2, torch)
    P.profile_enable(True)
    for _ in range(3):
        P.segmented_partition(keys, shape, pred, tune=tiling, out_keys=g.out_keys,
                              out_idx=g.out_idx, seg_split=g.seg_split, flags=g.flags)
    torch.cuda.synchronize()
    P.profile_enable(False)
    kern = _prof(P)
    # the plain per-call form: one flat partition per row (row-local indices,
    # no descriptor), 10^4 host calls on the same stream
    offs = np.concatenate([[0], np.cumsum(shape_np)])
    ok = torch.empty_like(keys)
    oi = torch.empty(n, dtype=torch.int32, device=dev)
    sp = torch.empty(W.SEG_M, dtype=torch.int64, device=dev)

    def per_call():
        for k in range(W.SEG_M):
            lo, hi = int(offs[k]), int(offs[k + 1])
            if hi > lo:
                P.partition(keys[lo:hi], pred, P.MODE_PARTITION, torch.int32,
                            out_keys=ok[lo:hi], out_idx=oi[lo:hi], split=sp[k:k + 1])
    t_calls = timed(per_call, 2, 1, torch)
    gold = _golden()["segmented_1e4_rows"]

    def outputs(o):
        return {"keys": _sha(o.out_keys), "idx_i32": _sha(o.out_idx), "seg_split": _sha(o.seg_split),
                "flags": _sha(o.flags)}

    # the eager call above wrote the graph's buffers last: replay the graph
    # once more and check what it writes
    g.launch()
    torch.cuda.synchronize()
    ok_graph = _verify("segmented graph", outputs(g), gold)
    g.close()
    # the same tiling with the other way of learning T_k of multi-item rows
    row_sync = tiling[3] if len(tiling) > 3 else P._lib.ROW_SYNC_AUTO
    other = tuple(tiling[:3]) + (P._lib.ROW_SYNC_COUNT if row_sync != P._lib.ROW_SYNC_COUNT
                                 else P._lib.ROW_SYNC_WAIT,)
    g2 = P.SegmentedGraph(keys, shape, pred, tune=other)
    t_other = timed(g2.launch, steps, 2, torch)
    ok_other = _verify("segmented graph, other row sync", outputs(g2), gold)
    g2.close()
    alg = n * (4 + 4 + 4 + 1) + W.SEG_M * 16
    main = kern.get("seg_main_partition")
    if main:
        main["alg_bytes_per_launch"] = n * 13
        main["alg_GBps"] = n * 13 / (main["avg_ms"] * 1e-3) / 1e9
        main["traffic"] = _traffic("seg_main_partition", n)
    return {"n": n, "m": W.SEG_M, "tiling": {"block": tiling[0], "rows": tiling[1],
                                             "wgs_per_cu": tiling[2],
                                             "row_sync": ["auto", "count", "nowait", "wait"][row_sync]},
            "verified_against_oracle": ok_graph and ok_other,
            "graph_ms_other_row_sync": t_other * 1e3,
            "other_row_sync": ["auto", "count", "nowait", "wait"][other[3]],
            "tuner_ms": tune_ms, "tiling_from_cache": cached,
            "graph_ms": t_graph * 1e3, "graph_GElem_s": n / t_graph / 1e9,
            "graph_alg_GBps": alg / t_graph / 1e9, "graph_frac_of_8TBps": alg / t_graph / 8e12,
            "eager_ms": t_eager * 1e3, "per_call_10^4_ms": t_calls * 1e3,
            "speedup_vs_per_call": t_calls / t_graph, "alg_bytes": alg, "kernels": kern}


def section_autograd(args, torch, np, P, W, dev):
    """Differentiable partition: int32 keys n = 2^24, key % 2 == 0, payload f32
    [n, 16] ~ N(0,1); one step = forward (partition + row scatter) + backward
    (row gather)."""
    n, cols = W.AUTOGRAD_N, W.AUTOGRAD_ROW
    keys = torch.from_numpy(W.int_keys(n, W.AUTOGRAD_SEEDS[0])).to(dev)
    payload = torch.from_numpy(W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[1])).to(dev)
    gy = torch.from_numpy(W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[2])).to(dev)
    pred = P.Pred.mod_eq(2, 0)
    steps = max(5, args.steps)
    p = payload.clone().requires_grad_(True)

    def ours():
        p.grad = None
        y, _, _, _ = P.partition_scatter(keys, p, pred)
        y.backward(gy)

    t_ours = timed(ours, steps, 2, torch)
    P.profile_enable(True)
    for _ in range(3):
        ours()
    torch.cuda.synchronize()
    P.profile_enable(False)
    kern = _prof(P)
    ib = 4 if n < (1 << 31) else 8   # index width the differentiable partition uses
    for k in ("scatter_rows", "gather_rows"):
        if k in kern:
            kern[k]["alg_bytes_per_launch"] = n * (ib + 2 * cols * 4)
            kern[k]["alg_GBps"] = n * (ib + 2 * cols * 4) / (kern[k]["avg_ms"] * 1e-3) / 1e9
            kern[k]["traffic"] = _traffic(k, n)
    gold = _golden()["fwd_bwd_2e24x16"]
    p.grad = None
    y, _, _, _ = P.partition_scatter(keys, p, pred)
    y.backward(gy)
    verified = _verify("fwd+bwd", {"y": _sha(y), "grad_payload": _sha(p.grad)}, gold)
    del y

    def per_call():
        _, idx, _ = P.partition(keys, pred, P.MODE_PARTITION, torch.int64, want_keys=False)
        y = torch.empty_like(payload).index_copy_(0, idx, payload)
        gp = gy.index_select(0, idx)
        return y, gp

    t_plain = timed(per_call, steps, 2, torch)
    q = payload.clone().requires_grad_(True)
    ar = torch.arange(n, device=dev)

    def torch_autograd():
        q.grad = None
        _, idx, _ = P.partition(keys, pred, P.MODE_PARTITION, torch.int64, want_keys=False)
        inv = torch.empty_like(idx)
        inv[idx] = ar
        y = q.index_select(0, inv)
        y.backward(gy)

    t_ta = timed(torch_autograd, steps, 2, torch)
    row = cols * 4
    # partition (read keys, write indices and partitioned keys) + fwd + bwd
    alg = n * (4 + ib + 4) + n * (ib + row + row) + n * (ib + row + row)
    return {"n": n, "row_bytes": row, "verified_against_oracle": verified, "ours_ms": t_ours * 1e3, "ours_alg_GBps": alg / t_ours / 1e9,
            "ours_frac_of_8TBps": alg / t_ours / 8e12,
            "per_call_index_copy_select_ms": t_plain * 1e3,
            "torch_autograd_index_select_ms": t_ta * 1e3,
            "speedup_vs_per_call": t_plain / t_ours, "speedup_vs_torch_autograd": t_ta / t_ours,
            "alg_bytes": alg, "kernels": kern}


def section_props(args, torch, np, P, W, dev):
    """int64 n = 2^28: Range+Inj+Bij on a permutation, Mono on a sorted array,
    all four on the permutation with 1000 planted faults."""
    n = W.PROPS_N
    gold = _golden()["check_props_2e28_i64"]
    perm_np = W.permutation(n, W.PROPS_PERM_SEED)
    perm = torch.from_numpy(perm_np).to(dev)
    steps = max(3, args.steps // 2)
    out = {}

    def named(v, names):
        rows = P.verdicts(v)
        col = {"range": 0, "mono": 1, "inj": 2, "bij": 3}
        return {k: list(rows[col[k]]) for k in names}

    m3 = P.RANGE | P.INJ | P.BIJ
    t = timed(lambda: P.check_props(perm, m3, 0, n, 0, n), steps, 1, torch)
    v = named(P.check_props(perm, m3, 0, n, 0, n), ("range", "inj", "bij"))
    out["perm_range_inj_bij"] = {"ms": t * 1e3, "GElem_s": n / t / 1e9, "alg_GBps": 8 * n / t / 1e9,
                                 "frac_of_8TBps": 8 * n / t / 8e12, "verdicts": v,
                                 "verified_against_oracle": _verify("props perm", v, gold["perm"])}
    P.profile_enable(True)
    P.check_props(perm, m3, 0, n, 0, n)
    torch.cuda.synchronize()
    P.profile_enable(False)
    kern = _prof(P)
    for k in ("props_scan", "props_check"):
        if k in kern:
            kern[k]["traffic"] = _traffic(k, n)
    out["perm_kernels"] = kern
    bad = torch.from_numpy(W.inject_faults(perm_np, 1000, 1052, "mixed")).to(dev)
    del perm_np
    m4 = m3 | P.MONO
    t = timed(lambda: P.check_props(bad, m4, 0, n, 0, n), steps, 1, torch)
    v = named(P.check_props(bad, m4, 0, n, 0, n), ("range", "mono", "inj", "bij"))
    out["faulty_all4"] = {"ms": t * 1e3, "GElem_s": n / t / 1e9, "verdicts": v,
                          "verified_against_oracle": _verify("props faulty", v, gold["faulty_1000_mixed"])}
    P.profile_enable(True)
    P.check_props(bad, m4, 0, n, 0, n)
    torch.cuda.synchronize()
    P.profile_enable(False)
    fk = _prof(P)
    if "props_rescan" in fk:
        fk["props_rescan"]["traffic"] = _traffic("props_rescan", n)
    out["faulty_kernels"] = fk
    del bad, perm
    srt = torch.from_numpy(W.sorted_keys(n, W.PROPS_SORTED_SEED)).to(dev)
    t = timed(lambda: P.check_props(srt, P.MONO), steps, 1, torch)
    v = named(P.check_props(srt, P.MONO), ("mono",))
    out["sorted_mono"] = {"ms": t * 1e3, "GElem_s": n / t / 1e9, "alg_GBps": 8 * n / t / 1e9,
                          "verdicts": v, "verified_against_oracle": _verify("props sorted", v, gold["sorted"])}
    return out


# The paper's A100 times of partition2 (Section 6, table "tab:eval" right),
# milliseconds: other hardware, context only.
PAPER_A100_MS = {50_000_000: {"base": 12.357, "static": 2.814, "static_opt": 2.614},
                 100_000_000: {"base": 38.947, "static": 5.565, "static_opt": 5.145},
                 200_000_000: {"base": 135.742, "static": 11.097, "static_opt": 10.557}}


def section_verify(args, torch, np, P, W, dev):
    """partition2 of N random f32 (x < 0.5) with its scatter verified three
    ways: Base = the indices are materialised, then a dynamically checked
    scatter (zeroed output, reduce-by-index of atomic minima, check, winner
    writes); Static = zeroed output, then the fused partition that scatters
    without checks; Static+Opt = the fused partition alone (the output is not
    initialised: the index array is a bijection)."""
    res = {}
    steps = max(3, args.steps // 4)
    pred = P.Pred.lt(W.VERIFY_S)
    for n in W.VERIFY_NS:
        x = torch.from_numpy(W.f32_uniform(n, W.VERIFY_SEED)).to(dev)
        dst = torch.empty_like(x)
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        split = torch.empty(1, dtype=torch.int64, device=dev)
        verdict = torch.empty(3, dtype=torch.int64, device=dev)

        def static_opt():
            P.partition(x, pred, P.MODE_PARTITION, torch.int32, out_keys=dst, want_idx=False, split=split)

        def static():
            P.zero_(dst)
            static_opt()

        def base():
            P.partition(x, pred, P.MODE_PARTITION, torch.int32, want_keys=False, out_idx=idx, split=split)
            P.scatter_checked(n, idx, x, out=dst, verdict=verdict)

        base()
        torch.cuda.synchronize()
        ref = dst.clone()
        assert int(verdict[0].item()) == 1, "partition indices must verify as injective"
        r = {}
        for name, fn in (("base", base), ("static", static), ("static_opt", static_opt)):
            fn()
            torch.cuda.synchronize()
            assert torch.equal(dst, ref), f"{name} differs from the checked scatter"
            t = timed(fn, steps, 1, torch)
            r[name] = {"ms": t * 1e3, "GElem_s": n / t / 1e9}
        r["verified_against_oracle"] = _verify(
            f"verify {n}", {"keys": _sha(ref), "split": int(split.item())},
            _golden()["verify_partition2"][f"{n // 1_000_000}M"])
        r["speedup_static"] = r["base"]["ms"] / r["static"]["ms"]
        r["speedup_static_opt"] = r["base"]["ms"] / r["static_opt"]["ms"]
        r["paper_a100_ms"] = PAPER_A100_MS[n]
        res[f"{n // 1_000_000}M"] = r
        del x, dst, idx, ref
    P.profile_enable(True)
    n = W.VERIFY_NS[-1]
    x = torch.from_numpy(W.f32_uniform(n, W.VERIFY_SEED)).to(dev)
    dst = torch.empty_like(x)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    P.partition(x, pred, P.MODE_PARTITION, torch.int32, want_keys=False, out_idx=idx)
    P.scatter_checked(n, idx, x, out=dst)
    torch.cuda.synchronize()
    P.profile_enable(False)
    res["base_kernels_200M"] = _prof(P)
    return res


def section_pairs(args, torch, np, P, W, dev):
    """get_smallest_pairs on a random graph of 2^26 entries over 2^24 vertices:
    hist min, the keep flags, a filter of the flags and two 8-byte scatters,
    all enqueued without a host synchronisation; then Inj of both outputs
    with the device checker.  Compared with the same steps in plain torch
    (scatter_reduce amin, gather, boolean masks)."""
    n_verts, m = W.PAIRS_VERTS, W.PAIRS_M
    e, i = W.graph_entries(n_verts, m, W.PAIRS_SEEDS)
    es = torch.from_numpy(e).to(dev)
    is_ = torch.from_numpy(i).to(dev)
    sp = P.SmallestPairs(n_verts, m, es, is_)
    steps = max(3, args.steps // 2)
    t = timed(sp.run, steps, 2, torch)
    kept = int(sp.split.item())
    eo, io = sp.es_out[:kept], sp.is_out[:kept]

    def check():
        return (P.check_props(eo, P.INJ, lo=0, hi=n_verts), P.check_props(io, P.INJ, lo=0, hi=m))

    t_check = timed(check, steps, 1, torch)
    v1, v2 = (P.verdicts(v)[2] for v in check())

    def torch_ref():
        h = torch.full((n_verts,), m, dtype=torch.int64, device=dev)
        h.scatter_reduce_(0, es, is_, reduce="amin", include_self=True)
        keep = h[es] == is_
        return es[keep], is_[keep]

    re, ri = torch_ref()
    assert torch.equal(re, eo) and torch.equal(ri, io), "torch reference disagrees"
    t_torch = timed(torch_ref, steps, 1, torch)
    P.profile_enable(True)
    sp.run()
    torch.cuda.synchronize()
    P.profile_enable(False)
    return {"n_verts": n_verts, "entries": m, "kept": kept, "ms": t * 1e3, "G_entries_s": m / t / 1e9,
            "inj_check_ms": t_check * 1e3, "inj_es_out": v1, "inj_is_out": v2,
            "torch_ms": t_torch * 1e3, "speedup_vs_torch": t_torch / t, "kernels": _prof(P)}


def section_partition3(args, torch, np, P, W, dev, x=None):
    """3-way stable partition of the headline's 2^28 f32 input into
    x < 1/3, 1/3 <= x < 2/3 and the rest, int32 positions: 12 algorithmic
    bytes per element (16 with the counting pass), as partition2."""
    if x is None:
        x = torch.from_numpy(W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)).to(dev)
    n = x.numel()
    ok = torch.empty_like(x)
    oi = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(3, dtype=torch.int64, device=dev)
    cl = P.Classes.thresholds(1 / 3, 2 / 3)
    steps = max(3, args.steps // 2)
    t = timed(lambda: P.partition_v(x, cl, torch.int32, out_keys=ok, out_idx=oi, counts=cnt), steps, 2, torch)
    P.profile_enable(True)
    P.partition_v(x, cl, torch.int32, out_keys=ok, out_idx=oi, counts=cnt)
    torch.cuda.synchronize()
    P.profile_enable(False)
    k = _prof(P)
    sc = k.get("flatv_scatter", {}).get("avg_ms", 0.0)
    ok_ = _verify("partition3", {"keys": _sha(ok), "idx_i32": _sha(oi), "counts": cnt.cpu().tolist()},
                  _golden()["partition3_2e28_f32"])
    return {"ms": t * 1e3, "GElem_s": n / t / 1e9, "counts": cnt.cpu().tolist(),
            "verified_against_oracle": ok_,
            "scatter_alg_GBps": 12 * n / (sc * 1e-3) / 1e9 if sc else None, "kernels": k}


def section_shape_tools(args, torch, np, P, W, dev):
    """mkII and mkSgmDescr of the 10^4-row shape (7.04e7 elements, int32 row
    numbers) and sgmSum of 2^26 int64 values with a flag at every row start
    of the same kind of shape."""
    shape = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
    n = int(shape.sum())
    st = torch.from_numpy(shape).to(dev)
    steps = max(3, args.steps // 2)
    ii = torch.empty(n, dtype=torch.int32, device=dev)
    t_ii = timed(lambda: P.mk_ii(st, n, torch.int32), steps, 2, torch)
    xs_rows = torch.arange(1, W.SEG_M + 1, dtype=torch.int64, device=dev)
    t_descr = timed(lambda: P.mk_sgm_descr(st, xs_rows, n), steps, 2, torch)
    del ii
    m = 1 << 26
    flags = torch.zeros(m, dtype=torch.uint8, device=dev)
    flags[torch.from_numpy(np.unique(np.random.default_rng(W.SEG_KEYS_SEED).integers(0, m, m >> 12))).to(dev)] = 1
    xs = torch.from_numpy(W.int_keys(m, W.SEG_KEYS_SEED).astype(np.int64)).to(dev)
    out = torch.empty_like(xs)
    t_sg = timed(lambda: P.sgm_sum(flags, xs, out), steps, 2, torch)
    return {"mk_ii_int32": {"n": n, "ms": t_ii * 1e3, "alg_GBps": 4 * n / t_ii / 1e9},
            "mk_sgm_descr_int64": {"n": n, "ms": t_descr * 1e3, "alg_GBps": 8 * n / t_descr / 1e9},
            "sgm_sum_2^26_int64": {"ms": t_sg * 1e3, "alg_GBps": 17 * m / t_sg / 1e9}}


def profile_run(args, torch, np, P, W, dev):
    """One workload's launches only (inputs built first, outside the loop):
    for rocprofv3, whose per-kernel summaries and counters are taken from
    these runs.  A plain device copy of 1 GiB runs once first, to calibrate
    FETCH_SIZE / WRITE_SIZE against known bytes."""
    cal = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    torch.empty_like(cal).copy_(cal)
    del cal
    name = args.profile
    if name in ("flat", "filter"):
        x = torch.from_numpy(W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)).to(dev)
        ok = torch.empty_like(x)
        oi = torch.empty(x.numel(), dtype=torch.int32, device=dev)
        sp = torch.empty(1, dtype=torch.int64, device=dev)
        mode = P.MODE_PARTITION if name == "flat" else P.MODE_FILTER
        preds = [P.Pred.lt(s) for s in W.FLAT_LARGE_SELECTIVITIES] if name == "flat" else [P.Pred.lt(0.5)]

        def fn():
            for p in preds:
                P.partition(x, p, mode, torch.int32, out_keys=ok, out_idx=oi, split=sp)
    elif name == "flat_small":
        ks = torch.from_numpy(W.int_keys(W.FLAT_SMALL_N, W.FLAT_SMALL_SEED)).to(dev)
        oks = torch.empty_like(ks)
        ois = torch.empty(ks.numel(), dtype=torch.int64, device=dev)
        sp = torch.empty(1, dtype=torch.int64, device=dev)
        p = P.Pred.mod_eq(2, 0)

        def fn():
            P.partition(ks, p, P.MODE_PARTITION, torch.int64, out_keys=oks, out_idx=ois, split=sp)
    elif name == "segmented":
        shape_np = W.segment_sizes(W.SEG_M, W.SEG_SIZES_SEED)
        keys = torch.from_numpy(W.int_keys(int(shape_np.sum()), W.SEG_KEYS_SEED)).to(dev)
        shape = torch.from_numpy(shape_np).to(dev)
        pred = P.Pred.mod_eq(3, 0)
        g = P.SegmentedGraph(keys, shape, pred, tune=(256, 4, 64, P._lib.ROW_SYNC_WAIT))
        fn = g.launch
    elif name == "fwd_bwd":
        n, cols = W.AUTOGRAD_N, W.AUTOGRAD_ROW
        keys = torch.from_numpy(W.int_keys(n, W.AUTOGRAD_SEEDS[0])).to(dev)
        p = torch.from_numpy(W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[1])).to(dev).requires_grad_(True)
        gy = torch.from_numpy(W.f32_normal((n, cols), W.AUTOGRAD_SEEDS[2])).to(dev)
        pred = P.Pred.mod_eq(2, 0)

        def fn():
            p.grad = None
            y, _, _, _ = P.partition_scatter(keys, p, pred)
            y.backward(gy)
    else:
        n = W.PROPS_N
        perm = W.permutation(n, W.PROPS_PERM_SEED)
        if name == "props_faulty":
            perm = W.inject_faults(perm, 1000, 1052, "mixed")
        x = torch.from_numpy(perm).to(dev)
        del perm
        mask = P.RANGE | P.INJ | P.BIJ | (P.MONO if name == "props_faulty" else 0)

        def fn():
            P.check_props(x, mask, 0, n, 0, n)
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    print(json.dumps({"profile": name, "steps": args.steps,
                      "ms_per_step": (time.perf_counter() - t0) / args.steps * 1e3}))


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(W, np, min_seconds=10.0, max_passes=8):
    """The oracle (single-threaded C) on the headline's 2^28 f32 input, whole
    passes over the three selectivities repeated until at least `min_seconds`
    have elapsed (at most `max_passes`), with this process pinned to one host
    core."""
    import oracle as O
    xs = W.f32_uniform(W.FLAT_LARGE_N, W.FLAT_LARGE_SEED)
    ns = xs.size
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    passes = 0
    try:
        t0 = time.perf_counter()
        while True:
            for s in W.FLAT_LARGE_SELECTIVITIES:
                O.partition2(xs, O.Pred.lt(s))
            passes += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds or passes >= max_passes:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    done = passes * len(W.FLAT_LARGE_SELECTIVITIES) * ns
    return {"value": done / dt / 1e9, "unit": "GElem/s",
            "cores": 1, "kind": "oracle",
            "host": {"cpu_model": _host_cpu(), "os_cpu_count": os.cpu_count(),
                     "cores_allowed": len(allowed), "pinned_core": core},
            "sample": f"partition2 of the 2^28 f32 input once per s in "
                      f"{list(W.FLAT_LARGE_SELECTIVITIES)}, {passes} pass(es): {dt:.1f} s on one "
                      f"host core (process pinned to core {core})"}


if __name__ == "__main__":
    main()
