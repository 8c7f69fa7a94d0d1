"""Benchmark: exact radius queries/s on the gmm16 workload (n = 1e6 points,
d = 16, float32, 20-cluster Gaussian mixture, 1e5 out-of-sample queries,
R = 1.5) -- the mixed-precision screen (bf16 matrix cores + float64
recheck) against the plain float64 GPU kernel.

One step = one snn_query call over all 1e5 queries with the index and the
queries resident in HBM.  W untimed warm-up steps, then K timed steps
bracketed by torch.cuda.synchronize(); the value is m * K / elapsed.

Prints one JSON line.  ``roofline`` describes the dominant kernel (the
candidate screen): algorithmic work per launch (sum over queries of the
window size |J_q| times 2d flop, the count of Section 4 for eq. (ip2)) over
its average duration, timed with HIP events the library records on its own
stream around that kernel.  ``cpu_baseline`` times the CPU oracle (CPU SNN,
Algorithms 1-2 with float64 BLAS) on a bounded sample of the same queries.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_FLOPS = 2.5e15  # MI355X dense bf16 matrix peak
PEAK_FP64_VALU_OPS = 256 * 4 * 16 * 2.4e9  # non-fused float64 lane-ops/s: CUs x SIMDs x lanes x clock
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=100_000)
    ap.add_argument("--R", type=float, default=1.5)
    ap.add_argument("--precisions", default="mixed,fp64")
    ap.add_argument("--cpu-sample", type=int, default=2000, help="queries the CPU oracle times (0: skip)")
    ap.add_argument("--check", type=int, default=200, help="queries checked against the oracle (0: skip)")
    return ap.parse_args()


def time_precision(idx, Q, R, prec, steps, warmup, torch):
    for _ in range(warmup):
        out = idx.query(Q, R, precision=prec, stats=True)
    torch.cuda.synchronize()
    screen = []
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(idx.stream)
    for _ in range(steps):
        out = idx.query(Q, R, precision=prec, stats=True)
        screen.append(out[3]["screen_ms"])
    stop.record(idx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    return out, wall, ev_ms, sum(screen) / len(screen)


def cpu_baseline(w, sample):
    import numpy as np

    import oracle

    try:
        from threadpoolctl import threadpool_info

        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    g = np.random.default_rng(0)
    sel = np.sort(g.choice(w.m, size=min(sample, w.m), replace=False))
    t0 = time.perf_counter()
    idx = oracle.build_index(w.P)
    t1 = time.perf_counter()
    nb, st = oracle.snn_query(idx, w.Q[sel], w.R)
    t2 = time.perf_counter()
    return {
        "value": len(sel) / (t2 - t1),
        "unit": "queries/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{len(sel)} of the {w.m} queries (seeded), index built separately in {t1 - t0:.1f} s",
    }, (sel, nb)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); queries shard without communication, "
              "see the design notes for the multi-GPU mapping", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2212_07679_amd import binding, workloads

    w = workloads.gmm16(n=a.n, m=a.m, R=a.R)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.P).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = binding.Index(X)
    torch.cuda.synchronize()
    index_ms = (time.perf_counter() - t0) * 1e3

    results = {}
    for prec in [p for p in a.precisions.split(",") if p]:
        out, wall, ev_ms, screen_ms = time_precision(idx, Q, w.R, prec, a.steps, a.warmup, torch)
        st = out[3]
        results[prec] = {
            "qps": w.m * a.steps / (ev_ms / 1e3),
            "ms_per_step": ev_ms / a.steps,
            "wall_ms_per_step": wall * 1e3 / a.steps,
            "screen_ms": screen_ms,
            "stats": st,
            "out": out,
        }
        print(f"[bench] {prec}: {results[prec]['ms_per_step']:.3f} ms/step, screen {screen_ms:.3f} ms, "
              f"nnz {st['nnz']}, window pairs {st['pairs_window']}, rechecked {st['pairs_recheck']}",
              file=sys.stderr, flush=True)

    # identical results across precisions
    precs = list(results)
    for p in precs[1:]:
        for x, y in zip(results[precs[0]]["out"][:3], results[p]["out"][:3]):
            assert torch.equal(x, y), f"{precs[0]} and {p} differ"

    cpu = None
    if a.cpu_sample > 0:
        cpu, (sel, nb) = cpu_baseline(w, a.cpu_sample)
        # the sampled rows agree with the oracle
        rp, col, _ = (t.cpu().numpy() for t in results[precs[0]]["out"][:3])
        for k, qi in enumerate(sel[: a.check]):
            assert np.array_equal(col[rp[qi]:rp[qi + 1]], nb.col[nb.row_ptr[k]:nb.row_ptr[k + 1]]), f"query {qi}"

    head = "mixed" if "mixed" in results else precs[0]
    r = results[head]
    st = r["stats"]
    d = w.d
    if head == "mixed":
        achieved = st["pairs_window"] * 2 * d / (r["screen_ms"] / 1e3)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16_FLOPS / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_BF16_FLOPS, "traffic": None}
    else:
        achieved = st["pairs_window"] * (3 * d) / (r["screen_ms"] / 1e3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU_OPS / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU_OPS, "traffic": None}
    line = {
        "metric": "exact radius queries/s at n=1e6,d=16: MFMA+FP64 recheck vs plain FP64 GPU",
        "value": r["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "gmm16: n=1e6 d=16 float32, 20-cluster Gaussian mixture, 1e5 out-of-sample "
                               "queries, R=1.5", "n": w.n, "d": d, "m": w.m, "R": w.R, "precision": head},
        "fp64_gpu_qps": results.get("fp64", {}).get("qps"),
        "speedup_vs_fp64_gpu": (r["qps"] / results["fp64"]["qps"]) if ("fp64" in results and head != "fp64") else None,
        "pairs_window": st["pairs_window"],
        "pairs_recheck": st["pairs_recheck"],
        "recheck_fraction": st["pairs_recheck"] / max(st["pairs_window"], 1),
        "nnz": st["nnz"],
        "screen_ms": r["screen_ms"],
        "index_ms": index_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
