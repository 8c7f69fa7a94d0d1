"""Benchmark: exact radius queries/s.

Default (the headline): the gmm16 workload -- n = 1e6 points, d = 16,
float32, 20-cluster Gaussian mixture, 1e5 out-of-sample queries, R = 1.5 --
with the precision form (the matrix-core screen AUTO picks -- fp16 operands
on this set -- plus the float64 recheck) timed against the bf16 three-term
screen and the plain float64 GPU kernel.  ``--workload`` selects another
configuration (uniform2d, gmm128z, blobs3d, ...); those print the same kind
of line for that workload.

One step = one snn_query (or snn_query_self) call over all queries with the
index and the queries resident in HBM.  W untimed warm-up steps, then K timed
steps bracketed by torch.cuda.synchronize(), each step also bracketed by HIP
events on the library's stream; value = m / (median step time).

Prints one JSON line.  ``roofline`` describes the dominant kernel (the
candidate screen): algorithmic work per launch (the sum over queries of the
window size |J_q| times the flop count Section 4 gives per candidate: 2d for
eq. (ip2), 3d - 1 for eq. (ip1)) over the kernel's average duration, timed with
HIP events the library records on its own stream around that kernel.
``cpu_baseline`` times the CPU oracle (CPU SNN, Algorithms 1-2, float64 BLAS)
on a bounded sample of the same queries.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_FLOPS = 2.5e15  # MI355X dense bf16 matrix peak
PEAK_FP32_FLOPS = 157.3e12  # MI355X fp32 matrix (and vector) peak
PEAK_FP64_VALU_OPS = 256 * 4 * 16 * 2.4e9  # non-fused float64 lane-ops/s: CUs x SIMDs x lanes x clock
PEAK_HBM = 8.0e12
INDEX_BUILDS = 9  # index builds timed (median reported)

HEADLINE_METRIC = "exact radius queries/s at n=1e6,d=16: MFMA+FP64 recheck vs plain FP64 GPU"

WORKLOADS = {
    "gmm16": dict(desc="gmm16: n=1e6 d=16 float32, 20-cluster Gaussian mixture, 1e5 out-of-sample queries, R=1.5",
                  precisions="auto,mixed,fp64", cpu_sample=2000),
    "uniform2d": dict(desc="uniform2d: n=1e4 d=2 float64 uniform in [0,1]^2, 1e3 queries sampled from the data, "
                           "R=0.05", precisions="auto,fp64", cpu_sample=1000),
    "gmm128z": dict(desc="gmm128z: n=2e6 d=128 float32, 50-cluster mixture z-scored per feature, all-points "
                         "self-query, R=4.0", precisions="auto", cpu_sample=200),
    "blobs3d": dict(desc="blobs3d: n=5e6 d=3 float32, 1000 Gaussian blobs (std 0.01) + 20% uniform background in "
                         "[0,1]^3, all-points self-query, R=0.005", precisions="auto", cpu_sample=500),
    "angular100": dict(desc="angular100: n=1183514 d=100 float32 clustered directions (GloVe-100 shape), rows "
                            "normalised on the device, 1e4 out-of-sample queries, angle <= 39 degrees "
                            "(Euclidean R = sqrt(2 - 2 cos 39deg) on unit rows)", precisions="auto,fp64",
                       cpu_sample=300),
    "stream_gmm16": dict(desc="stream_gmm16: gmm16 mixture, index built on 1e6 points, then --steps inserts of 1e5 "
                              "points each (streaming); queries of the grown index against a rebuilt one",
                         precisions="auto", cpu_sample=200000),
    "dbscan_blobs3d": dict(desc="dbscan_blobs3d: DBSCAN (Section 6.4) of blobs3d, n=5e6 d=3 float32, eps=R=0.005, "
                                "min_samples=5; one step = all-points self-query + clustering on a built index",
                           precisions="auto", cpu_sample=50000),
    "blobs3d_batch": dict(desc="blobs3d_batch: the blobs3d particle set (n=5e6, d=3, R=0.005, all-points self-query) "
                               "as an instance of the batched form, on the fp32 matrix-core screen inside the captured "
                               "graph (precision and batching forms combined)", precisions="auto", cpu_sample=0),
    "batch256": dict(desc="batch256: 256 instances, n log-uniform in [1e3,1e5], d in {3,8,32}, float32 uniform in "
                          "the unit cube, 10% of the points as queries, R for ~30 expected neighbours; one captured "
                          "graph, autotuned tiles", precisions="mixed", cpu_sample=4000),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "mixed": "paper_2212_07679_amd/csrc/k_cand_mfma.hip",
    "fp16": "paper_2212_07679_amd/csrc/k_cand_mfma.hip",
    "fp32": "paper_2212_07679_amd/csrc/k_cand_mfma.hip",
    "fp64": "paper_2212_07679_amd/csrc/k_cand_fp64.hip",
}


def source_hash(rel):
    import hashlib

    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload, used):
    """HBM bytes per launch of the screen kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    try:
        rec = json.load(open(TRAFFIC_FILE)).get(f"{workload}/{used}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256_16") != source_hash(KERNEL_SOURCES[used]):
        return None
    return rec["traffic_bytes"]


def copy_probe(nbytes):
    """A plain device-to-device copy of known size, for calibrating the
    FETCH_SIZE / WRITE_SIZE counters (profile this command with --pmc)."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 3}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gmm16", choices=sorted(WORKLOADS) + ["copyprobe"])
    ap.add_argument("--n", type=int, default=0, help="override the number of points (0: the workload's)")
    ap.add_argument("--m", type=int, default=0, help="override the number of queries (gmm16, uniform2d)")
    ap.add_argument("--R", type=float, default=0.0, help="override the radius (0: the workload's)")
    ap.add_argument("--precisions", default="", help="comma list; the first is the reported value")
    ap.add_argument("--cpu-sample", type=int, default=-1, help="queries the CPU oracle times (0: skip)")
    ap.add_argument("--check", type=int, default=200, help="queries checked against the oracle (0: skip)")
    return ap.parse_args()


def make_workload(name, n, m):
    from paper_2212_07679_amd import workloads as W

    if name == "gmm16":
        return W.gmm16(**({"n": n} if n else {}), **({"m": m} if m else {}))
    if name == "uniform2d":
        return W.uniform2d(**({"n": n} if n else {}), **({"m": m} if m else {}))
    if name == "gmm128z":
        return W.gmm128z(**({"n": n} if n else {}))
    if name == "blobs3d":
        return W.blobs3d(**({"n": n} if n else {}))
    if name == "angular100":
        return W.angular100(**({"n": n} if n else {}), **({"m": m} if m else {}))
    raise ValueError(name)


def run_query(idx, w, Qdev, prec):
    if w.alpha is not None:  # angular neighbours of unit rows: the library takes the angle
        return idx.query(Qdev, w.alpha, precision=prec, stats=True, metric="angular")
    if w.Q is None:
        return idx.query_self(w.R, precision=prec, stats=True)
    return idx.query(Qdev, w.R, precision=prec, stats=True)


def query_args(w, Qdev):
    """(Q or None, radius, metric) of the workload's query call."""
    if w.alpha is not None:  # angular neighbours of unit rows: the library takes the angle
        return Qdev, w.alpha, "angular"
    return (None if w.Q is None else Qdev), w.R, "l2"


def time_precision(idx, w, Qdev, prec, steps, warmup, torch):
    """W warm-ups, then K steps bracketed by synchronisations; each step is
    also bracketed by its own events on the library's stream, for the median.
    A step is one C-ABI call into output buffers allocated once (sized by a
    first call), as a serving loop makes it; the same call through the
    allocating binding (fresh output tensors per call) is timed after it."""
    first = run_query(idx, w, Qdev, prec)
    nnz0 = int(first[1].numel())
    m = first[0].numel() - 1
    dev = Qdev.device if Qdev is not None else torch.device("cuda:0")
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz0, 1), dtype=torch.int32, device=dev)
    dist = torch.empty(max(nnz0, 1), dtype=torch.float32, device=dev)
    Q, R, metric = query_args(w, Qdev)

    def step():
        return idx.query_into(Q, R, rp, col, dist, precision=prec, stats=True, metric=metric)

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        screen = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        t0 = time.perf_counter()
        ev[0].record(idx.stream)
        for j in range(k):
            r = fn()
            ev[j + 1].record(idx.stream)
            screen.append(r[-1]["screen_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = sorted(ev[j].elapsed_time(ev[j + 1]) for j in range(k))
        med = per[k // 2] if k % 2 else 0.5 * (per[k // 2 - 1] + per[k // 2])
        return r, wall, ev[0].elapsed_time(ev[k]), med, sum(screen) / len(screen)

    (nnz, st), wall, ev_ms, med, screen_ms = timed(step, steps)
    out = (rp, col[:nnz], dist[:nnz], st)
    _, _, _, alloc_med, _ = timed(lambda: run_query(idx, w, Qdev, prec), min(steps, 10))
    return out, wall, ev_ms, med, screen_ms, alloc_med  # screen_ms: the screen kernel's average duration


def host_cpu():
    """Model name and logical core count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(w, sample):
    """The oracle's CPU SNN (Algorithms 1-2 with float64 BLAS) on a seeded
    sample of the queries, with the BLAS threads the host offers and again on
    one thread (the paper's own timings are single-threaded)."""
    import numpy as np

    import oracle

    cores = oracle_cores()
    g = np.random.default_rng(0)
    sel = np.sort(g.choice(w.m, size=min(sample, w.m), replace=False))
    t0 = time.perf_counter()
    idx = oracle.build_index(w.P)
    t1 = time.perf_counter()

    def run(rows):
        if w.alpha is not None:
            from oracle.metrics import snn_angular

            return snn_angular(idx, w.queries[rows], w.alpha)
        return oracle.snn_query(idx, w.queries[rows], w.R)

    nb, st = run(sel)
    t2 = time.perf_counter()
    one = None
    try:
        from threadpoolctl import threadpool_limits

        sel1 = sel[: max(1, len(sel) // 4)]
        with threadpool_limits(limits=1):
            t3 = time.perf_counter()
            run(sel1)
            one = {"value": len(sel1) / (time.perf_counter() - t3), "sample": f"first {len(sel1)} of the sample"}
    except Exception as e:  # threadpoolctl unavailable: report only the multi-thread figure
        one = {"value": None, "error": str(e)}
    model, ncpu = host_cpu()
    return {
        "value": len(sel) / (t2 - t1),
        "unit": "queries/s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": f"{len(sel)} of the {w.m} queries (seeded), index built separately in {t1 - t0:.1f} s",
        "single_thread": one,
        "host_cpu": model,
        "host_logical_cpus": ncpu,
    }, (sel, nb)


def roofline(prec_used, terms, st, screen_ms, d):
    if prec_used in ("mixed", "fp16"):  # bf16 and fp16 share the dense matrix peak
        achieved = st["pairs_window"] * 2 * d / (screen_ms / 1e3)
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16_FLOPS / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_BF16_FLOPS, "traffic": None}
    if prec_used == "fp32":
        achieved = st["pairs_window"] * 2 * d / (screen_ms / 1e3)
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_FLOPS / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_FLOPS, "traffic": None}
    achieved = st["pairs_window"] * (3 * d - 1) / (screen_ms / 1e3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU_OPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU_OPS, "traffic": None}


def index_hbm(n, d, b, index_ms):
    """Algorithmic HBM bytes of the index build (Algorithm 1 on the device)
    over its wall time: the rows are read four times (centring, Gram matrix,
    scores, gather) and written once in key order in the input dtype and
    centred in fp32, plus key, id, h and norm per row (20 bytes) and four
    radix passes over 8-byte (key, id) pairs read and written (64 bytes per
    row).  The float64 copy of the rows is not part of the build: the first
    float64 screen or self-query makes it."""
    nbytes = 4 * n * d * b + n * (d * b + 4 * d + 20) + 64 * n
    achieved = nbytes / (index_ms / 1e3)
    return {"bytes": nbytes, "achieved_GBps": achieved / 1e9, "peak_GBps": PEAK_HBM / 1e9,
            "frac": achieved / PEAK_HBM}


def oracle_cores():
    try:
        from threadpoolctl import threadpool_info

        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def main_batch(a):
    """The batching form: all 256 instances in one captured graph.  One step
    is one launch of the query graph over every instance (the indexes are
    built by the index graph, timed separately); the same step is also timed
    with the index pass included, and against a loop of per-instance calls
    of the plain float64 kernel and of the mixed screen."""
    import numpy as np
    import torch

    import oracle
    from paper_2212_07679_amd import binding
    from paper_2212_07679_amd import workloads as W

    spec = WORKLOADS["batch256"]
    insts = W.batch256()
    M = sum(w.m for w in insts)
    print(f"[bench] batch256: {len(insts)} instances, sum n={sum(w.n for w in insts)} sum m={M}", file=sys.stderr,
          flush=True)
    dev = [(torch.from_numpy(w.P).cuda(), torch.from_numpy(w.Q).cuda(), w.R) for w in insts]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = binding.Batch(dev, autotune=True)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    info = plan.info()
    print(f"[bench] plan created (incl. autotune) in {create_s:.2f} s: {info}", file=sys.stderr, flush=True)

    def timed(fn, steps, stream):
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        out = None
        for _ in range(steps):
            out = fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, out

    for _ in range(a.warmup):
        plan.run(index=False, stats=True)
    screens = []

    # a step: one launch of the captured query pass and its read-back (the
    # lists stay in the plan's output buffers, as a serving loop reads them)
    def q_step():
        r = plan.run(index=False, stats=True, views=False)
        screens.append(r[1]["screen_ms"])
        return r

    ms, (_, st) = timed(q_step, a.steps, plan.stream)
    full_ms, _ = timed(lambda: plan.run(index=True, stats=True, views=False), max(1, a.steps // 2), plan.stream)
    res = plan.run(index=False)  # the lists, for the check below
    screen_ms = sum(screens) / len(screens)
    print(f"[bench] batched query graph {ms:.3f} ms/step (screen {screen_ms:.3f} ms), index+query {full_ms:.3f} ms,"
          f" stats {st}", file=sys.stderr, flush=True)

    # per-instance calls of the single-instance path (indexes built outside the timing)
    idxs = [binding.Index(X) for X, _, _ in dev]
    loops = {}
    for prec in ("fp64", "mixed"):
        def loop():
            return [ix.query(Q, R, precision=prec) for ix, (_, Q, R) in zip(idxs, dev)]

        loop()
        loops[prec], lres = timed(loop, max(1, min(a.steps, 3)), idxs[0].stream)
        for i in range(len(insts)):
            for x, y in zip(lres[i], res[i]):
                assert torch.equal(x, y), f"instance {i}: batched and per-instance {prec} results differ"
        print(f"[bench] per-instance loop {prec}: {loops[prec]:.3f} ms/step", file=sys.stderr, flush=True)
    for ix in idxs:
        ix.close()

    cpu = None
    if a.cpu_sample != 0:
        budget = spec["cpu_sample"] if a.cpu_sample < 0 else a.cpu_sample
        g = np.random.default_rng(1)
        order = g.permutation(len(insts))
        done = 0
        tq = 0.0
        used = 0
        for i in order:
            w = insts[i]
            take = min(w.m, 64, budget - done)
            if take <= 0:
                break
            ix = oracle.build_index(w.P)
            t1 = time.perf_counter()
            nb, _ = oracle.snn_query(ix, w.Q[:take], w.R)
            tq += time.perf_counter() - t1
            done += take
            used += 1
            rp, col, _ = (t.cpu().numpy() for t in res[i])
            for k in range(min(take, 8)):
                assert np.array_equal(col[rp[k]:rp[k + 1]], nb.col[nb.row_ptr[k]:nb.row_ptr[k + 1]]), \
                    f"instance {i} query {k} differs from the oracle"
        cpu = {"value": done / tq, "unit": "queries/s", "cores": oracle_cores(), "kind": "oracle", "host_cpu": host_cpu()[0],
               "sample": f"first {done} queries (up to 64 each) of {used} seeded-random instances; "
                         "index builds not timed"}

    flops = st["flops_window"]
    roof = None
    if screen_ms > 0:
        ach = flops / (screen_ms / 1e3)
        roof = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_BF16_FLOPS / 1e12, "unit": "TFLOP/s",
                "frac": ach / PEAK_BF16_FLOPS, "traffic": None}
    line = {
        "metric": "exact radius queries/s (batched instances)",
        "value": M / (ms / 1e3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "instances": len(insts), "sum_n": sum(w.n for w in insts), "sum_m": M,
                   "tiles": info},
        "index_and_query_ms_per_step": full_ms,
        "per_instance_fp64_ms_per_step": loops["fp64"],
        "per_instance_mixed_ms_per_step": loops["mixed"],
        "speedup_vs_fp64_gpu": loops["fp64"] / ms,
        "pairs_window": st["pairs_window"],
        "pairs_executed": st["pairs_executed"],
        "pairs_recheck": st["pairs_recheck"],
        "recheck_fraction": st["pairs_recheck"] / max(st["pairs_window"], 1),
        "nnz": st["nnz"],
        "screen_ms": screen_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main_blobs_batch(a):
    """The particle set with the precision and batching forms combined: the
    blobs3d self-query as an instance of the batched form (one captured
    graph; its three-term bf16 band would pass too many pairs, so the plan
    puts it on the fp32 matrix-core screen).  One step is one launch of the
    query graph (the index graph is timed separately); the result is checked
    byte for byte against the single-instance path."""
    import torch

    from paper_2212_07679_amd import binding
    from paper_2212_07679_amd import workloads as W

    spec = WORKLOADS["blobs3d_batch"]
    w = W.blobs3d(**({"n": a.n} if a.n else {}))
    print(f"[bench] blobs3d_batch: n={w.n} d={w.d} R={w.R}", file=sys.stderr, flush=True)
    X = torch.from_numpy(w.P).cuda()
    torch.cuda.synchronize()
    plan = binding.Batch([(X, None, w.R)])
    info = plan.info()
    assert info["fp32_instances"] == 1, info
    print(f"[bench] plan: {info}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        plan.run(index=False, stats=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    screens = []
    ev[0].record(plan.stream)
    for k in range(a.steps):
        res, st = plan.run(index=False, stats=True)
        ev[k + 1].record(plan.stream)
        screens.append(st["screen_ms"])
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(a.steps))
    ms = per[a.steps // 2]
    screen_ms = sum(screens) / len(screens)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(plan.stream)
    plan.run(index=True, query=False)
    t1.record(plan.stream)
    torch.cuda.synchronize()
    index_ms = t0.elapsed_time(t1)
    # the single-instance path on the same points: identical CSR
    idx = binding.Index(X)
    single = idx.query_self(w.R, stats=True)
    torch.cuda.synchronize()
    for x, y in zip(single[:3], res[0]):
        assert torch.equal(x, y), "batched and single-instance results differ"
    print(f"[bench] batched self-query {ms:.3f} ms/step (screen {screen_ms:.3f} ms), index {index_ms:.3f} ms; "
          f"single-instance {single[3]['total_ms']:.3f} ms (screen {single[3]['screen_ms']:.3f} ms, symmetric scan)",
          file=sys.stderr, flush=True)
    idx.close()
    ach = st["flops_window"] / (screen_ms / 1e3) if screen_ms > 0 else 0.0
    line = {
        "metric": "exact radius queries/s (particle self-query, precision and batching forms combined)",
        "value": w.n / (ms / 1e3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": w.n, "d": w.d, "R": w.R, "tiles": info},
        "index_ms": index_ms,
        "single_instance_ms": single[3]["total_ms"],
        "pairs_window": st["pairs_window"],
        "pairs_executed": st["pairs_executed"],
        "pairs_recheck": st["pairs_recheck"],
        "nnz": st["nnz"],
        "screen_ms": screen_ms,
        "roofline": {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_FP32_FLOPS / 1e12,
                     "unit": "TFLOP/s", "frac": ach / PEAK_FP32_FLOPS, "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(line))


def main_dbscan(a):
    """DBSCAN of the particle workload (Section 6.4's application).  One step
    is the clustering of the indexed points: the all-points self-query with
    radius eps feeding the union-find labelling on the device.  The index
    build is timed separately (as for the query workloads), and the route
    through explicit neighbour lists (snn_query_self + snn_dbscan) is timed
    beside it."""
    import numpy as np
    import torch

    import oracle
    from paper_2212_07679_amd import binding
    from paper_2212_07679_amd import workloads as W

    spec = WORKLOADS["dbscan_blobs3d"]
    min_samples = 5
    w = W.blobs3d(**({"n": a.n} if a.n else {}))
    eps = w.R
    X = torch.from_numpy(w.P).to("cuda:0")
    torch.cuda.synchronize()
    binding.Index(X).close()  # first build: allocations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = binding.Index(X)
    torch.cuda.synchronize()
    index_ms = (time.perf_counter() - t0) * 1e3
    stream = idx.stream

    def timed(fn, steps):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        out = None
        for _ in range(steps):
            out = fn()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, out

    fused = lambda: idx.dbscan(eps, min_samples, stats=True)  # noqa: E731

    def lists():
        rp, col, _ = idx.query_self(eps)
        return binding.dbscan_csr(rp, col, min_samples, stream=stream)

    for _ in range(a.warmup):
        fused()
    ms, (labels, core, k, st) = timed(fused, a.steps)
    lists()
    lists_ms, (labels2, core2, k2) = timed(lists, max(1, min(a.steps, 3)))
    assert torch.equal(labels, labels2) and torch.equal(core, core2) and k == k2, "the two routes differ"
    lab = labels.cpu().numpy()
    assert k == int(lab.max()) + 1 and lab.min() >= -1
    print(f"[bench] dbscan: {ms:.3f} ms/step (screen {st['screen_ms']:.3f}), via neighbour lists {lists_ms:.3f} ms, "
          f"index {index_ms:.1f} ms, clusters {k}, noise {int((lab == -1).sum())}", file=sys.stderr, flush=True)

    cpu = None
    if a.cpu_sample != 0:
        ns = spec["cpu_sample"] if a.cpu_sample < 0 else a.cpu_sample
        # the same recipe at a size the oracle finishes in seconds: blob count
        # scaled with n, so the points per blob (and the density) stay the same
        kb = max(1, round(1000 * ns / w.n))
        ws = W.blobs3d(n=ns, k=kb)
        t0 = time.perf_counter()
        oracle.dbscan(ws.P, eps, min_samples)
        tc = time.perf_counter() - t0
        cpu = {"value": ns / tc, "unit": "points/s", "cores": oracle_cores(), "kind": "oracle", "host_cpu": host_cpu()[0],
               "sample": f"the blobs3d recipe at n={ns} with {kb} blobs (same points per blob), eps={eps}, "
                         f"min_samples={min_samples}; brute-force lists + DBSCAN, {tc:.1f} s"}
    line = {
        "metric": "DBSCAN points/s (self-query + clustering on a built index)",
        "value": w.n / (ms / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": w.n, "d": w.d, "eps": eps, "min_samples": min_samples},
        "index_ms": index_ms,
        "via_lists_ms_per_step": lists_ms,
        "clusters": k,
        "noise": int((lab == -1).sum()),
        "nnz": st["nnz"],
        "pairs_window": st["pairs_window"],
        "pairs_recheck": st["pairs_recheck"],
        "screen_ms": st["screen_ms"],
        "roofline": roofline(binding.PRECISION_NAMES[st["precision_used"]], st["terms_used"], st, st["screen_ms"],
                             w.d),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main_stream(a):
    """Streaming inserts: one step is one insert of 1e5 points into a grown
    index (centre and direction kept from the first build).  Reported beside
    it: the build of the first 1e6 points, a rebuild of the grown set, and
    queries of the grown index against the rebuilt one (same results)."""
    import numpy as np
    import torch

    import oracle
    from paper_2212_07679_amd import binding
    from paper_2212_07679_amd import workloads as W

    spec = WORKLOADS["stream_gmm16"]
    n0, batch = 1_000_000, 100_000
    total = n0 + batch * (a.steps + 1)
    w = W.gmm16(n=total, m=100_000)
    X = torch.from_numpy(w.P).to("cuda:0")
    Q = torch.from_numpy(w.Q).to("cuda:0")
    torch.cuda.synchronize()

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, out

    binding.Index(X[:n0]).close()  # allocations
    build_ms, idx = wall(lambda: binding.Index(X[:n0]))
    idx.insert(X[n0:n0 + batch])  # warm-up insert
    times = []
    for k in range(a.steps):
        lo = n0 + batch * (k + 1)
        ms, _ = wall(lambda: idx.insert(X[lo:lo + batch]))
        times.append(ms)
    ins_ms = float(np.mean(times))
    rebuild_ms, full = wall(lambda: binding.Index(X))
    for i in (idx, full):
        i.query(Q, w.R)
    q_grown, r1 = wall(lambda: idx.query(Q, w.R, stats=True))
    q_full, r2 = wall(lambda: full.query(Q, w.R, stats=True))
    for x, y in zip(r1[:3], r2[:3]):
        assert torch.equal(x, y), "grown and rebuilt indexes differ"
    # bytes the merge moves per insert: every row of the grown arrays read
    # once (old or new part) and written once
    d, dp = w.d, ((w.d + 3) // 4) * 4
    row_bytes = 8 + 4 + 4 * d + 8 * dp + 4 * d + 4 + 4
    n_mid = n0 + batch * (a.steps / 2 + 1)
    achieved = 2.0 * row_bytes * n_mid / (ins_ms / 1e3)
    print(f"[bench] stream: build {build_ms:.1f} ms, insert {ins_ms:.2f} ms per 1e5, rebuild of {total} "
          f"{rebuild_ms:.1f} ms, query grown {q_grown:.2f} ms vs rebuilt {q_full:.2f} ms", file=sys.stderr, flush=True)

    cpu = None
    if a.cpu_sample != 0:
        ns = spec["cpu_sample"] if a.cpu_sample < 0 else a.cpu_sample
        t0 = time.perf_counter()
        oracle.build_index(w.P[:ns])
        tc = time.perf_counter() - t0
        cpu = {"value": ns / tc, "unit": "points/s", "cores": oracle_cores(), "kind": "oracle", "host_cpu": host_cpu()[0],
               "sample": f"the oracle's index build (Algorithm 1) of {ns} rows of the same mixture, {tc:.2f} s"}
    line = {
        "metric": "streaming insert points/s into an exact SNN index",
        "value": batch / (ins_ms / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": 1,
        "ms_per_step": ins_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n0": n0, "batch": batch, "n_final": total, "d": d},
        "build_ms": build_ms,
        "rebuild_ms": rebuild_ms,
        "query_ms_grown": q_grown,
        "query_ms_rebuilt": q_full,
        "pairs_window_grown": r1[3]["pairs_window"],
        "pairs_window_rebuilt": r2[3]["pairs_window"],
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); queries shard across GPUs without "
              "communication, see the design notes for the multi-GPU mapping", file=sys.stderr)
        sys.exit(2)
    if a.workload == "copyprobe":
        copy_probe(1 << 30)
        return
    if a.workload == "batch256":
        main_batch(a)
        return
    if a.workload == "dbscan_blobs3d":
        main_dbscan(a)
        return
    if a.workload == "stream_gmm16":
        main_stream(a)
        return
    if a.workload == "blobs3d_batch":
        main_blobs_batch(a)
        return
    import numpy as np
    import torch

    from paper_2212_07679_amd import binding

    spec = WORKLOADS[a.workload]
    precisions = [p for p in (a.precisions or spec["precisions"]).split(",") if p]
    cpu_sample = spec["cpu_sample"] if a.cpu_sample < 0 else a.cpu_sample
    t_gen = time.perf_counter()
    w = make_workload(a.workload, a.n, a.m)
    if a.R > 0:
        import dataclasses

        w = dataclasses.replace(w, R=a.R)
    print(f"[bench] {a.workload}: n={w.n} d={w.d} m={w.m} R={w.R} generated in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.P).to(dev)
    Qdev = torch.from_numpy(w.Q).to(dev) if w.Q is not None else None
    normalize_ms = None
    if w.alpha is not None:
        # angular neighbours: rows normalised on the device, then a search by
        # angle (the library compares S with the squared chord 2 - 2 cos alpha)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.normalize_rows(X, out=X)
        binding.normalize_rows(Qdev, out=Qdev)
        torch.cuda.synchronize()
        normalize_ms = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()
    idx = binding.Index(X)  # first build: allocations
    idx.close()
    # the build ends with a read-back, so its wall time is the device time
    # plus the host's launches; the median of several builds
    builds = []
    for _ in range(INDEX_BUILDS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = binding.Index(X)
        torch.cuda.synchronize()
        builds.append((time.perf_counter() - t0) * 1e3)
        if len(builds) < INDEX_BUILDS:
            idx.close()
    index_ms = statistics.median(builds)

    results = {}
    for prec in precisions:
        out, wall, ev_ms, med_ms, screen_ms, alloc_ms = time_precision(idx, w, Qdev, prec, a.steps, a.warmup, torch)
        st = out[3]
        results[prec] = {
            "qps": w.m / (med_ms / 1e3),
            "ms_per_step": med_ms,
            "alloc_ms_per_step": alloc_ms,
            "mean_ms_per_step": ev_ms / a.steps,
            "wall_ms_per_step": wall * 1e3 / a.steps,
            "screen_ms": screen_ms,
            "stats": st,
            "out": out,
        }
        used = binding.PRECISION_NAMES[st["precision_used"]]
        print(f"[bench] {prec} ({used}, terms {st['terms_used']}): {results[prec]['ms_per_step']:.3f} ms/step, "
              f"screen {screen_ms:.3f} ms, nnz {st['nnz']}, window pairs {st['pairs_window']}, "
              f"rechecked {st['pairs_recheck']}", file=sys.stderr, flush=True)

    # one more call of the first precision with per-stage device times
    # (SNN_PROFILE: launched kernel by kernel, outside the timed steps)
    os.environ["SNN_PROFILE"] = "1"
    try:
        prof = run_query(idx, w, Qdev, precisions[0])[3]
    finally:
        del os.environ["SNN_PROFILE"]
    stage_ms = dict(zip(("order", "window", "screen", "recheck", "assemble"), prof["stage_ms"]))
    stage_ms["call"] = prof["total_ms"]
    print(f"[bench] stages (profiled call): {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})}",
          file=sys.stderr, flush=True)

    # identical results across precisions
    for p in precisions[1:]:
        for x, y in zip(results[precisions[0]]["out"][:3], results[p]["out"][:3]):
            assert torch.equal(x, y), f"{precisions[0]} and {p} differ"

    cpu = None
    if cpu_sample > 0:
        wc = w
        if w.alpha is not None:
            import dataclasses

            from oracle.metrics import normalize_rows

            wc = dataclasses.replace(w, P=normalize_rows(w.P), Q=normalize_rows(w.Q))
        cpu, (sel, nb) = cpu_baseline(wc, cpu_sample)
        rp, col, dist = (t.cpu().numpy() for t in results[precisions[0]]["out"][:3])
        for k, qi in enumerate(sel[: a.check]):
            got = col[rp[qi]:rp[qi + 1]]
            assert np.array_equal(got, nb.col[nb.row_ptr[k]:nb.row_ptr[k + 1]]), f"query {qi} differs from the oracle"

    head = precisions[0]
    r = results[head]
    st = r["stats"]
    used = binding.PRECISION_NAMES[st["precision_used"]]
    fp64 = results.get("fp64")
    line = {
        "metric": HEADLINE_METRIC if a.workload == "gmm16" else (
            "exact angular radius queries/s" if w.alpha is not None else "exact radius queries/s"),
        "value": r["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "timing": "value and ms_per_step: median of the K steps, each bracketed by HIP events on the library's "
                  "stream, a step being one C-ABI query call into output buffers allocated once; mean_ms_per_step: "
                  "the K steps between one pair of events; alloc_ms_per_step: the median step of the binding's "
                  "allocating call (new output tensors per call)",
        "mean_ms_per_step": r["mean_ms_per_step"],
        "alloc_ms_per_step": r["alloc_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16+f64", "fp16": "f16+f64", "fp32": "f32+f64", "fp64": "f64"}[used],
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": w.n, "d": w.d, "m": w.m, "R": (None if w.alpha is not None else w.R), "self_query": w.Q is None,
                   "precision": used, "terms": st["terms_used"],
                   **({"alpha_deg": math.degrees(w.alpha), "normalize_ms": normalize_ms} if w.alpha is not None
                      else {})},
        "fp64_gpu_qps": fp64["qps"] if fp64 else None,
        "speedup_vs_fp64_gpu": (r["qps"] / fp64["qps"]) if (fp64 and head != "fp64") else None,
        "pairs_window": st["pairs_window"],
        "pairs_executed": st["pairs_executed"],
        "pairs_window_per_s": st["pairs_window"] / (r["screen_ms"] / 1e3),
        "pairs_executed_per_s": st["pairs_executed"] / (r["screen_ms"] / 1e3),
        "pairs_recheck": st["pairs_recheck"],
        "recheck_fraction": st["pairs_recheck"] / max(st["pairs_window"], 1),
        "nnz": st["nnz"],
        "screen_ms": r["screen_ms"],
        "stage_ms": stage_ms,
        "index_ms": index_ms,
        "index_timing": f"median wall time of {INDEX_BUILDS} builds (min {min(builds):.3f} ms), after one untimed build",
        "index_hbm": index_hbm(w.n, w.d, w.P.dtype.itemsize, index_ms),
        "roofline": roofline(used, st["terms_used"], st, r["screen_ms"], w.d),
        "cpu_baseline": cpu,
    }
    line["roofline"]["traffic"] = measured_traffic(a.workload, used)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
