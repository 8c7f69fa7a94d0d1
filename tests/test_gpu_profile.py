"""Per-stage device times (SNN_PROFILE) and log lines (SNN_LOG) on the GPU.

A profiled call reports one non-negative time per stage of Algorithm 2
(ordering, windows, screen, recheck, assembly) whose sum stays within the
call's device time, the screen stage close to screen_ms; the results are
the same as without profiling (checked against the oracle).  Without
SNN_PROFILE every stage time is -1.
"""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2212_07679_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_07679_amd import binding

    return binding


@pytest.fixture
def env(monkeypatch):
    return monkeypatch


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check(got, ref, what):
    row_ptr, col, dist = (t.cpu().numpy() for t in got[:3])
    assert np.array_equal(row_ptr, ref.row_ptr), f"{what}: row_ptr"
    assert np.array_equal(col, ref.col), f"{what}: col"
    nz = ref.dist != 0
    assert np.all(np.abs(dist[nz] - ref.dist[nz]) <= 1e-5 * ref.dist[nz]), f"{what}: dist"


def check_stages(st, what):
    t = st["stage_ms"]
    assert len(t) == 5 and all(x >= 0 for x in t), f"{what}: {t}"
    # the screen stage runs event to event, screen_ms from the first
    # workgroup's start to the last one's end: a little shorter
    assert st["screen_ms"] <= t[2] + 2e-3, f"{what}: screen stage {t[2]} vs {st['screen_ms']}"
    assert t[2] <= st["screen_ms"] * 1.05 + 0.05, f"{what}: screen stage {t[2]} vs {st['screen_ms']}"
    assert sum(t) <= st["total_ms"] * 1.001 + 1e-3, f"{what}: stages {t} exceed the call {st['total_ms']}"


@pytest.fixture(scope="module")
def gmm():
    w = W.gmm16(n=20_000, m=2_000, R=3.0)
    return w, oracle.brute_radius(w.P, w.Q, w.R)


@pytest.mark.parametrize("precision", ["auto", "mixed", "fp64"])
def test_profiled_query_stages(B, gmm, env, precision):
    w, ref = gmm
    say(f"profile: gmm16 n={w.n} m={w.m} R={w.R} precision={precision}")
    idx = B.Index(to_dev(w.P))
    Q = to_dev(w.Q)
    env.delenv("SNN_PROFILE", raising=False)
    got = idx.query(Q, w.R, precision=precision, stats=True)
    check(got, ref, "unprofiled")
    assert got[3]["stage_ms"] == [-1.0] * 5
    assert 0 < got[3]["screen_ms"] < got[3]["total_ms"], got[3]
    env.setenv("SNN_PROFILE", "1")
    for k in range(3):  # the same call again: never replayed from a graph while profiled
        got = idx.query(Q, w.R, precision=precision, stats=True)
        check(got, ref, f"profiled call {k}")
        check_stages(got[3], f"profiled call {k}")
    say(f"  stages {['%.3f' % x for x in got[3]['stage_ms']]} total {got[3]['total_ms']:.3f} ms")


def test_profiled_self_query_and_dbscan(B, env):
    w = W.blobs3d(n=20_000, R=0.02)
    ref = oracle.brute_radius(w.P, w.P, w.R)
    say(f"profile: blobs3d self-query n={w.n} R={w.R}")
    env.setenv("SNN_PROFILE", "1")
    idx = B.Index(to_dev(w.P))
    got = idx.query_self(w.R, stats=True)
    check(got, ref, "self-query")
    check_stages(got[3], "self-query")
    labels, core, k, st = idx.dbscan(w.R, 5, stats=True)
    assert k >= 1
    assert all(x >= 0 for x in st["stage_ms"]), st["stage_ms"]


def test_profiled_batch_stages(B, env):
    g = np.random.default_rng([2212, 7679, 41])
    insts, refs = [], []
    for n, m, d, R in ((3000, 300, 3, 0.08), (2000, None, 8, 0.5), (4000, 500, 16, 1.0)):
        P = g.normal(size=(n, d)).astype(np.float32)
        Qn = None if m is None else g.normal(size=(m, d)).astype(np.float32)
        insts.append((to_dev(P), None if Qn is None else to_dev(Qn), R))
        refs.append(oracle.brute_radius(P, P if Qn is None else Qn, R))
    say("profile: batch of 3 instances")
    env.setenv("SNN_PROFILE", "1")
    bt = B.Batch(insts)
    for k in range(2):
        res, st = bt.run(index=False, query=True, stats=True)
        for i, r in enumerate(refs):
            check(res[i], r, f"batch run {k} instance {i}")
        t = st["stage_ms"]
        assert all(x >= 0 for x in t), t
        if st["screen_ms"] >= 0:
            assert abs(t[2] - st["screen_ms"]) <= 1e-3 + 1e-3 * st["screen_ms"], (t, st["screen_ms"])
        assert sum(t) <= st["total_ms"] * 1.001 + 1e-3, (t, st["total_ms"])
    bt.close()
    env.delenv("SNN_PROFILE")
    bt = B.Batch(insts)
    res, st = bt.run(index=False, query=True, stats=True)
    assert st["stage_ms"] == [-1.0] * 5
    bt.close()


def test_log_lines(B, gmm, env, capfd):
    w, ref = gmm
    idx = B.Index(to_dev(w.P))
    Q = to_dev(w.Q)
    env.setenv("SNN_LOG", "2")
    got = idx.query(Q, w.R, stats=True)
    check(got, ref, "logged call")
    err = capfd.readouterr().err
    assert "[snn] query n=20000 d=16 m=2000" in err, err
    assert f"nnz={ref.col.size}" in err, err
    env.setenv("SNN_LOG", "0")
    idx.query(Q, w.R, stats=True)
    assert "[snn]" not in capfd.readouterr().err
