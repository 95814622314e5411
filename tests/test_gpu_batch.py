"""GPU: batched solves over many 2-D patterns of uneven size in one launch.

Members follow the 512-member workload recipe (non-diagonal M with 7-smooth
|det M|, rank-1 and rank-2 Smith forms, 2-6 ellipses, contrast 2-50).  Small
members are compared with the FP64 oracle element by element; the full-size
batch against oracle values of sampled members (tests/golden/batch_c4.json).
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import elasticity as E
from oracle.dft import make_transform
from tests.gpu_util import perm_between, tensors_to_fields, rel_err

pytestmark = pytest.mark.gpu
ahom = pytest.importorskip("paper_1605_05712_amd.ahom")

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def loads3():
    eb = np.zeros((3, 3, 3))
    eb[0, 0, 0] = 1.0
    eb[1, 1, 1] = 1.0
    eb[2, 0, 1] = eb[2, 1, 0] = 1.0 / np.sqrt(2.0)
    return eb


def make_batch(seeds, lo=1024, hi=65536, **kw):
    mbs = [synth.batch_2d_member(s, lo, hi) for s in seeds]
    B = ahom.Batch([mb["M"] for mb in mbs], **kw)
    for i, mb in enumerate(mbs):
        m, _ = B.info(i)
        B.set_material(i, np.array(mb["lame"]), synth.ellipses_phase(B.points(i), m, mb["ellipses"]))
    return B, mbs


def test_batch_fields_match_oracle_after_fixed_iterations():
    """12 small members (rank-1 and rank-2), FP64, 3 updates: fields and residual histories."""
    seeds = list(range(9000, 9012))
    say("batch fixed iterations", seeds)
    B, mbs = make_batch(seeds, lo=64, hi=1024, precision=ahom.FP64, tol=0.0, max_iter=3)
    out = B.solve(loads3())
    es = [B.info(i)[1] for i in range(len(seeds))]
    print("Smith forms", [e.tolist() for e in es], flush=True)
    assert any(e[0] == 1 for e in es) and any(e[0] > 1 for e in es)
    assert np.all(out["iters"] == 3)
    for i, mb in enumerate(mbs):
        M = mb["M"].tolist()
        T = make_transform(M)
        ph = synth.ellipses_phase(T.points, T.m, mb["ellipses"])
        lame = np.array(mb["lame"])
        ip = perm_between(T.points, B.points(i))
        for l, eb in enumerate(loads3()):
            r = E.basic_scheme(M, ph, lame, E.default_reference(lame), eb[:2, :2], transform=T, fixed_iters=3)
            assert rel_err(B.strain(i, l), tensors_to_fields(r.eps[:, :, ip])) < 1e-10, (seeds[i], l)
            assert np.allclose(B.history(i, l), r.history, rtol=1e-9), (seeds[i], l)
            assert np.allclose(B.cauchy_history(i, l)[:3], r.cauchy, rtol=1e-9), (seeds[i], l)
            assert np.allclose(out["mean_stress"][i, l][:2, :2], r.mean_stress, rtol=1e-10, atol=1e-14)


def test_batch_equals_single_pattern_solver():
    """FP64 to 1e-8: each member's iterations and mean stress equal the single-pattern solver's."""
    seeds = [4000, 4001, 4002, 4003, 4004, 4005]
    say("batch vs solver", seeds)
    B, mbs = make_batch(seeds, precision=ahom.FP64, tol=1e-8, max_iter=5000)
    out = B.solve(loads3(), allow=(ahom.AHOM_OK,))
    for i, mb in enumerate(mbs):
        P = ahom.Pattern(mb["M"])
        S = ahom.Solver(P, precision=ahom.FP64, tol=1e-8, max_iter=5000)
        S.set_material(np.array(mb["lame"]), synth.ellipses_phase(P.points(), P.m, mb["ellipses"]))
        o = S.solve(loads3(), allow=(ahom.AHOM_OK,))
        assert np.all(np.abs(out["iters"][i] - o["iters"]) <= 1), (seeds[i], out["iters"][i], o["iters"])
        assert rel_err(out["mean_stress"][i], o["mean_stress"]) < 1e-7, seeds[i]


def test_batch_group_barrier_timeout_ends_cleanly(monkeypatch):
    """Failure handling forced from the host: a zero wait limit at the group
    barriers makes every barrier that does not find all arrivals at once give
    up.  The launch must still end; such items report status 3 (and the call
    AHOM_E_DEVICE); every item that reports status 0 equals the normal run."""
    seeds = [4000, 4001, 4002, 4003]
    say("batch group time-out", seeds)
    B, _ = make_batch(seeds, precision=ahom.FP64, tol=1e-8, max_iter=5000)
    ref = B.solve(loads3(), allow=(ahom.AHOM_OK,))
    assert np.all(ref["item_status"] == 0)
    del B
    monkeypatch.setenv("AHOM_BATCH_GROUP_WAIT", "0")
    B, _ = make_batch(seeds, precision=ahom.FP64, tol=1e-8, max_iter=5000)
    out = B.solve(loads3(), allow=(ahom.AHOM_OK, ahom.AHOM_W_NOT_CONVERGED, ahom.AHOM_E_DEVICE))
    st = out["item_status"]
    print("statuses", st.tolist(), flush=True)
    assert set(np.unique(st).tolist()) <= {0, 3}
    ok = st == 0
    assert np.array_equal(out["iters"][ok], ref["iters"][ok])
    assert np.allclose(out["mean_stress"][ok], ref["mean_stress"][ok], rtol=1e-12, atol=0.0)


def test_batch_fp32_strain_fields_match_fp64():
    """FP32 + restarts to 1e-6: each item's strain field (FP64 base + FP32
    correction, read back by ahom_batch_strain) against an FP64 batch solved
    to 1e-10 on the same members."""
    seeds = list(range(4100, 4108))
    say("batch fp32 strain vs fp64", seeds)
    B32, _ = make_batch(seeds, precision=ahom.FP32_MIXED, tol=1e-6, max_iter=5000)
    o32 = B32.solve(loads3(), allow=(ahom.AHOM_OK,))
    assert B32.last_timing()[1] >= len(seeds)
    B64, _ = make_batch(seeds, precision=ahom.FP64, tol=1e-10, max_iter=5000)
    B64.solve(loads3(), allow=(ahom.AHOM_OK,))
    worst = 0.0
    for i in range(len(seeds)):
        for l in range(3):
            a = B32.strain(i, l)
            b = B64.strain(i, l)
            e = np.abs(a - b).max() / np.abs(b).max()
            worst = max(worst, e)
            assert np.all(np.isfinite(a))
    print(f"worst strain error {worst:.2e}, FP32 iterations {int(o32['iters'].min())}..{int(o32['iters'].max())}",
          flush=True)
    assert worst < 1e-4


def test_batch_restart_rounds_beyond_the_graph():
    """FP32 with restart factor 0.5 (a restart per halving of the residual):
    the first solve runs the rounds beyond the two a graph holds from the
    host, the next capture plans for all of them; eager and graph results
    agree bit for bit and every item converges."""
    seeds = list(range(4100, 4106))
    say("batch restart rounds beyond the graph", seeds)
    B, _ = make_batch(seeds, precision=ahom.FP32_MIXED, tol=1e-6, max_iter=5000, refine=0.5)
    ref = B.solve(loads3(), use_graph=False, allow=(ahom.AHOM_OK,))
    n_restart = B.last_timing()[1]
    print("restarts", n_restart, "iterations", ref["iters"].min(), "..", ref["iters"].max(), flush=True)
    assert n_restart > 2 * len(seeds) * 3
    assert np.all(ref["item_status"] == 0) and np.all(ref["resid"] <= 1e-6)
    for k in range(2):
        out = B.solve(loads3(), use_graph=True, allow=(ahom.AHOM_OK,))
        assert B.last_timing()[1] == n_restart, k
        assert np.array_equal(out["iters"], ref["iters"]), k
        assert np.array_equal(out["mean_stress"], ref["mean_stress"]), k
        assert np.array_equal(out["resid"], ref["resid"]), k


def test_batch_graph_replays_equal_eager():
    """FP32 + restarts: three graph replays reproduce the eager launch bit for bit."""
    seeds = list(range(4100, 4116))
    say("batch graph replays", seeds)
    B, _ = make_batch(seeds, precision=ahom.FP32_MIXED, tol=1e-6, max_iter=5000)
    ref = B.solve(loads3(), use_graph=False, allow=(ahom.AHOM_OK,))
    assert B.last_timing()[1] >= 1
    for k in range(3):
        out = B.solve(loads3(), use_graph=True, allow=(ahom.AHOM_OK,))
        assert np.array_equal(out["iters"], ref["iters"]), k
        assert np.array_equal(out["mean_stress"], ref["mean_stress"]), k
        assert np.array_equal(out["resid"], ref["resid"]), k
        # eager work between replays
        P = ahom.Pattern([[8, 0], [2, 8]])
        S = ahom.Solver(P, tol=0.0, max_iter=2)
        S.set_material([[1.0, 1.0], [2.0, 2.0]], (np.arange(P.m) % 2).astype(np.uint8))
        S.solve(np.eye(3)[None])
    s0 = B.strain(0, 0)
    assert np.all(np.isfinite(s0))


def test_batch_512_members_fp32_against_oracle_samples():
    """The full workload: 512 members x 3 loads, FP32 + FP64 residual, tol 1e-6, graph launch."""
    gold = json.load(open(os.path.join(GOLD, "batch_c4.json")))
    seeds = list(range(4000, 4512))
    say("batch 512 members fp32", len(seeds))
    B, mbs = make_batch(seeds, precision=ahom.FP32_MIXED, tol=1e-6, max_iter=5000)
    out = B.solve(loads3(), use_graph=True, allow=(ahom.AHOM_OK,))
    ms, restarts = B.last_timing()
    pts = sum(B.info(i)[0] for i in range(len(seeds)))
    print(f"512 members, {pts} points, device {ms:.1f} ms, restarts {restarts}, "
          f"iterations {int(out['iters'].min())}..{int(out['iters'].max())}", flush=True)
    assert np.all(out["item_status"] == 0)
    assert np.all(out["resid"] <= 1e-6)
    assert all(0 <= B.variant(i) < 4 for i in range(len(seeds)))
    for s, g in gold["members"].items():
        i = seeds.index(int(s))
        for l in range(3):
            ref = np.array(g["loads"][l]["mean_stress"])
            got = out["mean_stress"][i, l][:2, :2]
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print("seed", s, "m", g["m"], "load", l, "iters", out["iters"][i, l], "oracle", g["loads"][l]["iters"],
                  f"mean-stress error {err:.2e}", flush=True)
            assert err < 1e-5
