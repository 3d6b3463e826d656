"""GPU parity of the restart score and of the batched persistent STGD.

Bars:
* score (FP32 rows, FP32 products, FP64 sums across batches) within 1e-5 of
  the oracle's restart_score, relative to |score| + ||T||^2;
* batched runs in the default tile layout are bit-identical to otm_sgd_run of
  the same problem and restarts (same kernel body, same arithmetic order);
* the other tile layout (forced through the tuning cache) changes only the
  order of the column-sum reduction: factor error <= 1e-4 against the oracle
  run (the FP32 run bar) and <= 1e-5 against the default layout;
* best restart = argmin of the scores; graph replays bit-identical to the
  eager run.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_round, host, padded, phi_cols, rel, to_dev

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu

BATCH, PASSES, BETA0, TAU = 100, 2, 0.01, 50.0


def _problem(n, k, seed, three, restarts):
    g = np.random.default_rng(seed)
    scale = 0.3
    YA = f32_round(g.standard_normal((n, k)) * scale + 0.2)
    YB = f32_round(g.standard_normal((n, k)) * scale + 0.1) if three else YA
    YC = f32_round(g.standard_normal((n, k)) * scale - 0.1) if three else YA
    ybar = f32_round(np.stack([YA.mean(0), YB.mean(0), YC.mean(0)]))
    Phi0 = [f32_round(synth.initial_factors(k, seed=seed, restart=r) * 1.2) for r in range(restarts)]
    perms = [synth.permutations(n, PASSES, seed=seed, sub=r) for r in range(restarts)]
    return dict(YA=YA, YB=YB, YC=YC, ybar=ybar, Phi0=Phi0, perms=perms, k=k, n=n, alpha0=0.5 if three else 0.1)


def _device_problem(P):
    k = P["k"]
    ldy = otm.default_ldy(k)
    A = padded(P["YA"], ldy, torch.float32)
    B = A if P["YB"] is P["YA"] else padded(P["YB"], ldy, torch.float32)
    C = A if P["YC"] is P["YA"] else padded(P["YC"], ldy, torch.float32)
    Phi0 = to_dev(np.stack([x.T for x in P["Phi0"]]), torch.float32)
    perms = to_dev(np.stack(P["perms"]), torch.int32)
    return otm.Problem(A, B, C, to_dev(P["ybar"]), Phi0, k, P["alpha0"], perms)


def _params():
    return otm.SgdParams(k=1, batch=BATCH, passes=PASSES, y_dtype=otm.F32, beta0=BETA0, beta_tau=TAU)


SHAPES = [(150, 5, True), (777, 16, False), (1000, 33, True), (2100, 64, False), (640, 100, True),
          (333, 128, False), (90, 12, True)]


@pytest.mark.parametrize("k,three", [(7, True), (16, False), (50, True), (128, False)])
def test_score_vs_oracle(k, three):
    P = _problem(333, k, seed=k, three=three, restarts=3)
    D = _device_problem(P)
    p = otm.SgdParams(k=k, batch=BATCH, y_dtype=otm.F32, alpha0=P["alpha0"])
    sc = host(otm.sgd_score(p, P["n"], D.YA, D.YB, D.YC, D.ybar3, D.Phi0.contiguous(), restarts=3))
    T = oracle.whitened_tensor(P["YA"], P["YB"], P["YC"], P["ybar"], P["alpha0"])
    tt = float(np.sum(T * T))
    ref = np.array([oracle.restart_score(T, Phi) for Phi in P["Phi0"]])
    assert np.all(np.abs(sc - ref) <= 1e-5 * (np.abs(ref) + tt)), (sc, ref)


def _run_batched(problems, restarts, cache=None):
    D = [_device_problem(P) for P in problems]
    run = otm.BatchedRun(D, restarts, _params(), tune_cache=cache)
    run.run()
    torch.cuda.synchronize()
    return D, run


def test_batched_equals_single_runs_and_scores():
    restarts = 3
    problems = [_problem(n, k, seed=100 + i, three=t, restarts=restarts) for i, (n, k, t) in enumerate(SHAPES)]
    D, run = _run_batched(problems, restarts)
    assert int(run.nonfinite.item()) == 0
    for i, (P, d) in enumerate(zip(problems, D)):
        # the single-problem entry point on the same inputs
        Phi = d.Phi0.clone()
        p = otm.SgdParams(k=P["k"], batch=BATCH, passes=PASSES, y_dtype=otm.F32, alpha0=P["alpha0"], beta0=BETA0,
                          beta_tau=TAU)
        otm.sgd_run(p, P["n"], d.YA, d.YB, d.YC, d.ybar3, d.perms, Phi, restarts=restarts,
                    perm_stride=d.perms[0].numel())
        torch.cuda.synchronize()
        assert torch.equal(Phi, run.Phi[i]), f"problem {i}"
        # scores of the final factors against the oracle's, best = argmin
        T = oracle.whitened_tensor(P["YA"], P["YB"], P["YC"], P["ybar"], P["alpha0"])
        tt = float(np.sum(T * T))
        got = host(run.scores[i])
        ref = np.array([oracle.restart_score(T, phi_cols(run.Phi[i][r])) for r in range(restarts)])
        assert np.all(np.abs(got - ref) <= 1e-5 * (np.abs(ref) + tt)), (i, got, ref)
        assert int(run.best[i].item()) == int(np.argmin(got))


def test_batched_same_result_with_every_group_on_its_own_queue(tmp_path):
    """With 16 hardware queues every variant group gets a branch of its own and
    a whole-device grid; the jobs' arithmetic does not depend on scheduling, so
    the factors and scores equal (bit for bit) those of the default 4 queues
    (groups sharing branches).  The 16-queue run is a child process: the queue
    count is fixed when the HIP runtime starts."""
    import subprocess
    import sys
    restarts = 3
    problems = [_problem(n, k, seed=100 + i, three=t, restarts=restarts) for i, (n, k, t) in enumerate(SHAPES)]
    _, run = _run_batched(problems, restarts)
    out = tmp_path / "child.npz"
    env = dict(os.environ, GPU_MAX_HW_QUEUES="16")
    child = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_child.py")
    r = subprocess.run([sys.executable, child, str(out)], env=env, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    got = np.load(out)
    for i in range(len(problems)):
        np.testing.assert_array_equal(got[f"phi{i}"], run.Phi[i].cpu().numpy())
        np.testing.assert_array_equal(got[f"score{i}"], run.scores[i].cpu().numpy())


def test_batched_vs_oracle_runs_both_layouts(tmp_path):
    restarts = 2
    problems = [_problem(n, k, seed=200 + i, three=t, restarts=restarts)
                for i, (n, k, t) in enumerate([(500, 12, True), (400, 40, False), (300, 100, True)])]
    ref = oracle.sgd_batched(problems, batch=BATCH, beta0=BETA0, tau=TAU)
    _, run0 = _run_batched(problems, restarts)
    cache = tmp_path / "tune.txt"
    cache.write_text("".join(f"sgd_batched f32 kp={kp} views={v} layout=1 us_step=2,1\n"
                             for kp in range(16, 129, 16) for v in (1, 3)))
    _, run1 = _run_batched(problems, restarts, cache=str(cache))
    for i in range(len(problems)):
        for r in range(restarts):
            want = ref[i][0][r]
            assert rel(phi_cols(run0.Phi[i][r]), want) < 1e-4
            assert rel(phi_cols(run1.Phi[i][r]), want) < 1e-4
            assert rel(host(run1.Phi[i][r]), host(run0.Phi[i][r])) < 1e-5
        assert int(run0.best[i].item()) == ref[i][2] or abs(ref[i][1][ref[i][2]] - ref[i][1][int(run0.best[i].item())]) \
            < 1e-6 * abs(ref[i][1][ref[i][2]])


def test_graph_replays_match_eager():
    restarts = 2
    problems = [_problem(n, k, seed=300 + i, three=t, restarts=restarts)
                for i, (n, k, t) in enumerate([(800, 24, True), (1200, 64, False), (256, 100, True)])]
    D, run = _run_batched(problems, restarts)
    eager = [x.clone() for x in run.Phi]
    eager_scores = [x.clone() for x in run.scores]
    eager_best = run.best.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        run.capture(s)
    for rep in range(3):
        for x in run.Phi:
            x.fill_(float("nan"))
        run.best.fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            run.replay(s)
        s.synchronize()
        # unrelated eager work between replays
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
        for i in range(len(problems)):
            assert torch.equal(run.Phi[i], eager[i]), (rep, i)
            assert torch.equal(run.scores[i], eager_scores[i]), (rep, i)
        assert torch.equal(run.best, eager_best)
    run.close()


def test_nonfinite_flag_is_set_and_cleared():
    P = _problem(400, 20, seed=5, three=True, restarts=1)
    d = _device_problem(P)
    hot = otm.SgdParams(k=1, batch=BATCH, passes=PASSES, y_dtype=otm.F32, beta0=1e6, beta_tau=1e9)
    run = otm.BatchedRun([d], 1, hot)
    run.run()
    torch.cuda.synchronize()
    assert int(run.nonfinite.item()) == 1
    cold = otm.BatchedRun([d], 1, _params())
    cold.nonfinite.fill_(1)          # a stale flag is cleared by the run
    cold.run()
    torch.cuda.synchronize()
    assert int(cold.nonfinite.item()) == 0


def test_autotune_writes_cache_and_plans_with_it(tmp_path):
    cache = str(tmp_path / "tune.txt")
    otm.sgd_autotune([16, 100], BATCH, cache)
    torch.cuda.synchronize()
    lines = [l.split() for l in open(cache) if l.startswith("sgd_batched")]
    keys = {(l[2], l[3]) for l in lines}
    assert keys == {("kp=16", "views=1"), ("kp=16", "views=3"), ("kp=112", "views=1"), ("kp=112", "views=3")}
    for l in lines:
        t0, t1 = (float(x) for x in l[5].split("=")[1].split(","))
        assert t0 > 0 and t1 > 0
        assert l[4] == ("layout=1" if t1 < t0 else "layout=0")
    problems = [_problem(500, 16, seed=7, three=False, restarts=2), _problem(300, 100, seed=8, three=True, restarts=2)]
    ref = oracle.sgd_batched(problems, batch=BATCH, beta0=BETA0, tau=TAU)
    _, run = _run_batched(problems, 2, cache=cache)
    for i in range(2):
        for r in range(2):
            assert rel(phi_cols(run.Phi[i][r]), ref[i][0][r]) < 1e-4
