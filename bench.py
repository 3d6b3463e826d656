#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: mixed-membership graph, n = 100000 nodes (X/A = 50000/50000),
k = 100 communities, alpha0 = 0.5, p = 0.05, q = 0.001, seeded synthetic.
One step = the whole path on one batch of input already resident in HBM:
power-iterated M2 sketch (FP64) -> randomized whitener (FP64) -> whitening
SpMM (BF16 W and Y, FP32 accumulation) -> STGD run (50 passes, mini-batch 100,
BF16 matrix-core contractions, FP32 master with the plain update) -> memberships
(FP64).

value = whitened samples pushed through STGD per second of a whole step
(n_X * passes / step time).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = dict(name="mmsb_large", n=100000, n_x=50000, k=100, alpha0=0.5, p=0.05, q=0.001, batch=100, passes=50,
                q_power=3, beta0=1e-3, beta_tau=2500.0, tau_pi=0.1, compensated=False)
PEAK_BF16 = 2.5e15          # dense MFMA bf16, FLOP/s
PEAK_HBM = 8.0e12           # bytes/s
# HBM counters of the STGD kernel (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE), per launch,
# valid only for the kernel source they were taken on.
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sgd_kernel_mmsb_large_counters.json")
WHITEN_COUNTERS_FILE = os.path.join(ROOT, "profiles", "whiten_kernel_counters.json")


def sgd_flops(n: int, batch: int, k: int, passes: int) -> float:
    """Algorithmic flops of one STGD run: per step 2 PA/PB products (2*2*B*k^2),
    YC^T Q (2*B*k^2), Phi^T Phi and Phi (G*G) (2*2*k^3)."""
    full, rem = divmod(n, batch)
    per_pass = full * (6.0 * batch * k * k + 4.0 * k ** 3)
    if rem:
        per_pass += 6.0 * rem * k * k + 4.0 * k ** 3
    return per_pass * passes


def kernel_hash(files=("stgd.hip", "stgd_kernel.h")) -> str:
    """Hash of a kernel's sources without comments and blank lines (the
    counters are valid for this code only); by default the STGD kernel's."""
    import re
    h = hashlib.sha256()
    for f in files:
        src = open(os.path.join(ROOT, "paper_1309_0787_amd", "csrc", f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(line.rstrip() for line in src.splitlines() if line.strip()).encode())
    return h.hexdigest()[:16]


def counters_traffic():
    try:
        c = json.load(open(COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if c.get("kernel_sha256_16") != kernel_hash():
        return None
    return c.get("bytes_per_launch")


def whiten_traffic(workload: str):
    """HBM bytes per launch of the whitening SpMM on `workload` ("documents":
    one view; "graph": the benchmark graph's block) from the committed
    counters, or None when spmm.hip has changed since they were taken."""
    try:
        c = json.load(open(WHITEN_COUNTERS_FILE))
    except (OSError, ValueError):
        return None
    if c.get("kernel_sha256_16") != kernel_hash(("spmm.hip",)):
        return None
    return c.get("workloads", {}).get(workload, {}).get("bytes_per_launch")


def cpu_baseline(inst, w):
    """The FP64 oracle on the same workload (whole path, one decomposition).
    Returns the baseline record and the oracle's results (for the per-result
    errors of the GPU path)."""
    import numpy as np
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # noqa: BLE001
        cores = os.cpu_count()
    k = w["k"]
    S = synth.projection(inst.C.n_cols, 2 * k, seed=1)
    perms = synth.permutations(inst.C.n_rows, w["passes"], seed=2)
    Phi0 = synth.initial_factors(k, seed=4)
    t0 = time.perf_counter()
    Q, O = oracle.power_sketch(inst.C, S, w["alpha0"], False, w["q_power"])
    W, _ = oracle.whitener_rsvd(O, Q, k)
    Y, ybar = oracle.whiten(inst.C, W, False)
    yb = np.stack([ybar] * 3)
    Phi = oracle.sgd_run(Y, Y, Y, yb, Phi0, perms, w["batch"], w["beta0"], w["beta_tau"], w["alpha0"])
    Pi = oracle.recover_pi(Y, Phi, w["tau_pi"])
    el = time.perf_counter() - t0
    rec = {"value": inst.C.n_rows * w["passes"] / el, "unit": "samples/s", "cores": int(cores), "kind": "oracle",
           "sample": f"whole path once on the same graph (FP64): sketch q={w['q_power']}, whitener, whitening, "
                     f"{w['passes']} STGD passes, memberships; {el:.1f} s"}
    return rec, dict(W=W, Y=Y, ybar=yb, Phi=Phi, Pi=Pi, Phi0=Phi0, perms=perms)


def _rel(a, b) -> float:
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _host(t):
    return t.detach().to("cpu", dtype=__import__("torch").float64).numpy()


def errors_graph(res, ores, w, inst=None) -> dict:
    """Error of each result of the benchmark step (BF16 W/Y and contractions,
    FP64 sketch/whitener/post) against the FP64 oracle's whole path on the
    same graph, projection, initial factors and permutations; then FP32 runs
    with and without the compensated update on the oracle's rows (FP32
    rounded) against the oracle run on the same rows."""
    import numpy as np
    import torch
    from paper_1309_0787_amd import otm
    k, n = w["k"], ores["Y"].shape[0]
    Yg = _host(res.Y[0])[:, :k]
    row_err = np.linalg.norm(Yg - ores["Y"], axis=1) / np.maximum(np.linalg.norm(ores["Y"], axis=1), 1e-300)
    Pi_g = _host(res.Pi)
    out = {"W": _rel(_host(res.W), ores["W"]),
           "Y": _rel(Yg, ores["Y"]), "Y_row_max": float(row_err.max()),
           "Phi": _rel(_host(res.Phi[0]).T, ores["Phi"]),
           "Pi": _rel(Pi_g, ores["Pi"]), "Pi_max_abs": float(np.abs(Pi_g - ores["Pi"]).max()),
           "precision": "W FP64 (BF16 copy for the SpMM), Y BF16, STGD BF16 operands / FP32 accumulate and "
                        "plain FP32 master, Pi FP64 arithmetic; Y and Phi include the BF16 rounding"}
    dev = res.W.device
    permd = torch.as_tensor(ores["perms"], device=dev)
    # the same BF16 run with the compensated master update, on the step's own
    # BF16 rows: factor error and microseconds per step beside the plain one
    Yb = res.Y[0]
    ybg = res.ybar3
    pb = otm.SgdParams(k=k, batch=w["batch"], passes=w["passes"], y_dtype=otm.BF16, compensated=True,
                       alpha0=w["alpha0"], beta0=w["beta0"], beta_tau=w["beta_tau"], ldy=Yb.shape[1])
    Phi = torch.as_tensor(ores["Phi0"].T.copy(), dtype=torch.float32, device=dev)[None].contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    otm.sgd_run(pb, n, Yb, Yb, Yb, ybg, permd, Phi)
    e1.record()
    torch.cuda.synchronize()
    steps = w["passes"] * ((n + w["batch"] - 1) // w["batch"])
    out["Phi_bf16_compensated"] = _rel(_host(Phi[0]).T, ores["Phi"])
    out["stgd_us_per_step_bf16_compensated"] = e0.elapsed_time(e1) * 1e3 / steps
    ldy = otm.default_ldy(k)
    Y32 = torch.zeros((n, ldy), dtype=torch.float32, device=dev)
    Y32[:, :k] = torch.as_tensor(ores["Y"], dtype=torch.float32, device=dev)
    yb3 = torch.as_tensor(ores["ybar"].astype(np.float32).reshape(-1), device=dev)
    for comp in (True, False):
        p = otm.SgdParams(k=k, batch=w["batch"], passes=w["passes"], y_dtype=otm.F32, compensated=comp,
                          alpha0=w["alpha0"], beta0=w["beta0"], beta_tau=w["beta_tau"], ldy=ldy)
        Phi = torch.as_tensor(ores["Phi0"].T.copy(), dtype=torch.float32, device=dev)[None].contiguous()
        otm.sgd_run(p, n, Y32, Y32, Y32, yb3, permd, Phi)
        torch.cuda.synchronize()
        out["Phi_fp32_" + ("compensated" if comp else "plain")] = _rel(_host(Phi[0]).T, ores["Phi"])
    out["fp32_steps"] = w["passes"] * ((n + w["batch"] - 1) // w["batch"])
    if inst is not None:   # the method's own limit on this graph: the oracle's memberships against the planted
        out["recovery_error_oracle"] = recovery_error(torch.as_tensor(ores["Pi"]), inst.pi[inst.X])
        out["recovery_error_gpu"] = recovery_error(res.Pi, inst.pi[inst.X])
    return out


DOCS = dict(k=50, alpha0=1.0, q_power=3, batch=100, passes=50, beta0=1e-3, beta_tau=2500.0)


def errors_documents(inst) -> dict:
    """The document workload (d = 10000, k = 50, 1e5 documents, three views,
    FP32 W/Y/STGD, FP64 sketch/whitener/topics) through the whole path on the
    GPU, each result against the FP64 oracle's path on the same inputs:
    W, the three views' Y, Phi, the topic-word matrix and the weights."""
    import numpy as np
    import torch
    import oracle
    import synth
    from paper_1309_0787_amd import otm, pipeline
    w = DOCS
    dev = torch.device("cuda:0")
    k, n = w["k"], inst.C.n_rows
    S = synth.projection(inst.C.n_cols, 2 * k, seed=1)
    perms = synth.permutations(n, w["passes"], seed=2)
    Phi0 = synth.initial_factors(k, seed=4)
    views = [otm.DeviceCSR.from_host(v, dev) for v in inst.views]
    C, CT = otm.DeviceCSR.from_host(inst.C, dev), otm.DeviceCSR.from_host(inst.CT, dev)
    cfg = pipeline.FitConfig(k=k, alpha0=w["alpha0"], normalize=True, q_power=w["q_power"], y_dtype=otm.F32,
                             batch=w["batch"], passes=w["passes"], beta0=w["beta0"], beta_tau=w["beta_tau"],
                             topics=True)
    Phi = torch.as_tensor(Phi0.T.copy(), dtype=torch.float32, device=dev)[None].contiguous()
    tm = pipeline.Timer(True)
    res = pipeline.fit(views, C, CT, torch.as_tensor(S, device=dev), Phi, torch.as_tensor(perms, device=dev), cfg,
                       timer=tm)
    torch.cuda.synchronize()
    gpu_ms = {a: round(b, 3) for a, b in tm.spans_ms().items()}
    t0 = time.perf_counter()
    Q, O = oracle.power_sketch(inst.C, S, w["alpha0"], True, w["q_power"])
    Wo, _ = oracle.whitener_rsvd(O, Q, k)
    Ys = [oracle.whiten(v, Wo, True) for v in inst.views]
    yb = np.stack([y[1] for y in Ys])
    Phio = oracle.sgd_run(Ys[0][0], Ys[1][0], Ys[2][0], yb, Phi0, perms, w["batch"], w["beta0"], w["beta_tau"],
                          w["alpha0"])
    muo, aho, _ = oracle.unwhiten_topics(Wo, Phio)
    el = time.perf_counter() - t0
    mug = _host(res.mu)
    return {"workload": f"documents d={inst.C.n_cols}, k={k}, n={n}, three views, FP32, {w['passes']} passes",
            "W": _rel(_host(res.W), Wo),
            "Y": max(_rel(_host(res.Y[i])[:, :k], Ys[i][0]) for i in range(3)),
            "Phi": _rel(_host(res.Phi[0]).T, Phio),
            "mu": _rel(mug, muo), "mu_max_abs": float(np.abs(mug - muo).max()),
            "alpha_hat": _rel(_host(res.alpha_hat), aho),
            "gpu_stage_ms": gpu_ms, "oracle_s": round(el, 2)}


# beta0 3e-4: at 1e-3 the three-view problems with k = 100 and alpha0 = 1 diverge
BATCHED = dict(problems=256, ks=(16, 32, 64, 100, 128), n_lo=1e3, n_hi=1e5, restarts=8, passes=50, batch=100,
               beta0=3e-4, beta_tau=2500.0)
PEAK_FP32_MFMA = 157.3e12


def bench_batched(steps: int, warmup: int, real_rows=None) -> dict:
    """Many decompositions with restarts in one launch sequence (FP32): 256
    problems, k uniform over {16, 32, 64, 100, 128}, n log-uniform in
    [1e3, 1e5], half three-view (documents) and half one-view (graphs), 8
    restarts each; the tile layouts come from the autotuner (run first, timed
    separately).  The launch sequence is captured into a graph once and the
    replays are timed (HIP events on the replay stream).  real_rows: the
    benchmark graph's whitened FP32 rows, for the equal-work check (one k = 100
    one-view job on them and on planted rows of the same shape)."""
    import tempfile

    import torch
    from paper_1309_0787_amd import otm
    import synth

    w = BATCHED
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    table = synth.batched_table(w["problems"], w["ks"], w["n_lo"], w["n_hi"])
    problems = []
    for i, sp in enumerate(table):
        k, n = sp["k"], sp["n"]
        ldy = otm.default_ldy(k)
        YA, YB, YC, _ = synth.planted_views(n, k, sp["alpha0"], sp["views"], sub=i, device=dev, ldy=ldy)
        ybar = torch.stack([YA[:, :k].mean(0), YB[:, :k].mean(0), YC[:, :k].mean(0)]).contiguous()
        Phi0 = torch.as_tensor(np.ascontiguousarray(np.stack([synth.initial_factors(k, restart=r + 100 * i).T
                                                               for r in range(w["restarts"])])),
                               dtype=torch.float32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + i)
        perms = torch.argsort(torch.rand((w["passes"], n), device=dev, generator=g), dim=1).to(torch.int32)
        problems.append(otm.Problem(YA, YB, YC, ybar, Phi0, k, sp["alpha0"], perms))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    p = otm.SgdParams(k=1, batch=w["batch"], passes=w["passes"], y_dtype=otm.F32, beta0=w["beta0"],
                      beta_tau=w["beta_tau"])
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")
        t0 = time.perf_counter()
        otm.sgd_autotune(sorted(set(w["ks"])), w["batch"], cache)
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
        tuned = open(cache).read().splitlines()[1:]
        run = otm.BatchedRun(problems, w["restarts"], p, tune_cache=cache)
    s = torch.cuda.Stream()
    run.capture(s)
    for _ in range(warmup):
        run.replay(s)
    s.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(steps):
        run.replay(s)
    ev1.record(s)
    s.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    samples = sum(sp["n"] for sp in table) * w["passes"] * w["restarts"]
    flops = 0.0
    for sp in table:
        full, rem = divmod(sp["n"], w["batch"])
        per_pass = full * (6.0 * w["batch"] * sp["k"] ** 2 + 4.0 * sp["k"] ** 3)
        if rem:
            per_pass += 6.0 * rem * sp["k"] ** 2 + 4.0 * sp["k"] ** 3
        flops += per_pass * (w["passes"] + 1) * w["restarts"]     # training passes + the scoring pass
    achieved = flops / (ms * 1e-3)
    out = {
        "workload": f"{w['problems']} problems, k in {list(w['ks'])}, n log-uniform [{int(w['n_lo'])}, {int(w['n_hi'])}], "
                    f"half three-view / half one-view, {w['restarts']} restarts, {w['passes']} passes, FP32, "
                    f"captured launch sequence replayed",
        "samples_per_s": samples / (ms * 1e-3), "ms_per_run": ms, "jobs": len(problems) * w["restarts"],
        "kernel_groups": run.groups,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA, "flops_per_run": flops},
        "nonfinite": int(run.nonfinite.item()), "generation_s": round(t_gen, 2), "autotune_s": round(t_tune, 2),
        "tuned_layouts": tuned,
    }
    run.close()
    if real_rows is not None:
        out["equal_work_check"] = _equal_work_check(real_rows)
    return out


def _equal_work_check(Yreal) -> dict:
    """One k = 100 one-view job (the benchmark graph's whitened rows, FP32,
    10 passes) against planted rows of the same shape: microseconds per step."""
    import torch
    from paper_1309_0787_amd import otm
    import synth
    dev = Yreal.device
    n, ldy = Yreal.shape
    k = 100
    res = {}
    for name in ("whitened_graph_rows", "planted_rows"):
        if name == "planted_rows":
            Y, _, _, _ = synth.planted_views(n, k, 0.5, 1, sub=7, device=dev, ldy=ldy)
        else:
            Y = Yreal
        ybar = torch.stack([Y[:, :k].mean(0)] * 3).contiguous()
        Phi0 = torch.as_tensor(synth.initial_factors(k, restart=3).T.copy(), dtype=torch.float32, device=dev)[None]
        pr = [otm.Problem(Y, Y, Y, ybar, Phi0.contiguous(), k, 0.5, None)]
        p = otm.SgdParams(k=1, batch=100, passes=10, y_dtype=otm.F32, beta0=3e-4, beta_tau=2500.0)
        run = otm.BatchedRun(pr, 1, p)
        run.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run.run()
        e1.record()
        torch.cuda.synchronize()
        steps = 11 * ((n + 99) // 100)       # 10 passes and the scoring pass
        res[name] = {"us_per_step": e0.elapsed_time(e1) * 1e3 / steps, "nonfinite": int(run.nonfinite.item())}
        run.close()
    return res


WARM = dict(instances=50000, exact_share=0.8, sampled_n=2000, epochs=6, batch=256, lr=1e-3, heldout=1000)


def train_warm_start(inst, pool_res, w) -> tuple:
    """The learned warm start trained on instances from the three workloads'
    generators: 80% exact-moment instances of block models drawn by
    the small graph, document and large graph generators (k = 10, 50, 100),
    20% sampled instances: seeded subsets of 2000 whitened rows of the
    benchmark graph with its planted directions as targets."""
    import torch
    from paper_1309_0787_amd import otm
    from paper_1309_0787_amd import warmstart as pws
    dev = torch.device("cuda:0")
    cfg = WARM
    k = w["k"]
    # planted directions of the benchmark graph in its whitened coordinates:
    # u_i = sqrt(ahat_i) W^T F_i, F = Pi_A^T P^T, ahat = 1/k
    W = pool_res.W.double().cpu().numpy()
    F = inst.pi[inst.A] @ inst.P.T
    U = (W.T @ F) / np.sqrt(k)
    Yp = pool_res.Y[0].float()
    pool = {"Y": Yp, "U": U, "lam": np.full(k, np.sqrt(k)), "alpha0": w["alpha0"]}
    g = np.random.default_rng(0)
    fams = list(pws.FAMILIES)
    specs = []
    for i in range(cfg["instances"]):
        if g.random() < cfg["exact_share"]:
            specs.append(dict(kind="exact", family=fams[int(g.integers(3))], seed=5000 + i))
        else:
            specs.append(dict(kind="sampled", seed=5000 + i, n=cfg["sampled_n"]))
    t0 = time.perf_counter()
    tr = pws.build_generated(specs, dev, sampled_pool=pool,
                             progress=lambda i: print(f"bench: warm start, {i} instances built", file=sys.stderr,
                                                      flush=True))
    warm = pws.WarmStart(dev, seed=3)
    _, _, X, tgt, _ = warm.prepare(tr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = warm.train(X, tgt, tr.ks, epochs=cfg["epochs"], batch=cfg["batch"], lr=cfg["lr"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"train_instances": len(specs), "exact": sum(s["kind"] == "exact" for s in specs),
            "epochs": cfg["epochs"], "build_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
            "adam_steps": len(losses), "final_loss": float(np.mean(losses[-20:]))}
    del X, tgt, tr
    return warm, info


def bench_heldout(warm) -> dict:
    """SGD iterations to R <= 1e-3 on 1000 held-out exact-moment instances
    (disjoint seeds; the three generators, k = 10, 50, 100), FP32, from the
    warm start and from random orthonormal factors, all instances of an arm in
    one batched launch per chunk of passes; R after each chunk from the
    batched kernel's restart score (R = 1 + score / ||T||^2, ||T||^2 =
    sum lambda^2)."""
    import torch
    from paper_1309_0787_amd import otm
    from paper_1309_0787_amd import warmstart as pws
    import synth
    dev = torch.device("cuda:0")
    cnt = WARM["heldout"]
    fams = list(pws.FAMILIES)
    g = np.random.default_rng(1)
    specs = [dict(kind="exact", family=fams[int(g.integers(3))], seed=900000 + i) for i in range(cnt)]
    hs = pws.build_generated(specs, dev, progress=lambda i: print(f"bench: held-out, {i} instances built",
                                                                  file=sys.stderr, flush=True))
    Pw = pws.warm_factors_batch(warm, hs)
    ks = hs.ks.cpu().numpy()
    rows, tnorm = [], []
    for i, sp in enumerate(specs):
        Y, _, lam = pws.generated_exact_instance(sp["family"], sp["seed"])
        k = Y.shape[0]
        ldy = otm.default_ldy(k)
        Yd = torch.zeros((k, ldy), dtype=torch.float32, device=dev)
        Yd[:, :k] = torch.as_tensor(Y, device=dev)
        rows.append((Yd, torch.stack([Yd[:, :k].mean(0)] * 3).contiguous(), k))
        tnorm.append(float(np.sum(lam ** 2)))
    tnorm = np.asarray(tnorm)
    chunks = [25, 25, 50, 100, 200, 400, 400, 800]
    beta0 = 0.02
    out = {}
    for arm in ("random", "warm"):
        if arm == "warm":
            phis = [Pw[i, :rows[i][2] ** 2].reshape(1, rows[i][2], rows[i][2]).clone() for i in range(cnt)]
        else:
            phis = [torch.as_tensor(synth.initial_factors(rows[i][2], seed=7, restart=i).T.copy(), dtype=torch.float32,
                                    device=dev)[None].contiguous() for i in range(cnt)]
        done = np.full(cnt, -1)
        steps = 0
        ms = 0.0
        for c in chunks:
            problems = [otm.Problem(Y, Y, Y, yb, phis[i], k, 0.0) for i, (Y, yb, k) in enumerate(rows)]
            p = otm.SgdParams(k=1, batch=100, passes=c, y_dtype=otm.F32, beta0=beta0, beta_tau=1e12)
            run = otm.BatchedRun(problems, 1, p)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run.run()
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            steps += c
            R = 1.0 + np.array([float(sc.item()) for sc in run.scores]) / tnorm
            newly = (done < 0) & (R <= 1e-3)
            done[newly] = steps
            phis = [ph.clone() for ph in run.Phi]
            run.close()
            print(f"bench: held-out {arm}, {steps} steps, {int((done > 0).sum())} reached 1e-3", file=sys.stderr,
                  flush=True)
        ok = done > 0
        out[arm] = {"success_rate": float(ok.mean()),
                    "median_steps_to_1e-3": float(np.median(done[ok])) if ok.any() else None,
                    "success_by_k": {int(kk): float(ok[ks == kk].mean()) for kk in sorted(set(ks.tolist()))},
                    "gpu_ms": round(ms, 1)}
    out["workload"] = (f"{cnt} held-out exact-moment instances (block-model limits of the three generators, k in "
                       f"{{10, 50, 100}}), FP32, full batch, beta {beta0}, up to {sum(chunks)} steps; "
                       f"iterations counted at chunk ends {list(np.cumsum(chunks))}")
    return out


def bench_time_to_loss(inst, C, CT, S, Phi_init, w, warm, warm_info) -> dict:
    """Time to the converged loss on the benchmark graph, four arms:
    {FP32, BF16} x {random: best of 8 random restarts in one launch; warm: the
    learned warm start as restart 0 beside 7 random restarts}, 100 passes
    each.  R of every restart at every pass end from snapshots (outside the
    timed stages), all against the FP32 arm's tensor.  Two thresholds: the
    best converged R over the arms plus 1e-3 (an arm stuck in a worse basin
    never reaches it: null), and the worst arm's converged R plus 1e-3, which
    every arm reaches.  An arm's time to a threshold is its prefix (sketch,
    whitener, whitening, warm start) plus its STGD time up to the first pass
    whose best restart reaches it.  Memberships of each arm's best restart
    against the planted ones."""
    import torch
    from paper_1309_0787_amd import otm, pipeline
    import synth
    dev = torch.device("cuda:0")
    k, R, passes = w["k"], 8, 100
    n = inst.C.n_rows
    perms = torch.as_tensor(np.stack([synth.permutations(n, passes, seed=2, sub=r) for r in range(R)]), device=dev)
    Phi_rand = torch.as_tensor(np.stack([synth.initial_factors(k, seed=4, restart=r).T for r in range(R)]),
                               dtype=torch.float32, device=dev).contiguous()
    runs, T_ref = {}, None
    pi_true = inst.pi[inst.X]
    for name, ydt, use_warm in (("fp32_random", otm.F32, False), ("fp32_warm", otm.F32, True),
                                ("bf16_random", otm.BF16, False), ("bf16_warm", otm.BF16, True)):
        # FP32 arms with the compensated master update, BF16 arms with the
        # plain one (as the benchmark step)
        cfg = pipeline.FitConfig(k=k, alpha0=w["alpha0"], normalize=False, q_power=w["q_power"], y_dtype=ydt,
                                 batch=w["batch"], passes=passes, beta0=w["beta0"], beta_tau=w["beta_tau"],
                                 tau_pi=w["tau_pi"], restarts=R, compensated=(ydt == otm.F32))
        Phi = Phi_rand.clone()
        tm = pipeline.Timer(True)
        res = pipeline.fit([C], C, CT, S, Phi, perms, cfg, snapshots=True, timer=tm, warm=warm if use_warm else None)
        torch.cuda.synchronize()
        if T_ref is None:
            T_ref = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, w["alpha0"])
        Rs = otm.residual(T_ref, res.snapshots.reshape(-1, k, k).contiguous()).cpu().numpy().reshape(R, passes)
        best_r = int(np.argmin(Rs[:, -1]))
        Pi = otm.recover_pi(res.Y[0], k, res.Phi[best_r], tau=w["tau_pi"])
        runs[name] = dict(stages=tm.spans_ms(), Rs=Rs, best=best_r, rec=recovery_error(Pi, pi_true))
    finals = [float(r["Rs"][:, -1].min()) for r in runs.values()]
    r_inf = min(finals)
    thr = r_inf + 1e-3
    thr_common = max(finals) + 1e-3
    out = {"threshold": thr, "R_inf": r_inf, "threshold_common": thr_common, "passes": passes, "restarts": R}

    def first_pass(best_by_pass, t):
        hit = np.nonzero(best_by_pass <= t)[0]
        return int(hit[0]) + 1 if hit.size else None

    for name, r in runs.items():
        best_by_pass = r["Rs"].min(axis=0)
        pz, pc = first_pass(best_by_pass, thr), first_pass(best_by_pass, thr_common)
        st = r["stages"]
        prefix = st.get("sketch", 0) + st.get("whitener", 0) + st.get("whiten", 0) + st.get("warm", 0)
        out[name] = {"time_to_loss_ms": (prefix + st["stgd"] * pz / passes) if pz else None,
                     "passes_to_loss": pz,
                     "time_to_common_ms": (prefix + st["stgd"] * pc / passes) if pc else None,
                     "passes_to_common": pc, "R_final_best": float(r["Rs"][:, -1].min()),
                     "R_pass1_best": float(r["Rs"][:, 0].min()), "R_final_warm_restart": float(r["Rs"][0, -1]),
                     "best_restart": r["best"], "stgd_ms": round(st["stgd"], 2), "prefix_ms": round(prefix, 2),
                     "recovery_error": r["rec"]}
    def ratio(a, b, key):
        x, y = out[a][key], out[b][key]
        return (x / y) if (x and y) else None
    for key, tag in (("time_to_loss_ms", ""), ("time_to_common_ms", "_common")):
        out["speedup_warm_fp32" + tag] = ratio("fp32_random", "fp32_warm", key)
        out["speedup_warm_bf16" + tag] = ratio("bf16_random", "bf16_warm", key)
        out["speedup_bf16_warm_vs_fp32_random" + tag] = ratio("fp32_random", "bf16_warm", key)
    out["warm_start"] = warm_info
    return out


def bench_spmm(inst, reps: int = 20) -> dict:
    """Whitening SpMM on the document workload (d = 10000, k = 50, 1e5
    documents of Poisson(200) tokens, three views, FP32 counts, FP32 W and Y):
    the HBM-bound case.  W is a seeded Gaussian d x k matrix (the values do not
    change the work) in the whitener's layout (rows padded to 16 bytes).
    Algorithmic bytes per view: nnz (4 + 4) + 4 (n + 1) + n ldy 4 written, plus
    W (d k 4) once; the W rows gathered per entry come from L2."""
    import numpy as np
    import torch
    from paper_1309_0787_amd import otm
    import synth

    dev = torch.device("cuda:0")
    k, d, n = 50, inst.C.n_cols, inst.C.n_rows
    views = [otm.DeviceCSR.from_host(v, dev) for v in inst.views]
    ldw = otm.default_ldw(k, otm.F32)
    Wbuf = torch.zeros((d, ldw), dtype=torch.float32, device=dev)
    Wbuf[:, :k] = torch.as_tensor(np.random.default_rng(0).standard_normal((d, k)), dtype=torch.float32, device=dev)
    W = Wbuf[:, :k]
    ldy = otm.default_ldy(k)
    Ys = [torch.empty((n, ldy), dtype=torch.float32, device=dev) for _ in views]
    for v, Y in zip(views, Ys):
        otm.whiten(v, True, W, y_dtype=otm.F32, out=Y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for v, Y in zip(views, Ys):
            otm.whiten(v, True, W, y_dtype=otm.F32, out=Y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps                       # three views
    nnz = sum(v.nnz for v in inst.views)
    algo = nnz * 8 + 3 * 4 * (n + 1) + 3 * n * ldy * 4 + d * k * 4
    achieved = algo / (ms * 1e-3)
    per = whiten_traffic("documents")
    traffic = 3 * per if per else None
    return {"workload": f"documents d={d}, k={k}, n={n}, three views, nnz={nnz}, FP32",
            "ms_per_three_views": ms, "algorithmic_bytes": algo,
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM, "traffic": traffic,
                         "traffic_gb_s": (traffic / (ms * 1e-3) / 1e9) if traffic else None,
                         "traffic_over_algorithmic": (traffic / algo) if traffic else None},
            "w_gather_bytes": nnz * ldw * 4, "w_gather_tb_per_s": nnz * ldw * 4 / (ms * 1e-3) / 1e12}


def bench_whiten_graph(C, W, k: int, reps: int = 20) -> dict:
    """Whitening SpMM of the benchmark graph's block G[X, A] (BF16 W and Y,
    no weights), as the step runs it: algorithmic HBM bytes nnz 4 + 4 (n + 1)
    + d k 2 + n ldy 2 per launch, HIP events over `reps` launches, and the
    counter traffic when it is current."""
    import torch
    from paper_1309_0787_amd import otm
    n, d = C.n_rows, C.n_cols
    ldy = otm.default_ldy(k)
    # the whitener's BF16 copy of W: rows padded to 16 bytes
    Wbuf = torch.zeros((d, otm.default_ldw(k, otm.BF16)), dtype=torch.bfloat16, device=W.device)
    Wbuf[:, :k] = W.to(torch.bfloat16)
    W_lo = Wbuf[:, :k]
    Y = torch.empty((n, ldy), dtype=torch.bfloat16, device=W.device)
    otm.whiten(C, False, W_lo, y_dtype=otm.BF16, out=Y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        otm.whiten(C, False, W_lo, y_dtype=otm.BF16, out=Y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    algo = C.nnz * 4 + 4 * (n + 1) + d * k * 2 + n * ldy * 2
    achieved = algo / (ms * 1e-3)
    traffic = whiten_traffic("graph")
    return {"workload": f"graph block G[X, A], {n} x {d}, nnz={C.nnz}, k={k}, BF16 W and Y",
            "ms_per_launch": ms, "algorithmic_bytes": algo,
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM, "traffic": traffic,
                         "traffic_gb_s": (traffic / (ms * 1e-3) / 1e9) if traffic else None,
                         "traffic_over_algorithmic": (traffic / algo) if traffic else None},
            "w_gather_bytes": C.nnz * otm.default_ldw(k, otm.BF16) * 2}


def recovery_error(Pi: "torch.Tensor", pi_true: "np.ndarray") -> float:
    """||Pi_hat - pi^T||_F / ||pi||_F after matching communities (Hungarian on correlations)."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    P = Pi.detach().double().cpu().numpy()                     # k x n
    T = pi_true.T                                              # k x n
    Pc = P - P.mean(1, keepdims=True)
    Tc = T - T.mean(1, keepdims=True)
    corr = (Pc @ Tc.T) / (np.linalg.norm(Pc, axis=1)[:, None] * np.linalg.norm(Tc, axis=1)[None, :] + 1e-300)
    r, c = linear_sum_assignment(-corr)
    M = np.zeros_like(T)
    M[c] = P[r]
    return float(np.linalg.norm(M - T) / np.linalg.norm(T))


def _validation_record(Pi_hat, pi_true) -> dict:
    """Recovery ratio and error of Section 5.2 (p-value matching, BH-adjusted,
    threshold 0.01) of estimated memberships (k x n, GPU) against the planted
    ones (n x k host), computed by the library's validation kernels."""
    import torch
    from paper_1309_0787_amd import otm
    P = torch.as_tensor(pi_true.T.astype(np.float32), device=Pi_hat.device).contiguous()
    V = otm.validate(Pi_hat.float().contiguous(), P, 0.01)
    sc = V.scores.cpu().numpy()
    return {"recovery_ratio": float(sc[0]), "error": float(sc[1]), "edges": int(V.edges.sum().item())}


def bench_validation_small() -> dict:
    """The small graph (n = 1000, X/A 500/500, k = 10, alpha0 = 0.1, p = 0.3,
    q = 0.05): whole path on the GPU (FP32), 8 restarts in one launch, the
    lowest residual kept; R and E of its memberships, and the same for the
    oracle's path."""
    import torch
    import oracle
    import synth
    from paper_1309_0787_amd import otm, pipeline
    dev = torch.device("cuda:0")
    g = synth.make("mmsb_small")
    k, a0, R = 10, 0.1, 8
    S = synth.projection(g.C.n_cols, 2 * k, seed=1)
    n = g.C.n_rows
    perms = synth.permutations(n, 50, seed=2)
    Phi0 = np.stack([synth.initial_factors(k, seed=3, restart=r).T for r in range(R)])
    C, CT = otm.DeviceCSR.from_host(g.C, dev), otm.DeviceCSR.from_host(g.CT, dev)
    cfg = pipeline.FitConfig(k=k, alpha0=a0, q_power=3, y_dtype=otm.F32, batch=100, passes=50, beta0=0.05,
                             beta_tau=500.0, restarts=R, tau_pi=0.1)
    Phi = torch.as_tensor(Phi0, dtype=torch.float32, device=dev).contiguous()
    res = pipeline.fit([C], C, CT, torch.as_tensor(S, device=dev), Phi, torch.as_tensor(perms, device=dev), cfg)
    T = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, a0)
    Rs = otm.residual(T, res.Phi).cpu().numpy()
    best = int(np.argmin(Rs))
    Pi = otm.recover_pi(res.Y[0], k, res.Phi[best], tau=0.1)
    out = {"workload": "MMSB n=1000 (X/A 500/500) k=10 alpha0=0.1 p=0.3 q=0.05, FP32, 50 passes, best of 8 restarts",
           "R_best": float(Rs[best]), "gpu": _validation_record(Pi, g.pi[g.X]),
           "recovery_error": recovery_error(Pi, g.pi[g.X])}
    Q, O = oracle.power_sketch(g.C, S, a0, False, 3)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    Y, yb = oracle.whiten(g.C, W, False)
    yb3 = np.stack([yb] * 3)
    Tn = oracle.whitened_tensor(Y, Y, Y, yb3, a0)
    best_o, bR = None, np.inf
    for r in range(R):
        P_o = oracle.sgd_run(Y, Y, Y, yb3, Phi0[r].T, perms, 100, 0.05, 500.0, a0)
        Rr = oracle.residual(Tn, P_o)
        if Rr < bR:
            best_o, bR = P_o, Rr
    Pi_o = oracle.recover_pi(Y, best_o, 0.1)
    out["oracle"] = _validation_record(torch.as_tensor(Pi_o, dtype=torch.float32, device=dev), g.pi[g.X])
    out["oracle"]["R_best"] = float(bR)
    return out


def bench_four_partition(w) -> dict:
    """Section 2.2's four-partition estimator (nodes split into X/A/B/C,
    transition matrices through the randomized pseudo-inverse) on the
    benchmark's graph model (n = 1e5, k = 100, BF16 views and STGD), and on a
    denser graph (n = 2e4, k = 5, FP32) beside the single-leaf-set path on
    the same X and A blocks: stage times, residual, memberships."""
    import time as _t
    import torch
    import synth
    from paper_1309_0787_amd import otm, pipeline
    dev = torch.device("cuda:0")
    out = {}
    for name, n, k, a0, p, q, ydt, passes in (("large", w["n"], w["k"], w["alpha0"], w["p"], w["q"], otm.BF16, 50),
                                             ("dense", 20000, 5, 0.5, 0.3, 0.02, otm.F32, 50)):
        t0 = _t.perf_counter()
        g = synth.mmsb_four(n, k, a0, p, q)
        t_gen = _t.perf_counter() - t0
        B = g.blocks
        G = otm.DevicePartition.from_blocks(B, dev)
        nA, nB, nC = (B[("X", s)].n_cols for s in "ABC")
        nx = B[("X", "A")].n_rows
        S = torch.as_tensor(synth.projection(nA, k, seed=1), device=dev)
        SB = torch.as_tensor(synth.projection(nB, 2 * k, seed=11), device=dev)
        SC = torch.as_tensor(synth.projection(nC, 2 * k, seed=12), device=dev)
        perms = torch.as_tensor(synth.permutations(nx, passes, seed=2), device=dev)
        Phi0 = torch.as_tensor(synth.initial_factors(k, seed=4).T.copy(), dtype=torch.float32, device=dev)[None]
        cfg = pipeline.FitConfig(k=k, alpha0=a0, q_power=1, y_dtype=ydt, batch=100, passes=passes, beta0=1e-3,
                                 beta_tau=2500.0, tau_pi=0.1)
        blocks = [otm.DeviceCSR.from_host(B[(s, "A")], dev) for s in "BC"]
        Phi = Phi0.clone()
        pipeline.fit_four(G, S, SB, SC, Phi, perms, cfg, q_pinv=1, node_blocks=blocks)   # warm-up
        Phi = Phi0.clone()
        tm = pipeline.Timer(True)
        res = pipeline.fit_four(G, S, SB, SC, Phi, perms, cfg, q_pinv=1, node_blocks=blocks, timer=tm)
        torch.cuda.synchronize()
        T = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, a0)
        rec = {"workload": f"MMSB n={n} k={k} alpha0={a0} p={p} q={q}, X/A/B/C quarters, "
                           f"{'BF16' if ydt == otm.BF16 else 'FP32'}, {passes} passes",
               "stage_ms": {a: round(b, 3) for a, b in tm.spans_ms().items()},
               "R": float(otm.residual(T, res.Phi[0]).item()), "nonfinite": int(res.nonfinite.item()),
               "recovery_error_X": recovery_error(res.Pi, g.pi[g.sets["X"]]),
               "recovery_error_B": recovery_error(res.Pi_nodes[0], g.pi[g.sets["B"]]),
               "validation_X": _validation_record(res.Pi, g.pi[g.sets["X"]]),
               "generation_s": round(t_gen, 2)}
        if name == "dense":   # the single-leaf-set path on the same X, A blocks
            C, CT = G.XA, G.AX
            cfg1 = pipeline.FitConfig(k=k, alpha0=a0, q_power=3, y_dtype=ydt, batch=100, passes=passes, beta0=1e-3,
                                      beta_tau=2500.0, tau_pi=0.1)
            Phi = Phi0.clone()
            S2 = torch.as_tensor(synth.projection(nA, 2 * k, seed=1), device=dev)
            r1 = pipeline.fit([C], C, CT, S2, Phi, perms, cfg1, pi_view=0)
            T1 = otm.tensor_form(r1.Y[0], r1.Y[1], r1.Y[2], k, r1.ybar3, a0)
            rec["single_leaf_set"] = {"R": float(otm.residual(T1, r1.Phi[0]).item()),
                                      "recovery_error_X": recovery_error(r1.Pi, g.pi[g.sets["X"]])}
        out[name] = rec
        del G, B, g
    return out


def oracle_stage_timing(inst, w) -> dict:
    """The FP64 oracle per stage on the benchmark graph (one M2 application
    to the 2k-column sketch, the whitener, the whitening, 200 STGD steps, the
    memberships), median of 5 runs after one warm-up, with the linear algebra
    libraries held to one thread and then to all of the host's cores."""
    import platform
    import statistics

    import oracle
    import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    k, a0 = w["k"], w["alpha0"]
    C = inst.C
    S = synth.projection(C.n_cols, 2 * k, seed=1)
    O = oracle.m2_apply(C, S, a0, False)
    Q, O = oracle.power_sketch(C, S, a0, False, 1)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    Y, yb = oracle.whiten(C, W, False)
    yb3 = np.stack([yb] * 3)
    steps = 200
    spp = (C.n_rows + w["batch"] - 1) // w["batch"]
    perms = synth.permutations(C.n_rows, (steps + spp - 1) // spp, seed=2)
    Phi0 = synth.initial_factors(k, seed=4)
    stages = {
        "m2_apply": lambda: oracle.m2_apply(C, S, a0, False),
        "whitener": lambda: oracle.whitener_rsvd(O, Q, k),
        "whiten": lambda: oracle.whiten(C, W, False),
        "stgd_200_steps": lambda: oracle.sgd_run(Y, Y, Y, yb3, Phi0, perms, w["batch"], w["beta0"], w["beta_tau"], a0,
                                                 end_step=steps),
        "memberships": lambda: oracle.recover_pi(Y, Phi0, w["tau_pi"]),
    }
    cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    model = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
           "blas_threads_all": int(cores), "runs": "median of 5 after 1 warm-up"}
    for label, limit in (("1_thread", 1), ("all_cores", int(cores))):
        rec = {}
        with threadpool_limits(limits=limit):
            for name, fn in stages.items():
                fn()
                ts = []
                for _ in range(5):
                    t0 = time.perf_counter()
                    fn()
                    ts.append(time.perf_counter() - t0)
                rec[name + "_ms"] = round(statistics.median(ts) * 1e3, 3)
        rec["stgd_samples_per_s"] = steps * w["batch"] / (rec["stgd_200_steps_ms"] * 1e-3)
        out[label] = rec
    return out


def bench_peaks() -> dict:
    """The device's own rates measured by the library's probes: a 16-byte
    vector copy of 4 GiB (HBM read + write bytes over the time; best of 5)
    and whole-device matrix-core chains in BF16, FP32 and FP64 (best of 3)."""
    import torch
    from paper_1309_0787_amd import otm
    dev = torch.device("cuda:0")
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    blocks = 256 * 16
    otm.probe_copy(src, dst, blocks)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        otm.probe_copy(src, dst, blocks)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    out = {"hbm_copy_gb_s": 2.0 * nbytes / (best * 1e-3) / 1e9, "copy_bytes": nbytes}
    del src, dst
    sink = torch.empty(256 * 8 * 256, dtype=torch.float32, device=dev)
    for name, dt, iters in (("bf16", otm.BF16, 4000), ("fp32", otm.F32, 4000), ("fp64", otm.F64, 2000)):
        blocks = 256 * 8
        otm.probe_mfma(dt, 100, blocks, sink)
        best = float("inf")
        flops = 0
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            flops = otm.probe_mfma(dt, iters, blocks, sink)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[f"mfma_{name}_tflop_s"] = flops / (best * 1e-3) / 1e12
    out["datasheet"] = {"hbm_gb_s": 8000.0, "mfma_bf16_tflop_s": 2500.0, "mfma_fp32_tflop_s": 157.3,
                        "mfma_fp64_tflop_s": 78.6}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quality", action="store_true", help="also report the residual of the final factors")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched many-problem measurement")
    ap.add_argument("--no-time-to-loss", action="store_true", help="skip the warm-start time-to-loss measurement")
    ap.add_argument("--no-spmm", action="store_true", help="skip the document whitening SpMM measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip validation, four-partition, measured peaks and per-stage oracle timing")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (scale for the HBM counters)")
    ap.add_argument("--print-kernel-hash", action="store_true", help="print the STGD kernel source hash and exit")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(kernel_hash())
        return
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the hot path is single-GPU here",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_0787_amd import otm
    if not os.path.exists(otm.LIB_PATH):
        from paper_1309_0787_amd import build
        build.build()
    from paper_1309_0787_amd import pipeline
    import synth

    w = WORKLOAD
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    inst = synth.mmsb(w["n"], w["k"], w["alpha0"], w["p"], w["q"], w["n_x"], seed=synth.BASE_SEED)
    t_gen = time.perf_counter() - t_gen
    k, n = w["k"], inst.C.n_rows
    C = otm.DeviceCSR.from_host(inst.C, dev)
    CT = otm.DeviceCSR.from_host(inst.CT, dev)
    S = torch.as_tensor(synth.projection(inst.C.n_cols, 2 * k, seed=1), device=dev)
    perms = torch.as_tensor(synth.permutations(n, w["passes"], seed=2), device=dev)
    Phi_init = torch.as_tensor(synth.initial_factors(k, seed=4).T.copy(), dtype=torch.float32, device=dev)[None]
    Phi = torch.empty_like(Phi_init)
    cfg = pipeline.FitConfig(k=k, alpha0=w["alpha0"], normalize=False, q_power=w["q_power"], y_dtype=otm.BF16,
                             batch=w["batch"], passes=w["passes"], beta0=w["beta0"], beta_tau=w["beta_tau"],
                             tau_pi=w["tau_pi"], compensated=w["compensated"])

    def step(timer=None):
        Phi.copy_(Phi_init)
        return pipeline.fit([C], C, CT, S, Phi, perms, cfg, pi_view=0, timer=timer)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    timers = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tm = pipeline.Timer(True)
        res = step(tm)
        timers.append(tm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    stages = {}
    for tm in timers:
        for kname, v in tm.spans_ms().items():
            stages[kname] = stages.get(kname, 0.0) + v / args.steps
    sgd_ms = stages["stgd"]
    flops = sgd_flops(n, w["batch"], k, w["passes"])
    achieved = flops / (sgd_ms * 1e-3)
    out = {
        "metric": "whitened samples/sec through tensor SGD at k=100",
        "value": n * w["passes"] / (ms_per_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"MMSB n={w['n']} (X/A {w['n_x']}/{w['n'] - w['n_x']}) k={k} alpha0={w['alpha0']} "
                               f"p={w['p']} q={w['q']} nnz(G[X,A])={inst.C.nnz}",
                   "batch": w["batch"], "passes": w["passes"], "restarts": 1, "sketch_power_iterations": w["q_power"],
                   "precision": "BF16 W/Y and STGD contractions, FP32 accumulate and FP32 master (plain update), "
                                "FP64 sketch/whitener/post"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16, "traffic": counters_traffic(),
                     "kernel": "sgd_kernel<MmaBF16,128,1,plain>", "flops_per_launch": flops, "launch_ms": sgd_ms,
                     "frac_one_cu": achieved / (PEAK_BF16 / 256)},
        "stage_ms": {kname: round(v, 4) for kname, v in stages.items()},
        "sgd_samples_per_s": n * w["passes"] / (sgd_ms * 1e-3),
        "sgd_us_per_step": sgd_ms * 1e3 / (w["passes"] * ((n + w["batch"] - 1) // w["batch"])),
        "generation_s": round(t_gen, 2),
    }
    if not args.no_extras:
        print("bench: measured peaks", file=sys.stderr, flush=True)
        out["measured_peaks"] = bench_peaks()
        pk = out["measured_peaks"]
        out["roofline"]["frac_measured_peak"] = achieved / (pk["mfma_bf16_tflop_s"] * 1e12)
        print("bench: validation (recovery ratio, error)", file=sys.stderr, flush=True)
        out["validation"] = {"large": dict(_validation_record(res.Pi, inst.pi[inst.X]),
                                           recovery_error=recovery_error(res.Pi, inst.pi[inst.X])),
                             "small": bench_validation_small()}
        print("bench: four-partition estimator", file=sys.stderr, flush=True)
        out["four_partition"] = bench_four_partition(w)
    if args.quality:
        T = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, w["alpha0"])
        out["quality"] = {"residual": float(otm.residual(T, res.Phi[0]).item()),
                          "nonfinite": int(res.nonfinite.item())}
    if not args.no_time_to_loss:
        print("bench: warm-start training (instances of the three generators)", file=sys.stderr, flush=True)
        warm, warm_info = train_warm_start(inst, res, w)
        print("bench: held-out instances, warm against random", file=sys.stderr, flush=True)
        out["warm_start_heldout"] = bench_heldout(warm)
        print("bench: time to loss, four arms", file=sys.stderr, flush=True)
        out["time_to_loss"] = bench_time_to_loss(inst, C, CT, S, Phi_init, w, warm, warm_info)
    docs = None
    if not args.no_spmm or not args.no_cpu_baseline:
        t0 = time.perf_counter()
        docs = synth.make("lda_medium")
        print(f"bench: document workload generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if not args.no_spmm:
        print("bench: whitening SpMM on the document workload and the graph", file=sys.stderr, flush=True)
        out["spmm"] = bench_spmm(docs)
        out["spmm_graph"] = bench_whiten_graph(C, res.W, k)
    if not args.no_batched:
        print("bench: batched workload", file=sys.stderr, flush=True)
        Yr = res.Y[0].float().contiguous() if res.Y[0].dtype != torch.float32 else res.Y[0]
        out["batched"] = bench_batched(max(1, min(args.steps, 3)), 1, real_rows=Yr)
    if not args.no_cpu_baseline:
        print("bench: oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"], ores = cpu_baseline(inst, w)
        print("bench: per-result errors against the oracle (graph)", file=sys.stderr, flush=True)
        out["error_vs_oracle"] = {"graph": errors_graph(res, ores, w, inst)}
        print("bench: per-result errors against the oracle (documents)", file=sys.stderr, flush=True)
        out["error_vs_oracle"]["documents"] = errors_documents(docs)
        if not args.no_extras:
            print("bench: oracle per stage, one thread and all cores", file=sys.stderr, flush=True)
            out["cpu_baseline"]["per_stage"] = oracle_stage_timing(inst, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    # The batched leg runs one persistent kernel per kernel variant (ten here)
    # side by side; HIP gives a process GPU_MAX_HW_QUEUES hardware queues (4 by
    # default), so the benchmark asks for 16 before the runtime starts.
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    main()
