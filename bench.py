#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: mixed-membership graph, n = 100000 nodes (X/A = 50000/50000),
k = 100 communities, alpha0 = 0.5, p = 0.05, q = 0.001, seeded synthetic.
One step = the whole path on one batch of input already resident in HBM:
power-iterated M2 sketch (FP64) -> randomized whitener (FP64) -> whitening
SpMM (BF16 W and Y, FP32 accumulation) -> STGD run (50 passes, mini-batch 100,
BF16 matrix-core contractions, FP32 compensated update) -> memberships (FP64).

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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = dict(name="mmsb_large", n=100000, n_x=50000, k=100, alpha0=0.5, p=0.05, q=0.001, batch=100, passes=50,
                q_power=3, beta0=1e-3, beta_tau=2500.0, tau_pi=0.1)
PEAK_BF16 = 2.5e15          # dense MFMA bf16, FLOP/s
PEAK_HBM = 8.0e12           # bytes/s
# HBM counters of the STGD kernel (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE), per launch,
# valid only for the kernel source they were taken on.
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sgd_kernel_mmsb_large_counters.json")


def sgd_flops(n: int, batch: int, k: int, passes: int) -> float:
    """Algorithmic flops of one STGD run: per step 2 PA/PB products (2*2*B*k^2),
    YC^T Q (2*B*k^2), Phi^T Phi and Phi (G*G) (2*2*k^3)."""
    full, rem = divmod(n, batch)
    per_pass = full * (6.0 * batch * k * k + 4.0 * k ** 3)
    if rem:
        per_pass += 6.0 * rem * k * k + 4.0 * k ** 3
    return per_pass * passes


def kernel_hash() -> str:
    """Hash of the STGD kernel's sources without comments and blank lines (the
    counters are valid for this code only)."""
    import re
    h = hashlib.sha256()
    for f in ("stgd.hip", "stgd_kernel.h"):
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


def cpu_baseline(inst, w):
    """The FP64 oracle on the same workload (whole path, one decomposition)."""
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
    oracle.recover_pi(Y, Phi, w["tau_pi"])
    el = time.perf_counter() - t0
    return {"value": inst.C.n_rows * w["passes"] / el, "unit": "samples/s", "cores": int(cores), "kind": "oracle",
            "sample": f"whole path once on the same graph (FP64): sketch q={w['q_power']}, whitener, whitening, "
                      f"{w['passes']} STGD passes, memberships; {el:.1f} s"}


# beta0 3e-4: at 1e-3 the three-view problems with k = 100 and alpha0 = 1 diverge
BATCHED = dict(problems=256, ks=(16, 32, 64, 100, 128), n_lo=1e3, n_hi=1e5, restarts=8, passes=50, batch=100,
               beta0=3e-4, beta_tau=2500.0)
PEAK_FP32_MFMA = 157.3e12


def bench_batched(steps: int, warmup: int) -> dict:
    """Many decompositions with restarts in one launch (FP32): 256 problems, k
    uniform over {16, 32, 64, 100, 128}, n log-uniform in [1e3, 1e5], half
    three-view (documents) and half one-view (graphs), 8 restarts each; the
    tile layouts come from the autotuner (run first, timed separately)."""
    import tempfile

    import numpy as np
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
        Phi0 = torch.as_tensor(np.ascontiguousarray(np.stack([synth.initial_factors(k, restart=r + 100 * i).T for r in range(w["restarts"])])),
                               dtype=torch.float32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + i)
        perms = torch.argsort(torch.rand((w["passes"], n), device=dev, generator=g), dim=1).to(torch.int32)
        problems.append(otm.Problem(YA, YB, YC, ybar, Phi0, k, sp["alpha0"], perms))   # perms shared by the restarts
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
    for _ in range(warmup):
        run.run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        run.run()
    ev1.record()
    torch.cuda.synchronize()
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
    return {
        "workload": f"{w['problems']} problems, k in {list(w['ks'])}, n log-uniform [{int(w['n_lo'])}, {int(w['n_hi'])}], "
                    f"half three-view / half one-view, {w['restarts']} restarts, {w['passes']} passes, FP32",
        "samples_per_s": samples / (ms * 1e-3), "ms_per_run": ms, "jobs": len(problems) * w["restarts"],
        "kernel_groups": run.groups,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_MFMA, "flops_per_run": flops},
        "nonfinite": int(run.nonfinite.item()), "generation_s": round(t_gen, 2), "autotune_s": round(t_tune, 2),
        "tuned_layouts": tuned,
    }


WARM = dict(instances=8000, epochs=15, batch=256, lr=1e-3, exact_share=0.8, sampled_n=2000)


def bench_spmm(reps: int = 20) -> dict:
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
    t0 = time.perf_counter()
    inst = synth.make("lda_medium")
    t_gen = time.perf_counter() - t0
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
    return {"workload": f"documents d={d}, k={k}, n={n}, three views, nnz={nnz}, FP32",
            "ms_per_three_views": ms, "algorithmic_bytes": algo,
            "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM},
            "w_gather_bytes": nnz * ldw * 4, "w_gather_tb_per_s": nnz * ldw * 4 / (ms * 1e-3) / 1e12,
            "generation_s": round(t_gen, 2)}


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


def bench_time_to_loss(inst, C, CT, S, perms, Phi_init, w) -> dict:
    """Time to the converged loss: FP32 path from random factors against the
    BF16 path from the learned warm start, on the benchmark graph.  R(Phi) is
    evaluated at every pass end from snapshots, outside the timed stages; the
    threshold is the FP32 path's final R plus 1e-3.  The warm start is trained
    first (timed separately) on exact-moment instances (k in {10, 50, 100}) and
    planted-mixture rows."""
    import numpy as np
    import torch
    from paper_1309_0787_amd import otm, pipeline
    from paper_1309_0787_amd import warmstart as pws

    dev = torch.device("cuda:0")
    ws_cfg = WARM
    g = np.random.default_rng(0)
    specs = []
    for i in range(ws_cfg["instances"]):
        if g.random() < ws_cfg["exact_share"]:
            specs.append(dict(k=int(g.choice([10, 50, 100, 100, 100])), seed=5000 + i, kind="exact"))
        else:
            specs.append(dict(k=w["k"], seed=5000 + i, kind="sampled", n=ws_cfg["sampled_n"], alpha0=w["alpha0"],
                              views=1))
    t0 = time.perf_counter()
    tr = pws.build_instances(specs, dev)
    warm = pws.WarmStart(dev, seed=3)
    _, _, X, tgt, _ = warm.prepare(tr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = warm.train(X, tgt, tr.ks, epochs=ws_cfg["epochs"], batch=ws_cfg["batch"], lr=ws_cfg["lr"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del X, tgt, tr
    k = w["k"]
    runs = {}
    pi_true = inst.pi[inst.X]
    for name, ydt, use_warm in (("fp32_random", otm.F32, False), ("bf16_warm", otm.BF16, True)):
        cfg = pipeline.FitConfig(k=k, alpha0=w["alpha0"], normalize=False, q_power=w["q_power"], y_dtype=ydt,
                                 batch=w["batch"], passes=w["passes"], beta0=w["beta0"], beta_tau=w["beta_tau"],
                                 tau_pi=w["tau_pi"])
        Phi = Phi_init.clone()
        tm = pipeline.Timer(True)
        res = pipeline.fit([C], C, CT, S, Phi, perms, cfg, pi_view=0, snapshots=True, timer=tm,
                           warm=warm if use_warm else None)
        torch.cuda.synchronize()
        spans = tm.spans_ms()
        T = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, w["alpha0"])
        Rs = otm.residual(T, res.snapshots[0].contiguous()).cpu().numpy()
        runs[name] = dict(stages_ms={a: round(b, 3) for a, b in spans.items()}, R_by_pass=[float(x) for x in Rs],
                          recovery_error=recovery_error(res.Pi, pi_true))
    r_inf = runs["fp32_random"]["R_by_pass"][-1]
    thr = r_inf + 1e-3
    out = {"threshold": thr, "R_inf_fp32": r_inf}
    for name, r in runs.items():
        hit = [i for i, x in enumerate(r["R_by_pass"]) if x <= thr]
        passes = hit[0] + 1 if hit else None
        st = r["stages_ms"]
        prefix = st.get("sketch", 0) + st.get("whitener", 0) + st.get("whiten", 0) + st.get("warm", 0)
        ttl = prefix + st["stgd"] * passes / w["passes"] if passes else None
        out[name] = {"time_to_loss_ms": ttl, "passes_to_loss": passes, "R_final": r["R_by_pass"][-1],
                     "R_pass1": r["R_by_pass"][0], "stgd_ms_50_passes": st["stgd"], "prefix_ms": prefix,
                     "warm_ms": st.get("warm"), "recovery_error": r["recovery_error"]}
    a, b = out["fp32_random"]["time_to_loss_ms"], out["bf16_warm"]["time_to_loss_ms"]
    out["speedup"] = (a / b) if (a and b) else None
    out["warm_start"] = {"train_instances": ws_cfg["instances"], "epochs": ws_cfg["epochs"],
                         "build_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                         "final_loss": float(np.mean(losses[-10:])), "adam_steps": len(losses)}
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
                             tau_pi=w["tau_pi"])

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
                   "precision": "BF16 W/Y and STGD contractions, FP32 accumulate and master, FP64 sketch/whitener/post"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16, "traffic": counters_traffic(),
                     "kernel": "sgd_kernel<MmaBF16,128>", "flops_per_launch": flops, "launch_ms": sgd_ms,
                     "frac_one_cu": achieved / (PEAK_BF16 / 256)},
        "stage_ms": {kname: round(v, 4) for kname, v in stages.items()},
        "sgd_samples_per_s": n * w["passes"] / (sgd_ms * 1e-3),
        "sgd_us_per_step": sgd_ms * 1e3 / (w["passes"] * ((n + w["batch"] - 1) // w["batch"])),
        "generation_s": round(t_gen, 2),
    }
    if args.quality:
        T = otm.tensor_form(res.Y[0], res.Y[1], res.Y[2], k, res.ybar3, w["alpha0"])
        out["quality"] = {"residual": float(otm.residual(T, res.Phi[0]).item()),
                          "nonfinite": int(res.nonfinite.item())}
    if not args.no_time_to_loss:
        print("bench: time to loss, BF16 + warm start against FP32", file=sys.stderr, flush=True)
        out["time_to_loss"] = bench_time_to_loss(inst, C, CT, S, perms, Phi_init, w)
    if not args.no_spmm:
        print("bench: whitening SpMM on the document workload", file=sys.stderr, flush=True)
        out["spmm"] = bench_spmm()
    if not args.no_batched:
        print("bench: batched workload", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(max(1, min(args.steps, 3)), 1)
    if not args.no_cpu_baseline:
        print("bench: oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    # The batched leg runs one persistent kernel per kernel variant (ten here)
    # side by side; HIP gives a process GPU_MAX_HW_QUEUES hardware queues (4 by
    # default), so the benchmark asks for 16 before the runtime starts.
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    main()
