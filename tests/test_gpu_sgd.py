"""GPU parity of the STGD step and run (Section 3.2, Lemma update; stacked
form of Section 4.3) against the FP64 oracle on identical inputs.

Bars (stated per precision):
* FP32 step: the GPU update Phi1 - Phi0 matches the oracle's within 1e-5
  relative (Frobenius), i.e. the step is right to FP32 accumulation error;
* BF16 step (Y stored in BF16, Phi and the exchanged G*G / Q rounded to BF16 as
  matrix-core operands, FP32 accumulation): update within 3e-2 relative, with
  the compensated update and with the variant that keeps no compensation
  terms;
* FP32 run: factor error ||Phi_gpu - Phi_ref||_F / ||Phi_ref||_F <= 1e-4;
* runs split at any step, restarts in one launch and per-pass snapshots are
  bit-identical to the corresponding single runs on the GPU (FP32, and BF16
  at k = 100 with and without compensation).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import bf16_round, dev, f32_round, padded, phi_cols, phi_rows, rel, to_dev

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu


def _inputs(n, k, seed, scale=0.3, three=True):
    g = np.random.default_rng(seed)
    YA = g.standard_normal((n, k)) * scale + 0.2
    YB = g.standard_normal((n, k)) * scale + 0.1 if three else YA
    YC = g.standard_normal((n, k)) * scale - 0.1 if three else YA
    ybar = np.stack([YA.mean(0), YB.mean(0), YC.mean(0)])
    Phi = synth.initial_factors(k, seed=seed) * 1.3
    return YA, YB, YC, ybar, Phi


def _dev_views(YA, YB, YC, k, dtype):
    ldy = otm.default_ldy(k)
    tdt = torch.bfloat16 if dtype == otm.BF16 else torch.float32
    A = padded(YA, ldy, tdt)
    B = A if YB is YA else padded(YB, ldy, tdt)
    C = A if YC is YA else padded(YC, ldy, tdt)
    return A, B, C


@pytest.mark.parametrize("k", [4, 10, 17, 32, 50, 100, 128])
@pytest.mark.parametrize("rows", [1, 7, 100, 128])
@pytest.mark.parametrize("alpha0", [0.0, 0.5])
def test_step_fp32(k, rows, alpha0):
    YA, YB, YC, ybar, Phi0 = _inputs(rows, k, seed=k * 1000 + rows)
    YA, YB, YC, ybar, Phi0 = (f32_round(x) for x in (YA, YB, YC, ybar, Phi0))
    beta = 0.01
    ref = oracle.sgd_step(YA, YB, YC, ybar, Phi0, beta, alpha0, theta=1.0)
    A, B, C = _dev_views(YA, YB, YC, k, otm.F32)
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=128, alpha0=alpha0, y_dtype=otm.F32)
    otm.sgd_step(p, rows, A, B, C, to_dev(ybar), beta, P)
    torch.cuda.synchronize()
    got = phi_cols(P)
    assert rel(got - Phi0, ref - Phi0) < 1e-5


@pytest.mark.parametrize("k", [10, 64, 100, 128])
@pytest.mark.parametrize("alpha0", [0.0, 1.0])
@pytest.mark.parametrize("compensated", [True, False])
def test_step_bf16(k, alpha0, compensated):
    rows = 100
    YA, YB, YC, ybar, Phi0 = _inputs(rows, k, seed=k + 7)
    YA, YB, YC = (bf16_round(x) for x in (YA, YB, YC))
    ybar, Phi0 = f32_round(ybar), f32_round(Phi0)
    beta = 0.01
    ref = oracle.sgd_step(YA, YB, YC, ybar, Phi0, beta, alpha0)
    A, B, C = _dev_views(YA, YB, YC, k, otm.BF16)
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=100, alpha0=alpha0, y_dtype=otm.BF16, compensated=compensated)
    otm.sgd_step(p, rows, A, B, C, to_dev(ybar), beta, P)
    torch.cuda.synchronize()
    assert rel(phi_cols(P) - Phi0, ref - Phi0) < 3e-2


@pytest.mark.parametrize("k", [14, 15, 46, 47, 78, 79, 110, 111])
@pytest.mark.parametrize("three", [False, True])
@pytest.mark.parametrize("compensated", [True, False])
def test_step_bf16_padding_tiles(k, three, compensated):
    """BF16 pads k to a multiple of 32; when k + 2 (components and the two
    folded means) fits in one 16-wide tile less, the products skip the last
    tile row and column.  k on both sides of each threshold, one shared view
    (staged rows, plain or compensated update) and three views."""
    rows = 100
    YA, YB, YC, ybar, Phi0 = _inputs(rows, k, seed=k + 11, three=three)
    YA, YB, YC = (bf16_round(x) for x in (YA, YB, YC))
    if not three:
        YB = YC = YA
    ybar, Phi0 = f32_round(ybar), f32_round(Phi0)
    beta = 0.01
    ref = oracle.sgd_step(YA, YB, YC, ybar, Phi0, beta, 0.5)
    if three:
        A, B, C = _dev_views(YA, YB, YC, k, otm.BF16)
    else:
        A, _, _ = _dev_views(YA, YA, YA, k, otm.BF16)
        B = C = A
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=100, alpha0=0.5, y_dtype=otm.BF16, compensated=compensated)
    otm.sgd_step(p, rows, A, B, C, to_dev(ybar), beta, P)
    torch.cuda.synchronize()
    assert rel(phi_cols(P) - Phi0, ref - Phi0) < 3e-2


def test_step_aliased_views_theta():
    k, rows = 20, 50
    YA, _, _, ybar, Phi0 = _inputs(rows, k, seed=3, three=False)
    YA, ybar, Phi0 = f32_round(YA), f32_round(ybar), f32_round(Phi0)
    ref = oracle.sgd_step(YA, YA, YA, ybar, Phi0, 0.02, 0.3, theta=3.0)
    A, _, _ = _dev_views(YA, YA, YA, k, otm.F32)
    P = phi_rows(Phi0)
    otm.sgd_step(otm.SgdParams(k=k, batch=64, alpha0=0.3, theta=3.0), rows, A, A, A, to_dev(ybar), 0.02, P)
    torch.cuda.synchronize()
    assert rel(phi_cols(P) - Phi0, ref - Phi0) < 1e-5


def _graph_instance():
    """Small MMSB instance (n = 1000, X/A = 500/500, k = 10) whitened by the oracle."""
    g = synth.make("mmsb_small")
    k = 10
    S = synth.projection(g.C.n_cols, 2 * k, seed=1)
    Q, O = oracle.power_sketch(g.C, S, 0.1, False, 3)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    Y, ybar = oracle.whiten(g.C, W, normalize=False)
    return g, f32_round(Y), f32_round(np.stack([ybar] * 3))


@pytest.mark.parametrize("compensated", [True, False])
def test_run_fp32_graph_parity(compensated):
    g, Y, ybar = _graph_instance()
    n, k = Y.shape
    perms = synth.permutations(n, 50, seed=2)
    Phi0 = f32_round(synth.initial_factors(k, seed=4))
    beta0, tau = 0.05, 500.0
    ref = oracle.sgd_run(Y, Y, Y, ybar, Phi0, perms, 100, beta0, tau, 0.1)
    A, _, _ = _dev_views(Y, Y, Y, k, otm.F32)
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=100, passes=50, alpha0=0.1, beta0=beta0, beta_tau=tau, compensated=compensated)
    nonfinite = torch.zeros(1, dtype=torch.int32, device=dev())
    otm.sgd_run(p, n, A, A, A, to_dev(ybar), to_dev(perms, torch.int32), P, nonfinite=nonfinite)
    torch.cuda.synchronize()
    assert int(nonfinite.item()) == 0
    assert rel(phi_cols(P), ref) < 1e-4


def test_run_three_views_ragged_batches():
    n, k = 237, 24         # 237 = 2*100 + 37: ragged last batch
    YA, YB, YC, ybar, Phi0 = _inputs(n, k, seed=11)
    YA, YB, YC, ybar, Phi0 = (f32_round(x) for x in (YA, YB, YC, ybar, Phi0 * 0.8))
    perms = synth.permutations(n, 4, seed=5)
    ref = oracle.sgd_run(YA, YB, YC, ybar, Phi0, perms, 100, 0.01, 20.0, 0.7)
    A, B, C = _dev_views(YA, YB, YC, k, otm.F32)
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=100, passes=4, alpha0=0.7, beta0=0.01, beta_tau=20.0)
    otm.sgd_run(p, n, A, B, C, to_dev(ybar), to_dev(perms, torch.int32), P)
    torch.cuda.synchronize()
    assert rel(phi_cols(P), ref) < 1e-5


@pytest.mark.parametrize("k,three", [(100, True), (128, False), (112, True)])
def test_run_fp32_unstaged_rows_multi_pass(k, three):
    """k >= 112 (padded): FP32 rows are not staged in LDS; the products read
    them from global memory after an L2 prefetch one step ahead.  Several
    passes with a ragged last batch, against the oracle run."""
    n, passes = 437, 3
    YA, YB, YC, ybar, Phi0 = _inputs(n, k, seed=k + 3, three=three)
    YA, YB, YC, ybar, Phi0 = (f32_round(x) for x in (YA, YB, YC, ybar, Phi0 * 0.8))
    if not three:
        YB = YC = YA
    perms = synth.permutations(n, passes, seed=k)
    ref = oracle.sgd_run(YA, YB, YC, ybar, Phi0, perms, 100, 0.01, 20.0, 0.4)
    A, B, C = _dev_views(YA, YB, YC, k, otm.F32)
    P = phi_rows(Phi0)
    p = otm.SgdParams(k=k, batch=100, passes=passes, alpha0=0.4, beta0=0.01, beta_tau=20.0)
    otm.sgd_run(p, n, A, B, C, to_dev(ybar), to_dev(perms, torch.int32), P)
    torch.cuda.synchronize()
    assert rel(phi_cols(P), ref) < 1e-5


def test_run_split_restarts_snapshots_bit_identical():
    n, k, passes = 300, 16, 3
    YA, YB, YC, ybar, _ = _inputs(n, k, seed=13)
    YA, YB, YC, ybar = (f32_round(x) for x in (YA, YB, YC, ybar))
    A, B, C = _dev_views(YA, YB, YC, k, otm.F32)
    yb = to_dev(ybar)
    R = 3
    perms = np.stack([synth.permutations(n, passes, seed=20 + r) for r in range(R)])
    pd = to_dev(perms, torch.int32)
    Phi0 = np.stack([f32_round(synth.initial_factors(k, seed=9, restart=r)).T for r in range(R)])
    p = otm.SgdParams(k=k, batch=64, passes=passes, alpha0=0.2, beta0=0.02, beta_tau=30.0)
    spp = (n + 63) // 64
    # R restarts in one launch, with snapshots
    P_all = to_dev(Phi0)
    snaps = torch.zeros((R, passes, k, k), dtype=torch.float32, device=dev())
    otm.sgd_run(p, n, A, B, C, yb, pd, P_all, restarts=R, perm_stride=passes * n, snapshots=snaps)
    # each restart alone, split in two with the compensation carried over
    for r in range(R):
        P1 = to_dev(Phi0[r])
        comp = torch.zeros((k, k), dtype=torch.float32, device=dev())
        cut = spp + 2
        otm.sgd_run(p, n, A, B, C, yb, pd[r], P1, start_step=0, end_step=cut, Phi_comp=comp)
        otm.sgd_run(p, n, A, B, C, yb, pd[r], P1, start_step=cut, end_step=-1, Phi_comp=comp)
        torch.cuda.synchronize()
        assert torch.equal(P1, P_all[r])
        assert torch.equal(snaps[r, passes - 1], P_all[r])
        P2 = to_dev(Phi0[r])
        otm.sgd_run(p, n, A, B, C, yb, pd[r], P2, end_step=spp)
        torch.cuda.synchronize()
        assert torch.equal(P2, snaps[r, 0])


@pytest.mark.parametrize("compensated", [False, True])
def test_run_bf16_split_restarts_bit_identical(compensated):
    """BF16 rows, one shared view, k = 100 (the benchmark's kernel shape):
    restarts in one launch equal separate runs split in two, with the
    compensation carried over when it is on (the plain update keeps no state
    besides Phi)."""
    n, k, passes = 700, 100, 2
    YA, _, _, ybar, _ = _inputs(n, k, seed=17, three=False)
    YA, ybar = bf16_round(YA), f32_round(ybar)
    A, _, _ = _dev_views(YA, YA, YA, k, otm.BF16)
    yb = to_dev(ybar)
    R = 2
    perms = np.stack([synth.permutations(n, passes, seed=40 + r) for r in range(R)])
    pd = to_dev(perms, torch.int32)
    Phi0 = np.stack([f32_round(synth.initial_factors(k, seed=19, restart=r)).T for r in range(R)])
    p = otm.SgdParams(k=k, batch=100, passes=passes, y_dtype=otm.BF16, alpha0=0.5, beta0=0.01, beta_tau=100.0,
                      compensated=compensated)
    spp = (n + 99) // 100
    P_all = to_dev(Phi0)
    otm.sgd_run(p, n, A, A, A, yb, pd, P_all, restarts=R, perm_stride=passes * n)
    for r in range(R):
        P1 = to_dev(Phi0[r])
        comp = torch.zeros((k, k), dtype=torch.float32, device=dev())
        cut = spp + 3
        otm.sgd_run(p, n, A, A, A, yb, pd[r], P1, start_step=0, end_step=cut, Phi_comp=comp)
        otm.sgd_run(p, n, A, A, A, yb, pd[r], P1, start_step=cut, end_step=-1, Phi_comp=comp)
        torch.cuda.synchronize()
        assert torch.equal(P1, P_all[r])
        assert torch.isfinite(P1).all()


def test_run_nonfinite_flag_and_bad_arguments():
    n, k = 120, 8
    YA, YB, YC, ybar, Phi0 = _inputs(n, k, seed=1)
    A, B, C = _dev_views(*(f32_round(x) for x in (YA, YB, YC)), k, otm.F32)
    P = phi_rows(f32_round(Phi0) * 50.0)
    flag = torch.zeros(1, dtype=torch.int32, device=dev())
    p = otm.SgdParams(k=k, batch=40, passes=3, beta0=10.0)
    otm.sgd_run(p, n, A, B, C, to_dev(ybar), None, P, nonfinite=flag)
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    with pytest.raises(otm.OtmError) as e:
        otm.sgd_run(otm.SgdParams(k=129, batch=40), n, A, B, C, to_dev(ybar), None, P)
    assert e.value.status == -8
    with pytest.raises(otm.OtmError) as e:
        otm.sgd_run(otm.SgdParams(k=k, batch=129), n, A, B, C, to_dev(ybar), None, P)
    assert e.value.status == -8
    with pytest.raises(otm.OtmError):
        otm.sgd_run(p, n, A, B, C, to_dev(ybar), None, P, start_step=5, end_step=2)
