"""GPU parity of the learned warm start against its FP64 oracle, and the gain
it brings to the stochastic updates.

Bars: sketch (FP64 sums, FP32 output) 1e-5 relative; frames on exact moments
(FP32 Jacobi) 1e-4 on Q, the features and sigma; targets 1e-4; perceptron
forward and backward in FP32 (sums of up to 40400 terms) 1e-4 relative, BF16
inference 3e-2; Adam 1e-5; loss 1e-6; factors 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import warmstart as ows
import synth
from gpu_util import f32_round, host, padded, rel, to_dev

from paper_1309_0787_amd import otm
from paper_1309_0787_amd import warmstart as pws

pytestmark = pytest.mark.gpu


def _views(n, k, seed, three):
    g = np.random.default_rng(seed)
    YA = f32_round(g.standard_normal((n, k)) * 0.4 + 0.1)
    YB = f32_round(g.standard_normal((n, k)) * 0.4 - 0.05) if three else YA
    YC = f32_round(g.standard_normal((n, k)) * 0.4 + 0.02) if three else YA
    ybar = f32_round(np.stack([YA.mean(0), YB.mean(0), YC.mean(0)]))
    return YA, YB, YC, ybar


@pytest.mark.parametrize("n,k,alpha0,three,dt", [(1, 5, 0.0, True, otm.F32), (333, 16, 0.7, True, otm.F32),
                                                 (3000, 100, 0.5, False, otm.F32), (700, 37, 1.0, True, otm.BF16)])
def test_sketch_vs_oracle(n, k, alpha0, three, dt):
    YA, YB, YC, ybar = _views(n, k, seed=n + k, three=three)
    tdt = torch.bfloat16 if dt == otm.BF16 else torch.float32
    ldy = otm.default_ldy(k)
    A = padded(YA, ldy, tdt)
    B = A if not three else padded(YB, ldy, tdt)
    C = A if not three else padded(YC, ldy, tdt)
    if dt == otm.BF16:   # the oracle sees the same rounded rows
        YA, YB, YC = (host(t)[:, :k] for t in (A, B, C))
    Theta = f32_round(np.random.default_rng(k).standard_normal((k, 4)))
    S = otm.ws_sketch(A, B, C, k, to_dev(ybar), alpha0, to_dev(Theta))
    torch.cuda.synchronize()
    ref = ows.sketch(YA, YB, YC, ybar, alpha0, Theta)
    assert rel(host(S), ref) < 1e-5


def _exact_set(ks, seed0=0, P=100):
    dev = torch.device("cuda:0")
    inst = pws.build_instances([dict(k=k, seed=seed0 + i, kind="exact") for i, k in enumerate(ks)], dev, P)
    return inst


def test_frames_and_targets_on_exact_moments():
    ks = [3, 10, 50, 100, 17]
    inst = _exact_set(ks, seed0=40)
    Q, sigma, X, tgt, info = pws.WarmStart.prepare(inst)
    torch.cuda.synchronize()
    assert np.all(host(info) >= 0)
    P = 100
    for i, k in enumerate(ks):
        S = host(inst.S[i])[:, :k, :k]
        Th = host(inst.Theta[i])[:k]
        # the instance's sketch is the oracle's sketch of its rows
        Y, _, _ = pws.exact_instance(k, 40 + i)
        Y = Y.astype(np.float64)
        So = ows.sketch(Y, Y, Y, np.stack([Y.mean(0)] * 3), 0.0, Th)
        assert rel(S, So) < 1e-5
        Qo = ows.canonical_frame(S, Th)
        # FP32 eigenvectors are accurate to about eps * |mu|_max / gap
        mu = np.sort(np.abs(np.linalg.eigvalsh(0.5 * (S[0] + S[0].T))))
        gap = max(np.min(np.diff(mu)) if k > 1 else mu[-1], 1e-12)
        tol = 1e-4 + 2e-6 * mu[-1] / gap
        Qg = host(Q[i])[:k, :k]
        assert np.abs(Qg - Qo).max() < tol, (k, np.abs(Qg - Qo).max(), tol)
        so = ows.sketch_scale(S)
        assert abs(float(sigma[i]) - so) < 1e-5 * so
        xo = ows.features(S, Th, Qo, P)
        assert rel(host(X[i]), xo) < tol
        Uo = host(inst.U[i])[:k, :k]
        lo = host(inst.lam[i])[:k]
        to = ows.frame_target(Qo, Uo, lo, so, P)
        assert rel(host(tgt[i]), to.ravel()) < tol
        # the target maps back to the planted factors
        Phi = otm.ws_factors(inst.ks[i:i + 1], tgt[i:i + 1], Q[i:i + 1], sigma[i:i + 1])
        V0 = host(Phi[0])[:k * k].reshape(k, k).T          # column j = phi_j
        Vo = ows.warm_factors(to.ravel(), Qo, so, P)
        assert rel(V0, Vo) < tol


@pytest.mark.parametrize("batch", [7, 64])
def test_perceptron_forward_backward_adam_vs_oracle(batch):
    d = otm.ws_dims()
    g = np.random.default_rng(batch)
    ws = pws.WarmStart(torch.device("cuda:0"), seed=batch)
    p = host(ws.params)
    n_in, hid, n_out = d["n_in"], d["hidden"], d["n_out"]
    params = {"W1": p[:hid * n_in].reshape(hid, n_in), "b1": p[hid * n_in:hid * n_in + hid],
              "W2": p[hid * n_in + hid:hid * n_in + hid + n_out * hid].reshape(n_out, hid),
              "b2": p[hid * n_in + hid + n_out * hid:]}
    X = f32_round(g.standard_normal((batch, n_in)) * (g.random((batch, n_in)) < 0.3))
    Xd = to_dev(X)
    H, out = otm.mlp_forward(ws.params, Xd)
    ref, cache = ows.mlp_forward(params, X)
    torch.cuda.synchronize()
    assert rel(host(H), cache[2]) < 1e-4
    assert rel(host(out), ref) < 1e-4
    dout = f32_round(g.standard_normal((batch, n_out)) * 1e-2)
    grads = otm.mlp_backward(ws.params, Xd, H, to_dev(dout))
    gref = ows.mlp_backward(params, (X, cache[1], host(H)), dout)
    gh = host(grads)
    assert rel(gh[:hid * n_in], gref["W1"].ravel()) < 1e-4
    assert rel(gh[hid * n_in:hid * n_in + hid], gref["b1"]) < 1e-4
    off = hid * n_in + hid
    assert rel(gh[off:off + n_out * hid], gref["W2"].ravel()) < 1e-4
    assert rel(gh[off + n_out * hid:], gref["b2"]) < 1e-4
    # Adam, two steps with the same gradients, against the oracle on a slice
    m = torch.zeros_like(ws.params)
    v = torch.zeros_like(ws.params)
    P0 = ws.params.clone()
    for t in (1, 2):
        otm.mlp_adam(ws.params, grads, m, v, t, 1e-3)
    sl = slice(off - 1000, off + 1000)
    po = {"w": host(P0)[sl]}
    mo, vo = {"w": np.zeros(2000)}, {"w": np.zeros(2000)}
    for t in (1, 2):
        ows.adam_step(po, {"w": gh[sl]}, mo, vo, t, 1e-3)
    assert rel(host(ws.params)[sl], po["w"]) < 1e-5
    # BF16 inference
    ob = otm.mlp_forward_bf16(otm.mlp_to_bf16(P0), P0, Xd)
    assert rel(host(ob), ref) < 3e-2


def test_mse_vs_oracle():
    g = np.random.default_rng(3)
    ks = [4, 100, 9]
    out = f32_round(g.standard_normal((3, 10000)))
    tgt = f32_round(g.standard_normal((3, 10000)))
    kd = torch.tensor(ks, dtype=torch.int32, device="cuda")
    live = sum(k * k for k in ks)
    loss, dout = otm.ws_mse(kd, live, to_dev(out), to_dev(tgt))
    Lo, do = ows.mse(out, tgt, ks)
    assert abs(float(loss.item()) - Lo) < 1e-6 * Lo
    assert rel(host(dout), do) < 1e-6


def test_training_reduces_the_loss_and_the_warm_start_beats_random():
    """Short training on exact-moment instances (k = 4..10), then STGD from
    the network's factors and from random orthonormal factors on held-out
    instances: the warm start reaches R <= 1e-3 on more instances and needs
    fewer steps."""
    dev = torch.device("cuda:0")
    g = np.random.default_rng(0)
    train = pws.build_instances([dict(k=int(k), seed=1000 + i, kind="exact") for i, k in
                                 enumerate(g.integers(4, 11, size=4096))], dev)
    ws = pws.WarmStart(dev, seed=1)
    Q, sigma, X, tgt, info = ws.prepare(train)
    losses = ws.train(X, tgt, train.ks, epochs=20, batch=128, lr=1e-3)
    assert np.mean(losses[-8:]) < 0.2 * np.mean(losses[:8])
    held = [dict(k=int(k), seed=900000 + i, kind="exact") for i, k in enumerate(g.integers(4, 11, size=24))]
    wins = {"warm": 0, "random": 0}
    steps = {"warm": [], "random": []}
    for i, spec in enumerate(held):
        k = spec["k"]
        Y, U, lam = pws.exact_instance(k, spec["seed"])
        Yd = to_dev(Y)
        ybar = torch.stack([Yd.mean(0)] * 3).contiguous()
        T = oracle.whitened_tensor(Y.astype(np.float64), Y.astype(np.float64), Y.astype(np.float64),
                                   np.stack([Y.mean(0)] * 3).astype(np.float64), 0.0)
        Pw = ws.initial_factors(Yd, Yd, Yd, ybar, k, 0.0, seed=spec["seed"])
        Pr = to_dev(synth.initial_factors(k, seed=spec["seed"], restart=5).T.copy())
        beta = 0.05 / float(lam.max()) ** (4.0 / 3.0)
        p = otm.SgdParams(k=k, batch=k, passes=1, y_dtype=otm.F32, alpha0=0.0, beta0=beta, beta_tau=1e12)
        Ypad = padded(Y.astype(np.float64), otm.default_ldy(k), torch.float32)
        for name, P0 in (("warm", Pw), ("random", Pr)):
            Phi = P0.clone().contiguous()
            done = None
            for block in range(40):                 # 40 x 50 full-batch steps
                p50 = otm.SgdParams(k=k, batch=k, passes=50, y_dtype=otm.F32, alpha0=0.0, beta0=beta,
                                    beta_tau=1e12)
                otm.sgd_run(p50, k, Ypad, Ypad, Ypad, ybar, None, Phi)
                R = oracle.residual(T, host(Phi).T)
                if R <= 1e-3:
                    done = (block + 1) * 50
                    break
            if done is not None:
                wins[name] += 1
                steps[name].append(done)
    assert wins["warm"] > wins["random"], (wins, steps)
    assert wins["warm"] >= 0.75 * len(held)
