"""GPU parity of the four-partition community estimator (Section 2.2, Eq.
transitionMat; Section 4.1; Section 4.2 "Randomized Pseudoinverse") against
the FP64 oracle on the same seeded graphs and projections.

FP64 stages: pairs products 1e-12 relative; the pseudo-inverse (exact rank k:
against the library pseudo-inverse, 1e-9; sampled: against the oracle's as a
product, 1e-9); Z_B^T V, Z_C^T V and the four-partition M2 operator 1e-9;
W 1e-8 after the sign rule.  FP32 stages: whitened views 1e-6 per row from the
oracle's rows of its own W, W_B, W_C rounded to FP32; the STGD run 1e-4
relative factor error; memberships of X, B and C nodes 1e-4 absolute.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_round, host, rel, to_dev
from oracle import community as cm

from paper_1309_0787_amd import otm, pipeline

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def graph():
    g = synth.mmsb_four(20000, 5, 0.5, 0.3, 0.02, seed=17)
    dev = torch.device("cuda:0")
    return g, otm.DevicePartition.from_blocks(g.blocks, dev)


def test_pairs_apply_vs_oracle(graph):
    g, G = graph
    B = g.blocks
    V = np.random.default_rng(0).standard_normal((B[("X", "C")].n_cols, 12))
    got = otm.pairs_apply(G.BX, G.XC, to_dev(V, torch.float64))
    V2 = np.random.default_rng(1).standard_normal((B[("X", "A")].n_cols, 7))
    got2 = otm.pairs_apply(G.CX, G.XA, to_dev(V2, torch.float64))
    torch.cuda.synchronize()
    assert rel(host(got), cm.pairs_apply(B[("X", "B")], B[("X", "C")], V)) < 1e-12
    assert rel(host(got2), cm.pairs_apply(B[("X", "C")], B[("X", "A")], V2)) < 1e-12


def test_pinv_factors_exact_rank_k():
    g = np.random.default_rng(2)
    n1, n2, k, m = 300, 250, 5, 10
    P = g.standard_normal((n1, k)) @ g.standard_normal((k, n2))
    SL, SR = synth.projection(n1, m, seed=3), synth.projection(n2, m, seed=4)
    F = otm.pinv_factors(to_dev(P @ SR, torch.float64), to_dev(P.T @ SL, torch.float64), to_dev(SL, torch.float64), k)
    torch.cuda.synchronize()
    X = host(F.QK) @ host(F.core) @ host(F.QJ).T
    ref = np.linalg.pinv(P, rcond=1e-10)
    assert rel(X, ref) < 1e-9
    sv = np.linalg.svd(SL.T @ P @ SR, compute_uv=False)[:k]
    np.testing.assert_allclose(host(F.sv), sv, rtol=1e-10)


def test_pinv_factors_sampled_vs_oracle_and_rank_deficient():
    g = np.random.default_rng(5)
    n1, n2, k, m = 400, 350, 6, 12
    P = g.standard_normal((n1, k)) @ g.standard_normal((k, n2)) + 0.3 * g.standard_normal((n1, n2))
    SL, SR = synth.projection(n1, m, seed=6), synth.projection(n2, m, seed=7)
    J, K = P @ SR, P.T @ SL
    F = otm.pinv_factors(to_dev(J, torch.float64), to_dev(K, torch.float64), to_dev(SL, torch.float64), k)
    torch.cuda.synchronize()
    QK, core, QJ = cm.pinv_factors(J, K, SL, k)
    assert rel(host(F.QK) @ host(F.core) @ host(F.QJ).T, QK @ core @ QJ.T) < 1e-9
    # a sketch of rank 2 has no rank-4 part
    P2 = g.standard_normal((n1, 2)) @ g.standard_normal((2, n2))
    with pytest.raises(otm.OtmNotPSD):
        otm.pinv_factors(to_dev(P2 @ SR, torch.float64), to_dev(P2.T @ SL, torch.float64), to_dev(SL, torch.float64), 4)


def _factors_both(g, G, k, q_pinv):
    B = g.blocks
    nB, nC = B[("X", "B")].n_cols, B[("X", "C")].n_cols
    SB0, SC0 = synth.projection(nB, 2 * k, seed=11), synth.projection(nC, 2 * k, seed=12)
    Fo = cm.transition_factors(B[("X", "A")], B[("X", "B")], B[("X", "C")], SB0, SC0, k, q=q_pinv)
    SB, SC = to_dev(SB0, torch.float64), to_dev(SC0, torch.float64)
    for _ in range(q_pinv):
        SB = otm.orthonormalize(otm.pairs_apply(G.BX, G.XC, SC))
        SC = otm.orthonormalize(otm.pairs_apply(G.CX, G.XB, SB))
    Fg = otm.pinv_factors(otm.pairs_apply(G.BX, G.XC, SC), otm.pairs_apply(G.CX, G.XB, SB), SB, k)
    return Fo, Fg


@pytest.mark.parametrize("q_pinv", [0, 1])
def test_transition_products_and_m2_four_vs_oracle(graph, q_pinv):
    g, G = graph
    k = 5
    Fo, Fg = _factors_both(g, G, k, q_pinv)
    nA = g.blocks[("X", "A")].n_cols
    V = np.random.default_rng(8).standard_normal((nA, 2 * k))
    Vd = to_dev(V, torch.float64)
    zb = otm.transition_t_apply(G, Fg, 1, Vd)
    zc = otm.transition_t_apply(G, Fg, 2, Vd)
    O = otm.m2_apply_four(G, Fg, 0.5, Vd)
    torch.cuda.synchronize()
    assert rel(host(zb), cm.zb_t(Fo, V)) < 1e-9
    assert rel(host(zc), cm.zc_t(Fo, V)) < 1e-9
    assert rel(host(O), cm.m2_apply_four(Fo, V, 0.5)) < 1e-9


def test_cast_rows_rounding_and_padding():
    X = np.random.default_rng(9).standard_normal((37, 13))
    for dt, rnd in ((otm.F32, f32_round), (otm.BF16, None)):
        out = otm.cast_rows(to_dev(X, torch.float64), dt)
        torch.cuda.synchronize()
        full = out.as_strided((37, out.stride(0)), (out.stride(0), 1))
        assert torch.all(full[:, 13:] == 0)
        want = rnd(X) if rnd else torch.as_tensor(X.astype(np.float32)).to(torch.bfloat16).double().numpy()
        np.testing.assert_array_equal(host(out), want)


def test_fit_four_vs_oracle_and_planted(graph):
    """The whole four-partition path (FP32 views and STGD) against the
    oracle's, and its memberships against the planted ones."""
    g, G = graph
    k, a0 = 5, 0.5
    B = g.blocks
    sets = g.sets
    nA, nB, nC = (B[("X", s)].n_cols for s in "ABC")
    S, SB0, SC0 = (synth.projection(nA, k, seed=1), synth.projection(nB, 2 * k, seed=11),
                   synth.projection(nC, 2 * k, seed=12))
    n = B[("X", "A")].n_rows
    passes = 30
    perms = synth.permutations(n, passes, seed=2)
    Phi0 = synth.initial_factors(k, seed=4)
    cfg = pipeline.FitConfig(k=k, alpha0=a0, q_power=1, y_dtype=otm.F32, batch=100, passes=passes, beta0=1e-3,
                             beta_tau=2500.0, tau_pi=0.0)
    dev = torch.device("cuda:0")
    Phi = to_dev(Phi0.T.copy(), torch.float32)[None].contiguous()
    blocks = [otm.DeviceCSR.from_host(B[(s, "A")], dev) for s in "BC"]
    res = pipeline.fit_four(G, to_dev(S, torch.float64), to_dev(SB0, torch.float64), to_dev(SC0, torch.float64), Phi,
                            to_dev(perms, torch.int32), cfg, q_pinv=1, node_blocks=blocks)
    torch.cuda.synchronize()
    assert int(res.nonfinite.item()) == 0
    # oracle path
    Fo = cm.transition_factors(B[("X", "A")], B[("X", "B")], B[("X", "C")], SB0, SC0, k, q=1)
    Qo, Oo = cm.power_sketch_four(Fo, S, a0, 1)
    Wo, _ = oracle.whitener_rsvd(Oo, Qo, k)
    assert rel(host(res.W), Wo) < 1e-8
    WBo, WCo = cm.zb_t(Fo, Wo), cm.zc_t(Fo, Wo)
    assert rel(host(res.WB), WBo) < 1e-8 and rel(host(res.WC), WCo) < 1e-8
    Ys = []
    for i, (blk, Wv) in enumerate(((B[("X", "A")], Wo), (B[("X", "B")], WBo), (B[("X", "C")], WCo))):
        Yo, _ = oracle.whiten(blk, f32_round(Wv), False)
        Yg = host(res.Y[i])[:, :k]
        err = np.linalg.norm(Yg - Yo, axis=1) / np.maximum(np.linalg.norm(Yo, axis=1), 1e-300)
        assert err.max() < 1e-6, (i, err.max())
        Ys.append(f32_round(Yo))
    yb = np.stack([Y.mean(0) for Y in Ys])
    Phi_o = oracle.sgd_run(Ys[0], Ys[1], Ys[2], yb, Phi0, perms, 100, 1e-3, 2500.0, a0)
    assert rel(host(res.Phi[0]).T, Phi_o) <= 1e-4
    Pi_o = oracle.recover_pi(Ys[0], Phi_o, 0.0)
    assert np.abs(host(res.Pi) - Pi_o).max() < 1e-4
    for s, Pg in zip("BC", res.Pi_nodes):
        Pn = oracle.recover_pi(cm.node_views(B[(s, "A")], Wo), Phi_o, 0.0)
        assert np.abs(host(Pg) - Pn).max() < 1e-4
