"""GPU parity of the model variants against the FP64 oracle on the same seeded
inputs:

* column-selection projection for a sparse M2 (Section 4.2): O = M2 S for
  documents, graphs and weighted graphs (1e-12 relative), its dense S, and the
  whitener from it on an exact rank-k M2 (1e-9);
* the Poisson model of Section 2.2 (weighted edges): the whole path (FP32
  views and STGD) on a weighted graph (W 1e-8; views per row within
  4 sqrt(entries) 2^-24 of the row's absolute mass, the FP32 accumulation
  bound; factors 1e-4, memberships 1e-4);
* the role swap of Lemma postprocessing: memberships of the leaf set A from
  the same path with samples and leaves exchanged (1e-4);
* a bipartite weighted graph (the business-user setting of Section 6):
  memberships of both sides (1e-4);
* the four-partition estimator on a weighted graph, and with X and A
  exchanged (memberships of A, 1e-4).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import f32_round, host, rel, to_dev
from oracle import community as cm
from planted import exact_m2, planted_topics

from paper_1309_0787_amd import otm, pipeline

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("kind", ["documents", "graph", "weighted"])
def test_m2_apply_select_vs_oracle(kind):
    if kind == "documents":
        inst = synth.lda(d=3000, k=5, alpha0=1.0, beta=0.1, n_docs=20000, mean_len=60.0, seed=3)
        C, CT, norm, a0 = inst.C, inst.CT, True, 1.0
    elif kind == "graph":
        g = synth.mmsb(20000, 5, 0.5, 0.3, 0.02, n_x=10000, seed=4)
        C, CT, norm, a0 = g.C, g.CT, False, 0.5
    else:
        g = synth.mmsb_weighted(20000, 5, 0.5, 0.3, 0.02, n_x=10000, seed=5)
        C, CT, norm, a0 = g.C, g.CT, False, 0.5
    d = C.n_cols
    rows, signs = synth.column_selection(d, 24, seed=7)
    O = otm.m2_apply_select(otm.DeviceCSR.from_host(C, _dev()), otm.DeviceCSR.from_host(CT, _dev()), norm, a0,
                            to_dev(rows, torch.int32), to_dev(signs, torch.float64))
    Sd = otm.selection_dense(to_dev(rows, torch.int32), to_dev(signs, torch.float64), d)
    torch.cuda.synchronize()
    S = synth.selection_dense(rows, signs, d)
    np.testing.assert_array_equal(host(Sd), S)
    assert rel(host(O), oracle.m2_apply(C, S, a0, norm)) < 1e-12


def test_m2_apply_select_rejects_a_row_out_of_range():
    g = synth.mmsb(2000, 3, 0.5, 0.3, 0.02, n_x=1000, seed=4)
    rows = np.array([0, 5, g.C.n_cols], dtype=np.int32)
    with pytest.raises(otm.OtmError):
        otm.m2_apply_select(otm.DeviceCSR.from_host(g.C, _dev()), otm.DeviceCSR.from_host(g.CT, _dev()), False, 0.5,
                            to_dev(rows, torch.int32), to_dev(np.ones(3), torch.float64))


def test_whitener_from_a_column_selection_on_exact_rank_k():
    d, k = 800, 8
    mu, ahat = planted_topics(d, k, seed=9, beta=1.0)
    M2 = exact_m2(mu, ahat)
    rows, signs = synth.column_selection(d, 2 * k, seed=1)
    S = synth.selection_dense(rows, signs, d)
    W, ev, _ = otm.whitener(to_dev(M2 @ S, torch.float64), to_dev(S, torch.float64), k, w_lo_dtype=None)
    torch.cuda.synchronize()
    Wo, _ = oracle.whitener_rsvd(M2 @ S, S, k)
    assert rel(host(W), Wo) < 1e-9
    np.testing.assert_allclose(host(W).T @ M2 @ host(W), np.eye(k), atol=1e-10)


def _aliased_both(C, CT, k, a0, passes, seed, pi_rows):
    """GPU fit and the oracle's path on the same samples C (rows), FP32."""
    S = synth.projection(C.n_cols, 2 * k, seed=seed)
    n = C.n_rows
    perms = synth.permutations(n, passes, seed=seed + 1)
    Phi0 = synth.initial_factors(k, seed=seed + 2)
    cfg = pipeline.FitConfig(k=k, alpha0=a0, q_power=3, y_dtype=otm.F32, batch=100, passes=passes, beta0=1e-3,
                             beta_tau=2500.0, tau_pi=0.0)
    Cd, CTd = otm.DeviceCSR.from_host(C, _dev()), otm.DeviceCSR.from_host(CT, _dev())
    Phi = to_dev(Phi0.T.copy(), torch.float32)[None].contiguous()
    res = pipeline.fit([Cd], Cd, CTd, to_dev(S, torch.float64), Phi, to_dev(perms, torch.int32), cfg, pi_view=0)
    torch.cuda.synchronize()
    Q, O = oracle.power_sketch(C, S, a0, False, 3)
    Wo, _ = oracle.whitener_rsvd(O, Q, k)
    assert rel(host(res.W), Wo) < 1e-8
    Wf = f32_round(Wo)
    Yo, _ = oracle.whiten(C, Wf, False)
    Yg = host(res.Y[0])[:, :k]
    # FP32 accumulation over a row's stored entries: 4 sqrt(entries) 2^-24 of
    # the row's absolute mass sum_j |c_j| |W_j| (weighted rows cancel more)
    Cs = C.to_scipy(np.float64)
    mass = np.linalg.norm(abs(Cs) @ np.abs(Wf), axis=1)
    bound = 4.0 * np.sqrt(np.maximum(np.diff(Cs.indptr), 1)) * 2.0 ** -24 * mass
    assert np.all(np.linalg.norm(Yg - Yo, axis=1) <= bound + 1e-30)
    Yh = f32_round(Yo)
    yb = np.stack([Yh.mean(0)] * 3)
    Phi_o = oracle.sgd_run(Yh, Yh, Yh, yb, Phi0, perms, 100, 1e-3, 2500.0, a0)
    assert rel(host(res.Phi[0]).T, Phi_o) <= 1e-4
    Pi_o = oracle.recover_pi(Yh, Phi_o, 0.0)
    assert np.abs(host(res.Pi) - Pi_o).max() < 1e-4
    return res


def test_poisson_weighted_graph_path_and_role_swap_vs_oracle():
    g = synth.mmsb_weighted(20000, 5, 0.5, 0.3, 0.02, n_x=10000, seed=11)
    assert g.C.vals is not None and g.C.vals.max() >= 2.0
    _aliased_both(g.C, g.CT, 5, 0.5, 20, 21, g.pi[g.X])
    # memberships of the leaf set: samples and leaves exchanged
    _aliased_both(g.CT, g.C, 5, 0.5, 20, 31, g.pi[g.A])


def test_bipartite_weighted_graph_both_sides_vs_oracle():
    b = synth.bipartite(12000, 9000, 5, 0.5, 0.3, 0.02, poisson=True, seed=13)
    _aliased_both(b.C, b.CT, 5, 0.5, 20, 41, b.pi_u)
    _aliased_both(b.CT, b.C, 5, 0.5, 20, 51, b.pi_v)


def _four_both(blocks, names, k, a0, passes, seed):
    """fit_four on the partition named (samples, leaf A, leaf B, leaf C) and
    the oracle's path; memberships of the samples compared."""
    Xn, An, Bn, Cn = names
    B = blocks
    part = {("X", "A"): B[(Xn, An)], ("X", "B"): B[(Xn, Bn)], ("X", "C"): B[(Xn, Cn)],
            ("A", "X"): B[(An, Xn)], ("B", "X"): B[(Bn, Xn)], ("C", "X"): B[(Cn, Xn)]}
    G = otm.DevicePartition.from_blocks(part, _dev())
    nA, nB, nC = (part[("X", s)].n_cols for s in "ABC")
    S, SB0, SC0 = (synth.projection(nA, k, seed=seed), synth.projection(nB, 2 * k, seed=seed + 1),
                   synth.projection(nC, 2 * k, seed=seed + 2))
    n = part[("X", "A")].n_rows
    perms = synth.permutations(n, passes, seed=seed + 3)
    Phi0 = synth.initial_factors(k, seed=seed + 4)
    cfg = pipeline.FitConfig(k=k, alpha0=a0, q_power=1, y_dtype=otm.F32, batch=100, passes=passes, beta0=1e-3,
                             beta_tau=2500.0)
    Phi = to_dev(Phi0.T.copy(), torch.float32)[None].contiguous()
    res = pipeline.fit_four(G, to_dev(S, torch.float64), to_dev(SB0, torch.float64), to_dev(SC0, torch.float64), Phi,
                            to_dev(perms, torch.int32), cfg, q_pinv=1)
    torch.cuda.synchronize()
    Fo = cm.transition_factors(part[("X", "A")], part[("X", "B")], part[("X", "C")], SB0, SC0, k, q=1)
    Qo, Oo = cm.power_sketch_four(Fo, S, a0, 1)
    Wo, _ = oracle.whitener_rsvd(Oo, Qo, k)
    assert rel(host(res.W), Wo) < 1e-8
    Ys = [f32_round(oracle.whiten(part[("X", s)], f32_round(Wv), False)[0])
          for s, Wv in zip("ABC", (Wo, cm.zb_t(Fo, Wo), cm.zc_t(Fo, Wo)))]
    yb = np.stack([Y.mean(0) for Y in Ys])
    Phi_o = oracle.sgd_run(Ys[0], Ys[1], Ys[2], yb, Phi0, perms, 100, 1e-3, 2500.0, a0)
    assert rel(host(res.Phi[0]).T, Phi_o) <= 1e-4
    assert np.abs(host(res.Pi) - oracle.recover_pi(Ys[0], Phi_o, 0.0)).max() < 1e-4


def test_four_partition_weighted_graph_and_role_swap_vs_oracle():
    g = synth.mmsb_four(20000, 5, 0.5, 0.3, 0.02, seed=17, poisson=True)
    _four_both(g.blocks, "XABC", 5, 0.5, 20, 61)
    _four_both(g.blocks, "AXBC", 5, 0.5, 20, 71)
