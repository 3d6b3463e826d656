"""Pins of the four-partition community oracle (Section 2.2 transition
matrices and moments; Section 4.1; Section 4.2 "Randomized Pseudoinverse").

* the randomized pseudo-inverse: exact on a rank-k non-square matrix (equals
  the library pseudo-inverse); with a symmetric matrix and one sketch it is the
  printed algorithm's formula; on a full-rank matrix it is the Moore-Penrose
  inverse of the two-sided Nystrom approximant (the four defining identities);
* exact moments (expected adjacency of a planted model): Z_B Pairs(B, C) =
  Pairs(A, C), Z_B F_B = F_A, Z_C F_C = F_A (the views are carried into the A
  view), and M2 equals its closed form (alpha0+1) F_A E_X[pi pi^T] F_A^T -
  alpha0 M1 M1^T; the whitened views agree row by row and W^T M2 W = I;
* end to end on exact moments of a block model (alpha0 = 0): the memberships
  of the X, B and C nodes are recovered exactly after STGD with restarts;
* Monte Carlo on sampled graphs: the three-view tensor of the four-partition
  estimator is unbiased (within sampling noise of the planted tensor) where
  the aliased single-leaf-set tensor carries the repeated-leaf bias.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import community as cm
from planted import planted_four


def _lowrank(n1, n2, k, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((n1, k)) @ g.standard_normal((k, n2))


def test_pinv_exact_rank_k_nonsquare():
    P = _lowrank(30, 23, 4, seed=1)
    X = cm.pinv_dense(P, synth.projection(30, 8, seed=2), synth.projection(23, 8, seed=3), 4)
    ref = np.linalg.pinv(P, rcond=1e-10)
    np.testing.assert_allclose(X, ref, atol=1e-10 * np.abs(ref).max())


def test_pinv_symmetric_one_sketch_is_the_printed_formula():
    """P symmetric positive semi-definite of rank k, one sketch S of k columns:
    J = P S, Psi = S^T J, SVD(J) = U_J L_J V_J^T and
    P^+ = U_J L_J^-1 V_J^T Psi V_J L_J^-1 U_J^T (Section 4.2)."""
    g = np.random.default_rng(4)
    A = g.standard_normal((20, 4))
    P = A @ A.T
    S = synth.projection(20, 4, seed=5)
    J = P @ S
    Psi = S.T @ J
    UJ, LJ, VJt = np.linalg.svd(J, full_matrices=False)
    printed = UJ @ np.diag(1.0 / LJ) @ VJt @ Psi @ VJt.T @ np.diag(1.0 / LJ) @ UJ.T
    X = cm.pinv_dense(P, S, S, 4)
    np.testing.assert_allclose(X, printed, atol=1e-11 * np.abs(printed).max())
    np.testing.assert_allclose(X, np.linalg.pinv(P, rcond=1e-10), atol=1e-11 * np.abs(printed).max())


def test_pinv_is_moore_penrose_inverse_of_the_nystrom_approximant():
    """Full-rank (noisy) P: X is the pseudo-inverse of P~ = J Psi_k^+ K^T, the
    two-sided Nystrom approximation with Psi truncated to rank k."""
    g = np.random.default_rng(6)
    P = _lowrank(40, 35, 5, seed=7) + 0.05 * g.standard_normal((40, 35))
    SL, SR = synth.projection(40, 10, seed=8), synth.projection(35, 10, seed=9)
    J, K = P @ SR, P.T @ SL
    U, s, Vt = np.linalg.svd(SL.T @ J)
    Psi_k_pinv = Vt[:5].T @ np.diag(1.0 / s[:5]) @ U[:, :5].T
    Pt = J @ Psi_k_pinv @ K.T
    X = cm.pinv_dense(P, SL, SR, 5)
    tol = 1e-10
    np.testing.assert_allclose(Pt @ X @ Pt, Pt, atol=tol * np.abs(Pt).max())
    np.testing.assert_allclose(X @ Pt @ X, X, atol=tol * np.abs(X).max())
    np.testing.assert_allclose((Pt @ X).T, Pt @ X, atol=tol)
    np.testing.assert_allclose((X @ Pt).T, X @ Pt, atol=tol)
    assert np.linalg.matrix_rank(X, tol=1e-8 * np.abs(X).max()) == 5


def test_pinv_rejects_rank_deficient_sketch():
    P = _lowrank(12, 10, 2, seed=10)
    with pytest.raises(oracle.NotPSDError):
        cm.pinv_dense(P, synth.projection(12, 6, seed=1), synth.projection(10, 6, seed=2), 4)


def _exact(alpha0, seed, sizes=None, k=4):
    sizes = sizes or dict(X=400, A=48, B=52, C=44)
    pis, P, E = planted_four(sizes, k, 0.6, 0.1, seed=seed, alpha0=alpha0)
    F = cm.transition_factors(E[("X", "A")], E[("X", "B")], E[("X", "C")],
                              synth.projection(sizes["B"], 2 * k, seed=seed + 1),
                              synth.projection(sizes["C"], 2 * k, seed=seed + 2), k)
    return pis, P, E, F


@pytest.mark.parametrize("alpha0", [0.0, 0.7])
def test_exact_moments_transition_matrices(alpha0):
    pis, P, E, F = _exact(alpha0, seed=11)
    nB, nC = 52, 44
    ZB = cm.zb(F, np.eye(nB))                  # n_A x n_B
    ZC = cm.zc(F, np.eye(nC))
    pairs = lambda r, c: cm.pairs_apply(E[("X", r)], E[("X", c)], np.eye(E[("X", c)].shape[1]))
    PAC, PBC, PAB, PCB = pairs("A", "C"), pairs("B", "C"), pairs("A", "B"), pairs("C", "B")
    np.testing.assert_allclose(ZB @ PBC, PAC, atol=1e-12 * np.abs(PAC).max())
    np.testing.assert_allclose(ZC @ PCB, PAB, atol=1e-12 * np.abs(PAB).max())
    FA, FB, FC = (pis[s].T @ P.T for s in "ABC")
    np.testing.assert_allclose(ZB @ FB, FA, atol=1e-11)
    np.testing.assert_allclose(ZC @ FC, FA, atol=1e-11)
    # the transposed products agree with the explicit matrices
    V = np.random.default_rng(0).standard_normal((48, 3))
    np.testing.assert_allclose(cm.zb_t(F, V), ZB.T @ V, atol=1e-12 * np.abs(ZB.T @ V).max())
    np.testing.assert_allclose(cm.zc_t(F, V), ZC.T @ V, atol=1e-12 * np.abs(ZC.T @ V).max())


@pytest.mark.parametrize("alpha0", [0.0, 0.7])
def test_exact_moments_m2_closed_form(alpha0):
    """Eq. 2moment_graph on the expected adjacency: the sum over samples of
    Z_C E[g_C] E[g_B]^T Z_B^T is F_A (sum_x pi_x pi_x^T) F_A^T, so
    M2 = (alpha0+1) F_A C_X F_A^T - alpha0 M1 M1^T with C_X = E_X[pi pi^T]
    and M1 = F_A E_X[pi]."""
    pis, P, E, F = _exact(alpha0, seed=12)
    FA = pis["A"].T @ P.T
    PX = pis["X"]
    CX = PX @ PX.T / PX.shape[1]
    M1 = FA @ PX.mean(axis=1)
    np.testing.assert_allclose(cm.first_moment_four(E[("X", "A")]), M1, atol=1e-14)
    ref = (alpha0 + 1.0) * FA @ CX @ FA.T - alpha0 * np.outer(M1, M1)
    M2 = cm.m2_apply_four(F, np.eye(48), alpha0)
    np.testing.assert_allclose(M2, ref, atol=1e-12 * np.abs(ref).max())


def _whiten_exact_sbm(seed):
    pis, P, E, F = _exact(0.0, seed=seed)
    k = 4
    Q, O = cm.power_sketch_four(F, synth.projection(48, k, seed=seed + 3), 0.0, 1)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    return pis, P, E, F, W


def test_exact_sbm_views_agree_and_w_whitens():
    pis, P, E, F, W = _whiten_exact_sbm(seed=13)
    M2 = cm.m2_apply_four(F, np.eye(48), 0.0)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(4), atol=1e-12)
    YA, YB, YC, ybar, WB, WC = cm.whiten_four(F, W)
    np.testing.assert_allclose(YB, YA, atol=1e-11 * np.abs(YA).max())
    np.testing.assert_allclose(YC, YA, atol=1e-11 * np.abs(YA).max())


def test_exact_sbm_memberships_recovered_for_x_b_and_c():
    pis, P, E, F, W = _whiten_exact_sbm(seed=14)
    k = 4
    YA, YB, YC, ybar, _, _ = cm.whiten_four(F, W)
    T = oracle.whitened_tensor(YA, YB, YC, ybar, 0.0)
    n = YA.shape[0]
    perms = np.tile(np.arange(n, dtype=np.int32), (800, 1))
    best, best_R = None, np.inf
    for r in range(16):             # several restarts stall one component short (R = 1/4)
        Phi = oracle.sgd_run(YA, YB, YC, ybar, synth.initial_factors(k, seed=15, restart=r), perms, batch=n,
                             beta0=0.05, tau=1e9, alpha0=0.0)
        R = oracle.residual(T, Phi)
        if R < best_R:
            best, best_R = Phi, R
    assert best_R < 1e-13          # the expanded residual's FP64 cancellation floor is about 1e-15
    Pi_X = oracle.recover_pi(YA, best, 0.0)
    # the estimated communities come in some order: match by the X nodes
    order = np.argmax(Pi_X @ pis["X"].T, axis=0)              # estimated row of each true community
    assert sorted(order) == list(range(k))
    np.testing.assert_allclose(Pi_X[order], pis["X"], atol=1e-9)
    for s in "BC":
        Pi_s = oracle.recover_pi(cm.node_views(E[(s, "A")], W), best, 0.0)
        np.testing.assert_allclose(Pi_s[order], pis[s], atol=1e-9)


def test_sampled_graph_four_partition_is_unbiased_where_aliased_is_not():
    """Sampled Bernoulli rows of a planted block model (6000 samples, 40
    leaves per set) with the transition matrices and W of the exact moments:
    the three-view tensor lies within sampling noise (3%) of the planted
    tensor, while the tensor of the aliased views (y_A = y_B = y_C) is off by
    more than 20%: its repeated-leaf terms sum_a G_xa w_a (x) w_a (x) w_a
    do not vanish in expectation."""
    k = 3
    sizes = dict(X=6000, A=40, B=40, C=40)
    pis, P, E = planted_four(sizes, k, 0.5, 0.1, seed=3)
    F = cm.transition_factors(E[("X", "A")], E[("X", "B")], E[("X", "C")], synth.projection(40, 6, seed=1),
                              synth.projection(40, 6, seed=2), k)
    Q, O = cm.power_sketch_four(F, synth.projection(40, k, seed=5), 0.0, 1)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    YA, YB, YC, yb, WB, WC = cm.whiten_four(F, W)
    T_exact = oracle.whitened_tensor(YA, YB, YC, yb, 0.0)
    g = np.random.default_rng(0)
    draw = lambda s: (g.random(E[("X", s)].shape) < E[("X", s)].toarray()).astype(float)
    GA, GB, GC = draw("A"), draw("B"), draw("C")
    ya, yb_, yc = GA @ W, GB @ WB, GC @ WC
    T4 = oracle.whitened_tensor(ya, yb_, yc, np.stack([ya.mean(0), yb_.mean(0), yc.mean(0)]), 0.0)
    Tal = oracle.whitened_tensor(ya, ya, ya, np.stack([ya.mean(0)] * 3), 0.0)
    rel = lambda T: np.linalg.norm(T - T_exact) / np.linalg.norm(T_exact)
    assert rel(T4) < 0.03
    assert rel(Tal) > 0.2


@pytest.mark.parametrize("q", [1, 2])
def test_pinv_sketches_are_krylov_images(q):
    """The refined sketches of a sampled Pairs(B, C): S_B and S_C have
    orthonormal columns, span(S_C) = span((P^T P)^q S_C0) and
    span(S_B) = span(P (P^T P)^(q-1) S_C0) (P formed explicitly)."""
    g = synth.mmsb_four(1200, 3, 0.5, 0.4, 0.05, seed=5)
    B = g.blocks
    nB, nC = B[("X", "B")].n_cols, B[("X", "C")].n_cols
    SB0, SC0 = synth.projection(nB, 6, seed=1), synth.projection(nC, 6, seed=2)
    SB, SC = cm.pinv_sketches(B[("X", "B")], B[("X", "C")], SB0, SC0, q)
    np.testing.assert_allclose(SB.T @ SB, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(SC.T @ SC, np.eye(6), atol=1e-12)
    P = cm.pairs_apply(B[("X", "B")], B[("X", "C")], np.eye(nC))
    PtP = P.T @ P
    KC = np.linalg.matrix_power(PtP, q) @ SC0
    KB = P @ np.linalg.matrix_power(PtP, q - 1) @ SC0

    def sin_max(A, Bm):
        Qa, Qb = np.linalg.qr(A)[0], np.linalg.qr(Bm)[0]
        return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))

    assert sin_max(SC, KC) < 1e-9
    assert sin_max(SB, KB) < 1e-9
    assert sin_max(SC, np.linalg.matrix_power(PtP, q - 1) @ SC0) > 1e-3


def test_refined_sketches_open_the_gap_of_a_sampled_pairs_matrix():
    """On a sampled graph the Gaussian sketch of Pairs(B, C) shows no gap at k
    in the singular values of Psi; one refinement makes s_(k+1) / s_k small
    and the whitened views B and A then point the same way."""
    k = 5
    g = synth.mmsb_four(20000, k, 0.5, 0.3, 0.02)
    B = g.blocks
    nB, nC = B[("X", "B")].n_cols, B[("X", "C")].n_cols
    SB0, SC0 = synth.projection(nB, 2 * k, seed=11), synth.projection(nC, 2 * k, seed=12)
    ratios = []
    for q in (0, 1):
        SB, SC = cm.pinv_sketches(B[("X", "B")], B[("X", "C")], SB0, SC0, q)
        s = np.linalg.svd(SB.T @ cm.pairs_apply(B[("X", "B")], B[("X", "C")], SC), compute_uv=False)
        ratios.append(s[k] / s[k - 1])
    assert ratios[0] > 0.5 and ratios[1] < 0.05


def test_poisson_counts_second_moment_is_unbiased_through_the_diagonal_correction():
    """Section 2.2 Poisson model: for counts g ~ Poisson(lambda),
    E[g g^T - diag g] = lambda lambda^T (the diagonal correction of the pair
    moment is the Poisson factorial moment).  With alpha0 = 0 the oracle's M2
    on a sampled weighted graph matches (1/n_X) sum_x lambda_x lambda_x^T, the
    conditional expectation given the memberships, within sampling noise on the
    diagonal as off it; without the correction the diagonal is off by the mean
    of lambda (about 3 times its size here)."""
    g = synth.mmsb_weighted(12000, 3, 0.3, 0.5, 0.05, n_x=11000, seed=5)
    lam = g.pi[g.X] @ g.P @ g.pi[g.A].T
    nA = len(g.A)
    M2 = oracle.m2_apply(g.C, np.eye(nA), 0.0, False)
    ref = lam.T @ lam / lam.shape[0]
    Cs = g.C.to_scipy()
    raw = np.asarray((Cs.T @ Cs).todense()) / lam.shape[0]
    off = ~np.eye(nA, dtype=bool)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(np.diag(M2), np.diag(ref)) < 0.1
    assert rel(M2[off], ref[off]) < 0.08
    assert rel(np.diag(raw), np.diag(ref)) > 2.0


def test_role_swap_recovers_the_leaf_set_memberships_exactly():
    """Lemma postprocessing: the memberships of the leaf set A come from the
    same estimator with the roles of X and A exchanged (samples A, leaves X,
    B, C).  On the exact moments of a block model they are exact."""
    k = 4
    sizes = dict(X=60, A=200, B=52, C=44)
    pis, P, E = planted_four(sizes, k, 0.6, 0.1, seed=21)
    Fs = cm.transition_factors(E[("A", "X")], E[("A", "B")], E[("A", "C")], synth.projection(52, 2 * k, seed=1),
                               synth.projection(44, 2 * k, seed=2), k)
    Q, O = cm.power_sketch_four(Fs, synth.projection(60, k, seed=3), 0.0, 1)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    YA, YB, YC, ybar, _, _ = cm.whiten_four(Fs, W)
    T = oracle.whitened_tensor(YA, YB, YC, ybar, 0.0)
    n = YA.shape[0]
    perms = np.tile(np.arange(n, dtype=np.int32), (800, 1))
    best, best_R = None, np.inf
    for r in range(16):
        Phi = oracle.sgd_run(YA, YB, YC, ybar, synth.initial_factors(k, seed=23, restart=r), perms, batch=n,
                             beta0=0.05, tau=1e9, alpha0=0.0)
        R = oracle.residual(T, Phi)
        if R < best_R:
            best, best_R = Phi, R
    assert best_R < 1e-13
    Pi_A = oracle.recover_pi(YA, best, 0.0)
    order = np.argmax(Pi_A @ pis["A"].T, axis=0)
    assert sorted(order) == list(range(k))
    np.testing.assert_allclose(Pi_A[order], pis["A"], atol=1e-9)


def test_four_partition_m2_has_rank_k_plus_one_and_a_width_k_sketch_whitens_it():
    """Z_B and Z_C have rank k (the rank-k pseudo-inverse), so the sampled
    four-partition M2 has rank at most k + 1 (the alpha0 M1 M1^T term adds
    one): a sketch of 2k columns is rank deficient.  One power step of a
    width-k sketch lies in M2's column space, and the whitener built from it
    whitens M2 on that space (READING of Section 3.1's k-SVD for this M2)."""
    k = 5
    g = synth.mmsb_four(4000, k, 0.5, 0.5, 0.05)
    B = g.blocks
    nA, nB, nC = (B[("X", s)].n_cols for s in "ABC")
    F = cm.transition_factors(B[("X", "A")], B[("X", "B")], B[("X", "C")], synth.projection(nB, 2 * k, seed=11),
                              synth.projection(nC, 2 * k, seed=12), k, q=1)
    M2 = cm.m2_apply_four(F, np.eye(nA), 0.5)
    s = np.linalg.svd(M2, compute_uv=False)
    assert s[k + 1] < 1e-10 * s[0] and s[k] > 1e-9 * s[0]
    Q, O = cm.power_sketch_four(F, synth.projection(nA, k, seed=1), 0.5, 1)
    W, _ = oracle.whitener_rsvd(O, Q, k)
    # exact: W whitens the Nystrom approximation it is built from
    Om = Q.T @ O
    Om = 0.5 * (Om + Om.T)
    sig, U = np.linalg.eigh(Om)
    Bm = O @ U / np.sqrt(sig)[None, :]
    np.testing.assert_allclose(W.T @ (Bm @ Bm.T) @ W, np.eye(k), atol=1e-11)
    # approximately M2 itself (sampled, hence not exactly symmetric)
    assert np.abs(W.T @ M2 @ W - np.eye(k)).max() < 1e-2
