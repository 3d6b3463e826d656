"""Pins of the oracle's whitening (Section 3.1 and Section 4.2).

* closed form: on an exact rank-k M2 the randomized whitener equals the
  definition W = U_M2 Sigma_M2^(-1/2) computed from a dense eigendecomposition
  of the explicit M2 (same sign rule), and W^T M2 W = I;
* the whitened samples are the definition y = W^T c / l, checked row by row.
"""
import numpy as np
import pytest

import oracle
import synth
from planted import exact_m2, planted_topics


@pytest.mark.parametrize("d,k", [(12, 3), (40, 7), (200, 10)])
def test_whitener_exact_rank_k(d, k):
    mu, ahat = planted_topics(d, k, seed=d + k)
    M2 = exact_m2(mu, ahat)
    S = synth.projection(d, 2 * k, seed=7)
    W, evals = oracle.whitener_rsvd(M2 @ S, S, k)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(k), atol=1e-12)
    # the definition of Section 3.1 through a dense eigendecomposition
    lam, U = np.linalg.eigh(M2)
    order = np.argsort(-lam)[:k]
    W_def = oracle.canonical_signs(U[:, order] / np.sqrt(lam[order])[None, :])
    np.testing.assert_allclose(W, W_def, atol=1e-10 * np.abs(W_def).max())
    np.testing.assert_allclose(evals, lam[order], rtol=1e-11)


def test_whitener_projection_size_independent():
    """Nystrom with any k_tilde >= k recovers the same W on an exact rank-k M2."""
    mu, ahat = planted_topics(30, 4, seed=9)
    M2 = exact_m2(mu, ahat)
    Ws = []
    for kt in (4, 8, 13):
        S = synth.projection(30, kt, seed=kt)
        Ws.append(oracle.whitener_rsvd(M2 @ S, S, 4)[0])
    np.testing.assert_allclose(Ws[0], Ws[1], atol=1e-10)
    np.testing.assert_allclose(Ws[0], Ws[2], atol=1e-10)


@pytest.mark.parametrize("q", [1, 3])
def test_power_sketch_exact_rank_k_gives_the_definition(q):
    """Power iterations keep an exact rank-k M2's whitener: W = U Sigma^(-1/2)."""
    d, k = 60, 5
    mu, ahat = planted_topics(d, k, seed=17)
    M2 = exact_m2(mu, ahat)
    S = synth.projection(d, 2 * k, seed=3)
    Q = S
    for _ in range(q):
        Q = np.linalg.qr(M2 @ Q)[0]
    W, _ = oracle.whitener_rsvd(M2 @ Q, Q, k)
    lam, U = np.linalg.eigh(M2)
    order = np.argsort(-lam)[:k]
    W_def = oracle.canonical_signs(U[:, order] / np.sqrt(lam[order])[None, :])
    np.testing.assert_allclose(W, W_def, atol=1e-9 * np.abs(W_def).max())


def test_power_sketch_repairs_indefinite_projection():
    """Sampled graph moment: the plain width-2k sketch is indefinite at rank k,
    three power iterations make it definite and the whitener is then as good
    as the dense top-k eigendecomposition of the same M2."""
    g = synth.make("mmsb_small")
    k = 10
    S = synth.projection(g.C.n_cols, 2 * k, seed=1)
    with pytest.raises(oracle.NotPSDError):
        oracle.whitener_rsvd(oracle.m2_apply(g.C, S, 0.1, False), S, k)
    Q, O = oracle.power_sketch(g.C, S, 0.1, False, 3)
    W, ev = oracle.whitener_rsvd(O, Q, k)
    M2 = oracle.m2_apply(g.C, np.eye(g.C.n_cols), 0.1, False)
    lam = np.sort(np.linalg.eigvalsh(M2))[::-1][:k]
    np.testing.assert_allclose(ev, lam, rtol=0.05)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(k), atol=0.1)


def test_whitener_rejects_indefinite():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((10, 10))
    M2 = -(A @ A.T)
    S = synth.projection(10, 6, seed=1)
    with pytest.raises(oracle.NotPSDError):
        oracle.whitener_rsvd(M2 @ S, S, 3)


def test_canonical_signs_rule():
    W = np.array([[1.0, -3.0, 2.0], [-2.0, 1.0, -2.0], [0.5, 2.9, 1.0]])
    V = oracle.canonical_signs(W)
    np.testing.assert_array_equal(V[:, 0], [-1.0, 2.0, -0.5])
    np.testing.assert_array_equal(V[:, 1], [3.0, -1.0, -2.9])
    np.testing.assert_array_equal(V[:, 2], [2.0, -2.0, 1.0])   # tie: lowest row wins


def test_whiten_rows_definition():
    inst = synth.lda(d=15, k=2, alpha0=1.0, beta=0.5, n_docs=30, mean_len=9.0, seed=4)
    W = synth.projection(15, 4, seed=2)
    for v in inst.views:
        Y, ybar = oracle.whiten(v, W, normalize=True)
        dense = v.to_scipy(np.float64).toarray()
        for t in range(dense.shape[0]):
            np.testing.assert_allclose(Y[t], W.T @ dense[t] / dense[t].sum(), atol=1e-14)
        np.testing.assert_allclose(ybar, Y.sum(0) / Y.shape[0], atol=1e-15)
    g = synth.mmsb(n=50, k=2, alpha0=0.3, p=0.5, q=0.1, n_x=25, seed=1)
    Wg = synth.projection(g.C.n_cols, 3, seed=5)
    Y, _ = oracle.whiten(g.C, Wg, normalize=False)
    np.testing.assert_allclose(Y, g.C.to_scipy(np.float64).toarray() @ Wg, atol=1e-13)


def test_sampled_graph_whitener_invariant_on_low_rank_m2():
    """On sampled data W whitens the Nystrom approximation O Omega^+ O^T
    restricted to its top k (the matrix it is built from)."""
    g = synth.mmsb(n=400, k=4, alpha0=0.2, p=0.5, q=0.05, n_x=200, seed=3)
    S = synth.projection(g.C.n_cols, 8, seed=9)
    O = oracle.m2_apply(g.C, S, 0.2, normalize=False)
    W, _ = oracle.whitener_rsvd(O, S, 4)
    Om = S.T @ O
    Om = 0.5 * (Om + Om.T)
    sig, U = np.linalg.eigh(Om)
    idx = np.argsort(-sig)[:4]
    B = O @ U[:, idx] / np.sqrt(sig[idx])
    np.testing.assert_allclose(W.T @ (B @ B.T) @ W, np.eye(4), atol=1e-11)


def _principal_angle_max(A: np.ndarray, B: np.ndarray) -> float:
    """Sine of the largest principal angle between span(A) and span(B) (equal
    widths): the spectral norm of the part of B's basis outside span(A)."""
    Qa = np.linalg.qr(A)[0]
    Qb = np.linalg.qr(B)[0]
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


@pytest.mark.parametrize("q", [0, 1, 3])
def test_power_sketch_steps_against_dense_m2(q):
    """The power-iterated sketch (reading of Section 4.2 for sampled moments),
    checked against the explicitly formed M2 of a sampled graph: the returned
    O is M2 applied to the returned Q, Q has orthonormal columns (q >= 1;
    q = 0 returns S itself), and span(Q) is span(M2^q S), the q-th Krylov
    image of the projection (an extra or missing iteration moves the span)."""
    g = synth.make("mmsb_small")
    d = g.C.n_cols
    M2 = oracle.m2_apply(g.C, np.eye(d), 0.1, False)
    # the explicit M2 is the pair enumeration's: symmetric, as Section 2.2 defines it
    np.testing.assert_allclose(M2, M2.T, atol=1e-14)
    S = synth.projection(d, 20, seed=1)
    Q, O = oracle.power_sketch(g.C, S, 0.1, False, q)
    np.testing.assert_allclose(O, M2 @ Q, atol=1e-12 * np.abs(M2 @ Q).max())
    if q == 0:
        np.testing.assert_array_equal(Q, S)
    else:
        np.testing.assert_allclose(Q.T @ Q, np.eye(20), atol=1e-12)
    K = S.copy()
    for _ in range(q):
        K = M2 @ K
    assert _principal_angle_max(Q, K) < 1e-10
    # the spans of neighbouring iteration counts are far apart on this graph
    if q >= 1:
        assert _principal_angle_max(Q, np.linalg.matrix_power(M2, q - 1) @ S) > 1e-3
    assert _principal_angle_max(Q, np.linalg.matrix_power(M2, q + 1) @ S) > 1e-3


@pytest.mark.parametrize("normalize", [True, False])
def test_column_selection_sketch_is_signed_columns_of_m2(normalize):
    """Section 4.2, sparse M2: with S a column selection with random signs,
    O = M2 S holds the selected columns of M2 with their signs, and
    S^T O holds the selected entries M2[r_i, r_j] s_i s_j."""
    if normalize:
        inst = synth.lda(d=40, k=3, alpha0=0.8, beta=0.3, n_docs=300, mean_len=12.0, seed=6)
        C, a0 = inst.C, 0.8
    else:
        C, a0 = synth.mmsb(300, 3, 0.3, 0.4, 0.05, n_x=150, seed=6).C, 0.3
    d = C.n_cols
    M2 = oracle.m2_apply(C, np.eye(d), a0, normalize)
    rows, signs = synth.column_selection(d, 9, seed=2)
    S = synth.selection_dense(rows, signs, d)
    assert len(set(rows.tolist())) == 9 and set(np.abs(signs)) == {1.0}
    O = oracle.m2_apply(C, S, a0, normalize)
    np.testing.assert_allclose(O, M2[:, rows] * signs[None, :], atol=1e-14 * np.abs(M2).max())
    np.testing.assert_allclose(S.T @ O, M2[np.ix_(rows, rows)] * np.outer(signs, signs), atol=1e-14 * np.abs(M2).max())


def test_whitener_with_column_selection_on_exact_rank_k():
    """A column-selection sketch of width 2k of an exact rank-k M2 (whose
    selected columns span its range) gives the whitener of the definition."""
    d, k = 60, 5
    mu, ahat = planted_topics(d, k, seed=31, beta=2.0)
    M2 = exact_m2(mu, ahat)
    rows, signs = synth.column_selection(d, 2 * k, seed=3)
    S = synth.selection_dense(rows, signs, d)
    W, evals = oracle.whitener_rsvd(M2 @ S, S, k)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(k), atol=1e-11)
    lam, U = np.linalg.eigh(M2)
    order = np.argsort(-lam)[:k]
    W_def = oracle.canonical_signs(U[:, order] / np.sqrt(lam[order])[None, :])
    np.testing.assert_allclose(W, W_def, atol=1e-9 * np.abs(W_def).max())
