"""FP64 oracle of the four-partition community estimator (TEST
INFRASTRUCTURE, like the rest of this package: only tests, the smoke check and
the benchmark's CPU-baseline leg use it).

Section 2.2 splits the nodes into a sample set X and three leaf sets A, B, C.
With Pairs(Y1, Y2) = G[X, Y1]^T G[X, Y2] (the pair counts of the samples'
edges into Y1 and Y2), the transition matrices of Eq. transitionMat,
    Z_B = Pairs(A, C) Pairs(B, C)^+,      Z_C = Pairs(A, B) Pairs(C, B)^+,
carry the B and C views into the A view, so that the three whitened views
    y_A = W^T G[x, A]^T,  y_B = W^T Z_B G[x, B]^T,  y_C = W^T Z_C G[x, C]^T
(Section 4.1 and Appendix A) are conditionally independent copies of one
vector and the third moment has no repeated-leaf terms.  The second moment is
Eq. 2moment_graph:
    M2 = (alpha0+1)/n_X sum_x Z_C G[x, C]^T G[x, B] Z_B^T - alpha0 M1 M1^T,
    M1 = (1/n_X) sum_x G[x, A]^T                       (Eq. 1moment_graph).
Nothing n x n is formed: the pseudo-inverse stays in factored low-rank form
(Section 4.1) and every product is applied to a thin matrix.

READINGS:
* Pairs carries the factor 1/n_X of the moments; Z_B and Z_C do not depend on
  it.
* The randomized pseudo-inverse (Section 4.2, algorithm "Randomized
  Pseudoinverse") is printed for a square, symmetric Pairs with one sketch S:
  J = Pairs S, Psi = S^T J, Pairs^+ ~ U_J L_J^-1 V_J^T Psi V_J L_J^-1 U_J^T.
  Pairs(B, C) is neither square nor symmetric, so the same Nystrom form is
  taken from both sides: J = P S_C, K = P^T S_B, Psi = S_B^T P S_C, which
  approximates P by J Psi^+ K^T and gives P^+ ~ (K^T)^+ Psi J^+; with P
  symmetric and S_B = S_C this is the printed formula (pinned).  As for the
  whitener, the sketches have k_tilde = 2k columns and Psi is truncated to
  its top k singular triplets before it is inverted.
* Also as for the whitener, a Gaussian sketch of a sampled Pairs matrix is
  swamped by its flat noise spectrum (no gap at k in the singular values of
  Psi), so the two sketches are refined by q alternating range-finder steps
  S_B <- orth(P S_C), S_C <- orth(P^T S_B) before J, K and Psi are taken;
  q = 0 is the printed algorithm.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .otm import NotPSDError, as_sparse, power_sketch_op, whiten

__all__ = ["pairs_apply", "pinv_sketches", "pinv_factors", "pinv_dense", "transition_factors", "zb_t", "zc_t", "zb", "zc",
           "first_moment_four", "m2_apply_four", "power_sketch_four", "whiten_four", "node_views"]


def pairs_apply(G1, G2, V: np.ndarray) -> np.ndarray:
    """Pairs(Y1, Y2) V = (1/n_X) G[X, Y1]^T (G[X, Y2] V) for G1 = G[X, Y1],
    G2 = G[X, Y2] (Section 2.2, Pairs(Y1, Y2) = G[X, Y1]^T (x) G[X, Y2]^T
    summed over the samples)."""
    A1, A2 = as_sparse(G1), as_sparse(G2)
    return np.asarray(A1.T @ (A2 @ V)) / A1.shape[0]


def pinv_factors(J: np.ndarray, K: np.ndarray, S_left: np.ndarray, k: int, rel_floor: float = 1e-12):
    """Rank-k randomized pseudo-inverse of P (n1 x n2) from its sketches
    J = P S_right (n1 x m), K = P^T S_left (n2 x m) (Section 4.2, algorithm
    "Randomized Pseudoinverse", two-sided READING of the module docstring):
      Psi = S_left^T J = U diag(s) V^T (SVD), top k kept;
      J' = J V_k = Q_J R_J,  K' = K U_k = Q_K R_K   (thin QR);
      P ~ J' diag(s_k)^-1 K'^T  and  P^+ ~ Q_K Core Q_J^T,
      Core = R_K^-T diag(s_k) R_J^-1.
    Returns (Q_K (n2 x k), Core (k x k), Q_J (n1 x k)).  Raises NotPSDError
    when s_k <= rel_floor s_1 (Psi has no rank-k part to invert)."""
    Psi = S_left.T @ J
    U, s, Vt = np.linalg.svd(Psi)
    if not (s[k - 1] > rel_floor * s[0]):
        raise NotPSDError(f"s_k = {s[k - 1]:.3e} (s_1 = {s[0]:.3e})")
    Jk = J @ Vt[:k].T
    Kk = K @ U[:, :k]
    QJ, RJ = np.linalg.qr(Jk)
    QK, RK = np.linalg.qr(Kk)
    core = np.linalg.solve(RK.T, np.diag(s[:k])) @ np.linalg.inv(RJ)
    return QK, core, QJ


def pinv_dense(P: np.ndarray, S_left: np.ndarray, S_right: np.ndarray, k: int) -> np.ndarray:
    """The randomized pseudo-inverse of a dense P as an explicit n2 x n1 matrix."""
    QK, core, QJ = pinv_factors(P @ S_right, P.T @ S_left, S_left, k)
    return QK @ core @ QJ.T


def pinv_sketches(GXB, GXC, S_B: np.ndarray, S_C: np.ndarray, q: int):
    """The sketches of P = Pairs(B, C) after q alternating range-finder steps
    (READING of the module docstring): S_B <- orth(P S_C), S_C <- orth(P^T S_B).
    span(S_C) is then span((P^T P)^q S_C) and span(S_B) span(P (P^T P)^(q-1) S_C)."""
    for _ in range(q):
        S_B = np.linalg.qr(pairs_apply(GXB, GXC, S_C))[0]
        S_C = np.linalg.qr(pairs_apply(GXC, GXB, S_B))[0]
    return S_B, S_C


def transition_factors(GXA, GXB, GXC, S_B: np.ndarray, S_C: np.ndarray, k: int, q: int = 0) -> dict:
    """Factors of Pairs(B, C)^+ (Eq. transitionMat) from the sketches
    J = Pairs(B, C) S_C (n_B x m) and K = Pairs(C, B) S_B (n_C x m), after q
    refinements of the sketches (pinv_sketches):
    Pairs(B, C)^+ ~ Q_K Core Q_J^T and Pairs(C, B)^+ = its transpose, so both
    Z_B and Z_C use one factorisation."""
    S_B, S_C = pinv_sketches(GXB, GXC, S_B, S_C, q)
    J = pairs_apply(GXB, GXC, S_C)
    K = pairs_apply(GXC, GXB, S_B)
    QK, core, QJ = pinv_factors(J, K, S_B, k)
    return {"QK": QK, "core": core, "QJ": QJ, "GXA": GXA, "GXB": GXB, "GXC": GXC}


def zb_t(F: dict, V: np.ndarray) -> np.ndarray:
    """Z_B^T V = (Pairs(B, C)^+)^T Pairs(A, C)^T V = Q_J Core^T Q_K^T Pairs(C, A) V."""
    X = pairs_apply(F["GXC"], F["GXA"], V)
    return F["QJ"] @ (F["core"].T @ (F["QK"].T @ X))


def zc_t(F: dict, V: np.ndarray) -> np.ndarray:
    """Z_C^T V = (Pairs(C, B)^+)^T Pairs(A, B)^T V = Q_K Core Q_J^T Pairs(B, A) V."""
    X = pairs_apply(F["GXB"], F["GXA"], V)
    return F["QK"] @ (F["core"] @ (F["QJ"].T @ X))


def zb(F: dict, U: np.ndarray) -> np.ndarray:
    """Z_B U = Pairs(A, C) Q_K Core Q_J^T U  (U: n_B x m)."""
    return pairs_apply(F["GXA"], F["GXC"], F["QK"] @ (F["core"] @ (F["QJ"].T @ U)))


def zc(F: dict, U: np.ndarray) -> np.ndarray:
    """Z_C U = Pairs(A, B) Q_J Core^T Q_K^T U  (U: n_C x m)."""
    return pairs_apply(F["GXA"], F["GXB"], F["QJ"] @ (F["core"].T @ (F["QK"].T @ U)))


def first_moment_four(GXA) -> np.ndarray:
    """M1 = (1/n_X) sum_x G[x, A]^T (Eq. 1moment_graph)."""
    A = as_sparse(GXA)
    return np.asarray(A.sum(axis=0)).ravel() / A.shape[0]


def m2_apply_four(F: dict, S: np.ndarray, alpha0: float) -> np.ndarray:
    """O = M2 S for M2 of Eq. 2moment_graph, applied right to left without
    forming it: (alpha0+1)/n_X Z_C G[X, C]^T (G[X, B] (Z_B^T S)) - alpha0 M1 (M1^T S)."""
    GXB, GXC = as_sparse(F["GXB"]), as_sparse(F["GXC"])
    n_x = GXB.shape[0]
    u = zb_t(F, S)
    w = np.asarray(GXC.T @ (GXB @ u)) / n_x
    M1 = first_moment_four(F["GXA"])
    return (alpha0 + 1.0) * zc(F, w) - alpha0 * np.outer(M1, M1 @ S)


def power_sketch_four(F: dict, S: np.ndarray, alpha0: float, q: int):
    """The power-iterated sketch of the whitener (the reading of Section 4.2
    used for every sampled moment) with the four-partition M2."""
    return power_sketch_op(lambda V: m2_apply_four(F, V, alpha0), S, q)


def whiten_four(F: dict, W: np.ndarray):
    """The three whitened views (Section 4.1, Appendix A):
    y_A = W^T G[x, A]^T, y_B = (Z_B^T W)^T G[x, B]^T, y_C = (Z_C^T W)^T G[x, C]^T.
    Returns (Y_A, Y_B, Y_C, ybar (3 x k), W_B = Z_B^T W, W_C = Z_C^T W)."""
    WB = zb_t(F, W)
    WC = zc_t(F, W)
    YA, ya = whiten(F["GXA"], W, False)
    YB, yb = whiten(F["GXB"], WB, False)
    YC, yc = whiten(F["GXC"], WC, False)
    return YA, YB, YC, np.stack([ya, yb, yc]), WB, WC


def node_views(G_SA, W: np.ndarray) -> np.ndarray:
    """Whitened adjacency of nodes S into A, W^T G[A, s] per node s (the
    columns of W^T G[A, A^c] in Lemma postprocessing), for memberships of
    nodes outside X."""
    return np.asarray(as_sparse(G_SA) @ W)


def dense_csr(M: np.ndarray) -> sp.csr_matrix:
    """A dense block as a sparse matrix (exact-moment instances)."""
    return sp.csr_matrix(M)
