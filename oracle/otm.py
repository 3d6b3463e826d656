"""FP64 oracle of the hot path: moments, whitening, STGD, loss, post-processing.

TEST INFRASTRUCTURE (see the package docstring): only tests, the smoke check
and the benchmark's CPU-baseline leg may use it.

Section references are to Huang, Niranjan, Hakeem, Anandkumar, "Online Tensor
Methods for Learning Latent Variable Models".  Readings taken where the paper
is silent or inconsistent are marked READING where they are applied.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "NotPSDError", "as_sparse", "row_weights", "dirichlet_coefficients", "first_moment",
    "m2_apply", "power_sketch", "power_sketch_op", "whitener_rsvd", "canonical_signs", "whiten", "sgd_step", "sgd_direction",
    "sgd_run", "beta_schedule", "steps_per_pass", "whitened_tensor", "residual",
    "unwhiten_topics", "recover_pi", "eigen_from_factors", "restart_score", "best_restart", "sgd_batched",
]


class NotPSDError(ValueError):
    """The projected second moment has no k positive eigenvalues."""


# ----------------------------------------------------------------------------
# Data as sparse matrices
# ----------------------------------------------------------------------------
def as_sparse(C) -> sp.csr_matrix:
    """CSR (synth.CSR or scipy) -> scipy CSR in float64."""
    if sp.issparse(C):
        return sp.csr_matrix(C, dtype=np.float64)
    return C.to_scipy(np.float64)


def row_weights(C, normalize: bool):
    """Per-sample weights of the moments.

    READING (Section 2.1): for documents the moments are taken per document on
    the normalised counts, the first moment with weight 1/l_t and the pair
    term with weight 1/(l_t (l_t - 1)), where l_t is the document length; this
    is what makes the expectations of Lemma (topic) hold for documents of
    different lengths.  For graphs (Section 2.2) every sample has weight 1.
    Returns (w1, w2) of length n.
    """
    Cs = as_sparse(C)
    n = Cs.shape[0]
    if not normalize:
        return np.ones(n), np.ones(n)
    lengths = np.asarray(Cs.sum(axis=1)).ravel()
    if np.any(lengths < 2):
        raise ValueError("document with fewer than 2 tokens")
    return 1.0 / lengths, 1.0 / (lengths * (lengths - 1.0))


def dirichlet_coefficients(alpha0: float):
    """Coefficients of the Dirichlet-corrected tensor (Section 3.2, tensor T):
    a = (alpha0+1)(alpha0+2)/2, b = alpha0(alpha0+1)/2, c = alpha0^2."""
    a = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0
    b = alpha0 * (alpha0 + 1.0) / 2.0
    c = alpha0 * alpha0
    return a, b, c


# ----------------------------------------------------------------------------
# Moments (Section 2, Eqs. 1moment_topic / 2moment_topic and the graph forms)
# ----------------------------------------------------------------------------
def first_moment(C, normalize: bool) -> np.ndarray:
    """M1 = (1/n) sum_t w1_t c_t (Eq. 1moment_topic; Eq. 1moment_graph with w1 = 1)."""
    Cs = as_sparse(C)
    w1, _ = row_weights(Cs, normalize)
    return np.asarray(Cs.T @ w1).ravel() / Cs.shape[0]


def m2_apply(C, S: np.ndarray, alpha0: float, normalize: bool) -> np.ndarray:
    """O = M2 S without forming M2 (Section 4.2, randomized low-rank approximation).

    M2 = (alpha0+1)/n sum_t w2_t (c_t c_t^T - diag(c_t)) - alpha0 M1 M1^T
    (Eq. 2moment_topic; for a graph with a single leaf set, c_t is the row
    G[x, A] and w2 = 1).  Applied to S column by column:
      sum_t w2_t c_t c_t^T S  = C^T diag(w2) (C S)
      sum_t w2_t diag(c_t) S  = diag(C^T w2) S
    """
    Cs = as_sparse(C)
    n = Cs.shape[0]
    _, w2 = row_weights(Cs, normalize)
    M1 = first_moment(Cs, normalize)
    CS = Cs @ S
    pair = Cs.T @ (w2[:, None] * CS)
    diag = np.asarray(Cs.T @ w2).ravel()[:, None] * S
    return (alpha0 + 1.0) / n * (pair - diag) - alpha0 * np.outer(M1, M1 @ S)


def power_sketch(C, S: np.ndarray, alpha0: float, normalize: bool, q: int):
    """Sketch of M2 for the whitener with q power iterations.

    READING (Section 4.2 on sampled data): the Nystrom step needs
    S^T M2 S to be positive definite on its top k eigenpairs, which fails for
    sampled moments whose many small noise eigenvalues (of both signs) swamp a
    sketch of width 2k.  The sketch is therefore refined by
    Q_0 = S, Q_j = orth(M2 Q_{j-1}) (a basis of the span; QR here), the power
    method sketch of the Nystrom analysis the paper cites; q = 0 is the
    paper's algorithm.  Returns (Q_q, O = M2 Q_q) for whitener_rsvd(O, Q_q, k).
    """
    return power_sketch_op(lambda V: m2_apply(C, V, alpha0, normalize), S, q)


def power_sketch_op(apply_m2, S: np.ndarray, q: int):
    """The power iteration of power_sketch for any second-moment operator
    apply_m2(V) = M2 V: Q_0 = S, Q_j = orth(M2 Q_{j-1}); returns (Q_q, M2 Q_q)."""
    Q = S
    for _ in range(q):
        Q = np.linalg.qr(apply_m2(Q))[0]
    return Q, apply_m2(Q)


def canonical_signs(W: np.ndarray) -> np.ndarray:
    """Flip each column so that its entry of largest magnitude is positive
    (ties: the lowest row index).  Whitening matrices are defined up to such
    signs (Section 3.1), so both implementations fix them the same way."""
    W = W.copy()
    for j in range(W.shape[1]):
        r = int(np.argmax(np.abs(W[:, j])))      # argmax returns the first maximum
        if W[r, j] < 0:
            W[:, j] = -W[:, j]
    return W


def whitener_rsvd(O: np.ndarray, S: np.ndarray, k: int, rel_floor: float = 1e-12):
    """Whitening matrix from the random projection O = M2 S (Section 4.2,
    algorithm "Randomized Tall-thin SVD" and its tall-thin QR variant).

    Steps (READING: the projected matrix is truncated to its top k
    eigenpairs before the square root, so that W has k columns):
      Omega = sym(S^T O);  Omega = U diag(sigma) U^T, sigma descending;
      B = O U_k diag(sigma_k)^(-1/2), so that M2 ~ O Omega^+ O^T ~ B B^T;
      B = U_B diag(s_B) V_B^T (thin SVD);  W = U_B diag(s_B)^(-1)
    which gives W^T (B B^T) W = I (Section 3.1: W^T M2 W = I).
    Returns (W, eigenvalues s_B^2 of the low-rank M2, descending).
    """
    Omega = S.T @ O
    Omega = 0.5 * (Omega + Omega.T)
    sig, U = np.linalg.eigh(Omega)
    order = np.argsort(-sig, kind="stable")
    sig, U = sig[order], U[:, order]
    if not (sig[k - 1] > rel_floor * max(sig[0], 0.0)) or sig[k - 1] <= 0:
        raise NotPSDError(f"sigma_k = {sig[k - 1]:.3e} (sigma_1 = {sig[0]:.3e})")
    B = O @ (U[:, :k] / np.sqrt(sig[:k])[None, :])
    UB, sB, _ = np.linalg.svd(B, full_matrices=False)
    W = canonical_signs(UB / sB[None, :])
    return W, sB ** 2


def whiten(C, W: np.ndarray, normalize: bool):
    """Whitened samples Y = diag(r) C W and their mean (Section 3.1, whitened
    data y_t = <W, c_t>; Appendix A, y_A = <G[x, A]^T, W>).

    READING (Section 2.1): each document view is normalised by its own token
    count, r_t = 1/l_t, so that E[y | h] = W^T mu h; graphs use r = 1.
    Returns (Y (n x k), ybar (k,)) with ybar = mean over all n samples
    (Appendix A: ybar := E_t[y^t]).
    """
    Cs = as_sparse(C)
    if normalize:
        r = 1.0 / np.asarray(Cs.sum(axis=1)).ravel()
    else:
        r = np.ones(Cs.shape[0])
    Y = r[:, None] * np.asarray(Cs @ W)
    return Y, Y.mean(axis=0)


# ----------------------------------------------------------------------------
# Stochastic tensor gradient descent (Section 3.2, Lemma "update")
# ----------------------------------------------------------------------------
def sgd_direction(YA, YB, YC, ybar, Phi, alpha0: float, theta: float = 1.0):
    """Update direction Delta (k x k) of Lemma (update) averaged over a batch,
    so that Phi_new = Phi + beta * Delta.  Column i belongs to phi_i.

    For each sample t and component i (Lemma update, with kappa = (1+theta)/2):
      Delta_i = -kappa sum_j <phi_j, phi_i>^2 phi_j
                + a <phi_i, yA_t><phi_i, yB_t> yC_t + c <phi_i, ybarA><phi_i, ybarB> ybarC
                - b <phi_i, yA_t><phi_i, yB_t> ybarC
                - b <phi_i, yA_t><phi_i, ybarB> yC_t
                - b <phi_i, ybarA><phi_i, yB_t> yC_t
    READING: a mini-batch averages these per-sample directions; ybar are the
    global means (the superscript t on ybar_B in the Lemma is taken as a typo).
    Written in the stacked matrix form the paper uses for its BLAS-3 version:
      PA = YA Phi, PB = YB Phi, mA = Phi^T ybarA, mB = Phi^T ybarB
      Q  = a PA*PB - b PA diag(mB) - b diag(mA) PB          (elementwise *)
      D  = YC^T Q / B + ybarC (c mA*mB - b colsum(PA*PB) / B)^T
      G  = Phi^T Phi;  O = Phi (G*G)
      Delta = D - kappa O
    """
    a, b, c = dirichlet_coefficients(alpha0)
    kappa = 0.5 * (1.0 + theta)
    ybA, ybB, ybC = ybar[0], ybar[1], ybar[2]
    nb = YA.shape[0]
    PA = YA @ Phi
    PB = YB @ Phi
    mA = Phi.T @ ybA
    mB = Phi.T @ ybB
    H = PA * PB
    Q = a * H - b * PA * mB[None, :] - b * mA[None, :] * PB
    D = YC.T @ Q / nb + np.outer(ybC, c * mA * mB - b * H.sum(axis=0) / nb)
    G = Phi.T @ Phi
    O = Phi @ (G * G)
    return D - kappa * O


def sgd_step(YA, YB, YC, ybar, Phi, beta: float, alpha0: float, theta: float = 1.0):
    """One STGD step on a batch: phi_i <- phi_i - beta dL/dv_i (Lemma update)."""
    return Phi + beta * sgd_direction(YA, YB, YC, ybar, Phi, alpha0, theta)


def steps_per_pass(n: int, batch: int) -> int:
    return (n + batch - 1) // batch


def beta_schedule(t: int, beta0: float, tau: float) -> float:
    """READING: the paper names beta^t the learning rate without a schedule;
    here beta_t = beta0 / (1 + t / tau), t the global step index."""
    return beta0 / (1.0 + t / tau)


def sgd_run(YA, YB, YC, ybar, Phi0, perms, batch: int, beta0: float, tau: float,
            alpha0: float, theta: float = 1.0, start_step: int = 0, end_step: int | None = None,
            snapshot_every_pass: bool = False):
    """Online STGD over the data (Section 3.2 and Section 4.3).

    perms is (passes x n): pass p visits samples perms[p, 0], perms[p, 1], ...
    in batches of `batch`; the last batch of a pass may be shorter and is
    averaged over its true size.  Global step t runs pass t // S, batch t % S,
    with S = ceil(n / batch) steps per pass and rate beta_t.  Every step
    updates all k components from the previous Phi (stacked form).
    Steps [start_step, end_step) are run, which makes a run resumable.
    Returns Phi, or (Phi, snapshots at the end of every completed pass).
    """
    n = YA.shape[0]
    spp = steps_per_pass(n, batch)
    total = perms.shape[0] * spp
    end = total if end_step is None else min(end_step, total)
    Phi = np.array(Phi0, dtype=np.float64, copy=True)
    snaps = []
    for t in range(start_step, end):
        p, s = divmod(t, spp)
        idx = perms[p, s * batch: min((s + 1) * batch, n)]
        Phi = sgd_step(YA[idx], YB[idx], YC[idx], ybar, Phi,
                       beta_schedule(t, beta0, tau), alpha0, theta)
        if snapshot_every_pass and s == spp - 1:
            snaps.append(Phi.copy())
    return (Phi, snaps) if snapshot_every_pass else Phi


# ----------------------------------------------------------------------------
# Loss (for measurement only: the hot path never forms the tensor)
# ----------------------------------------------------------------------------
def whitened_tensor(YA, YB, YC, ybar, alpha0: float, chunk: int = 1024) -> np.ndarray:
    """The whitened tensor T (k x k x k) of Section 3.2, formed explicitly:
      T = a/n sum_t yA_t x yB_t x yC_t
          - b/n sum_t [yA_t x yB_t x ybarC + yA_t x ybarB x yC_t + ybarA x yB_t x yC_t]
          + c ybarA x ybarB x ybarC."""
    a, b, c = dirichlet_coefficients(alpha0)
    n, k = YA.shape
    ybA, ybB, ybC = ybar[0], ybar[1], ybar[2]
    T = np.zeros((k, k, k))
    for s in range(0, n, chunk):
        A, Bv, Cv = YA[s:s + chunk], YB[s:s + chunk], YC[s:s + chunk]
        # sum_t yA_t x yB_t x yC_t as (rows of yA kron yB)^T yC, one matmul
        kron = (A[:, :, None] * Bv[:, None, :]).reshape(A.shape[0], k * k)
        T += a / n * (kron.T @ Cv).reshape(k, k, k)
        T -= b / n * np.einsum("ij,l->ijl", A.T @ Bv, ybC)
        T -= b / n * np.einsum("il,j->ijl", A.T @ Cv, ybB)
        T -= b / n * np.einsum("jl,i->ijl", Bv.T @ Cv, ybA)
    T += c * np.einsum("i,j,l->ijl", ybA, ybB, ybC)
    return T


def residual(T: np.ndarray, Phi: np.ndarray) -> float:
    """Relative residual R = ||sum_i phi_i^(x3) - T||_F^2 / ||T||_F^2 (the
    objective of Section 3.2 at theta = 0), expanded as
      ||sum phi^3||^2 = sum_ij (phi_i^T phi_j)^3,
      <sum phi^3, T>  = sum_i T(phi_i, phi_i, phi_i)."""
    G = Phi.T @ Phi
    self_term = float(np.sum(G ** 3))
    cross = float(np.einsum("ijl,ia,ja,la->", T, Phi, Phi, Phi))
    tt = float(np.sum(T * T))
    return (self_term - 2.0 * cross + tt) / tt


def restart_score(T: np.ndarray, Phi: np.ndarray) -> float:
    """Score of a restart's final factors: ||sum_i phi_i^(x3) - T||_F^2 - ||T||_F^2
    = sum_ij (phi_i^T phi_j)^3 - 2 sum_i T(phi_i, phi_i, phi_i).  READING (the
    paper leaves the choice among restarts open): restarts are ranked by the
    residual of the objective of Section 3.2; ||T||^2 is the same for every
    restart of a problem, so it is left out."""
    G = Phi.T @ Phi
    return float(np.sum(G ** 3)) - 2.0 * float(np.einsum("ijl,ia,ja,la->", T, Phi, Phi, Phi))


def best_restart(scores) -> int:
    """Index of the lowest score; ties go to the lower index."""
    return int(np.argmin(np.asarray(scores)))


def sgd_batched(problems, batch: int, beta0: float, tau: float, theta: float = 1.0):
    """Independent decompositions, each with several restarts: every restart
    is an online run (sgd_run) of its problem, scored by restart_score; the
    best restart is the lowest score.  problems: dicts with YA, YB, YC, ybar
    (3 x k), alpha0, Phi0 (list of k x k, phi_i as columns) and perms (list of
    passes x n, one per restart).  Returns, per problem, (list of final Phi,
    list of scores, best index)."""
    out = []
    for P in problems:
        T = whitened_tensor(P["YA"], P["YB"], P["YC"], P["ybar"], P["alpha0"])
        phis, scores = [], []
        for Phi0, perms in zip(P["Phi0"], P["perms"]):
            Phi = sgd_run(P["YA"], P["YB"], P["YC"], P["ybar"], Phi0, perms, batch, beta0, tau, P["alpha0"], theta)
            phis.append(Phi)
            scores.append(restart_score(T, Phi))
        out.append((phis, scores, best_restart(scores)))
    return out


# ----------------------------------------------------------------------------
# Post-processing (Section 3.3, Lemma "postprocessing")
# ----------------------------------------------------------------------------
def eigen_from_factors(Phi: np.ndarray, theta: float = 1.0):
    """lambda_i = ||phi_i||^3 (Section 3.3) and unit u_i = phi_i / ||phi_i||.

    READING: the fixed point of the update has kappa ||phi||^3 = lambda with
    kappa = (1+theta)/2; at theta = 1 this is the paper's lambda = ||phi||^3.
    """
    norms = np.linalg.norm(Phi, axis=0)
    lam = 0.5 * (1.0 + theta) * norms ** 3
    return lam, Phi / norms[None, :]


def unwhiten_topics(W: np.ndarray, Phi: np.ndarray, theta: float = 1.0):
    """Topic-word matrix and Dirichlet weights (Lemma postprocessing).

    mu_hat = (W^T)^+ Phi up to a per-column scale.  READING: with the unit
    eigenvectors u_i the scale is lambda_i, mu_i = lambda_i (W^T)^+ u_i, where
    (W^T)^+ = W (W^T W)^(-1); then negative entries are clipped to 0 and each
    column is normalised to sum 1.  alpha_hat_i = lambda_i^(-2) / sum_j lambda_j^(-2).
    Returns (mu (d x k), alpha_hat (k,), lambda (k,)).
    """
    lam, U = eigen_from_factors(Phi, theta)
    WtW = W.T @ W
    pinvT = W @ np.linalg.inv(WtW)
    mu = pinvT @ (U * lam[None, :])
    mu = np.maximum(mu, 0.0)
    sums = mu.sum(axis=0)
    mu = np.where(sums[None, :] > 0, mu / np.where(sums > 0, sums, 1.0)[None, :], 0.0)
    inv2 = lam ** -2.0
    return mu, inv2 / inv2.sum(), lam


def recover_pi(Y: np.ndarray, Phi: np.ndarray, tau: float, theta: float = 1.0) -> np.ndarray:
    """Community memberships of the samples (Lemma postprocessing):
      Pi_hat = diag(lambda)^(-1) U^T W^T G[A, X] = diag(lambda)^(-1) U^T Y^T
    (k x n), READING: with unit eigenvectors U and gamma = 1.  Then the
    thresholding step: clip negatives to 0, normalise each column to sum 1,
    zero the entries below tau, normalise again (a column whose sum is 0 stays 0).
    """
    lam, U = eigen_from_factors(Phi, theta)
    Pi = (U.T @ Y.T) / lam[:, None]
    Pi = np.maximum(Pi, 0.0)

    def _norm(M):
        s = M.sum(axis=0)
        return np.where(s[None, :] > 0, M / np.where(s > 0, s, 1.0)[None, :], 0.0)

    Pi = _norm(Pi)
    Pi = np.where(Pi < tau, 0.0, Pi)
    return _norm(Pi)
