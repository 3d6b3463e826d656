"""Planted (exact-moment) instances used by the CPU pins and GPU parity tests.

These build the exact population quantities of the exact-moment lemmas from
the planted parameters, independently of the oracle's estimators:
  LDA  (Lemma topic):  M2 = sum_i ahat_i mu_i mu_i^T
  MMSB (Lemma exact moments): M2 = sum_i ahat_i F_i F_i^T with F = Pi_A^T P^T
and exact "samples" whose implicit tensor equals the exact whitened tensor.
"""
from __future__ import annotations

import numpy as np

import synth


def planted_topics(d: int, k: int, seed: int, beta: float = 0.3, alpha: np.ndarray | None = None):
    g = synth.rng(seed, synth.S_MISC, 1)
    mu = g.dirichlet(np.full(d, beta), size=k).T.copy()      # (d, k)
    if alpha is None:
        alpha = g.dirichlet(np.full(k, 5.0)) * 1.0
    ahat = alpha / alpha.sum()
    return mu, ahat


def exact_m2(F: np.ndarray, ahat: np.ndarray) -> np.ndarray:
    return (F * ahat[None, :]) @ F.T


def exact_samples(W: np.ndarray, F: np.ndarray, ahat: np.ndarray) -> np.ndarray:
    """k samples y_j = (k ahat_j)^(1/3) W^T F_j; with alpha0 = 0 (a=1, b=c=0)
    their implicit tensor (1/k) sum_j y_j^(x3) equals sum_j ahat_j (W^T F_j)^(x3),
    the whitened exact third moment."""
    k = F.shape[1]
    return ((W.T @ F) * np.cbrt(k * ahat)[None, :]).T.copy()


def planted_whitened_factors(W: np.ndarray, F: np.ndarray, ahat: np.ndarray):
    """u_i = sqrt(ahat_i) W^T F_i (orthonormal when W whitens the exact M2),
    lambda_i = ahat_i^(-1/2), planted STGD fixed point phi_i = lambda_i^(1/3) u_i."""
    U = (W.T @ F) * np.sqrt(ahat)[None, :]
    lam = ahat ** -0.5
    return U, lam, U * np.cbrt(lam)[None, :]


def planted_four(sizes: dict, k: int, p: float, q: float, seed: int, alpha0: float = 0.0):
    """Exact-moment four-partition graph (Section 2.2): node memberships pi
    (pure, every community present in every set, when alpha0 = 0; else
    Dir(alpha0/k)), P = q 1 1^T + (p - q) I, and the expected adjacency blocks
    E[G[R, S]] = Pi_R^T P Pi_S as dense matrices (sparse containers).
    Returns (pi per set (k x n_set), P, blocks)."""
    import scipy.sparse as sp
    g = synth.rng(seed, synth.S_MISC, 7)
    P = np.full((k, k), q) + (p - q) * np.eye(k)
    pis = {}
    for name, n in sizes.items():
        if alpha0 == 0.0:
            lab = g.permutation(np.arange(n) % k)
            pis[name] = np.eye(k)[:, lab]
        else:
            pis[name] = g.dirichlet(np.full(k, alpha0 / k), size=n).T
    blocks = {}
    for r, c in synth.FOUR_BLOCKS:
        blocks[(r, c)] = sp.csr_matrix(pis[r].T @ P @ pis[c])
    return pis, P, blocks
