"""FP64 oracle of the validation layer (TEST INFRASTRUCTURE, like the rest
of this package): matching estimated communities to ground truth by p-value
testing (Section 5.1) and the evaluation metrics of Section 5.2.

Pi_hat (k_hat x n) holds an estimated membership row per community, Pi
(k x n) the true memberships of the same n nodes.

* rho(i, j): Pearson correlation of the rows Pi_hat_i and Pi_j.
* T_ij = rho sqrt(n - 2) / sqrt(1 - rho^2), Student t with n - 2 degrees of
  freedom under independence.
* READING: the right p-value is described as the probability of a value
  greater than T_ij, while its formula is printed as 1 - P(t > T); the
  description (and its footnote: anti-correlated communities are not paired)
  fixes p_ij = P(t_(n-2) > T_ij).
* READING: the p-values are "adjusted to ensure a small enough false
  discovery rate" with a citation of a local-fdr tool; the adjustment here is
  the Benjamini-Hochberg step-up over all k_hat * k tests,
  p_adj(r) = min(1, min_(s >= r) m p_(s) / s) for the r-th smallest p.
* G_Pval: the pairs (i, j) with p_adj <= 0.01 (the paper's threshold).
* Recovery ratio R = (1/k) #{true communities j with an edge}.
* Error E = (1/k) sum over the edges (i, j) of (1/n) sum_x |Pi_hat_i(x) - Pi_j(x)|.
* Bridgeness (Eq. bridgeness) of node x with membership vector m over
  k_hat communities: b_x = 1 - sqrt(k_hat/(k_hat - 1) sum_j (m_j - 1/k_hat)^2);
  degree-corrected (Eq. degreebridgeness): D_x b_x.
"""
from __future__ import annotations

import numpy as np
from scipy import stats

__all__ = ["correlation", "t_statistic", "right_pvalue", "pvalue_matrix", "bh_adjust", "pvalue_graph",
           "recovery_ratio", "l1_distances", "error", "bridgeness", "validate"]


def correlation(Pi_hat: np.ndarray, Pi: np.ndarray) -> np.ndarray:
    """rho (k_hat x k): Pearson correlation of every estimated row with every
    true row over the n nodes (a constant row has correlation 0)."""
    A = Pi_hat - Pi_hat.mean(axis=1, keepdims=True)
    B = Pi - Pi.mean(axis=1, keepdims=True)
    na = np.sqrt(np.sum(A * A, axis=1))
    nb = np.sqrt(np.sum(B * B, axis=1))
    cov = A @ B.T
    den = na[:, None] * nb[None, :]
    return np.where(den > 0, cov / np.where(den > 0, den, 1.0), 0.0)


def t_statistic(rho: np.ndarray, n: int) -> np.ndarray:
    """T = rho sqrt(n - 2) / sqrt(1 - rho^2) (Section 5.1); +-inf at |rho| = 1."""
    rho = np.asarray(rho, dtype=np.float64)
    # both branches are evaluated: |rho| >= 1 (rounding can give 1 + ulp)
    # divides by zero or takes the root of a negative there, and is discarded
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(np.abs(rho) >= 1.0, np.sign(rho) * np.inf, rho * np.sqrt(n - 2.0) / np.sqrt(1.0 - rho * rho))


def right_pvalue(T: np.ndarray, dof: float) -> np.ndarray:
    """P(t_dof > T), the Student t survival function (library routine)."""
    return stats.t.sf(T, dof)


def pvalue_matrix(Pi_hat: np.ndarray, Pi: np.ndarray) -> np.ndarray:
    """Pval(i, j) = P(t_(n-2) > T_ij) for estimated i, true j."""
    n = Pi.shape[1]
    return right_pvalue(t_statistic(correlation(Pi_hat, Pi), n), n - 2.0)


def bh_adjust(p: np.ndarray) -> np.ndarray:
    """Benjamini-Hochberg adjusted p-values over all entries of p (same shape):
    sort ascending (ties by position), q_r = m p_(r) / r, running minimum from
    the largest down, capped at 1."""
    flat = np.asarray(p, dtype=np.float64).ravel()
    m = flat.size
    order = np.argsort(flat, kind="stable")
    q = flat[order] * m / np.arange(1, m + 1)
    q = np.minimum.accumulate(q[::-1])[::-1]
    out = np.empty(m)
    out[order] = np.minimum(q, 1.0)
    return out.reshape(np.shape(p))


def pvalue_graph(p_adj: np.ndarray, threshold: float = 0.01) -> np.ndarray:
    """Edges of G_Pval: E[i, j] = p_adj(i, j) <= threshold (estimated i, true j)."""
    return p_adj <= threshold


def recovery_ratio(E: np.ndarray) -> float:
    """R = (1/k) sum_j 1{degree of true community j in G_Pval > 0}."""
    return float(np.mean(E.any(axis=0)))


def l1_distances(Pi_hat: np.ndarray, Pi: np.ndarray) -> np.ndarray:
    """D(i, j) = (1/n) sum_x |Pi_hat_i(x) - Pi_j(x)|."""
    return np.abs(Pi_hat[:, None, :] - Pi[None, :, :]).mean(axis=2)


def error(Pi_hat: np.ndarray, Pi: np.ndarray, E: np.ndarray) -> float:
    """E = (1/k) sum over the edges of D(i, j) (Section 5.2)."""
    k = Pi.shape[0]
    return float(np.sum(l1_distances(Pi_hat, Pi)[E]) / k)


def bridgeness(Pi_hat: np.ndarray, degree: np.ndarray | None = None):
    """b_x = 1 - sqrt(k_hat/(k_hat-1) sum_j (Pi_hat_j(x) - 1/k_hat)^2) per node
    (Eq. bridgeness); with degrees also D_x b_x (Eq. degreebridgeness)."""
    kh = Pi_hat.shape[0]
    b = 1.0 - np.sqrt(kh / (kh - 1.0) * np.sum((Pi_hat - 1.0 / kh) ** 2, axis=0))
    return b if degree is None else (b, degree * b)


def validate(Pi_hat: np.ndarray, Pi: np.ndarray, threshold: float = 0.01) -> dict:
    """The whole validation: p-values, adjusted p-values, edges, R and E."""
    p = pvalue_matrix(Pi_hat, Pi)
    p_adj = bh_adjust(p)
    E = pvalue_graph(p_adj, threshold)
    return {"p": p, "p_adj": p_adj, "edges": E, "recovery_ratio": recovery_ratio(E),
            "error": error(Pi_hat, Pi, E)}
