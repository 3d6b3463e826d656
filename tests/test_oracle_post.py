"""Pins of the oracle's post-processing (Section 3.3, Lemma postprocessing).

* exact recovery: from the planted fixed point on an exact M2, the topic-word
  matrix mu, the Dirichlet weights ahat and the memberships pi come back
  exactly (up to the permutation of the factors);
* thresholding on a worked example computed by hand.
"""
import numpy as np

import oracle
import synth
from planted import exact_m2, planted_topics, planted_whitened_factors


def test_exact_topic_recovery():
    d, k = 40, 5
    mu, ahat = planted_topics(d, k, seed=71)
    S = synth.projection(d, 2 * k, seed=2)
    W, _ = oracle.whitener_rsvd(exact_m2(mu, ahat) @ S, S, k)
    _, lam, Phi = planted_whitened_factors(W, mu, ahat)
    perm = np.array([3, 0, 4, 1, 2])
    mu_hat, ahat_hat, lam_hat = oracle.unwhiten_topics(W, Phi[:, perm])
    np.testing.assert_allclose(mu_hat, mu[:, perm], atol=1e-10)
    np.testing.assert_allclose(ahat_hat, ahat[perm], atol=1e-12)
    np.testing.assert_allclose(lam_hat, lam[perm], rtol=1e-12)


def test_exact_membership_recovery():
    """E[G[x, A]] = F_A pi_x with F_A = Pi_A^T P^T (exact-moment lemma of
    Section 2.2); whitening the exact rows and post-processing returns pi_x."""
    g = synth.mmsb(n=300, k=4, alpha0=0.4, p=0.7, q=0.1, n_x=150, seed=8)
    PiA = g.pi[g.A]
    PiX = g.pi[g.X]
    F = PiA @ g.P.T
    ahat = g.alpha / g.alpha.sum()
    S = synth.projection(len(g.A), 8, seed=5)
    W, _ = oracle.whitener_rsvd(exact_m2(F, ahat) @ S, S, 4)
    _, _, Phi = planted_whitened_factors(W, F, ahat)
    Y = (F @ PiX.T).T @ W                     # rows y_x = W^T F pi_x
    Pi_hat = oracle.recover_pi(Y, Phi, tau=0.0)
    np.testing.assert_allclose(Pi_hat, PiX.T, atol=1e-10)


def test_threshold_worked_example():
    """One sample, two unit factors with lambda = (1, 2); raw memberships
    Lambda^-1 U^T y = (0.9, 0.1) -> normalised (0.9, 0.1); tau = 0.2 zeroes
    the second -> (1, 0).  A negative raw entry is clipped first."""
    Phi = np.array([[1.0, 0.0], [0.0, 2.0 ** (1 / 3)]])
    y = np.array([[0.9, 0.2]])
    np.testing.assert_allclose(oracle.recover_pi(y, Phi, 0.0)[:, 0], [0.9, 0.1], atol=1e-15)
    np.testing.assert_allclose(oracle.recover_pi(y, Phi, 0.2)[:, 0], [1.0, 0.0], atol=1e-15)
    y2 = np.array([[0.9, -0.2]])
    np.testing.assert_allclose(oracle.recover_pi(y2, Phi, 0.0)[:, 0], [1.0, 0.0], atol=1e-15)
    y3 = np.array([[-0.9, -0.2]])
    np.testing.assert_array_equal(oracle.recover_pi(y3, Phi, 0.0)[:, 0], [0.0, 0.0])


def test_eigenvalues_theta():
    Phi = np.diag([1.0, 2.0])
    lam, U = oracle.eigen_from_factors(Phi, theta=1.0)
    np.testing.assert_allclose(lam, [1.0, 8.0])
    lam3, _ = oracle.eigen_from_factors(Phi, theta=3.0)
    np.testing.assert_allclose(lam3, [2.0, 16.0])
    np.testing.assert_allclose(U, np.eye(2))
