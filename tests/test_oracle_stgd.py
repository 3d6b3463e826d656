"""Pins of the oracle's stochastic tensor gradient descent (Section 3.2).

* closed form: exact-moment samples give T = sum_i lambda_i u_i^(x3) with
  orthonormal u_i and lambda_i = ahat_i^(-1/2) (Lemma topic + W^T M2 W = I);
* Monte Carlo: sampled LDA views with alpha0 > 0 give E[T] = the same
  orthogonal tensor, which fails if a Dirichlet correction term or sign is off;
* finite differences: in the symmetric case the update direction is minus the
  gradient of f = (kappa/6) ||sum phi^3||^2 - (1/3) <sum phi^3, T_batch>, with
  both tensors formed explicitly;
* explicit contraction: with three different views the data part is
  T_batch(phi_i, phi_i, .) and the orthogonality part sum_j <phi_j,phi_i>^2 phi_j;
* fixed point: exact-moment runs converge to phi_i = lambda_i^(1/3) u_i,
  i.e. ||phi_i||^3 = lambda_i (Section 3.3);
* resume: a run split at any step equals the uninterrupted run bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from planted import exact_m2, exact_samples, planted_topics, planted_whitened_factors


def _exact_instance(d, k, seed):
    mu, ahat = planted_topics(d, k, seed=seed)
    M2 = exact_m2(mu, ahat)
    S = synth.projection(d, 2 * k, seed=seed + 1)
    W, _ = oracle.whitener_rsvd(M2 @ S, S, k)
    return mu, ahat, W


@pytest.mark.parametrize("d,k", [(10, 3), (50, 8)])
def test_exact_samples_give_orthogonal_tensor(d, k):
    mu, ahat, W = _exact_instance(d, k, seed=31)
    Y = exact_samples(W, mu, ahat)
    ybar = np.stack([Y.mean(0)] * 3)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, alpha0=0.0)
    U, lam, _ = planted_whitened_factors(W, mu, ahat)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    T_ref = np.einsum("i,ai,bi,ci->abc", lam, U, U, U)
    np.testing.assert_allclose(T, T_ref, atol=1e-12 * np.abs(T_ref).max())


@pytest.mark.slow
def test_dirichlet_corrected_tensor_expectation():
    """E[T] from three independent token views of sampled documents at alpha0=1
    equals sum_i lambda_i u_i^(x3) (the three correction terms cancel the
    Dirichlet cross moments)."""
    d, k, alpha0 = 6, 3, 1.0
    mu, _ = planted_topics(d, k, seed=41, beta=0.8)
    ahat = np.full(k, 1.0 / k)
    S = synth.projection(d, 2 * k, seed=2)
    W, _ = oracle.whitener_rsvd(exact_m2(mu, ahat) @ S, S, k)
    inst = synth.lda(d=d, k=k, alpha0=alpha0, beta=1.0, n_docs=300000, mean_len=12.0, seed=43, mu=mu)
    Ys = [oracle.whiten(v, W, normalize=True) for v in inst.views]
    ybar = np.stack([y[1] for y in Ys])
    T = oracle.whitened_tensor(Ys[0][0], Ys[1][0], Ys[2][0], ybar, alpha0)
    U, lam, _ = planted_whitened_factors(W, mu, ahat)
    T_ref = np.einsum("i,ai,bi,ci->abc", lam, U, U, U)
    err = np.abs(T - T_ref).max() / np.abs(T_ref).max()
    assert err < 0.03, err
    # flipping the sign of the middle (b) terms breaks it
    a, b, c = oracle.dirichlet_coefficients(alpha0)
    T_plain = oracle.whitened_tensor(Ys[0][0], Ys[1][0], Ys[2][0], ybar, 0.0)   # = mean yA x yB x yC
    T_flip = T + 2 * (T - a * T_plain - c * np.einsum("i,j,l->ijl", *ybar))
    assert np.abs(T_flip - T_ref).max() / np.abs(T_ref).max() > 10 * err


def _f_symmetric(Phi, Y, ybar, alpha0, kappa):
    T = oracle.whitened_tensor(Y, Y, Y, ybar, alpha0)
    k = Phi.shape[1]
    Sphi = np.zeros_like(T)
    for i in range(k):
        Sphi += np.einsum("a,b,c->abc", Phi[:, i], Phi[:, i], Phi[:, i])
    return kappa / 6.0 * np.sum(Sphi * Sphi) - np.sum(Sphi * T) / 3.0


@pytest.mark.parametrize("alpha0,theta,nb", [(0.0, 1.0, 1), (0.5, 1.0, 7), (1.0, 3.0, 20), (0.1, 0.2, 5)])
def test_direction_is_minus_gradient_symmetric(alpha0, theta, nb):
    k = 5
    g = np.random.default_rng(7)
    Y = g.standard_normal((nb, k))
    yb = g.standard_normal(k) * 0.3
    ybar = np.stack([yb, yb, yb])
    Phi = g.standard_normal((k, k)) * 0.7
    kappa = 0.5 * (1 + theta)
    Dlt = oracle.sgd_direction(Y, Y, Y, ybar, Phi, alpha0, theta)
    h = 1e-5
    grad = np.zeros_like(Phi)
    for a_ in range(k):
        for i in range(k):
            E = np.zeros_like(Phi)
            E[a_, i] = h
            grad[a_, i] = (_f_symmetric(Phi + E, Y, ybar, alpha0, kappa)
                           - _f_symmetric(Phi - E, Y, ybar, alpha0, kappa)) / (2 * h)
    np.testing.assert_allclose(Dlt, -grad, rtol=0, atol=2e-8 * np.abs(grad).max())


@pytest.mark.parametrize("alpha0,nb", [(0.0, 1), (0.7, 9), (2.0, 4)])
def test_direction_explicit_contraction_three_views(alpha0, nb):
    k = 4
    g = np.random.default_rng(3)
    YA, YB, YC = (g.standard_normal((nb, k)) for _ in range(3))
    ybar = g.standard_normal((3, k)) * 0.4
    Phi = g.standard_normal((k, k))
    T = oracle.whitened_tensor(YA, YB, YC, ybar, alpha0)
    expect = np.zeros((k, k))
    for i in range(k):
        data = np.einsum("abc,a,b->c", T, Phi[:, i], Phi[:, i])
        orth = sum(float(Phi[:, j] @ Phi[:, i]) ** 2 * Phi[:, j] for j in range(k))
        expect[:, i] = data - orth
    np.testing.assert_allclose(oracle.sgd_direction(YA, YB, YC, ybar, Phi, alpha0, 1.0), expect,
                               atol=1e-12 * np.abs(expect).max())


def test_residual_matches_explicit_frobenius():
    k = 4
    g = np.random.default_rng(5)
    T = g.standard_normal((k, k, k))
    Phi = g.standard_normal((k, k))
    Sphi = np.einsum("ai,bi,ci->abc", Phi, Phi, Phi)
    ref = np.sum((Sphi - T) ** 2) / np.sum(T * T)
    assert abs(oracle.residual(T, Phi) - ref) < 1e-12 * ref


def test_exact_moment_fixed_point_and_convergence():
    d, k = 20, 4
    mu, ahat, W = _exact_instance(d, k, seed=51)
    Y = exact_samples(W, mu, ahat)
    ybar = np.stack([Y.mean(0)] * 3)
    U, lam, Phi_star = planted_whitened_factors(W, mu, ahat)
    # the planted factors are a fixed point of the full-batch update
    D = oracle.sgd_direction(Y, Y, Y, ybar, Phi_star, alpha0=0.0)
    assert np.abs(D).max() < 1e-12
    # start near the truth and run full-batch steps: converge to it
    g = np.random.default_rng(1)
    Phi0 = Phi_star + 0.05 * g.standard_normal((k, k))
    perms = np.tile(np.arange(k, dtype=np.int32), (400, 1))
    Phi = oracle.sgd_run(Y, Y, Y, ybar, Phi0, perms, batch=k, beta0=0.05, tau=1e9, alpha0=0.0)
    np.testing.assert_allclose(np.linalg.norm(Phi, axis=0) ** 3, lam, rtol=1e-10)
    np.testing.assert_allclose(Phi, Phi_star, atol=1e-10)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, 0.0)
    assert oracle.residual(T, Phi) < 1e-18


def test_random_restarts_find_planted_factors():
    d, k = 16, 4
    mu, ahat, W = _exact_instance(d, k, seed=61)
    Y = exact_samples(W, mu, ahat)
    ybar = np.stack([Y.mean(0)] * 3)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, 0.0)
    U, lam, _ = planted_whitened_factors(W, mu, ahat)
    perms = np.tile(np.arange(k, dtype=np.int32), (3000, 1))
    best = min(oracle.residual(T, oracle.sgd_run(Y, Y, Y, ybar, synth.initial_factors(k, 5, r), perms,
                                                 batch=k, beta0=0.05, tau=1e9, alpha0=0.0))
               for r in range(8))
    assert best < 1e-12


def test_run_resume_is_bit_identical():
    g = np.random.default_rng(2)
    n, k = 53, 5
    YA, YB, YC = (g.standard_normal((n, k)) for _ in range(3))
    ybar = np.stack([YA.mean(0), YB.mean(0), YC.mean(0)])
    perms = synth.permutations(n, 3, seed=4)
    Phi0 = synth.initial_factors(k, seed=3)
    full = oracle.sgd_run(YA, YB, YC, ybar, Phi0, perms, 10, 0.01, 50.0, 0.3)
    half = oracle.sgd_run(YA, YB, YC, ybar, Phi0, perms, 10, 0.01, 50.0, 0.3, end_step=7)
    rest = oracle.sgd_run(YA, YB, YC, ybar, half, perms, 10, 0.01, 50.0, 0.3, start_step=7)
    np.testing.assert_array_equal(full, rest)
    # the last batch of a pass is the ragged remainder (53 = 5*10 + 3)
    assert oracle.steps_per_pass(n, 10) == 6


def test_batch_of_one_is_the_lemma():
    """B = 1: the update of every phi_i is the Lemma's six-term expression."""
    k, alpha0, beta = 3, 0.4, 0.02
    g = np.random.default_rng(9)
    yA, yB, yC = (g.standard_normal(k) for _ in range(3))
    ybar = g.standard_normal((3, k))
    Phi = g.standard_normal((k, k))
    a, b, c = oracle.dirichlet_coefficients(alpha0)
    new = oracle.sgd_step(yA[None], yB[None], yC[None], ybar, Phi, beta, alpha0)
    for i in range(k):
        p = Phi[:, i]
        upd = p - beta * sum((Phi[:, j] @ p) ** 2 * Phi[:, j] for j in range(k))
        upd = upd + beta * a * (p @ yA) * (p @ yB) * yC + beta * c * (p @ ybar[0]) * (p @ ybar[1]) * ybar[2]
        upd = upd - beta * b * ((p @ yA) * (p @ yB) * ybar[2] + (p @ yA) * (p @ ybar[1]) * yC
                                + (p @ ybar[0]) * (p @ yB) * yC)
        np.testing.assert_allclose(new[:, i], upd, atol=1e-14)


def test_restart_score_is_residual_minus_constant():
    """score = (R - 1) ||T||^2 with R from the explicitly formed difference tensor."""
    k = 5
    g = np.random.default_rng(9)
    T = g.standard_normal((k, k, k))
    tt = float(np.sum(T * T))
    for _ in range(3):
        Phi = g.standard_normal((k, k))
        Sphi = np.einsum("ai,bi,ci->abc", Phi, Phi, Phi)
        ref = float(np.sum((Sphi - T) ** 2)) - tt
        assert abs(oracle.restart_score(T, Phi) - ref) < 1e-12 * (abs(ref) + tt)


def test_best_restart_ties_and_order():
    assert oracle.best_restart([3.0, 1.0, 1.0, 2.0]) == 1
    assert oracle.best_restart([0.5]) == 0


def test_batched_picks_a_restart_that_recovers_the_planted_factors():
    """Exact moments: the restart with the lowest score reaches R = 0, i.e. the
    planted factors (closed form of the fixed point); several restarts stall."""
    d, k = 16, 4
    mu, ahat, W = _exact_instance(d, k, seed=61)
    Y = exact_samples(W, mu, ahat)
    ybar = np.stack([Y.mean(0)] * 3)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, 0.0)
    perms = np.tile(np.arange(k, dtype=np.int32), (3000, 1))
    P = dict(YA=Y, YB=Y, YC=Y, ybar=ybar, alpha0=0.0,
             Phi0=[synth.initial_factors(k, 5, r) for r in range(8)], perms=[perms] * 8)
    (phis, scores, best), = oracle.sgd_batched([P], batch=k, beta0=0.05, tau=1e9)
    tt = float(np.sum(T * T))
    assert scores[best] == min(scores)
    assert max(oracle.residual(T, P_) for P_ in phis) > 0.1      # some restarts stall
    assert oracle.residual(T, phis[best]) < 1e-12
    assert abs(scores[best] + tt) < 1e-10 * tt          # R = 0  <=>  score = -||T||^2
    U, lam, Phi_star = planted_whitened_factors(W, mu, ahat)
    # every planted factor is matched by one recovered column (up to order)
    cos = np.abs((phis[best] / np.linalg.norm(phis[best], axis=0)).T @ U)
    assert np.all(np.abs(np.sort(cos.max(axis=0)) - 1.0) < 1e-9)
