"""CPU pins of the warm-start oracle: the sketch against the explicitly formed
tensor, the canonical frame and the target on exact moments (closed form:
the planted factors), the perceptron's gradients by finite differences, the
Adam step against its closed form at t = 1, the greedy matching."""
import numpy as np
import pytest

import oracle
from oracle import warmstart as ws
import synth


def _views(n, k, seed, three=True):
    g = np.random.default_rng(seed)
    YA = g.standard_normal((n, k)) * 0.4 + 0.1
    YB = g.standard_normal((n, k)) * 0.4 - 0.05 if three else YA
    YC = g.standard_normal((n, k)) * 0.4 + 0.02 if three else YA
    ybar = np.stack([YA.mean(0), YB.mean(0), YC.mean(0)])
    return YA, YB, YC, ybar


@pytest.mark.parametrize("alpha0,three", [(0.0, True), (0.7, True), (0.3, False)])
def test_sketch_is_the_contracted_tensor(alpha0, three):
    k = 6
    YA, YB, YC, ybar = _views(57, k, seed=3, three=three)
    Theta = np.random.default_rng(4).standard_normal((k, 4))
    T = oracle.whitened_tensor(YA, YB, YC, ybar, alpha0)          # T[i, j, l]: views A, B, C
    S = ws.sketch(YA, YB, YC, ybar, alpha0, Theta)
    for r in range(4):
        ref = np.einsum("ijl,l->ij", T, Theta[:, r])
        np.testing.assert_allclose(S[r], ref, atol=1e-12 * np.abs(ref).max())


def _exact(k, seed):
    """T = sum_l lambda_l u_l^(x3) from k exact samples y_l = (k lambda_l)^(1/3) u_l (alpha0 = 0)."""
    g = np.random.default_rng(seed)
    ahat = g.dirichlet(np.full(k, 2.0))
    lam = ahat ** -0.5
    U = synth.initial_factors(k, seed=seed)
    Y = (U * np.cbrt(k * lam)[None, :]).T.copy()
    ybar = np.stack([Y.mean(0)] * 3)
    return Y, ybar, U, lam


@pytest.mark.parametrize("k", [3, 8, 20])
def test_frame_recovers_planted_directions_on_exact_moments(k):
    Y, ybar, U, lam = _exact(k, seed=k)
    Theta = np.random.default_rng(k + 1).standard_normal((k, 4))
    S = ws.sketch(Y, Y, Y, ybar, 0.0, Theta)
    Q = ws.canonical_frame(S, Theta)
    C = Q.T @ U
    perm = ws.greedy_match(C)
    # every frame vector is +u of one planted component (orientation included)
    np.testing.assert_allclose(C[np.arange(k), perm], 1.0, atol=1e-9)
    # ordered by decreasing |eigenvalue| of S_1 = sum lambda_l (u_l . theta_1) u_l u_l^T
    mu = np.abs(lam[perm] * (U[:, perm].T @ Theta[:, 0]))
    assert np.all(np.diff(mu) <= 1e-9 * mu.max())


def test_target_maps_back_to_the_planted_factors():
    k, P = 7, 12
    Y, ybar, U, lam = _exact(k, seed=11)
    Theta = np.random.default_rng(2).standard_normal((k, 4))
    S = ws.sketch(Y, Y, Y, ybar, 0.0, Theta)
    Q = ws.canonical_frame(S, Theta)
    sigma = ws.sketch_scale(S)
    # E_theta ||T(I, I, theta)||_F^2 = ||T||_F^2: sigma estimates ||T||_F
    tnorm = np.sqrt(np.sum(lam ** 2))
    assert 0.2 < sigma / tnorm < 5.0
    Tg = ws.frame_target(Q, U, lam, sigma, P)
    V0 = ws.warm_factors(Tg.ravel(), Q, sigma, P)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, 0.0)
    assert oracle.residual(T, V0) < 1e-20
    x = ws.features(S, Theta, Q, P)
    assert x.shape == (4 * P * P + 4 * P,)
    F1 = x[:P * P].reshape(P, P)
    np.testing.assert_allclose(F1[:k, :k], Q.T @ S[0] @ Q / sigma, atol=1e-14)
    assert np.all(F1[k:, :] == 0) and np.all(F1[:, k:] == 0)


def test_mlp_gradients_match_finite_differences():
    g = np.random.default_rng(5)
    p = ws.init_params(7, 5, 4, g)
    X = g.standard_normal((3, 7))
    tgt = g.standard_normal((3, 4))

    def loss(pp):
        out, _ = ws.mlp_forward(pp, X)
        return 0.5 * float(np.sum((out - tgt) ** 2))

    out, cache = ws.mlp_forward(p, X)
    grads = ws.mlp_backward(p, cache, out - tgt)
    h = 1e-6
    for name in p:
        num = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[name][idx] += h
            lp = loss(pp)
            pp[name][idx] -= 2 * h
            num[idx] = (lp - loss(pp)) / (2 * h)
        np.testing.assert_allclose(grads[name], num, rtol=1e-6, atol=1e-8)


def test_mse_gradient_and_mask():
    g = np.random.default_rng(6)
    P, ks = 3, [2, 3]
    out = g.standard_normal((2, P * P))
    tgt = g.standard_normal((2, P * P))
    L, d = ws.mse(out, tgt, ks)
    mask = np.zeros((2, P, P))
    mask[0, :2, :2] = 1
    mask[1] = 1
    mask = mask.reshape(2, -1)
    assert abs(L - np.sum(((out - tgt) * mask) ** 2) / 13) < 1e-14
    h = 1e-6
    for idx in [(0, 0), (0, 2), (1, 8)]:
        o2 = out.copy()
        o2[idx] += h
        Lp, _ = ws.mse(o2, tgt, ks)
        o2[idx] -= 2 * h
        Lm, _ = ws.mse(o2, tgt, ks)
        assert abs((Lp - Lm) / (2 * h) - d[idx]) < 1e-7


def test_adam_first_step_closed_form():
    """At t = 1 the bias corrections cancel: delta = -lr g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-9])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    ws.adam_step(p, g, m, v, 1, lr=0.01)
    np.testing.assert_allclose(p["w"], [1.0, -2.0, 0.5] - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12)
    # second step with the same gradient: m = 0.19 g, v = 0.001999 g^2 (bias-corrected: g, g^2)
    ws.adam_step(p, g, m, v, 2, lr=0.01)
    np.testing.assert_allclose(m["w"], 0.19 * g["w"], rtol=1e-12)
    np.testing.assert_allclose(v["w"], (0.001 * 0.999 + 0.001) * g["w"] ** 2, rtol=1e-12)


def test_greedy_match():
    perm = np.array([2, 0, 3, 1])
    C = np.zeros((4, 4))
    C[np.arange(4), perm] = [0.9, -0.8, 0.7, -0.95]
    np.testing.assert_array_equal(ws.greedy_match(C), perm)
    # greedy, not optimal: the largest entry is taken first
    C = np.array([[0.9, 0.8], [0.85, 0.1]])
    np.testing.assert_array_equal(ws.greedy_match(C), [0, 1])


def test_sketch_scale_exact_values():
    """sigma = sqrt(mean_r ||S_r||_F^2) on hand-built sketches: squared norms
    2, 8, 0 and 25 give sqrt(35 / 4) (a sum in place of the mean, or a norm
    in place of its square, gives another number)."""
    S = np.zeros((4, 2, 2))
    S[0] = np.eye(2)
    S[1] = 2.0 * np.eye(2)
    S[3] = [[3.0, 0.0], [4.0, 0.0]]
    assert ws.sketch_scale(S) == pytest.approx(np.sqrt(35.0 / 4.0), rel=1e-15)
    assert ws.sketch_scale(np.zeros((4, 3, 3))) == 0.0


def test_sketch_scale_is_the_tensor_norm_for_an_orthonormal_design():
    """For T = sum_l lambda_l u_l^(x3) (k = 4) and theta_r = 2 u_r,
    ||T(I, I, theta_r)||_F^2 = 4 lambda_r^2, so the mean over the four
    sketches is sum_l lambda_l^2 = ||T||_F^2 exactly: sigma = ||T||_F."""
    k = 4
    lam = np.array([1.0, 2.0, 3.0, 4.0])
    U = synth.initial_factors(k, seed=21)
    Y = (U * np.cbrt(k * lam)[None, :]).T.copy()          # exact samples, alpha0 = 0
    ybar = np.stack([Y.mean(0)] * 3)
    Theta = 2.0 * U
    S = ws.sketch(Y, Y, Y, ybar, 0.0, Theta)
    assert ws.sketch_scale(S) == pytest.approx(np.sqrt(30.0), rel=1e-13)
    T = oracle.whitened_tensor(Y, Y, Y, ybar, 0.0)
    assert ws.sketch_scale(S) == pytest.approx(np.sqrt(np.sum(T * T)), rel=1e-13)
