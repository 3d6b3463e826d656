"""FP64 oracle of the learned warm start (TEST INFRASTRUCTURE, like the rest
of this package): a sketch of the whitened third moment, its canonical frame,
the network's features, a two-layer perceptron (forward, backward, Adam) and
the map from the network's output to initial factors.

The paper initialises the stochastic updates randomly (Section 3.2); the warm
start is an addition.  Its pieces:

* sketch: S_r = T(I, I, theta_r), r = 1..4, the tensor T of Section 3.2
  contracted along its third mode with Gaussian vectors theta_r, computed from
  the whitened rows without forming T;
* canonical frame (READING, an addition): the whitened basis is arbitrary
  (W is unique only up to rotation, Section 3.1), and a perceptron cannot
  learn to undo a random rotation, so the sketches are presented in the
  eigenbasis Q of S_1 (eigenvalues by decreasing magnitude), each eigenvector
  oriented so that its contraction with the theta_r of largest |q^T theta_r|
  has the sign of q^T S_r q (for T = sum_l lambda_l u_l^(x3), lambda_l > 0,
  this makes q = +u_l);
* network: x = [Q^T S_r Q / sigma (r = 1..4, zero-padded to P x P),
  Q^T theta_r (padded to P)], sigma = sqrt(mean_r ||S_r||_F^2);
  h = relu(W1 x + b1), out = W2 h + b2 (P x P, row-major);
* initial factors: V0 = Q out[:k, :k] sigma^(1/3), column i = phi_i;
* training target: the planted factors lambda_l^(1/3) u_l written in the frame
  and divided by sigma^(1/3), each assigned to the frame vector it is most
  aligned with (greedy matching by decreasing |cos|); loss = mean squared
  error over the live k x k block.
"""
from __future__ import annotations

import numpy as np

from .otm import dirichlet_coefficients

N_SKETCH = 4


def sketch(YA, YB, YC, ybar, alpha0: float, Theta) -> np.ndarray:
    """S_r = T(I, I, theta_r) for the columns theta_r of Theta (k x 4):
      S_r = (1/n) YA^T diag(a z_r - b (ybarC . theta_r)) YB
            - b ybarA ((1/n) YB^T z_r)^T - b ((1/n) YA^T z_r) ybarB^T
            + c (ybarC . theta_r) ybarA ybarB^T,       z_r = YC theta_r.
    Returns (4, k, k)."""
    a, b, c = dirichlet_coefficients(alpha0)
    n = YA.shape[0]
    ybA, ybB, ybC = ybar[0], ybar[1], ybar[2]
    out = []
    for r in range(Theta.shape[1]):
        th = Theta[:, r]
        z = YC @ th
        gc = float(ybC @ th)
        w = a * z - b * gc
        S = (YA * w[:, None]).T @ YB / n
        S -= b * np.outer(ybA, YB.T @ z / n)
        S -= b * np.outer(YA.T @ z / n, ybB)
        S += c * gc * np.outer(ybA, ybB)
        out.append(S)
    return np.stack(out)


def canonical_frame(S: np.ndarray, Theta: np.ndarray) -> np.ndarray:
    """Eigenvectors of sym(S_1), by decreasing |eigenvalue| (ties: lower
    index), each oriented as in the module docstring.  Returns Q (k x k)."""
    S1 = 0.5 * (S[0] + S[0].T)
    ev, Q = np.linalg.eigh(S1)
    order = sorted(range(len(ev)), key=lambda i: (-abs(ev[i]), i))
    Q = Q[:, order]
    qt = Q.T @ Theta                                   # k x 4
    for l in range(Q.shape[1]):
        r = int(np.argmax(np.abs(qt[l])))              # ties: lowest r
        mu = float(Q[:, l] @ S[r] @ Q[:, l])
        if qt[l, r] * mu < 0:
            Q[:, l] = -Q[:, l]
    return Q


def sketch_scale(S: np.ndarray) -> float:
    return float(np.sqrt(np.mean([np.sum(Sr * Sr) for Sr in S])))


def features(S: np.ndarray, Theta: np.ndarray, Q: np.ndarray, P: int) -> np.ndarray:
    """Network input (4 P^2 + 4 P): frame sketches over sigma, then frame thetas."""
    k = Q.shape[0]
    sigma = sketch_scale(S)
    x = np.zeros(N_SKETCH * P * P + N_SKETCH * P)
    for r in range(N_SKETCH):
        F = np.zeros((P, P))
        F[:k, :k] = Q.T @ S[r] @ Q / sigma
        x[r * P * P:(r + 1) * P * P] = F.ravel()
        x[N_SKETCH * P * P + r * P: N_SKETCH * P * P + r * P + k] = Q.T @ Theta[:, r]
    return x


def init_params(n_in: int, n_hidden: int, n_out: int, gen: np.random.Generator) -> dict:
    """Uniform +-1/sqrt(fan_in) weights and biases (the usual default)."""
    s1, s2 = 1.0 / np.sqrt(n_in), 1.0 / np.sqrt(n_hidden)
    return {"W1": gen.uniform(-s1, s1, (n_hidden, n_in)), "b1": gen.uniform(-s1, s1, n_hidden),
            "W2": gen.uniform(-s2, s2, (n_out, n_hidden)), "b2": gen.uniform(-s2, s2, n_out)}


def mlp_forward(params: dict, X: np.ndarray):
    """X: (batch, n_in).  Returns (out, cache)."""
    Z = X @ params["W1"].T + params["b1"]
    H = np.maximum(Z, 0.0)
    out = H @ params["W2"].T + params["b2"]
    return out, (X, Z, H)


def mlp_backward(params: dict, cache, dout: np.ndarray) -> dict:
    """Gradients of a scalar loss given dL/dout (batch, n_out)."""
    X, Z, H = cache
    gW2 = dout.T @ H
    gb2 = dout.sum(axis=0)
    dH = dout @ params["W2"]
    dZ = dH * (Z > 0.0)
    gW1 = dZ.T @ X
    gb1 = dZ.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2}


def adam_step(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update (Kingma and Ba, 2015, Algorithm 1), step t >= 1, in place."""
    for name in params:
        g = grads[name]
        m[name] = beta1 * m[name] + (1.0 - beta1) * g
        v[name] = beta2 * v[name] + (1.0 - beta2) * g * g
        mhat = m[name] / (1.0 - beta1 ** t)
        vhat = v[name] / (1.0 - beta2 ** t)
        params[name] = params[name] - lr * mhat / (np.sqrt(vhat) + eps)


def warm_factors(out_row: np.ndarray, Q: np.ndarray, sigma: float, P: int) -> np.ndarray:
    """Initial factors V0 = Q out[:k, :k] sigma^(1/3) (column i = phi_i)."""
    k = Q.shape[0]
    O = out_row.reshape(P, P)[:k, :k]
    return Q @ O * np.cbrt(sigma)


def greedy_match(C: np.ndarray) -> np.ndarray:
    """perm[l] = the column assigned to frame vector l: repeatedly take the
    largest remaining |C[l, j]| (ties: lowest l, then lowest j)."""
    k = C.shape[0]
    A = np.abs(C).astype(np.float64)
    perm = np.full(k, -1)
    used_r, used_c = np.zeros(k, bool), np.zeros(k, bool)
    for _ in range(k):
        best, bl, bj = -1.0, -1, -1
        for l in range(k):
            if used_r[l]:
                continue
            for j in range(k):
                if not used_c[j] and A[l, j] > best:
                    best, bl, bj = A[l, j], l, j
        perm[bl] = bj
        used_r[bl] = used_c[bj] = True
    return perm


def frame_target(Q: np.ndarray, U: np.ndarray, lam: np.ndarray, sigma: float, P: int) -> np.ndarray:
    """Training target (P x P): column l holds Q^T phi*_{perm[l]} / sigma^(1/3)
    with phi*_j = lambda_j^(1/3) u_j and perm = greedy_match(Q^T U)."""
    k = Q.shape[0]
    perm = greedy_match(Q.T @ U)
    Phi_star = U * np.cbrt(lam)[None, :]
    Tg = np.zeros((P, P))
    Tg[:k, :k] = (Q.T @ Phi_star[:, perm]) / np.cbrt(sigma)
    return Tg


def mse(out: np.ndarray, target: np.ndarray, ks) -> tuple[float, np.ndarray]:
    """Mean squared error over the live k x k blocks and its gradient."""
    B = out.shape[0]
    P = int(round(np.sqrt(out.shape[1])))
    mask = np.zeros((B, P, P))
    for i, k in enumerate(ks):
        mask[i, :k, :k] = 1.0
    mask = mask.reshape(B, -1)
    cnt = mask.sum()
    d = (out - target) * mask
    return float(np.sum(d * d) / cnt), 2.0 * d / cnt
