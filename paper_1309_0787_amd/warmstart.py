"""Learned warm start of the stochastic updates: instance generation, training
and inference of the perceptron that maps a sketch of the whitened third
moment (in its canonical frame) to initial factors.  Orchestration only: the
sketch, frames, targets, perceptron products, Adam and the factors run in the
library's HIP kernels (``otm.ws_*``, ``otm.mlp_*``); torch holds the buffers.

Random initial factors (``synth.initial_factors``) remain the fallback, e.g.
for k above the network's P = 100.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import otm


@dataclass
class InstanceSet:
    """count instances, padded to the network's P: ks (int32), sketches S
    (count x 4 x P x P), Theta (count x P x 4), planted directions U
    (count x P x P, column j = u_j) and eigenvalues lam (count x P)."""
    ks: torch.Tensor
    S: torch.Tensor
    Theta: torch.Tensor
    U: torch.Tensor
    lam: torch.Tensor

    def __len__(self):
        return self.ks.numel()


def _thetas(k: int, seed: int, P: int) -> np.ndarray:
    g = np.random.default_rng([seed, 7])
    th = np.zeros((P, 4), dtype=np.float32)
    th[:k] = g.standard_normal((k, 4))
    return th


def exact_instance(k: int, seed: int, conc: float = 2.0):
    """Exact moments in whitened coordinates: T = sum_j lambda_j u_j^(x3) with
    lambda_j = ahat_j^(-1/2), ahat ~ Dir(conc), U Haar; the k rows
    y_j = (k lambda_j)^(1/3) u_j with alpha0 = 0 have exactly this tensor.
    Returns (Y (k x k) float32, U, lam) as numpy."""
    import synth
    g = np.random.default_rng([seed, 3])
    ahat = g.dirichlet(np.full(k, conc))
    lam = ahat ** -0.5
    U = synth.initial_factors(k, seed=seed, restart=77)
    Y = np.ascontiguousarray((U * np.cbrt(k * lam)[None, :]).T, dtype=np.float32)
    return Y, U, lam


def build_instances(specs: list[dict], device, P: int | None = None) -> InstanceSet:
    """specs: dicts with k, seed and kind 'exact' (exact moments) or 'sampled'
    (planted mixture rows: n, alpha0, views; their planted tensor has
    lambda_j = sqrt(k) and directions U).  Sketches run on the GPU."""
    import synth
    P = P or otm.ws_dims()["P"]
    cnt = len(specs)
    ks = torch.tensor([s["k"] for s in specs], dtype=torch.int32, device=device)
    S = torch.zeros((cnt, 4, P, P), dtype=torch.float32, device=device)
    Th = torch.zeros((cnt, P, 4), dtype=torch.float32, device=device)
    U = torch.zeros((cnt, P, P), dtype=torch.float32, device=device)
    lam = torch.zeros((cnt, P), dtype=torch.float32, device=device)
    for i, s in enumerate(specs):
        k = s["k"]
        if s.get("kind", "exact") == "exact":
            Y, Ui, li = exact_instance(k, s["seed"])
            Yd = torch.as_tensor(Y, device=device)
            YA = YB = YC = Yd
            a0 = 0.0
        else:
            YA, YB, YC, Ut = synth.planted_views(s["n"], k, s["alpha0"], s["views"], seed=s["seed"], sub=i,
                                                 device=device)
            Ui, li = Ut.numpy().astype(np.float64), np.full(k, np.sqrt(k))
            a0 = s["alpha0"]
        ybar = torch.stack([YA[:, :k].mean(0), YB[:, :k].mean(0), YC[:, :k].mean(0)]).contiguous()
        th = torch.as_tensor(_thetas(k, s["seed"], P), device=device)
        Th[i] = th
        otm.ws_sketch(YA, YB, YC, k, ybar, a0, th[:k].contiguous(), S[i])
        U[i, :k, :k] = torch.as_tensor(Ui, dtype=torch.float32, device=device)
        lam[i, :k] = torch.as_tensor(li, dtype=torch.float32, device=device)
    return InstanceSet(ks, S, Th, U, lam)


class WarmStart:
    """The perceptron and its Adam state (FP32 on the device)."""

    def __init__(self, device, seed: int = 0):
        d = otm.ws_dims()
        self.d = d
        self.device = device
        g = torch.Generator(device="cpu").manual_seed(seed)
        parts = []
        for rows, cols in ((d["hidden"], d["n_in"]), (d["n_out"], d["hidden"])):
            bound = 1.0 / np.sqrt(cols)
            parts.append((torch.rand((rows * cols,), generator=g) * 2 - 1) * bound)
            parts.append((torch.rand((rows,), generator=g) * 2 - 1) * bound)
        self.params = torch.cat(parts).to(device)
        assert self.params.numel() == d["n_params"]
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self._bf16 = None

    @staticmethod
    def prepare(inst: InstanceSet):
        """Frames, inputs and training targets of a set of instances."""
        Q, sigma, X, info = otm.ws_frames(inst.ks, inst.S, inst.Theta)
        tgt = otm.ws_target(inst.ks, Q, sigma, inst.U, inst.lam)
        return Q, sigma, X, tgt, info

    def train(self, X, tgt, ks, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0) -> list[float]:
        """Adam on the mean squared error over the live blocks; returns the
        loss of every step (host floats, read once at the end)."""
        cnt = X.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        ks_host = ks.cpu().numpy().astype(np.int64)
        losses = []
        for _ in range(epochs):
            order = torch.randperm(cnt, generator=g)
            for s in range(0, cnt, batch):
                idx = order[s:s + batch].to(self.device)
                Xb, tb, kb = X[idx], tgt[idx], ks[idx]
                live = int(np.sum(ks_host[order[s:s + batch].numpy()] ** 2))
                H, out = otm.mlp_forward(self.params, Xb)
                loss, dout = otm.ws_mse(kb, live, out, tb)
                otm.mlp_backward(self.params, Xb, H, dout, self.grads)
                self.t += 1
                otm.mlp_adam(self.params, self.grads, self.m, self.v, self.t, lr)
                losses.append(loss)
        self._bf16 = None
        return [float(x.item()) for x in losses]

    def infer(self, X, bf16: bool = True):
        if not bf16:
            return otm.mlp_forward(self.params, X)[1]
        if self._bf16 is None:
            self._bf16 = otm.mlp_to_bf16(self.params)
        return otm.mlp_forward_bf16(self._bf16, self.params, X)

    def initial_factors(self, YA, YB, YC, ybar3, k: int, alpha0: float, seed: int = 0, bf16: bool = True):
        """Warm-start factors for one problem (k x k FP32 on the device, phi_i
        contiguous, the layout of the STGD entry points)."""
        P = self.d["P"]
        if k > P:
            raise otm.OtmError(-8, f"the network takes k <= {P}; use random initial factors")
        S = torch.zeros((1, 4, P, P), dtype=torch.float32, device=self.device)
        th = torch.as_tensor(_thetas(k, seed, P), device=self.device)
        otm.ws_sketch(YA, YB, YC, k, ybar3, alpha0, th[:k].contiguous(), S[0])
        ks = torch.tensor([k], dtype=torch.int32, device=self.device)
        Q, sigma, X, info = otm.ws_frames(ks, S, th[None])
        out = self.infer(X, bf16)
        Phi = otm.ws_factors(ks, out, Q, sigma)
        return Phi[0, :k * k].reshape(k, k)


# ---------------------------------------------------------------------------
# Training and held-out instances drawn from the three workloads' generators
# ---------------------------------------------------------------------------
FAMILIES = {
    # the graph and document workloads: components, samples, Dirichlet total
    "mmsb_small": dict(k=10, n=500, alpha0=0.1),
    "lda_medium": dict(k=50, n=100000, alpha0=1.0),
    "mmsb_large": dict(k=100, n=50000, alpha0=0.5),
}


def family_weights(family: str, seed: int) -> np.ndarray:
    """Community shares of a workload's samples as its generator draws them,
    at the block-model limit (each sample in its largest community, which
    keeps the whitened third moment exactly orthogonal): the memberships are
    pi ~ Dir(alpha0/k 1) (Section 2), a symmetric law, so the index of the
    largest entry is uniform over the k communities and the counts of the n
    samples are Multinomial(n, 1/k) (drawn directly).  Returns alpha_hat_j,
    the share of community j (an empty community gets one sample)."""
    import synth
    f = FAMILIES[family]
    k, n = f["k"], f["n"]
    g = synth.rng(seed, synth.S_MISC, 31)
    counts = g.multinomial(n, np.full(k, 1.0 / k)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    return counts / counts.sum()


def generated_exact_instance(family: str, seed: int):
    """Exact moments of a block model from a workload's generator, in
    whitened coordinates: T = sum_j lambda_j u_j^(x3), lambda_j =
    alpha_hat_j^(-1/2) from family_weights, U Haar (the whitened basis is
    arbitrary, Section 3.1); the k rows y_j = (k lambda_j)^(1/3) u_j with
    alpha0 = 0 have exactly this tensor.  Returns (Y, U, lam) as numpy."""
    import synth
    ahat = family_weights(family, seed)
    k = ahat.size
    lam = ahat ** -0.5
    U = synth.initial_factors(k, seed=seed, restart=78)
    Y = np.ascontiguousarray((U * np.cbrt(k * lam)[None, :]).T, dtype=np.float32)
    return Y, U, lam


def build_generated(specs: list[dict], device, sampled_pool=None, P: int | None = None, progress=None) -> InstanceSet:
    """specs: dicts with family and seed, kind 'exact' (generated_exact_instance)
    or 'sampled': rows[i] of a whitened sample pool (sampled_pool: dict with Y
    (n x ldy FP32, device), U (k x k planted directions in the whitened
    coordinates), lam (k), alpha0) restricted to a seeded subset of size
    spec['n'].  Sketches run on the GPU.  progress: None or a callable
    taking the number of instances built (called every 5000)."""
    P = P or otm.ws_dims()["P"]
    cnt = len(specs)
    ks = torch.zeros(cnt, dtype=torch.int32, device=device)
    S = torch.zeros((cnt, 4, P, P), dtype=torch.float32, device=device)
    Th = torch.zeros((cnt, P, 4), dtype=torch.float32, device=device)
    U = torch.zeros((cnt, P, P), dtype=torch.float32, device=device)
    lam = torch.zeros((cnt, P), dtype=torch.float32, device=device)
    kk = []
    for i, s in enumerate(specs):
        if s.get("kind", "exact") == "exact":
            Y, Ui, li = generated_exact_instance(s["family"], s["seed"])
            k = Y.shape[0]
            YA = YB = YC = torch.as_tensor(Y, device=device)
            a0 = 0.0
        else:
            pool = sampled_pool
            k = pool["U"].shape[0]
            g = np.random.default_rng([s["seed"], 11])
            rows = torch.as_tensor(np.sort(g.choice(pool["Y"].shape[0], s["n"], replace=False)), device=device)
            YA = YB = YC = pool["Y"].index_select(0, rows).contiguous()
            Ui, li, a0 = pool["U"], pool["lam"], pool["alpha0"]
        kk.append(k)
        ybar = torch.stack([YA[:, :k].mean(0), YB[:, :k].mean(0), YC[:, :k].mean(0)]).contiguous()
        th = torch.as_tensor(_thetas(k, s["seed"], P), device=device)
        Th[i] = th
        otm.ws_sketch(YA, YB, YC, k, ybar, a0, th[:k].contiguous(), S[i])
        U[i, :k, :k] = torch.as_tensor(np.asarray(Ui), dtype=torch.float32, device=device)
        lam[i, :k] = torch.as_tensor(np.asarray(li), dtype=torch.float32, device=device)
        if progress is not None and (i + 1) % 5000 == 0:
            progress(i + 1)
    ks.copy_(torch.tensor(kk, dtype=torch.int32))
    return InstanceSet(ks, S, Th, U, lam)


def warm_factors_batch(warm: "WarmStart", inst: InstanceSet, bf16: bool = True) -> torch.Tensor:
    """Warm-start factors of every instance of a set (count x P*P, instance i's
    phi_j at row i, offset j*k), from the set's own sketches."""
    Q, sigma, X, info = otm.ws_frames(inst.ks, inst.S, inst.Theta)
    out = warm.infer(X, bf16)
    return otm.ws_factors(inst.ks, out, Q, sigma)
