"""The hot path end to end on one GPU: M2 sketch -> whitener -> whitening
SpMM -> STGD run -> post-processing.  Orchestration only: every stage is a
libotm entry point; this module allocates device buffers and orders calls on
one stream."""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import otm


@dataclass
class FitConfig:
    k: int
    alpha0: float
    normalize: bool = False          # documents: True (length weights), graphs: False
    q_power: int = 3                 # power iterations of the sketch (0 = the paper's plain Nystrom)
    k_tilde: int = 0                 # sketch width, 0 = 2k
    y_dtype: int = otm.F32           # whitened samples and STGD contractions: F32 or BF16
    batch: int = 100
    passes: int = 50
    beta0: float = 1e-3
    beta_tau: float = 2500.0
    theta: float = 1.0
    compensated: bool = True
    restarts: int = 1
    tau_pi: float = 0.0              # membership threshold (graphs)
    topics: bool = False             # documents: unwhiten to topic-word matrix and Dirichlet weights

    @property
    def kt(self) -> int:
        return self.k_tilde if self.k_tilde else 2 * self.k


@dataclass
class FitResult:
    W: torch.Tensor
    evals: torch.Tensor
    Y: list
    ybar3: torch.Tensor
    Phi: torch.Tensor
    Pi: torch.Tensor | None = None
    snapshots: torch.Tensor | None = None
    nonfinite: torch.Tensor | None = None
    mu: torch.Tensor | None = None
    alpha_hat: torch.Tensor | None = None
    lam: torch.Tensor | None = None
    infos: torch.Tensor | None = None
    info_kinds: list = field(default_factory=list)
    events: dict = field(default_factory=dict)

    def check(self):
        """Raises for a device status set by any stage (one synchronisation)."""
        otm.check_info(self.infos, self.info_kinds)


class Timer:
    """HIP events on the stream the stages run on."""

    def __init__(self, enabled: bool):
        self.enabled = enabled
        self.marks = []

    def mark(self, name: str):
        if self.enabled:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.marks.append((name, e))

    def spans_ms(self) -> dict:
        out = {}
        for (n0, e0), (n1, e1) in zip(self.marks, self.marks[1:]):
            out[n1] = e0.elapsed_time(e1)
        return out


def fit(views, C_m2, CT_m2, S: torch.Tensor, Phi0: torch.Tensor, perms: torch.Tensor | None, cfg: FitConfig,
        pi_view=None, snapshots: bool = False, timer: Timer | None = None, warm=None,
        warm_seed: int = 0, check: bool = True) -> FitResult:
    """views: 1 DeviceCSR (graph: the three views alias) or 3 (document views A, B, C).
    C_m2/CT_m2: the observations the second moment is built from and their transpose.
    Phi0: restarts x k x k FP32 (row i = phi_i), consumed in place.
    perms: passes x n int32 shared by the restarts, or restarts x passes x n.
    pi_view: index of the view whose rows get memberships (graphs), or None.
    warm: a trained warmstart.WarmStart; its factors replace Phi0[0] (the
    other restarts keep theirs).
    The stages' device status words go to one buffer that is read once at the
    end (check=True) or left to the caller (FitResult.check), so no stage
    waits for the device in between."""
    t = timer or Timer(False)
    k = cfg.k
    kinds = otm.power_sketch_kinds(cfg.q_power) + ["whitener"] + (["unwhiten_topics"] if cfg.topics else [])
    infos = torch.zeros(len(kinds), dtype=torch.int32, device=S.device)
    t.mark("start")
    Q, O = otm.power_sketch(C_m2, CT_m2, cfg.normalize, cfg.alpha0, S, cfg.q_power, infos=infos)
    t.mark("sketch")
    nsk = 2 * cfg.q_power + 1
    W, ev, W_lo = otm.whitener(O, Q, k, w_lo_dtype=cfg.y_dtype, info=infos[nsk:nsk + 1])
    t.mark("whitener")
    ys, ybars = [], []
    for v in views:
        Y, yb = otm.whiten(v, cfg.normalize, W_lo, y_dtype=cfg.y_dtype)
        ys.append(Y)
        ybars.append(yb)
    if len(ys) == 1:
        ys = ys * 3
        ybars = ybars * 3
    ybar3 = torch.cat(ybars).contiguous()
    t.mark("whiten")
    if warm is not None:
        Phi0[0].copy_(warm.initial_factors(ys[0], ys[1], ys[2], ybar3, k, cfg.alpha0, seed=warm_seed))
        t.mark("warm")
    n = views[0].n_rows
    p = otm.SgdParams(k=k, batch=cfg.batch, passes=cfg.passes, y_dtype=cfg.y_dtype, compensated=cfg.compensated,
                      alpha0=cfg.alpha0, theta=cfg.theta, beta0=cfg.beta0, beta_tau=cfg.beta_tau,
                      ldy=ys[0].shape[1])
    R = cfg.restarts
    snaps = torch.empty((R, cfg.passes, k, k), dtype=torch.float32, device=S.device) if snapshots else None
    flag = torch.zeros(1, dtype=torch.int32, device=S.device)
    stride = 0 if (perms is None or perms.dim() == 2) else perms.shape[1] * perms.shape[2]
    otm.sgd_run(p, n, ys[0], ys[1], ys[2], ybar3, perms, Phi0, restarts=R, perm_stride=stride,
                snapshots=snaps, nonfinite=flag)
    t.mark("stgd")
    Pi = mu = ah = lam = None
    if pi_view is not None:
        Pi = otm.recover_pi(ys[pi_view], k, Phi0[0], theta=cfg.theta, tau=cfg.tau_pi)
    if cfg.topics:
        mu, ah, lam = otm.unwhiten_topics(W, Phi0[0], theta=cfg.theta, info=infos[nsk + 1:nsk + 2])
    t.mark("post")
    res = FitResult(W=W, evals=ev, Y=ys, ybar3=ybar3, Phi=Phi0, Pi=Pi, snapshots=snaps, nonfinite=flag, mu=mu,
                    alpha_hat=ah, lam=lam, infos=infos, info_kinds=kinds)
    if check:
        res.check()
    return res


@dataclass
class FourResult:
    factors: "otm.PinvFactors"
    W: torch.Tensor
    WB: torch.Tensor
    WC: torch.Tensor
    evals: torch.Tensor
    Y: list
    ybar3: torch.Tensor
    Phi: torch.Tensor
    Pi: torch.Tensor | None
    Pi_nodes: list
    nonfinite: torch.Tensor
    infos: torch.Tensor
    info_kinds: list

    def check(self):
        otm.check_info(self.infos, self.info_kinds)


def fit_four(G: "otm.DevicePartition", S: torch.Tensor, S_B: torch.Tensor, S_C: torch.Tensor, Phi0: torch.Tensor,
             perms: torch.Tensor | None, cfg: FitConfig, q_pinv: int = 1, node_blocks=(), timer: Timer | None = None,
             check: bool = True) -> FourResult:
    """The four-partition graph path (Section 2.2, Eq. transitionMat; Section
    4.1; Section 4.2): refined sketches of Pairs(B, C) (q_pinv range-finder
    steps) -> randomized pseudo-inverse factors -> power-iterated sketch of
    the four-partition M2 -> whitener -> W_B = Z_B^T W, W_C = Z_C^T W ->
    three whitened views -> STGD -> memberships of the X nodes (Pi) and of
    the nodes of each block G[S, A] in node_blocks (Pi_nodes).
    S: n_A x k, S_B: n_B x 2k, S_C: n_C x 2k FP64 projections.  This M2 has
    rank at most k + 1 (Z_B and Z_C have rank k), so its sketch has k
    columns and cfg.q_power = 1 power step puts it in M2's column space; a
    wider sketch is rank deficient and its orthonormalisation is refused.
    Phi0: restarts x k x k (row i = phi_i), consumed in place."""
    t = timer or Timer(False)
    k, q = cfg.k, cfg.q_power
    kinds = ["orthonormalize"] * (2 * q_pinv) + ["pinv_factors"] + ["orthonormalize"] * q + ["whitener"]
    infos = torch.zeros(len(kinds), dtype=torch.int32, device=S.device)
    slot = lambda i: infos[i:i + 1]
    t.mark("start")
    SB, SC = S_B, S_C
    for j in range(q_pinv):
        SB = otm.orthonormalize(otm.pairs_apply(G.BX, G.XC, SC), info=slot(2 * j))
        SC = otm.orthonormalize(otm.pairs_apply(G.CX, G.XB, SB), info=slot(2 * j + 1))
    J = otm.pairs_apply(G.BX, G.XC, SC)
    K = otm.pairs_apply(G.CX, G.XB, SB)
    n0 = 2 * q_pinv
    F = otm.pinv_factors(J, K, SB, k, info=slot(n0))
    t.mark("transition")
    Q, O = otm.power_sketch_four(G, F, cfg.alpha0, S, q, infos=infos[n0 + 1:n0 + 1 + q])
    t.mark("sketch")
    W, ev, W_lo = otm.whitener(O, Q, k, w_lo_dtype=cfg.y_dtype, info=slot(n0 + 1 + q))
    t.mark("whitener")
    WB = otm.transition_t_apply(G, F, 1, W)
    WC = otm.transition_t_apply(G, F, 2, W)
    ys, ybars = [], []
    for blk, Wv in ((G.XA, W_lo), (G.XB, otm.cast_rows(WB, cfg.y_dtype)), (G.XC, otm.cast_rows(WC, cfg.y_dtype))):
        Y, yb = otm.whiten(blk, False, Wv, y_dtype=cfg.y_dtype)
        ys.append(Y)
        ybars.append(yb)
    ybar3 = torch.cat(ybars).contiguous()
    t.mark("whiten")
    n = G.n_x
    p = otm.SgdParams(k=k, batch=cfg.batch, passes=cfg.passes, y_dtype=cfg.y_dtype, compensated=cfg.compensated,
                      alpha0=cfg.alpha0, theta=cfg.theta, beta0=cfg.beta0, beta_tau=cfg.beta_tau, ldy=ys[0].shape[1])
    flag = torch.zeros(1, dtype=torch.int32, device=S.device)
    stride = 0 if (perms is None or perms.dim() == 2) else perms.shape[1] * perms.shape[2]
    otm.sgd_run(p, n, ys[0], ys[1], ys[2], ybar3, perms, Phi0, restarts=cfg.restarts, perm_stride=stride,
                nonfinite=flag)
    t.mark("stgd")
    Pi = otm.recover_pi(ys[0], k, Phi0[0], theta=cfg.theta, tau=cfg.tau_pi)
    Pi_nodes = []
    for blk in node_blocks:
        Yn, _ = otm.whiten(blk, False, W_lo, y_dtype=cfg.y_dtype, want_ybar=False)
        Pi_nodes.append(otm.recover_pi(Yn, k, Phi0[0], theta=cfg.theta, tau=cfg.tau_pi))
    t.mark("post")
    res = FourResult(factors=F, W=W, WB=WB, WC=WC, evals=ev, Y=ys, ybar3=ybar3, Phi=Phi0, Pi=Pi, Pi_nodes=Pi_nodes,
                     nonfinite=flag, infos=infos, info_kinds=kinds)
    if check:
        res.check()
    return res
