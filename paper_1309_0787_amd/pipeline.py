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
    events: dict = field(default_factory=dict)


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
        warm_seed: int = 0) -> FitResult:
    """views: 1 DeviceCSR (graph: the three views alias) or 3 (document views A, B, C).
    C_m2/CT_m2: the observations the second moment is built from and their transpose.
    Phi0: restarts x k x k FP32 (row i = phi_i), consumed in place.
    perms: passes x n int32 shared by the restarts, or restarts x passes x n.
    pi_view: index of the view whose rows get memberships (graphs), or None.
    warm: a trained warmstart.WarmStart; its factors replace Phi0[0] (the
    other restarts keep theirs)."""
    t = timer or Timer(False)
    k = cfg.k
    t.mark("start")
    Q, O = otm.power_sketch(C_m2, CT_m2, cfg.normalize, cfg.alpha0, S, cfg.q_power)
    t.mark("sketch")
    W, ev, W_lo = otm.whitener(O, Q, k, w_lo_dtype=cfg.y_dtype)
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
    Pi = None
    if pi_view is not None:
        Pi = otm.recover_pi(ys[pi_view], k, Phi0[0], theta=cfg.theta, tau=cfg.tau_pi)
    t.mark("post")
    return FitResult(W=W, evals=ev, Y=ys, ybar3=ybar3, Phi=Phi0, Pi=Pi, snapshots=snaps, nonfinite=flag)
