"""Helpers shared by the GPU parity tests: host <-> device conversion and BF16
rounding of test inputs (round to nearest even, done by torch on the CPU)."""
from __future__ import annotations

import numpy as np
import torch

from paper_1309_0787_amd import otm


def dev():
    return torch.device("cuda:0")


def to_dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=dev(), dtype=dtype)


def host(t) -> np.ndarray:
    return t.detach().to("cpu", torch.float64).numpy()


def bf16_round(x: np.ndarray) -> np.ndarray:
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def f32_round(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def csr_dev(csr):
    return otm.DeviceCSR.from_host(csr, dev())


def padded(Y: np.ndarray, ldy: int, dtype) -> torch.Tensor:
    n, k = Y.shape
    out = np.zeros((n, ldy), dtype=np.float64)
    out[:, :k] = Y
    return to_dev(out, dtype)


def phi_rows(Phi: np.ndarray) -> torch.Tensor:
    """Oracle Phi (column i = phi_i) -> device k x k FP32 with row i = phi_i."""
    return to_dev(Phi.T.copy(), torch.float32)


def phi_cols(t: torch.Tensor) -> np.ndarray:
    """Device Phi (row i = phi_i) -> oracle layout (column i = phi_i)."""
    return host(t).T.copy()


def rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
