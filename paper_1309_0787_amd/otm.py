"""Thin Python binding of libotm (ctypes).  Argument marshalling only: every
step runs in the library's HIP kernels.  torch provides device memory and the
current stream; nothing here computes the method.

The library must be built (``paper_1309_0787_amd.build.build()``); without it
every call raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotm.so")

F64, F32, BF16 = 0, 1, 2
_TORCH_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
_DTYPE_CODE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_dbl = ctypes.c_double


class OtmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"otm error {status}: {msg}")
        self.status = status


class OtmNotPSD(OtmError):
    pass


class OtmNonFinite(OtmError):
    pass


class _CSR(ctypes.Structure):
    _fields_ = [("n_rows", _i32), ("n_cols", _i32), ("nnz", _i64),
                ("rowptr", _vp), ("colidx", _vp), ("vals", _vp)]


class _Partition(ctypes.Structure):
    _fields_ = [("XA", _CSR), ("XB", _CSR), ("XC", _CSR), ("AX", _CSR), ("BX", _CSR), ("CX", _CSR)]


class _SgdParams(ctypes.Structure):
    _fields_ = [("k", _i32), ("batch", _i32), ("passes", _i32), ("ldy", _i32), ("y_dtype", _i32),
                ("compensated", _i32), ("alpha0", _dbl), ("theta", _dbl), ("beta0", _dbl),
                ("beta_tau", _dbl)]


class _Problem(ctypes.Structure):
    _fields_ = [("YA", _vp), ("YB", _vp), ("YC", _vp), ("ybar", _vp), ("perms", _vp), ("perm_stride", _i64),
                ("Phi0", _vp), ("Phi", _vp), ("score", _vp), ("n", _i32), ("k", _i32), ("ldy", _i32),
                ("pad_", _i32), ("alpha0", _dbl)]


_SIGS = {
    "otm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "otm_last_error": (ctypes.c_char_p, []),
    "otm_version": (ctypes.c_int, []),
    "otm_max_k": (ctypes.c_int, []),
    "otm_max_batch": (ctypes.c_int, []),
    "otm_csr_check_workspace": (_sz, []),
    "otm_csr_check": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.POINTER(_i64), _vp, _sz, _vp]),
    "otm_m2_apply_workspace": (_sz, [_i32, _i32, _i32]),
    "otm_m2_apply": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.POINTER(_CSR), ctypes.c_int, _dbl, _vp, _i32,
                                    _vp, _vp, _vp, _sz, _vp]),
    "otm_m2_apply_select_workspace": (_sz, [_i32, _i32]),
    "otm_m2_apply_select": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.POINTER(_CSR), ctypes.c_int, _dbl, _vp, _vp,
                                           _i32, _vp, _vp, _vp, _sz, _vp]),
    "otm_selection_dense": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _vp]),
    "otm_whitener_workspace": (_sz, [_i32, _i32, _i32]),
    "otm_whitener": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, ctypes.c_int, _i32, _vp, _vp, _sz,
                                    _vp]),
    "otm_orthonormalize_workspace": (_sz, [_i32, _i32]),
    "otm_orthonormalize": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "otm_pairs_apply_workspace": (_sz, [_i32, _i32]),
    "otm_pairs_apply": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.POINTER(_CSR), _vp, _i32, _vp, _vp, _sz, _vp]),
    "otm_pinv_factors_workspace": (_sz, [_i32, _i32, _i32, _i32]),
    "otm_pinv_factors": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                        _vp]),
    "otm_factored_apply_workspace": (_sz, [_i32, _i32, _i32]),
    "otm_factored_apply": (ctypes.c_int, [_vp, _i32, _vp, ctypes.c_int, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _sz,
                                          _vp]),
    "otm_transition_t_workspace": (_sz, [ctypes.POINTER(_Partition), _i32, _i32]),
    "otm_transition_t_apply": (ctypes.c_int, [ctypes.POINTER(_Partition), _vp, _vp, _vp, _i32, ctypes.c_int, _vp,
                                              _i32, _vp, _vp, _sz, _vp]),
    "otm_m2_apply_four_workspace": (_sz, [ctypes.POINTER(_Partition), _i32, _i32]),
    "otm_m2_apply_four": (ctypes.c_int, [ctypes.POINTER(_Partition), _vp, _vp, _vp, _i32, _dbl, _vp, _i32, _vp, _vp,
                                         _sz, _vp]),
    "otm_cast_rows": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, ctypes.c_int, _i32, _vp]),
    "otm_whiten_noalloc_capacity": (_sz, []),
    "otm_whiten_noalloc": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.c_int, _vp, ctypes.c_int, _i32, _i32, _vp,
                                          ctypes.c_int, _i32, _vp, _vp]),
    "otm_whiten_workspace": (_sz, [_i32, _i32]),
    "otm_whiten": (ctypes.c_int, [ctypes.POINTER(_CSR), ctypes.c_int, _vp, ctypes.c_int, _i32, _i32, _vp,
                                  ctypes.c_int, _i32, _vp, _vp, _sz, _vp]),
    "otm_sgd_step": (ctypes.c_int, [ctypes.POINTER(_SgdParams), _i32, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _vp]),
    "otm_sgd_run": (ctypes.c_int, [ctypes.POINTER(_SgdParams), _i32, _vp, _vp, _vp, _vp, _vp, _i64, _i32, _i64,
                                   _i64, _vp, _vp, _vp, _vp, _vp]),
    "otm_sgd_score_workspace": (_sz, [_i32]),
    "otm_sgd_score": (ctypes.c_int, [ctypes.POINTER(_SgdParams), _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _sz,
                                     _vp]),
    "otm_sgd_batched_plan": (ctypes.c_int, [ctypes.POINTER(_Problem), _i32, _i32, ctypes.POINTER(_SgdParams),
                                            ctypes.c_char_p, _vp, _vp, ctypes.POINTER(_vp)]),
    "otm_plan_size": (_sz, [_vp]),
    "otm_plan_image": (_vp, [_vp]),
    "otm_plan_groups": (_i32, [_vp]),
    "otm_plan_group_info": (ctypes.c_int, [_vp, _i32] + [ctypes.POINTER(_i32)] * 4),
    "otm_plan_free": (ctypes.c_int, [_vp]),
    "otm_sgd_batched_workspace": (_sz, [_vp]),
    "otm_sgd_batched": (ctypes.c_int, [_vp, _vp, _vp, _sz, _vp]),
    "otm_sgd_batched_graph": (ctypes.c_int, [_vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "otm_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "otm_graph_destroy": (ctypes.c_int, [_vp]),
    "otm_sgd_autotune": (ctypes.c_int, [ctypes.POINTER(_i32), _i32, _i32, ctypes.c_char_p, _vp]),
    "otm_ws_dims": (ctypes.c_int, [ctypes.POINTER(_i32)] * 4 + [ctypes.POINTER(_i64)]),
    "otm_ws_sketch_workspace": (_sz, [_i32, _i32]),
    "otm_ws_sketch": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _i32, _i32, _i32, _vp, _dbl, _vp, _vp, _i32, _vp,
                                     _sz, _vp]),
    "otm_ws_frames_workspace": (_sz, [_i32]),
    "otm_ws_frames": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_ws_target": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "otm_mlp_workspace": (_sz, [_i32]),
    "otm_mlp_forward": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_mlp_backward": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _dbl, _dbl, _dbl, _dbl, _vp]),
    "otm_mlp_to_bf16": (ctypes.c_int, [_vp, _vp, _vp]),
    "otm_mlp_bf16_workspace": (_sz, [_i32]),
    "otm_mlp_forward_bf16": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "otm_ws_mse_workspace": (_sz, [_i32]),
    "otm_ws_mse": (ctypes.c_int, [_i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_ws_factors": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "otm_unwhiten_workspace": (_sz, [_i32, _i32]),
    "otm_unwhiten_topics": (ctypes.c_int, [_vp, _i32, _i32, _vp, _dbl, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_recover_pi_workspace": (_sz, [_i32]),
    "otm_recover_pi": (ctypes.c_int, [_vp, ctypes.c_int, _i32, _i32, _i32, _vp, _dbl, _dbl, _vp, _vp, _sz, _vp]),
    "otm_validate_workspace": (_sz, [_i32, _i32, _i32]),
    "otm_validate": (ctypes.c_int, [_vp, _i32, _vp, _i32, _i32, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "otm_bridgeness": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(_CSR), _vp, _vp, _vp]),
    "otm_probe_copy": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp]),
    "otm_probe_mfma_flops": (_i64, [ctypes.c_int, _i64, _i32]),
    "otm_probe_mfma": (ctypes.c_int, [ctypes.c_int, _i64, _i32, _vp, _vp]),
    "otm_tensor_form": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _i32, _i32, _i32, _vp, _dbl, _vp, _vp]),
    "otm_residual_workspace": (_sz, [_i32, _i32]),
    "otm_residual": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp, _vp, _sz, _vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libotm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OtmError(-6, f"{LIB_PATH} not found: build the HIP library first "
                               "(paper_1309_0787_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            # a library older than this binding lacks some entry points:
            # only calls of those fail (the ABI test checks every export)
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        msg = lib().otm_last_error().decode()
        raise OtmError(status, msg)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise OtmError(-1, "tensor must live on the GPU")
    if not t.is_contiguous():
        # the library reads dense row-major buffers; a strided view would be misread
        raise OtmError(-1, "tensor must be contiguous (row-major)")
    return t.data_ptr()


def _ptr_rows(t) -> tuple[int, int]:
    """(pointer, row stride) of a 2-D GPU tensor with unit column stride (a
    row-padded buffer or a column slice of one)."""
    if not t.is_cuda:
        raise OtmError(-1, "tensor must live on the GPU")
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise OtmError(-1, "matrix must be row-major with unit column stride")
    return t.data_ptr(), t.stride(0)


def _need(t, name: str, dtype, shape=None, min_rows: int | None = None):
    """Refuses a tensor of another element type or shape than the entry point
    reads: the C ABI takes bare pointers, so a mismatch would make a kernel
    read or write outside the buffer.  shape entries of None match anything;
    min_rows (instead of shape[0]) accepts longer buffers."""
    if t is None:
        raise OtmError(-1, f"{name} must not be None")
    if t.dtype != dtype:
        raise OtmError(-3, f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None:
        bad = t.dim() != len(shape) or any(s is not None and int(a) != int(s) for a, s in zip(t.shape, shape))
        if bad:
            want = tuple("*" if s is None else int(s) for s in shape)
            raise OtmError(-2, f"{name} must have shape {want}, got {tuple(t.shape)}")
    if min_rows is not None and (t.dim() < 1 or t.shape[0] < min_rows):
        raise OtmError(-2, f"{name} must have at least {min_rows} rows, got {tuple(t.shape)}")


def _need_numel(t, name: str, dtype, numel: int):
    if t is None:
        raise OtmError(-1, f"{name} must not be None")
    if t.dtype != dtype:
        raise OtmError(-3, f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise OtmError(-2, f"{name} must hold {numel} values, got {t.numel()}")


def _need_w(W, C):
    if W.dtype not in (torch.float32, torch.bfloat16):
        raise OtmError(-3, f"W must be FP32 or BF16, got {W.dtype}")
    if W.dim() != 2 or W.shape[0] != C.n_cols:
        raise OtmError(-2, f"W must have one row per column of C ({C.n_cols}), got {tuple(W.shape)}")


def _beyond_capacity(p) -> bool:
    """k or batch past what the kernels are compiled for: the library refuses
    the call itself (OTM_ECAPACITY), before any buffer is read."""
    return p.k > int(lib().otm_max_k()) or p.batch > int(lib().otm_max_batch())


def _need_views(p, n: int, YA, YB, YC, ybar3):
    """The three views of an STGD call: y_dtype, ldy columns, at least n rows;
    ybar3 the 3 x k FP32 means."""
    ldy = p.ldy if p.ldy else default_ldy(p.k)
    dt = _TORCH_DTYPE[p.y_dtype]
    for name, Y in (("YA", YA), ("YB", YB), ("YC", YC)):
        _need(Y, name, dt, (None, ldy), min_rows=n)
    _need_numel(ybar3, "ybar3", torch.float32, 3 * p.k)


def _need_csr_pair(C, CT):
    if CT.n_rows != C.n_cols or CT.n_cols != C.n_rows or CT.nnz != C.nnz:
        raise OtmError(-2, "CT must be the transpose of C (n_cols x n_rows, same nnz)")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ CSR
class DeviceCSR:
    """A CSR whose arrays live on the GPU (int32 rowptr/colidx, float32 vals or None)."""

    def __init__(self, n_rows, n_cols, rowptr, colidx, vals=None):
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.rowptr, self.colidx, self.vals = rowptr, colidx, vals
        self.nnz = int(colidx.numel())

    @staticmethod
    def from_host(csr, device) -> "DeviceCSR":
        rp = torch.from_numpy(csr.rowptr).to(device=device, dtype=torch.int32)
        ci = torch.from_numpy(csr.colidx).to(device=device, dtype=torch.int32)
        v = None if csr.vals is None else torch.from_numpy(csr.vals).to(device=device, dtype=torch.float32)
        return DeviceCSR(csr.n_rows, csr.n_cols, rp, ci, v)

    def c(self) -> _CSR:
        return _CSR(self.n_rows, self.n_cols, self.nnz, _ptr(self.rowptr), _ptr(self.colidx), _ptr(self.vals))

    @property
    def device(self):
        return self.rowptr.device


def csr_check(C: DeviceCSR, stream=None) -> int:
    ws = _ws(lib().otm_csr_check_workspace(), C.device)
    bad = _i64(0)
    cc = C.c()
    _check(lib().otm_csr_check(ctypes.byref(cc), ctypes.byref(bad), _ptr(ws), ws.numel(), _stream(stream)))
    return int(bad.value)


# ------------------------------------------------------------------ a1, a2
def _info_slot(info, device):
    """(slot, deferred): a caller's 1-element int32 device tensor receives the
    entry point's device status and is checked later (check_info); without one
    a fresh slot is checked right after the call (a stream synchronisation)."""
    if info is None:
        return torch.zeros(1, dtype=torch.int32, device=device), False
    if info.dtype != torch.int32 or info.numel() != 1 or not info.is_cuda:
        raise OtmError(-1, "info must be a 1-element int32 GPU tensor")
    return info, True


_INFO_ERRORS = {
    "pinv_factors": (OtmNotPSD, -4, "sketched pairs matrix has no rank-k part (s_k <= 1e-12 s_1)"),
    "m2_apply": (OtmError, -1, "a document has fewer than 2 tokens"),
    "m2_apply_select": (OtmError, -1, "a document has fewer than 2 tokens or a selected row is out of range"),
    "whitener": (OtmNotPSD, -4, "projected second moment has no k positive eigenvalues"),
    "orthonormalize": (OtmError, -4, "sketch is rank deficient"),
    "unwhiten_topics": (OtmError, -4, "W^T W is not positive definite"),
}


def _raise_info(kind: str):
    cls, code, msg = _INFO_ERRORS[kind]
    raise cls(code, msg)


def check_info(infos: torch.Tensor, kinds: list[str]):
    """Raises for the first non-zero device status among infos[i] (written by
    the entry point kinds[i]); one synchronisation for all of them."""
    codes = infos.cpu().tolist()
    for c, kind in zip(codes, kinds):
        if c != 0:
            _raise_info(kind)


def m2_apply(C: DeviceCSR, CT: DeviceCSR, normalize: bool, alpha0: float, S: torch.Tensor, stream=None,
             info: torch.Tensor | None = None):
    """O = M2 S (FP64).  Raises OtmError if a document has fewer than 2 tokens
    (at once, or through check_info when the caller passes an info slot)."""
    _need(S, "S", torch.float64, (C.n_cols, None))
    _need_csr_pair(C, CT)
    d, kt = S.shape
    O = torch.empty((d, kt), dtype=torch.float64, device=S.device)
    info, deferred = _info_slot(info, S.device)
    ws = _ws(lib().otm_m2_apply_workspace(C.n_rows, C.n_cols, kt), S.device)
    c1, c2 = C.c(), CT.c()
    _check(lib().otm_m2_apply(ctypes.byref(c1), ctypes.byref(c2), int(normalize), float(alpha0), _ptr(S), kt,
                              _ptr(O), _ptr(info), _ptr(ws), ws.numel(), _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("m2_apply")
    return O


def m2_apply_select(C: DeviceCSR, CT: DeviceCSR, normalize: bool, alpha0: float, sel_rows: torch.Tensor,
                    sel_signs: torch.Tensor, stream=None, info: torch.Tensor | None = None):
    """O = M2 S for the column selection S[sel_rows[j], j] = sel_signs[j] (FP64)."""
    if sel_rows.dtype != torch.int32 or sel_signs.dtype != torch.float64 or sel_rows.numel() != sel_signs.numel():
        raise OtmError(-3, "sel_rows must be int32 and sel_signs FP64 of the same length")
    _need_csr_pair(C, CT)
    kt = sel_rows.numel()
    d = C.n_cols
    O = torch.empty((d, kt), dtype=torch.float64, device=sel_rows.device)
    info, deferred = _info_slot(info, sel_rows.device)
    ws = _ws(lib().otm_m2_apply_select_workspace(C.n_rows, d), sel_rows.device)
    c1, c2 = C.c(), CT.c()
    _check(lib().otm_m2_apply_select(ctypes.byref(c1), ctypes.byref(c2), int(normalize), float(alpha0), _ptr(sel_rows),
                                     _ptr(sel_signs), kt, _ptr(O), _ptr(info), _ptr(ws), ws.numel(), _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("m2_apply_select")
    return O


def selection_dense(sel_rows: torch.Tensor, sel_signs: torch.Tensor, d: int, stream=None) -> torch.Tensor:
    if sel_rows.dtype != torch.int32 or sel_signs.dtype != torch.float64 or sel_rows.numel() != sel_signs.numel():
        raise OtmError(-3, "sel_rows must be int32 and sel_signs FP64 of the same length")
    kt = sel_rows.numel()
    S = torch.empty((d, kt), dtype=torch.float64, device=sel_rows.device)
    _check(lib().otm_selection_dense(_ptr(sel_rows), _ptr(sel_signs), d, kt, _ptr(S), _stream(stream)))
    return S


def default_ldw(k: int, dtype: int) -> int:
    """Row stride of W for the whitening SpMM: k rounded up to 16 bytes."""
    per = 8 if dtype == BF16 else 4
    return (k + per - 1) // per * per


def whitener(O: torch.Tensor, S: torch.Tensor, k: int, w_lo_dtype: int | None = F32, ldw_lo: int | None = None,
             stream=None, info: torch.Tensor | None = None):
    """(W FP64 d x k, evals FP64 k, W_lo in w_lo_dtype or None).  W_lo is the
    d x k view of a d x ldw_lo buffer (default: k rounded up to 16 bytes) whose
    padding columns hold 0.  Raises OtmNotPSD."""
    _need(O, "O", torch.float64, (None, None))
    _need(S, "S", torch.float64, tuple(O.shape))
    d, kt = O.shape
    W = torch.empty((d, k), dtype=torch.float64, device=O.device)
    ev = torch.empty(k, dtype=torch.float64, device=O.device)
    W_lo, ld = None, k
    if w_lo_dtype is not None:
        ld = default_ldw(k, w_lo_dtype) if ldw_lo is None else int(ldw_lo)
        W_lo = torch.empty((d, ld), dtype=_TORCH_DTYPE[w_lo_dtype], device=O.device)
    info, deferred = _info_slot(info, O.device)
    ws = _ws(lib().otm_whitener_workspace(d, kt, k), O.device)
    _check(lib().otm_whitener(_ptr(O), _ptr(S), d, kt, k, _ptr(W), _ptr(ev), _ptr(W_lo),
                              F32 if w_lo_dtype is None else w_lo_dtype, ld, _ptr(info), _ptr(ws), ws.numel(),
                              _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("whitener")
    return W, ev, (None if W_lo is None else W_lo[:, :k])


def orthonormalize(Y: torch.Tensor, stream=None, info: torch.Tensor | None = None) -> torch.Tensor:
    """Q = Y (Y^T Y)^(-1/2) (FP64)."""
    _need(Y, "Y", torch.float64, (None, None))
    d, m = Y.shape
    Q = torch.empty_like(Y)
    info, deferred = _info_slot(info, Y.device)
    ws = _ws(lib().otm_orthonormalize_workspace(d, m), Y.device)
    _check(lib().otm_orthonormalize(_ptr(Y), d, m, _ptr(Q), _ptr(info), _ptr(ws), ws.numel(), _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("orthonormalize")
    return Q


def power_sketch(C: DeviceCSR, CT: DeviceCSR, normalize: bool, alpha0: float, S: torch.Tensor, q: int,
                 stream=None, infos: torch.Tensor | None = None):
    """Sketch for the whitener: Q_0 = S, Q_j = orth(M2 Q_{j-1}); returns
    (Q_q, O = M2 Q_q).  q = 0 returns (S, M2 S).  infos: None (each status
    checked at once) or 2q + 1 int32 device slots, in call order
    m2_apply, orthonormalize, ..., m2_apply (power_sketch_kinds(q))."""
    if infos is not None and infos.numel() < 2 * q + 1:
        raise OtmError(-1, f"power_sketch needs {2 * q + 1} info slots")
    slot = (lambda i: None) if infos is None else (lambda i: infos[i:i + 1])
    Q = S
    for j in range(q):
        Q = orthonormalize(m2_apply(C, CT, normalize, alpha0, Q, stream, info=slot(2 * j)), stream,
                           info=slot(2 * j + 1))
    return Q, m2_apply(C, CT, normalize, alpha0, Q, stream, info=slot(2 * q))


def power_sketch_kinds(q: int) -> list[str]:
    return ["m2_apply", "orthonormalize"] * q + ["m2_apply"]


# ------------------------------------------------------------------ four-partition graph moments
class DevicePartition:
    """The blocks G[X, A], G[X, B], G[X, C] of a graph and their transposes,
    as DeviceCSRs (Section 2.2 node partition)."""

    def __init__(self, XA, XB, XC, AX, BX, CX):
        self.XA, self.XB, self.XC, self.AX, self.BX, self.CX = XA, XB, XC, AX, BX, CX

    @staticmethod
    def from_blocks(blocks: dict, device) -> "DevicePartition":
        names = (("X", "A"), ("X", "B"), ("X", "C"), ("A", "X"), ("B", "X"), ("C", "X"))
        return DevicePartition(*[DeviceCSR.from_host(blocks[n], device) for n in names])

    def c(self) -> _Partition:
        return _Partition(self.XA.c(), self.XB.c(), self.XC.c(), self.AX.c(), self.BX.c(), self.CX.c())

    @property
    def n_x(self):
        return self.XA.n_rows

    @property
    def sizes(self):
        return self.XA.n_cols, self.XB.n_cols, self.XC.n_cols

    @property
    def device(self):
        return self.XA.device


def pairs_apply(G1T: DeviceCSR, G2: DeviceCSR, V: torch.Tensor, stream=None) -> torch.Tensor:
    """Pairs(Y1, Y2) V = (1/n_X) G[Y1, X] (G[X, Y2] V) (FP64)."""
    _need(V, "V", torch.float64, (G2.n_cols, None))
    if G1T.n_cols != G2.n_rows:
        raise OtmError(-2, "G1T must have one column per sample row of G2")
    n2, m = V.shape
    out = torch.empty((G1T.n_rows, m), dtype=torch.float64, device=V.device)
    ws = _ws(lib().otm_pairs_apply_workspace(G2.n_rows, m), V.device)
    a, b = G1T.c(), G2.c()
    _check(lib().otm_pairs_apply(ctypes.byref(a), ctypes.byref(b), _ptr(V), m, _ptr(out), _ptr(ws), ws.numel(),
                                 _stream(stream)))
    return out


@dataclass
class PinvFactors:
    """P^+ ~ QK core QJ^T (n2 x n1); sv: the top k singular values of Psi."""
    QJ: torch.Tensor
    QK: torch.Tensor
    core: torch.Tensor
    sv: torch.Tensor
    k: int


def pinv_factors(J: torch.Tensor, K: torch.Tensor, S_left: torch.Tensor, k: int, stream=None,
                 info: torch.Tensor | None = None) -> PinvFactors:
    """Rank-k randomized pseudo-inverse of P from J = P S_right, K = P^T S_left."""
    _need(J, "J", torch.float64, (None, None))
    n1, m = J.shape
    _need(K, "K", torch.float64, (None, m))
    _need(S_left, "S_left", torch.float64, (n1, m))
    n2 = K.shape[0]
    dev = J.device
    QJ = torch.empty((n1, k), dtype=torch.float64, device=dev)
    QK = torch.empty((n2, k), dtype=torch.float64, device=dev)
    core = torch.empty((k, k), dtype=torch.float64, device=dev)
    sv = torch.empty(k, dtype=torch.float64, device=dev)
    info, deferred = _info_slot(info, dev)
    ws = _ws(lib().otm_pinv_factors_workspace(n1, n2, m, k), dev)
    _check(lib().otm_pinv_factors(_ptr(J), _ptr(K), _ptr(S_left), n1, n2, m, k, _ptr(QJ), _ptr(QK), _ptr(core),
                                  _ptr(sv), _ptr(info), _ptr(ws), ws.numel(), _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("pinv_factors")
    return PinvFactors(QJ, QK, core, sv, k)


def factored_apply(Q_in: torch.Tensor, core: torch.Tensor, trans: bool, Q_out: torch.Tensor, X: torch.Tensor,
                   stream=None) -> torch.Tensor:
    """Q_out M (Q_in^T X), M = core or core^T."""
    _need(Q_in, "Q_in", torch.float64, (None, None))
    _need(core, "core", torch.float64, (Q_in.shape[1], Q_in.shape[1]))
    _need(Q_out, "Q_out", torch.float64, (None, Q_in.shape[1]))
    _need(X, "X", torch.float64, (Q_in.shape[0], None))
    n_in, k = Q_in.shape
    n_out = Q_out.shape[0]
    m = X.shape[1]
    Y = torch.empty((n_out, m), dtype=torch.float64, device=X.device)
    ws = _ws(lib().otm_factored_apply_workspace(n_in, k, m), X.device)
    _check(lib().otm_factored_apply(_ptr(Q_in), n_in, _ptr(core), int(bool(trans)), _ptr(Q_out), n_out, k, _ptr(X), m,
                                    _ptr(Y), _ptr(ws), ws.numel(), _stream(stream)))
    return Y


def transition_t_apply(G: DevicePartition, F: PinvFactors, view: int, V: torch.Tensor, stream=None) -> torch.Tensor:
    """view 1: Z_B^T V (n_B x m); view 2: Z_C^T V (n_C x m)."""
    _need(V, "V", torch.float64, (G.XA.n_cols, None))
    m = V.shape[1]
    rows = G.XB.n_cols if view == 1 else G.XC.n_cols
    out = torch.empty((rows, m), dtype=torch.float64, device=V.device)
    gc = G.c()
    ws = _ws(lib().otm_transition_t_workspace(ctypes.byref(gc), F.k, m), V.device)
    _check(lib().otm_transition_t_apply(ctypes.byref(gc), _ptr(F.QJ), _ptr(F.QK), _ptr(F.core), F.k, int(view), _ptr(V),
                                        m, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def m2_apply_four(G: DevicePartition, F: PinvFactors, alpha0: float, S: torch.Tensor, stream=None) -> torch.Tensor:
    """O = M2 S for the four-partition second moment (FP64)."""
    _need(S, "S", torch.float64, (G.XA.n_cols, None))
    m = S.shape[1]
    O = torch.empty((G.XA.n_cols, m), dtype=torch.float64, device=S.device)
    gc = G.c()
    ws = _ws(lib().otm_m2_apply_four_workspace(ctypes.byref(gc), F.k, m), S.device)
    _check(lib().otm_m2_apply_four(ctypes.byref(gc), _ptr(F.QJ), _ptr(F.QK), _ptr(F.core), F.k, float(alpha0), _ptr(S),
                                   m, _ptr(O), _ptr(ws), ws.numel(), _stream(stream)))
    return O


def power_sketch_four(G: DevicePartition, F: PinvFactors, alpha0: float, S: torch.Tensor, q: int, stream=None,
                      infos: torch.Tensor | None = None):
    """The power-iterated sketch with the four-partition M2; infos: None or q
    int32 device slots (the orthonormalisations)."""
    if infos is not None and infos.numel() < q:
        raise OtmError(-1, f"power_sketch_four needs {q} info slots")
    Q = S
    for j in range(q):
        Q = orthonormalize(m2_apply_four(G, F, alpha0, Q, stream), stream,
                           info=None if infos is None else infos[j:j + 1])
    return Q, m2_apply_four(G, F, alpha0, Q, stream)


def cast_rows(X: torch.Tensor, dtype: int, ld: int | None = None, stream=None) -> torch.Tensor:
    """FP64 rows to an F32/BF16 copy with row stride ld (default: 16-byte rows);
    returns the rows x cols view of the padded buffer."""
    _need(X, "X", torch.float64, (None, None))
    rows, cols = X.shape
    ld = default_ldw(cols, dtype) if ld is None else int(ld)
    out = torch.empty((rows, ld), dtype=_TORCH_DTYPE[dtype], device=X.device)
    _check(lib().otm_cast_rows(_ptr(X), rows, cols, X.stride(0), _ptr(out), dtype, ld, _stream(stream)))
    return out[:, :cols]


# ------------------------------------------------------------------ a3
def default_ldy(k: int) -> int:
    return (k + 7) // 8 * 8


def whiten(C: DeviceCSR, normalize: bool, W: torch.Tensor, y_dtype: int = F32, ldy: int | None = None,
           want_ybar: bool = True, out: torch.Tensor | None = None, stream=None):
    """Y (n x ldy, y_dtype) and ybar (k FP32, or None).  W (d x k) may be a
    column slice of a row-padded buffer; its row stride is passed as ldw."""
    _need_w(W, C)
    d, k = W.shape
    w_ptr, ldw = _ptr_rows(W)
    if out is not None:   # the row stride is the output's own
        if out.dim() != 2 or out.shape[0] != C.n_rows or (ldy is not None and ldy != out.shape[1]):
            raise ValueError(f"out must be {C.n_rows} x ldy, got {tuple(out.shape)} (ldy={ldy})")
        if out.dtype != _TORCH_DTYPE[y_dtype]:
            raise ValueError(f"out is {out.dtype}, y_dtype asks for {_TORCH_DTYPE[y_dtype]}")
        ldy = out.shape[1]
    ldy = default_ldy(k) if ldy is None else ldy
    Y = out if out is not None else torch.empty((C.n_rows, ldy), dtype=_TORCH_DTYPE[y_dtype], device=W.device)
    ybar = torch.empty(k, dtype=torch.float32, device=W.device) if want_ybar else None
    ws = _ws(lib().otm_whiten_workspace(C.n_rows, k), W.device)
    cc = C.c()
    _check(lib().otm_whiten(ctypes.byref(cc), int(normalize), w_ptr, _DTYPE_CODE[W.dtype], k, ldw, _ptr(Y),
                            y_dtype, ldy, _ptr(ybar), _ptr(ws), ws.numel(), _stream(stream)))
    return Y, ybar


def whiten_noalloc(C: DeviceCSR, normalize: bool, W: torch.Tensor, Y: torch.Tensor, ybar: torch.Tensor | None,
                   y_dtype: int = F32, stream=None):
    """otm_whiten_noalloc into caller-given Y (n x ldy) and ybar (k FP32 or
    None): no workspace, nothing allocated by the library or here."""
    _need_w(W, C)
    d, k = W.shape
    w_ptr, ldw = _ptr_rows(W)
    if Y.dim() != 2 or Y.shape[0] != C.n_rows or Y.dtype != _TORCH_DTYPE[y_dtype]:
        raise ValueError("Y must be n x ldy in y_dtype")
    cc = C.c()
    _check(lib().otm_whiten_noalloc(ctypes.byref(cc), int(normalize), w_ptr, _DTYPE_CODE[W.dtype], k, ldw, _ptr(Y),
                                    y_dtype, Y.shape[1], _ptr(ybar), _stream(stream)))
    return Y, ybar


# ------------------------------------------------------------------ a4, a5
@dataclass
class SgdParams:
    k: int
    batch: int = 100
    passes: int = 1
    ldy: int = 0
    y_dtype: int = F32
    compensated: bool = True
    alpha0: float = 0.0
    theta: float = 1.0
    beta0: float = 0.01
    beta_tau: float = 1e12

    def c(self) -> _SgdParams:
        ldy = self.ldy if self.ldy else default_ldy(self.k)
        return _SgdParams(self.k, self.batch, self.passes, ldy, self.y_dtype, int(self.compensated), self.alpha0,
                          self.theta, self.beta0, self.beta_tau)


def sgd_step(p: SgdParams, rows: int, YA, YB, YC, ybar3: torch.Tensor, beta: float, Phi: torch.Tensor,
             Phi_comp: torch.Tensor | None = None, stream=None):
    """One STGD step on the first `rows` rows; Phi (k x k FP32, row i = phi_i) updated in place."""
    if not _beyond_capacity(p):
        _need_views(p, rows, YA, YB, YC, ybar3)
        _need_numel(Phi, "Phi", torch.float32, p.k * p.k)
        if Phi_comp is not None:
            _need_numel(Phi_comp, "Phi_comp", torch.float32, p.k * p.k)
    cp = p.c()
    _check(lib().otm_sgd_step(ctypes.byref(cp), rows, _ptr(YA), _ptr(YB), _ptr(YC), _ptr(ybar3), float(beta),
                              _ptr(Phi), _ptr(Phi_comp), _stream(stream)))
    return Phi


def check_perms(perms: torch.Tensor | None, n: int, passes: int, restarts: int, perm_stride: int):
    """The kernels read perms[r*perm_stride + p*n + i] for every run r, pass p
    and row i (they range-check the values, not the buffer): refuse a buffer
    of another type or too short for that."""
    if perms is None:
        return
    if perms.dtype != torch.int32:
        raise OtmError(-3, f"perms must be int32, got {perms.dtype}")
    if not perms.is_contiguous():
        raise OtmError(-1, "perms must be contiguous")
    if perm_stride < 0:
        raise OtmError(-1, "perm_stride must be >= 0")
    need = (restarts - 1) * perm_stride + passes * n
    if perms.numel() < need:
        raise OtmError(-2, f"perms holds {perms.numel()} entries, the runs read {need} "
                           f"((restarts-1)*perm_stride + passes*n)")


def sgd_run(p: SgdParams, n: int, YA, YB, YC, ybar3: torch.Tensor, perms: torch.Tensor | None, Phi: torch.Tensor,
            restarts: int = 1, perm_stride: int = 0, start_step: int = 0, end_step: int = -1,
            Phi_comp: torch.Tensor | None = None, snapshots: torch.Tensor | None = None,
            nonfinite: torch.Tensor | None = None, stream=None):
    """Runs STGD steps [start_step, end_step) for `restarts` independent runs
    (Phi: restarts x k x k FP32, updated in place)."""
    check_perms(perms, n, p.passes, restarts, perm_stride)
    if not _beyond_capacity(p):
        _need_views(p, n, YA, YB, YC, ybar3)
        kk = p.k * p.k
        _need_numel(Phi, "Phi", torch.float32, restarts * kk)
        if Phi_comp is not None:
            _need_numel(Phi_comp, "Phi_comp", torch.float32, restarts * kk)
        if snapshots is not None and (snapshots.dtype != torch.float32
                                      or snapshots.numel() < restarts * p.passes * kk):
            raise OtmError(-2, "snapshots must be FP32 with restarts x passes x k x k values")
        if nonfinite is not None and (nonfinite.dtype != torch.int32 or nonfinite.numel() < 1):
            raise OtmError(-3, "nonfinite must be an int32 tensor")
    cp = p.c()
    _check(lib().otm_sgd_run(ctypes.byref(cp), n, _ptr(YA), _ptr(YB), _ptr(YC), _ptr(ybar3), _ptr(perms),
                             perm_stride, restarts, start_step, end_step, _ptr(Phi), _ptr(Phi_comp),
                             _ptr(snapshots), _ptr(nonfinite), _stream(stream)))
    return Phi


def sgd_score(p: SgdParams, n: int, YA, YB, YC, ybar3: torch.Tensor, Phi: torch.Tensor, restarts: int = 1,
              stream=None) -> torch.Tensor:
    """score_r = sum_ij (phi_i^T phi_j)^3 - 2 sum_i T(phi_i, phi_i, phi_i) for each of
    the `restarts` factor matrices in Phi (restarts x k x k FP32); FP64 result."""
    if not _beyond_capacity(p):
        _need_views(p, n, YA, YB, YC, ybar3)
        _need_numel(Phi, "Phi", torch.float32, restarts * p.k * p.k)
    score = torch.empty(restarts, dtype=torch.float64, device=Phi.device)
    ws = _ws(lib().otm_sgd_score_workspace(restarts), Phi.device)
    cp = p.c()
    _check(lib().otm_sgd_score(ctypes.byref(cp), n, _ptr(YA), _ptr(YB), _ptr(YC), _ptr(ybar3), _ptr(Phi), restarts,
                               _ptr(score), _ptr(ws), ws.numel(), _stream(stream)))
    return score


@dataclass
class Problem:
    """One decomposition of a batched run: FP32 whitened views (n x ldy; the
    three may be the same tensor), global means (3 x k), initial factors
    (restarts x k x k) and optional permutations (int32, restarts x passes x n,
    or passes x n shared by every restart)."""
    YA: torch.Tensor
    YB: torch.Tensor
    YC: torch.Tensor
    ybar3: torch.Tensor
    Phi0: torch.Tensor
    k: int
    alpha0: float
    perms: torch.Tensor | None = None


class BatchedRun:
    """A planned batched STGD run: results Phi[i] (restarts x k x k), scores[i]
    (restarts) per problem and best (the lowest-score restart per problem).
    run() enqueues it; capture() turns it into a replayable graph."""

    def __init__(self, problems: list[Problem], restarts: int, p: SgdParams, tune_cache: str | None = None):
        dev = problems[0].Phi0.device
        self.device = dev
        self.problems = problems
        self.restarts = restarts
        self.Phi = [torch.empty(P.Phi0.shape, dtype=torch.float32, device=dev) for P in problems]
        self.scores = [torch.empty(restarts, dtype=torch.float64, device=dev) for _ in problems]
        self.best = torch.empty(len(problems), dtype=torch.int32, device=dev)
        self.nonfinite = torch.zeros(1, dtype=torch.int32, device=dev)
        arr = (_Problem * len(problems))()
        for i, P in enumerate(problems):
            n, ldy = P.YA.shape
            for t in (P.YA, P.YB, P.YC):
                if t.dtype != torch.float32 or t.shape != (n, ldy):
                    raise OtmError(-3, "batched views must be FP32 tensors of one shape")
            if P.Phi0.shape != (restarts, P.k, P.k):
                raise OtmError(-2, "Phi0 must be restarts x k x k")
            # perms: restarts x passes x n (one order per run) or passes x n (shared)
            stride = 0 if P.perms is None or P.perms.dim() == 2 else P.perms[0].numel()
            check_perms(P.perms, n, p.passes, restarts, stride)
            arr[i] = _Problem(_ptr(P.YA), _ptr(P.YB), _ptr(P.YC), _ptr(P.ybar3), _ptr(P.perms), stride,
                              _ptr(P.Phi0), _ptr(self.Phi[i]), _ptr(self.scores[i]), n, P.k, ldy, 0,
                              float(P.alpha0))
        cp = p.c()
        plan = _vp()
        _check(lib().otm_sgd_batched_plan(arr, len(problems), restarts, ctypes.byref(cp),
                                          tune_cache.encode() if tune_cache else None, _ptr(self.best),
                                          _ptr(self.nonfinite), ctypes.byref(plan)))
        self._plan = plan
        nbytes = lib().otm_plan_size(plan)
        image = ctypes.string_at(lib().otm_plan_image(plan), nbytes)
        self.groups = lib().otm_plan_groups(plan)
        self.image = torch.frombuffer(bytearray(image), dtype=torch.uint8).to(dev)
        self.ws = _ws(lib().otm_sgd_batched_workspace(plan), dev)
        self._graph = None

    def run(self, stream=None):
        _check(lib().otm_sgd_batched(self._plan, _ptr(self.image), _ptr(self.ws), self.ws.numel(), _stream(stream)))

    def capture(self, stream: torch.cuda.Stream):
        """Captures the launch sequence into a graph on `stream` (not the null stream)."""
        g = _vp()
        _check(lib().otm_sgd_batched_graph(self._plan, _ptr(self.image), _ptr(self.ws), self.ws.numel(),
                                           _stream(stream), ctypes.byref(g)))
        self._graph = g

    def replay(self, stream=None):
        if self._graph is None:
            raise OtmError(-1, "no graph captured")
        _check(lib().otm_graph_launch(self._graph, _stream(stream)))

    def close(self):
        if self._graph is not None:
            _check(lib().otm_graph_destroy(self._graph))
            self._graph = None
        if getattr(self, "_plan", None) is not None:
            lib().otm_plan_free(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def sgd_autotune(ks, batch: int, cache_path: str, stream=None):
    """Times the batched kernel's tile layouts for each padded k of ks and
    records the fastest in cache_path."""
    arr = (_i32 * len(ks))(*[int(k) for k in ks])
    _check(lib().otm_sgd_autotune(arr, len(ks), batch, cache_path.encode(), _stream(stream)))


# ------------------------------------------------------------------ a6
def unwhiten_topics(W: torch.Tensor, Phi: torch.Tensor, theta: float = 1.0, stream=None,
                    info: torch.Tensor | None = None):
    _need(W, "W", torch.float64, (None, None))
    d, k = W.shape
    _need_numel(Phi, "Phi", torch.float32, k * k)
    mu = torch.empty((d, k), dtype=torch.float64, device=W.device)
    ah = torch.empty(k, dtype=torch.float64, device=W.device)
    lam = torch.empty(k, dtype=torch.float64, device=W.device)
    info, deferred = _info_slot(info, W.device)
    ws = _ws(lib().otm_unwhiten_workspace(d, k), W.device)
    _check(lib().otm_unwhiten_topics(_ptr(W), d, k, _ptr(Phi), float(theta), _ptr(mu), _ptr(ah), _ptr(lam),
                                     _ptr(info), _ptr(ws), ws.numel(), _stream(stream)))
    if not deferred and int(info.item()) != 0:
        _raise_info("unwhiten_topics")
    return mu, ah, lam


def recover_pi(Y: torch.Tensor, k: int, Phi: torch.Tensor, theta: float = 1.0, tau: float = 0.0, stream=None):
    if Y.dtype not in (torch.float32, torch.bfloat16) or Y.dim() != 2 or Y.shape[1] < k:
        raise OtmError(-3, "Y must be n x ldy (ldy >= k) in FP32 or BF16")
    _need_numel(Phi, "Phi", torch.float32, k * k)
    n, ldy = Y.shape
    Pi = torch.empty((k, n), dtype=torch.float32, device=Y.device)
    ws = _ws(lib().otm_recover_pi_workspace(k), Y.device)
    _check(lib().otm_recover_pi(_ptr(Y), _DTYPE_CODE[Y.dtype], ldy, n, k, _ptr(Phi), float(theta), float(tau),
                                _ptr(Pi), _ptr(ws), ws.numel(), _stream(stream)))
    return Pi


# ------------------------------------------------------------------ validation
@dataclass
class Validation:
    rho: torch.Tensor
    p: torch.Tensor
    p_adj: torch.Tensor
    edges: torch.Tensor
    l1: torch.Tensor
    scores: torch.Tensor        # [recovery ratio, error]


def validate(Pi_hat: torch.Tensor, Pi: torch.Tensor, threshold: float = 0.01, stream=None) -> Validation:
    """p-value matching of estimated to true communities and the recovery
    ratio / error (FP32 k_hat x n and k x n inputs, FP64 results)."""
    kh, n = Pi_hat.shape
    k = Pi.shape[0]
    if Pi.shape[1] != n or Pi_hat.dtype != torch.float32 or Pi.dtype != torch.float32:
        raise OtmError(-2, "Pi_hat and Pi must be FP32 with the same number of nodes")
    dev = Pi_hat.device
    out = [torch.empty((kh, k), dtype=torch.float64, device=dev) for _ in range(3)]
    edges = torch.empty((kh, k), dtype=torch.int32, device=dev)
    l1 = torch.empty((kh, k), dtype=torch.float64, device=dev)
    scores = torch.empty(2, dtype=torch.float64, device=dev)
    ws = _ws(lib().otm_validate_workspace(kh, k, n), dev)
    _check(lib().otm_validate(_ptr(Pi_hat), kh, _ptr(Pi), k, n, float(threshold), _ptr(out[0]), _ptr(out[1]),
                              _ptr(out[2]), _ptr(edges), _ptr(l1), _ptr(scores), _ptr(ws), ws.numel(),
                              _stream(stream)))
    return Validation(out[0], out[1], out[2], edges, l1, scores)


def bridgeness(Pi_hat: torch.Tensor, G: DeviceCSR | None = None, stream=None):
    """(b, b_degree or None) per node."""
    _need(Pi_hat, "Pi_hat", torch.float32, (None, None))
    kh, n = Pi_hat.shape
    b = torch.empty(n, dtype=torch.float64, device=Pi_hat.device)
    bd = torch.empty(n, dtype=torch.float64, device=Pi_hat.device) if G is not None else None
    gc = G.c() if G is not None else None
    _check(lib().otm_bridgeness(_ptr(Pi_hat), kh, n, ctypes.byref(gc) if gc is not None else None, _ptr(b), _ptr(bd),
                                _stream(stream)))
    return b, bd


# ------------------------------------------------------------------ measurement probes
def probe_copy(src: torch.Tensor, dst: torch.Tensor, blocks: int, stream=None):
    _check(lib().otm_probe_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), int(blocks), _stream(stream)))


def probe_mfma(dtype: int, iters: int, blocks: int, out: torch.Tensor, stream=None) -> int:
    """Launches the matrix-core probe; returns its flops."""
    _check(lib().otm_probe_mfma(int(dtype), int(iters), int(blocks), _ptr(out), _stream(stream)))
    return int(lib().otm_probe_mfma_flops(int(dtype), int(iters), int(blocks)))


# ------------------------------------------------------------------ loss
def tensor_form(YA, YB, YC, k: int, ybar3: torch.Tensor, alpha0: float, stream=None):
    if YA.dtype not in (torch.float32, torch.bfloat16) or YA.dim() != 2 or YA.shape[1] < k:
        raise OtmError(-3, "YA must be n x ldy (ldy >= k) in FP32 or BF16")
    _need(YB, "YB", YA.dtype, tuple(YA.shape))
    _need(YC, "YC", YA.dtype, tuple(YA.shape))
    _need_numel(ybar3, "ybar3", torch.float32, 3 * k)
    n, ldy = YA.shape
    T = torch.empty((k, k, k), dtype=torch.float64, device=YA.device)
    _check(lib().otm_tensor_form(_ptr(YA), _ptr(YB), _ptr(YC), _DTYPE_CODE[YA.dtype], ldy, n, k, _ptr(ybar3),
                                 float(alpha0), _ptr(T), _stream(stream)))
    return T


def residual(T: torch.Tensor, Phis: torch.Tensor, stream=None):
    k = T.shape[0]
    _need(T, "T", torch.float64, (k, k, k))
    if Phis.dtype != torch.float32 or Phis.numel() % (k * k) != 0:
        raise OtmError(-3, "Phis must be FP32 with a multiple of k x k values")
    Phis = Phis.reshape(-1, k, k)
    cnt = Phis.shape[0]
    R = torch.empty(cnt, dtype=torch.float64, device=T.device)
    ws = _ws(lib().otm_residual_workspace(k, cnt), T.device)
    _check(lib().otm_residual(_ptr(T), k, _ptr(Phis), cnt, _ptr(R), _ptr(ws), ws.numel(), _stream(stream)))
    return R


# ------------------------------------------------------------------ warm start
def ws_dims() -> dict:
    v = [_i32() for _ in range(4)]
    npar = _i64()
    _check(lib().otm_ws_dims(*[ctypes.byref(x) for x in v], ctypes.byref(npar)))
    return {"n_in": v[0].value, "hidden": v[1].value, "n_out": v[2].value, "P": v[3].value, "n_params": npar.value}


def ws_sketch(YA, YB, YC, k: int, ybar3: torch.Tensor, alpha0: float, Theta: torch.Tensor, S: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
    """S_r = T(I, I, theta_r), r = 0..3 (4 x lds x lds FP32; lds = S.shape[-1])."""
    if YA.dtype not in (torch.float32, torch.bfloat16) or YA.dim() != 2 or YA.shape[1] < k:
        raise OtmError(-3, "YA must be n x ldy (ldy >= k) in FP32 or BF16")
    _need(YB, "YB", YA.dtype, tuple(YA.shape))
    _need(YC, "YC", YA.dtype, tuple(YA.shape))
    _need_numel(ybar3, "ybar3", torch.float32, 3 * k)
    _need_numel(Theta, "Theta", torch.float32, 4 * k)
    if S is not None and (S.dtype != torch.float32 or S.dim() != 3 or S.shape[0] != 4 or S.shape[1] != S.shape[2]
                          or S.shape[2] < k):
        raise OtmError(-2, "S must be 4 x lds x lds FP32 with lds >= k")
    n, ldy = YA.shape
    if S is None:
        S = torch.zeros((4, k, k), dtype=torch.float32, device=YA.device)
    lds = S.shape[-1]
    ws = _ws(lib().otm_ws_sketch_workspace(n, k), YA.device)
    _check(lib().otm_ws_sketch(_ptr(YA), _ptr(YB), _ptr(YC), _DTYPE_CODE[YA.dtype], ldy, n, k, _ptr(ybar3),
                               float(alpha0), _ptr(Theta), _ptr(S), lds, _ptr(ws), ws.numel(), _stream(stream)))
    return S


def ws_frames(ks: torch.Tensor, S: torch.Tensor, Theta: torch.Tensor, stream=None):
    """Canonical frames and network inputs: returns (Q, sigma, X, info)."""
    d = ws_dims()
    cnt = ks.numel()
    _need_numel(ks, "ks", torch.int32, cnt)
    _need_numel(S, "S", torch.float32, cnt * 4 * d["P"] * d["P"])
    _need_numel(Theta, "Theta", torch.float32, cnt * d["P"] * 4)
    dev = S.device
    Q = torch.empty((cnt, d["P"], d["P"]), dtype=torch.float32, device=dev)
    sig = torch.empty(cnt, dtype=torch.float32, device=dev)
    X = torch.empty((cnt, d["n_in"]), dtype=torch.float32, device=dev)
    info = torch.empty(cnt, dtype=torch.int32, device=dev)
    ws = _ws(lib().otm_ws_frames_workspace(cnt), dev)
    _check(lib().otm_ws_frames(cnt, _ptr(ks), _ptr(S), _ptr(Theta), _ptr(Q), _ptr(sig), _ptr(X), _ptr(info), _ptr(ws),
                               ws.numel(), _stream(stream)))
    return Q, sig, X, info


def ws_target(ks, Q, sigma, U, lam, stream=None) -> torch.Tensor:
    cnt = ks.numel()
    P = ws_dims()["P"]
    _need_numel(ks, "ks", torch.int32, cnt)
    _need_numel(Q, "Q", torch.float32, cnt * P * P)
    _need_numel(sigma, "sigma", torch.float32, cnt)
    _need_numel(U, "U", torch.float32, cnt * P * P)
    _need_numel(lam, "lam", torch.float32, cnt * P)
    tgt = torch.empty((cnt, P * P), dtype=torch.float32, device=Q.device)
    _check(lib().otm_ws_target(cnt, _ptr(ks), _ptr(Q), _ptr(sigma), _ptr(U), _ptr(lam), _ptr(tgt), _stream(stream)))
    return tgt


def _need_mlp(d, params, X):
    _need_numel(params, "params", torch.float32, d["n_params"])
    _need(X, "X", torch.float32, (None, d["n_in"]))


def mlp_forward(params, X, stream=None):
    d = ws_dims()
    _need_mlp(d, params, X)
    B = X.shape[0]
    H = torch.empty((B, d["hidden"]), dtype=torch.float32, device=X.device)
    out = torch.empty((B, d["n_out"]), dtype=torch.float32, device=X.device)
    ws = _ws(lib().otm_mlp_workspace(B), X.device)
    _check(lib().otm_mlp_forward(_ptr(params), B, _ptr(X), _ptr(H), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return H, out


def mlp_backward(params, X, H, dout, grads=None, stream=None):
    d = ws_dims()
    _need_mlp(d, params, X)
    B = X.shape[0]
    _need(H, "H", torch.float32, (B, d["hidden"]))
    _need(dout, "dout", torch.float32, (B, d["n_out"]))
    if grads is not None:
        _need_numel(grads, "grads", torch.float32, d["n_params"])
    if grads is None:
        grads = torch.empty_like(params)
    ws = _ws(lib().otm_mlp_workspace(B), X.device)
    _check(lib().otm_mlp_backward(_ptr(params), B, _ptr(X), _ptr(H), _ptr(dout), _ptr(grads), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return grads


def mlp_adam(params, grads, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    npar = ws_dims()["n_params"]
    for name, t_ in (("params", params), ("grads", grads), ("m", m), ("v", v)):
        _need_numel(t_, name, torch.float32, npar)
    _check(lib().otm_mlp_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(t), float(lr), float(beta1),
                              float(beta2), float(eps), _stream(stream)))


def mlp_to_bf16(params, stream=None) -> torch.Tensor:
    _need_numel(params, "params", torch.float32, ws_dims()["n_params"])
    pb = torch.empty(params.numel(), dtype=torch.bfloat16, device=params.device)
    _check(lib().otm_mlp_to_bf16(_ptr(params), _ptr(pb), _stream(stream)))
    return pb


def mlp_forward_bf16(params_bf16, params, X, stream=None) -> torch.Tensor:
    d = ws_dims()
    _need_mlp(d, params, X)
    _need_numel(params_bf16, "params_bf16", torch.bfloat16, d["n_params"])
    B = X.shape[0]
    out = torch.empty((B, d["n_out"]), dtype=torch.float32, device=X.device)
    ws = _ws(lib().otm_mlp_bf16_workspace(B), X.device)
    _check(lib().otm_mlp_forward_bf16(_ptr(params_bf16), _ptr(params), B, _ptr(X), _ptr(out), _ptr(ws), ws.numel(),
                                      _stream(stream)))
    return out


def ws_mse(ks, live: int, out, target, stream=None):
    cnt = ks.numel()
    n_out = ws_dims()["n_out"]
    _need_numel(ks, "ks", torch.int32, cnt)
    _need_numel(out, "out", torch.float32, cnt * n_out)
    _need_numel(target, "target", torch.float32, cnt * n_out)
    loss = torch.empty(1, dtype=torch.float64, device=out.device)
    dout = torch.empty_like(out)
    ws = _ws(lib().otm_ws_mse_workspace(cnt), out.device)
    _check(lib().otm_ws_mse(cnt, _ptr(ks), int(live), _ptr(out), _ptr(target), _ptr(loss), _ptr(dout), _ptr(ws),
                            ws.numel(), _stream(stream)))
    return loss, dout


def ws_factors(ks, out, Q, sigma, stream=None) -> torch.Tensor:
    cnt = ks.numel()
    d = ws_dims()
    P = d["P"]
    _need_numel(ks, "ks", torch.int32, cnt)
    _need_numel(out, "out", torch.float32, cnt * d["n_out"])
    _need_numel(Q, "Q", torch.float32, cnt * P * P)
    _need_numel(sigma, "sigma", torch.float32, cnt)
    Phi = torch.zeros((cnt, P * P), dtype=torch.float32, device=out.device)
    _check(lib().otm_ws_factors(cnt, _ptr(ks), _ptr(out), _ptr(Q), _ptr(sigma), _ptr(Phi), _stream(stream)))
    return Phi
