"""GPU parity of the whitening SpMM (Section 3.1 whitened data) against the
FP64 oracle, on the same rounded W.

Bars: FP32 Y within 2e-6 relative per row (FP32 accumulation of <= a few
hundred terms); BF16 Y within 2^-8 relative per entry of the row scale plus
the FP32 bar; ybar within 1e-6 relative (FP64 reduction of FP32 rows)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import bf16_round, csr_dev, dev, f32_round, host, to_dev

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu


def _check_rows(Yg, Yref, k, tol_rel):
    Yg = Yg[:, :k]
    scale = np.maximum(np.abs(Yref).max(axis=1, keepdims=True), 1e-30)
    err = np.abs(Yg - Yref) / scale
    assert err.max() <= tol_rel, (err.max(), np.unravel_index(err.argmax(), err.shape))


@pytest.mark.parametrize("k", [3, 10, 16, 50, 100, 128])
@pytest.mark.parametrize("w_dt,y_dt", [(otm.F32, otm.F32), (otm.BF16, otm.BF16), (otm.BF16, otm.F32),
                                       (otm.F32, otm.BF16)])
def test_whiten_graph_rows(k, w_dt, y_dt):
    g = synth.mmsb(n=1300, k=4, alpha0=0.3, p=0.2, q=0.02, n_x=700, seed=k)
    W = synth.projection(g.C.n_cols, k, seed=3)
    Wr = bf16_round(W) if w_dt == otm.BF16 else f32_round(W)
    Wd = to_dev(Wr, torch.bfloat16 if w_dt == otm.BF16 else torch.float32)
    Y, ybar = otm.whiten(csr_dev(g.C), False, Wd, y_dtype=y_dt)
    torch.cuda.synchronize()
    Yref, ybref = oracle.whiten(g.C, Wr, normalize=False)
    Yg = host(Y)
    tol = 2e-6 if y_dt == otm.F32 else 2.0 ** -8
    _check_rows(Yg, Yref, k, tol)
    assert np.all(Yg[:, k:] == 0.0)
    np.testing.assert_allclose(host(ybar), ybref, rtol=0, atol=1e-6 * np.abs(ybref).max())


@pytest.mark.parametrize("k", [7, 50, 64])
def test_whiten_document_views_normalised(k):
    inst = synth.lda(d=3000, k=5, alpha0=1.0, beta=0.1, n_docs=2051, mean_len=40.0, seed=k)
    W = f32_round(synth.projection(3000, k, seed=5))
    for v in inst.views:
        Y, ybar = otm.whiten(csr_dev(v), True, to_dev(W), y_dtype=otm.F32)
        torch.cuda.synchronize()
        Yref, ybref = oracle.whiten(v, W, normalize=True)
        _check_rows(host(Y), Yref, k, 2e-6)
        np.testing.assert_allclose(host(ybar), ybref, rtol=0, atol=1e-6 * np.abs(ybref).max())


@pytest.mark.parametrize("k", [3, 10, 50, 100, 129, 200])
@pytest.mark.parametrize("w_dt,y_dt", [(otm.F32, otm.F32), (otm.BF16, otm.BF16), (otm.BF16, otm.F32)])
def test_whiten_padded_row_stride(k, w_dt, y_dt):
    """W as the d x k slice of a row-padded buffer whose padding holds NaN (the
    16-byte vector gathers read it; it must not reach Y or ybar), and as a
    slice that starts one column in (unaligned: narrower gathers)."""
    g = synth.mmsb(n=1500, k=4, alpha0=0.3, p=0.2, q=0.02, n_x=900, seed=k + 1)
    W = synth.projection(g.C.n_cols, k, seed=4)
    Wr = bf16_round(W) if w_dt == otm.BF16 else f32_round(W)
    tdt = torch.bfloat16 if w_dt == otm.BF16 else torch.float32
    ldw = otm.default_ldw(k, w_dt)
    for off, ld in ((0, ldw), (1, ldw + 8)):
        buf = torch.full((g.C.n_cols, ld), float("nan"), dtype=tdt, device=dev())
        buf[:, off:off + k] = to_dev(Wr, tdt)
        if off and k > 64:                          # one element per lane: k <= 64
            with pytest.raises(otm.OtmError) as e:
                otm.whiten(csr_dev(g.C), False, buf[:, off:off + k], y_dtype=y_dt)
            assert e.value.status == -8
            continue
        Y, ybar = otm.whiten(csr_dev(g.C), False, buf[:, off:off + k], y_dtype=y_dt)
        torch.cuda.synchronize()
        Yref, ybref = oracle.whiten(g.C, Wr, normalize=False)
        Yg = host(Y)
        _check_rows(Yg, Yref, k, 2e-6 if y_dt == otm.F32 else 2.0 ** -8)
        assert np.all(Yg[:, k:] == 0.0)
        np.testing.assert_allclose(host(ybar), ybref, rtol=0, atol=1e-6 * np.abs(ybref).max())


def test_whiten_into_given_output_uses_its_row_stride():
    """An output buffer wider than the default row stride: the rows land at
    its own stride with zero padding; a buffer of the wrong dtype or row
    count is refused before any launch."""
    g = synth.mmsb(n=800, k=4, alpha0=0.3, p=0.2, q=0.02, n_x=500, seed=3)
    k = 20
    W = f32_round(synth.projection(g.C.n_cols, k, seed=8))
    Cd = csr_dev(g.C)
    out = torch.full((g.C.n_rows, 40), float("nan"), dtype=torch.float32, device=dev())
    Y, _ = otm.whiten(Cd, False, to_dev(W), y_dtype=otm.F32, out=out)
    torch.cuda.synchronize()
    assert Y.data_ptr() == out.data_ptr()
    Yref, _ = oracle.whiten(g.C, W, normalize=False)
    Yg = host(Y)
    _check_rows(Yg, Yref, k, 2e-6)
    assert np.all(Yg[:, k:] == 0.0)
    with pytest.raises(ValueError):
        otm.whiten(Cd, False, to_dev(W), y_dtype=otm.BF16, out=out)
    with pytest.raises(ValueError):
        otm.whiten(Cd, False, to_dev(W), y_dtype=otm.F32, out=out[:-1])
    with pytest.raises(ValueError):
        otm.whiten(Cd, False, to_dev(W), y_dtype=otm.F32, ldy=24, out=out)


def test_whiten_document_views_padded_stride():
    """The document-workload shape (k = 50 FP32, W padded to 52 columns)."""
    inst = synth.lda(d=3000, k=5, alpha0=1.0, beta=0.1, n_docs=3001, mean_len=60.0, seed=11)
    k = 50
    W = f32_round(synth.projection(3000, k, seed=6))
    buf = torch.full((3000, otm.default_ldw(k, otm.F32)), float("nan"), dtype=torch.float32, device=dev())
    buf[:, :k] = to_dev(W)
    for v in inst.views:
        Y, ybar = otm.whiten(csr_dev(v), True, buf[:, :k], y_dtype=otm.F32)
        torch.cuda.synchronize()
        Yref, ybref = oracle.whiten(v, W, normalize=True)
        _check_rows(host(Y), Yref, k, 2e-6)
        np.testing.assert_allclose(host(ybar), ybref, rtol=0, atol=1e-6 * np.abs(ybref).max())


@pytest.mark.parametrize("k", [50, 100])
@pytest.mark.parametrize("w_dt,y_dt", [(otm.F32, otm.F32), (otm.BF16, otm.BF16), (otm.BF16, otm.F32)])
def test_whiten_w_in_lds(k, w_dt, y_dt):
    """A small W (300 rows) gathered by many stored entries (over 512 per
    column, rows of 80 entries on average) is copied into LDS once per
    workgroup; the rows equal the oracle's and, bit for bit, those of the
    kernel that gathers W from global memory (forced by a row stride that
    allows only narrow vectors).  Row lengths are ragged, some rows empty, and
    the row count is not a multiple of the rows a workgroup takes."""
    rng = np.random.default_rng(k)
    d, n = 300, 6001
    lens = rng.integers(48, 113, n)
    lens[rng.choice(n, 20, replace=False)] = 0
    cols = [np.sort(rng.choice(d, int(m), replace=False)) for m in lens]
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    colidx = np.concatenate(cols).astype(np.int32)
    vals = rng.integers(1, 5, colidx.size).astype(np.float32)
    assert colidx.size >= 512 * d and colidx.size >= 64 * n
    C = synth.CSR(n, d, rowptr, colidx, vals)
    W = synth.projection(d, k, seed=12)
    Wr = bf16_round(W) if w_dt == otm.BF16 else f32_round(W)
    tdt = torch.bfloat16 if w_dt == otm.BF16 else torch.float32
    Cd = csr_dev(C)
    fast = torch.zeros((d, otm.default_ldw(k, w_dt)), dtype=tdt, device=dev())
    fast[:, :k] = to_dev(Wr, tdt)
    slow = torch.zeros((d, k + 1 if k % 2 else k + 2), dtype=tdt, device=dev())   # narrow vectors, 64 lanes
    slow[:, :k] = to_dev(Wr, tdt)
    for norm in (False, True):
        Y, ybar = otm.whiten(Cd, norm, fast[:, :k], y_dtype=y_dt)
        Y2, ybar2 = otm.whiten(Cd, norm, slow[:, :k], y_dtype=y_dt)
        torch.cuda.synchronize()
        Yref, ybref = oracle.whiten(C, Wr, normalize=False)
        if norm:     # an empty row has no token count: the kernel writes zeros there
            Yref = np.where(lens[:, None] > 0, Yref / np.asarray(C.to_scipy().sum(1)).clip(1e-30), 0.0)
            ybref = Yref.mean(0)
        _check_rows(host(Y), Yref, k, 2e-6 if y_dt == otm.F32 else 2.0 ** -8)
        assert torch.equal(Y, Y2)
        np.testing.assert_allclose(host(ybar), ybref, rtol=0, atol=1e-6 * np.abs(ybref).max())
        np.testing.assert_allclose(host(ybar), host(ybar2), rtol=0, atol=1e-6 * np.abs(ybref).max())


def test_whiten_empty_rows_and_empty_matrix():
    # rows 0, 3 and the last are empty
    rowptr = np.array([0, 0, 2, 3, 3, 5, 5], dtype=np.int32)
    colidx = np.array([1, 4, 0, 2, 3], dtype=np.int32)
    C = synth.CSR(6, 5, rowptr, colidx, np.array([1, 2, 3, 4, 5], dtype=np.float32))
    W = f32_round(synth.projection(5, 6, seed=1))
    for norm in (False, True):
        Y, ybar = otm.whiten(csr_dev(C), norm, to_dev(W), y_dtype=otm.F32)
        torch.cuda.synchronize()
        Yref, ybref = oracle.whiten(C, W, normalize=False)
        if norm:
            rs = np.asarray(C.to_scipy().sum(1)).ravel()
            Yref = np.where(rs[:, None] > 0, Yref / np.where(rs > 0, rs, 1)[:, None], 0.0)
            ybref = Yref.mean(0)
        np.testing.assert_allclose(host(Y)[:, :6], Yref, atol=1e-6)
        np.testing.assert_allclose(host(ybar), ybref, atol=1e-6)
    E = synth.CSR(0, 5, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32), None)
    Y, ybar = otm.whiten(csr_dev(E), False, to_dev(W), y_dtype=otm.F32)
    torch.cuda.synchronize()
    assert Y.shape[0] == 0 and np.all(host(ybar) == 0)


def test_whiten_skips_out_of_range_columns_and_check_reports_them():
    rowptr = np.array([0, 2, 4], dtype=np.int32)
    colidx = np.array([0, 9, -3, 1], dtype=np.int32)     # 9 and -3 are outside [0, 3)
    C = synth.CSR(2, 3, rowptr, colidx, None)
    W = f32_round(synth.projection(3, 4, seed=2))
    Cd = csr_dev(C)
    assert otm.csr_check(Cd) == 2
    Y, _ = otm.whiten(Cd, False, to_dev(W), y_dtype=otm.F32)
    torch.cuda.synchronize()
    np.testing.assert_allclose(host(Y)[:, :4], np.stack([W[0], W[1]]), atol=1e-7)
    good = csr_dev(synth.mmsb(n=100, k=2, alpha0=0.3, p=0.3, q=0.1, seed=1).C)
    assert otm.csr_check(good) == 0


def test_whiten_rejects_bad_arguments():
    C = csr_dev(synth.CSR(2, 3, np.array([0, 1, 2], dtype=np.int32), np.array([0, 1], dtype=np.int32), None))
    W = to_dev(np.ones((3, 4)))
    with pytest.raises(otm.OtmError) as e:
        otm.whiten(C, False, W, y_dtype=otm.BF16, ldy=4)           # BF16 needs ldy % 8 == 0
    assert e.value.status == -2
    with pytest.raises(otm.OtmError):
        otm.whiten(C, False, to_dev(np.ones((3, 4)), torch.float64), y_dtype=otm.F32)   # FP64 W
