"""The whitening entry point that allocates nothing (otm_whiten_noalloc),
called through the C ABI, against otm_whiten on the same inputs: the same
kernels write Y and ybar, so both must be bit-identical; two calls in a row
with the second on a smaller input (the shared scratch array keeps the first
call's partial sums, which the second must not see); a size whose partial
sums exceed the array is refused on the host with OTM_EWORKSPACE."""
import numpy as np
import pytest
import torch

import synth

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu


def _inputs(n_docs, d, k, seed, w_dtype):
    dev = torch.device("cuda:0")
    inst = synth.lda(d=d, k=3, alpha0=1.0, beta=0.1, n_docs=n_docs, mean_len=40.0, seed=seed)
    C = otm.DeviceCSR.from_host(inst.views[seed % 3], dev)
    ldw = otm.default_ldw(k, w_dtype)
    Wb = torch.zeros((d, ldw), dtype=torch.float32)
    Wb[:, :k] = torch.as_tensor(np.random.default_rng(seed).standard_normal((d, k)), dtype=torch.float32)
    W = Wb.to(device=dev, dtype=otm._TORCH_DTYPE[w_dtype])[:, :k]
    return C, W


@pytest.mark.parametrize("w_dtype,y_dtype", [(otm.F32, otm.F32), (otm.BF16, otm.BF16), (otm.F32, otm.BF16)])
def test_noalloc_equals_whiten_on_two_calls(w_dtype, y_dtype):
    print(f"whiten_noalloc w={w_dtype} y={y_dtype}", flush=True)
    for n_docs, d, k, seed in ((40000, 3000, 50, 1), (777, 500, 17, 2)):   # second call smaller
        C, W = _inputs(n_docs, d, k, seed, w_dtype)
        Y_ref, yb_ref = otm.whiten(C, True, W, y_dtype=y_dtype)
        Y = torch.full_like(Y_ref, float("nan"))
        yb = torch.full_like(yb_ref, float("nan"))
        otm.whiten_noalloc(C, True, W, Y, yb, y_dtype=y_dtype)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_ref), (n_docs, k)
        assert torch.equal(yb, yb_ref), (n_docs, k)


def test_noalloc_without_ybar_and_empty_input():
    C, W = _inputs(500, 400, 9, 3, otm.F32)
    Y_ref, _ = otm.whiten(C, True, W, y_dtype=otm.F32)
    Y = torch.zeros_like(Y_ref)
    otm.whiten_noalloc(C, True, W, Y, None, y_dtype=otm.F32)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y_ref)
    empty = otm.DeviceCSR(0, 400, torch.zeros(1, dtype=torch.int32, device="cuda"),
                          torch.zeros(0, dtype=torch.int32, device="cuda"))
    yb = torch.full((9,), 7.0, device="cuda")
    otm.whiten_noalloc(empty, True, W, torch.empty((0, Y.shape[1]), device="cuda"), yb, y_dtype=otm.F32)
    torch.cuda.synchronize()
    assert torch.all(yb == 0)


def test_noalloc_refuses_partial_sums_beyond_the_array():
    cap = otm.lib().otm_whiten_noalloc_capacity()
    assert cap == 1 << 20
    C, W = _inputs(40000, 600, 400, 4, otm.BF16)   # 8192 blocks x 400 columns > 2^20
    Y = torch.empty((C.n_rows, otm.default_ldy(400)), dtype=torch.bfloat16, device="cuda")
    yb = torch.empty(400, dtype=torch.float32, device="cuda")
    with pytest.raises(otm.OtmError) as e:
        otm.whiten_noalloc(C, True, W, Y, yb, y_dtype=otm.BF16)
    assert e.value.status == -7
