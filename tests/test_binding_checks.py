"""Host-side argument checks of the binding that keep the kernels' reads in
bounds (no GPU needed): the permutation buffer of an STGD run must be int32,
contiguous and hold (restarts - 1) * perm_stride + passes * n entries; dense
operands must have the element type and shape the entry point reads."""
import pytest
import torch

from paper_1309_0787_amd import otm


def test_perms_buffer_size_type_and_layout():
    n, passes = 50, 3
    ok = torch.zeros(passes * n, dtype=torch.int32)
    otm.check_perms(ok, n, passes, 1, 0)
    otm.check_perms(None, n, passes, 4, 0)
    otm.check_perms(torch.zeros((2, passes, n), dtype=torch.int32), n, passes, 2, passes * n)
    otm.check_perms(ok, n, passes, 4, 0)                                 # shared by every restart
    with pytest.raises(otm.OtmError, match="entries"):
        otm.check_perms(ok[:-1], n, passes, 1, 0)
    with pytest.raises(otm.OtmError, match="entries"):
        otm.check_perms(torch.zeros((2, passes, n), dtype=torch.int32), n, passes, 3, passes * n)
    with pytest.raises(otm.OtmError, match="int32"):
        otm.check_perms(ok.to(torch.int64), n, passes, 1, 0)
    with pytest.raises(otm.OtmError, match="contiguous"):
        otm.check_perms(torch.zeros((passes, 2 * n), dtype=torch.int32)[:, ::2], n, passes, 1, 0)
    with pytest.raises(otm.OtmError, match="perm_stride"):
        otm.check_perms(ok, n, passes, 2, -1)


def test_info_slot_must_be_one_int32_on_the_gpu():
    with pytest.raises(otm.OtmError, match="info"):
        otm._info_slot(torch.zeros(2, dtype=torch.int32), "cpu")
    with pytest.raises(otm.OtmError, match="info"):
        otm._info_slot(torch.zeros(1, dtype=torch.int64), "cpu")


def test_deferred_info_raises_the_entry_points_error():
    otm.check_info(torch.zeros(3, dtype=torch.int32), ["m2_apply", "whitener", "unwhiten_topics"])
    with pytest.raises(otm.OtmNotPSD):
        otm.check_info(torch.tensor([0, 1], dtype=torch.int32), ["m2_apply", "whitener"])
    with pytest.raises(otm.OtmError, match="fewer than 2 tokens"):
        otm.check_info(torch.tensor([1, 1], dtype=torch.int32), ["m2_apply", "whitener"])


def _csr(n_rows, n_cols):
    import numpy as np
    import synth
    rp = np.arange(n_rows + 1, dtype=np.int32)
    ci = (np.arange(n_rows, dtype=np.int32) % n_cols).astype(np.int32)
    return synth.CSR(n_rows, n_cols, rp, ci, None)


def test_dense_operands_must_match_what_the_kernels_read():
    """Element type and shape of every dense operand are checked before the
    call, since the C ABI takes bare pointers (CPU tensors suffice: the checks
    come first)."""
    C = _csr(6, 4)
    Cd, CTd = otm.DeviceCSR.from_host(C, "cpu"), otm.DeviceCSR.from_host(C.transpose(), "cpu")
    with pytest.raises(otm.OtmError) as e:
        otm.m2_apply(Cd, CTd, False, 0.5, torch.zeros((4, 2), dtype=torch.float32))
    assert e.value.status == -3
    with pytest.raises(otm.OtmError) as e:
        otm.m2_apply(Cd, CTd, False, 0.5, torch.zeros((5, 2), dtype=torch.float64))
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.m2_apply(Cd, Cd, False, 0.5, torch.zeros((4, 2), dtype=torch.float64))   # not the transpose
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.whitener(torch.zeros((4, 2), dtype=torch.float64), torch.zeros((4, 3), dtype=torch.float64), 1)
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.orthonormalize(torch.zeros((4, 2), dtype=torch.float32))
    assert e.value.status == -3
    with pytest.raises(otm.OtmError) as e:
        otm.whiten(Cd, False, torch.zeros((5, 3), dtype=torch.float32))
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.pairs_apply(CTd, Cd, torch.zeros((3, 2), dtype=torch.float64))
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.pinv_factors(torch.zeros((5, 3), dtype=torch.float64), torch.zeros((4, 2), dtype=torch.float64),
                         torch.zeros((5, 3), dtype=torch.float64), 2)
    assert e.value.status == -2


def test_stgd_views_factors_and_means_are_checked():
    k, n = 6, 10
    ldy = otm.default_ldy(k)
    Y = torch.zeros((n, ldy), dtype=torch.float32)
    yb = torch.zeros((3, k), dtype=torch.float32)
    Phi = torch.zeros((1, k, k), dtype=torch.float32)
    p = otm.SgdParams(k=k, batch=4, passes=1)
    bad = [
        (dict(YA=torch.zeros((n, ldy + 2), dtype=torch.float32)), -2),     # row stride
        (dict(YA=torch.zeros((n - 1, ldy), dtype=torch.float32)), -2),     # too few rows
        (dict(YA=torch.zeros((n, ldy), dtype=torch.bfloat16)), -3),        # element type
        (dict(ybar3=torch.zeros((2, k), dtype=torch.float32)), -2),
        (dict(Phi=torch.zeros((2, k, k), dtype=torch.float32)), -2),       # restarts = 1
        (dict(Phi=torch.zeros((1, k, k), dtype=torch.float64)), -3),
    ]
    for over, status in bad:
        a = dict(YA=Y, YB=Y, YC=Y, ybar3=yb, Phi=Phi)
        a.update(over)
        with pytest.raises(otm.OtmError) as e:
            otm.sgd_run(p, n, a["YA"], a["YB"], a["YC"], a["ybar3"], None, a["Phi"])
        assert e.value.status == status, over


def test_warm_start_buffers_are_checked():
    d = otm.ws_dims()
    params = torch.zeros(d["n_params"], dtype=torch.float32)
    with pytest.raises(otm.OtmError) as e:
        otm.mlp_forward(params, torch.zeros((2, d["n_in"] - 1), dtype=torch.float32))
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.mlp_forward(params[:-1], torch.zeros((2, d["n_in"]), dtype=torch.float32))
    assert e.value.status == -2
    with pytest.raises(otm.OtmError) as e:
        otm.mlp_adam(params, params, params, params.double(), 1, 1e-3)
    assert e.value.status == -3
    ks = torch.tensor([4, 5], dtype=torch.int32)
    with pytest.raises(otm.OtmError) as e:
        otm.ws_frames(ks, torch.zeros((1, 4, d["P"], d["P"]), dtype=torch.float32),
                      torch.zeros((2, d["P"], 4), dtype=torch.float32))
    assert e.value.status == -2
