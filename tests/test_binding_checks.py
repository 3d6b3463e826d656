"""Host-side argument checks of the binding that keep the kernels' reads in
bounds (no GPU needed): the permutation buffer of an STGD run must be int32,
contiguous and hold (restarts - 1) * perm_stride + passes * n entries."""
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
