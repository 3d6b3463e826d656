"""The measurement probes: the copy probe copies (every byte equal), the
matrix-core probe runs to completion with finite sums, and its flop count
follows the instruction shapes (2 m n k per instruction, eight chains per
wave, four waves per workgroup)."""
import pytest
import torch

from paper_1309_0787_amd import otm

pytestmark = pytest.mark.gpu


def test_probe_copy_copies():
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    otm.probe_copy(src, dst, 64)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    with pytest.raises(otm.OtmError):
        otm.probe_copy(src[1:], dst[1:], 64)          # not 16-byte aligned


@pytest.mark.parametrize("dtype,shape", [(otm.BF16, 16 * 16 * 32), (otm.F32, 16 * 16 * 4), (otm.F64, 16 * 16 * 4)])
def test_probe_mfma_runs_and_counts(dtype, shape):
    blocks, iters = 8, 10
    out = torch.full((blocks * 256,), float("nan"), device="cuda")
    flops = otm.probe_mfma(dtype, iters, blocks, out)
    torch.cuda.synchronize()
    assert flops == 2 * shape * 8 * iters * blocks * 4
    assert torch.isfinite(out).all()
