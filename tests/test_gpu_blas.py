"""The library's bandwidth reference kernels (used by the benchmark for its
ceilings), checked for what they move."""

import pytest
import torch

from paper_1904_08616_amd import dirac as D

pytestmark = pytest.mark.gpu


def test_bandwidth_probe_moves_what_it_says():
    n = (1 << 20) + 48  # not a multiple of the grid's stride
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    D.bandwidth_probe("copy", src, dst, n)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    D.bandwidth_probe("write", None, dst, n)
    torch.cuda.synchronize()
    pattern = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").view(torch.uint8).repeat(n // 16)
    assert torch.equal(dst, pattern)
    before = dst.clone()
    D.bandwidth_probe("read", src, dst, n)  # dst is only a sink
    torch.cuda.synchronize()
    assert torch.equal(dst, before)
