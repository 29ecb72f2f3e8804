"""The STREAM copy probe (the attainable-bandwidth reference of the bench)
copies bitwise, including a ragged tail shorter than one workgroup."""
import pytest
import torch

import paper_0910_3915_amd as scd
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 255, 256 * 65536 + 77])
def test_stream_copy_is_bitwise(n):
    announce(f"stream copy: {n} doubles")
    g = torch.Generator(device="cpu").manual_seed(n)
    src = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    dst = torch.full_like(src, float("nan"))
    s = torch.cuda.Stream()
    scd.stream_copy(src, dst, s)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
