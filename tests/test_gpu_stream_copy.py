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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pull_copy_is_the_streaming_step(dtype):
    """scd_pull_copy keeps the state and writes, at every fluid node of the
    other buffer, exactly the oracle's pull-streaming (periodic neighbours,
    bounce-back) of the same seeded populations: pure copies, so bit for
    bit."""
    import numpy as np
    import oracle as O
    import workloads as W
    announce(f"pull copy: 20x18x14 droplet box, seeded populations, {dtype}")
    c = W.droplet_case(20, 18, 14, 5.0, 0.12, 0.2, dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"])
    rng = np.random.default_rng(11)
    plain = rng.uniform(0.0, 0.1, size=(2, 19, 14, 18, 20)).astype(
        np.float64 if dtype == "f64" else np.float32)
    L.set_state(torch.from_numpy(plain).cuda())
    before = L.get_state(blocked=True).clone()
    L.pull_copy()
    torch.cuda.synchronize()
    assert torch.equal(L.get_state(blocked=True), before)
    other = L.pop[1] if torch.equal(L.pop[0], before) else L.pop[0]
    Lo = O.Lattice(W.params(20, 18, 14, 0.12), c["solid"])
    want = O.to_gpu_layout(Lo.stream(O.from_gpu_layout(plain.astype(np.float64))))
    got = L.unpack(other).cpu().double().numpy()
    fluid = c["solid"] == 0
    assert np.array_equal(got[:, :, fluid], want[:, :, fluid])
