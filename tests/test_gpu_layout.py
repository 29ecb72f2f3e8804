"""The blocked population layout: scd_pop_pack places element (a, k, x, y, z)
where the header's formula says, scd_pop_unpack inverts it, and a state set
in the plain order comes back unchanged."""
import ctypes

import numpy as np
import pytest
import torch

import paper_0910_3915_amd as scd
from gpu_helpers import announce

B = scd.binding
pytestmark = pytest.mark.gpu


def blocked_index(nx, ny, nz):
    """Flat blocked offset of every plain element, shape (2, 19, nz, ny, nx),
    from the formula a sp + ((z pb + c // 32) 19 + k) 32 + c % 32."""
    pb = (nx * ny + 31) // 32
    sp = 19 * 32 * pb * nz
    a = np.arange(2).reshape(2, 1, 1, 1, 1)
    k = np.arange(19).reshape(1, 19, 1, 1, 1)
    z = np.arange(nz).reshape(1, 1, nz, 1, 1)
    c = (np.arange(ny).reshape(ny, 1) * nx + np.arange(nx).reshape(1, nx)).reshape(1, 1, 1, ny, nx)
    return a * sp + ((z * pb + c // 32) * 19 + k) * 32 + c % 32, 2 * sp


@pytest.mark.parametrize("dims", [(20, 18, 14), (7, 5, 3), (64, 2, 5)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pack_follows_the_formula_and_unpack_inverts_it(dims, dtype):
    import workloads as W
    nx, ny, nz = dims
    announce(f"pop pack/unpack: {dims} {dtype}")
    L = scd.Lattice(W.params(nx, ny, nz, 0.1, dtype=dtype), np.zeros((nz, ny, nx), np.uint8))
    idx, total = blocked_index(nx, ny, nz)
    assert L.pop_numel == total
    g = torch.Generator(device="cpu").manual_seed(nx * 1000 + ny * 10 + nz)
    plain = torch.randn((2, 19, nz, ny, nx), generator=g, dtype=L.dtype)
    blocked = L.pack(plain.cuda())
    torch.cuda.synchronize()
    got = blocked.cpu().numpy()
    assert np.array_equal(got[idx.reshape(-1)], plain.numpy().reshape(-1))
    back = L.unpack(blocked)
    torch.cuda.synchronize()
    assert torch.equal(back.cpu(), plain)
    # set_state / get_state in the plain order round-trip exactly
    L.set_state(plain.cuda(), 7)
    assert torch.equal(L.get_state().cpu(), plain)
    assert L.step_count == 7


def test_pack_rejects_overlap():
    import workloads as W
    announce("pop pack: overlapping buffers")
    L = scd.Lattice(W.params(8, 8, 4, 0.1), np.zeros((4, 8, 8), np.uint8))
    buf = torch.zeros(2 * L.pop_numel, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    q = ctypes.c_void_p(buf.data_ptr() + 8 * 64)
    assert B.lib().scd_pop_pack(L.h, p, q) == B.SCD_EINVAL
    assert B.lib().scd_pop_unpack(L.h, p, None) == B.SCD_EINVAL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_padding_slots_stay_zero(dtype):
    """On a box whose planes are not a whole number of blocks, the padding
    slots of the state the binding hands out are zero after stepping: the
    kernels write node slots only."""
    import workloads as W
    announce(f"pop padding after 10 steps: 20x18x14 droplet, {dtype}")
    c = W.droplet_case(20, 18, 14, 5.0, 0.12, 0.2, dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(10)
    idx, total = blocked_index(20, 18, 14)
    node = np.zeros(total, bool)
    node[idx.reshape(-1)] = True
    st = L.get_state(blocked=True).cpu().numpy()
    assert not node.all()
    assert np.all(st[~node] == 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_poisoned_padding_never_reaches_a_result(dtype):
    """NaN in every padding slot of the blocked state, and of lambda', on a
    box whose planes are not a whole number of blocks: three steps under
    every compiled variant, the observables, the contact angle and a reverse
    step give bit for bit what they give from clean padding (the kernels
    address node slots only)."""
    import workloads as W
    announce(f"poisoned padding: 20x18x16 droplet, every variant, {dtype}")
    c = W.droplet_case(20, 18, 16, 6.5, 0.12, 0.2, dtype=dtype, offset=4)
    idx, total = blocked_index(20, 18, 16)
    node = np.zeros(total, bool)
    node[idx.reshape(-1)] = True
    pad = torch.from_numpy(~node).cuda()
    out = {}
    for poison in (False, True):
        L = scd.Lattice(c["params"], c["solid"], adjoint=True)
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        st = L.get_state(blocked=True)
        if poison:
            st[pad] = float("nan")
        L.set_state(st, blocked=True)
        states = []
        for v in range(len(scd.tile_list())):
            L.set_tile(v, 4)
            L.step(3)
            states.append(L.get_state(blocked=True).cpu().numpy()[node])
        o = L.observables()
        ca = L.contact_angle(c["ca"])
        s2 = L.get_state(blocked=True)
        lam = L.ca_seed(c["ca"], 1.0, blocked=True)
        if poison:
            lam[pad] = float("nan")
        lo, dp = L.adjoint_step(s2, lam, blocked=True)
        out[poison] = (states, o, ca, lo.cpu().numpy()[node], dp)
    clean, dirty = out[False], out[True]
    for a, b in zip(clean[0], dirty[0]):
        assert np.array_equal(a, b)
    assert dirty[1]["finite"] and dirty[1]["mass"] == clean[1]["mass"]
    assert dirty[1]["momentum"] == clean[1]["momentum"]
    assert dirty[2]["theta_e1"] == clean[2]["theta_e1"] and dirty[2]["theta_e2"] == clean[2]["theta_e2"]
    assert np.array_equal(clean[3], dirty[3]) and np.all(np.isfinite(dirty[3]))
    assert clean[4] == dirty[4]
