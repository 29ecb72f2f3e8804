"""The contact angle for callers that cannot allocate
(scd_contact_angle_static, scratch in the library's fixed device array)
against scd_contact_angle (scratch in the lattice's work area), through the
C ABI: the same kernels on the same state, so every field agrees bit for bit;
two calls in a row, the second on a smaller lattice (the array keeps the
first call's contents), then a lattice beyond the array's limit, which is
rejected."""
import ctypes
import math

import numpy as np
import pytest

import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce

pytestmark = pytest.mark.gpu

FIELDS = ("theta_e1", "h_e1", "a_e1", "R_e1", "aref_e1", "H_e1", "theta_e2", "h_e2", "a_e2", "R_e2",
          "aref_e2", "H_e2", "cx", "cy", "flags")


def _same(a, b):
    for k in FIELDS:
        x, y = a[k], b[k]
        if isinstance(x, float) and math.isnan(x):
            assert isinstance(y, float) and math.isnan(y), k
        else:
            assert x == y, (k, x, y)
    assert a["status"] == b["status"]


def _lattice(nx, ny, nz, r, dtype, steps):
    c = W.droplet_case(nx, ny, nz, r, 0.12, 0.2, dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(steps)
    return L, c


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_static_contact_angle_matches_work_area(dtype):
    announce(f"no-alloc contact angle: 64x48x32 then 24x20x16, {dtype}")
    big, cb = _lattice(64, 48, 32, 10.0, dtype, 60)
    small, cs = _lattice(24, 20, 16, 6.0, dtype, 40)
    a = big.contact_angle(cb["ca"], static_scratch=True)
    b = small.contact_angle(cs["ca"], static_scratch=True)  # smaller, right after
    _same(a, big.contact_angle(cb["ca"]))
    _same(b, small.contact_angle(cs["ca"]))
    assert a["status"] == 0 and b["status"] == 0 and not np.isnan(a["theta_e1"])
    # a state with no droplet gives the same status and flags both ways
    nx = ny = nz = 16
    p = W.params(nx, ny, nz, 0.1, dtype=dtype)
    L = scd.Lattice(p, W.walls_mask(nx, ny, nz))
    L.init_equilibrium(np.full((nz, ny, nx), 0.04), np.full((nz, ny, nx), 0.7))
    cfg = W.ca_cfg(nx, ny)
    e = L.contact_angle(cfg, static_scratch=True)
    assert e["status"] == scd.binding.SCD_ENOINTERFACE
    _same(e, L.contact_angle(cfg))


def test_static_contact_angle_rejects_large_planes():
    announce("no-alloc contact angle: a 1024 x 260 plane is rejected")
    nx, ny, nz = 1024, 260, 4
    p = W.params(nx, ny, nz, 0.1, dtype="f32")
    L = scd.Lattice(p, W.walls_mask(nx, ny, nz))
    out = scd.binding.ScdCa()
    c = scd.binding.make_ca_cfg(W.ca_cfg(nx, ny, offset=1))
    st = scd.binding.lib().scd_contact_angle_static(L.h, ctypes.byref(c), ctypes.byref(out))
    assert st == scd.binding.SCD_EUNSUPPORTED
    assert b"512 x 512" in scd.binding.lib().scd_last_error() or b"262144" in scd.binding.lib().scd_last_error()
