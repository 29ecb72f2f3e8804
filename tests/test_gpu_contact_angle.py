"""Parity of the HIP contact-angle observable and of its E2 seed with the
oracle on analytic caps (Sec. 3, Eq. geoCA): the same tanh cap profile as the
oracle's pins, loaded on both sides as resting equilibrium populations with
rho_A = 0.7 + phi / 2 and rho_B = 0.7 - phi / 2, so that phi = rho_A - rho_B.
Covers E1, E2, the E2 window around the column (a second droplet in the
reference layer), the direct-base fallback and the seed.  Angles within
1e-8 degrees (phi differs from the oracle's only by the rounding of the
population sums)."""
import numpy as np
import pytest

import oracle as O
import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce

pytestmark = pytest.mark.gpu

SHAPE = (52, 64, 64)


def cap_phi(R, theta_deg, center_xy, z_wall=0.5, width=2.0, amp=0.6):
    nz, ny, nx = SHAPE
    c = -R * np.cos(np.radians(theta_deg))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center_xy[0]) ** 2 + (y - center_xy[1]) ** 2 + (z - z_wall - c) ** 2)
    return amp * np.tanh((R - r) / width)


def with_corner_droplet(phi):
    nz, ny, nx = SHAPE
    out = phi
    for dx in (0.0, float(nx)):
        for dy in (0.0, float(ny)):
            out = np.maximum(out, cap_phi(7.0, 90.0, (dx, dy)))
    return out


def _pair(phi, adjoint=False):
    nz, ny, nx = SHAPE
    p = W.params(nx, ny, nz, 0.1)
    solid = W.walls_mask(nx, ny, nz)
    ra, rb = 0.7 + 0.5 * phi, 0.7 - 0.5 * phi
    L = scd.Lattice(p, solid, adjoint=adjoint)
    L.init_equilibrium(ra, rb)
    Lo = O.Lattice(p, solid)
    Lo.init_equilibrium(ra, rb)
    return L, Lo


CASES = [("cap", 40.0), ("cap", 90.0), ("cap", 120.0), ("cap", 150.0),
         ("two", 90.0), ("two", 120.0), ("flat", 25.0)]


@pytest.mark.parametrize("kind,theta", CASES)
def test_contact_angle_matches_oracle(kind, theta):
    announce(f"contact angle parity: {kind} {theta}")
    nz, ny, nx = SHAPE
    cfg = W.ca_cfg(nx, ny)
    phi = cap_phi(24.0, theta, (cfg["ic"], cfg["jc"]))
    if kind == "two":
        phi = with_corner_droplet(phi)
    L, Lo = _pair(phi)
    g, o = L.contact_angle(cfg), Lo.contact_angle(cfg)
    assert g["flags"] == o["flags"]
    if kind == "flat":
        assert g["flags"] & scd.binding.CA_FLAGS["E2_WHOLE_LAYER"]
    else:
        assert abs(g["theta_e2"] - theta) < 0.5
    for k in ("theta_e1", "theta_e2", "aref_e1", "aref_e2", "H_e1", "H_e2"):
        if np.isnan(o[k]):
            assert np.isnan(g[k]), k
        else:
            assert abs(g[k] - o[k]) < 1e-8, k


@pytest.mark.parametrize("kind", ["cap", "two"])
def test_seed_matches_oracle_on_caps(kind):
    nz, ny, nx = SHAPE
    cfg = W.ca_cfg(nx, ny)
    phi = cap_phi(24.0, 120.0, (cfg["ic"], cfg["jc"]))
    if kind == "two":
        phi = with_corner_droplet(phi)
    L, Lo = _pair(phi, adjoint=True)
    lam = O.from_gpu_layout(L.ca_seed(cfg, 1.5).cpu().numpy())
    lo, rc = Lo.ca_seed(cfg, 1.5)
    assert rc == 0
    assert np.max(np.abs(lam - lo)) <= 1e-9 * np.max(np.abs(lo))
