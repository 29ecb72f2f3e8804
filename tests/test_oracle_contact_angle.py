"""Pins of the contact-angle observable (Sec. 3, Eq. geoCA) on analytic
caps, with no lattice Boltzmann run: the order parameter of a sphere of
radius R_s whose centre sits c = -R_s cos(theta) above the wall is
phi = 0.6 tanh((R_s - |x - x_c|) / 2), and both estimators must return
theta.  Also checks the E2 seed against central differences of theta_E2."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def cap_phi(shape, R, theta_deg, z_wall, center_xy, width=2.0, amp=0.6):
    nz, ny, nx = shape
    c = -R * np.cos(np.radians(theta_deg))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - center_xy[0]) ** 2 + (y - center_xy[1]) ** 2 + (z - z_wall - c) ** 2)
    return amp * np.tanh((R - r) / width)


def _lattice(ora, nx, ny, nz):
    return ora.Lattice(W.params(nx, ny, nz, 0.1), W.walls_mask(nx, ny, nz))


@pytest.fixture(scope="module")
def box(ora):
    nx, ny, nz = 64, 64, 52
    return _lattice(ora, nx, ny, nz), (nz, ny, nx)


@pytest.mark.parametrize("theta", [40.0, 60.0, 90.0, 120.0, 150.0])
def test_analytic_caps_both_estimators(box, theta):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1], z_solid_top=0, offset=5)
    phi = cap_phi(shape, 24.0, theta, 0.5, (cfg["ic"], cfg["jc"]))
    out = L.contact_angle_phi(cfg, phi)
    assert out["status"] == 0
    assert out["flags"] & ~O.CA_RAY_LIMIT == 0
    assert abs(out["theta_e1"] - theta) < 0.5
    assert abs(out["theta_e2"] - theta) < 0.5
    assert abs(out["cx"] - cfg["ic"]) < 0.5 and abs(out["cy"] - cfg["jc"]) < 0.5


def test_small_offset_flat_cap(box):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1], z_solid_top=0, offset=2)
    phi = cap_phi(shape, 24.0, 30.0, 0.5, (cfg["ic"], cfg["jc"]))
    out = L.contact_angle_phi(cfg, phi)
    assert out["flags"] == 0
    assert abs(out["theta_e1"] - 30.0) < 0.5
    assert abs(out["theta_e2"] - 30.0) < 0.5


def test_cap_flatter_than_reference_falls_back(box):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1], z_solid_top=0, offset=5)
    phi = cap_phi(shape, 24.0, 25.0, 0.5, (cfg["ic"], cfg["jc"]))
    out = L.contact_angle_phi(cfg, phi)
    assert out["flags"] & O.CA_NO_REF
    # base measured half a spacing above the wall: a few degrees of bias
    assert abs(out["theta_e1"] - 25.0) < 4.0


def test_no_droplet(box):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1])
    out = L.contact_angle_phi(cfg, -0.5 * np.ones(shape))
    assert out["status"] == -4 and out["flags"] & O.CA_NO_DROP
    assert np.isnan(out["theta_e1"]) and np.isnan(out["theta_e2"])


def test_second_region_above_is_ignored(box):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1])
    phi = cap_phi(shape, 24.0, 90.0, 0.5, (cfg["ic"], cfg["jc"]))
    film = phi.copy()
    film[44:50] = 0.6  # an A film under the ceiling
    a = L.contact_angle_phi(cfg, phi)
    b = L.contact_angle_phi(cfg, film)
    assert abs(a["theta_e1"] - b["theta_e1"]) < 1e-12
    assert abs(a["theta_e2"] - b["theta_e2"]) < 1e-12


def test_e2_seed_matches_central_differences(ora):
    c = W.config_gradient_tiny()
    L = ora.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(20)
    s0 = L.get_state()
    lam, rc = L.ca_seed(c["ca"], 1.0)
    assert rc == 0
    rng = np.random.default_rng(11)
    fluid = (c["solid"] == 0)[..., None, None]
    for _ in range(3):
        v = rng.normal(size=s0.shape) * fluid
        h = 1e-6
        L.set_state(s0 + h * v)
        tp = L.contact_angle(c["ca"])["theta_e2"]
        L.set_state(s0 - h * v)
        tm = L.contact_angle(c["ca"])["theta_e2"]
        fd = (tp - tm) / (2 * h) * np.pi / 180.0
        ad = float(np.sum(lam * v))
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3)
    L.set_state(s0)


@pytest.mark.parametrize("theta", [90.0, 120.0])
def test_second_droplet_in_reference_layer_is_ignored(box, theta):
    """A second, small droplet on the wall away from the column (centred on
    the box corner, so it wraps over all four corners) adds A-rich nodes to
    the reference layer; E2 sums only the disk around the column, so neither
    estimator moves."""
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1])
    phi = cap_phi(shape, 24.0, theta, 0.5, (cfg["ic"], cfg["jc"]))
    other = np.maximum(phi, cap_phi(shape, 7.0, 90.0, 0.5, (0.0, 0.0)))
    for dx in (shape[2], 0):
        for dy in (shape[1], 0):
            other = np.maximum(other, cap_phi(shape, 7.0, 90.0, 0.5, (float(dx), float(dy))))
    a = L.contact_angle_phi(cfg, phi)
    b = L.contact_angle_phi(cfg, other)
    kref = cfg["z_solid_top"] + cfg["offset"]
    assert (other[kref] > 0).sum() > (phi[kref] > 0).sum() + 50
    assert b["flags"] & ~O.CA_RAY_LIMIT == 0
    assert abs(a["theta_e1"] - b["theta_e1"]) < 1e-12
    assert abs(a["theta_e2"] - b["theta_e2"]) < 1e-12
    assert abs(b["theta_e2"] - theta) < 0.5


def test_whole_layer_when_reference_is_outside(box):
    L, shape = box
    cfg = W.ca_cfg(shape[2], shape[1], z_solid_top=0, offset=5)
    out = L.contact_angle_phi(cfg, cap_phi(shape, 24.0, 25.0, 0.5, (cfg["ic"], cfg["jc"])))
    assert out["flags"] & O.CA_NO_REF and out["flags"] & O.CA_E2_WHOLE_LAYER
