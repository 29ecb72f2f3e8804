"""Pins of the oracle's pressure tensor (Sec. 4.1) and of the planar surface
tension integral (Eq. gammaMechDef).

* Uniform states: the kinetic part of an equilibrium with velocity u is
  rho/3 I exactly (its second central moment), and the interaction part of a
  uniform state is g psi_A psi_B (2 W_axis + 8 W_diag) I, because the 18
  neighbours give sum_k W_k c_k c_k = (2 W_axis + 8 W_diag) I.
* A relaxed planar interface is in mechanical equilibrium: the normal
  component P_zz is the same on every plane (within 1 %), while the
  tangential component dips in the interface; far from it P_N - P_T
  vanishes and P_N equals the bulk pressure (rho_A + rho_B)/3 + 10 g psi psi.
* Walls: with the same wall content for both species, the A-wall and B-wall
  systems are mirror images, so their tensions are equal and Young's angle
  is 90 degrees; a wall richer in A lowers the A-wall tension (A wets).
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("psi,w", [(0, (1.0, 1.0)), (1, (1.0, 1.0)), (0, (2.0, 0.5))])
def test_uniform_state_pressure(ora, psi, w):
    n, g = 6, 0.13
    p = W.params(n, n, n, g, psi=psi, w_axis=w[0], w_diag=w[1])
    L = ora.Lattice(p)
    ra, rb = 0.61, 0.23
    L.init_equilibrium(np.full((n, n, n), ra), np.full((n, n, n), rb))
    P = L.pressure_tensor()
    f = (lambda r: 1.0 - np.exp(-r)) if psi else (lambda r: r)
    expect = (ra + rb) / 3.0 + g * f(ra) * f(rb) * (2.0 * w[0] + 8.0 * w[1])
    assert np.allclose(P[..., :3], expect, rtol=0, atol=1e-14)
    assert np.allclose(P[..., 3:], 0.0, atol=1e-15)


def test_moving_equilibrium_kinetic_part(ora):
    n, g = 6, 0.1
    L = ora.Lattice(W.params(n, n, n, g))
    ra, rb = 0.5, 0.3
    u = np.zeros((n, n, n, 3))
    u[...] = (0.05, -0.03, 0.02)
    L.init_equilibrium(np.full((n, n, n), ra), np.full((n, n, n), rb), u)
    P = L.pressure_tensor()
    expect = (ra + rb) / 3.0 + 10.0 * g * ra * rb
    assert np.allclose(P[..., :3], expect, rtol=0, atol=1e-14)
    assert np.allclose(P[..., 3:], 0.0, atol=1e-15)


def _lamella(ora, g=0.1, n=4, nz=64, steps=8000):
    L = ora.Lattice(W.params(n, n, nz, g))
    z = np.arange(nz)[:, None, None] * np.ones((1, n, n))
    inside = (z >= nz // 4) & (z < 3 * nz // 4)
    L.init_equilibrium(np.where(inside, 0.7, 0.04), np.where(inside, 0.04, 0.7))
    L.step(steps)
    return L


def test_planar_interface_mechanical_balance(ora):
    g = 0.1
    L = _lamella(ora, g)
    P = L.pressure_tensor()
    r = L.density()
    pn = P[..., 2].mean(axis=(1, 2))
    pt = 0.5 * (P[..., 0] + P[..., 1]).mean(axis=(1, 2))
    assert (pn.max() - pn.min()) / pn.mean() < 0.01
    assert (pt.max() - pt.min()) / pt.mean() > 0.05
    bulk = (r[..., 0] + r[..., 1]) / 3.0 + 10.0 * g * r[..., 0] * r[..., 1]
    for z in (0, 32):  # lamella centres, 16 planes from either interface
        assert abs(pn[z] - pt[z]) < 1e-8
        assert abs(pn[z] - bulk[z].mean()) < 1e-8
    gamma, prof = L.surface_tension_z()
    assert gamma > 0
    assert abs(gamma - prof.sum()) < 1e-14
    # the two interfaces are mirror images about the lamella centre plane
    nz = prof.size
    mirror = prof[(nz // 2 - 1 - np.arange(nz)) % nz]
    assert np.allclose(prof, mirror, atol=1e-9)


def _wall_slab(ora, rho_fluid, rho_wall, g=0.1, n=4, nz=48, wall=16, steps=3000):
    solid = np.zeros((nz, n, n), np.uint8)
    solid[:wall] = 1
    p = W.params(n, n, nz, g, rho_wall=rho_wall)
    L = ora.Lattice(p, solid)
    ra = np.full((nz, n, n), rho_fluid[0])
    rb = np.full((nz, n, n), rho_fluid[1])
    ra[:wall] = 0.0
    rb[:wall] = 0.0
    L.init_equilibrium(ra, rb)
    L.step(steps)
    return L.surface_tension_z()[0]


def test_wall_tensions_and_young(ora):
    gA = _wall_slab(ora, (0.7, 0.04), (0.5, 0.5))
    gB = _wall_slab(ora, (0.04, 0.7), (0.5, 0.5))
    assert abs(gA - gB) <= 1e-12 * abs(gA)
    # a wall richer in A (delta = +0.2) attracts A relative to B
    gA2 = _wall_slab(ora, (0.7, 0.04), W.asymmetric_wall(0.2))
    gB2 = _wall_slab(ora, (0.04, 0.7), W.asymmetric_wall(0.2))
    assert gA2 < gB2


def test_young_and_huang_closed_forms(ora):
    import oracle as O
    assert O.young_angle(0.03, 0.03, 0.05) == pytest.approx(90.0, abs=1e-12)
    assert O.young_angle(0.05, 0.02, 0.06) == pytest.approx(60.0, abs=1e-9)
    assert O.young_angle(0.02, 0.05, 0.06) == pytest.approx(120.0, abs=1e-9)
    assert O.young_angle(0.2, 0.0, 0.05) == 0.0 and O.young_angle(0.0, 0.2, 0.05) == 180.0
    # symmetric wall content: 90 degrees for any bulk densities
    p = W.params(8, 8, 8, 0.12)
    assert O.huang_angle(p, 0.74, 0.01) == pytest.approx(90.0, abs=1e-12)
    # wall richer in A by 0.2: cos = g_wall 0.2 / (g (0.74 - 0.01) / 2) with g_wall = g
    p = W.params(8, 8, 8, 0.12, rho_wall=W.asymmetric_wall(0.2))
    expect = np.degrees(np.arccos(0.2 / (0.73 / 2.0)))
    assert O.huang_angle(p, 0.74, 0.01) == pytest.approx(expect, abs=1e-9)
    # the exponential pseudopotential enters through psi(rho_wall)
    p = W.params(8, 8, 8, 0.12, rho_wall=(0.7, 0.3), psi=1)
    c = (np.exp(-0.3) - np.exp(-0.7)) / (0.5 / 2.0)
    assert O.huang_angle(p, 0.6, 0.1) == pytest.approx(np.degrees(np.arccos(c)), abs=1e-9)


def test_radial_tension_uniform_state(ora):
    n = 12
    L = ora.Lattice(W.params(n, n, n, 0.1))
    L.init_equilibrium(np.full((n, n, n), 0.5), np.full((n, n, n), 0.3))
    g, rs, prof, pphi = L.radial_tension([6.0, 6.0, 6.0], 5.0, 6)
    assert np.isnan(g) and np.isnan(rs)
    assert np.allclose(prof, 0.0, atol=1e-14) and np.allclose(pphi, 0.2, atol=1e-14)


def test_radial_tension_open_axis_equals_padded_box(ora):
    """A sessile droplet between walls at z = 0 and nz - 1: its radial
    profile with the plain z distance equals the fully periodic profile of
    the same state in a box of twice the height whose added layers are all
    wall, where no shell can wrap across z.  With the minimum image in z the
    original box wraps the upper nodes onto the inner shells, so that
    profile differs."""
    c = W.droplet_case(16, 16, 12, 5.0, 0.1, 0.2)
    L = ora.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(40)
    s = L.get_state()
    nz = 12
    p2 = dict(c["params"], nz=2 * nz)
    solid2 = np.concatenate([c["solid"], np.ones_like(c["solid"])], axis=0)
    L2 = ora.Lattice(p2, solid2)
    L2.set_state(np.concatenate([s, np.zeros_like(s)], axis=0))
    centre = [8.0, 8.0, 0.5]
    g_open, rs_open, prof_open, phi_open = L.radial_tension(centre, 7.0, 8, periodic=(True, True, False))
    g_pad, rs_pad, prof_pad, phi_pad = L2.radial_tension(centre, 7.0, 8)
    assert np.array_equal(prof_open, prof_pad) and np.array_equal(phi_open, phi_pad)
    assert (np.isnan(g_open) and np.isnan(g_pad)) or g_open == g_pad
    _, _, prof_wrap, _ = L.radial_tension(centre, 7.0, 8)
    assert not np.allclose(prof_wrap, prof_open, rtol=0, atol=1e-6)


@pytest.mark.slow
def test_radial_tension_free_droplet(ora):
    """A relaxed free droplet: the radial mechanical-equilibrium identity
    p_in - p_out = 2 int (P_N - P_T) / r dr holds within 10 %, R_s is the
    radius of the droplet's volume within 0.2, and Eq. mechRadGamma agrees
    with the Laplace tension dp R_s / 2 within 10 %."""
    n, g = 48, 0.1
    L = ora.Lattice(W.params(n, n, n, g))
    ra, rb = W.sphere_densities(n, 8.0)
    L.init_equilibrium(ra, rb)
    L.step(3000)
    rmax = n / 2 - 5
    gam, rs, prof, pphi = L.radial_tension([n / 2] * 3, rmax, n // 2)
    r = L.density()
    p = (r[..., 0] + r[..., 1]) / 3.0 + 10.0 * g * r[..., 0] * r[..., 1]
    c = n // 2
    dp = p[c - 1:c + 2, c - 1:c + 2, c - 1:c + 2].mean() - p[0:2, 0:2, 0:2].mean()
    rb_ = np.arange(n // 2) + 0.5
    ident = (2.0 * prof / rb_)[rb_ <= rmax].sum()
    assert abs(ident - dp) < 0.10 * dp
    volume = np.count_nonzero(r[..., 0] > r[..., 1])
    assert abs(rs - (3.0 * volume / (4.0 * np.pi)) ** (1.0 / 3.0)) < 0.2
    assert abs(gam - dp * rs / 2.0) < 0.10 * dp * rs / 2.0
