"""Pins of the Shan-Chen force and of the wall force (Sec. 2, Eq. SCforce
and the wall model), by closed forms of the nearest-neighbour sum:

* uniform psi gives no force;
* psi^B linear in x gives F^A = -g psi^A (2 w_axis + 8 w_diag) b x_hat:
  the sum over the 18 neighbours of c_x c equals (2 + 8) x_hat
  (2 axis and 8 diagonal vectors have c_x = +-1);
* one species only feels the *other* species' gradient;
* next to a flat wall with uniform fluid the wall adds
  5 psi^a (g_wall^a psi_wall^b - g_ab psi^b) z_hat (5 neighbours below);
* in a periodic box the forces on A and B cancel pairwise.
"""
import numpy as np
import pytest

import workloads as W


def _rho(shape, a, b):
    r = np.zeros(shape + (2,))
    r[..., 0] = a
    r[..., 1] = b
    return r


def test_uniform_psi_no_force(ora):
    L = ora.Lattice(W.params(5, 6, 7, 0.13))
    F = L.force(_rho((7, 6, 5), 0.6, 0.2))
    assert np.max(np.abs(F)) < 1e-16


@pytest.mark.parametrize("weights", [(1.0, 1.0), (2.0, 1.0), (1.0, 0.5)])
def test_linear_psi_gradient(ora, weights):
    nx, ny, nz = 12, 4, 4
    g = 0.1
    L = ora.Lattice(W.params(nx, ny, nz, g, w_axis=weights[0], w_diag=weights[1]))
    b = 0.01
    x = np.arange(nx, dtype=float)
    rho = _rho((nz, ny, nx), 0.3, 0.0)
    rho[..., 1] = 0.2 + b * x[None, None, :]
    F = L.force(rho)
    factor = 2 * weights[0] + 8 * weights[1]
    inner = slice(1, nx - 1)  # away from the periodic wrap of the ramp
    assert np.allclose(F[:, :, inner, 0, 0], -g * 0.3 * factor * b, rtol=1e-13, atol=0)
    assert np.allclose(F[:, :, inner, 0, 1:], 0.0, atol=1e-16)
    # B sees a uniform psi^A: no force on B
    assert np.allclose(F[:, :, inner, 1, :], 0.0, atol=1e-16)


def test_flat_wall_force(ora):
    nx, ny, nz = 4, 4, 6
    solid = W.walls_mask(nx, ny, nz)
    g_ab, gw = 0.11, (0.07, 0.05)
    rw = (0.3, 0.6)
    L = ora.Lattice(W.params(nx, ny, nz, g_ab, rho_wall=rw, g_wall=gw), solid)
    ra, rb = 0.5, 0.25
    F = L.force(_rho((nz, ny, nx), ra, rb))
    # first fluid layer above the floor
    fa = 5 * ra * (gw[0] * rw[1] - g_ab * rb)
    fb = 5 * rb * (gw[1] * rw[0] - g_ab * ra)
    assert np.allclose(F[1, :, :, 0, 2], fa, rtol=1e-13)
    assert np.allclose(F[1, :, :, 1, 2], fb, rtol=1e-13)
    assert np.allclose(F[1, :, :, :, :2], 0.0, atol=1e-16)
    # mirror image below the ceiling
    assert np.allclose(F[nz - 2, :, :, 0, 2], -fa, rtol=1e-13)
    # bulk layers feel nothing
    assert np.allclose(F[2:nz - 2], 0.0, atol=1e-16)
    # the wall's psi goes through psi(): check the exponential form as well
    p = W.params(nx, ny, nz, 0.0, rho_wall=rw, g_wall=gw, psi=1)
    L1 = ora.Lattice(p, solid)
    F1 = L1.force(_rho((nz, ny, nx), ra, rb))
    expect = 5 * (1 - np.exp(-ra)) * gw[0] * (1 - np.exp(-rw[1]))
    assert np.allclose(F1[1, :, :, 0, 2], expect, rtol=1e-13)


def test_periodic_forces_cancel(ora):
    nx, ny, nz = 7, 6, 5
    L = ora.Lattice(W.params(nx, ny, nz, 0.16))
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.05, 0.9, size=(nz, ny, nx, 2))
    F = L.force(rho)
    total = F.sum(axis=(0, 1, 2, 3))
    assert np.max(np.abs(total)) < 1e-13
    # and each species alone does not cancel (the test is not vacuous)
    assert np.max(np.abs(F[..., 0, :].sum(axis=(0, 1, 2)))) > 1e-3
