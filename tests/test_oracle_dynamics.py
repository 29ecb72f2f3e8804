"""Pins of the full oracle step against invariants and closed forms:

* uniform states, at rest or moving, are fixed points (Sec. 2: collision
  toward the equilibrium of the same density and velocity, no force);
* a shear wave decays as exp(-nu q^2 t) with nu = (2 tau - 1)/6 (Sec. 4);
* mass of each species is conserved (BGK and bounce-back conserve it);
* total momentum is conserved in a fully periodic box (the Shan-Chen forces
  cancel pairwise and the velocity shift adds exactly the force);
* the mixed state loses stability at the spinodal of the psi = rho model.
  For a long composition wave the species flux is the velocity-shift drift
  tau F^a (mobility tau / rho^a per unit force, Sec. 2) against the lattice
  diffusion c_s^2 (tau - 1/2) grad rho^a; with F^a = -10 g psi^a grad psi^b
  (the unweighted 18-neighbour sum has sum_k c_k c_k = 10 I) the uniform
  mixture rho^A = rho^B = rho_tot/2 becomes unstable above
      g_c = (tau - 1/2) / (15 tau rho_tot).
  A small wave decays at 0.9 g_c and grows at 1.1 g_c, for two values of tau.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("tau", [(1.0, 1.0), (0.8, 1.3)])
@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.04, -0.02, 0.03)])
def test_uniform_state_is_fixed_point(ora, tau, u):
    nx, ny, nz = 4, 5, 3
    L = ora.Lattice(W.params(nx, ny, nz, 0.15, tau=tau))
    shape = (nz, ny, nx)
    ra, rb = np.full(shape, 0.6), np.full(shape, 0.3)
    uu = np.broadcast_to(np.array(u), shape + (3,)).copy()
    L.init_equilibrium(ra, rb, uu)
    s0 = L.get_state()
    L.step(3)
    assert np.max(np.abs(L.get_state() - s0)) < 1e-15


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_shear_wave_viscosity(ora, tau):
    nx, ny, nz = 2, 2, 32
    L = ora.Lattice(W.params(nx, ny, nz, 0.0, tau=(tau, tau)))
    shape = (nz, ny, nx)
    q = 2 * np.pi / nz
    U = 1e-3
    z = np.arange(nz)
    u = np.zeros(shape + (3,))
    u[..., 0] = U * np.sin(q * z)[:, None, None]
    L.init_equilibrium(np.full(shape, 0.5), np.full(shape, 0.5), u)
    c, _, _ = ora.tables()

    def amplitude():
        s = L.get_state()
        jx = np.einsum("zyxak,k->zyx", s, c[:, 0].astype(float))
        rho = s.sum(axis=(3, 4))
        ux = (jx / rho)[:, 0, 0]
        return 2.0 / nz * np.sum(ux * np.sin(q * z))

    nu = (2 * tau - 1) / 6.0
    a0 = amplitude()
    T = 400
    L.step(T)
    a1 = amplitude()
    # the stored state is post-collision: its velocity lags the physical
    # one by half a step of decay at both ends, which cancels in the ratio
    assert abs(a1 / a0 - np.exp(-nu * q * q * T)) < 0.01 * np.exp(-nu * q * q * T)


def test_mass_conservation_small_droplet(ora):
    c = W.config_small_fp64()
    L = ora.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    m0 = L.observables()["mass"]
    L.step(1000)
    o = L.observables()
    assert o["finite"]
    for a in range(2):
        assert abs(o["mass"][a] - m0[a]) <= 1e-12 * m0[a]


def test_momentum_conservation_periodic(ora):
    n = 16
    L = ora.Lattice(W.params(n, n, n, 0.12, tau=(1.0, 0.9)))
    ra, rb = W.sphere_densities(n, 5.0, center=(7.3, 8.1, 8.6))
    ra, rb = ra + 0.0, rb + 0.0
    rng = np.random.default_rng(5)
    u = rng.uniform(-0.01, 0.01, size=(n, n, n, 3))
    L.init_equilibrium(ra, rb, u)
    P0 = np.array(L.observables()["momentum"])
    mass = sum(L.observables()["mass"])
    L.step(300)
    P1 = np.array(L.observables()["momentum"])
    assert np.max(np.abs(P1 - P0)) <= 1e-12 * mass
    assert np.max(np.abs(P0)) > 1e-3  # a nonzero momentum is carried along


def _mode_amplitudes(ora, g, tau, steps, checkpoints=2):
    nx, ny, nz = 64, 2, 2
    L = ora.Lattice(W.params(nx, ny, nz, g, tau=(tau, tau)))
    x = np.arange(nx)
    pert = 1e-4 * np.sin(2 * np.pi * x / nx)[None, None, :] * np.ones((nz, ny, nx))
    L.init_equilibrium(0.37 + pert, 0.37 - pert)
    out = [2e-4]
    for _ in range(checkpoints):
        L.step(steps // checkpoints)
        r = L.density()
        phi = r[..., 0] - r[..., 1]
        out.append(2.0 / nx * np.sum(phi[0, 0] * np.sin(2 * np.pi * x / nx)))
    return out


@pytest.mark.parametrize("tau", [1.0, 1.5])
def test_demixing_threshold(ora, tau):
    gc = (tau - 0.5) / (15.0 * tau * 0.74)
    below = _mode_amplitudes(ora, 0.9 * gc, tau, 2000)
    above = _mode_amplitudes(ora, 1.1 * gc, tau, 2000)
    assert below[2] < below[1] < below[0]  # decays monotonically
    assert above[2] > above[1] > above[0]  # grows
    # a plain mean-field threshold without the (tau - 1/2)/tau factor would
    # put both couplings deep inside the stable region
    assert 1.1 * gc < 1.0 / (15.0 * 0.74)


def test_result_independent_of_thread_count(ora):
    """The oracle's per-node loops run on host threads; reductions run in a
    fixed serial order, so one thread and all threads give the same state
    and observables bit for bit."""
    c = W.droplet_case(20, 18, 14, 5.0, 0.12, 0.2)
    n0 = ora.num_threads()
    out = []
    for n in (1, max(2, n0)):
        ora.set_threads(n)
        L = ora.Lattice(c["params"], c["solid"])
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(6)
        out.append((L.get_state(), L.observables()["mass"], L.contact_angle(c["ca"])["theta_e2"]))
    ora.set_threads(n0)
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
