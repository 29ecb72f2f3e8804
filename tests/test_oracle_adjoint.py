"""Pins of the oracle's adjoint step (an extension: the exact transpose of
one lattice step, Sec. 2 sub-steps in reverse).

* Transpose test: for a random state C, random cotangent lam and random
  direction v, <adjoint(lam), v> must equal the central difference of
  <lam, S(C + h v)>, and the parameter gradient must equal the central
  difference of <lam, S(C; p + h e_i)> for each of the five parameters.
* End to end: gradient of (theta_E2 - 120 deg)^2 after 50 steps on a
  16 x 16 x 12 box against central differences with step 1e-5.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

PARAM_KEYS = ("rho_wall_A", "rho_wall_B", "g_ab", "g_wall_A", "g_wall_B")


def perturbed(p, i, h):
    q = dict(p)
    rw, gw = list(q["rho_wall"]), list(q["g_wall"])
    if i == 0:
        rw[0] += h
    elif i == 1:
        rw[1] += h
    elif i == 2:
        q["g_ab"] += h
    elif i == 3:
        gw[0] += h
    else:
        gw[1] += h
    q["rho_wall"], q["g_wall"] = tuple(rw), tuple(gw)
    return q


def one_step(ora, p, solid, state):
    L = ora.Lattice(p, solid)
    L.set_state(state)
    L.step(1)
    return L.get_state()


@pytest.mark.parametrize("psi", [0, 1])
def test_single_step_transpose(ora, psi):
    c = W.config_gradient_tiny()
    p = dict(c["params"], psi=psi, tau=(1.0, 0.8), g_wall=(0.09, 0.14))
    solid = c["solid"].copy()
    solid[1:4, 3:6, 4:7] = 1  # a post: walls on several sides
    L = ora.Lattice(p, solid)
    ra, rb = W.cap_densities(16, 16, 12, 5.0, 0.5, solid, noise=0.02, seed=4)
    L.init_equilibrium(ra, rb)
    L.step(5)
    s0 = L.get_state()
    rng = np.random.default_rng(2)
    fluid = (solid == 0)[..., None, None]
    lam = rng.normal(size=s0.shape) * fluid
    lam_t, dparams = L.adjoint_step(s0, lam)
    h = 1e-6
    for _ in range(2):
        v = rng.normal(size=s0.shape) * fluid
        fp = np.sum(lam * one_step(ora, p, solid, s0 + h * v))
        fm = np.sum(lam * one_step(ora, p, solid, s0 - h * v))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - np.sum(lam_t * v)) <= 1e-7 * abs(fd)
    for i in range(5):
        fp = np.sum(lam * one_step(ora, perturbed(p, i, h), solid, s0))
        fm = np.sum(lam * one_step(ora, perturbed(p, i, -h), solid, s0))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - dparams[i]) <= 1e-6 * max(abs(fd), 1e-3), PARAM_KEYS[i]


def _loss(p, c, nsteps, target):
    L = O.Lattice(p, c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(nsteps)
    th = L.contact_angle(c["ca"])["theta_e2"]
    return (th - target) ** 2


def test_end_to_end_gradient_vs_finite_differences(ora):
    c = W.config_gradient_tiny()
    p = dict(c["params"], rho_wall=(0.55, 0.45))
    nsteps, target = 50, 120.0
    loss, theta, grad = O.theta_e2_gradient_run(p, c["solid"], c["rho_a"], c["rho_b"],
                                                 nsteps, c["ca"], target)
    assert np.isfinite(theta) and abs(loss - _loss(p, c, nsteps, target)) < 1e-12
    h = 1e-5
    for i in range(5):
        fd = (_loss(perturbed(p, i, h), c, nsteps, target) -
              _loss(perturbed(p, i, -h), c, nsteps, target)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), abs(grad[i])), (PARAM_KEYS[i], fd, grad[i])
