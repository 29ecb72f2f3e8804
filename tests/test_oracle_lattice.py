"""Pins of the oracle's lattice tables and equilibrium (Sec. 2, Eq. Equil).

The equilibrium is checked against facts that do not restate its formula:
the D3Q19 moment identities, the exact 0th/1st/2nd moments that the
third-order equilibrium must carry, and its agreement with the discrete
Maxwellian zeta_k rho exp(c.u/cs^2 - u^2/2cs^2) up to third order in u
(the truncation error must shrink as u^4).
"""
import itertools

import numpy as np
import pytest

CS2 = 1.0 / 3.0


def test_d3q19_velocity_set(ora):
    c, w, opp = ora.tables()
    # 19 distinct vectors: the rest vector, 6 axis and 12 face diagonals
    assert len({tuple(v) for v in c}) == 19
    norms = sorted(int(v @ v) for v in c)
    assert norms == [0] + [1] * 6 + [2] * 12
    assert np.all(np.abs(c) <= 1)
    for k in range(19):
        assert np.array_equal(c[opp[k]], -c[k])


def test_d3q19_weight_moments(ora):
    c, w, _ = ora.tables()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    second = np.einsum("k,ki,kj->ij", w, c, c)
    assert np.allclose(second, CS2 * np.eye(3), atol=1e-16)
    third = np.einsum("k,ki,kj,kl->ijl", w, c, c, c)
    assert np.allclose(third, 0.0, atol=1e-16)
    fourth = np.einsum("k,ki,kj,kl,km->ijlm", w, c, c, c, c)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ij,lm->ijlm", d, d) + np.einsum("il,jm->ijlm", d, d)
                      + np.einsum("im,jl->ijlm", d, d))
    assert np.allclose(fourth, iso, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(ora, seed):
    c, w, _ = ora.tables()
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.01, 2.0)
    u = rng.uniform(-0.3, 0.3, 3)
    f = ora.equilibrium(rho, u)
    assert abs(f.sum() - rho) < 1e-15 * 10
    assert np.allclose(f @ c, rho * u, atol=1e-15 * 10)
    second = np.einsum("k,ki,kj->ij", f, c, c)
    assert np.allclose(second, rho * (np.outer(u, u) + CS2 * np.eye(3)), atol=1e-14)


def test_equilibrium_at_rest_is_weights(ora):
    _, w, _ = ora.tables()
    assert np.array_equal(ora.equilibrium(0.7, np.zeros(3)), 0.7 * w)


def test_equilibrium_is_third_order_maxwellian(ora):
    c, w, _ = ora.tables()
    rng = np.random.default_rng(7)
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    errs = []
    for eps in (0.08, 0.04, 0.02):
        u = eps * direction
        maxwell = w * np.exp(c @ u / CS2 - (u @ u) / (2 * CS2))
        errs.append(np.max(np.abs(ora.equilibrium(1.0, u) - maxwell)))
    # fourth-order truncation: halving u divides the error by ~16
    for e0, e1 in zip(errs, errs[1:]):
        assert 12.0 < e0 / e1 < 20.0


def test_equilibrium_velocity_symmetry(ora):
    c, w, opp = ora.tables()
    u = np.array([0.05, -0.11, 0.07])
    f = ora.equilibrium(0.9, u)
    g = ora.equilibrium(0.9, -u)
    # reversing u mirrors the distribution onto the opposite velocities
    assert np.allclose(f[opp], g, atol=1e-16)
    # permuting the axes permutes the distribution accordingly
    for perm in itertools.permutations(range(3)):
        up = u[list(perm)]
        fp = ora.equilibrium(0.9, up)
        cp = c[:, list(perm)]
        for k in range(19):
            kk = next(j for j in range(19) if np.array_equal(c[j], cp[k]))
            assert abs(fp[kk] - f[k]) < 1e-16
