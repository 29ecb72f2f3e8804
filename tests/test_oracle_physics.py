"""Physics pins of the oracle that need a relaxed droplet (tens of seconds).

* Laplace law: free droplets of three radii in a periodic box have the same
  surface tension gamma = dp R / 2, and dp against 1/R extrapolates to zero.
  The pressure is the bulk limit of the paper's pressure tensor (Sec. 4.1):
  p = (rho_A + rho_B)/3 + 10 g psi_A psi_B, because the second term of P_ij
  sums 2 g psi_A psi_B (x - x')(x - x') over the 18 neighbours with
  sum_k c_k c_k = 10 I and a prefactor 1/4 over the two ordered pairs.
* Symmetric walls: with the same wall content for both species, Young's
  equation (Sec. 1, Eq. young) gives cos(theta) = 0.  Finite droplets carry
  a 1/R correction (Laplace compression of the droplet), so the pin is the
  1/R extrapolation of E1 from two droplet sizes: 90 +- 1 degrees.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.slow
def test_laplace_law_three_radii(ora):
    n, g, T = 32, 0.1, 3000
    dps, Rs = [], []
    for R0 in (6.0, 8.0, 10.0):
        L = ora.Lattice(W.params(n, n, n, g))
        ra, rb = W.sphere_densities(n, R0)
        L.init_equilibrium(ra, rb)
        L.step(T)
        r = L.density()
        p = (r[..., 0] + r[..., 1]) / 3.0 + 10.0 * g * r[..., 0] * r[..., 1]
        c = n // 2
        p_in = p[c - 1:c + 2, c - 1:c + 2, c - 1:c + 2].mean()
        p_out = p[0:2, 0:2, 0:2].mean()
        volume = np.count_nonzero(r[..., 0] > r[..., 1])
        dps.append(p_in - p_out)
        Rs.append((3.0 * volume / (4.0 * np.pi)) ** (1.0 / 3.0))
    dps, Rs = np.array(dps), np.array(Rs)
    gamma = dps * Rs / 2.0
    assert np.all(dps > 0)
    assert (gamma.max() - gamma.min()) / gamma.mean() < 0.03
    slope, intercept = np.polyfit(1.0 / Rs, dps, 1)
    assert abs(intercept) < 0.05 * dps.max()


@pytest.mark.slow
def test_symmetric_walls_ninety_degrees(ora):
    thetas, radii = [], []
    for n, r0, T in ((32, 8.0, 2000), (48, 12.0, 3000)):
        c = W.droplet_case(n, n, n, r0, 0.1, 0.0)
        L = ora.Lattice(c["params"], c["solid"])
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(T)
        out = L.contact_angle(c["ca"])
        assert out["flags"] == 0
        thetas.append(out["theta_e1"])
        radii.append(out["R_e1"])
    k = (thetas[1] - thetas[0]) / (1.0 / radii[0] - 1.0 / radii[1])
    theta_inf = thetas[1] + k / radii[1]
    assert abs(theta_inf - 90.0) < 1.0
    assert all(abs(t - 90.0) < 4.0 for t in thetas)
