"""How far FP32 agrees with FP64 on the long throughput run, and why the
pointwise density bound holds only on short runs.

The 128 x 128 x 64 droplet (wall asymmetry 0.2) runs 20 000 steps three
ways from the same seeded densities: in FP64; in FP32; and in FP64 with the
state rounded to FP32 after every step (FP64 arithmetic, FP32 storage).  The
third run carries only the storage rounding of FP32, none of the FP32
kernel's arithmetic, yet its densities leave the FP64 run's by as much as
the FP32 run's do (measured max |drho| 0.83 against 0.43 after 20 000 steps;
1.2e-4 and 2.9e-6 after 1000): the spreading droplet's interface amplifies
any rounding at the FP32 level to O(0.1) pointwise differences, so the
per-result statement for long runs is the contact angle, which FP32 keeps
within 0.5 degrees.  FP32 mass drifts by rounding only (measured
-7.4e-6 and -1.0e-5 relative over 20 000 steps).
"""
import numpy as np
import pytest
import torch

import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce, gpu_density

pytestmark = pytest.mark.gpu

STEPS = 20000


def _run(c, dtype, round_storage=False):
    L = scd.Lattice(dict(c["params"], dtype=dtype), c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    m0 = L.observables()["mass"]
    early = None
    if round_storage:
        buf = L.empty_blocked()
        for t in range(1, STEPS + 1):
            L.step(1)
            st = L.get_state(out=buf, blocked=True)
            st.copy_(st.float().double())
            L.set_state(st, step=t, blocked=True)
            if t == 1000:
                early = gpu_density(L)
    else:
        L.step(1000)
        early = gpu_density(L)
        L.step(STEPS - 1000)
    m1 = L.observables()["mass"]
    out = (early, gpu_density(L), L.contact_angle(c["ca"]), [(m1[a] - m0[a]) / m0[a] for a in range(2)])
    L.close()
    torch.cuda.empty_cache()
    return out


def test_fp32_long_run_against_fp64_and_storage_rounding():
    c = W.config_throughput(delta=0.2)
    announce("fp32 scope: 128x128x64, 20000 steps: FP64, FP32, FP64 with FP32 storage")
    e64, r64, ca64, m64 = _run(c, "f64")
    e32, r32, ca32, m32 = _run(c, "f32")
    er, rr, car, mr = _run(c, "f64", round_storage=True)
    d32 = float(np.max(np.abs(r32 - r64)))
    dr = float(np.max(np.abs(rr - r64)))
    announce(f"fp32 scope: max|drho| FP32 {d32:.3e}, FP32 storage {dr:.3e}; after 1000 steps "
             f"{np.max(np.abs(e32 - e64)):.3e}, {np.max(np.abs(er - e64)):.3e}; "
             f"theta_E1 {ca64['theta_e1']:.4f} {ca32['theta_e1']:.4f} {car['theta_e1']:.4f}; "
             f"FP32 mass drift {m32}")
    # the contact angle is the per-result statement of the long run
    for k in ("theta_e1", "theta_e2"):
        assert abs(ca32[k] - ca64[k]) <= 0.5, (k, ca32[k], ca64[k])
    # early on the densities still agree pointwise at the FP32 level
    assert np.max(np.abs(e32 - e64)) <= 1e-3
    # storage rounding alone diverges as far as FP32 does: the dynamics, not
    # the FP32 kernel, sets the pointwise difference of the long run
    assert dr >= 0.5 * d32, (dr, d32)
    assert max(abs(v) for v in m64) <= 1e-12
    assert max(abs(v) for v in m32) <= 3e-5
