"""Checkpoint/resume and the guards around the step.

* A run saved to disk and resumed in a fresh lattice continues bit for bit
  like the uninterrupted run.
* Wall nodes' population entries are never read: poisoning them with NaN
  leaves every fluid node's populations, the observables and the contact
  angle exactly as in the clean run (also on posts, with walls inside the
  box).
"""
import numpy as np
import pytest
import torch

import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_save_resume_is_bitwise(tmp_path, dtype):
    announce(f"resume: {dtype}")
    c = W.droplet_case(40, 32, 24, 8.0, 0.12, -0.2, dtype=dtype)
    A = scd.Lattice(c["params"], c["solid"])
    A.init_equilibrium(c["rho_a"], c["rho_b"])
    A.step(60)
    path = str(tmp_path / "ckpt.pt")
    A.save(path)
    A.step(60)
    R = scd.Lattice.load(path)
    assert R.step_count == 60
    R.step(60)
    assert R.step_count == A.step_count == 120
    assert torch.equal(A.get_state().cpu(), R.get_state().cpu())


@pytest.mark.parametrize("case", ["walls", "posts"])
def test_wall_entries_are_never_read(case):
    announce(f"poisoned wall entries: {case}")
    if case == "walls":
        c = W.droplet_case(40, 32, 24, 8.0, 0.12, 0.2)
    else:
        nx, ny, nz = 48, 48, 32
        solid = W.posts_mask(nx, ny, nz, width=6, pitch=12, height=8)
        c = W.droplet_case(nx, ny, nz, 14.0, 0.12, -0.3, mask=solid, z_solid_top=8)
    solid = torch.as_tensor(c["solid"].astype(bool))
    runs = []
    for poison in (False, True):
        L = scd.Lattice(c["params"], c["solid"])
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        if poison:
            st = L.get_state()
            st[:, :, solid.to(st.device)] = float("nan")
            L.set_state(st, 0)
        L.step(50)
        st = L.get_state().cpu()
        runs.append((st, L.observables(), L.contact_angle(c["ca"])))
    fluid = ~solid
    clean, dirty = runs[0][0][:, :, fluid], runs[1][0][:, :, fluid]
    assert torch.isfinite(dirty).all()
    assert torch.equal(clean, dirty)
    assert runs[0][1]["mass"] == runs[1][1]["mass"] and runs[1][1]["finite"]
    assert runs[0][2]["theta_e1"] == runs[1][2]["theta_e1"] or (
        np.isnan(runs[0][2]["theta_e1"]) and np.isnan(runs[1][2]["theta_e1"]))


def test_mass_drift_watchdog():
    """The watchdog measures each species' relative mass change since the
    first observables call after the state was set, flags it exactly when it
    exceeds the tolerance (the tolerance is set from the measured drift
    itself, so the case is forced from the host), and a new state resets
    the reference."""
    announce("mass-drift watchdog: f32, 2000 steps")
    c = W.droplet_case(40, 32, 24, 8.0, 0.12, -0.2, dtype="f32")
    L = scd.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    o0 = L.observables()
    assert o0["drift"] == (0.0, 0.0)
    L.step(2000)
    L.set_mass_watchdog(0.0)  # measure only; the reference stays
    o1 = L.observables()
    for a in range(2):
        assert o1["drift"][a] == pytest.approx((o1["mass"][a] - o0["mass"][a]) / o0["mass"][a], rel=1e-12, abs=0)
    worst = max(abs(v) for v in o1["drift"])
    assert worst <= 1e-5  # FP32 rounding only
    if worst > 0:
        L.set_mass_watchdog(0.5 * worst)
        with pytest.raises(scd.ScdError) as e:
            L.observables()
        assert e.value.status == scd.SCD_EDRIFT
        o = L.observables(raise_drift=False)
        assert o["status"] == scd.SCD_EDRIFT and o["drift"] == o1["drift"]
    L.set_mass_watchdog(2.0 * worst + 1e-30)
    assert L.observables()["status"] == scd.SCD_OK
    # a state set from outside is the new reference
    L.set_mass_watchdog(1e-30)
    L.set_state(L.get_state(), step=0)
    assert L.observables()["drift"] == (0.0, 0.0)
    with pytest.raises(scd.ScdError):
        L.set_mass_watchdog(-1.0)
