"""Parity of the HIP adjoint step, the E2 seed and the checkpointed gradient
driver with the oracle's FP64 adjoint (itself pinned against central
differences), plus a GPU-only central-difference check."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _tiny(delta=0.1):
    c = W.config_gradient_tiny()
    c["params"] = dict(c["params"], rho_wall=W.asymmetric_wall(delta))
    return c


def test_seed_matches_oracle():
    c = _tiny()
    L = scd.Lattice(c["params"], c["solid"], adjoint=True)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(30)
    lam = O.from_gpu_layout(L.ca_seed(c["ca"], 2.5).cpu().numpy())
    Lo = O.Lattice(c["params"], c["solid"])
    Lo.init_equilibrium(c["rho_a"], c["rho_b"])
    Lo.step(30)
    lo, rc = Lo.ca_seed(c["ca"], 2.5)
    assert rc == 0
    assert np.max(np.abs(lam - lo)) <= 1e-9 * np.max(np.abs(lo))


@pytest.mark.parametrize("variant", ["plain", "post_tau_psi"])
def test_adjoint_step_matches_oracle(variant):
    c = _tiny()
    p = dict(c["params"])
    solid = c["solid"].copy()
    if variant == "post_tau_psi":
        solid[1:4, 3:6, 4:7] = 1
        p = dict(p, tau=(1.0, 0.8), psi=1, g_wall=(0.09, 0.14))
    ra, rb = W.cap_densities(16, 16, 12, 5.0, 0.5, solid, noise=0.02, seed=4)
    announce(f"adjoint parity: 16x16x12 {variant}")
    L = scd.Lattice(p, solid, adjoint=True)
    L.init_equilibrium(ra, rb)
    L.step(5)
    st = L.get_state()
    rng = np.random.default_rng(9)
    fluid = (solid == 0)[None, None]
    lam = rng.normal(size=(2, 19) + solid.shape) * fluid
    lam_t = torch.from_numpy(lam).cuda()
    out, dp = L.adjoint_step(st, lam_t)
    Lo = O.Lattice(p, solid)
    Lo.init_equilibrium(ra, rb)
    Lo.step(5)
    lo, dpo = Lo.adjoint_step(Lo.get_state(), O.from_gpu_layout(lam))
    g = O.from_gpu_layout(out.cpu().numpy())
    assert np.max(np.abs(g - lo)) <= 1e-11 * np.max(np.abs(lo))
    assert np.allclose(dp, dpo, rtol=1e-10, atol=1e-10 * np.max(np.abs(dpo)))


@pytest.mark.parametrize("variant", ["plain", "post_tau_psi"])
def test_fp32_adjoint_step_matches_oracle(variant):
    """The FP32 reverse step (its own local, stencil and push passes) against
    the oracle's FP64 transpose at the same FP32 state and the same
    FP32-rounded lambda', so that only the reverse step's own FP32
    arithmetic differs: every entry within 2e-6 of the largest (measured
    1.9e-7 and 2.1e-7) and the parameter gradient within 1e-5 of its largest
    component (measured 2.5e-7 and 8.3e-7)."""
    c = _tiny()
    p = dict(c["params"], dtype="f32")
    solid = c["solid"].copy()
    if variant == "post_tau_psi":
        solid[1:4, 3:6, 4:7] = 1
        p = dict(p, tau=(1.0, 0.8), psi=1, g_wall=(0.09, 0.14))
    ra, rb = W.cap_densities(16, 16, 12, 5.0, 0.5, solid, noise=0.02, seed=4)
    announce(f"FP32 adjoint parity: 16x16x12 {variant}")
    L = scd.Lattice(p, solid, adjoint=True)
    L.init_equilibrium(ra, rb)
    L.step(5)
    st = L.get_state()
    rng = np.random.default_rng(9)
    fluid = (solid == 0)[None, None]
    lam = (rng.normal(size=(2, 19) + solid.shape) * fluid).astype(np.float32)
    out, dp = L.adjoint_step(st, torch.from_numpy(lam).cuda())
    Lo = O.Lattice(dict(p, dtype="f64"), solid)
    lo, dpo = Lo.adjoint_step(O.from_gpu_layout(st.double().cpu().numpy()),
                              O.from_gpu_layout(lam.astype(np.float64)))
    g = O.from_gpu_layout(out.double().cpu().numpy())
    err = np.max(np.abs(g - lo)) / np.max(np.abs(lo))
    derr = np.max(np.abs(np.array(dp) - dpo)) / np.max(np.abs(dpo))
    announce(f"FP32 adjoint parity: lambda {err:.3e}, parameter gradient {derr:.3e}")
    assert err <= 2e-6
    assert derr <= 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_step_ragged_box_matches_oracle(dtype):
    """A 15 x 13 x 11 box (195 nodes per plane, not a multiple of the 32-node
    population block; 2145 nodes, not a multiple of the 32 nodes a wave of
    the split local pass takes) with floor, ceiling and a post, psi =
    1 - exp(-rho), tau_A != tau_B: the reverse step against the oracle's
    transpose at the same state and lambda', to 1e-11 (FP64, measured
    5.2e-16) and 2e-6 (FP32, measured 2.2e-7) of the largest entry, the
    parameter gradient to 1e-10 and 1e-5 (measured 7.4e-15 and 4.9e-7)."""
    c = W.droplet_case(15, 13, 11, 4.0, 0.12, -0.2, dtype=dtype)
    solid = c["solid"].copy()
    solid[1:5, 5:8, 6:9] = 1
    p = dict(c["params"], tau=(1.0, 0.85), psi=1, g_wall=(0.1, 0.13))
    ra, rb = W.cap_densities(15, 13, 11, 4.0, 1.5, solid, noise=0.02, seed=3)
    announce(f"adjoint parity: ragged 15x13x11 {dtype}")
    L = scd.Lattice(p, solid, adjoint=True)
    L.init_equilibrium(ra, rb)
    L.step(7)
    st = L.get_state()
    rng = np.random.default_rng(5)
    fluid = (solid == 0)[None, None]
    lam = rng.normal(size=(2, 19) + solid.shape) * fluid
    if dtype == "f32":
        lam = lam.astype(np.float32)
    out, dp = L.adjoint_step(st, torch.from_numpy(lam).cuda())
    Lo = O.Lattice(dict(p, dtype="f64"), solid)
    lo, dpo = Lo.adjoint_step(O.from_gpu_layout(st.double().cpu().numpy()),
                              O.from_gpu_layout(lam.astype(np.float64)))
    g = O.from_gpu_layout(out.double().cpu().numpy())
    err = np.max(np.abs(g - lo)) / np.max(np.abs(lo))
    derr = np.max(np.abs(np.array(dp) - dpo)) / np.max(np.abs(dpo))
    announce(f"adjoint parity ragged {dtype}: lambda {err:.3e}, parameter gradient {derr:.3e}")
    assert err <= (1e-11 if dtype == "f64" else 2e-6)
    assert derr <= (1e-10 if dtype == "f64" else 1e-5)


def test_checkpointed_gradient_matches_oracle_and_fd():
    c = _tiny(0.1)
    nsteps, K, target = 50, 7, 120.0
    announce("gradient: 16x16x12, 50 steps, checkpoints every 7")
    setup = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target)
    wall = torch.tensor([0.55, 0.45, 0.12, 0.12, 0.12], dtype=torch.float64, requires_grad=True)
    loss = scd.ContactAngleFn.apply(wall, setup)
    loss.backward()
    g = wall.grad.numpy()
    p = dict(c["params"], rho_wall=(0.55, 0.45))
    lo, th, go = O.theta_e2_gradient_run(p, c["solid"], c["rho_a"], c["rho_b"], nsteps, c["ca"], target)
    assert abs(loss.item() - lo) <= 1e-9 * lo
    assert np.allclose(g, go, rtol=1e-8, atol=0), (g, go)
    # central differences through the GPU forward only
    h = 1e-5
    v0 = wall.detach().numpy()
    for i in range(5):
        vp, vm = v0.copy(), v0.copy()
        vp[i] += h
        vm[i] -= h
        setup.apply_params(vp)
        fp = setup.forward()
        setup.apply_params(vm)
        fm = setup.forward()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), abs(g[i])), (i, fd, g[i])


def test_gradient_workload_full_size_matches_finite_differences():
    """The gradient workload at its own size (64 x 64 x 48, cap radius 14,
    2000 steps, checkpoints every 100, moment cache on): the checkpointed
    gradient of (theta_E2 - 120)^2 with respect to the five wall and
    coupling parameters against central differences of the GPU forward
    pass (the oracle would need every state of the run at this size)."""
    c = W.config_gradient()
    announce("gradient: 64x64x48, 2000 steps, K=100, against central differences")
    setup = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], 2000, 100, c["ca"], 120.0)
    p = c["params"]
    v0 = np.array([p["rho_wall"][0], p["rho_wall"][1], p["g_ab"], p["g_wall"][0], p["g_wall"][1]])
    setup.apply_params(v0)
    setup.forward()
    g = np.array(setup.backward())
    assert np.all(np.isfinite(g)) and np.max(np.abs(g)) > 0
    h = 1e-5
    for i in range(5):
        vp, vm = v0.copy(), v0.copy()
        vp[i] += h
        vm[i] -= h
        setup.apply_params(vp)
        fp = setup.forward()
        setup.apply_params(vm)
        fm = setup.forward()
        fd = (fp - fm) / (2 * h)
        announce(f"gradient: component {i} adjoint {g[i]:.6e} central difference {fd:.6e}")
        # against the largest component, and each component against itself
        # (the five components lie within a factor 5 of each other here)
        assert abs(fd - g[i]) <= 1e-4 * np.max(np.abs(g)), (i, fd, g[i])
        assert abs(fd - g[i]) <= 5e-4 * abs(g[i]), (i, fd, g[i])


def test_two_level_checkpoints_match_one_level():
    c = _tiny(-0.1)
    nsteps, target = 60, 110.0
    one = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, 12, c["ca"], target)
    two = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, 12, c["ca"], target, inner=5)
    la, lb = one.forward(), two.forward()
    assert la == lb
    ga, gb = one.backward(), two.backward()
    assert ga == gb  # same recomputed states, same adjoint order


def test_gradient_from_current_state_matches_oracle():
    c = _tiny(0.15)
    announce("gradient over the last 30 steps of a 50-step run")
    L = scd.Lattice(c["params"], c["solid"], adjoint=True)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(20)
    setup = scd.GradSetup(c["params"], c["solid"], None, None, 30, 8, c["ca"], 100.0, lattice=L, inner=3)
    loss = setup.forward()
    g = setup.backward()
    Lo = O.Lattice(c["params"], c["solid"])
    Lo.init_equilibrium(c["rho_a"], c["rho_b"])
    Lo.step(20)
    states = []
    for _ in range(30):
        states.append(Lo.get_state())
        Lo.step(1)
    th = Lo.contact_angle(c["ca"])["theta_e2"]
    assert abs(loss - (th - 100.0) ** 2) <= 1e-9 * loss
    lam, _ = Lo.ca_seed(c["ca"], 2.0 * (th - 100.0) * 180.0 / np.pi)
    go = np.zeros(5)
    for t in range(29, -1, -1):
        lam, dp = Lo.adjoint_step(states[t], lam)
        go += dp
    assert np.allclose(g, go, rtol=1e-8, atol=0), (g, go)


def test_cached_segments_keep_two_states():
    """With the moment cache covering a segment and a step variant that
    writes the moments, a recomputed segment needs two state buffers (the
    adjoint of a cached state reads nothing else of it); a variant that
    writes none needs one per recomputed step, and the gradients agree."""
    c = _tiny(0.1)
    nsteps, K, target = 30, 10, 110.0
    s = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target)
    s.forward()
    g2 = s.backward()
    assert s.seg.shape[0] == 2
    r = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target)
    r.lat.set_tile(scd.variant_index(64, 4, 0, 1), 4)
    r.forward()
    gk = r.backward()
    assert r.seg.shape[0] == K - 1
    assert np.allclose(g2, gk, rtol=1e-9, atol=0), (g2, gk)  # the variants round differently


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("inner", [None, 4])
def test_moment_cache_gives_the_same_gradient(dtype, inner):
    """The densities and momenta a recomputed step writes are those the
    adjoint computes from its own pull (same pulls, same sums in the same
    order), so the cached sweep reproduces the plain one bit for bit; a
    variant that writes no moments falls back to the full path."""
    announce(f"moment cache: {dtype}, inner {inner}")
    c = _tiny(0.1)
    c["params"] = dict(c["params"], dtype=dtype)
    nsteps, K, target = 40, 9, 115.0
    out = []
    for cache in (False, True):
        s = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target,
                          inner=inner, moment_cache=cache)
        out.append((s.forward(), s.backward()))
    assert out[0] == out[1]
    reg = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target,
                        inner=inner, moment_cache=True)
    reg.lat.set_tile(scd.variant_index(64, 4, 0, 1), 4)
    ref = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], nsteps, K, c["ca"], target,
                        inner=inner, moment_cache=False)
    ref.lat.set_tile(scd.variant_index(64, 4, 0, 1), 4)
    assert (reg.forward(), reg.backward()) == (ref.forward(), ref.backward())


@pytest.mark.parametrize("size", ["tiny", "workload"])
def test_fp32_gradient_against_fp64(size):
    """The FP32 checkpointed gradient (FP32 states and adjoint, FP64 parameter
    sums) against the FP64 gradient of the same run, per component relative
    to the largest: the 16 x 16 x 12 box over 50 steps within 1e-5 (measured
    4.0e-7); the gradient workload (64 x 64 x 48, 2000 steps, checkpoints
    every 100) within 1e-2 (measured 2.6e-3, on the g_ab component, 0.6 % of
    itself: the FP32 forward run and its adjoint carry 2000 steps of
    rounding)."""
    out = {}
    for dt in ("f64", "f32"):
        if size == "tiny":
            c = _tiny(0.1)
            c["params"] = dict(c["params"], dtype=dt)
            n, K = 50, 7
        else:
            c = W.config_gradient(dtype=dt)
            n, K = 2000, 100
        announce(f"gradient: {size} {dt}, {n} steps, K={K}")
        s = scd.GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], n, K, c["ca"], 120.0)
        s.forward()
        out[dt] = np.array(s.backward())
    g64, g32 = out["f64"], out["f32"]
    rel = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    announce(f"gradient: FP32 against FP64, max difference / largest component {rel:.3e}")
    assert rel <= (1e-5 if size == "tiny" else 1e-2), (g32, g64)
