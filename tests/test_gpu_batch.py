"""Batched persistent launch: members of uneven sizes and parameters must
evolve bitwise as the same lattices stepped one by one, with and without a
captured HIP graph; the autotuner must keep results unchanged; and every
member, stepped in the batch, must match the oracle's own run of it (FP64 to
1e-12, FP32 within the rounding of a few tens of steps, the bound of the
full-size FP32 parity test)."""
import numpy as np
import pytest
import torch

import paper_0910_3915_amd as scd
import workloads as W
from gpu_helpers import announce, gpu_state_as_oracle, oracle_run

pytestmark = pytest.mark.gpu


def _members(dtype):
    cases = []
    for (nx, ny, nz, g, d) in ((40, 32, 24, 0.12, 0.2), (24, 48, 16, 0.10, -0.3), (64, 16, 20, 0.15, 0.0)):
        c = W.droplet_case(nx, ny, nz, 0.2 * min(nx, ny), g, d, dtype=dtype)
        cases.append(c)
    return cases


@pytest.mark.parametrize("dtype,grid", [("f64", 64), ("f32", 64), ("f32", 0)])
def test_batch_equals_sequential(dtype, grid):
    announce(f"batch: 3 uneven members, {dtype}, grid {grid}, 40 steps")
    cases = _members(dtype)
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    var = [i for i, r in enumerate(scd.tile_list()) if r[2] == 2][0]  # a species-split variant
    B.set_tile(var, 8, grid)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B.step(20)
    B.graph_capture(10)
    B.graph_replay(2)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        L = scd.Lattice(c["params"], c["solid"])
        L.set_tile(var, 8)
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(40)
        v = B.view(i)
        assert v.step_count == 40
        assert torch.equal(v.get_state().cpu(), L.get_state().cpu()), i
        a, b = v.contact_angle(c["ca"]), L.contact_angle(c["ca"])
        assert a["theta_e1"] == b["theta_e1"] or (np.isnan(a["theta_e1"]) and np.isnan(b["theta_e1"]))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_members_against_oracle(dtype):
    """Three uneven members (one of them with a 64-wide tile's worth of idle
    lanes) stepped 40 times in the batch with its default tile (20 eager
    steps, then a captured graph of 10 replayed twice) against the oracle's
    run of each member from the same seeded densities, every population."""
    announce(f"batch: 3 uneven members, {dtype}, default tile, 40 steps against the oracle")
    cases = _members(dtype)
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B.step(20)
    B.graph_capture(10)
    B.graph_replay(2)
    torch.cuda.synchronize()
    bound = 1e-12 if dtype == "f64" else 2e-6  # measured 1.5e-15 and 1.8e-7
    for i, c in enumerate(cases):
        got = gpu_state_as_oracle(B.view(i))
        d = float(np.max(np.abs(got - oracle_run(c, 40).get_state())))
        announce(f"batch: member {i} max |dC| {d:.3e}")
        assert d <= bound, (i, d)


def test_mixed_member_tiles_equal_sequential():
    """Members with different step variants and chunks (three launch groups
    per step) evolve bit for bit as each lattice stepped alone with its own
    tile, eagerly and from a captured graph."""
    announce("batch: 3 members with three different variants, f32, 30 steps")
    cases = _members("f32")
    tl = scd.tile_list()
    picks = [scd.variant_index(64, 4, 6, 2), scd.variant_index(32, 8, 0, 1), scd.variant_index(32, 4, 7, 1)]
    zcs = [8, 5, 20]
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
        B.set_member_tile(i, picks[i], zcs[i])
    assert B.member_tiles() == list(zip(picks, zcs))
    B.step(10)
    B.graph_capture(10)
    B.graph_replay(2)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        L = scd.Lattice(c["params"], c["solid"])
        L.set_tile(picks[i], min(zcs[i], c["params"]["nz"]))
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(30)
        assert torch.equal(B.view(i).get_state().cpu(), L.get_state().cpu()), (i, tl[picks[i]])


def test_cache_blocked_sets_equal_sequential():
    """Members packed into cache-blocking sets (two sets, then one member per
    set), stepped an odd number of steps eagerly and from a captured graph,
    evolve bit for bit as each lattice stepped alone: only the order of the
    launches changes."""
    announce("batch: cache-blocking sets, f32, 32 steps")
    cases = _members("f32")
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    var = scd.variant_index(64, 4, 6, 2)
    B.set_tile(var, 8, 0)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    # about 9.5, 5.7 and 6.3 MB of state: the first two members share a set
    B.set_blocking(16 << 20)
    assert B.blocking() == (16 << 20, 2)
    B.step(7)
    B.graph_capture(10)
    B.graph_replay(2)
    B.set_blocking(1)
    assert B.blocking() == (1, 3)
    B.step(5)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        L = scd.Lattice(c["params"], c["solid"])
        L.set_tile(var, 8)
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(32)
        v = B.view(i)
        assert v.step_count == 32
        assert torch.equal(v.get_state().cpu(), L.get_state().cpu()), i
    B.set_blocking(0)
    assert B.blocking() == (0, 1)


def test_autotune_keeps_results(tmp_path):
    c = W.droplet_case(48, 40, 24, 9.0, 0.12, 0.1)
    L = scd.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    cache = str(tmp_path / "tune.jsonl")
    best, ms = L.autotune(4, cache)
    assert ms > 0 and 0 <= best[0] < len(scd.tile_list())
    best2, ms2 = L.autotune(4, cache)  # served from the cache
    assert tuple(best2) == tuple(best) and ms2 == pytest.approx(ms)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(30)
    R = scd.Lattice(c["params"], c["solid"])
    R.init_equilibrium(c["rho_a"], c["rho_b"])
    R.step(30)
    assert torch.max(torch.abs(L.get_state().cpu() - R.get_state().cpu())).item() <= 1e-13


def test_batch_autotune_then_default_tiles_match_sequential(tmp_path):
    """After the batch autotuner (which advances the members) a fresh start
    with the chosen tile equals the members stepped one by one with it."""
    cases = _members("f32")
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    cache = str(tmp_path / "btune.jsonl")
    best, ms = B.autotune(2, cache)
    assert ms > 0 and len(best) == 3
    members = B.member_tiles()
    assert B.autotune(2, cache) == (best, ms)  # served from the cache
    assert B.member_tiles() == members
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B.step(24)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        L = scd.Lattice(c["params"], c["solid"])
        L.set_tile(members[i][0], min(members[i][1], c["params"]["nz"]))
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(24)
        assert torch.equal(B.view(i).get_state().cpu(), L.get_state().cpu()), i


def test_full_batch_sweep_equals_sequential():
    """The 64-droplet FP32 sweep the bench times (42 M nodes, boxes of
    64-128 x 64-128 x 48-96), in the bench's launch configuration (batch
    autotuner, re-initialised, a captured graph of 20 steps): every member
    equals the same droplet stepped alone with the tile the autotuner chose,
    bit for bit, and the library's default tile up to FP32 rounding (the
    variants order the force sum differently)."""
    announce("batch: the 64-droplet FP32 sweep, autotuned, 20 steps in a graph, vs one by one")
    draws = W.batch_draw(64, seed=0)
    cases = [W.droplet_case(d["nx"], d["ny"], d["nz"], d["radius"], d["g_ab"], d["delta"], dtype="f32")
             for d in draws]
    s = torch.cuda.Stream()
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=s)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    best, _ = B.autotune(3, None)
    members = B.member_tiles()
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B.graph_capture(20)
    B.graph_replay(1)
    torch.cuda.synchronize()
    worst = 0.0
    for i, c in enumerate(cases):
        v = B.view(i)
        assert v.step_count == 20, i
        got = v.get_state()
        L = scd.Lattice(c["params"], c["solid"], stream=s)
        L.set_tile(members[i][0], min(members[i][1], c["params"]["nz"]))
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(20)
        assert torch.equal(got, L.get_state()), i
        L.close()
        D = scd.Lattice(c["params"], c["solid"], stream=s)
        D.init_equilibrium(c["rho_a"], c["rho_b"])
        D.step(20)
        worst = max(worst, torch.max(torch.abs(got - D.get_state())).item())
        D.close()
    announce(f"batch: largest difference from the default tile {worst:.3e}")
    assert worst <= 1e-5
    # the smallest member against the oracle's own 20-step run of it
    small = min(range(len(cases)), key=lambda i: cases[i]["solid"].size)
    d = float(np.max(np.abs(gpu_state_as_oracle(B.view(small)) - oracle_run(cases[small], 20).get_state())))
    announce(f"batch: member {small} against the oracle, max |dC| {d:.3e}")
    assert d <= 2e-6, d
