#!/usr/bin/env python3
"""Throughput benchmark of the two-component Shan-Chen D3Q19 relaxation run.

Workload (the single-droplet throughput case): a 128 x 128 x 64 box with
walls at z = 0 and 63, a cap of radius 24 of A on the floor (rho 0.7 / 0.04,
noise 1e-3, seed 0), tau = 1, psi = rho, g_ab = g_wall = 0.12, wall
asymmetry rho_wall_A - rho_wall_B = 0.2.  A "step" is one lattice time step
(pull-stream + bounce-back, Shan-Chen and wall force, velocity shift, BGK
collide, fused in one kernel); the timed region also takes the FP64
mass/momentum reduction and both contact-angle estimators every 100 steps,
as a relaxation run does.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  Extra objects: roofline of the fused step kernel
(algorithmic bytes 2 species x 19 x (read + write) x sizeof(real) per fluid
node), the FP32 run, FP32-vs-FP64 results after --theta-steps steps, the
adjoint/forward cost ratio (64 x 64 x 48), the batched sweep against
sequential launches (64 droplets drawn from seed 0), and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "D3Q19 2-comp MLUPS & % HBM roofline; adjoint/forward cost; FP32 vs FP64 dtheta"
COUNTERS = {dt: os.path.join(ROOT, "profiles", "step_fused_128x128x64_%s_counters.json" % dt)
            for dt in ("f64", "f32")}
KERNEL_SOURCES = ["paper_0910_3915_amd/csrc/step.hip", "paper_0910_3915_amd/csrc/common.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def fluid_nodes(solid):
    import numpy as np
    return int(np.count_nonzero(np.asarray(solid) == 0))


def timed_relaxation(scd, W, torch, dtype, steps, warmup, samples, obs_every, tile, stream):
    """MLUPS of the relaxation run (median over samples, each exactly `steps`
    steps after exactly `warmup` untimed ones) and the per-launch time of
    the step kernel."""
    import numpy as np
    c = W.config_throughput(delta=0.2, dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"], stream=stream)
    if tile is not None:
        L.set_tile(*tile)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    nf = fluid_nodes(c["solid"])
    L.step(warmup)
    L.observables()
    torch.cuda.synchronize()
    # a graph of g steps (even, at most obs_every) serves the blocks; an odd
    # or short remainder runs eagerly; observables and both contact-angle
    # estimators after every obs_every-th step and after the last one
    g = min(obs_every, steps) // 2 * 2
    walls = []
    for _ in range(samples):
        if g >= 2:
            L.graph_capture(g)  # on the current buffer parity; runs nothing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            if g >= 2 and steps - done >= g:
                L.graph_replay(1)
                done += g
            else:
                L.step(steps - done)
                done = steps
            if done % obs_every == 0 or done == steps:
                L.observables()
                L.contact_angle(c["ca"])
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    wall = float(np.median(walls))
    # kernel-only region on the kernel's stream: average launch duration
    gk = max(2, g)
    L.graph_capture(gk)
    reps = max(1, steps // gk)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.graph_replay(reps)
    e1.record(stream)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / (reps * gk)
    # layout ceiling: the step's pulls and stores without its arithmetic
    e0.record(stream)
    for _ in range(reps * gk):
        L.pull_copy()
    e1.record(stream)
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / (reps * gk)
    ca = L.contact_angle(c["ca"])
    variant, zc = L.tile()
    tx, ty, zmarch, waves = scd.tile_list()[variant]
    return {"mlups": nf * steps / wall / 1e6, "ms_per_step": wall * 1e3 / steps, "steps": steps,
            "samples_mlups": [round(nf * steps / w / 1e6, 1) for w in walls],
            "launch_ms": launch_ms, "pull_copy_ms": copy_ms, "fluid_nodes": nf,
            "theta_e1": ca["theta_e1"],
            "theta_e2": ca["theta_e2"],
            "tile": {"tx": tx, "ty": ty, "zmarch": zmarch, "waves_per_simd": waves, "zchunk": zc}}


def roofline(res, bytes_per_node, traffic):
    achieved = bytes_per_node * res["fluid_nodes"] / (res["launch_ms"] * 1e-3) / 1e9
    layout = bytes_per_node * res["fluid_nodes"] / (res["pull_copy_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_step (fused pull-stream, force, collide)",
            "bytes_per_fluid_node": bytes_per_node, "launch_us": round(res["launch_ms"] * 1e3, 2),
            # the same pulls and stores with no arithmetic (k_pull_copy): the
            # rate the state layout itself allows
            "layout_copy": {"GBs": round(layout, 1), "us": round(res["pull_copy_ms"] * 1e3, 2),
                            "step_frac": round(achieved / layout, 4)}}


def measured_traffic(dtype):
    """HBM bytes per launch of the step in this dtype from the committed
    rocprofv3 counter summary, or None when there is none or the kernel
    sources changed since the counters were taken."""
    if not os.path.exists(COUNTERS[dtype]):
        return None
    d = json.load(open(COUNTERS[dtype]))
    if d.get("kernel_sha") != kernel_sha():
        return None
    return d.get("traffic_bytes_per_launch")


def autotuned_tile(scd, W, dtype, stream):
    c = W.config_throughput(delta=0.2, dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"], stream=stream)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    best, ms = L.autotune(10, None)
    return tuple(best), ms


def fp32_vs_fp64(scd, W, torch, steps, tile64, tile32, stream):
    """The throughput run for `steps` steps in FP64, in FP32, in FP64 with
    the state rounded to FP32 after every step (FP64 arithmetic, FP32
    storage), and in FP64 from initial densities perturbed by 6e-8 relative
    (uniform, seeded): the last two show how far rounding at the FP32 level
    alone, once per step or once at the start, moves the densities over the
    run, next to the FP32 run's difference."""
    import numpy as np
    out = {}
    dens = {}
    mass = {}
    for name, dt, tile in (("f64", "f64", tile64), ("f32", "f32", tile32), ("f64_f32_storage", "f64", tile64),
                           ("f64_perturbed", "f64", tile64)):
        c = W.config_throughput(delta=0.2, dtype=dt)
        L = scd.Lattice(c["params"], c["solid"], stream=stream)
        if tile is not None:
            L.set_tile(*tile)
        ra, rb = c["rho_a"], c["rho_b"]
        if name == "f64_perturbed":
            rng = np.random.default_rng(7)
            ra = ra * (1.0 + 6e-8 * rng.uniform(-1.0, 1.0, ra.shape))
            rb = rb * (1.0 + 6e-8 * rng.uniform(-1.0, 1.0, rb.shape))
        L.init_equilibrium(ra, rb)
        m0 = L.observables()["mass"]
        if name == "f64_f32_storage":
            buf = L.empty_blocked()
            for t in range(1, steps + 1):
                L.step(1)
                st = L.get_state(out=buf, blocked=True)
                st.copy_(st.float().double())
                L.set_state(st, step=t, blocked=True)
        else:
            L.step(steps)
        m1 = L.observables()["mass"]
        mass[name] = [(m1[a] - m0[a]) / m0[a] for a in range(2)]
        out[name] = L.contact_angle(c["ca"])
        dens[name] = L.density().cpu().numpy()
        L.close()
    return {"steps": steps,
            "max_abs_drho": float(np.max(np.abs(dens["f64"] - dens["f32"]))),
            "max_abs_drho_f64_f32_storage": float(np.max(np.abs(dens["f64"] - dens["f64_f32_storage"]))),
            "max_abs_drho_f64_perturbed_6e-8": float(np.max(np.abs(dens["f64"] - dens["f64_perturbed"]))),
            "theta_e1_f64": out["f64"]["theta_e1"], "theta_e1_f32": out["f32"]["theta_e1"],
            "theta_e2_f64": out["f64"]["theta_e2"], "theta_e2_f32": out["f32"]["theta_e2"],
            "dtheta_e1": abs(out["f64"]["theta_e1"] - out["f32"]["theta_e1"]),
            "dtheta_e2": abs(out["f64"]["theta_e2"] - out["f32"]["theta_e2"]),
            "mass_drift_rel": mass}


def adjoint_cost(scd, W, torch, stream, dtype="f64", nsteps=40):
    """Adjoint step against forward step on the gradient workload, both
    launched the same way: one C call per step sequence, no graph, timed
    with HIP events on the lattice's stream (the library captures forward
    steps in graphs too; that time is reported as well)."""
    import ctypes
    c = W.config_gradient(dtype=dtype)
    L = scd.Lattice(c["params"], c["solid"], adjoint=True, stream=stream)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    L.step(200)
    st = L.get_state(blocked=True)
    lam = L.ca_seed(c["ca"], 1.0, blocked=True)
    lam2 = torch.empty_like(lam)
    L.graph_capture(20)
    lib = scd.binding.lib()
    p = scd.binding._ptr
    e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    torch.cuda.synchronize()
    e[0].record(stream)
    L.graph_replay(nsteps // 20)
    e[1].record(stream)
    scd.binding.check(lib.scd_step(L.h, ctypes.c_int64(nsteps)))
    e[2].record(stream)
    L.adjoint_reset()
    e[3].record(stream)
    a, b = lam, lam2
    for _ in range(nsteps):
        scd.binding.check(lib.scd_adjoint_step(L.h, p(st), p(a), p(b), None))
        a, b = b, a
    e[4].record(stream)
    torch.cuda.synchronize()
    g = L.adjoint_read()
    fwd_graph = e[0].elapsed_time(e[1]) / nsteps
    fwd = e[1].elapsed_time(e[2]) / nsteps
    adj = e[3].elapsed_time(e[4]) / nsteps
    # the whole checkpointed gradient of the gradient workload: 2000 forward
    # steps with a checkpoint every 100, then the reverse sweep (segment
    # recompute + adjoint steps)
    from paper_0910_3915_amd.grad import GradSetup
    gs = GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], 2000, 100, c["ca"], 120.0,
                   stream=stream)
    gs.forward()
    gs.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs.forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad = gs.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"workload": "64x64x48 droplet r=14, " + dtype, "forward_ms": round(fwd, 4),
            "forward_graph_ms": round(fwd_graph, 4),
            "adjoint_ms": round(adj, 4), "ratio": round(adj / fwd, 3),
            "grad_finite": all(x == x for x in g),
            "checkpointed_2000_steps": {"forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
                                        "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
                                        "theta_e2": gs.theta, "grad": grad}}


def _angles(lat, cfg):
    """(theta_E1, theta_E2), or None when no droplet is left (members below
    the coexistence coupling dissolve)."""
    ca = lat.contact_angle(cfg)
    if ca.get("status", 0) != 0 or ca["theta_e1"] != ca["theta_e1"] or ca["theta_e2"] != ca["theta_e2"]:
        return None
    return (ca["theta_e1"], ca["theta_e2"])


def batched_vs_sequential(scd, W, torch, stream, steps=10000, graph_steps=100, seq_default_steps=200,
                          n=64):
    """The batched parameter sweep: 64 FP32 droplets drawn from seed 0, run
    for `steps` steps by the batch (tiles and cache-blocking sets picked by
    the batch autotuner, a captured graph of graph_steps steps replayed),
    against the same 64 droplets run one after another, one launch per step
    each, with each lattice's autotuned tile for the same number of steps
    (and, for the rate only, with the library's default tile over
    seq_default_steps, both one lattice at a time and all lattices in turn
    every step).  Both sides start from the same seeded state; the contact
    angles of every droplet at the end are compared."""
    draws = W.batch_draw(n, seed=0)
    cases = [W.droplet_case(d["nx"], d["ny"], d["nz"], d["radius"], d["g_ab"], d["delta"], dtype="f32")
             for d in draws]
    nf = sum(fluid_nodes(c["solid"]) for c in cases)
    B = scd.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=stream)
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    tile, _ = B.autotune(6, None)
    members = B.member_tiles()
    set_bytes, nsets = B.blocking()
    for i, c in enumerate(cases):
        B.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B.graph_capture(graph_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.graph_replay(steps // graph_steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    th_b = [_angles(B.view(i), c["ca"]) for i, c in enumerate(cases)]
    del B
    torch.cuda.empty_cache()

    def timed_runs(lats, nsteps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for L in lats:
            L.step(nsteps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def fresh(tuned):
        lats = []
        for c in cases:
            L = scd.Lattice(c["params"], c["solid"], stream=stream)
            L.init_equilibrium(c["rho_a"], c["rho_b"])
            if tuned:
                L.autotune(3, None)
                L.init_equilibrium(c["rho_a"], c["rho_b"])
            lats.append(L)
        return lats

    lats = fresh(False)
    timed_runs(lats, 2)  # warm-up
    ts_default = timed_runs(lats, seq_default_steps) / seq_default_steps
    # the same lattices advanced in turn, one launch each per step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(seq_default_steps):
        for L in lats:
            L.step(1)
    torch.cuda.synchronize()
    ts_inter = (time.perf_counter() - t0) / seq_default_steps
    lats = fresh(True)
    ts_tuned = timed_runs(lats, steps) / steps
    th_s = [_angles(L, c["ca"]) for L, c in zip(lats, cases)]
    del lats
    torch.cuda.empty_cache()
    both = [(a, b) for a, b in zip(th_b, th_s) if a is not None and b is not None]
    tl = scd.tile_list()
    per_step_b = tb / steps
    return {"droplets": n, "fluid_nodes": nf, "dtype": "f32", "steps": steps,
            "graph_steps": graph_steps,
            "batched_mlups": round(nf / per_step_b / 1e6, 1),
            "batched_tile": {"shape": list(tl[tile[0]]), "zchunk": tile[1], "grid": tile[2],
                             "set_bytes": set_bytes, "sets": nsets,
                             "member_variants": {"x".join(map(str, tl[v])): sum(1 for m in members if m[0] == v)
                                                 for v in sorted(set(m[0] for m in members))}},
            "sequential_tuned_mlups": round(nf / ts_tuned / 1e6, 1),
            "sequential_default_mlups": round(nf / ts_default / 1e6, 1),
            "sequential_default_steps": seq_default_steps,
            "sequential_interleaved_mlups": round(nf / ts_inter / 1e6, 1),
            "speedup": round(min(ts_default, ts_tuned) / per_step_b, 3),
            "speedup_vs_sequential_default": round(ts_default / per_step_b, 3),
            "speedup_vs_interleaved": round(ts_inter / per_step_b, 3),
            "theta": {"droplets_compared": len(both),
                      "no_droplet_both": sum(1 for a, b in zip(th_b, th_s) if a is None and b is None),
                      "no_droplet_one_side": sum(1 for a, b in zip(th_b, th_s) if (a is None) != (b is None)),
                      "max_dtheta_e1": max((abs(a[0] - b[0]) for a, b in both), default=None),
                      "max_dtheta_e2": max((abs(a[1] - b[1]) for a, b in both), default=None)}}


def copy_probe(torch, scd, stream, nbytes=1 << 30, reps=20):
    """Attainable HBM bandwidth of a read-once write-once sweep: the library's
    STREAM copy kernel over nbytes (read + write counted), timed with events
    on the same stream; torch's own device copy is reported beside it."""
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()

    def timed(fn):
        with torch.cuda.stream(stream):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(lambda: scd.stream_copy(src, dst, stream))
    if not torch.equal(src, dst):
        raise RuntimeError("STREAM copy probe produced a wrong copy")
    ms_torch = timed(lambda: dst.copy_(src))
    return {"bytes_per_copy": 2 * n * 8, "kernel": "k_stream_copy", "us": round(ms * 1e3, 2),
            "GBs": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1),
            "torch_copy_GBs": round(2 * n * 8 / (ms_torch * 1e-3) / 1e9, 1)}


def cpu_baseline(W, seconds):
    """The oracle on the host cores: all its threads for `seconds`, then one
    thread for a third of that (a shorter sample of the same run)."""
    import oracle
    c = W.config_throughput(delta=0.2)
    L = oracle.Lattice(c["params"], c["solid"])
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    nf = fluid_nodes(c["solid"])

    def sample(limit):
        L.step(1)  # first touch
        steps = 0
        t0 = time.perf_counter()
        while True:
            L.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= limit or steps >= 1000:
                return steps, el

    cores = oracle.num_threads()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    steps, el = sample(seconds)
    oracle.set_threads(1)
    steps1, el1 = sample(seconds / 3)
    oracle.set_threads(cores)
    return {"value": round(nf * steps / el / 1e6, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"128x128x64 droplet, FP64, {steps} steps ({el:.1f} s)",
            "one_core": {"value": round(nf * steps1 / el1 / 1e6, 3),
                         "sample": f"{steps1} steps ({el1:.1f} s), 1 thread"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--samples", type=int, default=3,
                    help="timed samples of --steps steps each; the median is reported")
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--theta-steps", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true", help="main workload only")
    ap.add_argument("--autotune", action="store_true",
                    help="time every compiled variant first instead of the library defaults")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64",
                    help="precision of the main workload; f32 times the FP32 relaxation run "
                         "alone (no extras, no CPU baseline)")
    args = ap.parse_args()
    if args.dtype == "f32":
        args.no_extras = args.no_cpu = True
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(one process drives one GPU)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.samples < 1 or args.obs_every < 1:
        print("bench.py: need --steps >= 1, --warmup >= 0, --samples >= 1, --obs-every >= 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0910_3915_amd as scd
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    tile64 = tile32 = None  # library default variant and z-chunk
    if args.autotune:
        tile64, ms64 = autotuned_tile(scd, W, "f64", stream)
        tile32, ms32 = autotuned_tile(scd, W, "f32", stream)
        log(f"autotune: f64 {tile64} {ms64:.4f} ms/step, f32 {tile32} {ms32:.4f} ms/step")

    dt = args.dtype
    log("timing %s relaxation run" % dt.upper())
    r64 = timed_relaxation(scd, W, torch, dt, args.steps, args.warmup, args.samples, args.obs_every,
                           tile64 if dt == "f64" else tile32, stream)
    log(json.dumps(r64))
    result = {
        "metric": METRIC, "value": round(r64["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": r64["steps"], "warmup": args.warmup, "samples": args.samples,
        "samples_mlups": r64["samples_mlups"], "ms_per_step": round(r64["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": "synthetic (seeded droplet, no dataset)",
        "config": {"workload": "single droplet 128x128x64, cap r=24, g_ab=g_wall=0.12, tau=1, "
                               "rho_wall=(0.6,0.4), %s, observables every %d steps"
                               % (dt.upper(), args.obs_every),
                   "fluid_nodes": r64["fluid_nodes"], "tile": r64["tile"], "parallelism": "single GPU"},
        "roofline": roofline(r64, 608 if dt == "f64" else 304, measured_traffic(dt)),
    }
    if not args.no_extras:
        log("timing FP32 relaxation run")
        r32 = timed_relaxation(scd, W, torch, "f32", args.steps, args.warmup, args.samples,
                               args.obs_every, tile32, stream)
        result["fp32"] = {"value": round(r32["mlups"], 1), "unit": "MLUPS",
                          "ms_per_step": round(r32["ms_per_step"], 5), "tile": r32["tile"],
                          "roofline": roofline(r32, 304, measured_traffic("f32"))}
        log("FP32 vs FP64 after %d steps" % args.theta_steps)
        result["fp32_vs_fp64"] = fp32_vs_fp64(scd, W, torch, args.theta_steps, tile64, tile32, stream)
        log("adjoint / forward cost")
        adj = {"f64": adjoint_cost(scd, W, torch, stream, "f64"),
               "f32": adjoint_cost(scd, W, torch, stream, "f32")}
        g64 = adj["f64"]["checkpointed_2000_steps"]["grad"]
        g32 = adj["f32"]["checkpointed_2000_steps"]["grad"]
        gmax = max(abs(v) for v in g64)
        # the FP32 gradient of (theta_E2 - 120)^2 over the 2000-step run
        # against the FP64 one, per component relative to the largest
        adj["f32_vs_f64_grad"] = {"max_rel_to_largest": max(abs(a - b) for a, b in zip(g32, g64)) / gmax,
                                  "per_component_rel": [abs(a - b) / abs(b) for a, b in zip(g32, g64)]}
        result["adjoint"] = adj
        log("batched vs sequential")
        result["batched"] = batched_vs_sequential(scd, W, torch, stream)
    result["copy_probe"] = copy_probe(torch, scd, stream)
    log("copy probe", result["copy_probe"])
    if not args.no_cpu:
        log("CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
