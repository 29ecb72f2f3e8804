"""Workload drivers on top of the library: the wall-asymmetry sweep, the
gradient fit of the wall parameters to a target angle, the structured-
surface (posts) run, and the planar surface-tension route to the contact
angle with Huang's estimate.  Each prints JSON lines and returns a dict.

    python -m paper_0910_3915_amd.experiments sweep --dtype f64
    python -m paper_0910_3915_amd.experiments fit --dtype f64
    python -m paper_0910_3915_amd.experiments posts --steps 100000
    python -m paper_0910_3915_amd.experiments young --dtype f64
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import binding as B
from .grad import ContactAngleFn, GradSetup

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import workloads as W  # noqa: E402


def emit(d):
    print(json.dumps(d), flush=True)
    return d


def fluid_nodes(solid):
    return int(np.count_nonzero(np.asarray(solid) == 0))


def timed_steps(L, steps, stream, chunk=1000):
    """Advance L by steps with captured graphs; returns seconds."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    g = min(chunk, steps) // 2 * 2
    if g >= 2:
        L.graph_capture(g)
        while steps - done >= g:
            L.graph_replay(1)
            done += g
    L.step(steps - done)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def sessile_radial_tension(L, ca, cfg):
    """Eq. mechRadGamma on a sessile droplet: shells about the centre of the
    sphere of its E1 cap, on the droplet's axis column at height
    k_ref + H - R (the cap's sphere, R = (a_ref^2 + H^2) / 2H measured from
    the reference layer), out to 5 lattice units before the nearest
    border.  z distances are plain differences (the box is bounded by walls
    in z; x and y stay periodic).  Returns (gamma, R_s, centre)."""
    nz, ny, nx = L.shape
    k_ref = cfg["z_solid_top"] + cfg["offset"]
    zc = k_ref + ca["H_e1"] - ca["R_e1"]
    centre = [float(cfg["ic"]), float(cfg["jc"]), float(zc)]
    rmax = min(nx / 2.0, ny / 2.0, (nz - 1) - zc) - 5.0
    g, rs, _, _ = L.radial_tension(centre, rmax, int(rmax) + 2, periodic=(True, True, False))
    return g, rs, centre


def sweep(dtype="f64", steps=20000, box="full", deltas=W.THROUGHPUT_DELTAS, radial=False):
    """Contact angle against the wall asymmetry rho_wall_A - rho_wall_B; with
    radial, also the radial surface tension of each sessile droplet."""
    stream = torch.cuda.Stream()
    out = []
    for d in deltas:
        c = (W.config_throughput(delta=float(d), dtype=dtype) if box == "full"
             else dict(W.config_throughput_twin(delta=float(d)), params=dict(
                 W.config_throughput_twin(delta=float(d))["params"], dtype=dtype)))
        L = B.Lattice(c["params"], c["solid"], stream=stream)
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        sec = timed_steps(L, steps, stream)
        ca = L.contact_angle(c["ca"])
        obs = L.observables()
        row = {"exp": "sweep", "box": box, "dtype": dtype, "delta": float(d), "steps": steps,
               "theta_e1": ca["theta_e1"], "theta_e2": ca["theta_e2"], "flags": ca["flags"],
               "mlups": fluid_nodes(c["solid"]) * steps / sec / 1e6, "mass": list(obs["mass"])}
        if radial:
            g, rs, centre = sessile_radial_tension(L, ca, c["ca"])
            row.update({"gamma_radial": g, "R_s": rs, "R_e1": ca["R_e1"], "centre": centre})
        out.append(emit(row))
        del L
    return {"sweep": out}


def fit(dtype="f64", iters=50, steps=2000, ckpt=100, target=120.0, max_step=0.05):
    """Gradient descent on the wall contents (rho_wall_A, rho_wall_B) through
    the hand-written adjoint: loss L = (theta_E2 - target)^2 (deg^2) after
    steps steps of the 64 x 64 x 48 droplet (cap radius 14), g_ab = g_wall =
    0.12 held fixed (their gradients are reported).

    Step along -grad L with the Gauss-Newton length for the single residual
    r = theta - target (dp = -2 L grad L / |grad L|^2, the step that zeroes
    the linearised r), capped at max_step in parameter space; a trial point
    that raises the loss or loses the droplet halves the step (at most five
    times).  Trials are forward-only; the gradient is taken through
    ContactAngleFn at accepted points."""
    c = W.config_gradient(dtype=dtype)
    setup = GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], steps, ckpt, c["ca"], target)
    g_ab = 0.12

    def wall_of(p):
        return torch.cat([p, torch.tensor([g_ab, g_ab, g_ab], dtype=torch.float64)])

    def value_and_grad(p):
        wall = wall_of(p).requires_grad_(True)
        loss = ContactAngleFn.apply(wall, setup)
        loss.backward()
        return loss.item(), setup.theta, wall.grad.clone()

    def trial(p):
        setup.apply_params(wall_of(p).tolist())
        try:
            return setup.forward()
        except B.ScdError:
            return float("inf")

    p = torch.tensor([0.5, 0.5], dtype=torch.float64)
    loss, theta, gfull = value_and_grad(p)
    hist = []
    for it in range(iters):
        gx = gfull[:2]
        hist.append(emit({"exp": "fit", "dtype": dtype, "iter": it, "loss": loss, "theta_e2": theta,
                          "rho_wall_A": float(p[0]), "rho_wall_B": float(p[1]),
                          "grad_full": [float(v) for v in gfull]}))
        nrm2 = float(gx @ gx)
        if loss < 1e-8 or nrm2 == 0.0:
            break
        dp = -2.0 * loss / nrm2 * gx
        n = float(dp.norm())
        if n > max_step:
            dp *= max_step / n
        t, accepted = 1.0, False
        for _ in range(6):
            q = torch.clamp(p + t * dp, min=0.0)
            if trial(q) < loss:
                accepted = True
                break
            t *= 0.5
        if not accepted:
            break
        p = q
        loss, theta, gfull = value_and_grad(p)
    res = emit({"exp": "fit_final", "dtype": dtype, "theta_e2": theta, "loss": loss,
                "rho_wall": [float(v) for v in p], "g_ab": g_ab, "iters": len(hist),
                "optimizer": "gradient descent, Gauss-Newton step length capped at %g, backtracking" % max_step,
                "abs_error_deg": abs(theta - target)})
    return {"history": hist, "final": res}


def _planar_batch(cases, steps, stream, checkpoints=(0.5, 1.0)):
    """Relax planar systems together in one batched launch; returns, for
    each checkpoint fraction, the surface-tension sums and the views."""
    B_ = B.Batch([c["params"] for c in cases], [c["solid"] for c in cases], stream=stream)
    for i, c in enumerate(cases):
        B_.init_equilibrium(i, c["rho_a"], c["rho_b"])
    B_.autotune(2, None)  # advances the members: start again afterwards
    for i, c in enumerate(cases):
        B_.init_equilibrium(i, c["rho_a"], c["rho_b"])
    chunk = 1000
    B_.graph_capture(chunk)
    done, out = 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for frac in checkpoints:
        target = int(round(frac * steps))
        while done + chunk <= target:
            B_.graph_replay(1)
            done += chunk
        if target > done:
            B_.step(target - done)
            done = target
            B_.graph_capture(chunk)
        torch.cuda.synchronize()
        out.append((done, [B_.view(i).surface_tension_z()[0] for i in range(len(cases))]))
    sec = time.perf_counter() - t0
    return B_, out, sec


def young(dtype="f64", steps=20000, grid_steps=20000, with_droplets=True, with_grid=True):
    """Contact angles from planar surface tensions (Sec. 4.1, Eq. gammaMechDef
    and Eq. young) and Huang's estimate (Eq. huangSigmaLG), against the
    geometric angle.

    Part 1, g = 0.12 and the nine wall asymmetries of the droplet sweep:
    the A-B lamella and, per asymmetry, the A-wall and B-wall slabs
    (32 x 8 x 128, periodic), relaxed together in one batch; Young's angle
    cos = (gamma_Bw - gamma_Aw) / gamma_AB; Huang's estimate from the bulk A
    densities of the relaxed lamella; the geometric E1/E2 angles of the
    128 x 128 x 64 droplets after 20000 steps.
    The radial tension of a free droplet (64^3, initial radius 16) gives a
    second Young angle with the same wall tensions, and the radial tension
    of each sessile droplet itself (shells about its cap's sphere centre) a
    third, compared with its geometric angle as in Sec. 4.1.
    Part 2, the paper's grid: g = 0.00 .. 0.20 (step 0.02) against the wall
    density eta = 0.00 .. 0.60 (step 0.02) with wall content (0, eta), all
    693 planar systems in one batch.  Young's angle where an A-B interface
    exists (gamma_AB > 1e-6)."""
    stream = torch.cuda.Stream()
    res = {}
    # ---- part 1
    deltas = [float(d) for d in W.THROUGHPUT_DELTAS]
    g = 0.12
    cases = [W.planar_case("AB", g, dtype=dtype)]
    for d in deltas:
        wall = W.asymmetric_wall(d)
        cases += [W.planar_case("Aw", g, wall, dtype=dtype), W.planar_case("Bw", g, wall, dtype=dtype)]
    Bt, snaps, sec = _planar_batch(cases, steps, stream)
    nodes = sum(fluid_nodes(c["solid"]) for c in cases)
    (s_half, gam_half), (s_end, gam) = snaps
    dens = Bt.view(0).density().cpu().numpy()  # (2, nz, ny, nx)
    nz = cases[0]["params"]["nz"]
    rho_in, rho_out = float(dens[0, nz // 2].mean()), float(dens[0, 0].mean())
    g_ab = gam[0] / 2.0
    emit({"exp": "young_planar", "dtype": dtype, "steps": s_end, "gamma_AB": g_ab,
          "gamma_AB_half": gam_half[0] / 2.0, "rho_in": rho_in, "rho_out": rho_out,
          "members": len(cases), "mlups": nodes * s_end / sec / 1e6})
    del Bt
    # radial tension of a free droplet at the same coupling (Eq. mechRadGamma)
    n = 64
    ra, rb = W.sphere_densities(n, 16.0)
    fd = B.Lattice(W.params(n, n, n, g, dtype=dtype), np.zeros((n, n, n), np.uint8), stream=stream)
    fd.init_equilibrium(ra, rb)
    timed_steps(fd, steps, stream)
    g_rad, rs, _, _ = fd.radial_tension([n / 2.0] * 3, n / 2.0 - 5.0, n // 2)
    emit({"exp": "young_radial", "dtype": dtype, "steps": steps, "gamma_AB_radial": g_rad, "R_s": rs})
    del fd
    geo = {}
    if with_droplets:
        for r in sweep(dtype, 20000, "full", deltas, radial=True)["sweep"]:
            geo[r["delta"]] = r
    rows = []
    for j, d in enumerate(deltas):
        gAw, gBw = gam[1 + 2 * j] / 2.0, gam[2 + 2 * j] / 2.0
        p = W.params(8, 8, 8, g, rho_wall=W.asymmetric_wall(d))
        row = {"exp": "young", "delta": d, "gamma_Aw": gAw, "gamma_Bw": gBw, "gamma_AB": g_ab,
               "gamma_Aw_half": gam_half[1 + 2 * j] / 2.0, "gamma_Bw_half": gam_half[2 + 2 * j] / 2.0,
               "theta_young": B.young_angle(gBw, gAw, g_ab),
               "theta_young_radial": B.young_angle(gBw, gAw, g_rad),
               "theta_huang": B.huang_angle(p, rho_in, rho_out)}
        if d in geo:
            row["theta_e1"] = geo[d]["theta_e1"]
            row["theta_e2"] = geo[d]["theta_e2"]
            gs_ = geo[d]["gamma_radial"]
            row["gamma_AB_sessile"] = gs_
            row["R_s_sessile"] = geo[d]["R_s"]
            if gs_ == gs_:  # not NaN
                th = B.young_angle(gBw, gAw, gs_)
                row["theta_young_sessile"] = th
                row["deviation_percent"] = 100.0 * (th - geo[d]["theta_e1"]) / geo[d]["theta_e1"]
        rows.append(emit(row))
    res["g012"] = rows
    if not with_grid:
        return res
    # ---- part 2
    gs = [round(0.02 * i, 2) for i in range(11)]
    etas = [round(0.02 * i, 2) for i in range(31)]
    cases, index = [], {}
    for gg in gs:
        index[(gg, "AB")] = len(cases)
        cases.append(W.planar_case("AB", gg, dtype=dtype))
        for eta in etas:
            for kind in ("Aw", "Bw"):
                index[(gg, eta, kind)] = len(cases)
                cases.append(W.planar_case(kind, gg, (0.0, eta), dtype=dtype))
    Bt, snaps, sec = _planar_batch(cases, grid_steps, stream, checkpoints=(1.0,))
    nodes = sum(fluid_nodes(c["solid"]) for c in cases)
    _, gam = snaps[0]
    del Bt
    table = []
    for gg in gs:
        gab = gam[index[(gg, "AB")]] / 2.0
        line = []
        for eta in etas:
            gAw, gBw = gam[index[(gg, eta, "Aw")]] / 2.0, gam[index[(gg, eta, "Bw")]] / 2.0
            line.append(B.young_angle(gBw, gAw, gab) if gab > 1e-6 else None)
        table.append(emit({"exp": "young_grid", "g": gg, "gamma_AB": gab, "eta": etas, "theta_young": line}))
    res["grid"] = table
    res["grid_perf"] = emit({"exp": "young_grid_perf", "members": len(cases), "steps": grid_steps,
                             "seconds": sec, "mlups": nodes * grid_steps / sec / 1e6})
    return res


def sizes(dtype="f32", etas=(0.1, 0.2, 0.3, 0.35), boxes=((128, 40000), (256, 80000)), g=0.16,
          report_every=10000, stream=None, start="hemisphere", wall="psi", rho_out=0.04):
    """The paper's size/wettability study (Sec. 4): droplets of initial volume
    (L * 70 / 128)^3 -- 70^3 in the 128^3 box, 140^3 in 256^3 -- of A at
    (0.7, rho_out) in B at (rho_out, 0.7), noise 1e-3, seed 0, on one solid
    layer at z = 0 (periodic in z, so that layer is also the ceiling), the
    paper's pseudopotential psi = 1 - exp(-rho), g = 0.16, g_wall = g and
    the paper's single wall parameter eta.  Readings:
      start "hemisphere": a hemisphere of that volume on the wall; "cube": a
        cube of that volume (edge 70 or 140) standing on the wall;
      wall "psi": wall content (0, eta), which species A feels through
        psi(eta); "eta": the wall's pseudopotential itself is eta (Huang's
        G_ads = g eta), i.e. wall content (0, -ln(1 - eta)).
    Reports theta_E1/E2 every report_every steps and, per eta, the relative
    change from the small to the large box."""
    stream = stream or torch.cuda.Stream()
    out = {}
    for L_, steps in boxes:
        edge = 70.0 * L_ / 128.0
        vol = edge ** 3
        radius = (3.0 * vol / (2.0 * np.pi)) ** (1.0 / 3.0)
        solid = W.walls_mask(L_, L_, L_, floor=True, ceiling=False)
        nf = fluid_nodes(solid)
        for eta in etas:
            content = eta if wall == "psi" else -float(np.log1p(-eta))
            p = W.params(L_, L_, L_, g, rho_wall=(0.0, content), psi=1, dtype=dtype)
            if start == "cube":
                ra, rb = W.cube_densities(L_, L_, L_, round(edge), 0, solid, rho_out=rho_out)
            else:
                ra, rb = W.cap_densities(L_, L_, L_, radius, 0.5, solid, rho_out=rho_out)
            lat = B.Lattice(p, solid, stream=stream)
            lat.init_equilibrium(ra, rb)
            cfg = W.ca_cfg(L_, L_)
            done, sec = 0, 0.0
            while done < steps:
                n = min(report_every, steps - done)
                sec += timed_steps(lat, n, stream)
                done += n
                ca = lat.contact_angle(cfg)
                rec = {"exp": "sizes", "box": L_, "eta": eta, "start": start, "wall": wall,
                       "rho_out": rho_out, "dtype": dtype, "step": done, "radius0": radius,
                       "theta_e1": ca["theta_e1"], "theta_e2": ca["theta_e2"], "flags": ca["flags"],
                       "mlups": nf * done / sec / 1e6}
                if ca["flags"] & 32:  # no droplet at the column's first fluid node: where is it?
                    d = lat.density().cpu().numpy()
                    phi = d[0] - d[1]  # (nz, ny, nx)
                    col = np.nonzero(phi[1:, cfg["jc"], cfg["ic"]] > 0)[0]
                    rec["lift"] = {"bottom_on_column": int(col[0]) + 1 if col.size else None,
                                   "top_on_column": int(col[-1]) + 1 if col.size else None,
                                   "droplet_nodes": int(np.count_nonzero(phi > 0)),
                                   "wall_layer_a_nodes": int(np.count_nonzero(phi[1] > 0))}
                emit(rec)
            out[(L_, eta)] = rec
            del lat
            torch.cuda.empty_cache()
    small, large = boxes[0][0], boxes[-1][0]
    for eta in etas:
        if small != large and (small, eta) in out and (large, eta) in out:
            a, b = out[(small, eta)]["theta_e1"], out[(large, eta)]["theta_e1"]
            emit({"exp": "sizes_change", "eta": eta, "start": start, "wall": wall,
                  "theta_small": a, "theta_large": b, "relative_change_pct": 100.0 * (b - a) / a})
    return out


def adjoint_cost(reps=20):
    """Cost of the reverse step against the forward step, FP64 and FP32, on
    the gradient box (64 x 64 x 48) and the throughput box (128 x 128 x 64):
    reps plain adjoint steps (moments pass included), reps forward
    steps, then a one-level checkpointed gradient over 2 * reps steps with
    segments of reps steps, with and without the moment cache (the backward
    sweeps give the same gradient bit for bit).  Times from HIP events on
    the lattice's stream; run under rocprofv3 for per-kernel times."""
    stream = torch.cuda.Stream()
    out = []
    for dt in ("f64", "f32"):
        for name, c in (("64x64x48", W.config_gradient(dtype=dt)),
                        ("128x128x64", W.config_throughput(delta=0.2, dtype=dt))):
            L = B.Lattice(c["params"], c["solid"], adjoint=True, stream=stream)
            L.init_equilibrium(c["rho_a"], c["rho_b"])
            L.step(10)
            st = L.get_state(blocked=True)
            a = L.ca_seed(c["ca"], 1.0, blocked=True)
            b = torch.empty_like(a)
            L.adjoint_reset()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            # direct C calls (accumulating on the device, no synchronisation)
            ps, pl = B._ptr(st), [B._ptr(a), B._ptr(b)]
            torch.cuda.synchronize()
            B.check(B.lib().scd_adjoint_step(L.h, ps, pl[0], pl[1], None))
            e[0].record(stream)
            for r in range(reps):
                B.check(B.lib().scd_adjoint_step(L.h, ps, pl[r % 2], pl[1 - r % 2], None))
            e[1].record(stream)
            e[2].record(stream)
            L.step(reps)
            e[3].record(stream)
            torch.cuda.synchronize()
            adj, fwd = e[0].elapsed_time(e[1]) / reps, e[2].elapsed_time(e[3]) / reps
            del L, st, a, b
            sweeps = {}
            for cache in (False, True):
                s = GradSetup(c["params"], c["solid"], c["rho_a"], c["rho_b"], 2 * reps, reps, c["ca"],
                              120.0, stream=stream, moment_cache=cache)
                s.forward()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g = s.backward()
                torch.cuda.synchronize()
                sweeps[cache] = (time.perf_counter() - t0, g)
                del s
            torch.cuda.empty_cache()
            out.append(emit({"exp": "adjoint_cost", "dtype": dt, "box": name, "forward_us": fwd * 1e3,
                             "adjoint_us": adj * 1e3, "ratio": adj / fwd,
                             "backward_sweep_s": sweeps[False][0], "backward_sweep_cached_s": sweeps[True][0],
                             "same_gradient": sweeps[False][1] == sweeps[True][1]}))
    return out


def posts(steps=100000, adjoint_steps=1000, dtype="f32", K1=100, K2=10, report_every=10000, levels=0):
    """Droplet on a square array of posts (width 6, pitch 12, height 12) in
    a 384 x 384 x 192 box, wall asymmetry -0.3; then one adjoint pass over
    the last adjoint_steps steps: one level of checkpoints every K1 steps
    when its memory fits, else two levels (K2 inside each segment); levels
    1 or 2 forces the choice."""
    c = W.config_posts(dtype=dtype)
    stream = torch.cuda.Stream()
    L = B.Lattice(c["params"], c["solid"], adjoint=adjoint_steps > 0, stream=stream)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    nf = fluid_nodes(c["solid"])
    best, ms = L.autotune(6, None)
    L.init_equilibrium(c["rho_a"], c["rho_b"])
    # the mass-drift watchdog at the suggested tolerance of the dtype: the
    # run goes on, each report says whether the drift exceeds it
    L.set_mass_watchdog(1e-5 if dtype == "f32" else 1e-10)
    L.observables(raise_drift=False)  # the reference masses
    emit({"exp": "posts", "fluid_nodes": nf, "tile": list(best), "tune_ms": ms})
    run = steps - adjoint_steps
    done, total_sec = 0, 0.0
    while done < run:
        n = min(report_every, run - done)
        total_sec += timed_steps(L, n, stream)
        done += n
        ca = L.contact_angle(c["ca"])
        obs = L.observables(raise_nonfinite=False, raise_drift=False)
        emit({"exp": "posts", "step": L.step_count, "theta_e1": ca["theta_e1"], "theta_e2": ca["theta_e2"],
              "flags": ca["flags"], "mass": list(obs["mass"]), "finite": obs["finite"],
              "mass_drift": list(obs["drift"]), "drift_flagged": obs["status"] == B.SCD_EDRIFT,
              "mlups": nf * done / total_sec / 1e6})
    out = {"mlups": nf * done / total_sec / 1e6, "steps": done}
    if adjoint_steps > 0:
        # one level of checkpoints every K1 steps when its memory fits (the
        # moment cache serves the adjoint, so a segment keeps its moments,
        # 8 x N reals per step, and only two recomputed states), else a
        # second level every K2 steps inside each segment.  Only the
        # multi-plane marches write the moments: the gradient's forward and
        # recomputed steps use the dtype's default one, at the tuned chunk.
        L.set_tile(B.variant_index(64, 4, 6, 2) if dtype == "f32" else B.variant_index(32, 4, 7, 1), best[1])
        state = L.pop_bytes
        mom = 8 * int(np.prod(L.shape)) * (4 if dtype == "f32" else 8)
        one_level = (-(-adjoint_steps // K1) + 4) * state + (K1 - 1) * mom
        free, _ = torch.cuda.mem_get_info()
        inner = None if one_level < 0.85 * free else K2
        if levels:  # forced
            inner = None if levels == 1 else K2
        emit({"exp": "posts_adjoint_plan", "levels": 1 if inner is None else 2, "K1": K1, "K2": inner,
              "tile": list(L.tile()),
              "one_level_bytes": one_level, "free_bytes": free})
        setup = GradSetup(c["params"], c["solid"], None, None, adjoint_steps, K1, c["ca"], 150.0,
                          lattice=L, inner=inner)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = setup.forward()
        t1 = time.perf_counter()
        g = setup.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out.update(emit({"exp": "posts_adjoint", "steps": adjoint_steps, "levels": 1 if inner is None else 2,
                         "theta_e2": setup.theta, "loss": loss,
                         "grad": g, "forward_s": t1 - t0, "backward_s": t2 - t1,
                         "backward_over_forward": (t2 - t1) / (t1 - t0)}))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["sweep", "fit", "posts", "young", "sizes", "adjoint"])
    ap.add_argument("--box", type=int, default=None, help="sizes: run one box edge only")
    ap.add_argument("--dtype", default=None, help="f64 or f32 (posts default f32, others f64)")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--sweep-box", default="full")
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--no-grid", action="store_true", help="young: skip the 693-system grid")
    ap.add_argument("--start", default="hemisphere", choices=["hemisphere", "cube"], help="sizes")
    ap.add_argument("--wall", default="psi", choices=["psi", "eta"], help="sizes")
    ap.add_argument("--rho-out", type=float, default=0.04, help="sizes: minority density")
    ap.add_argument("--etas", default=None, help="sizes: comma-separated wall parameters")
    ap.add_argument("--levels", type=int, default=0, help="posts: checkpoint levels (0: one if it fits)")
    a = ap.parse_args()
    if a.what == "sweep":
        sweep(a.dtype or "f64", a.steps or 20000, a.sweep_box)
    elif a.what == "fit":
        fit(a.dtype or "f64", a.iters, a.steps or 2000)
    elif a.what == "sizes":
        boxes = ((128, 40000), (256, 80000))
        if a.box:  # one box edge (the paper checks 32, 64, 128 and 256)
            boxes = ((a.box, 80000 if a.box > 128 else 40000),)
        if a.steps:
            boxes = tuple((b[0], a.steps) for b in boxes)
        etas = tuple(float(e) for e in a.etas.split(",")) if a.etas else (0.1, 0.2, 0.3, 0.35)
        sizes(a.dtype or "f32", etas=etas, boxes=boxes, start=a.start, wall=a.wall, rho_out=a.rho_out)
    elif a.what == "young":
        young(a.dtype or "f64", a.steps or 20000, with_grid=not a.no_grid)
    elif a.what == "adjoint":
        adjoint_cost()
    else:
        posts(a.steps or 100000, a.adjoint_steps, a.dtype or "f32", levels=a.levels)


if __name__ == "__main__":
    main()
