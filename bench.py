#!/usr/bin/env python3
"""Throughput of the PNCG time step on one MI355X.

Workload: the ~110k-tet pile (24 voxelised spheres and tori dropped into a
0.4 m box; synthetic, seeded; dhat = 5e-4 m, h = 1/30 s, at most 25 PNCG
iterations per frame, dE tolerance 1e-3), stepped in the mixed float32 /
float64 form.  The pile first falls for S untimed frames (default 150:
input preparation, so that the timed frames are those of a pile at rest on
its floor and on itself, frames S+W .. S+W+K of the configured 200), then W
untimed warm-up frames, then K timed frames in one pncg_run_dev call.  The
primary value is PNCG iterations per second over the K frames; ms per frame
is reported beside it.  The same K frames are then run again from the saved
state through one pncg_step_dev call per frame, and again with per-launch
HIP events (profiling): the segmented pair scatter makes all three passes
follow the same trajectory bit for bit.

One JSON line is printed.  Besides the throughput it carries:
  roofline      the dominant kernel's algorithmic bytes per launch (the
                per-tet / per-vertex / per-pair byte model) over its average
                launch time: from HIP events on the library's stream in the
                profiled pass, and from the rocprofv3 summary committed in
                profiles/ (when it was made from the current kernel sources)
  iter_roofline the whole iteration's algorithmic bytes times iterations/s
  fp64          the plain float64 form over the same frames
  packed        the contact-rich packed pile (the same 24 shapes stacked with
                sub-dhat gaps, ~25k point-triangle / edge-edge pairs active)
  cpu_baseline  the float64 CPU oracle on bounded samples: pile iterations
                (headline), batched scene steps over the host's cores, and one
                adjoint step of the 30,000-tet bar
  batched       256 independent scenes (500-8000 tets each, 721k tets in
                all) stepped together by the batched kernel, several steps per
                captured graph: scene-steps/s and the kernel's byte rate
  adjoint       the differentiable rollout of the 30,000-tet bar (30 steps,
                checkpoints every 5): backward wall time per step
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
# Algorithmic bytes (compulsory traffic: each array touched once per pass),
# per tet, per vertex, per active point-triangle / edge-edge pair and per
# candidate pair, for one PNCG iteration: two element passes (index 16 B,
# D_m^-1 36 / 72 B, V mu and V lam 8 / 16 B), the vertex arrays of the
# gradient pass (x, xt, m read; g, diag written), of the direction pass (g,
# g_prev, diag, p_prev read; p written), of the curvature pass (x, p) and of
# the update (x, p read; x written); a contact record written and read.
BYTES = {
    "iter": {"mixed": (120, 232, 144, 8), "fp64": (208, 344, 144, 8)},
}
# The same model split over the kernels of one iteration (per tet, per vertex,
# per active pair, per candidate).
KERNEL_BYTES = {
    # grad (first launch of an iteration, with the pair pass and the pending
    # update folded in): element pass (60 / 104 B per tet); per vertex x_prev
    # read and x written (24 each), xt (24), m (8), g_prev and p read and g
    # and P g written (4 vectors of 12 / 24 B); per active pair its contact
    # record written and read (144 B); per candidate the pair (8 B)
    "grad": {"mixed": (60, 24 + 24 + 24 + 8 + 12 * 4, 144, 8), "fp64": (104, 24 + 24 + 24 + 8 + 24 * 4, 144, 8)},
    # dir: element pass; per vertex x (24), P g, p_prev, p_new (12 / 24 each),
    # mass (8); candidate pair (8)
    "dir": {"mixed": (60, 24 + 12 + 12 + 12 + 8, 0, 8), "fp64": (104, 24 + 24 + 24 + 24 + 8, 0, 8)},
    # narrow: pending update (x_prev, p read, x written) per vertex; the
    # written half of each active pair's record (72 B); candidate pair (8)
    "narrow": {"mixed": (0, 24 + 12 + 24, 72, 8), "fp64": (0, 24 + 24 + 24, 72, 8)},
}
SETTLE_FRAMES = 150        # frames the pile falls before the warm-up and timed frames


# kernels of the mixed single-scene path, by the name rocprofv3 records
# the Neo-Hookean, unsplit instantiations the pile runs (template arguments:
# real type, sweep mode, split, model, ...)
KERNEL_NAMES = {"grad": "k_grad<float, 0, false, 0, true,", "dir": "k_dir<float, false, 0,",
                "narrow": "k_narrow<float, false>"}
KERNEL_TIMES = os.path.join(ROOT, "profiles", "kernel_times.json")
CALIB_BYTES = 256 << 20          # the calibration copy reads and writes this many bytes
SOLVER_SOURCES = ("solver_kernels.hip", "sweep_common.h", "device_math.h", "internal.h")


def solver_source_hash():
    """sha256 over the sources of the single-scene solver kernels: traffic
    figures measured on other sources are not reported."""
    import hashlib
    hsh = hashlib.sha256()
    for f in SOLVER_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_08001_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def traffic_from_csv(fetch_csv, write_csv, out_path):
    """HBM bytes per launch of each solver kernel from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by the
    ratio of the calibration copy's known bytes to what the counter read for
    it."""
    import csv
    import re

    def per_kernel(path, counter):
        vals = {}
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                name = row["Kernel_Name"]
                key = None
                for k, pat in KERNEL_NAMES.items():
                    if pat in name:
                        key = k
                if key is None and re.search(r"copyBuffer|elementwise", name):
                    key = "copy"
                if key is not None:
                    vals.setdefault(key, []).append(float(row["Counter_Value"]) * 1024.0)
        out = {}
        for k, v in vals.items():
            v = np.sort(np.asarray(v))
            # the calibration copies are the three largest copy dispatches; a
            # solver kernel's launches vary little except those that return
            # at once after the step has stopped, so its median is taken
            out[k] = float(np.mean(v[-3:])) if k == "copy" else float(np.median(v))
        return out, {k: len(v) for k, v in vals.items()}

    fetch, nf = per_kernel(fetch_csv, "FETCH_SIZE")
    write, nw = per_kernel(write_csv, "WRITE_SIZE")
    f_scale = CALIB_BYTES / fetch["copy"]
    w_scale = CALIB_BYTES / write["copy"]
    out = {"source_sha256": solver_source_hash(),
           "calibration": {"copy_bytes_each_way": CALIB_BYTES, "fetch_counter_bytes": fetch["copy"],
                           "write_counter_bytes": write["copy"], "fetch_scale": f_scale, "write_scale": w_scale},
           "pile": {}, "detail": {}}
    for k in KERNEL_NAMES:
        if k in fetch and k in write:
            fb, wb = fetch[k] * f_scale, write[k] * w_scale
            out["pile"][k] = int(round(fb + wb))
            out["detail"][k] = {"fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)),
                                "dispatches": [nf[k], nw[k]]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def calibration_copy():
    import torch
    src = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def _clocks():
    """Host clocks (ns) that a profiler's timestamps may use, to mark a window."""
    out = {"monotonic": time.monotonic_ns()}
    for name in ("CLOCK_BOOTTIME", "CLOCK_MONOTONIC_RAW"):
        if hasattr(time, name):
            out[name.lower()] = time.clock_gettime_ns(getattr(time, name))
    return out


def trace_gaps(trace_csv, window_json, top=12):
    """Device busy and idle time inside the timed window of a headline run,
    from a rocprofv3 --kernel-trace CSV and the window bench.py wrote with
    --window-out: the host clock whose window holds the most solver
    launches is taken as the trace's time base.  Returns the span, the sum
    of kernel durations, the idle share, idle per frame and per iteration,
    and the largest gaps by the pair of kernels around them."""
    import csv
    import re
    win = json.load(open(window_json))
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))

    def short(n):
        n = n.replace("void ", "").replace("(anonymous namespace)::", "")
        i = n.find("(")
        return re.sub(r"pncg::", "", n[:i] if i > 0 else n)

    best = None
    for clock in win["start"]:
        t0, t1 = win["start"][clock], win["end"][clock]
        sel = [r for r in rows if int(r["Start_Timestamp"]) >= t0 and int(r["End_Timestamp"]) <= t1]
        n = sum(1 for r in sel if "k_grad" in r["Kernel_Name"])
        if best is None or n > best[0]:
            best = (n, clock, sel)
    n_grad, clock, sel = best
    if len(sel) < 2:
        raise SystemExit("no kernel of the trace falls inside the window")
    span = int(sel[-1]["End_Timestamp"]) - int(sel[0]["Start_Timestamp"])
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sel)
    gaps = {}
    for a, b in zip(sel, sel[1:]):
        g = max(int(b["Start_Timestamp"]) - int(a["End_Timestamp"]), 0)
        key = short(a["Kernel_Name"]) + " -> " + short(b["Kernel_Name"])
        c = gaps.setdefault(key, [0, 0])
        c[0] += 1
        c[1] += g
    idle = span - busy
    top_gaps = sorted(gaps.items(), key=lambda kv: -kv[1][1])[:top]
    return {"clock": clock, "kernels": len(sel), "grad_launches": n_grad, "frames": win["frames"],
            "iters": win["iters"], "span_us": round(span / 1e3, 1), "busy_us": round(busy / 1e3, 1),
            "idle_frac": round(idle / span, 4), "idle_us_per_frame": round(idle / 1e3 / win["frames"], 1),
            "idle_us_per_iter": round(idle / 1e3 / max(win["iters"], 1), 2),
            "us_per_iter": round(span / 1e3 / max(win["iters"], 1), 2),
            "top_gaps": [{"between": k, "count": c, "total_us": round(t / 1e3, 1), "mean_us": round(t / 1e3 / c, 2)}
                         for k, (c, t) in top_gaps]}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup_ctx(sc, precision, model="nh"):
    import paper_2405_08001_amd as P
    # the library runs on torch's current stream (see main), so its inputs
    # need no host-side wait
    ctx = P.Context(0, P.MIXED if precision == "mixed" else P.FP64, stream=_torch_stream())
    if model != "nh":
        ctx.pncg_set_model(model)
    ctx.pncg_set_mesh(sc.X, sc.tets, sc.tris, sc.edges, sc.object_id)
    ctx.pncg_set_material(sc.E, sc.nu, sc.rho)
    ctx.pncg_set_contact(sc.dhat, sc.kappa, sc.cell, sc.planes,
                         (P.CONTACT_SELF if sc.self_contact else 0) | P.CONTACT_REST_EXCLUDE)
    ctx.pncg_set_solver(sc.iter_max, sc.eps, P.TERM_DELTA_E, sc.gravity, 0)
    if len(sc.fixed):
        ctx.pncg_set_dirichlet(sc.fixed, sc.X[sc.fixed])
    return ctx


def _torch_stream():
    """Handle of torch's current stream, or None for its default stream (the
    library then uses a stream of its own)."""
    import torch
    h = torch.cuda.current_stream().cuda_stream
    return h or None


def run(sc, precision, settle, warmup, steps, model="nh", profile=True, per_call=True):
    """S settle frames and W warm-up frames (untimed), then K timed frames in
    one pncg_run_dev call (the state stays on the device and no host round
    trip separates the steps); then the same K frames from the saved state
    through one pncg_step_dev call per frame from Python, and again with
    per-launch HIP events (profiling on)."""
    import torch
    ctx = setup_ctx(sc, precision, model)
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.x0, dtype=torch.float64, device=dev)
    v = torch.tensor(sc.v0, dtype=torch.float64, device=dev)
    if settle + warmup > 0:
        ctx.pncg_run_dev(x, v, sc.h, settle + warmup)
    xs, vs = x.clone(), v.clone()
    state = (x.cpu().numpy().copy(), v.cpu().numpy().copy())
    # each pass below starts without a candidate list carried from earlier
    # steps (re-applying the default tuning drops it), so that all three run
    # the same trajectory bit for bit
    ctx.pncg_set_tuning(0.0, 0)
    torch.cuda.synchronize()
    clocks0 = _clocks()
    t0 = time.perf_counter()
    sts, _ = ctx.pncg_run_dev(x, v, sc.h, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    clocks1 = _clocks()
    x_end = x.cpu().numpy().copy()
    iters = sum(st["iters"] for st in sts)
    act = sum(st["n_active"] for st in sts)
    cand = sum(st["n_candidates"] for st in sts)
    reb = sum(st["rebuilds"] for st in sts)
    out = dict(seconds=dt, iters=iters, frames=steps, mean_active=act / steps, mean_cand=cand / steps,
               rebuilds_per_frame=reb / steps, state=state, stats=sts,
               window={"start": clocks0, "end": clocks1, "frames": steps, "iters": iters})
    if per_call:
        # the same frames through one Python call per step
        x.copy_(xs)
        v.copy_(vs)
        ctx.pncg_set_tuning(0.0, 0)
        x2, v2 = torch.empty_like(x), torch.empty_like(v)
        it_pc = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = ctx.pncg_step_dev(x, v, sc.h, x2, v2)
            x, x2, v, v2 = x2, x, v2, v
            it_pc += st["iters"]
        torch.cuda.synchronize()
        dt_pc = time.perf_counter() - t0
        out["per_call"] = {"iters_per_s": round(it_pc / dt_pc, 1), "ms_per_frame": round(1e3 * dt_pc / steps, 4),
                           "same_trajectory": bool(np.array_equal(x.cpu().numpy(), x_end))}
    if profile:
        # the same frames with HIP events around every launch
        x.copy_(xs)
        v.copy_(vs)
        ctx.pncg_set_tuning(0.0, 0)
        ctx.pncg_set_profiling(True)
        ctx.pncg_run_dev(x, v, sc.h, steps)
        out["prof"] = ctx.pncg_get_profile()
        ctx.pncg_set_profiling(False)
        out["prof_same_trajectory"] = bool(np.array_equal(x.cpu().numpy(), x_end))
    out["dmin"], out["jmin"] = ctx.pncg_min_distance(x_end)
    ctx.close()
    return out


def run_host_io(sc, state, frames=20):
    """The pile through pncg_step with host arrays (mixed form, from the state
    after warm-up): x and v go to the device and x', v' come back every
    step, so the rate includes the PCIe transfers."""
    ctx = setup_ctx(sc, "mixed")
    x, v = state[0].copy(), state[1].copy()
    its = 0
    t0 = time.perf_counter()
    for _ in range(frames):
        x, v, st = ctx.pncg_step(x, v, sc.h)
        its += st["iters"]
    dt = time.perf_counter() - t0
    ctx.close()
    return {"frames": frames, "iters_per_s": round(its / dt, 1), "ms_per_frame": round(1e3 * dt / frames, 4),
            "bytes_per_frame_over_pcie": 4 * 3 * 8 * sc.nV}


def _solve_once(sc, prec, x0, v0, iters, eps, term, flags=0, dhat=None):
    """One step of scene sc from (x0, v0) with the given stopping rule (and
    optionally another dhat): (x, v, stats, seconds)."""
    import torch
    import paper_2405_08001_amd as P
    dev = torch.device("cuda:0")
    ctx = setup_ctx(sc, prec)
    if dhat is not None:
        ctx.pncg_set_contact(dhat, sc.kappa, 0.0, sc.planes,
                             (P.CONTACT_SELF if sc.self_contact else 0) | P.CONTACT_REST_EXCLUDE)
    ctx.pncg_set_solver(iters, eps, term, sc.gravity, flags)
    x = torch.tensor(x0, device=dev)
    v = torch.tensor(v0, device=dev)
    xo, vo = torch.empty_like(x), torch.empty_like(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.pncg_step_dev(x, v, sc.h, xo, vo)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return xo.cpu().numpy(), vo.cpu().numpy(), st, dt


REF_TOL = 1e-11      # a study's reference minimiser: ||g|| <= REF_TOL ||g_0|| ...
REF_OK = 1e-9        # ... or, where rounding stops it short, at least this


def _reference(sc, x0, v0, dhat=None, tol=REF_TOL, cap=60000, flags=0):
    """x* of the step from (x0, v0): float64 Dai-Kou to ||g|| <= tol ||g_0||
    (at most cap iterations) and how far it got.  A looser gradient rule is
    not enough on contact steps: at 1e-7 the unsplit and the split solves of
    the stacked cubes stop 24 % (relative to |x* - x^t|) apart, at 1e-11
    2e-4 apart, so the studies use 1e-11 (the unsplit iteration gets there
    in far fewer iterations than the split one)."""
    import paper_2405_08001_amd as P
    xs, _, sref, _ = _solve_once(sc, "fp64", x0, v0, cap, tol, P.TERM_GRAD_REL, flags, dhat)
    ratio = sref["g_norm"] / sref["g0_norm"]
    return xs, {"reference_iters": int(sref["iters"]), "reference_grad_ratio": float(f"{ratio:.3e}"),
                "reference_converged": bool(ratio <= REF_OK)}


def _convergence(sc, prec, x0, v0, budgets, flags, dhat, xs):
    """Error of x after K iterations (each K in budgets) against the step's
    minimiser xs, relative to |xs - x^t|; iterations/s at the largest K."""
    import paper_2405_08001_amd as P
    scale = float(np.linalg.norm(xs - x0))
    errs, ips, act = [], 0.0, 0
    for K in budgets:
        xk, _, st, dt = _solve_once(sc, prec, x0, v0, K, 0.0, P.TERM_DELTA_E, flags, dhat)
        errs.append(float(f"{float(np.linalg.norm(xk - xs)) / scale:.3e}"))
        if K == budgets[-1]:
            ips, act = st["iters"] / dt, st["n_active"]
    return {"rel_error": errs, "iters_per_s": round(ips, 1), "active_pairs": int(act)}


def _study_cases():
    """Contact states for the convergence studies whose step minimiser the
    float64 reference reaches (||g|| <= 1e-11 ||g_0||, or 1e-9 where rounding
    stops it; a case whose reference falls short reports no errors): the cube resting on its floor after 12
    steps (plane barriers), the stacked cubes with the top one moving down
    into its sub-dhat gap (point-triangle, edge-edge and plane barriers), and
    the stacked bars (30,720 tets, about 5,400 pairs active at the start)."""
    import paper_2405_08001_amd as P
    import scenes
    cube = scenes.cube_scene()
    x, v = cube.x0.copy(), cube.v0.copy()
    for _ in range(12):
        x, v, _, _ = _solve_once(cube, "fp64", x, v, 2000, cube.eps, P.TERM_GRAD_REL)
    stack = scenes.small_contact_scene()
    sv = np.zeros_like(stack.X)
    sv[stack.object_id == 1, 2] = -0.05
    bars = scenes.stacked_bars_scene()
    return {"cube-resting": (cube, x, v), "stacked-cubes": (stack, stack.X.copy(), sv),
            "stacked-bars": (bars, bars.x0.copy(), bars.v0.copy())}


def _study(sc, prec, x0, v0, budgets, runs, dhat=None):
    """The reference of one case, then the error curve of each named run
    (flags) if the reference converged."""
    xs, ref = _reference(sc, x0, v0, dhat)
    res = {"precision": prec, "budgets": list(budgets), "reference_tol": REF_TOL, "reference_ok": REF_OK}
    res.update(ref)
    if not ref["reference_converged"]:
        res["note"] = "reference not converged: no errors reported"
        return res
    for name, flag in runs.items():
        res[name] = _convergence(sc, prec, x0, v0, budgets, flag, dhat, xs)
    return res


def run_beta_ablation(budgets=(25, 100, 400, 1600)):
    """The beta rules of the ablation (Sec. 7.1) on synthetic contact states:
    the error after K iterations of one step against the step's minimiser,
    float64, for each rule."""
    import paper_2405_08001_amd as P
    out = {}
    for name, (sc, x0, v0) in _study_cases().items():
        r = _study(sc, "fp64", x0, v0, budgets, dict(P.BETA_RULES))
        out[name] = {"reference": {k: r[k] for k in ("reference_iters", "reference_grad_ratio",
                                                     "reference_converged")},
                     "rules": {k: r[k] for k in P.BETA_RULES if k in r}}
        if "note" in r:
            out[name]["note"] = r["note"]
    return out


def run_split(budgets=(25, 100, 400, 1600)):
    """Splitting computation (Sec. 5.2) on the two-object contact states:
    the error after K iterations against the step's minimiser (the same
    energy either way), split and unsplit, float64 and mixed."""
    import paper_2405_08001_amd as P
    out = {"budgets": list(budgets), "reference_tol": REF_TOL}
    for name, (sc, x0, v0) in _study_cases().items():
        if len(np.unique(sc.object_id)) < 2:
            continue
        for prec in ("fp64", "mixed"):
            out[f"{name}/{prec}"] = _study(sc, prec, x0, v0, budgets,
                                            {"unsplit": 0, "split": P.SPLIT_OBJECTS})
    return out


def run_materials(sc, warmup=0, steps=30, models=("snh", "arap", "fcr"), batched=True,
                  adjoint_model="fcr"):
    """The pile as configured under each other material model (mixed form):
    iteration rate, frame time, iterations per frame, and the sweep's
    roofline (its algorithmic bytes do not depend on the model); the
    256-scene batch under each model (10 graph-captured steps); and the
    differentiable 30,000-tet rollout under one corotated model."""
    out = {"frames_settle": SETTLE_FRAMES, "frames_warmup": warmup, "frames_timed": steps}
    kt, kv, ka, kq = KERNEL_BYTES["grad"]["mixed"]
    for model in models:
        try:
            r = run(sc, "mixed", SETTLE_FRAMES, warmup, steps, model=model, per_call=False)
        except Exception as e:  # a model whose trajectory leaves its domain
            out[model] = {"error": str(e)}
            continue
        ips = r["iters"] / r["seconds"]
        prof = {k: v for k, v in r["prof"].items() if v[1] > 0}
        gus = prof["grad"][0] / prof["grad"][1]
        gb = kt * sc.nT + kv * sc.nV + ka * r["mean_active"] + kq * r["mean_cand"]
        out[model] = {"iters_per_s": round(ips, 1), "ms_per_frame": round(1e3 * r["seconds"] / r["frames"], 4),
                      "iters_per_frame": round(r["iters"] / r["frames"], 2),
                      "grad_us": round(gus, 3), "dir_us": round(prof["dir"][0] / prof["dir"][1], 3),
                      "grad_frac": round(gb / (gus * 1e-6) / HBM_PEAK, 4),
                      "min_distance_after": r["dmin"], "min_detF_after": r["jmin"]}
        if batched:
            bb = run_batched(10, 10, model=model)
            out[model]["batched"] = {k: bb[k] for k in ("scene_steps_per_s", "ms_per_batch_step",
                                                         "mean_iters_per_scene_step", "block", "max_team")}
    if adjoint_model:
        a = run_adjoint(model=adjoint_model)
        out[adjoint_model]["adjoint"] = {k: a[k] for k in ("adjoint_ms_per_step", "forward_ms_per_step",
                                                            "mean_forward_iters", "mean_cg_iters", "max_cg_iters")}
    return out


def run_dhat_strategy(fractions=(0.3, 0.5, 0.7), budgets=(25, 100, 400, 1600)):
    """The larger-dhat strategy (Sec. 5.1) on the stacked cubes, float64:
    dhat at 30/50/70 % of the mean boundary edge (same-object pairs closer
    than 1.5 dhat at rest excluded) against the configured dhat.  The
    strategy is a setting of the whole simulation, so each dhat gets the
    contact state it would keep: the cubes stacked with a gap of 0.4 dhat,
    the lower one 0.4 dhat above the floor, the upper one moving down at
    5 cm/s; one step from there against its own minimiser (the problem
    changes with dhat)."""
    import paper_2405_08001_amd as P
    import scenes
    base = scenes.small_contact_scene()
    ctx = setup_ctx(base, "fp64")
    lbar = ctx.pncg_mean_boundary_edge()
    ctx.close()
    out = {"scene": "stacked-cubes, gaps 0.4 dhat", "mean_boundary_edge": lbar, "budgets": list(budgets),
           "reference_tol": REF_TOL, "dhat": {}}
    for label, dh in [("configured", base.dhat)] + [(f"{f:.1f}*edge", f * lbar) for f in fractions]:
        sc = scenes.small_contact_scene(gap=0.4 * dh, dhat=dh)
        x0 = sc.X.copy()
        x0[:, 2] += 0.4 * dh - x0[:, 2].min()
        v0 = np.zeros_like(x0)
        v0[sc.object_id == 1, 2] = -0.05
        try:
            r = _study(sc, "fp64", x0, v0, budgets, {"pncg": 0}, dh)
            r["dhat"] = dh
            if "pncg" in r:
                r.update(r.pop("pncg"))
        except P.PncgError as e:      # e.g. a tet inverted on the way (no inversion guard, reading S4)
            r = {"dhat": dh, "error": str(e)}
        out["dhat"][label] = r
    return out


def run_batched(steps, warmup, model="nh", state_out=None):
    """The 256-scene batch, mixed precision: W eager steps (the scenes fall
    onto their planes), then K steps as one captured graph.  state_out: a
    directory that receives the state after the warm-up steps."""
    import torch
    import paper_2405_08001_amd as P
    import scenes
    scs = scenes.batched_scenes()
    b = scenes.pack_batch(scs)
    bt = P.Batch(b["vert_off"], b["X"], b["tet_off"], b["tets"], b["tri_off"], b["tris"], b["E"], b["nu"], b["rho"],
                 b["planes"], precision=P.MIXED)
    if model != "nh":
        bt.pncg_batch_set_model(model)
    s0 = scs[0]
    bt.pncg_batch_set_params(s0.dhat, s0.kappa, s0.iter_max, s0.eps, P.TERM_DELTA_E, s0.gravity, 0)
    dev = torch.device("cuda:0")
    x = torch.tensor(b["x"], dtype=torch.float64, device=dev)
    v = torch.tensor(b["v"], dtype=torch.float64, device=dev)
    bt.pncg_batch_run(x, v, s0.h, warmup)
    if state_out:
        np.savez(os.path.join(state_out, "batch_state.npz"), x=x.cpu().numpy(), v=v.cpu().numpy(),
                 vert_off=np.asarray(b["vert_off"]))
    block = bt.pncg_batch_autotune(x, v, s0.h, 2)     # on the state the timed steps start from
    cfg = bt.pncg_batch_get_config()
    _, _, tot0 = bt.pncg_batch_stats()
    bt.pncg_batch_run(x, v, s0.h, steps)      # captures the graph
    _, _, tot1 = bt.pncg_batch_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.pncg_batch_run(x, v, s0.h, steps)      # replays it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, _, tot2 = bt.pncg_batch_stats()
    it = (tot2 - tot1).astype(np.float64)
    T = np.diff(b["tet_off"]).astype(np.float64)
    V = np.diff(b["vert_off"]).astype(np.float64)
    bt_, bv_, _, _ = BYTES["iter"]["mixed"]
    nbytes = float(np.sum(it * (bt_ * T + bv_ * V)))
    xz = x[:, 2].min().item()
    bt.close()
    return {"scenes": len(scs), "tets": int(T.sum()), "steps_timed": steps, "steps_warmup": warmup,
            "block": block, "lds_staging": cfg["lds"], "max_team": cfg["max_team"], "teams": cfg["teams"],
            "scene_steps_per_s": round(len(scs) * steps / dt, 1),
            "ms_per_batch_step": round(1e3 * dt / steps, 4),
            "mean_iters_per_scene_step": round(float(it.sum()) / (len(scs) * steps), 2),
            "iters_per_s": round(float(it.sum()) / dt, 1),
            "roofline": {"bound": "hbm", "kernel": "batch_step", "achieved": round(nbytes / dt / 1e9, 1),
                         "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(nbytes / dt / HBM_PEAK, 4),
                         "bytes_per_launch": int(nbytes / steps)},
            "min_z_after": xz, "dtype": "f32+f64"}


def run_adjoint(steps=30, checkpoint=5, model="nh"):
    """Loss ||x_T - x_target||^2 of the 30,000-tet bar over 30 steps; the
    target is the forward result under a second seeded modulus field."""
    import torch
    import paper_2405_08001_amd as P
    import scenes
    sc = scenes.diff_bar_scene(seed=4)
    tgt = scenes.diff_bar_scene(seed=5)
    ctx = setup_ctx(sc, "fp64", model)
    ctx.pncg_set_solver(sc.iter_max, sc.eps, P.TERM_GRAD_ABS, sc.gravity, 0)
    sim = P.Simulation(ctx, sc.nu, sc.rho, sc.h, steps, checkpoint=checkpoint, cg_tol=1e-10, cg_max=20000)
    dev = torch.device("cuda:0")
    x0 = torch.tensor(sc.x0, dtype=torch.float64, device=dev)
    v0 = torch.tensor(sc.v0, dtype=torch.float64, device=dev)
    with torch.no_grad():
        x_tgt, _ = P.simulate(torch.tensor(tgt.E), x0, v0, sim)
    # one untimed rollout and backward pass first, so that the timed pair
    # excludes the one-time loading of torch's loss and autograd kernels
    Ew = torch.tensor(sc.E, dtype=torch.float64, requires_grad=True)
    xw, _ = P.simulate(Ew, x0, v0, sim)
    ((xw - x_tgt) ** 2).sum().backward()
    E = torch.tensor(sc.E, dtype=torch.float64, requires_grad=True)
    sim.recomputed_steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xT, _ = P.simulate(E, x0, v0, sim)
    loss = ((xT - x_tgt) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd_iters = [s["iters"] for s in sim.forward_stats]
    cg = [s["cg_iters"] for s in sim.adjoint_stats]
    ctx.close()
    return {"workload": "bar-50x10x10 (30000 tets), 30 steps, h=1/60, checkpoint 5",
            "adjoint_ms_per_step": round(1e3 * (t2 - t1) / steps, 3),
            "forward_ms_per_step": round(1e3 * (t1 - t0) / steps, 3),
            "backward_s": round(t2 - t1, 4), "forward_s": round(t1 - t0, 4),
            "recomputed_steps": sim.recomputed_steps, "mean_forward_iters": round(float(np.mean(fwd_iters)), 1),
            "mean_cg_iters": round(float(np.mean(cg)), 1), "max_cg_iters": int(max(cg)),
            "loss": float(loss.detach()), "grad_norm": float(E.grad.norm()), "dtype": "f64"}


def kernel_times_from(stats_csv, command):
    """profiles/kernel_times.json from a rocprofv3 --stats kernel statistics
    CSV: average and total duration and call count per kernel name, with the
    solver sources' hash and the command that made it."""
    import csv
    rows = {}
    with open(stats_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
            calls = int(r.get("Calls") or r.get("Count") or 0)
            total = float(r.get("TotalDurationNs") or r.get("Total_Duration_Ns") or 0.0)
            rows[name] = {"calls": calls, "avg_us": round(total / max(calls, 1) / 1e3, 3),
                          "total_us": round(total / 1e3, 1)}
    out = {"source_sha256": solver_source_hash(), "command": command, "kernels": rows}
    with open(KERNEL_TIMES, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def rocprof_avg_us(kern):
    """Average rocprofv3 duration of the kernel of KERNEL_NAMES[kern] from
    profiles/kernel_times.json, if that file was made from the current
    solver sources; else None."""
    try:
        kt = json.load(open(KERNEL_TIMES))
    except (OSError, ValueError):
        return None
    if kt.get("source_sha256") != solver_source_hash():
        return None
    pat = KERNEL_NAMES.get(kern)
    hits = [v for k, v in kt.get("kernels", {}).items() if pat and pat in k]
    if len(hits) != 1:
        return None
    return hits[0]["avg_us"], kt.get("command")


def kernel_roofline(kern, prof, sc, r, precision="mixed"):
    """Dominant-kernel roofline: algorithmic bytes per launch (KERNEL_BYTES
    with the frames' mean active pairs and candidates) over the average
    launch time from the profiled pass's HIP events, and over the rocprofv3
    average when profiles/kernel_times.json matches the sources."""
    us = prof[kern][0] / prof[kern][1]
    kt, kv, ka, kq = KERNEL_BYTES[kern][precision]
    kbytes = kt * sc.nT + kv * sc.nV + ka * r["mean_active"] + kq * r["mean_cand"]
    achieved = kbytes / (us * 1e-6)
    out = {"bound": "hbm", "kernel": kern, "achieved": round(achieved / 1e9, 1), "peak": HBM_PEAK / 1e9,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4), "bytes_per_launch": int(kbytes),
           "avg_launch_us": round(us, 3), "timing": "HIP events around each launch on the library's stream"}
    rp = rocprof_avg_us(kern) if precision == "mixed" else None
    if rp is not None:
        out["avg_launch_us_rocprof"] = rp[0]
        out["frac_rocprof"] = round(kbytes / (rp[0] * 1e-6) / HBM_PEAK, 4)
        out["rocprof_command"] = rp[1]
    return out


def summarize(sc, r, precision):
    ips = r["iters"] / r["seconds"]
    bt, bv, ba, bq = BYTES["iter"][precision]
    bytes_iter = bt * sc.nT + bv * sc.nV + ba * r["mean_active"] + bq * r["mean_cand"]
    out = {"iters_per_s": round(ips, 1), "ms_per_frame": round(1e3 * r["seconds"] / r["frames"], 4),
           "us_per_iter": round(1e6 / ips, 3), "mean_iters_per_frame": round(r["iters"] / r["frames"], 2),
           "mean_active_pairs": round(r["mean_active"], 1), "mean_candidates": round(r["mean_cand"], 1),
           "rebuilds_per_frame": round(r["rebuilds_per_frame"], 2),
           "iter_roofline": {"bytes_per_iter": int(bytes_iter), "achieved_GBps": round(bytes_iter * ips / 1e9, 1),
                             "frac": round(bytes_iter * ips / HBM_PEAK, 4)},
           "min_distance_after": r["dmin"], "min_detF_after": r["jmin"]}
    if "per_call" in r:
        out["per_call"] = r["per_call"]
    if "prof" in r:
        prof = {k: v for k, v in r["prof"].items() if v[1] > 0}
        out["kernels_us_avg"] = {k: round(v[0] / v[1], 3) for k, v in prof.items()}
        out["kernels_launches"] = {k: v[1] for k, v in prof.items()}
        out["profiled_same_trajectory"] = r["prof_same_trajectory"]
    return out


def cpu_baselines(workdir, n_pile_iters=3, n_batch_scenes=16, cores=8):
    """Run in a child process (no GPU): the float64 oracle on bounded
    samples of the three workloads, from states the GPU run saved in
    workdir."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:      # pragma: no cover
        pass
    import multiprocessing as mp
    import scenes
    from oracle import adjoint, pncg, problem
    out = {}
    # pile: n PNCG iterations of the step from the state the timed frames start from
    sc = scenes.pile_scene()
    st = np.load(os.path.join(workdir, "pile_state.npy"))
    prob = problem.Problem.from_scene(sc, rest_exclude=False)
    t0 = time.perf_counter()
    _, _, stt = pncg.step(prob, st[0], st[1], sc.h, iter_max=n_pile_iters, eps=0.0, term="delta_e")
    dt = time.perf_counter() - t0
    out["pile"] = {"value": round(stt.iters / dt, 4), "unit": "iters/s", "cores": 1, "kind": "oracle",
                   "seconds": round(dt, 2), "iters": stt.iters}
    # batched: one step of each of the first n scenes from the GPU state, over `cores` processes
    b = np.load(os.path.join(workdir, "batch_state.npz"))
    scs = scenes.batched_scenes()[:n_batch_scenes]
    jobs = [(i, b["x"][b["vert_off"][i]:b["vert_off"][i + 1]], b["v"][b["vert_off"][i]:b["vert_off"][i + 1]])
            for i in range(n_batch_scenes)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        iters = pool.map(_cpu_batch_scene, jobs)
    dt = time.perf_counter() - t0
    out["batched"] = {"value": round(n_batch_scenes / dt, 3), "unit": "scene-steps/s", "cores": cores,
                      "kind": "oracle", "seconds": round(dt, 2), "iters": int(sum(iters)),
                      "sample": f"one step of each of the first {n_batch_scenes} of the 256 scenes, "
                                f"from the batch's state after its warm-up steps"}
    # adjoint: one implicit-differentiation step of the 30,000-tet bar at a converged first step
    dsc = scenes.diff_bar_scene(seed=4)
    dp = problem.Problem.from_scene(dsc)
    x1, _ = adjoint.newton_solve(dp, dsc.x0, dsc.v0, dsc.h)
    xbar = np.random.default_rng(6).standard_normal(x1.shape)
    t0 = time.perf_counter()
    adjoint.step_adjoint(dp, x1, dsc.h, xbar, np.zeros_like(xbar))
    dt = time.perf_counter() - t0
    out["adjoint"] = {"value": round(1e3 * dt, 1), "unit": "ms/step", "cores": 1, "kind": "oracle",
                      "sample": "one adjoint step (assembled Hessian, sparse direct solve, modulus gradient) "
                                "of the 30,000-tet bar at its converged first step"}
    return out


def _cpu_batch_scene(job):
    import scenes
    from oracle import pncg, problem
    i, x, v = job
    s = scenes.batched_scenes()[i]
    p = problem.Problem.from_scene(s)
    _, _, st = pncg.step(p, x, v, s.h, iter_max=s.iter_max, eps=s.eps, term="delta_e")
    return st.iters


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed frames")
    ap.add_argument("--warmup", type=int, default=0, help="untimed frames after the settle frames")
    ap.add_argument("--settle", type=int, default=SETTLE_FRAMES,
                    help="frames the pile falls before the warm-up frames (input preparation)")
    ap.add_argument("--packed-frames", type=int, default=10, help="frames of the packed pile from rest")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison runs")
    ap.add_argument("--no-packed", action="store_true", help="skip the contact-rich packed pile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-scene batched run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable rollout")
    ap.add_argument("--no-beta-ablation", action="store_true", help="skip the beta-rule comparison")
    ap.add_argument("--no-dhat-strategy", action="store_true", help="skip the larger-dhat comparison")
    ap.add_argument("--no-split", action="store_true", help="skip the per-object splitting comparison")
    ap.add_argument("--no-materials", action="store_true", help="skip the pile and batch under the other material models")
    ap.add_argument("--headline-only", action="store_true", help="only the mixed pile (for kernel profiles)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB on the device (reference dispatch for rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calibrate-copy run into profiles/traffic.json")
    ap.add_argument("--kernel-times-from", nargs=2, metavar=("STATS_CSV", "COMMAND"),
                    help="no GPU run: turn a rocprofv3 --stats kernel statistics CSV into "
                         "profiles/kernel_times.json")
    ap.add_argument("--window-out", metavar="JSON",
                    help="write the host-clock window of the mixed pile's timed frames (for --trace-gaps-from)")
    ap.add_argument("--trace-gaps-from", nargs=2, metavar=("TRACE_CSV", "WINDOW_JSON"),
                    help="no GPU run: device busy and idle time inside the timed window of a rocprofv3 "
                         "--kernel-trace CSV")
    ap.add_argument("--cpu-baselines", metavar="DIR", help=argparse.SUPPRESS)
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--batched-warmup", type=int, default=10)
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from_csv(args.traffic_from[0], args.traffic_from[1],
                                          os.path.join(ROOT, "profiles", "traffic.json"))))
        return
    if args.kernel_times_from:
        print(json.dumps(kernel_times_from(*args.kernel_times_from)))
        return
    if args.trace_gaps_from:
        print(json.dumps(trace_gaps(*args.trace_gaps_from), indent=1))
        return
    if args.cpu_baselines:
        with open(os.path.join(args.cpu_baselines, "cpu.json"), "w") as fh:
            json.dump(cpu_baselines(args.cpu_baselines), fh)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU workload is one scene or one batch)", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_fp64 = args.no_packed = args.no_cpu_baseline = args.no_batched = args.no_adjoint = True
        args.no_beta_ablation = args.no_dhat_strategy = args.no_split = args.no_materials = True

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    # one stream (default priority) for torch and the library's contexts:
    # device inputs are then ordered without a host-side wait per step
    torch.cuda.set_stream(torch.cuda.Stream())
    if args.calibrate_copy:
        calibration_copy()
    import scenes
    sc = scenes.pile_scene()
    log(f"pile: {sc.nT} tets, {sc.nV} vertices, {len(sc.tris)} surface triangles")

    res = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        log(f"running {prec}: settle {args.settle}, warmup {args.warmup}, timed {args.steps}")
        res[prec] = run(sc, prec, args.settle, args.warmup, args.steps)
        r = res[prec]
        if args.window_out and prec == "mixed":
            with open(args.window_out, "w") as fh:
                json.dump(r["window"], fh)
        log(f"  {prec}: {r['iters']} iterations in {r['seconds'] * 1e3:.1f} ms "
            f"({r['iters'] / r['seconds']:.0f} it/s), active {r['mean_active']:.1f}, dmin={r['dmin']:.3e}")

    m = res["mixed"]
    ips = m["iters"] / m["seconds"]
    ms_frame = 1e3 * m["seconds"] / m["frames"]
    head = summarize(sc, m, "mixed")
    prof = {k: v for k, v in m["prof"].items() if v[1] > 0}
    kern = max((k for k in prof if k in KERNEL_BYTES), key=lambda k: prof[k][0])
    roof = kernel_roofline(kern, prof, sc, m)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tj = json.load(open(tpath))
            if tj.get("source_sha256") == solver_source_hash():
                traffic = tj.get("pile", {}).get(kern)
        except (OSError, ValueError):
            traffic = None
    roof["traffic"] = traffic
    first = args.settle + args.warmup
    out = {
        "metric": "PNCG iterations/s, 110k-tet pile, mixed float32/float64",
        "value": round(ips, 1),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_frame, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "pile-110k", "tets": sc.nT, "vertices": sc.nV, "h": sc.h,
                   "iter_max": sc.iter_max, "eps": sc.eps, "dhat": sc.dhat,
                   "frames": f"{first}-{first + args.steps} of the drop (settle {args.settle}, warm-up {args.warmup})",
                   "scatter": "segmented (deterministic)",
                   "mean_iters_per_frame": head["mean_iters_per_frame"],
                   "mean_active_pairs": head["mean_active_pairs"],
                   "mean_candidates": head["mean_candidates"]},
        "ms_per_frame": round(ms_frame, 4),
        "per_call": head.get("per_call"),
        "us_per_iter": head["us_per_iter"],
        "roofline": roof,
        "iter_roofline": head["iter_roofline"],
        "kernels_us_avg": head.get("kernels_us_avg"),
        "kernels_launches": head.get("kernels_launches"),
        "profiled_same_trajectory": head.get("profiled_same_trajectory"),
        "rebuilds_per_frame": head["rebuilds_per_frame"],
        "min_distance_after": m["dmin"],
        "min_detF_after": m["jmin"],
    }
    if "fp64" in res:
        f = res["fp64"]
        out["fp64"] = summarize(sc, f, "fp64")
        fprof = {k: v for k, v in f["prof"].items() if v[1] > 0}
        if "grad" in fprof:
            out["fp64"]["grad_roofline"] = kernel_roofline("grad", fprof, sc, f, "fp64")
        out["mixed_vs_fp64_speedup"] = round(ips / (f["iters"] / f["seconds"]), 3)
    if not args.no_packed:
        pk = scenes.packed_pile_scene()
        out["packed"] = {"workload": "pile-110k packed (24 shapes stacked with 0.3 dhat gaps, from rest)",
                         "frames": args.packed_frames}
        for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
            log(f"packed pile {prec}: {args.packed_frames} frames from rest ...")
            r = run(pk, prec, 0, 0, args.packed_frames)
            out["packed"][prec] = summarize(pk, r, prec)
            pprof = {k: v for k, v in r["prof"].items() if v[1] > 0}
            out["packed"][prec]["grad_roofline"] = kernel_roofline("grad", pprof, pk, r, prec)
            log(f"  {out['packed'][prec]['iters_per_s']} it/s, active {out['packed'][prec]['mean_active_pairs']}")
    if not args.no_cpu_baseline:
        import tempfile
        workdir = tempfile.mkdtemp(prefix="pncg_bench_")
        np.save(os.path.join(workdir, "pile_state.npy"), np.stack(m["state"]))
    log("pile through host arrays (PCIe-inclusive) ...")
    out["host_io"] = run_host_io(sc, m["state"])
    log(f"  {out['host_io']['iters_per_s']} it/s, {out['host_io']['ms_per_frame']} ms/frame")
    if not args.no_batched:
        log("batched: 256 scenes ...")
        out["batched"] = run_batched(args.batched_steps, args.batched_warmup,
                                     state_out=None if args.no_cpu_baseline else workdir)
        log(f"  {out['batched']['scene_steps_per_s']} scene-steps/s")
    if not args.no_adjoint:
        log("adjoint: 30,000-tet bar, 30 steps ...")
        out["adjoint"] = run_adjoint()
        log(f"  {out['adjoint']['adjoint_ms_per_step']} ms/step backward")
    if not args.no_materials:
        log("pile under the SNH, ARAP and FCR models ...")
        out["materials"] = run_materials(sc)
        log("  " + ", ".join(f"{k} {v.get('iters_per_s', v.get('error'))}" for k, v in out["materials"].items()
                             if isinstance(v, dict)))
    if not args.no_beta_ablation:
        log("beta rules on the study states ...")
        out["beta_ablation"] = run_beta_ablation()
        for case, r in out["beta_ablation"].items():
            log(f"  {case}: reference {r['reference']}; " +
                ", ".join(f"{k} {v['rel_error']}" for k, v in r["rules"].items()))
    if not args.no_split:
        log("splitting computation on the two-object states ...")
        out["split"] = run_split()
        for case, r in out["split"].items():
            if isinstance(r, dict):
                log(f"  {case}: ratio {r['reference_grad_ratio']} unsplit {r.get('unsplit', {}).get('rel_error')} "
                    f"split {r.get('split', {}).get('rel_error')}")
    if not args.no_dhat_strategy:
        log("larger-dhat strategy on the stacked cubes ...")
        out["dhat_strategy"] = run_dhat_strategy()
        log("  " + ", ".join(f"{k} {v.get('rel_error', v.get('error', v.get('note')))}"
                             for k, v in out["dhat_strategy"]["dhat"].items()))
    if not args.no_cpu_baseline and not args.no_batched:
        log("timing the CPU oracle on bounded samples (child process, no GPU) ...")
        import subprocess
        cp = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baselines", workdir],
                            capture_output=True, text=True)
        if cp.returncode == 0:
            cb = json.load(open(os.path.join(workdir, "cpu.json")))
            pile = cb["pile"]
            ipf = head["mean_iters_per_frame"]
            out["cpu_baseline"] = {
                "value": pile["value"], "unit": "iters/s", "cores": pile["cores"], "kind": "oracle",
                "sample": f"{pile['iters']} PNCG iterations of the step from the state the timed frames start "
                          f"from (float64 NumPy oracle, 1 thread, {pile['seconds']} s); at the GPU's "
                          f"{ipf} iterations per frame that is {ipf / pile['value']:.0f} s per frame "
                          f"(extrapolated, not timed)",
                "batched": cb["batched"], "adjoint": cb["adjoint"]}
        else:
            out["cpu_baseline"] = {"error": cp.stderr[-2000:]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
