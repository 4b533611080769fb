#!/usr/bin/env python3
"""Throughput of the PNCG time step on one MI355X.

Workload: the ~110k-tet pile (24 voxelised spheres and tori dropped into a
0.4 m box; synthetic, seeded; dhat = 5e-4 m, h = 1/30 s, at most 25 PNCG
iterations per frame, dE tolerance 1e-3), stepped in the mixed float32 /
float64 form, with the plain float64 form timed on the same frames for
comparison.  W untimed warm-up frames bring the shapes into contact; the
timed region is K frames.  The primary value is PNCG iterations per second
(summed over the K frames); ms per frame is reported beside it.

One JSON line is printed.  Besides the throughput it carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average launch time (HIP events on the library's stream,
                from a separate profiled pass), against 8 TB/s
  iter_roofline the whole iteration's algorithmic bytes (per-tet, per-vertex,
                per-contact byte model) times iterations/s, against 8 TB/s
  cpu_baseline  the float64 CPU oracle timed on a bounded sample of the same
                workload (one PNCG iteration from the state after warm-up)
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
# algorithmic bytes (compulsory traffic, each array touched once per pass)
BYTES = {
    # per tet, per vertex, per active contact, per candidate, for one iteration
    "iter": {"mixed": (120, 232, 144, 8), "fp64": (208, 344, 144, 8)},
}
# per-launch algorithmic bytes of each kernel: per tet, per vertex, per candidate
KERNEL_BYTES = {
    # dir: tet record; x (24), P g, p_prev, p_new, mass (8); candidate pair (8)
    "dir": {"mixed": (60, 24 + 12 + 12 + 12 + 8, 8), "fp64": (104, 24 + 24 + 24 + 24 + 8, 8)},
    # grad: tet record; x, xt, mass, g_prev, p_prev, g, P g, contact accumulators (48)
    "grad": {"mixed": (60, 24 + 24 + 8 + 12 * 4 + 48, 0), "fp64": (104, 24 + 24 + 8 + 24 * 4 + 48, 0)},
    # narrow: pending update (x_prev, p, x) per vertex; candidate pair (8)
    "narrow": {"mixed": (0, 24 + 12 + 24, 8), "fp64": (0, 24 + 24 + 24, 8)},
}


# kernels of the mixed single-scene path, by the name rocprofv3 records
# the Neo-Hookean, unsplit instantiations the pile runs (template arguments:
# real type, sweep mode, split, model, ...)
KERNEL_NAMES = {"grad": "k_grad<float, 1, false, 0,", "dir": "k_dir<float, false, 0,", "narrow": "k_narrow<float, false>"}
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
    return ctx


def _torch_stream():
    """Handle of torch's current stream, or None for its default stream (the
    library then uses a stream of its own)."""
    import torch
    h = torch.cuda.current_stream().cuda_stream
    return h or None


def run(sc, precision, warmup, steps, profile_frames, model="nh"):
    """W warm-up frames, then K timed frames in one pncg_run_dev call (the
    state stays on the device and no host round trip separates the steps);
    then K frames by separate pncg_step_dev calls from Python, for
    comparison, and the profiled frames."""
    import torch
    ctx = setup_ctx(sc, precision, model)
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.x0, dtype=torch.float64, device=dev)
    v = torch.tensor(sc.v0, dtype=torch.float64, device=dev)
    if warmup > 0:
        ctx.pncg_run_dev(x, v, sc.h, warmup)
    state = (x.cpu().numpy().copy(), v.cpu().numpy().copy())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts, _ = ctx.pncg_run_dev(x, v, sc.h, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(st["iters"] for st in sts)
    act = sum(st["n_active"] for st in sts)
    cand = sum(st["n_candidates"] for st in sts)
    # the same number of frames through one Python call per step
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
    # profiled pass (events around every launch) on further frames
    ctx.pncg_set_profiling(True)
    if profile_frames > 0:
        ctx.pncg_run_dev(x, v, sc.h, profile_frames)
    prof = ctx.pncg_get_profile()
    ctx.pncg_set_profiling(False)
    dmin, jmin = ctx.pncg_min_distance(x.cpu().numpy())
    ctx.close()
    return dict(seconds=dt, iters=iters, frames=steps, mean_active=act / steps, mean_cand=cand / steps,
                prof=prof, dmin=dmin, jmin=jmin, state=state,
                per_call={"iters_per_s": round(it_pc / dt_pc, 1), "ms_per_frame": round(1e3 * dt_pc / steps, 4)})


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


def _reference(sc, x0, v0, dhat=None, tol=1e-7, cap=5000, flags=None):
    """x* of the step from (x0, v0): float64 Dai-Kou to ||g|| <= tol ||g_0||
    (at most cap iterations) and how far it got.  Scenes of several objects
    are solved split by object (Sec. 5.2), which reaches the minimiser where
    the unsplit iteration stalls; the minimiser is the same."""
    import paper_2405_08001_amd as P
    if flags is None:
        flags = P.SPLIT_OBJECTS if len(np.unique(sc.object_id)) > 1 else 0
    xs, _, sref, _ = _solve_once(sc, "fp64", x0, v0, cap, tol, P.TERM_GRAD_REL, flags, dhat)
    return xs, {"reference_iters": int(sref["iters"]),
                "reference_grad_ratio": float(f"{sref['g_norm'] / sref['g0_norm']:.3e}")}


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


def run_beta_ablation(pile, pile_state, budgets=(10, 25, 50, 100)):
    """The beta rules of the ablation (Sec. 7.1), re-run on synthetic scenes:
    the error after K iterations of one step against the step's minimiser
    (float64 Dai-Kou to ||g|| <= 1e-7 ||g_0||, at most 5,000 iterations),
    for the pile (mixed, from the state after warm-up) and the cube resting
    on its floor (float64, after 12 steps)."""
    import paper_2405_08001_amd as P
    import scenes
    cube = scenes.cube_scene()
    x, v = cube.x0.copy(), cube.v0.copy()
    for _ in range(12):
        x, v, _, _ = _solve_once(cube, "fp64", x, v, 2000, cube.eps, P.TERM_GRAD_REL)
    cases = {"cube": (cube, "fp64", x, v), "pile": (pile, "mixed", pile_state[0], pile_state[1])}
    out = {}
    for name, (sc, prec, x0, v0) in cases.items():
        xs, ref = _reference(sc, x0, v0)
        res = {"precision": prec, "budgets": list(budgets), "reference_tol": 1e-7, "rules": {}}
        res.update(ref)
        for rule, flag in P.BETA_RULES.items():
            res["rules"][rule] = _convergence(sc, prec, x0, v0, budgets, flag, None, xs)
        out[name] = res
    return out


def run_split(pile, pile_state, budgets=(10, 25, 50, 100)):
    """Splitting computation (Sec. 5.2) on the pile (24 objects), mixed, from
    the state after warm-up: the error after K iterations against the step's
    minimiser (the same energy either way), split and unsplit, and the
    iteration rate of each over 10 frames as configured.  The minimiser is
    taken from the split float64 solve, which gets much closer to it."""
    import torch
    import paper_2405_08001_amd as P
    dev = torch.device("cuda:0")
    xs, ref = _reference(pile, pile_state[0], pile_state[1])
    out = {"budgets": list(budgets), "objects": int(len(np.unique(pile.object_id))), "reference_tol": 1e-7}
    out.update(ref)
    for name, flag in (("unsplit", 0), ("split", P.SPLIT_OBJECTS)):
        r = _convergence(pile, "mixed", pile_state[0], pile_state[1], budgets, flag, None, xs)
        ctx = setup_ctx(pile, "mixed")
        ctx.pncg_set_solver(pile.iter_max, pile.eps, P.TERM_DELTA_E, pile.gravity, flag)
        x = torch.tensor(pile_state[0], device=dev)
        v = torch.tensor(pile_state[1], device=dev)
        x2, v2 = torch.empty_like(x), torch.empty_like(v)
        its = reb = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            st = ctx.pncg_step_dev(x, v, pile.h, x2, v2)
            its += st["iters"]
            reb += st["rebuilds"]
            x, x2, v, v2 = x2, x, v2, v
        torch.cuda.synchronize()
        r["frames_iters_per_s"] = round(its / (time.perf_counter() - t0), 1)
        r["frames_iters_per_frame"] = round(its / 10, 2)
        r["frames_rebuilds_per_frame"] = round(reb / 10, 2)
        ctx.close()
        out[name] = r
    return out


def run_materials(sc, warmup=10, steps=30, profile_frames=5, models=("snh", "arap", "fcr"), batched=True,
                  adjoint_model="fcr"):
    """The pile as configured under each other material model (mixed form):
    iteration rate, frame time, iterations per frame, and the sweep's
    roofline (its algorithmic bytes do not depend on the model); the
    256-scene batch under each model (10 graph-captured steps); and the
    differentiable 30,000-tet rollout under one corotated model."""
    out = {"frames_warmup": warmup, "frames_timed": steps}
    kt, kv, kq = KERNEL_BYTES["grad"]["mixed"]
    for model in models:
        try:
            r = run(sc, "mixed", warmup, steps, profile_frames, model=model)
        except Exception as e:  # a model whose trajectory leaves its domain
            out[model] = {"error": str(e)}
            continue
        ips = r["iters"] / r["seconds"]
        prof = {k: v for k, v in r["prof"].items() if v[1] > 0}
        gus = prof["grad"][0] / prof["grad"][1]
        gb = kt * sc.nT + kv * sc.nV + kq * r["mean_cand"]
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


def run_dhat_strategy(pile, warmup=10, fractions=(0.3, 0.5, 0.7), budgets=(10, 25, 50, 100)):
    """The larger-dhat strategy (Sec. 5.1) on the pile, mixed: dhat at
    30/50/70 % of the mean boundary edge (same-object pairs closer than
    1.5 dhat at rest excluded) against the configured dhat.  Each runs its
    own warm-up frames from the initial state with its dhat (the strategy is
    a setting of the whole simulation), then one step is measured against
    its own minimiser (the problem changes with dhat)."""
    import torch
    import paper_2405_08001_amd as P
    dev = torch.device("cuda:0")
    ctx = setup_ctx(pile, "mixed")
    lbar = ctx.pncg_mean_boundary_edge()
    ctx.close()
    out = {"mean_boundary_edge": lbar, "budgets": list(budgets), "reference_tol": 1e-7, "warmup_frames": warmup,
           "dhat": {}}
    for label, dh in [("configured", pile.dhat)] + [(f"{f:.1f}*edge", f * lbar) for f in fractions]:
        r = {"dhat": dh}
        try:
            ctx = setup_ctx(pile, "mixed")
            ctx.pncg_set_contact(dh, pile.kappa, 0.0, pile.planes,
                                 (P.CONTACT_SELF if pile.self_contact else 0) | P.CONTACT_REST_EXCLUDE)
            x = torch.tensor(pile.x0, device=dev)
            v = torch.tensor(pile.v0, device=dev)
            x2, v2 = torch.empty_like(x), torch.empty_like(v)
            its = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(warmup):
                its += ctx.pncg_step_dev(x, v, pile.h, x2, v2)["iters"]
                x, x2, v, v2 = x2, x, v2, v
            torch.cuda.synchronize()
            r["warmup_iters_per_s"] = round(its / (time.perf_counter() - t0), 1)
            ctx.close()
            x0, v0 = x.cpu().numpy(), v.cpu().numpy()
            xs, ref = _reference(pile, x0, v0, dh)
            r.update(_convergence(pile, "mixed", x0, v0, budgets, 0, dh, xs))
            r.update(ref)
        except P.PncgError as e:      # e.g. a tet inverted on the way (no inversion guard, reading S4)
            r["error"] = str(e)
        out["dhat"][label] = r
    return out


def cpu_baseline(sc, state, budget_iters=1):
    """The float64 oracle, single-threaded, on one PNCG iteration from the
    same state (the rest-pose exclusion set of this scene is empty, so it is
    skipped in the oracle's setup)."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:      # pragma: no cover
        threadpool_limits = None
    from oracle import pncg, problem
    prob = problem.Problem.from_scene(sc, rest_exclude=False)
    x, v = state
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        _, _, st = pncg.step(prob, x, v, sc.h, iter_max=budget_iters, eps=0.0, term="delta_e")
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    return dict(value=st.iters / dt, unit="iters/s", cores=1, kind="oracle",
                sample=f"{st.iters} PNCG iteration(s) of the 110k-tet pile from the state after warm-up "
                       f"(float64 NumPy oracle, 1 thread, {dt:.1f} s)")


def run_batched(steps, warmup, model="nh"):
    """The 256-scene batch, mixed precision: W eager steps (the scenes fall
    onto their planes), then K steps as one captured graph."""
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60, help="timed frames")
    ap.add_argument("--warmup", type=int, default=10, help="untimed frames before timing")
    ap.add_argument("--profile-frames", type=int, default=10)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-scene batched run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable rollout")
    ap.add_argument("--no-beta-ablation", action="store_true", help="skip the beta-rule comparison")
    ap.add_argument("--no-dhat-strategy", action="store_true", help="skip the larger-dhat comparison")
    ap.add_argument("--no-split", action="store_true", help="skip the per-object splitting comparison")
    ap.add_argument("--no-materials", action="store_true", help="skip the pile and batch under the other material models")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB on the device (reference dispatch for rocprofv3 byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calibrate-copy run into profiles/traffic.json")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--batched-warmup", type=int, default=10)
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from_csv(args.traffic_from[0], args.traffic_from[1],
                                          os.path.join(ROOT, "profiles", "traffic.json"))))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU workload is one scene or one batch)", file=sys.stderr)
        sys.exit(2)

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
        log(f"running {prec}: warmup {args.warmup}, timed {args.steps}")
        res[prec] = run(sc, prec, args.warmup, args.steps, args.profile_frames)
        r = res[prec]
        log(f"  {prec}: {r['iters']} iterations in {r['seconds'] * 1e3:.1f} ms "
            f"({r['iters'] / r['seconds']:.0f} it/s), dmin={r['dmin']:.3e} jmin={r['jmin']:.3f}")

    m = res["mixed"]
    ips = m["iters"] / m["seconds"]
    ms_frame = 1e3 * m["seconds"] / m["frames"]
    bt, bv, ba, bq = BYTES["iter"]["mixed"]
    bytes_iter = bt * sc.nT + bv * sc.nV + ba * m["mean_active"] + bq * m["mean_cand"]
    # dominant kernel of the profiled pass
    prof = {k: v for k, v in m["prof"].items() if v[1] > 0}
    kern = max((k for k in prof if k in KERNEL_BYTES), key=lambda k: prof[k][0])
    avg_us = prof[kern][0] / prof[kern][1]
    kt, kv, kq = KERNEL_BYTES[kern]["mixed"]
    kbytes = kt * sc.nT + kv * sc.nV + kq * m["mean_cand"]
    achieved = kbytes / (avg_us * 1e-6) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tj = json.load(open(tpath))
            if tj.get("source_sha256") == solver_source_hash():
                traffic = tj.get("pile", {}).get(kern)
        except (OSError, ValueError):
            traffic = None
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
                   "frames_timed": args.steps, "frames_warmup": args.warmup,
                   "mean_iters_per_frame": round(m["iters"] / m["frames"], 2),
                   "mean_active_pairs": round(m["mean_active"], 1),
                   "mean_candidates": round(m["mean_cand"], 1)},
        "ms_per_frame": round(ms_frame, 4),
        "per_call": m["per_call"],
        "us_per_iter": round(1e6 / ips, 3),
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(achieved * 1e9 / HBM_PEAK, 4),
                     "bytes_per_launch": int(kbytes), "avg_launch_us": round(avg_us, 3),
                     "traffic": traffic},
        "iter_roofline": {"bytes_per_iter": int(bytes_iter),
                          "achieved_GBps": round(bytes_iter * ips / 1e9, 1),
                          "frac": round(bytes_iter * ips / HBM_PEAK, 4)},
        "kernels_us_avg": {k: round(v[0] / v[1], 3) for k, v in prof.items()},
        "kernels_launches": {k: v[1] for k, v in prof.items()},
        "min_distance_after": m["dmin"],
        "min_detF_after": m["jmin"],
    }
    if "fp64" in res:
        f = res["fp64"]
        fips = f["iters"] / f["seconds"]
        out["fp64"] = {"iters_per_s": round(fips, 1), "ms_per_frame": round(1e3 * f["seconds"] / f["frames"], 4),
                       "us_per_iter": round(1e6 / fips, 3)}
        t8, v8, a8, q8 = BYTES["iter"]["fp64"]
        b8 = t8 * sc.nT + v8 * sc.nV + a8 * f["mean_active"] + q8 * f["mean_cand"]
        out["fp64"]["iter_roofline"] = {"bytes_per_iter": int(b8), "achieved_GBps": round(b8 * fips / 1e9, 1),
                                        "frac": round(b8 * fips / HBM_PEAK, 4)}
        fprof = {k: v for k, v in f["prof"].items() if v[1] > 0}
        if "grad" in fprof:
            gus = fprof["grad"][0] / fprof["grad"][1]
            kt, kv, kq = KERNEL_BYTES["grad"]["fp64"]
            gb = kt * sc.nT + kv * sc.nV + kq * f["mean_cand"]
            out["fp64"]["grad_roofline"] = {"achieved": round(gb / (gus * 1e-6) / 1e9, 1), "avg_launch_us": round(gus, 3),
                                            "bytes_per_launch": int(gb), "frac": round(gb / (gus * 1e-6) / HBM_PEAK, 4)}
        out["mixed_vs_fp64_speedup"] = round(ips / fips, 3)
    log("pile through host arrays (PCIe-inclusive) ...")
    out["host_io"] = run_host_io(sc, m["state"])
    log(f"  {out['host_io']['iters_per_s']} it/s, {out['host_io']['ms_per_frame']} ms/frame")
    if not args.no_batched:
        log("batched: 256 scenes ...")
        out["batched"] = run_batched(args.batched_steps, args.batched_warmup)
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
        log("beta rules: pile and cube ...")
        out["beta_ablation"] = run_beta_ablation(sc, m["state"])
        for case, r in out["beta_ablation"].items():
            log(f"  {case}: " + ", ".join(f"{k} {v['rel_error']}" for k, v in r["rules"].items()))
    if not args.no_split:
        log("splitting computation on the pile ...")
        out["split"] = run_split(sc, m["state"])
        log(f"  unsplit {out['split']['unsplit']['rel_error']} split {out['split']['split']['rel_error']}")
    if not args.no_dhat_strategy:
        log("larger-dhat strategy on the pile ...")
        out["dhat_strategy"] = run_dhat_strategy(sc)
        log("  " + ", ".join(f"{k} {v.get('rel_error', v.get('error'))}" for k, v in out["dhat_strategy"]["dhat"].items()))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one iteration ...")
        out["cpu_baseline"] = cpu_baseline(sc, m["state"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
