#!/usr/bin/env python3
"""Benchmark of the long-characteristics transport step on one MI355X.

Default workload (the batched form): 64 independent problems of uneven size
-- meshes from {32^2, 64^2, 128^2, 256^2} cells on 6x6 cm, G from {8, 17, 51}
groups, 16/64/128 directions, characteristic spacing h/2, seeded smooth
temperature fields -- advanced together in float32 (one launch per phase and
polar group, graph-captured steps; the timed steps are graph replays, and a
second, eager pass with the library's kernel timers gives the per-kernel
figures).  Beside it the same 64 problems are run with the plain float64
sweep, problem by problem, and the float32 moments are compared with the
float64 ones.

A "step" is one backward-Euler transport step of the whole workload: the
sweep (eq. (10)-(13)) over every characteristic, direction and group of every
problem, then the cell moments and boundary factors (eq. (7), (14)-(16)).
Inputs are resident in HBM before the timed region.  Throughput is in
segment-updates/s: one update is one evaluation of the segment propagation for
one (segment, traversal, polar angle, group).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_algorithmic_bytes(solver, elem):
    """Bytes one sweep of a problem must move at minimum: the stored segment
    intensities read and written once, each segment's geometry (cell index
    and length) once per traversal, the cell-coefficient table once, the
    entering intensities and the exit intensities."""
    r = solver.rays
    G = solver.prob.G
    upd = solver.updates_per_step()
    state = 2 * upd * elem
    geom = 2 * r.n_segments * (4 + elem)
    coef = r.cells * G * (2 * elem)
    io = 2 * r.n_rays * 2 * r.n_pol * G * 8
    return state + geom + coef + io


def step_algorithmic_bytes(solver, elem):
    """Bytes one whole transport step of a problem must move at minimum: the
    sweep's (above) plus the moments every step writes -- E, F and the
    Eddington tensor (7 float64 per cell and group) and the boundary factors
    (8 float64 per boundary face and group).  Re-reading the stored
    intensities to form the moments is not counted: it is the price of an
    unfused reduction, not of the method."""
    p, r = solver.prob, solver.rays
    return sweep_algorithmic_bytes(solver, elem) + p.cells * p.G * 7 * 8 + p.G * r.nb * 8 * 8


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sweep_batch_traffic.txt")
SWEEP_SOURCES = ("sweep.hip", "batch.hip", "lc_internal.hpp")


def recorded_traffic(tuning):
    """HBM bytes per sweep phase measured with rocprofv3 counters for this
    workload (the recorded bytes per launch of each polar group's sweep at
    its chosen sweep_unroll, summed), or None when the sweep sources differ
    from those the counters were taken with or a choice was not recorded."""
    import hashlib
    try:
        rec = dict(line.split(" ", 1) for line in open(TRAFFIC_RECORD).read().splitlines()
                   if line and not line.startswith("#"))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_11998_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if rec.get("source_sha256", "").strip() != h.hexdigest():
        return None
    per = json.loads(rec.get("traffic_bytes_per_launch", "null")) or {}
    total = 0.0
    for pm, v in tuning.items():
        b = per.get(str(pm), {}).get(str(v["sweep_unroll"]))
        if b is None:
            return None
        total += b
    return total


def moment_errors(got, ref):
    from tests.parity_util import err_E, err_F, err_f
    import workloads as W
    return dict(E=err_E(got["E"], ref["E"]), F=err_F(got["F"], ref["F"], ref["E"], W.C_LIGHT),
                f=err_f(got["f"], ref["f"], ref["E"]))


def run_batched(probs, steps, warmup, prec, snapshot_steps=0):
    """The batched form in precision `prec`: tuned, then `steps` steps
    replayed from the captured graph (timed with events around the replay),
    then the same steps eager with the library's kernel timers per phase.
    With snapshot_steps = T, the moments after 1, 2, ..., T steps from the
    initial state are kept on the device (for the per-step accuracy check)."""
    import torch
    from paper_2305_11998_amd import driver, lc, tune
    bs = driver.BatchSolver(probs, prec=prec, static_material=True)
    tuned = tune.tune_batch(bs, verbose=True)
    _say(f"batch tuning per polar class: {tuned['per_class']}")
    bs.reset()
    bs.step(warmup)                                   # graph of `warmup` steps
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # timed: `steps` steps replayed from the captured graph (the production
    # path); captured once, untimed
    bs.step(steps)
    torch.cuda.synchronize()
    e0.record()
    bs.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)
    # the same steps eager and phase after phase, with the library's kernel
    # timers around each phase (for the per-kernel figures)
    lc.lc_batch_profile(bs.batch, True)
    lc.lc_batch_profile_read(bs.batch)
    torch.cuda.synchronize()
    e0.record()
    bs.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    pro, npro, sw, nsw, mo, nmo = lc.lc_batch_profile_read(bs.batch)
    lc.lc_batch_profile(bs.batch, False)
    snaps = []
    for n in range(1, snapshot_steps + 1):
        bs.reset()
        bs.step(n)
        torch.cuda.synchronize()
        snaps.append([{k: getattr(s, k).clone() for k in ("E", "F", "f")} for s in bs.solvers])
    return dict(bs=bs, ms=ms_graph, ms_eager=ms, sweep_ms=sw / max(nsw, 1), moments_ms=mo / max(nmo, 1),
                prologue_ms=pro / max(npro, 1), tuning=tuned, snapshots=snaps)


def _dev_errors(a, b, G, cells, c):
    """Error metrics of moments a against b (device tensors in the library's
    cell-major layout) -- the metrics of tests/parity_util on the device:
    relative E over cells whose E is above 1e-30 of the group's largest, F
    relative to c E, f absolute."""
    import torch
    Ea, Eb = a["E"].view(cells, G), b["E"].view(cells, G)
    m = Eb > 1e-30 * Eb.max(dim=0, keepdim=True).values
    if not bool(m.any()):
        return dict(E=0.0, F=0.0, f=0.0)
    eE = ((Ea - Eb).abs() / torch.where(m, Eb, torch.ones_like(Eb)))[m].max().item()
    dF = (a["F"].view(cells, 2, G) - b["F"].view(cells, 2, G)).abs().amax(dim=1)
    eF = (dF / torch.where(m, c * Eb, torch.ones_like(Eb)))[m].max().item()
    df = (a["f"].view(cells, 4, G) - b["f"].view(cells, 4, G)).abs().amax(dim=1)
    return dict(E=eE, F=eF, f=df[m].max().item())


def run_plain_f64(probs, steps, snapshots=None):
    """The plain float64 sweep, problem by problem (eager sweep + moments),
    timed over `steps` steps per problem.  With float32 snapshots (moments
    after 1..T steps, per problem), each problem is then advanced T steps
    from the initial state and its moments after every step are compared
    with the float32 ones; returns the worst error over steps and problems,
    and per step."""
    import torch
    import workloads as W
    from paper_2305_11998_amd import driver, lc
    tot_ms, upd = 0.0, 0
    T = len(snapshots) if snapshots else 0
    worst = {k: 0.0 for k in ("E", "F", "f")}
    per_step = [{k: 0.0 for k in ("E", "F", "f")} for _ in range(T)]
    for q, p in enumerate(probs):
        s = driver.Solver(p, prec=lc.LC_F64)
        s.reset()
        s.bench_step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            s.bench_step()
        e1.record()
        torch.cuda.synchronize()
        tot_ms += e0.elapsed_time(e1) / steps
        upd += s.updates_per_step()
        if T:
            s.reset()
            for t in range(T):
                s.bench_step()
                e = _dev_errors(snapshots[t][q], dict(E=s.E, F=s.F, f=s.f), p.G, p.cells, W.C_LIGHT)
                for k in worst:
                    worst[k] = max(worst[k], e[k])
                    per_step[t][k] = max(per_step[t][k], e[k])
        del s
    torch.cuda.empty_cache()
    return dict(ms_per_step=tot_ms, updates=upd, worst=worst, per_step=per_step)


def _oracle_pair_sample(prob, a, budget_s):
    """The oracle's sweep (unchanged) of azimuth pair a of a problem, both
    traversals, all polar angles and groups, on batches of 16
    characteristics (the shortest quarter, corner clips, left out), repeated
    until `budget_s` seconds of sweeping.  Returns (updates, seconds,
    characteristics)."""
    import numpy as np
    from oracle import rays as orays, sweep as osweep
    P, G = prob.n_pol, prob.G
    half = prob.n_az // 2
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi[[a, a + half]], prob.h_moc)
    pr = g.pairs[0]
    cols = list(range(a * P, a * P + P)) + list(range((a + half) * P, (a + half) * P + P))
    I_in = prob.I_in[:, cols, :]
    order = np.argsort(-pr.nseg)
    ks = np.sort(order[len(order) // 4:])
    done_upd, t_used, n_rays = 0, 0.0, 0
    chunk, q = 16, 0
    while t_used < budget_s:
        if q >= len(ks):
            q = 0
        sel = ks[q:q + chunk]
        q += chunk
        rows = np.concatenate([np.broadcast_to(prob.state0[:, pr.cells[k]].T[:, None, None, :],
                                               (len(pr.cells[k]), 2, P, G)) for k in sel])
        t0 = time.perf_counter()
        osweep.sweep_pair(g, 0, prob.mu, prob.kappa[0], prob.planck[0], prob.c_dt, rows, I_in,
                          rays=sel, local_state=True)
        t_used += time.perf_counter() - t0
        done_upd += int(pr.nseg[sel].sum()) * 2 * P * G
        n_rays += len(sel)
    return done_upd, t_used, n_rays


def _oracle_pair_job(args):
    member, a, budget_s = args
    import workloads as W
    prob = W.batch_problems(steps=1, only=[member])[0]
    return _oracle_pair_sample(prob, a, budget_s)


def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(model=model, nproc=os.cpu_count(), affinity=avail)


def cpu_baseline(prob, member, budget_s=12.0):
    """The oracle's sweep (unchanged) on a bounded sample of the workload's
    largest member, timed on the host: one process per azimuth pair (up to
    16, spawned), each sweeping characteristics of its pair for `budget_s`
    seconds; the aggregate rate is the sum of the processes' rates.  The
    single-process rate on pair 0 is reported beside it."""
    import multiprocessing as mp
    host = _host_cpu()
    n_pairs = prob.n_az // 2
    nproc = max(1, min(16, host["affinity"] or 1, n_pairs))
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc) as pool:
        res = pool.map(_oracle_pair_job, [(member, a, budget_s) for a in range(nproc)], chunksize=1)
    rate = sum(u / t for u, t, _ in res)
    upd = sum(u for u, _, _ in res)
    rays = sum(r for _, _, r in res)
    u1, t1, r1 = _oracle_pair_sample(prob, 0, budget_s)
    return dict(value=rate, unit="segment-updates/s", cores=nproc, kind="oracle",
                sample=f"oracle FP64 sweep, one process per azimuth pair ({nproc} pairs) of member "
                       f"{prob.name} ({prob.nx}x{prob.ny}, G={prob.G}, {prob.M} directions), both "
                       f"traversals, {rays} characteristics, {upd} updates, about {budget_s:.0f} s per "
                       f"process; host: {host['model']}, {host['nproc']} CPUs ({host['affinity']} usable)",
                single_process=dict(value=u1 / t1, updates=u1, seconds=t1, characteristics=r1),
                host=host)


def time_grey_closures(s, reps=20):
    """lc_grey_closures on the solver's last moments: mean launch time
    (events on the stream it runs on), its algorithmic bytes (7 moment and 2
    material values per (cell, group) read, 13 fields per cell written) and
    the oracle's time on the same inputs (one host thread)."""
    import torch
    from oracle import closures as oc
    from paper_2305_11998_amd import lc
    p = s.prob
    G, cells = p.G, p.cells
    kap, pla = s.kappa.view(-1)[:G * cells], s.planck.view(-1)[:G * cells]
    out = torch.empty(lc.N_GREY * cells, dtype=torch.float64, device="cuda")
    lc.lc_grey_closures(s.plan, s.E, s.F, s.f, kap, pla, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lc.lc_grey_closures(s.plan, s.E, s.F, s.f, kap, pla, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = (9 * G + lc.N_GREY) * cells * 8
    m = s.moments()
    t0 = time.perf_counter()
    oc.grey_closures(m["E"], m["F"], m["f"], p.kappa[0], p.planck[0])
    cpu_ms = (time.perf_counter() - t0) * 1e3
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"kernel": "k_grey_closures", "ms": ms, "algorithmic_bytes": nbytes, "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "cpu_oracle_ms": cpu_ms}


def time_faces(s, reps=5):
    """Interior-face moments of eq. (16) on the solver's problem: the sweep
    that also stores the upwind-face intensities and the face gather
    (lc_face_moments), mean times over `reps` launches.  The gather's
    algorithmic bytes: the stored intensities read once (one value per
    segment update) plus its outputs (7 doubles per face and group)."""
    import torch
    from paper_2305_11998_amd import lc
    p = s.prob
    s.enable_faces()
    s.reset()
    kap, pla = s.kappa.view(-1), s.planck.view(-1)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    lc.lc_sweep_points(s.plan, kap, pla, p.c_dt, s.state[0], s.state[1], s.I_in, s.points, s.I_exit)
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        lc.lc_sweep_points(s.plan, kap, pla, p.c_dt, s.state[0], s.state[1], s.I_in, s.points, s.I_exit)
    e[1].record()
    for _ in range(reps):
        lc.lc_face_moments(s.plan, s.points, s.state[1], s.c, s.Ef, s.Ff, s.ff)
    e[2].record()
    torch.cuda.synchronize()
    sweep_ms = e[0].elapsed_time(e[1]) / reps
    face_ms = e[1].elapsed_time(e[2]) / reps
    nf = lc.n_interior_faces(s.rays)
    elem = 4 if s.prec == lc.LC_F32 else 8
    nbytes = s.updates_per_step() * elem + 7 * nf * p.G * 8
    gbs = nbytes / (face_ms * 1e-3) / 1e9
    return {"kernel": "k_cell_moments over the interior-face lists", "sweep_with_points_ms": sweep_ms,
            "face_moments_ms": face_ms, "faces": nf, "algorithmic_bytes": nbytes, "achieved": gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def run_single(k, steps, warmup):
    """One problem of the named workloads (workloads.config(k)) on the plain
    path, float32 and float64: eager steps timed with the library's kernel
    timers, plus the float32-vs-float64 moment errors after one step."""
    import torch
    import workloads as W
    from paper_2305_11998_amd import driver, lc, tune
    prob = W.config(k, steps=1)
    out = {}
    for prec, name in ((lc.LC_F32, "f32"), (lc.LC_F64, "f64")):
        s = driver.Solver(prob, prec=prec)
        tuned = tune.tune(s, cache=None)
        s.reset()
        for _ in range(warmup):
            s.bench_step()
        torch.cuda.synchronize()
        lc.lc_plan_profile_read(s.plan)
        lc.lc_plan_profile(s.plan, True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            s.bench_step()
        e1.record()
        torch.cuda.synchronize()
        sw, nsw, mo, nmo = lc.lc_plan_profile_read(s.plan)
        lc.lc_plan_profile(s.plan, False)
        s.reset()
        s.step(1)
        grey = time_grey_closures(s) if prec == lc.LC_F32 else None
        out[name] = dict(ms=e0.elapsed_time(e1) / steps, sweep_ms=sw / max(nsw, 1), moments_ms=mo / max(nmo, 1),
                         grey=grey,
                         upd=s.updates_per_step(), moments=s.moments(),
                         alg=sweep_algorithmic_bytes(s, 4 if prec == lc.LC_F32 else 8),
                         tuning={kk: tuned.get(kk, 0) for kk in ("sweep_unroll", "moments_entries", "sweep_capped",
                                                                 "split")})
        out[name]["faces"] = time_faces(s) if prec == lc.LC_F32 else None     # after the moments above
        _say(f"config {k} {name}: {out[name]['ms']:.3f} ms/step, sweep {out[name]['sweep_ms']:.3f} ms, "
             f"moments {out[name]['moments_ms']:.3f} ms")
        del s
        torch.cuda.empty_cache()
    return prob, out


def main_single(args):
    prob, out = run_single(args.config, args.steps, args.warmup)
    f32, f64 = out["f32"], out["f64"]
    errs = moment_errors(f32["moments"], f64["moments"])
    value = f32["upd"] / (f32["ms"] / 1e3)
    achieved = f32["alg"] / (f32["sweep_ms"] / 1e3) / 1e9
    res = {
        "metric": "segment-updates/s, FP32 vs FP64 sweep at <=1e-5 rel error (single problem)",
        "value": value, "unit": "segment-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f32["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"single problem {prob.name}: {prob.nx}x{prob.ny} cells, G={prob.G}, "
                               f"{prob.M} directions, spacing {prob.h_moc:.4g} cm",
                   "updates_per_step": f32["upd"], "tuning": f32["tuning"]},
        "fp64_plain": {"value": f64["upd"] / (f64["ms"] / 1e3), "ms_per_step": f64["ms"],
                       "sweep_ms": f64["sweep_ms"], "moments_ms": f64["moments_ms"], "tuning": f64["tuning"]},
        "fp32_vs_fp64_max_err": errs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sweep<float,P,U>",
                     "kernel_ms": f32["sweep_ms"], "moments_kernel_ms": f32["moments_ms"],
                     "algorithmic_bytes_per_launch": f32["alg"]},
        "grey_closures": f32["grey"],
        "interior_faces": f32["faces"],
    }
    print(json.dumps(res), flush=True)


def split_cases():
    """Few-lane problems, where a traversal's steps are the critical path:
    a 512^2 grid swept for one group with 8 x 2 directions (lanes = the
    characteristics only), and the two lowest groups of the 256^2, G = 51,
    32 x 4 problem on a characteristic grid four times finer (spacing h/8),
    the kind of group range that group-dependent grids put on a fine grid;
    with the 128^2, G = 17 problem for comparison."""
    import numpy as np
    import workloads as W
    rng = np.random.default_rng(W.SEED0 + 7)
    n, L = 512, 6.0
    T = W.t_field_gaussians(rng, n, n, L, L)
    grey = W.make_problem(n, n, L, L, 8, 2, 1, 0.001, 30.0, L / n / 2, 3.0, [T], name="512x512 G=1 8x2 dirs h/2")
    c2 = W.config(2, steps=1)
    low = W.group_subset(c2, 0, 2, h_moc=c2.lx / c2.nx / 8, name="256x256 groups 0-1 of 51, 32x4 dirs, h/8")
    c1 = W.config(1, steps=1)
    c1.name = "128x128 G=17 32x2 dirs h/4"
    return [grey, low, c1]


def main_split(args):
    """Whole-traversal vs split sweep (lc_plan_set_split) on few-lane
    problems: sweep milliseconds per chunk length, float32 and float64, and
    the largest relative difference of E between the two forms."""
    import numpy as np
    import torch
    from paper_2305_11998_amd import driver, lc, tune
    rows = []
    cases = split_cases()
    for prob in (cases if args.case is None else [cases[args.case]]):
        for prec, name in ((lc.LC_F32, "f32"), (lc.LC_F64, "f64")):
            s = driver.Solver(prob, prec=prec)
            tune.tune(s, cache=None)
            times, E = {}, {}
            for sp in (0, 16, 32, 64, 128, 256):
                lc.lc_plan_set_split(s.plan, sp)
                s.reset()
                for _ in range(args.warmup):
                    s.bench_step()
                torch.cuda.synchronize()
                lc.lc_plan_profile_read(s.plan)
                lc.lc_plan_profile(s.plan, True)
                for _ in range(args.steps):
                    s.bench_step()
                torch.cuda.synchronize()
                sw, nsw, _, _ = lc.lc_plan_profile_read(s.plan)
                lc.lc_plan_profile(s.plan, False)
                times[sp] = sw / max(nsw, 1)
                s.reset()
                s.step(1, graph=False)
                E[sp] = s.moments()["E"]
            best = min(times, key=times.get)
            dE = max(float(np.max(np.abs(E[sp] - E[0]) / np.maximum(np.abs(E[0]), 1e-300))) for sp in E)
            row = dict(problem=prob.name, prec=name, updates=s.updates_per_step(), whole_ms=times[0],
                       best_split=best, best_ms=times[best], speedup=times[0] / times[best],
                       ms={str(k): v for k, v in times.items()}, max_rel_dE=dE)
            _say(f"{prob.name} {name}: whole {times[0]:.4f} ms, split {best}: {times[best]:.4f} ms "
                 f"({row['speedup']:.2f}x), max rel dE {dE:.1e}")
            rows.append(row)
            del s
            torch.cuda.empty_cache()
    print(json.dumps({"workload": "split sweep on few-lane problems", "rows": rows}), flush=True)


def main_refinement(args):
    """Characteristic-grid refinement at fixed material grid, transport only:
    the paper's vertex-avoiding, width-halving grid with h_moc = h_mat / r,
    r = 8, 16, ..., on a Fleck-Cummings-like slab (6 x 6 cm, 1 keV Planckian
    entering at x = 0, opacity 27/nu^3 (1 - e^{-nu/T}), 17 groups, 36 x 4
    directions), one backward-Euler step (c dt = 0.6 cm, the paper's 0.02 ns)
    through a prescribed temperature profile T(x) = 1 keV e^{-x / 1 cm} + 1 eV.
    Reports ||Delta E|| = || E_{h_moc} - E_{h_moc / 2} || (grey E, area-weighted
    L2 over the cells) and rho = ||Delta E_{h}|| / ||Delta E_{h/2}||, with the
    characteristic counts and step times."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2305_11998_amd import driver, lc
    L = 6.0
    rows = []
    for n, ratios in ((10, (8, 16, 32, 64, 128, 256, 512)), (40, (8, 16, 32, 64, 128))):
        h = L / n
        x = (np.arange(n) + 0.5) * h
        T = np.tile(1.0 * np.exp(-x / 1.0) + 0.001, n)          # cell i = iy * n + ix
        prev = None
        for r in ratios:
            prob = W.make_problem(n, n, L, L, 36, 4, 17, 0.001, 30.0, h / r, 0.6, [T], name=f"fc{n}")
            s = driver.Solver(prob, prec=lc.LC_F64, mode=lc.LC_RAYS_TUBES)
            s.reset()
            s.step(1, graph=False)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.reset()
            e0.record()
            s.step(1, graph=False)
            e1.record()
            torch.cuda.synchronize()
            E = s.moments()["E"].sum(axis=0)                        # grey E per cell
            row = {"h_mat": h, "ratio": r, "h_moc": h / r, "characteristics": int(s.rays.n_rays),
                   "segments": int(s.rays.n_segments), "step_ms": e0.elapsed_time(e1),
                   "norm_E": float(np.sqrt(np.sum(E ** 2) * h * h))}
            if prev is not None:
                d = float(np.sqrt(np.sum((E - prev) ** 2) * h * h))
                row["dE"] = d
                row["dE_rel"] = d / row["norm_E"]
                if "dE" in rows[-1]:
                    row["rho"] = rows[-1]["dE"] / d if d > 0 else None
            rows.append(row)
            prev = E
            _say(f"h_mat {h:.3f} ratio {r}: {row['characteristics']} characteristics, "
                 f"{row['segments']} segments, {row['step_ms']:.2f} ms, dE {row.get('dE', float('nan')):.3e}, "
                 f"rho {row.get('rho') or float('nan'):.2f}")
            del s
            torch.cuda.empty_cache()
    print(json.dumps({"workload": "characteristic-grid refinement (tube mode), transport only", "rows": rows}),
          flush=True)


def _fc_energy_defect(prob, prev, got, C):
    """Relative mismatch between the energy a step gains (matter plus
    radiation, summed over the cells) and the energy that crossed the
    boundary in it (from the multigroup face fluxes)."""
    import numpy as np
    nx, ny = prob.nx, prob.ny
    hx, hy = prob.lx / nx, prob.ly / ny
    nint = (nx - 1) * ny + nx * (ny - 1)
    gained = np.sum(prob.c_v * (got["T"] - prev["T"]) + (got["E_cell"] - prev["E_cell"]).sum(0)) * hx * hy
    sgn = np.concatenate([-np.ones(ny), np.ones(ny), -np.ones(nx), np.ones(nx)])
    lens = np.concatenate([np.full(ny, hy), np.full(ny, hy), np.full(nx, hx), np.full(nx, hx)])
    inflow = -(prob.c_dt / C) * np.sum(sgn * got["F_face"].sum(0)[nint:] * lens)
    return abs(gained - inflow) / abs(inflow)


def _oracle_mlqd_sample():
    """The oracle's multilevel step (unchanged) on a small Fleck-Cummings
    case: 4 x 4 cells of 1.5 cm, 4 groups, 8 x 2 directions, h_moc 0.3 cm,
    one step from T^0 at eps 1e-10.  Returns seconds per step."""
    import warnings
    import numpy as np
    import workloads as W
    from oracle import mlqd, rays, sweep
    p = W.fc_mlqd(1.5, 0.3, 8, 2, 4, nu_lo=0.3, nu_hi=30.0)
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc)
    st = sweep.initial_state(g, p.n_pol, p.state0)
    E0, F0 = mlqd.initial_low_order(p, W.C_LIGHT)
    t = time.time()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r = mlqd.outer_step(g, p, st, np.full(p.cells, p.T0), E0, F0, W.C_LIGHT, W.A_RAD, eps=1e-10)
    return time.time() - t, r["outer"], r["inner"]


def _restrict(y, n):
    """Cell averages of an n x n field on the n/2 x n/2 grid (cell i = iy n + ix)."""
    a = y.reshape(n, n)
    return 0.25 * (a[0::2, 0::2] + a[1::2, 0::2] + a[0::2, 1::2] + a[1::2, 1::2]).ravel()


def _refinement_rows(runs, key, L=6.0):
    """||Delta y_h|| = ||y_h - y_{2h}||_L2 over the slab at the last step (the
    finer solution restricted to the coarser grid by cell averages when the
    material grids differ), rho = ||Delta y_{2h}|| / ||Delta y_h|| and the
    relative difference ||Delta y_h|| / ||y_h||, for T and the grey E."""
    import numpy as np
    rows = []
    for prev, cur in zip(runs, runs[1:]):
        row = {"h_mat": cur["h_mat"], "h_moc": cur["h_moc"]}
        for name in ("T", "E"):
            yf, yc = cur[name], prev[name]
            n = int(round(np.sqrt(yf.size)))
            if yf.size != yc.size:
                yf = _restrict(yf, n)
                n //= 2
            h2 = (L / n) ** 2
            d = float(np.sqrt(np.sum((yf - yc) ** 2) * h2))
            row[f"d{name}"] = d
            row[f"d{name}_rel"] = d / float(np.sqrt(np.sum(yf ** 2) * h2))
            if rows and rows[-1].get(f"d{name}"):
                row[f"rho_{name}"] = rows[-1][f"d{name}"] / d if d > 0 else None
        rows.append(row)
    return rows


def _mlqd_leg(steps=5, h_mat=0.3, h_moc=0.01):
    """A short run of the multilevel time step (the --workload fc_mlqd leg)
    for the default bench line: `steps` steps from T^0 on the 20 x 20
    Fleck-Cummings grid, 17 groups, 144 directions."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2305_11998_amd import driver
    prob = W.fc_mlqd(h_mat, h_moc, 36, 4, 17, nu_lo=0.3, nu_hi=30.0)
    s = driver.MlqdSolver(prob, eps=1e-12, max_outer=200, max_inner=2000)
    s.reset()
    prev = dict(T=np.full(prob.cells, prob.T0), E_cell=4 * np.pi * prob.state0 / W.C_LIGHT)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    defect = 0.0
    total = 0.0
    for _ in range(steps):
        e0.record()
        s.step(1)
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
        got = s.solution()
        defect = max(defect, _fc_energy_defect(prob, prev, got, W.C_LIGHT))
        prev = got
    _say(f"multilevel steps: {total / steps:.1f} ms per step")
    return {"metric": "fc_mlqd_time_steps_per_s", "value": 1000.0 * steps / total, "unit": "steps/s",
            "ms_per_step": total / steps, "steps": steps,
            "mean_transport_iterations": sum(h[0] for h in s.history) / steps,
            "mean_low_order_iterations": sum(h[1] for h in s.history) / steps, "max_energy_defect": defect,
            "dtype": "f64",
            "workload": f"multilevel time steps from T^0, Fleck-Cummings, {prob.nx}x{prob.ny} cells (h_mat {h_mat} cm), "
                        f"17 groups, 144 directions, h_moc {h_moc} cm, eps 1e-12"}


def main_fc_mlqd(args):
    """Multilevel (MLQD) time steps on the Fleck-Cummings problem at the
    paper's counts: 6 x 6 cm, 17 groups, 144 directions (36 x 4), Delta t =
    0.02 ns, eps = c_v T with c_v = 0.5917 a_R, 1 keV Planckian entering at
    x = 0, T^0 = 1 eV; for each h_mat of --h-mat and h_moc of --h-moc,
    --steps time steps at tolerance --eps (uniform characteristics, or the
    paper's vertex-avoiding grid with --tubes).  Per step: transport (outer)
    and low-order (inner) iterations, time, and the energy-balance mismatch;
    per run the kernel-time share of the transport sweep (plan events).
    With several h_mat (one h_moc) or several h_moc (one h_mat), the
    refinement norms of the last step's T and grey E follow.  One JSON line
    per run, then a summary line."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2305_11998_amd import driver, lc
    mode = lc.LC_RAYS_TUBES if args.tubes else lc.LC_RAYS_UNIFORM
    runs = []
    for h_mat in args.h_mat:
        for h_moc in args.h_moc:
            prob = W.fc_mlqd(h_mat, h_moc, 36, 4, 17, nu_lo=0.3, nu_hi=30.0)
            t0 = time.time()
            rays = lc.lc_build_rays(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, h_moc, mode)
            s = driver.MlqdSolver(prob, rays=rays, eps=args.eps, max_outer=200, max_inner=2000)
            build_s = time.time() - t0
            lc.lc_plan_profile(s.plan, True)
            s.reset()
            prev = dict(T=np.full(prob.cells, prob.T0), E_cell=4 * np.pi * prob.state0 / W.C_LIGHT)
            rows, total_ms = [], 0.0
            for n in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.step(1)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                total_ms += ms
                got = s.solution()
                outer, inner, ch = s.history[-1]
                rows.append({"step": n + 1, "outer": outer, "inner": inner, "ms": round(ms, 3),
                             "T_max": float(got["T"].max()),
                             "energy_defect": _fc_energy_defect(prob, prev, got, W.C_LIGHT)})
                prev = got
                _say(f"h_mat {h_mat} h_moc {h_moc}: step {n + 1} outer {outer} inner {inner} {ms:.1f} ms "
                     f"T_max {got['T'].max():.4f}")
            prof = lc.lc_plan_profile_read(s.plan)
            r = s.rays
            upd = r.n_segments * 2 * r.n_pol * prob.G
            line = {"workload": "fc_mlqd", "h_mat": h_mat, "cells": prob.cells, "h_moc": h_moc,
                    "grid": "tubes" if args.tubes else "uniform", "characteristics": int(r.n_rays),
                    "segments": int(r.n_segments), "groups": prob.G, "directions": len(prob.omega), "eps": args.eps,
                    "steps": args.steps, "build_s": round(build_s, 2), "ms_per_step": total_ms / args.steps,
                    "mean_outer": sum(x["outer"] for x in rows) / args.steps,
                    "mean_inner": sum(x["inner"] for x in rows) / args.steps,
                    "sweep_ms_total": prof[0] if prof else None, "sweep_launches": prof[1] if prof else None,
                    "moments_ms_total": prof[2] if prof else None, "updates_per_sweep": int(upd),
                    "max_energy_defect": max(x["energy_defect"] for x in rows), "per_step": rows}
            if prof and prof[1]:
                # float64 sweep with face points: the previous state read, the new
                # state and the entering intensities written, 8 bytes each per update
                line["sweep_achieved_GBs"] = 24.0 * upd * prof[1] / (prof[0] * 1e-3) / 1e9
                line["sweep_frac_of_hbm"] = line["sweep_achieved_GBs"] / 8000.0
                line["sweep_share_of_step"] = prof[0] / total_ms
            print(json.dumps(line), flush=True)
            runs.append(dict(line, T=prev["T"], E=prev["E_grey"]))
            del s
            torch.cuda.empty_cache()
    main = runs[0]
    out = {"metric": "fc_mlqd_time_steps_per_s", "value": 1000.0 / main["ms_per_step"], "unit": "steps/s",
           "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "vs_baseline": None,
           "config": {"workload": f"multilevel time steps, Fleck-Cummings, {main['cells']} cells (h_mat "
                                  f"{main['h_mat']} cm), 17 groups, 144 directions, h_moc {main['h_moc']} cm "
                                  f"({main['grid']}), eps {args.eps}"},
           "mean_transport_iterations": main["mean_outer"], "mean_low_order_iterations": main["mean_inner"]}
    if len(runs) > 1 and (len(args.h_mat) == 1 or len(args.h_moc) == 1):
        out["refinement"] = _refinement_rows(runs, "h_mat" if len(args.h_moc) == 1 else "h_moc")
    if not args.no_cpu_baseline:
        sec, outer, inner = _oracle_mlqd_sample()
        out["cpu_baseline"] = {"value": 1.0 / sec, "unit": "steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"one step of a 4x4-cell, 4-group, 16-direction Fleck-Cummings case "
                                         f"(h_moc 0.3 cm, eps 1e-10): {sec:.2f} s, {outer} transport and {inner} "
                                         f"low-order iterations; a far smaller problem than the timed one"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("batch", "single", "refinement", "split", "fc_mlqd"), default="batch",
                    help="batch: the 64-problem batched form (default); single: one problem of --config; "
                         "refinement: characteristic-grid refinement study; split: whole vs split sweep "
                         "on few-lane problems; fc_mlqd: multilevel time steps on Fleck-Cummings")
    ap.add_argument("--h-mat", type=float, nargs="+", default=[0.6], help="--workload fc_mlqd: material cell widths")
    ap.add_argument("--h-moc", type=float, nargs="+", default=[0.01], help="--workload fc_mlqd: characteristic spacings")
    ap.add_argument("--tubes", action="store_true", help="--workload fc_mlqd: the paper's vertex-avoiding grid")
    ap.add_argument("--eps", type=float, default=1e-12, help="--workload fc_mlqd: iteration tolerance")
    ap.add_argument("--config", type=int, default=2, help="workload index for --workload single (0, 1, 2 or 4)")
    ap.add_argument("--case", type=int, default=None, help="--workload split: run only this case (0, 1 or 2)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--f64-steps", type=int, default=2)
    ap.add_argument("--check-steps", type=int, default=5,
                    help="steps over which the float32 moments are compared with float64 ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-mlqd", action="store_true", help="leave the short multilevel-step leg out of the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 4 GiB buffer three times (scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding the groups over "
              "several GPUs is a design only, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2305_11998_amd import lc

    torch.cuda.init()
    if args.copy_calibration:
        n = 1 << 30                                      # 2^30 float32 = 4 GiB
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        _say(f"copied 3 x {n * 4} bytes")
        return
    if args.workload == "split":
        return main_split(args)
    if args.workload == "refinement":
        main_refinement(args)
        return
    if args.workload == "fc_mlqd":
        main_fc_mlqd(args)
        return
    if args.workload == "single":
        main_single(args)
        return
    t0 = time.time()
    probs = W.batch_problems(steps=1)
    _say(f"64 problems generated in {time.time() - t0:.0f} s")
    r32 = run_batched(probs, args.steps, args.warmup, lc.LC_F32,
                      snapshot_steps=0 if args.no_f64 else args.check_steps)
    bs = r32.pop("bs")
    upd = bs.updates_per_step()
    alg = sum(sweep_algorithmic_bytes(s, 4) for s in bs.solvers)
    step_alg = sum(step_algorithmic_bytes(s, 4) for s in bs.solvers)
    ms32 = r32["ms"] / args.steps
    _say(f"f32 batched: {ms32:.3f} ms/step (eager, phase by phase {r32['ms_eager'] / args.steps:.3f}), "
         f"sweep {r32['sweep_ms']:.3f} ms, moments {r32['moments_ms']:.3f} ms, "
         f"prologue {r32['prologue_ms']:.3f} ms, {upd} updates/step")
    snaps = r32.pop("snapshots")
    del bs
    torch.cuda.empty_cache()

    out_f64, out_f64b, errs = None, None, None
    if not args.no_f64:
        r64b = run_batched(probs, args.steps, args.warmup, lc.LC_F64)
        bs64 = r64b.pop("bs")
        alg64 = sum(sweep_algorithmic_bytes(s, 8) for s in bs64.solvers)
        del bs64
        torch.cuda.empty_cache()
        ms64b = r64b["ms"] / args.steps
        out_f64b = {"value": upd / (ms64b / 1e3), "unit": "segment-updates/s", "ms_per_step": ms64b,
                    "sweep_ms": r64b["sweep_ms"], "moments_ms": r64b["moments_ms"],
                    "sweep_achieved_GBs": alg64 / (r64b["sweep_ms"] / 1e3) / 1e9,
                    "tuning": r64b["tuning"]["per_class"],
                    "form": "float64 batched: the same launches and graph-captured steps as the float32 form"}
        _say(f"f64 batched: {ms64b:.3f} ms/step, sweep {r64b['sweep_ms']:.3f} ms, "
             f"moments {r64b['moments_ms']:.3f} ms")
        r64 = run_plain_f64(probs, args.f64_steps, snaps)
        errs = dict(r64["worst"], steps_checked=len(snaps), per_step=r64["per_step"])
        v64 = r64["updates"] / (r64["ms_per_step"] / 1e3)
        out_f64 = {"value": v64, "unit": "segment-updates/s", "ms_per_step": r64["ms_per_step"],
                   "form": "plain float64 sweep + moments, problem by problem"}
        _say(f"f64 plain: {r64['ms_per_step']:.3f} ms/step; f32 vs f64 max errors over "
             f"{len(snaps)} steps {r64['worst']}")
    del snaps
    torch.cuda.empty_cache()

    value = upd / (ms32 / 1e3)
    achieved = alg / (r32["sweep_ms"] / 1e3) / 1e9
    step_achieved = step_alg / (ms32 / 1e3) / 1e9
    traffic = recorded_traffic(r32["tuning"]["per_class"])
    out = {
        "metric": "segment-updates/s, FP32 batched vs FP64 sweep at <=1e-5 rel error",
        "value": value,
        "unit": "segment-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Fleck-Cummings-type problems, smooth temperature fields)",
        "config": {"workload": "batched form: 64 independent problems, meshes {32,64,128,256}^2 on 6x6 cm, "
                               "G in {8,17,51}, 16/64/128 directions, spacing h/2, float32 sweep with "
                               "Kahan moments, one launch per phase and polar group",
                   "updates_per_step": upd, "eager_ms_per_step": r32["ms_eager"] / args.steps,
                   "tuning": r32["tuning"]["per_class"]},
        "fp64_plain": out_f64,
        "fp64_batched": out_f64b,
        "speedup_vs_fp64": (value / out_f64["value"]) if out_f64 else None,
        "speedup_vs_fp64_batched": (value / out_f64b["value"]) if out_f64b else None,
        "fp32_vs_fp64_max_err": errs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": "recorded: rocprofv3 FETCH_SIZE + WRITE_SIZE of the same sweep sources "
                                       "(profiles/sweep_batch_traffic.txt, source hash checked), scaled by a "
                                       "plain copy's counts",
                     "kernel": "k_sweep_batch<float,PM,U> (one launch per polar group, summed)",
                     "kernel_ms": r32["sweep_ms"],
                     "moments_kernel_ms": r32["moments_ms"], "algorithmic_bytes_per_launch": alg,
                     "step_algorithmic_bytes": step_alg, "step_achieved": step_achieved,
                     "step_frac": step_achieved / HBM_PEAK_GBS},
    }
    if not args.no_mlqd:
        out["fc_mlqd"] = _mlqd_leg()
    if not args.no_cpu_baseline:
        _say("cpu baseline (oracle sample)")
        big = max(range(len(probs)), key=lambda j: probs[j].cells * probs[j].G * probs[j].M)
        out["cpu_baseline"] = cpu_baseline(probs[big], big)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
