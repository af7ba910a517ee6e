#!/usr/bin/env python3
"""Benchmark of the long-characteristics transport step on one MI355X.

A "step" is one backward-Euler transport step of the whole workload: the
sweep (eq. (10)-(13)) over every characteristic, direction and group, then
the cell moments and boundary factors (eq. (7), (14)-(16)).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

Throughput is in segment-updates/s: one update is one evaluation of the
segment propagation for one (segment, traversal, polar angle, group).
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
    """Bytes one sweep launch must move at minimum: the stored segment
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


def run_gpu(prob, prec, steps, warmup):
    import torch
    from paper_2305_11998_amd import driver, lc, tune
    s = driver.Solver(prob, prec=prec)
    s.reset()
    tuned = tune.tune(s, cache=None, verbose=True)
    _say(f"tuning: unroll {tuned['sweep_unroll']}, entries {tuned['moments_entries']}")
    s.reset()
    s.tuning = tuned
    lc.lc_plan_profile(s.plan, False)
    for _ in range(warmup):
        s.bench_step()
    torch.cuda.synchronize()
    lc.lc_plan_profile_read(s.plan)
    lc.lc_plan_profile(s.plan, True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        s.bench_step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sw_ms, sw_n, mo_ms, mo_n = lc.lc_plan_profile_read(s.plan)
    lc.lc_plan_profile(s.plan, False)
    return s, ms, sw_ms / max(sw_n, 1), mo_ms / max(mo_n, 1)


def cpu_baseline(prob, budget_s=12.0):
    """The oracle's sweep (unchanged) on a bounded sample of the same
    workload: characteristics of the first azimuth pair, both traversals, all
    polar angles and groups, as many characteristics as fit the budget."""
    import numpy as np
    from oracle import rays as orays, sweep as osweep
    P, G = prob.n_pol, prob.G
    half = prob.n_az // 2
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi[[0, half]], prob.h_moc)
    pr = g.pairs[0]
    cols = list(range(P)) + list(range(half * P, half * P + P))
    I_in = prob.I_in[:, cols, :]
    order = np.argsort(-pr.nseg)              # typical lengths: start from the middle
    ks = np.sort(order[len(order) // 4:])
    done_upd, t_used, n_rays = 0, 0.0, 0
    chunk = 16
    q = 0
    while t_used < budget_s:
        if q >= len(ks):                      # all sampled characteristics done: sweep them again
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
    return dict(value=done_upd / t_used, unit="segment-updates/s", cores=1, kind="oracle",
                sample=f"oracle FP64 sweep of {n_rays} characteristics of azimuth pair 0 "
                       f"(both traversals, {P} polar angles, {G} groups, {done_upd} updates, "
                       f"{t_used:.1f} s, numpy on one host thread)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "is a design described in DESIGN.md, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2305_11998_amd import lc
    from tests.parity_util import err_E, err_F, err_f

    torch.cuda.init()
    prob = W.config(2)
    _say("workload ready: 256x256, G=51, 32x4 directions, spacing h/2")
    s32, ms32, sw32, mo32 = run_gpu(prob, lc.LC_F32, args.steps, args.warmup)
    _say(f"f32: {ms32 / args.steps:.3f} ms/step, sweep kernel {sw32:.3f} ms, moments {mo32:.3f} ms")
    m32 = s32.moments()
    tun32 = {k: s32.tuning[k] for k in ("sweep_unroll", "moments_entries")}
    upd = s32.updates_per_step()
    alg32 = sweep_algorithmic_bytes(s32, 4)
    del s32
    torch.cuda.empty_cache()
    s64, ms64, sw64, mo64 = run_gpu(prob, lc.LC_F64, args.steps, args.warmup)
    _say(f"f64: {ms64 / args.steps:.3f} ms/step, sweep kernel {sw64:.3f} ms, moments {mo64:.3f} ms")
    m64 = s64.moments()
    del s64
    torch.cuda.empty_cache()
    c = W.C_LIGHT
    errs = dict(E=err_E(m32["E"], m64["E"]), F=err_F(m32["F"], m64["F"], m64["E"], c),
                f=err_f(m32["f"], m64["f"], m64["E"]))
    _say(f"f32 vs f64 GPU: {errs}")

    value = upd * args.steps / (ms32 / 1e3)
    value64 = upd * args.steps / (ms64 / 1e3)
    achieved = alg32 / (sw32 / 1e3) / 1e9
    out = {
        "metric": "segment-updates/s, FP32 batched vs FP64 sweep at <=1e-5 rel error",
        "value": value,
        "unit": "segment-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Fleck-Cummings-type sharp-front temperature field)",
        "config": {"workload": "single problem, 256x256 cells on 6x6 cm, G=51 groups 0.001-30 keV, "
                               "128 directions (32 azimuths x 4 polar), spacing h/2, FP32 sweep with "
                               "Kahan moments", "updates_per_step": upd, "tuning": tun32},
        "fp64": {"value": value64, "ms_per_step": ms64 / args.steps, "sweep_kernel_ms": sw64,
                 "moments_kernel_ms": mo64},
        "fp32_vs_fp64_max_err": errs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep<float,P=4,sym>", "kernel_ms": sw32,
                     "algorithmic_bytes_per_launch": alg32},
    }
    if not args.no_cpu_baseline:
        _say("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
