"""Autotuner for the launch parameters of a plan.

For a plan and its buffers it times every candidate of each tunable launch
parameter with the library's own kernel timers (HIP events around the sweep
and the cell-moment kernels) and keeps the fastest.  The sweep parameter and
the moments parameter are independent, so each is searched on its own.
Results are cached in a JSON file keyed by the shape class of the problem
(precision, groups, polar angles, azimuth pairs, and the cell and segment
counts rounded to powers of two), so a second problem of the same class
reuses them without timing.
"""
from __future__ import annotations

import json
import sys
import math
import os

from . import lc

SWEEP_CANDIDATES = (2, 4, 8)
SWEEP_CANDIDATES_F32 = (2, 4, 8, 16)   # 16: float32 with at most MAX_POL_UNROLL16 polar angles
MAX_POL_UNROLL16 = 4
MOMENT_CANDIDATES = (1, 2, 3, 4)
SPLIT_CANDIDATES = (0, 32, 64, 128, 256)   # chunk steps of the split sweep, 0 = whole traversals
MIN_GAIN = 0.97            # an uncapped or split sweep is kept only if at least 3% faster than the default
BASE = (4, 3)             # the setting the other parameter is held at while one is searched
DEFAULT_CACHE = os.environ.get(
    "LC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lc_tuning.json"))


def shape_key(plan) -> str:
    r = plan.rays
    b = lambda x: int(round(math.log2(max(int(x), 1))))
    return (f"v{lc.lc_version()}-prec{plan.prec}-G{plan.G}-P{r.n_pol}-A{r.n_pairs}-"
            f"c{b(r.cells)}-s{b(r.n_segments)}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def sweep_candidates(prec: int, n_pol: int):
    """The sweep_unroll values the library accepts for this precision and
    polar count, in search order."""
    return SWEEP_CANDIDATES_F32 if prec == lc.LC_F32 and n_pol <= MAX_POL_UNROLL16 else SWEEP_CANDIDATES


def tune(solver, reps: int = 3, cache: str | None = DEFAULT_CACHE, verbose: bool = False):
    """Pick (sweep_unroll, moments_entries), then the residency cap of the
    whole-traversal sweep, then the split sweep's chunk length (0 = whole
    traversals), for ``solver.plan`` by timing ``reps`` eager steps per
    candidate.  Leaves the choice set on the plan and returns it with the
    measured times (ms per launch)."""
    import torch
    plan = solver.plan
    key = shape_key(plan)
    db = _load(cache) if cache else {}
    if key in db:
        t = db[key]
        lc.lc_plan_set_tuning(plan, t["sweep_unroll"], t["moments_entries"])
        lc.lc_plan_set_sweep_residency(plan, t.get("sweep_capped", 1))
        lc.lc_plan_set_split(plan, t.get("split", 0))
        return dict(t, cached=True, key=key)
    lc.lc_plan_set_split(plan, 0)
    lc.lc_plan_set_sweep_residency(plan, 1)
    def timed():
        """(sweep, moments) ms per launch over reps eager steps, after one warm step."""
        solver.bench_step()
        torch.cuda.synchronize()
        lc.lc_plan_profile_read(plan)
        lc.lc_plan_profile(plan, True)
        for _ in range(reps):
            solver.bench_step()
        torch.cuda.synchronize()
        sw, nsw, mo, nmo = lc.lc_plan_profile_read(plan)
        lc.lc_plan_profile(plan, False)
        return sw / max(nsw, 1), mo / max(nmo, 1)

    times = {}
    # the two parameters act on different kernels: vary one with the other fixed
    ucands = sweep_candidates(plan.prec, plan.rays.n_pol)
    combos = sorted({(u, BASE[1]) for u in ucands} | {(BASE[0], e) for e in MOMENT_CANDIDATES})
    for u, e in combos:
        lc.lc_plan_set_tuning(plan, u, e)
        times[(u, e)] = timed()
        if verbose:
            print(f"  tune {key}: unroll {u} entries {e}: sweep {times[(u, e)][0]:.3f} ms, "
                  f"moments {times[(u, e)][1]:.3f} ms", file=sys.stderr, flush=True)
    best_u = min(ucands, key=lambda u: times[(u, BASE[1])][0])
    best_e = min(MOMENT_CANDIDATES, key=lambda e: times[(BASE[0], e)][1])
    lc.lc_plan_set_tuning(plan, best_u, best_e)
    # the residency cap of the whole-traversal sweep (kept unless lifting it
    # is at least 3% faster: small problems, where the tail dominates)
    cap_ms = {1: timed()[0]}
    lc.lc_plan_set_sweep_residency(plan, 0)
    cap_ms[0] = timed()[0]
    best_c = 0 if cap_ms[0] <= MIN_GAIN * cap_ms[1] else 1
    lc.lc_plan_set_sweep_residency(plan, best_c)
    if verbose:
        print(f"  tune {key}: residency capped {cap_ms[1]:.3f} ms, uncapped {cap_ms[0]:.3f} ms",
              file=sys.stderr, flush=True)
    # then the split sweep's chunk length (its own load chunk is fixed, so
    # the unroll above does not act on it); few-lane problems gain from it
    split_ms = {}
    for sp in SPLIT_CANDIDATES:
        lc.lc_plan_set_split(plan, sp)
        split_ms[sp] = timed()[0]
        if verbose:
            print(f"  tune {key}: split {sp}: sweep {split_ms[sp]:.3f} ms", file=sys.stderr, flush=True)
    best_s = min(split_ms, key=split_ms.get)
    if split_ms[best_s] > MIN_GAIN * split_ms[0]:
        best_s = 0
    lc.lc_plan_set_split(plan, best_s)
    res = dict(sweep_unroll=best_u, moments_entries=best_e, sweep_capped=best_c, split=best_s,
               sweep_ms={str(k): v[0] for k, v in times.items()},
               moments_ms={str(k): v[1] for k, v in times.items()},
               capped_ms={str(k): v for k, v in cap_ms.items()},
               split_ms={str(k): v for k, v in split_ms.items()})
    if cache:
        db[key] = res
        _save(cache, db)
    return dict(res, cached=False, key=key)


def tune_batch(bs, steps: int = 2, verbose: bool = False):
    """Pick (sweep_unroll, moments_entries) per polar class of a BatchSolver
    (the library launches each class separately, with the tuning of its
    members' plans).  Each class is searched in turn with the others held at
    their current choice, timing the batch's launches (lc_batch_profile);
    the batch is left rebuilt with the choice."""
    import torch
    classes = bs.classes()
    best = {pm: list(BASE) for pm in classes}

    def run(cfg):
        bs.rebuild({pm: tuple(v) for pm, v in cfg.items()})
        lc.lc_batch_profile(bs.batch, True)
        bs.reset()
        bs.step(steps)
        torch.cuda.synchronize()
        pro, npro, sw, nsw, mo, nmo = lc.lc_batch_profile_read(bs.batch)
        lc.lc_batch_profile(bs.batch, False)
        return sw / max(nsw, 1), mo / max(nmo, 1)

    times = {}
    for pm in classes:
        ucands = sweep_candidates(bs.solvers[0].plan.prec, pm)
        for k, cands in ((0, ucands), (1, MOMENT_CANDIDATES)):
            res = {}
            for v in cands:
                cfg = {c: list(x) for c, x in best.items()}
                cfg[pm][k] = v
                res[v] = run(cfg)[k]
                times[(pm, k, v)] = res[v]
                if verbose:
                    what = "unroll" if k == 0 else "entries"
                    print(f"  tune batch: polar class {pm} {what} {v}: "
                          f"{'sweep' if k == 0 else 'moments'} {res[v]:.3f} ms", file=sys.stderr, flush=True)
            best[pm][k] = min(res, key=res.get)
    bs.rebuild({pm: tuple(v) for pm, v in best.items()})
    return dict(per_class={str(pm): dict(sweep_unroll=v[0], moments_entries=v[1]) for pm, v in best.items()},
                times={f"{pm}/{'unroll' if k == 0 else 'entries'}/{v}": t for (pm, k, v), t in times.items()})
