"""The sampled oracle (``solve.run_sampled``) for several blocks of samples in
parallel worker processes.

Characteristics evolve independently under prescribed material data, so
the moments of a block of cells (and the factors of a block of boundary
faces) come from that block's characteristics alone: each worker rebuilds
the problem from its recipe, traces the characteristics its block needs and
runs the oracle's time loop over them.  The blocks' results are only put
side by side.  Workers are spawned (fresh interpreters): they import numpy,
the oracle and the input generators, never the GPU library or torch."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def problem(recipe):
    """("config", k, steps) -> workloads.config(k, steps);
    ("batch", j, steps) -> member j of workloads.batch_problems(steps)."""
    import workloads as W
    kind, idx, steps = recipe
    if kind == "config":
        return W.config(idx, steps=steps)
    if kind == "batch":
        return W.batch_problems(steps=steps, only=[idx])[0]
    raise ValueError(recipe)


def _job(args):
    recipe, cells, faces = args
    from oracle import rays, solve
    p = problem(recipe)
    g = rays.build(p.nx, p.ny, p.lx, p.ly, p.phi, p.h_moc, only_cells=cells,
                   only_faces=faces if len(faces) else None)
    out = solve.run_sampled(p, g, cells, faces=faces if len(faces) else None)
    return out["steps"]


def workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run_blocks(jobs):
    """jobs: list of (recipe, cells, faces).  Returns, per job, the oracle's
    per-step list of {E, F, f[, bnd]} for its cells (and faces)."""
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers(), len(jobs))) as pool:
        return pool.map(_job, [(r, np.asarray(c, dtype=np.int64), np.asarray(f, dtype=np.int64))
                               for r, c, f in jobs], chunksize=1)


def blocks(items, n):
    """Split a sorted sample into n nearly equal consecutive blocks."""
    return [b for b in np.array_split(np.asarray(items, dtype=np.int64), n)]
