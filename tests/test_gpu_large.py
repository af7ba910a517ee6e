"""GPU: the largest single-GPU workload -- 512x512 cells, 51 groups, 288
directions (48 azimuths x 6 polar), spacing h/2, a temperature front moving
0.25 cm per step, 10 backward-Euler steps -- run as the float32 sweep, with a
float64 run beside it checking the moments on 1% of the cells after every
step, and the oracle checking 64 cells (corners, domain edges, both sides of
moment-tile edges, random ones) and 16 boundary faces after the last
step."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays, solve as osolve
from tests import oracle_pool
from tests.parity_util import bnd_errors, err_E, err_F, err_f, sample_cells, sample_faces

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sampled(solver, idx):
    """Moments [g][component][sampled cell], gathered on the device."""
    return {k: v[:, :, idx].cpu().numpy() for k, v in solver.moment_views().items()}


@pytest.mark.timeout(900)
def test_largest_problem_fp32_with_per_step_fp64_check():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_11998_amd import driver, lc
    torch.cuda.empty_cache()
    prob = W.config(4)
    G, cells = prob.G, prob.cells
    _say(f"512^2: G={G}, M={prob.M}, {prob.steps} steps")
    s32 = driver.Solver(prob, prec=lc.LC_F32)
    s64 = driver.Solver(prob, prec=lc.LC_F64, rays=s32.rays)
    _say(f"  state bytes: f32 {s32.plan.state_bytes / 1e9:.1f} GB, f64 {s64.plan.state_bytes / 1e9:.1f} GB per buffer")
    rng = np.random.default_rng(2305)
    idx_np = np.sort(rng.choice(cells, cells // 100, replace=False))
    idx = torch.from_numpy(idx_np).cuda()
    s32.reset()
    s64.reset()
    c = W.C_LIGHT
    worst = dict(E=0.0, F=0.0, f=0.0)
    for t in range(prob.steps):
        s32.step(1)
        s64.step(1)
        torch.cuda.synchronize()
        a = _sampled(s32, idx)
        b = _sampled(s64, idx)
        e = dict(E=err_E(a["E"][:, 0], b["E"][:, 0]), F=err_F(a["F"], b["F"], b["E"][:, 0], c),
                 f=err_f(a["f"], b["f"], b["E"][:, 0]))
        _say(f"  step {t}: f32 vs f64 on {len(idx_np)} cells: E {e['E']:.2e} F {e['F']:.2e} f {e['f']:.2e}")
        for k in worst:
            worst[k] = max(worst[k], e[k])
    assert worst["E"] <= 1e-5 and worst["F"] <= 1e-5 and worst["f"] <= 1e-5, worst
    # the float64 run against the oracle on 64 cells and 16 boundary faces
    # after the last step
    few = sample_cells(prob.nx, prob.ny, 64, 4)
    faces, _ = sample_faces(prob, 16, 4)
    m64 = _sampled(s64, torch.from_numpy(few).cuda())
    b64 = s64.bnd.view(G, -1, 8)[:, torch.from_numpy(faces).cuda()].cpu().numpy()
    del s32, s64
    torch.cuda.empty_cache()
    nblk = 16
    jobs = [(("config", 4, prob.steps), cb, fb)
            for cb, fb in zip(oracle_pool.blocks(few, nblk), oracle_pool.blocks(faces, nblk))]
    _say(f"  oracle on {len(few)} cells and {len(faces)} faces, {prob.steps} steps, "
         f"{len(jobs)} blocks on {oracle_pool.workers()} processes")
    res = oracle_pool.run_blocks(jobs)
    last = [r[-1] for r in res]
    ref = {k: np.concatenate([r[k] for r in last], axis=-1) for k in ("E", "F", "f")}
    ref_b = np.concatenate([r["bnd"] for r in last], axis=1)
    eE = err_E(m64["E"][:, 0], ref["E"])
    eF = err_F(m64["F"], ref["F"], ref["E"], c)
    ef = err_f(m64["f"], ref["f"], ref["E"])
    eb, ebc = bnd_errors(b64, ref_b, floor=0.0)
    _say(f"  f64 vs oracle: E {eE:.2e} F {eF:.2e} f {ef:.2e} bnd {eb:.2e} / C,f_b {ebc:.2e}")
    assert eE <= 1e-12 and eF <= 1e-12 and ef <= 1e-12
    assert eb <= 1e-12 and ebc <= 1e-12
