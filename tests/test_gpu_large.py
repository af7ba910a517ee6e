"""GPU: the largest single-GPU workload -- 512x512 cells, 51 groups, 288
directions (48 azimuths x 6 polar), spacing h/2, a temperature front moving
0.25 cm per step, 10 backward-Euler steps -- run as the float32 sweep, with a
float64 run beside it checking the moments on 1% of the cells after every
step, and the oracle checking a few cells after the last step."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays, solve as osolve
from tests.parity_util import err_E, err_F, err_f

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sampled(solver, idx):
    """Moments [g][component][sampled cell], gathered on the device."""
    return {k: v[:, :, idx].cpu().numpy() for k, v in solver.moment_views().items()}


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
    # the float64 run against the oracle on a few cells after the last step
    few = np.concatenate([rng.choice(cells, 3, replace=False), [0, cells - 1]])
    m64 = _sampled(s64, torch.from_numpy(few).cuda())
    del s32, s64
    torch.cuda.empty_cache()
    _say("  oracle on 5 cells, 10 steps")
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, only_cells=few)
    ref = osolve.run_sampled(prob, g, few)["steps"][-1]
    eE = err_E(m64["E"][:, 0], ref["E"])
    eF = err_F(m64["F"], ref["F"], ref["E"], c)
    ef = err_f(m64["f"], ref["f"], ref["E"])
    _say(f"  f64 vs oracle: E {eE:.2e} F {eF:.2e} f {ef:.2e}")
    assert eE <= 1e-12 and eF <= 1e-12 and ef <= 1e-12
