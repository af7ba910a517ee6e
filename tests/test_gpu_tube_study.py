"""GPU: the paper's vertex-avoiding, width-halving characteristic grid at the
sizes of the transport-only refinement study (bench.py --workload
refinement): a Fleck-Cummings-like slab on 40 x 40 cells of 0.15 cm (6 x 6 cm),
17 groups, 36 x 4 directions, one backward-Euler step, float64, with
h_moc = h / 16 and h / 64 (the finest grid of the study at this material
mesh has about 92,000 characteristics and 3.8 million segments).  Sampled
cells (corners, domain edges, random ones) and boundary faces against the
oracle, which traces and sweeps only the characteristics reaching them."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import rays as orays, solve as osolve
from tests.parity_util import bnd_errors, err_E, err_F, err_f, sample_cells, sample_faces

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _slab(n, ratio):
    L = 6.0
    h = L / n
    x = (np.arange(n) + 0.5) * h
    T = np.tile(1.0 * np.exp(-x / 1.0) + 0.001, n)          # cell i = iy * n + ix
    return W.make_problem(n, n, L, L, 36, 4, 17, 0.001, 30.0, h / ratio, 0.6, [T], name=f"fc{n}_r{ratio}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("ratio", [16, 64])
def test_tube_grid_at_study_size(ratio):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_11998_amd import driver, lc
    prob = _slab(40, ratio)
    _say(f"case tube study 40x40 h/{ratio}: GPU")
    s = driver.Solver(prob, prec=lc.LC_F64, mode=lc.LC_RAYS_TUBES)
    _say(f"  {s.rays.n_rays} characteristics, {s.rays.n_segments} segments")
    s.reset()
    s.step(1)
    got = s.moments()
    cells = sample_cells(prob.nx, prob.ny, 12, ratio)
    faces, _ = sample_faces(prob, 6, ratio, mode=orays.TUBES)
    _say(f"  oracle on {len(cells)} cells and {len(faces)} faces")
    g = orays.build(prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.h_moc, orays.TUBES, only_cells=cells,
                    only_faces=faces)
    ref = osolve.run_sampled(prob, g, cells, faces=faces)["steps"][-1]
    c = W.C_LIGHT
    eE = err_E(got["E"][:, cells], ref["E"])
    eF = err_F(got["F"][:, :, cells], ref["F"], ref["E"], c)
    ef = err_f(got["f"][:, :, cells], ref["f"], ref["E"])
    eb, ebc = bnd_errors(got["bnd"][:, faces], ref["bnd"], floor=0.0)
    _say(f"  E {eE:.2e} F {eF:.2e} f {ef:.2e} bnd {eb:.2e} / C,f_b {ebc:.2e}")
    assert max(eE, eF, ef, eb, ebc) <= 1e-12
