"""Run whole transport problems through the C ABI with PyTorch device memory.

``Solver`` uploads a problem's inputs once (opacities, Planck sources and
boundary intensities for every step), builds the characteristic grid and a
plan, and advances the per-segment state with ``lc_step`` (graph-captured) or
with explicit ``lc_sweep`` / ``lc_moments`` calls.  All arithmetic of the
method happens in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lc


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


class Solver:
    def __init__(self, prob, prec=lc.LC_F64, mode=lc.LC_RAYS_UNIFORM, c=None, rays=None, split=0):
        """split > 0: sweep traversals in chunks of that many steps
        (lc_plan_set_split)."""
        from workloads import C_LIGHT
        self.prob = prob
        self.c = C_LIGHT if c is None else float(c)
        self.prec = prec
        self.rays = rays if rays is not None else lc.lc_build_rays(
            prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, prob.h_moc, mode)
        self.plan = lc.Plan(self.rays, prob.G, prec)
        if split:
            lc.lc_plan_set_split(self.plan, split)
        G, cells = prob.G, prob.cells
        self.kappa = _dev(np.stack(prob.kappa))          # [steps][G][cells]
        self.planck = _dev(np.stack(prob.planck))
        self.stride = G * cells if prob.steps > 1 else 0
        self.I_in = _dev(prob.I_in)
        self.state0 = _dev(prob.state0)
        self.state = [self.plan.new_state(), self.plan.new_state()]
        r = self.rays
        self.I_exit = torch.zeros(r.n_rays * 2 * r.n_pol * G, dtype=torch.float64, device="cuda")
        self.E = torch.zeros(G * cells, dtype=torch.float64, device="cuda")
        self.F = torch.zeros(2 * G * cells, dtype=torch.float64, device="cuda")
        self.f = torch.zeros(4 * G * cells, dtype=torch.float64, device="cuda")
        self.bnd = torch.zeros(G * r.nb * 8, dtype=torch.float64, device="cuda")
        self.cur = 0
        self.t = 0

    def reset(self):
        lc.lc_state_fill(self.plan, self.state0, self.state[0])
        self.cur = 0
        self.t = 0

    def step(self, n=1, graph=True):
        """Advance n steps from the current state (material data of steps
        t .. t+n-1) and leave the last step's moments in E, F, f, bnd."""
        p = self.prob
        t0 = self.t
        if t0 + n > p.steps:
            raise ValueError("not enough material steps")
        off = t0 * self.stride
        kap = self.kappa.view(-1)[off:]
        pla = self.planck.view(-1)[off:]
        if graph:
            lc.lc_step(self.plan, n, kap, pla, p.c_dt, self.c, self.state[self.cur],
                       self.state[1 - self.cur], self.I_in, self.I_exit, self.E, self.F, self.f,
                       self.bnd, material_stride=self.stride)
        else:
            for t in range(n):
                o = t * self.stride
                lc.lc_sweep(self.plan, kap[o:], pla[o:], p.c_dt, self.state[(self.cur + t) % 2],
                            self.state[(self.cur + t + 1) % 2], self.I_in, self.I_exit)
            lc.lc_moments(self.plan, self.state[(self.cur + n) % 2], self.c, self.E, self.F, self.f,
                          self.bnd, self.I_exit, self.I_in)
        self.cur = (self.cur + n) % 2
        self.t += n

    def enable_faces(self):
        """Interior-face lists on the plan, a buffer for the upwind-face
        intensities and the face outputs."""
        lc.lc_plan_enable_faces(self.plan)
        G = self.prob.G
        nf = lc.n_interior_faces(self.rays)
        self.points = self.plan.new_state()
        self.Ef = torch.zeros(nf * G, dtype=torch.float64, device="cuda")
        self.Ff = torch.zeros(2 * nf * G, dtype=torch.float64, device="cuda")
        self.ff = torch.zeros(4 * nf * G, dtype=torch.float64, device="cuda")

    def step_faces(self, n=1):
        """Like step(n, graph=False), storing the upwind-face intensities of
        every sweep; leaves the last step's cell and interior-face moments."""
        p = self.prob
        t0 = self.t
        if t0 + n > p.steps:
            raise ValueError("not enough material steps")
        off = t0 * self.stride
        kap = self.kappa.view(-1)[off:]
        pla = self.planck.view(-1)[off:]
        for t in range(n):
            o = t * self.stride
            lc.lc_sweep_points(self.plan, kap[o:], pla[o:], p.c_dt, self.state[(self.cur + t) % 2],
                               self.state[(self.cur + t + 1) % 2], self.I_in, self.points, self.I_exit)
        new = self.state[(self.cur + n) % 2]
        lc.lc_moments(self.plan, new, self.c, self.E, self.F, self.f, self.bnd, self.I_exit, self.I_in)
        lc.lc_face_moments(self.plan, self.points, new, self.c, self.Ef, self.Ff, self.ff)
        self.cur = (self.cur + n) % 2
        self.t += n

    def face_moments(self):
        """Interior-face E [G][faces], F [G][2][faces], f [G][4][faces]."""
        G = self.prob.G
        nf = lc.n_interior_faces(self.rays)
        return dict(E=self.Ef.cpu().numpy().reshape(nf, G).T,
                    F=self.Ff.cpu().numpy().reshape(nf, 2, G).transpose(2, 1, 0),
                    f=self.ff.cpu().numpy().reshape(nf, 4, G).transpose(2, 1, 0))

    def bench_step(self):
        """One step with the first step's material data (for timing): eager
        sweep then moments, state ping-pong."""
        p = self.prob
        nxt = 1 - self.cur
        lc.lc_sweep(self.plan, self.kappa, self.planck, p.c_dt, self.state[self.cur], self.state[nxt],
                    self.I_in, self.I_exit)
        lc.lc_moments(self.plan, self.state[nxt], self.c, self.E, self.F, self.f, self.bnd,
                      self.I_exit, self.I_in)
        self.cur = nxt

    def moments(self):
        p = self.prob
        G, cells = p.G, p.cells
        # The library writes cell-major arrays; hand out [G][...][cells] views.
        return dict(E=self.E.cpu().numpy().reshape(cells, G).T,
                    F=self.F.cpu().numpy().reshape(cells, 2, G).transpose(2, 1, 0),
                    f=self.f.cpu().numpy().reshape(cells, 4, G).transpose(2, 1, 0),
                    bnd=self.bnd.cpu().numpy().reshape(G, self.rays.nb, 8))

    def moment_views(self):
        """Device views of E, F, f indexed [g][component][cell] (E has one
        component); no copy."""
        G, cells = self.prob.G, self.prob.cells
        return {k: getattr(self, k).view(cells, n, G).permute(2, 1, 0)
                for k, n in (("E", 1), ("F", 2), ("f", 4))}

    def grey_closures(self):
        """Grey closures (lc_grey_closures) of the moments left by the last
        step, with that step's opacity and Planck source: [13][cells]."""
        p = self.prob
        G, cells = p.G, p.cells
        t = max(self.t - 1, 0)
        off = t * self.stride
        out = torch.empty(lc.N_GREY * cells, dtype=torch.float64, device="cuda")
        lc.lc_grey_closures(self.plan, self.E, self.F, self.f, self.kappa.view(-1)[off:off + G * cells],
                            self.planck.view(-1)[off:off + G * cells], out)
        return out.cpu().numpy().reshape(lc.N_GREY, cells)

    def state_canonical(self):
        out = torch.empty(self.plan.n_state, dtype=torch.float64, device="cuda")
        lc.lc_state_export(self.plan, self.state[self.cur], out)
        r = self.rays
        return out.cpu().numpy().reshape(r.n_segments, 2, r.n_pol, self.prob.G)

    def exits(self):
        r = self.rays
        return self.I_exit.cpu().numpy().reshape(r.n_rays, 2, r.n_pol, self.prob.G)

    def updates_per_step(self):
        """Segment updates of one sweep: stored segments x 2 traversals x
        polar angles x groups."""
        r = self.rays
        return r.n_segments * 2 * r.n_pol * self.prob.G


class GroupSplitSolver:
    """Group-dependent characteristic grids: the groups of one problem are
    split into ranges, each swept on a grid of characteristics with its own
    spacing (and, optionally, construction); the ranges advance together as
    one batch.  Moments and grey closures are those of the whole problem."""

    def __init__(self, prob, parts, prec=lc.LC_F64, static_material=False):
        """parts: list of (g0, g1, h_moc) covering the groups in order."""
        import workloads as W
        assert parts[0][0] == 0 and parts[-1][1] == prob.G
        assert all(a[1] == b[0] for a, b in zip(parts, parts[1:]))
        self.prob = prob
        self.parts = parts
        self.subs = [W.group_subset(prob, g0, g1, h) for g0, g1, h in parts]
        self.batch = BatchSolver(self.subs, prec=prec, static_material=static_material)
        self.kappa = _dev(np.stack(prob.kappa))          # [steps][G][cells], for the closures
        self.planck = _dev(np.stack(prob.planck))

    def reset(self):
        self.batch.reset()

    def step(self, n=1):
        self.batch.step(n)

    def moments(self):
        """E [G][cells], F [G][2][cells], f [G][4][cells], bnd [G][nb][8]."""
        ms = [s.moments() for s in self.batch.solvers]
        return {k: np.concatenate([m[k] for m in ms], axis=0) for k in ("E", "F", "f", "bnd")}

    def grey_closures(self, step):
        """Grey closures of the whole problem with the material data of
        `step` (lc_grey_closures_dims on the ranges' moments): [13][cells]."""
        p = self.prob
        cells, G = p.cells, p.G
        sv = self.batch.solvers
        E = torch.cat([s.E.view(cells, s.prob.G) for s in sv], dim=1).contiguous()
        F = torch.cat([s.F.view(cells, 2, s.prob.G) for s in sv], dim=2).contiguous()
        f = torch.cat([s.f.view(cells, 4, s.prob.G) for s in sv], dim=2).contiguous()
        out = torch.empty(lc.N_GREY * cells, dtype=torch.float64, device="cuda")
        lc.lc_grey_closures_dims(cells, G, E.view(-1), F.view(-1), f.view(-1), self.kappa[step].reshape(-1),
                                 self.planck[step].reshape(-1), out)
        return out.cpu().numpy().reshape(lc.N_GREY, cells)


class BatchSolver:
    """Many problems advanced together through the batched C entry points.
    Each member keeps its own Solver (buffers, rays, plan); the batch handle
    refers to their device buffers."""

    def __init__(self, probs, prec=lc.LC_F32, c=None, tuning=None, static_material=False):
        """static_material: every step uses the first step's material data
        (then any number of steps may be taken)."""
        self.solvers = [Solver(p, prec=prec, c=c) for p in probs]
        if tuning is not None:
            for s in self.solvers:
                lc.lc_plan_set_tuning(s.plan, *tuning)
        self.c = self.solvers[0].c
        self.static = static_material
        self.max_steps = None if static_material else min(s.prob.steps for s in self.solvers)
        self.batch = None
        self.rebuild()

    def polar_class(self, s):
        """Polar bound of a member: the power of two >= its polar count (the
        library launches each class separately)."""
        pm = 1
        while pm < s.prob.n_pol:
            pm *= 2
        return pm

    def classes(self):
        return sorted({self.polar_class(s) for s in self.solvers})

    def rebuild(self, tuning=None):
        """(Re)create the batch handle, optionally with a new launch tuning
        (sweep_unroll, moments_entries) set on every member's plan: one pair
        for all, or a dict {polar class: pair}."""
        if tuning is not None:
            for s in self.solvers:
                t = tuning[self.polar_class(s)] if isinstance(tuning, dict) else tuning
                lc.lc_plan_set_tuning(s.plan, *t)
        if self.batch is not None:
            self.batch.free()
        static_material = self.static
        self.batch = lc.lc_batch_create([dict(
            plan=s.plan, kappa=s.kappa, planck=s.planck, c_dt=s.prob.c_dt,
            material_stride=0 if static_material else s.stride,
            state_a=s.state[0], state_b=s.state[1], I_in=s.I_in, I_exit=s.I_exit, E=s.E, F=s.F,
            f=s.f, bnd=s.bnd, n_steps_max=s.prob.steps) for s in self.solvers])

    def reset(self):
        for s in self.solvers:
            s.reset()

    def step(self, n):
        """n steps from the states in state[0] (material steps 0 .. n-1)."""
        if self.max_steps is not None and n > self.max_steps:
            raise ValueError(f"only {self.max_steps} material steps are available")
        lc.lc_batch_step(self.batch, n, self.c)
        for s in self.solvers:
            s.cur = n % 2
            s.t = n

    def updates_per_step(self):
        return sum(s.updates_per_step() for s in self.solvers)



class MlqdSolver:
    """Time steps of the multilevel method (lc_mlqd_step) on a
    Fleck-Cummings problem (workloads.fc_mlqd): the transport state, the
    temperature and the multigroup low-order solution ping-pong between two
    buffers; history records (outer, inner, (dT, dE)) per step."""

    def __init__(self, prob, prec=lc.LC_F64, rays=None, eps=1e-12, max_outer=60, max_inner=1000, depth=3):
        from workloads import A_RAD, C_LIGHT
        self.prob = prob
        self.c = C_LIGHT
        self.eps, self.max_outer, self.max_inner = eps, max_outer, max_inner
        self.rays = rays if rays is not None else lc.lc_build_rays(
            prob.nx, prob.ny, prob.lx, prob.ly, prob.phi, prob.mu, prob.omega, prob.h_moc)
        self.plan = lc.Plan(self.rays, prob.G, prec)
        self.h = lc.Mlqd(self.plan, prob.nu, prob.edges, C_LIGHT, prob.c_v, A_RAD)
        lc.lc_mlqd_set_acceleration(self.h, depth)
        G, N, nf = prob.G, prob.cells, self.h.nf
        z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
        self.I_in = _dev(prob.I_in)
        self.state0 = _dev(prob.state0)
        self.state = [self.plan.new_state(), self.plan.new_state()]
        self.T = [z(N), z(N)]
        self.E = [z(G * N), z(G * N)]
        self.Ef = [z(G * nf), z(G * nf)]
        self.F = [z(G * nf), z(G * nf)]
        self.E_grey = z(N)
        self.cur = 0
        self.history = []

    def reset(self):
        p = self.prob
        lc.lc_state_fill(self.plan, self.state0, self.state[0])
        self.T[0].fill_(p.T0)
        self.E[0].copy_(4.0 * np.pi * self.state0.reshape(-1) / self.c)
        self.F[0].zero_()
        self.cur = 0
        self.history = []

    def step(self, n=1):
        p = self.prob
        for _ in range(n):
            a, b = self.cur, 1 - self.cur
            r = lc.lc_mlqd_step(self.h, p.c_dt, self.state[a], self.state[b], self.I_in, self.T[a], self.E[a],
                                self.F[a], self.T[b], self.E[b], self.Ef[b], self.F[b], self.E_grey, eps=self.eps,
                                max_outer=self.max_outer, max_inner=self.max_inner)
            self.history.append(r)
            self.cur = b

    def solution(self):
        G, N, nf = self.prob.G, self.prob.cells, self.h.nf
        k = self.cur
        return dict(T=self.T[k].cpu().numpy(), E_cell=self.E[k].cpu().numpy().reshape(G, N),
                    E_face=self.Ef[k].cpu().numpy().reshape(G, nf), F_face=self.F[k].cpu().numpy().reshape(G, nf),
                    E_grey=self.E_grey.cpu().numpy())

    def state_canonical(self):
        out = torch.empty(self.plan.n_state, dtype=torch.float64, device="cuda")
        lc.lc_state_export(self.plan, self.state[self.cur], out)
        r = self.rays
        return out.cpu().numpy().reshape(r.n_segments, 2, r.n_pol, self.prob.G)
