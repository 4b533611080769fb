"""Differentiable time stepping: a torch.autograd.Function over T steps of
the library's solver whose backward pass runs the library's adjoint step
(implicit differentiation of each converged step, pncg_adjoint_step_dev),
recomputing the states between checkpoints taken every k steps: k - 1
steps per segment, since a segment's last state is the next checkpoint,
and none for the last segment, whose states the forward pass keeps (the
backward pass needs them first).

Only marshalling and control flow live here; every step, Hessian-vector
product, CG iteration and parameter gradient runs in the HIP library.

    sim = Simulation(ctx, nu, rho, h, steps, checkpoint=5)
    xT, vT = simulate(E, x0, v0, sim)        # E: (nT,) float64, x0/v0: (nV, 3) CUDA float64
    loss = ((xT - x_target) ** 2).sum()
    loss.backward()                           # E.grad, x0.grad, v0.grad

The context must be float64 (``FP64``) and its solver set to a tight
gradient tolerance (e.g. ``TERM_GRAD_REL`` with eps 1e-10): the adjoint
assumes each step's result is a minimiser of the incremental potential.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


class Simulation:
    """A prepared float64 context plus the rollout settings.

    ctx         an ``_lib.Context`` with mesh, contact and solver set (its
                material is replaced by E on every forward and backward)
    nu, rho     per-tet Poisson ratio and density (arrays or scalars)
    h, steps    step size and number of steps
    checkpoint  keep the state every ``checkpoint`` steps; the backward pass
                recomputes the steps in between
    cg_tol, cg_max   adjoint CG stopping rule (relative residual, cap)
    warm_start  start each step's adjoint CG from the previous step's lambda
    """

    def __init__(self, ctx, nu, rho, h, steps, checkpoint=5, cg_tol=1e-10, cg_max=20000, warm_start=True):
        if ctx.precision != _lib.FP64:
            raise ValueError("differentiation needs a float64 context")
        if steps < 1 or checkpoint < 1:
            raise ValueError("steps and checkpoint must be >= 1")
        self.ctx = ctx
        self.nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (ctx.nT,)).copy()
        self.rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (ctx.nT,)).copy()
        self.h = float(h)
        self.steps = int(steps)
        self.checkpoint = int(checkpoint)
        self.cg_tol = float(cg_tol)
        self.cg_max = int(cg_max)
        self.warm_start = bool(warm_start)
        self.forward_stats = []
        self.adjoint_stats = []
        self.recomputed_steps = 0

    def _set_E(self, E):
        self.ctx.pncg_set_material(np.ascontiguousarray(E, dtype=np.float64), self.nu, self.rho)

    def _step(self, x, v, xo, vo):
        return self.ctx.pncg_step_dev(x, v, self.h, xo, vo)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, E, x0, v0, sim):
        E_np = E.detach().to("cpu", torch.float64).numpy().copy()
        sim._set_E(E_np)
        x = x0.detach().to(torch.float64).contiguous().clone()
        v = v0.detach().to(torch.float64).contiguous().clone()
        xn, vn = torch.empty_like(x), torch.empty_like(v)
        ck = [(x.clone(), v.clone())]
        tail = []          # states of the last segment, which the backward pass needs first
        sim.forward_stats = []
        for t in range(sim.steps):
            sim.forward_stats.append(sim._step(x, v, xn, vn))
            x, xn, v, vn = xn, x, vn, v
            if (t + 1) % sim.checkpoint == 0 and t + 1 < sim.steps:
                ck.append((x.clone(), v.clone()))
                tail = []
            else:
                tail.append(x.clone())
        fctx.sim = sim
        fctx.E_np = E_np
        fctx.ck = ck
        fctx.tail = tail
        fctx.E_meta = (E.dtype, E.device)
        return x.clone(), v.clone()

    @staticmethod
    def backward(fctx, gx, gv):
        sim, ck = fctx.sim, fctx.ck
        ctx = sim.ctx
        sim._set_E(fctx.E_np)
        ctx.pncg_set_adjoint_warm_start(sim.warm_start)
        x_ref = ck[0][0]
        xbar = torch.zeros_like(x_ref) if gx is None else gx.detach().to(torch.float64).contiguous().clone()
        vbar = torch.zeros_like(x_ref) if gv is None else gv.detach().to(torch.float64).contiguous().clone()
        xb2, vb2 = torch.empty_like(xbar), torch.empty_like(vbar)
        Ebar = torch.zeros(ctx.nT, dtype=torch.float64, device=x_ref.device)
        sim.adjoint_stats = []
        k = sim.checkpoint
        for s in reversed(range(len(ck))):
            t0 = s * k
            t1 = min(t0 + k, sim.steps)
            if s == len(ck) - 1:
                states = fctx.tail         # kept by the forward pass
            else:
                # recompute x_{t0+1} .. x_{t1-1} from the checkpoint; x_{t1}
                # is the next checkpoint
                x, v = ck[s][0].clone(), ck[s][1].clone()
                states = []
                xn, vn = torch.empty_like(x), torch.empty_like(v)
                for _ in range(t0, t1 - 1):
                    sim._step(x, v, xn, vn)
                    sim.recomputed_steps += 1
                    x, xn, v, vn = xn, x, vn, v
                    states.append(x.clone())
                states.append(ck[s + 1][0])
            for t in range(t1, t0, -1):
                st = ctx.pncg_adjoint_step_dev(states[t - t0 - 1], sim.h, xbar, vbar, xb2, vb2, Ebar,
                                               cg_tol=sim.cg_tol, cg_max=sim.cg_max)
                sim.adjoint_stats.append(st)
                xbar, xb2, vbar, vb2 = xb2, xbar, vb2, vbar
        dtype, device = fctx.E_meta
        return Ebar.to(device=device, dtype=dtype), xbar, vbar, None


def simulate(E, x0, v0, sim):
    """(x_T, v_T) after sim.steps steps from (x0, v0) with per-tet moduli E;
    differentiable with respect to E, x0 and v0."""
    return _Rollout.apply(E, x0, v0, sim)
