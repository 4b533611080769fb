"""Adjoint form on the GPU: one adjoint step against the oracle's (sparse
direct solve) on the same converged state, whole-trajectory gradients
against the oracle's adjoint recursion, against central finite differences
of the GPU forward in 16 random directions, and checkpointing against full
storage."""
import sys

import numpy as np
import pytest

import scenes
from helpers import elem, make_ctx, make_problem, rel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bar(nx, ny, nz, lift=0.0012):
    return scenes.diff_bar_scene(seed=4, nx=nx, ny=ny, nz=nz, dx=0.01, lift=lift)


def _sim(sc, steps, checkpoint=5, cg_tol=1e-12):
    import paper_2405_08001_amd as P
    ctx = make_ctx(sc, 0)                   # converged steps: absolute gradient rule of the scene
    return P.Simulation(ctx, sc.nu, sc.rho, sc.h, steps, checkpoint=checkpoint, cg_tol=cg_tol, cg_max=20000)


def _rollout_grad(sim, E, x0, v0, x_tgt):
    import torch
    import paper_2405_08001_amd as P
    dev = torch.device("cuda:0")
    Et = torch.tensor(E, dtype=torch.float64, requires_grad=True)
    x0t = torch.tensor(x0, dtype=torch.float64, device=dev, requires_grad=True)
    v0t = torch.tensor(v0, dtype=torch.float64, device=dev, requires_grad=True)
    xT, _ = P.simulate(Et, x0t, v0t, sim)
    loss = ((xT - torch.tensor(x_tgt, device=dev)) ** 2).sum()
    loss.backward()
    return float(loss.detach()), Et.grad.numpy().copy(), x0t.grad.cpu().numpy(), v0t.grad.cpu().numpy()


def _forward_loss(sim, E, x0, v0, x_tgt):
    import torch
    import paper_2405_08001_amd as P
    dev = torch.device("cuda:0")
    with torch.no_grad():
        xT, _ = P.simulate(torch.tensor(E), torch.tensor(x0, device=dev), torch.tensor(v0, device=dev), sim)
    return float(((xT.cpu().numpy() - x_tgt) ** 2).sum())


def test_adjoint_step_matches_oracle():
    """Same converged x^{t+1} (the oracle's Newton result), same seeded
    adjoints: lambda by device CG versus a sparse direct solve."""
    from oracle import adjoint
    sc = _bar(8, 3, 3)
    P = make_problem(sc)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    x1, _ = adjoint.newton_solve(P, sc.X, v0, sc.h, tol=1e-12)
    assert len(P.active_set(x1).pd) > 0          # the floor barrier is active
    rng = np.random.default_rng(8)
    xbar = rng.standard_normal(x1.shape)
    vbar = rng.standard_normal(x1.shape)
    xo, vo, Eo, _ = adjoint.step_adjoint(P, x1, sc.h, xbar, vbar)
    ctx = make_ctx(sc, 0)
    xg, vg, Eg, st = ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, cg_tol=1e-13, cg_max=20000)
    _say(f"adjoint step: cg {st['cg_iters']} res {st['rel_residual']:.1e} "
         f"rel xbar {rel(xg, xo):.2e} vbar {rel(vg, vo):.2e} Ebar {rel(Eg, Eo):.2e}")
    assert st["reason"] == 0
    assert rel(xg, xo) <= 1e-9 and rel(vg, vo) <= 1e-9 and rel(Eg, Eo) <= 1e-9
    # Ebar accumulates
    _, _, Eg2, _ = ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, Ebar=Eg, cg_tol=1e-13)
    assert rel(Eg2, 2 * Eo) <= 1e-9


def test_adjoint_warm_start_same_solution_fewer_iterations():
    """Starting the CG from the previous call's lambda (a nearby right-hand
    side, as consecutive steps of a backward pass give): the same solution
    as the oracle's direct solve, in fewer CG iterations than from zero."""
    from oracle import adjoint
    sc = _bar(8, 3, 3)
    P = make_problem(sc)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    x1, _ = adjoint.newton_solve(P, sc.X, v0, sc.h, tol=1e-12)
    rng = np.random.default_rng(9)
    xbar = rng.standard_normal(x1.shape)
    vbar = rng.standard_normal(x1.shape)
    xbar2 = xbar + 0.01 * rng.standard_normal(x1.shape)
    xo, vo, Eo, _ = adjoint.step_adjoint(P, x1, sc.h, xbar2, vbar)
    ctx = make_ctx(sc, 0)
    ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, cg_tol=1e-13, cg_max=20000)
    _, _, _, cold = ctx.pncg_adjoint_step(x1, sc.h, xbar2, vbar, cg_tol=1e-13, cg_max=20000)
    ctx.pncg_set_adjoint_warm_start(1)
    ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, cg_tol=1e-13, cg_max=20000)
    xg, vg, Eg, warm = ctx.pncg_adjoint_step(x1, sc.h, xbar2, vbar, cg_tol=1e-13, cg_max=20000)
    _say(f"warm start: cg {warm['cg_iters']} (cold {cold['cg_iters']}) res {warm['rel_residual']:.1e} "
         f"rel xbar {rel(xg, xo):.2e} Ebar {rel(Eg, Eo):.2e}")
    assert warm["reason"] == 0
    assert warm["cg_iters"] < cold["cg_iters"]
    assert rel(xg, xo) <= 1e-9 and rel(vg, vo) <= 1e-9 and rel(Eg, Eo) <= 1e-9


def test_trajectory_gradient_matches_oracle():
    """4 steps of the small bar falling onto the floor: dL/dE through the GPU
    forward (PNCG, absolute gradient rule) and adjoint versus the oracle's Newton
    trajectory and direct-solve adjoint recursion."""
    from oracle import adjoint, problem
    sc = _bar(4, 2, 2)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    steps = 4
    rng = np.random.default_rng(5)
    E_tgt = 1e5 * np.exp(0.5 * rng.standard_normal(sc.nT))
    P2 = problem.Problem.from_scene(sc)
    P2.set_material(E_tgt, sc.nu)
    x_tgt = adjoint.trajectory(P2, sc.X, v0, sc.h, steps)[0][-1]
    P = make_problem(sc)
    Lo, Eo, _ = adjoint.loss_and_gradient(P, sc.X, v0, sc.h, steps, x_tgt)
    sim = _sim(sc, steps, checkpoint=2)
    Lg, Eg, _, _ = _rollout_grad(sim, sc.E, sc.X, v0, x_tgt)
    _say(f"trajectory: L {Lg:.6e}/{Lo:.6e} rel dL/dE {rel(Eg, Eo):.2e} "
         f"cg {[s['cg_iters'] for s in sim.adjoint_stats]}")
    assert abs(Lg - Lo) <= 1e-8 * Lo
    assert rel(Eg, Eo) <= 1e-5


def test_checkpointing_equals_full_storage():
    import torch
    sc = _bar(10, 3, 3)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    x_tgt = sc.X + 0.001
    s5, s1 = _sim(sc, 7, checkpoint=5), _sim(sc, 7, checkpoint=1)
    g5 = _rollout_grad(s5, sc.E, sc.X, v0, x_tgt)
    g1 = _rollout_grad(s1, sc.E, sc.X, v0, x_tgt)
    _say(f"checkpoint 5 vs 1: dE {rel(g5[1], g1[1]):.2e} dx0 {rel(g5[2], g1[2]):.2e} dv0 {rel(g5[3], g1[3]):.2e}; "
         f"recomputed {s5.recomputed_steps} / {s1.recomputed_steps}")
    # segments [0, 5) and [5, 7): x_1..x_4 recomputed, x_5 is a checkpoint,
    # the last segment's states are kept by the forward pass
    assert s5.recomputed_steps == 4 and s1.recomputed_steps == 0
    assert g5[0] == g1[0]
    for a, b in zip(g5[1:], g1[1:]):
        assert rel(a, b) <= 1e-12


def test_gradient_matches_central_differences_16_directions():
    """A 1,920-tet bar, 10 steps with the floor engaged, checkpoints every 5:
    the adjoint directional derivative of L in log E along 16 seeded random
    directions against central differences of the GPU forward (1e-4)."""
    import time
    t_start = time.perf_counter()
    sc = _bar(20, 4, 4)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.05
    steps = 10
    rng = np.random.default_rng(6)
    E_tgt = 1e5 * np.exp(0.5 * rng.standard_normal(sc.nT))
    sim = _sim(sc, steps)
    x_tgt_sim = _sim(sc, steps)
    import torch
    import paper_2405_08001_amd as P
    with torch.no_grad():
        xT, _ = P.simulate(torch.tensor(E_tgt), torch.tensor(sc.X, device="cuda:0"),
                           torch.tensor(v0, device="cuda:0"), x_tgt_sim)
    x_tgt = xT.cpu().numpy()
    L, Eg, _, _ = _rollout_grad(sim, sc.E, sc.X, v0, x_tgt)
    _say(f"fd: L={L:.6e}, recomputed steps {sim.recomputed_steps}, "
         f"max cg {max(s['cg_iters'] for s in sim.adjoint_stats)}")
    assert L > 0
    eps = 1e-4
    worst = 0.0
    for i in range(16):
        u = rng.standard_normal(sc.nT)
        Lp = _forward_loss(sim, sc.E * np.exp(eps * u), sc.X, v0, x_tgt)
        Lm = _forward_loss(sim, sc.E * np.exp(-eps * u), sc.X, v0, x_tgt)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(Eg * sc.E * u))
        err = abs(an - fd) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        _say(f"  direction {i}: adjoint {an:.8e} fd {fd:.8e} rel {err:.1e}")
        assert err <= 1e-4
    _say(f"  worst {worst:.1e}; {time.perf_counter() - t_start:.1f} s, "
         f"forward iterations per step {np.mean([s['iters'] for s in sim.forward_stats]):.0f}")


def test_full_size_gradient_matches_central_differences_16_directions():
    """The differentiation configuration itself: the 30,000-tet bar (50 x 10
    x 10 cells) falling onto the floor, 30 steps, checkpoints every 5, loss
    ||x_30 - x_target||^2 with the target the forward result under a second
    seeded modulus field, CG tolerance 1e-10.  The adjoint directional
    derivative in log E along 16 seeded random directions against central
    differences of the GPU forward, 1e-4 relative.  (The oracle's own
    trajectory gradient is compared at the 1,920-tet size: its sparse direct
    solves at 30,000 tets over 30 steps take too long for a test.)"""
    import time
    import torch
    import paper_2405_08001_amd as P
    t_start = time.perf_counter()
    sc = scenes.diff_bar_scene(seed=4)
    tgt = scenes.diff_bar_scene(seed=5)
    steps = 30
    sim = _sim(sc, steps, checkpoint=5, cg_tol=1e-10)
    dev = torch.device("cuda:0")
    with torch.no_grad():
        xT, _ = P.simulate(torch.tensor(tgt.E), torch.tensor(sc.x0, device=dev), torch.tensor(sc.v0, device=dev),
                           sim)
    x_tgt = xT.cpu().numpy()
    L, Eg, _, _ = _rollout_grad(sim, sc.E, sc.x0, sc.v0, x_tgt)
    _say(f"full-size fd ({sc.nT} tets, {steps} steps): L={L:.6e}, recomputed steps {sim.recomputed_steps}, "
         f"mean cg {np.mean([s['cg_iters'] for s in sim.adjoint_stats]):.0f}, "
         f"mean forward iterations {np.mean([s['iters'] for s in sim.forward_stats]):.0f}")
    assert L > 0 and sim.recomputed_steps == 20
    rng = np.random.default_rng(6)
    eps = 1e-4
    worst = 0.0
    for i in range(16):
        u = rng.standard_normal(sc.nT)
        Lp = _forward_loss(sim, sc.E * np.exp(eps * u), sc.x0, sc.v0, x_tgt)
        Lm = _forward_loss(sim, sc.E * np.exp(-eps * u), sc.x0, sc.v0, x_tgt)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(Eg * sc.E * u))
        err = abs(an - fd) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        _say(f"  direction {i}: adjoint {an:.8e} fd {fd:.8e} rel {err:.1e}")
        assert err <= 1e-4
    _say(f"  worst {worst:.1e}; {time.perf_counter() - t_start:.1f} s")


@pytest.mark.parametrize("scatter", [2, 1])
def test_adjoint_step_with_self_contact_matches_oracle(scatter):
    """Point-triangle, edge-edge and plane barriers active (the pressed cube
    stack): the adjoint's linear solve H lambda = xbar + vbar / h on the
    device (CG with the pair H p of the segmented or the atomic scatter)
    against the oracle's sparse direct solve with the same pair Hessian model
    (the solver's PSD projection, reading S7), element by element."""
    from oracle import adjoint
    sc = scenes.small_contact_scene()
    x1 = sc.X.copy()
    top = sc.object_id == 1
    x1[top, 2] -= 5.5e-4
    x1[~top, 2] -= 3e-4
    # a deformed state (at the rest shape dG/dE vanishes and Ebar is only rounding)
    x1 += np.random.default_rng(10).uniform(-3e-5, 3e-5, x1.shape)
    P = make_problem(sc)
    a = P.active_set(x1)
    assert np.sum(a.kind == 0) > 0 and np.sum(a.kind == 1) > 0 and len(a.pd) > 0
    rng = np.random.default_rng(9)
    xbar = rng.standard_normal(x1.shape)
    vbar = rng.standard_normal(x1.shape)
    xo, vo, Eo, lo = adjoint.step_adjoint(P, x1, sc.h, xbar, vbar, pair_hessian="psd")
    ctx = make_ctx(sc, 0, scatter=scatter)
    xg, vg, Eg, st = ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, cg_tol=1e-13, cg_max=20000)
    _say(f"self-contact adjoint scatter={scatter}: cg {st['cg_iters']} res {st['rel_residual']:.1e} "
         f"xbar {elem(xg, xo):.2e} vbar {elem(vg, vo):.2e} Ebar {elem(Eg, Eo):.2e}")
    assert st["reason"] == 0
    # the stiff barriers make H ill-conditioned (thousands of CG iterations):
    # a 1e-13 residual leaves lambda accurate to about 1e-9
    assert elem(xg, xo) <= 1e-8 and elem(vg, vo) <= 1e-8 and elem(Eg, Eo) <= 1e-8
    # and the pair Hessian matters: the full (unprojected) model gives another lambda
    xf, _, _, _ = adjoint.step_adjoint(P, x1, sc.h, xbar, vbar, pair_hessian="full")
    assert elem(xf, xo) > 1e-6
