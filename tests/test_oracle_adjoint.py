"""Pins for the oracle's implicit-differentiation gradient: central finite
differences of the trajectory loss in random directions of log E."""
import numpy as np

import scenes
from oracle import adjoint, problem


def _setup():
    sc = scenes.diff_bar_scene(seed=4, nx=4, ny=2, nz=2, dx=0.01, lift=0.0012)
    P = problem.Problem.from_scene(sc)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    steps = 4
    rng = np.random.default_rng(5)
    E_tgt = 1e5 * np.exp(0.5 * rng.standard_normal(sc.nT))
    P2 = problem.Problem.from_scene(sc)
    P2.set_material(E_tgt, sc.nu)
    xs, _ = adjoint.trajectory(P2, sc.X, v0, sc.h, steps)
    return sc, P, v0, steps, xs[-1]


def test_newton_reference_converges():
    sc, P, v0, steps, _ = _setup()
    x, it = adjoint.newton_solve(P, sc.X, v0, sc.h)
    xt = P.predictor(sc.X, v0, sc.h)
    g = P.gradient(x, xt, sc.h)
    assert np.linalg.norm(g) < 1e-11 * np.linalg.norm(P.gradient(sc.X, xt, sc.h))
    a = P.active_set(x)
    assert len(a.pd) > 0          # the floor barrier is active


def test_adjoint_matches_finite_differences():
    sc, P, v0, steps, x_tgt = _setup()
    L, Ebar, _ = adjoint.loss_and_gradient(P, sc.X, v0, sc.h, steps, x_tgt)
    assert L > 0
    rng = np.random.default_rng(6)
    E0 = P.E.copy()
    for _ in range(4):
        u = rng.standard_normal(sc.nT)
        e = 1e-5
        vals = []
        for s in (+1, -1):
            P.set_material(E0 * np.exp(s * e * u), sc.nu)
            xs, _ = adjoint.trajectory(P, sc.X, v0, sc.h, steps)
            vals.append(np.sum((xs[-1] - x_tgt) ** 2))
        P.set_material(E0, sc.nu)
        fd = (vals[0] - vals[1]) / (2 * e)
        an = np.sum(Ebar * E0 * u)          # chain rule through E = E0 exp(e u)
        assert np.isclose(an, fd, rtol=2e-5), (an, fd)
