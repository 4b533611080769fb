"""Reference gradient of a trajectory loss with respect to per-tet Young's
moduli, by implicit differentiation of each time step (not in the paper;
the paper only notes that the IPC formulation is differentiable, Sec. 1).

Forward: each step's x^{t+1} is the minimiser of the incremental potential
(Sec. 3, equation E), so its plain definition is G(x^{t+1}) = 0 with
G = grad E on the free degrees of freedom.  The oracle reaches it with a
damped Newton iteration on the assembled exact Hessian (sparse direct
solves), which converges to rounding level; it is independent of the PNCG
iteration whose converged result it stands for.  Only planes are supported
as contact primitives here (a feasible Newton step then only needs the
per-vertex plane distances to stay positive).

Backward, for v^{t+1} = (x^{t+1} - x^t)/h and xt = x^t + h v^t + h^2 g:
    lambda   = H^{-1} (xbar_{t+1} + vbar_{t+1} / h)
    xbar_t   = M lambda - vbar_{t+1} / h
    vbar_t   = h M lambda
    Ebar_e  -= lambda^T dG/dE_e
with H the exact Hessian at x^{t+1} (barrier_mode "full"; exact for planes).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import elastic


def newton_solve(prob, x_t, v_t, h, tol=1e-10, max_iter=100):
    """argmin_x E(x) by Newton with backtracking; returns (x, iterations).
    Stops at ||g|| <= tol ||g_0|| or when ||g|| stops falling below
    1e-8 ||g_0|| (the rounding floor of the gradient)."""
    assert not prob.self_contact, "the Newton reference supports planes only"
    xt = prob.predictor(x_t, v_t, h)
    x = np.array(x_t, dtype=np.float64, copy=True)
    g0 = None
    g_last = np.inf
    for it in range(max_iter):
        aset = prob.active_set(x)
        g = prob.gradient(x, xt, h, aset)
        gn = np.linalg.norm(g)
        g0 = gn if g0 is None else g0
        if gn <= tol * max(g0, 1e-300) or (gn < 1e-8 * g0 and gn >= g_last):
            return x, it
        g_last = gn
        H = prob.hessian_matrix(x, h, aset, mode="full")
        dx = -spla.spsolve(H.tocsc(), g.ravel()).reshape(-1, 3)
        if np.sum(dx * g) >= 0:       # not a descent direction: use -g
            dx = -g / np.maximum(np.repeat(prob.mass[:, None], 3, 1), 1e-300)
        dx[~prob.free] = 0.0
        E0 = prob.energy(x, xt, h, aset)
        a = 1.0
        # keep every surface vertex strictly in front of every plane
        sv = prob.surf_verts
        for pl in prob.planes:
            n, o = pl[:3], pl[3]
            dist = x[sv] @ n - o
            rate = dx[sv] @ n
            neg = rate < 0
            if np.any(neg):
                a = min(a, 0.9 * float(np.min(-dist[neg] / rate[neg])))
        while True:
            xn = x + a * dx
            try:
                En = prob.energy(xn, xt, h)
            except (ValueError, FloatingPointError):
                En = np.inf
            if En <= E0 + 1e-4 * a * np.sum(g * dx) or a < 1e-12:
                break
            # near the minimiser the energy change drops below rounding;
            # then accept a step that reduces the gradient norm instead
            if np.isfinite(En) and abs(En - E0) <= 1e-13 * abs(E0) and \
                    np.linalg.norm(prob.gradient(xn, xt, h)) < gn:
                break
            a *= 0.5
        x = xn
    return x, max_iter


def param_gradient_matrix(prob, x, h):
    """dG/dE_e as a sparse (3V x T) matrix: the elastic gradient is
    h^2 sum_e V_e vec(dF/dx)^T vec(dPsi/dF) with mu = E mu', lam = E lam'."""
    F = elastic.deformation_gradient(x, prob.tets, prob.Bmat)
    dmu = 1.0 / (2.0 * (1.0 + prob.nu))
    dlam = prob.nu / ((1.0 + prob.nu) * (1.0 - 2.0 * prob.nu))
    ge = h * h * elastic.element_param_gradient(F, prob.b, prob.vol, dmu, dlam, prob.model)   # (T,4,3)
    T = prob.tets.shape[0]
    rows = (3 * prob.tets[:, :, None] + np.arange(3)[None, None, :]).ravel()
    cols = np.repeat(np.arange(T), 12)
    M = sp.coo_matrix((ge.ravel(), (rows, cols)), shape=(3 * prob.nV, T)).tocsr()
    if len(prob.fixed):
        M = sp.diags(np.repeat(prob.free, 3).astype(np.float64)) @ M
    return M


def trajectory(prob, x0, v0, h, steps, tol=1e-10):
    xs, vs = [np.asarray(x0, dtype=np.float64)], [np.asarray(v0, dtype=np.float64)]
    for _ in range(steps):
        x, _ = newton_solve(prob, xs[-1], vs[-1], h, tol=tol)
        vs.append((x - xs[-1]) / h)
        xs.append(x)
    return xs, vs


def step_adjoint(prob, x1, h, xbar, vbar, pair_hessian="full"):
    """One backward step at the converged x^{t+1} = x1, given the loss
    adjoints xbar = dL/dx^{t+1}, vbar = dL/dv^{t+1}: returns
    (dL/dx^t, dL/dv^t, this step's contribution to dL/dE, lambda).
    pair_hessian: the point-triangle / edge-edge barrier Hessian in H,
    "full" (equation eq9 with frozen closest-point coefficients) or "psd" (its
    projection, the solver's model); planes and elements are exact either
    way."""
    H = prob.hessian_matrix(x1, h, mode=pair_hessian)
    rhs = (np.asarray(xbar, dtype=np.float64) + np.asarray(vbar, dtype=np.float64) / h).copy()
    rhs[~prob.free] = 0.0
    lam = spla.spsolve(H.tocsc(), rhs.ravel()).reshape(-1, 3)
    lam[~prob.free] = 0.0
    dE = -(param_gradient_matrix(prob, x1, h).T @ lam.ravel())
    Ml = prob.mass[:, None] * lam
    # prescribed vertices of x^{t+1} do not depend on x^t, v^t
    return Ml - vbar / h, h * Ml, dE, lam


def loss_and_gradient(prob, x0, v0, h, steps, x_target, tol=1e-10):
    """L = ||x_T - x_target||^2 and dL/dE (T,) by the adjoint recursion."""
    xs, vs = trajectory(prob, x0, v0, h, steps, tol)
    L = float(np.sum((xs[-1] - x_target) ** 2))
    xbar = 2.0 * (xs[-1] - x_target)
    vbar = np.zeros_like(xbar)
    Ebar = np.zeros(prob.tets.shape[0])
    for t in range(steps, 0, -1):
        xbar, vbar, dE, _ = step_adjoint(prob, xs[t], h, xbar, vbar)
        Ebar += dE
    return L, Ebar, xs
