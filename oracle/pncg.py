"""Algorithm 1: one implicit-Euler time step by Jacobi-preconditioned Dai-Kou
nonlinear conjugate gradient (Sec. 4).

Per iteration k (Algorithm 1, Sec. 4.1-4.4):
  constraint set at x; gradient g_{k+1} and P_{k+1} = diag(H)^{-1};
  beta = 0 on the first iteration, else the preconditioned Dai-Kou formula
      beta = g^T P y / (y^T p) - (y^T P y / y^T p) (p^T g / y^T p),
      y = g_{k+1} - g_k, p = the previous direction;
  p_{k+1} = -P g_{k+1} + beta p_k;
  alpha = min(dhat / (2 ||p||), -g^T p / p^T H p)     (equations upper, alpha)
  x <- x + alpha p;  dE = -alpha g^T p - alpha^2/2 p^T H p;  dE_0 from the
  first iteration; stop when dE < eps dE_0.

Readings where the paper is silent or garbled:
  * x_0 = x^t (not xt); prescribed vertices are set to their targets first.
  * "If i = 0" in the listing means k = 0; beta uses only the previous
    direction p_k.
  * ||p|| in the step bound is the largest per-vertex Euclidean length
    max_v ||p_v||_2, which keeps every vertex's displacement below dhat/2 as
    the text requires ("component" reads it as the largest |p_i| instead).
    The bound is infinite when the scene has no collision primitives.
  * Guards: y^T p = 0 or a non-finite beta gives beta = 0; g^T p >= 0 restarts
    with p = -P g; p^T H p <= 0 gives an unbounded Newton step; a step that is
    still unbounded or not finite stops the iteration.
  * Termination "delta_e": the rule above.  "grad_rel": stop at the top of an
    iteration when ||g||_2 <= eps ||g_0||_2 (used for tight convergence);
    "grad_abs": the same test against eps itself (steps that start near
    equilibrium have ||g_0|| near the gradient's rounding floor).
  * v^{t+1} = (x^{t+1} - x^t) / h.

Other beta rules (the ablation of Sec. 7.1 names CD, HZ, FR and PRP beside
DK; their formulas are in the cited papers).  Each is preconditioned by
taking inner products that involve a gradient or y in the P metric of its
iteration, with d = p_k the previous direction and z = P g:
  fr   Fletcher-Reeves:   beta = g^T P g / (g_k^T P_k g_k)
  prp  Polak-Ribiere-Polyak: beta = g^T P y / (g_k^T P_k g_k)
  cd   Conjugate Descent: beta = -g^T P g / (d^T g_k)
  hz   Hager-Zhang:       beta = g^T P y / (y^T d) - 2 (y^T P y / y^T d) (d^T g / y^T d)
  dk   Dai-Kou (default): as above (the HZ form with factor 1)
The guards and the restart are the same for every rule.

Splitting computation (Sec. 5.2, split=True): every object (the vertices
sharing an object id) gets its own beta, search direction and step size.
Readings, since the details are in the missing supplemental:
  * beta_o by the chosen rule over the object's vertices; p_v = -P g_v +
    beta_o p_prev,v; the restart test g_o^T p_o >= 0 per object;
  * alpha_o = min(dhat / (2 max_{v in o} ||p_v||), -g_o^T p_o / p_o^T H p_o),
    where p_o is p on the object's vertices and zero elsewhere, so p_o^T H p_o
    is the object's diagonal block of H (a contact pair between two objects
    adds its term with the other object's p left out); every vertex still
    moves at most dhat / 2, which keeps the step penetration-free;
  * an object whose direction is zero does not move; the step stops as
    "unbounded" only if some moving object's alpha is not finite;
  * dE = sum_o (-alpha_o g_o^T p_o - alpha_o^2 / 2 p_o^T H p_o), with the same
    termination rules as the unsplit step.
With one object this is the unsplit step, operation for operation.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class StepStats:
    iters: int = 0
    reason: str = ""
    dE0: float = 0.0
    last_dE: float = 0.0
    g0: float = 0.0
    gk: float = 0.0
    alpha_upper_hits: int = 0
    n_active: int = 0
    n_plane: int = 0
    energy_increase: int = 0
    history: list = dataclasses.field(default_factory=list)


BETA_RULES = ("dk", "fr", "prp", "cd", "hz")


def beta_value(rule, g, P, g_prev, P_prev, p_prev):
    """beta of iteration k > 0 by the named rule (module docstring); 0 when
    a denominator is zero or the value is not finite."""
    y = g - g_prev
    if rule in ("fr", "prp"):
        den = float(np.sum(g_prev * P_prev * g_prev))
        num = float(np.sum(g * P * g)) if rule == "fr" else float(np.sum(g * P * y))
        b = num / den if den != 0.0 else 0.0
    elif rule == "cd":
        den = float(np.sum(p_prev * g_prev))
        b = -float(np.sum(g * P * g)) / den if den != 0.0 else 0.0
    elif rule in ("dk", "hz"):
        yp = float(np.sum(y * p_prev))
        if yp == 0.0:
            return 0.0
        gPy = float(np.sum(g * P * y))
        yPy = float(np.sum(y * P * y))
        pg = float(np.sum(p_prev * g))
        c = 1.0 if rule == "dk" else 2.0
        b = gPy / yp - c * (yPy / yp) * (pg / yp)
    else:
        raise ValueError(f"unknown beta rule {rule!r}")
    return b if np.isfinite(b) else 0.0


def step(prob, x_t, v_t, h, *, iter_max=100, eps=1e-3, term="delta_e",
         alpha_norm="vertex", fixed_targets=None, track_energy=False,
         record=False, beta_rule="dk", split=False):
    """Returns (x_new, v_new, stats)."""
    if split:
        return _step_split(prob, x_t, v_t, h, iter_max=iter_max, eps=eps, term=term, alpha_norm=alpha_norm,
                           fixed_targets=fixed_targets, beta_rule=beta_rule)
    x_t = np.asarray(x_t, dtype=np.float64)
    xt = prob.predictor(x_t, v_t, h)
    x = x_t.copy()
    if len(prob.fixed):
        x[prob.fixed] = x_t[prob.fixed] if fixed_targets is None else fixed_targets
    st = StepStats()
    g_prev = p_prev = P_prev = None
    dE0 = None
    g0n = None
    E_prev = prob.energy(x, xt, h) if track_energy else None
    k = 0
    while k < iter_max:
        aset = prob.active_set(x)
        g = prob.gradient(x, xt, h, aset)
        D = prob.diag(x, h, aset)
        gn = float(np.sqrt(np.sum(g * g)))
        if g0n is None:
            g0n = gn
            st.g0 = gn
        st.gk = gn
        if (term == "grad_rel" and gn <= eps * g0n) or (term == "grad_abs" and gn <= eps):
            st.reason = term
            break
        P = 1.0 / D
        beta = 0.0 if k == 0 else beta_value(beta_rule, g, P, g_prev, P_prev, p_prev)
        p = -P * g + (beta * p_prev if k > 0 else 0.0)
        gp = float(np.sum(g * p))
        if gp >= 0.0:
            p = -P * g
            gp = float(np.sum(g * p))
        p[~prob.free] = 0.0
        if gp == 0.0:
            st.reason = "zero_gradient"
            break
        pHp = prob.pHp(x, p, h, aset)
        a_bar = -gp / pHp if pHp > 0 else np.inf
        if prob.has_collision_primitives:
            pmax = float(np.max(np.linalg.norm(p, axis=1))) if alpha_norm == "vertex" \
                else float(np.max(np.abs(p)))
            a_up = prob.dhat / (2.0 * pmax) if pmax > 0 else np.inf
        else:
            a_up = np.inf
        alpha = min(a_up, a_bar)
        if not np.isfinite(alpha):
            st.reason = "unbounded"
            break
        if a_up < a_bar:
            st.alpha_upper_hits += 1
        x = x + alpha * p
        dE = -alpha * gp - 0.5 * alpha * alpha * pHp
        if record:
            st.history.append(dict(k=k, beta=beta, alpha=alpha, a_bar=a_bar, a_up=a_up,
                                   gp=gp, pHp=pHp, dE=dE, gn=gn,
                                   n_active=0 if aset is None else len(aset.d) + len(aset.pd)))
        if aset is not None:
            st.n_active = len(aset.d)
            st.n_plane = len(aset.pd)
        if track_energy:
            E_new = prob.energy(x, xt, h)
            if E_new > E_prev:
                st.energy_increase += 1
            E_prev = E_new
        k += 1
        if dE0 is None:
            dE0 = dE
            st.dE0 = dE
        st.last_dE = dE
        g_prev, p_prev, P_prev = g, p, P
        if term == "delta_e" and dE < eps * dE0:
            st.reason = "delta_e"
            break
    if not st.reason:
        st.reason = "iter_max"
    st.iters = k
    v = (x - x_t) / h
    return x, v, st


def _step_split(prob, x_t, v_t, h, *, iter_max, eps, term, alpha_norm, fixed_targets, beta_rule):
    """Algorithm 1 with a beta, direction and step size per object (module
    docstring, splitting computation)."""
    x_t = np.asarray(x_t, dtype=np.float64)
    xt = prob.predictor(x_t, v_t, h)
    x = x_t.copy()
    if len(prob.fixed):
        x[prob.fixed] = x_t[prob.fixed] if fixed_targets is None else fixed_targets
    objs = [prob.object_id == o for o in np.unique(prob.object_id)]
    st = StepStats()
    g_prev = p_prev = P_prev = None
    dE0 = g0n = None
    k = 0
    while k < iter_max:
        aset = prob.active_set(x)
        g = prob.gradient(x, xt, h, aset)
        D = prob.diag(x, h, aset)
        gn = float(np.sqrt(np.sum(g * g)))
        if g0n is None:
            g0n = gn
            st.g0 = gn
        st.gk = gn
        if (term == "grad_rel" and gn <= eps * g0n) or (term == "grad_abs" and gn <= eps):
            st.reason = term
            break
        P = 1.0 / D
        p = np.zeros_like(g)
        gps = []
        for m in objs:
            beta = 0.0 if k == 0 else beta_value(beta_rule, g[m], P[m], g_prev[m], P_prev[m], p_prev[m])
            pm = -P[m] * g[m] + (beta * p_prev[m] if k > 0 else 0.0)
            gp = float(np.sum(g[m] * pm))
            if gp >= 0.0:
                pm = -P[m] * g[m]
                gp = float(np.sum(g[m] * pm))
            p[m] = pm
            gps.append(gp)
        p[~prob.free] = 0.0
        if all(gp == 0.0 for gp in gps):
            st.reason = "zero_gradient"
            break
        alphas, dE, unbounded, hits = [], 0.0, False, 0
        for m, gp in zip(objs, gps):
            po = np.where(m[:, None], p, 0.0)
            if not np.any(po):
                alphas.append(0.0)
                continue
            pHp = prob.pHp(x, po, h, aset)
            a_bar = -gp / pHp if pHp > 0 else np.inf
            if prob.has_collision_primitives:
                pmax = float(np.max(np.linalg.norm(p[m], axis=1))) if alpha_norm == "vertex" \
                    else float(np.max(np.abs(p[m])))
                a_up = prob.dhat / (2.0 * pmax) if pmax > 0 else np.inf
            else:
                a_up = np.inf
            alpha = min(a_up, a_bar)
            if not np.isfinite(alpha):
                unbounded = True
            hits += a_up < a_bar
            alphas.append(alpha)
            dE += -alpha * gp - 0.5 * alpha * alpha * pHp
        if unbounded:
            st.reason = "unbounded"
            break
        st.alpha_upper_hits += hits
        for m, alpha in zip(objs, alphas):
            x[m] = x[m] + alpha * p[m]
        if aset is not None:
            st.n_active = len(aset.d)
            st.n_plane = len(aset.pd)
        k += 1
        if dE0 is None:
            dE0 = dE
            st.dE0 = dE
        st.last_dE = dE
        g_prev, p_prev, P_prev = g, p, P
        if term == "delta_e" and dE < eps * dE0:
            st.reason = "delta_e"
            break
    else:
        st.reason = "iter_max"
    st.iters = k
    v = (x - x_t) / h
    return x, v, st
