"""Shared test helpers: build a library context or an oracle problem from a
seeded scene with identical settings."""
import numpy as np


def make_ctx(sc, precision=0, barrier_full=False, alpha_component=False, iter_max=None, eps=None, term=None,
             rest_exclude=True, chunk=0, cell=None, beta="dk", split=False, model="nh", scatter=0,
             graphs=True):
    import paper_2405_08001_amd as P
    ctx = P.Context(0, precision, chunk=chunk, scatter=scatter, graphs=graphs)
    if model != "nh":
        ctx.pncg_set_model(model)
    ctx.pncg_set_mesh(sc.X, sc.tets, sc.tris, sc.edges, sc.object_id)
    ctx.pncg_set_material(sc.E, sc.nu, sc.rho)
    flags = (P.CONTACT_SELF if sc.self_contact else 0) | (P.CONTACT_REST_EXCLUDE if rest_exclude else 0)
    ctx.pncg_set_contact(sc.dhat, sc.kappa, sc.cell if cell is None else cell, sc.planes, flags)
    term = {"delta_e": P.TERM_DELTA_E, "grad_rel": P.TERM_GRAD_REL,
            "grad_abs": P.TERM_GRAD_ABS}[sc.term if term is None else term]
    sflags = (P.BARRIER_FULL if barrier_full else 0) | (P.ALPHA_INF_COMPONENT if alpha_component else 0) | \
        P.BETA_RULES[beta] | (P.SPLIT_OBJECTS if split else 0)
    ctx.pncg_set_solver(sc.iter_max if iter_max is None else iter_max, sc.eps if eps is None else eps, term,
                        sc.gravity, sflags)
    if len(sc.fixed):
        ctx.pncg_set_dirichlet(sc.fixed, sc.X[sc.fixed])
    return ctx


def make_problem(sc, barrier_full=False, rest_exclude=True, model="nh"):
    from oracle import problem
    return problem.Problem.from_scene(sc, barrier_mode="full" if barrier_full else "psd",
                                      rest_exclude=rest_exclude, model=model)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def elem(a, b):
    """Element-by-element deviation: max_i |a_i - b_i| / max_i |b_i|, so that
    every element satisfies |a_i - b_i| <= elem(a, b) * max|b|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


def check_solver_pairs(ctx, prob, x, r, rtol=1e-12):
    """The library's solver pair list at x against the oracle: the oracle's
    inflated-AABB candidates with inflation r, kept where the oracle's
    closest distance (Sec. 3.2) is below r.  Both sides decide d < r in
    float64 but by different closest-point formulas, so a pair whose
    distance lies within rtol * r of r may fall either way; every other pair
    must agree.  Returns (n_pt, n_ee) of the library's lists."""
    import paper_2405_08001_amd as L
    from oracle import candidates, distance
    x = np.asarray(x, dtype=np.float64)
    out = []
    for kind in (L.KIND_PT, L.KIND_EE):
        if kind == L.KIND_PT:
            cand = candidates.pt_candidates(x, prob.tris, prob.surf_verts, r, prob.excl_pt)
            cand = np.asarray(cand, np.int64).reshape(-1, 2)
            t = prob.tris[cand[:, 1]]
            d = distance.point_triangle(x[cand[:, 0]], x[t[:, 0]], x[t[:, 1]], x[t[:, 2]])[2] if len(cand) else \
                np.zeros(0)
        else:
            cand = candidates.ee_candidates(x, prob.edges, r, prob.excl_ee)
            cand = np.asarray(cand, np.int64).reshape(-1, 2)
            e1, e2 = prob.edges[cand[:, 0]], prob.edges[cand[:, 1]]
            d = distance.edge_edge(x[e1[:, 0]], x[e1[:, 1]], x[e2[:, 0]], x[e2[:, 1]])[2] if len(cand) else \
                np.zeros(0)
        g = np.asarray(ctx.pncg_solver_pairs(x, kind), np.int64).reshape(-1, 2)
        # sorted and free of repeats
        if len(g) > 1:
            key = g[:, 0] * (1 << 32) + g[:, 1]
            assert np.all(np.diff(key) > 0), "solver list not sorted or has repeats"
        sure = cand[d < r * (1 - rtol)]
        maybe = cand[np.abs(d - r) <= rtol * r]
        gs = {(int(a), int(b)) for a, b in g}
        ss = {(int(a), int(b)) for a, b in sure}
        ms = {(int(a), int(b)) for a, b in maybe}
        missing = ss - gs
        extra = gs - ss - ms
        assert not missing, (kind, len(missing), sorted(missing)[:5])
        assert not extra, (kind, len(extra), sorted(extra)[:5])
        out.append(len(g))
    return tuple(out)
