"""Shared test helpers: build a library context or an oracle problem from a
seeded scene with identical settings."""
import numpy as np


def make_ctx(sc, precision=0, barrier_full=False, alpha_component=False, iter_max=None, eps=None, term=None,
             rest_exclude=True, chunk=0, cell=None, beta="dk", split=False, model="nh", scatter=0):
    import paper_2405_08001_amd as P
    ctx = P.Context(0, precision, chunk=chunk, scatter=scatter)
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
