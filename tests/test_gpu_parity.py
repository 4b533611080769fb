"""GPU parity against the oracle: per-phase queries on identical inputs,
bit-exact candidate lists, and whole steps."""
import sys

import numpy as np
import pytest

import scenes
from helpers import check_solver_pairs, make_ctx, make_problem, rel

pytestmark = pytest.mark.gpu

TOL = {0: dict(e=1e-11, g=1e-10, d=1e-10, php=1e-10, hp=1e-10),
       1: dict(e=1e-6, g=1e-5, d=1e-5, php=1e-5, hp=1e-5)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cube_state():
    sc = scenes.cube_scene()
    rng = np.random.default_rng(21)
    x = sc.X.copy()
    x[:, 2] -= 0.05 - 4e-4                       # bottom within dhat of the floor
    x += rng.uniform(-2e-4, 2e-4, x.shape)
    xt = x + rng.uniform(-1e-3, 1e-3, x.shape)
    return sc, x, xt


def _stack_state():
    sc = scenes.small_contact_scene()
    x = sc.X.copy()
    top = sc.object_id == 1
    x[top, 2] -= 5.5e-4
    x[~top, 2] -= 3e-4
    rng = np.random.default_rng(3)
    xt = x + rng.uniform(-1e-4, 1e-4, x.shape)
    return sc, x, xt


STATES = {"cube": _cube_state, "stack": _stack_state}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["cube", "stack"])
@pytest.mark.parametrize("full", [False, True])
def test_queries_match_oracle(which, precision, full):
    _say(f"queries {which} precision={precision} full={full}")
    sc, x, xt = STATES[which]()
    P = make_problem(sc, barrier_full=full)
    ctx = make_ctx(sc, precision, barrier_full=full)
    t = TOL[precision]
    h = sc.h
    a = P.active_set(x)
    assert len(a.pd) > 0
    if which == "stack":
        assert np.sum(a.kind == 0) > 0 and np.sum(a.kind == 1) > 0
    E = ctx.pncg_energy(x, xt, h)
    assert abs(E - P.energy(x, xt, h, a)) <= t["e"] * abs(P.energy(x, xt, h, a))
    g, d = ctx.pncg_gradient(x, xt, h)
    assert rel(g, P.gradient(x, xt, h, a)) <= t["g"]
    assert rel(d, P.diag(x, h, a)) <= t["d"]
    p = np.random.default_rng(5).standard_normal(x.shape) * 1e-3
    hp, php = ctx.pncg_hvp(x, p, h)
    ref_hp = P.hvp(x, p, h, a)
    assert rel(hp, ref_hp) <= t["hp"]
    assert abs(php - P.pHp(x, p, h, a)) <= t["php"] * abs(P.pHp(x, p, h, a))


@pytest.mark.parametrize("which", ["cube", "stack", "bar"])
def test_candidates_bit_exact(which):
    _say(f"candidates {which}")
    if which == "bar":
        sc = scenes.twisted_bar_scene()
        x = sc.X.copy()
        # fold the bar over itself so that many surface primitives come close
        L = sc.meta["length"]
        sel = x[:, 0] > L / 2
        x[sel, 0] = L - x[sel, 0]
        x[sel, 2] += 0.08 + 6e-4
        x += np.random.default_rng(9).uniform(-2e-4, 2e-4, x.shape)
    else:
        sc, x, _ = STATES[which]()
    P = make_problem(sc)
    ctx = make_ctx(sc, 0)
    pt, ee, pg = P.candidate_lists(x)
    import paper_2405_08001_amd as L
    g_pt = ctx.pncg_candidates(x, L.KIND_PT)
    g_ee = ctx.pncg_candidates(x, L.KIND_EE)
    g_pg = ctx.pncg_candidates(x, L.KIND_PG)
    assert np.array_equal(g_pt, pt), (len(g_pt), len(pt))
    assert np.array_equal(g_ee, ee), (len(g_ee), len(ee))
    assert np.array_equal(g_pg, pg), (len(g_pg), len(pg))
    if which != "cube":
        assert len(pt) > 0 and len(ee) > 0
    # the solver's own list (distance-filtered, built by the step's kernels)
    ctx.pncg_set_tuning(skin=2.0 * sc.dhat)
    n_pt, n_ee = check_solver_pairs(ctx, P, x, 3.0 * sc.dhat)
    if which == "bar":
        assert n_pt > 0 and n_ee > 0


def _cube_drop():
    sc = scenes.cube_scene()
    x0 = sc.X.copy()
    x0[:, 2] -= 0.05 - 1.2e-3                    # just above the floor, moving down
    v0 = np.zeros_like(x0)
    v0[:, 2] = -0.1
    return sc, x0, v0


def _stack_drop():
    sc = scenes.small_contact_scene()
    v0 = np.zeros_like(sc.X)
    v0[sc.object_id == 1, 2] = -0.05
    return sc, sc.X.copy(), v0


DROPS = {"cube": _cube_drop, "stack": _stack_drop}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("K", [1, 2, 12])
@pytest.mark.parametrize("which", ["cube", "stack"])
def test_fixed_iterations_match_oracle(which, K, precision):
    """K iterations of Algorithm 1 from the same state (no early stop): every
    step of the iteration (beta, direction, alpha, update) is pinned."""
    _say(f"fixed-iteration step {which} K={K} precision={precision}")
    from oracle import pncg
    sc, x0, v0 = DROPS[which]()
    P = make_problem(sc)
    ctx = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e")
    xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=K, eps=0.0, term="delta_e")
    xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} rel_x={rx:.3e} rel_dx={rdx:.3e} hits={sg['alpha_upper_hits']}")
    assert sg["iters"] == st.iters == K
    assert sg["alpha_upper_hits"] == st.alpha_upper_hits
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= (1e-9 if precision == 0 else 1e-3)
    assert rel(vg, vo) <= (1e-9 if precision == 0 else 1e-3)


def _two_apart():
    Xa, Ta = scenes.hex_grid(3, 3, 3, 0.01, origin=(0.0, 0.0, 5e-4))
    Xb, Tb = scenes.hex_grid(3, 3, 3, 0.01, origin=(0.2, 0.0, 0.02))
    X, tets, oid = scenes.merge_meshes([(Xa, Ta), (Xb, Tb)])
    X = X + np.random.default_rng(12).uniform(-2e-4, 2e-4, X.shape)
    E = np.where(np.arange(len(tets)) < len(Ta), 1e5, 1e6)
    sc = scenes.configs._scene(X, tets, E=E, nu=0.4, rho=1000.0, planes=[[0.0, 0.0, 1.0, 0.0]], dhat=1e-3,
                               kappa=1e4, h=1.0 / 60.0, object_id=oid, self_contact=True, cell=4e-3)
    v0 = np.zeros_like(X)
    v0[oid == 0, 2] = -0.1
    return sc, sc.X.copy(), v0


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["stack", "apart", "cube"])
def test_split_step_matches_oracle(which, precision):
    """Splitting computation (Sec. 5.2): a beta, direction and step size per
    object.  10 fixed iterations against the oracle's split step: the stacked
    cubes (pairs between the two objects), two cubes apart (independent
    objects) and one cube (one object: the unsplit step)."""
    from oracle import pncg
    _say(f"split step {which} precision={precision}")
    sc, x0, v0 = {"stack": _stack_drop, "apart": _two_apart, "cube": _cube_drop}[which]()
    K = 10
    prob = make_problem(sc)
    xo, _, st = pncg.step(prob, x0, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", split=True)
    ctx = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e", split=True)
    xg, _, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    bx, bdx = (1e-12, 1e-9) if precision == 0 else (1e-6, 1e-3)
    if precision == 1:
        xq = x0 * (1.0 + 2.0 ** -24)
        xp, _, _ = pncg.step(prob, xq, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", split=True)
        bx = max(bx, 4.0 * rel(xp, xo))
        bdx = max(bdx, 4.0 * rel(xp - xq, xo - x0))
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} hits {st.alpha_upper_hits}/{sg['alpha_upper_hits']} "
         f"rel_x={rx:.3e} (bar {bx:.1e}) rel_dx={rdx:.3e} (bar {bdx:.1e})")
    assert sg["iters"] == st.iters == K
    assert sg["alpha_upper_hits"] == st.alpha_upper_hits
    assert rx <= bx and rdx <= bdx
    if which == "cube":        # one object: the unsplit step to rounding
        xu, _, _ = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e").pncg_step(x0, v0, sc.h)
        assert rel(xg - x0, xu - x0) <= (1e-9 if precision == 0 else 1e-4)


def test_split_needs_contiguous_objects():
    import paper_2405_08001_amd as P
    sc, _, _ = _stack_drop()
    ctx = P.Context(0, 0)
    oid = sc.object_id[::-1].copy()           # decreasing ids: not contiguous ranges in order
    ctx.pncg_set_mesh(sc.X, sc.tets, sc.tris, sc.edges, oid)
    ctx.pncg_set_material(sc.E, sc.nu, sc.rho)
    with pytest.raises(P.PncgError):
        ctx.pncg_set_solver(10, 0.0, P.TERM_DELTA_E, sc.gravity, P.SPLIT_OBJECTS)
    ctx.pncg_set_solver(10, 0.0, P.TERM_DELTA_E, sc.gravity, 0)


def test_mean_boundary_edge_matches_numpy():
    """The larger-dhat strategy's reference length (Sec. 5.1): the mean rest
    length of the surface edges."""
    import paper_2405_08001_amd as P
    sc = scenes.small_contact_scene()
    ctx = P.Context(0, 0)
    with pytest.raises(P.PncgError):
        ctx.pncg_mean_boundary_edge()            # before set_mesh
    ctx.pncg_set_mesh(sc.X, sc.tets, sc.tris, sc.edges, sc.object_id)
    want = float(np.mean(np.linalg.norm(sc.X[sc.edges[:, 0]] - sc.X[sc.edges[:, 1]], axis=1)))
    got = ctx.pncg_mean_boundary_edge()
    _say(f"mean boundary edge {got:.6e} (numpy {want:.6e})")
    assert got == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("precision", [0, 1])
def test_larger_dhat_with_rest_exclusion(precision):
    """Sec. 5.1's larger-dhat strategy on the stacked cubes: dhat = 0.5 x the
    mean boundary edge (about 5 mm against a 0.4 mm gap).  Within each cube,
    pairs closer than 1.5 dhat in the rest shape are excluded, a non-empty
    set at this dhat; the exact candidate lists at rest (where the exclusion
    removes every same-cube neighbour) and at a squeezed state equal the
    oracle's bit for bit, and two fixed iterations of the step from rest
    match the oracle."""
    import paper_2405_08001_amd as L
    from oracle import pncg
    base = scenes.small_contact_scene()
    lbar = float(np.mean(np.linalg.norm(base.X[base.edges[:, 0]] - base.X[base.edges[:, 1]], axis=1)))
    dhat = 0.5 * lbar
    sc = scenes.small_contact_scene(dhat=dhat)
    P = make_problem(sc)
    _say(f"larger dhat {dhat:.3e} (mean boundary edge {lbar:.3e}) precision={precision}: "
         f"excluded PT {len(P.excl_pt)} EE {len(P.excl_ee)}")
    assert len(P.excl_pt) > 100 and len(P.excl_ee) > 100
    ctx = make_ctx(sc, precision, iter_max=2, eps=0.0, term="delta_e", cell=2.0 * dhat)
    squeezed = sc.X.copy()
    squeezed[:, 2] *= 0.97
    for x in (sc.X, squeezed):
        pt, ee, pg = P.candidate_lists(x)
        g_pt = ctx.pncg_candidates(x, L.KIND_PT)
        g_ee = ctx.pncg_candidates(x, L.KIND_EE)
        g_pg = ctx.pncg_candidates(x, L.KIND_PG)
        _say(f"  candidates PT {len(g_pt)}/{len(pt)} EE {len(g_ee)}/{len(ee)} PG {len(g_pg)}/{len(pg)}")
        assert len(pt) > 0 and len(ee) > 0
        assert np.array_equal(g_pt, pt) and np.array_equal(g_ee, ee) and np.array_equal(g_pg, pg)
    v0 = np.zeros_like(sc.X)
    xo, vo, st = pncg.step(P, sc.X, v0, sc.h, iter_max=2, eps=0.0, term="delta_e")
    xg, vg, sg = ctx.pncg_step(sc.X, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - sc.X, xo - sc.X)
    _say(f"  step: iters {sg['iters']}/{st.iters} active {sg['n_active']} rel_x={rx:.3e} rel_dx={rdx:.3e}")
    assert sg["iters"] == st.iters == 2
    assert sg["n_active"] > 0
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= (1e-9 if precision == 0 else 1e-3)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("rule", ["fr", "prp", "cd", "hz"])
@pytest.mark.parametrize("which", ["cube", "stack"])
def test_beta_rules_match_oracle(which, rule, precision):
    """The other beta rules of the ablation (Sec. 7.1): 12 fixed iterations
    against the oracle with the same rule, and a rule outside the set is
    refused."""
    _say(f"beta rule {rule} {which} precision={precision}")
    import paper_2405_08001_amd as P
    from oracle import pncg
    sc, x0, v0 = DROPS[which]()
    K = 12
    ctx = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e", beta=rule)
    prob = make_problem(sc)
    xo, vo, st = pncg.step(prob, x0, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", beta_rule=rule)
    xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    bx, bdx = (1e-12, 1e-9) if precision == 0 else (1e-6, 1e-3)
    if precision == 1:
        # rules without the DK correction term (CD, FR) amplify the float32
        # rounding of the element arithmetic more: the bar follows the
        # oracle's own spread under a 2^-24 relative perturbation of x0
        xq = x0 * (1.0 + 2.0 ** -24)
        xp, _, _ = pncg.step(prob, xq, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", beta_rule=rule)
        bx = max(bx, 4.0 * rel(xp, xo))
        bdx = max(bdx, 4.0 * rel(xp - xq, xo - x0))
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} rel_x={rx:.3e} (bar {bx:.1e}) rel_dx={rdx:.3e} (bar {bdx:.1e})")
    assert sg["iters"] == st.iters == K
    assert rx <= bx
    assert rdx <= bdx
    with pytest.raises(P.PncgError):
        ctx.pncg_set_solver(K, 0.0, P.TERM_DELTA_E, sc.gravity, 5 << 4)


@pytest.mark.parametrize("precision", [0, 1])
def test_cube_converged_step_matches_oracle(precision):
    """Tightly converged step: both sides reach the same minimiser, so the
    positions agree far below the 1e-5 bar regardless of the path."""
    _say(f"converged cube step precision={precision}")
    from oracle import pncg
    sc, x0, v0 = _cube_drop()
    P = make_problem(sc)
    # the float32 gradient has a rounding floor near 1e-6 ||g_0||, so the mixed
    # form is run to its cap and judged on positions only
    eps = 1e-9 if precision == 0 else 1e-7
    ctx = make_ctx(sc, precision, iter_max=4000 if precision == 0 else 1500, eps=eps, term="grad_rel")
    xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=4000, eps=1e-9, term="grad_rel")
    xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} reason={sg['reason']} rel_x={rx:.3e} rel_dx={rdx:.3e}")
    if precision == 0:
        assert sg["reason"] == 1
    assert rx <= (1e-10 if precision == 0 else 1e-5)
    assert rdx <= (1e-7 if precision == 0 else 1e-2)
    dmin, jmin = ctx.pncg_min_distance(xg)
    assert dmin > 0 and jmin > 0


def test_cube_configured_step_within_rounding_envelope():
    """The cube as configured (100 iterations, gradient tolerance 1e-6) stops
    before convergence; after 100 nonlinear CG iterations the iterate is
    sensitive to rounding.  The GPU result must lie within a small multiple
    of the oracle's own spread under a 1e-15 relative input perturbation."""
    _say("configured cube step vs rounding envelope")
    from oracle import pncg
    sc, x0, v0 = _cube_drop()
    P = make_problem(sc)
    ctx = make_ctx(sc, 0)
    xo, _, st = pncg.step(P, x0, v0, sc.h, iter_max=sc.iter_max, eps=sc.eps, term=sc.term)
    xp, _, _ = pncg.step(P, x0 * (1 + 1e-15), v0, sc.h, iter_max=sc.iter_max, eps=sc.eps, term=sc.term)
    env = rel(xp, xo)
    xg, _, sg = ctx.pncg_step(x0, v0, sc.h)
    _say(f"  envelope={env:.3e} gpu rel_x={rel(xg, xo):.3e} iters={sg['iters']}/{st.iters}")
    assert sg["iters"] == st.iters
    assert rel(xg, xo) <= max(20 * env, 1e-9)


def test_grad_abs_rule_matches_scaled_grad_rel():
    """The absolute gradient rule with eps * ||g_0|| stops at the same
    iteration, with the same result, as the relative rule with eps."""
    _say("grad_abs vs grad_rel")
    sc, x0, v0 = _cube_drop()
    cr = make_ctx(sc, 0, iter_max=4000, eps=1e-8, term="grad_rel")
    xr, _, sr = cr.pncg_step(x0, v0, sc.h)
    ca = make_ctx(sc, 0, iter_max=4000, eps=1e-8 * sr["g0_norm"], term="grad_abs")
    xa, _, sa = ca.pncg_step(x0, v0, sc.h)
    _say(f"  iters {sr['iters']}/{sa['iters']} reasons {sr['reason']}/{sa['reason']}")
    assert sr["reason"] == sa["reason"] == 1
    assert sa["iters"] == sr["iters"]
    assert np.array_equal(xa, xr)


@pytest.mark.parametrize("K", [1, 12])
def test_in_place_step_after_capacity_rerun(K):
    """Outputs may alias the inputs.  On the stacked cubes (4 mm cells) a
    fresh context's first solver-list build needs more spatial-grid entries
    than the initial 8 (nF + nE) + nSV + 4096, so the step is run again from
    its inputs with a larger grid; the in-place step, the out-of-place step
    and the host-pointer step agree."""
    import torch
    _say(f"in-place step with a capacity rerun K={K}")
    sc, x0, v0 = _stack_drop()
    dev = torch.device("cuda:0")
    outs = []
    for how in ("apart", "in_place", "host"):
        ctx = make_ctx(sc, 0, iter_max=K, eps=0.0, term="delta_e")
        if how == "host":
            xh, vh, st = ctx.pncg_step(x0, v0, sc.h)
            outs.append((xh, vh, st))
            continue
        x = torch.tensor(x0, device=dev)
        v = torch.tensor(v0, device=dev)
        if how == "apart":
            xo, vo = torch.empty_like(x), torch.empty_like(v)
        else:
            xo, vo = x, v
        st = ctx.pncg_step_dev(x, v, sc.h, xo, vo)
        outs.append((xo.cpu().numpy(), vo.cpu().numpy(), st))
    (xa, va, sa), (xi, vi, si), (xh, vh, sh) = outs
    _say(f"  rebuilds {sa['rebuilds']}/{si['rebuilds']}/{sh['rebuilds']} "
         f"rel dx in place {rel(xi - x0, xa - x0):.2e} host {rel(xh - x0, xa - x0):.2e}")
    assert sa["iters"] == si["iters"] == sh["iters"] == K
    # the segmented pair scatter is deterministic: equal bits
    for xb, vb in ((xi, vi), (xh, vh)):
        assert np.array_equal(xb, xa) and np.array_equal(vb, va)


def test_failed_in_place_step_leaves_the_state():
    """A step whose start state has vertices below the floor plane fails
    with E_PENETRATION; the in-place state (outputs aliasing the inputs, as
    pncg_run_dev uses) is left as it was."""
    import torch
    import paper_2405_08001_amd as P
    sc, x0, v0 = _stack_drop()
    x = x0.copy()
    x[:, 2] -= x[:, 2].min() + 1e-3          # the lowest vertices 1 mm below the floor
    dev = torch.device("cuda:0")
    xt, vt = torch.tensor(x, device=dev), torch.tensor(v0, device=dev)
    ctx = make_ctx(sc, 0, iter_max=12, eps=0.0, term="delta_e")
    with pytest.raises(P.PncgError) as e:
        ctx.pncg_run_dev(xt, vt, sc.h, 2)
    _say(f"start below the floor: {e.value}")
    assert e.value.code == P.E_PENETRATION
    assert np.array_equal(xt.cpu().numpy(), x) and np.array_equal(vt.cpu().numpy(), v0)


def _run_pair(sc, x0, v0, precision, n, **kw):
    """(state, stats) after n steps by pncg_run_dev (in place) and by n
    separate pncg_step_dev calls, each on a fresh context."""
    import torch
    dev = torch.device("cuda:0")
    ca = make_ctx(sc, precision, **kw)
    x, v = torch.tensor(x0, device=dev), torch.tensor(v0, device=dev)
    sts, rc = ca.pncg_run_dev(x, v, sc.h, n)
    cb = make_ctx(sc, precision, **kw)
    xb, vb = torch.tensor(x0, device=dev), torch.tensor(v0, device=dev)
    ref = []
    for _ in range(n):
        xo, vo = torch.empty_like(xb), torch.empty_like(vb)
        ref.append(cb.pncg_step_dev(xb, vb, sc.h, xo, vo))
        xb, vb = xo, vo
    return (x.cpu().numpy(), v.cpu().numpy(), sts, rc), (xb.cpu().numpy(), vb.cpu().numpy(), ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_run_dev_equals_repeated_steps(precision):
    """pncg_run_dev: n steps in place with no return in between give the
    states and per-step statistics of n separate steps, bit for bit: the cube
    on its floor, and the stacked cubes (self contact, list rebuilds, 12 fixed
    iterations per step) under the default segmented pair scatter."""
    _say(f"run_dev vs repeated steps precision={precision}")
    sc, x0, v0 = _cube_drop()
    (xa, va, sts, rc), (xr, vr, ref) = _run_pair(sc, x0, v0, precision, 4)
    _say(f"  cube iters {[s['iters'] for s in sts]} / {[s['iters'] for s in ref]}")
    assert rc == max(s["status"] for s in ref)
    assert np.array_equal(xa, xr) and np.array_equal(va, vr)
    for s, r in zip(sts, ref):
        assert s["iters"] == r["iters"] and s["reason"] == r["reason"] and s["g_norm"] == r["g_norm"]
    sc, x0, v0 = _stack_drop()
    (xa, va, sts, rc), (xr, vr, ref) = _run_pair(sc, x0, v0, precision, 5, iter_max=12, eps=0.0, term="delta_e")
    _say(f"  stack iters {[s['iters'] for s in sts]} rebuilds {[s['rebuilds'] for s in sts]} "
         f"rel dx {rel(xa - x0, xr - x0):.2e}")
    assert [s["iters"] for s in sts] == [r["iters"] for r in ref] == [12] * 5
    assert np.array_equal(xa, xr) and np.array_equal(va, vr)
    for s, r in zip(sts, ref):
        assert s["iters"] == r["iters"] and s["n_active"] == r["n_active"] and s["g_norm"] == r["g_norm"]


def test_step_dev_reads_inputs_torch_has_just_written():
    """Device-pointer steps read their inputs on the library's stream: the
    binding first finishes torch's queued work, so a state that torch is
    still writing (a copy queued behind a long matrix product) is read only
    once written.  Same bits as the host-pointer step."""
    import torch
    _say("step_dev after pending torch work")
    sc, x0, v0 = _cube_drop()
    ctx = make_ctx(sc, 0)
    xh, vh, _ = ctx.pncg_step(x0, v0, sc.h)
    dev = torch.device("cuda:0")
    src_x = torch.tensor(x0, device=dev)
    src_v = torch.tensor(v0, device=dev)
    a = torch.randn(4096, 4096, device=dev)
    torch.cuda.synchronize()
    for rep in range(3):
        x = torch.zeros_like(src_x)
        v = torch.zeros_like(src_v)
        torch.cuda.synchronize()
        for _ in range(4):
            a = a @ a
            a = a / a.abs().max()
        x.copy_(src_x)
        v.copy_(src_v)
        xo, vo = torch.empty_like(x), torch.empty_like(v)
        ctx.pncg_step_dev(x, v, sc.h, xo, vo)
        same = bool(np.array_equal(xo.cpu().numpy(), xh) and np.array_equal(vo.cpu().numpy(), vh))
        _say(f"  rep {rep}: identical to the host step: {same}")
        assert same


@pytest.mark.parametrize("precision", [0, 1])
def test_twisted_bar_first_step_matches_oracle(precision):
    """The 15,360-tet bar, first twist step (end faces prescribed, rotated by
    3 degrees each way), 12 fixed iterations against the oracle."""
    from oracle import pncg
    _say(f"twisted bar step precision={precision}")
    sc = scenes.twisted_bar_scene()
    tgt = scenes.twist_targets(sc, 1)
    P = make_problem(sc)
    v0 = np.zeros_like(sc.X)
    xo, vo, st = pncg.step(P, sc.X, v0, sc.h, iter_max=12, eps=0.0, term="delta_e", fixed_targets=tgt)
    ctx = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e")
    ctx.pncg_set_dirichlet(sc.fixed, tgt)
    xg, vg, sg = ctx.pncg_step(sc.X, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - sc.X, xo - sc.X)
    _say(f"  iters {sg['iters']}/{st.iters} rel_x={rx:.3e} rel_dx={rdx:.3e}")
    assert sg["iters"] == st.iters == 12
    assert np.array_equal(xg[sc.fixed], tgt)
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= (1e-9 if precision == 0 else 1e-3)


def _stacked():
    sc = scenes.stacked_bars_scene()
    x0 = sc.X.copy()
    v0 = np.zeros_like(x0)
    v0[sc.object_id == 1, 2] = -0.02
    return sc, x0, v0


@pytest.mark.parametrize("precision", [0, 1])
def test_stacked_bars_self_contact_step_matches_oracle(precision):
    """Two twisted-bar meshes (30,720 tets) stacked with a 0.6 mm gap, the
    upper one moving down: point-triangle and edge-edge barriers active over
    the whole overlap (about 5,400 pairs), 2 fixed iterations."""
    from oracle import pncg
    _say(f"stacked bars step precision={precision}")
    sc, x0, v0 = _stacked()
    P = make_problem(sc)
    xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=2, eps=0.0, term="delta_e", fixed_targets=x0[sc.fixed])
    ctx = make_ctx(sc, precision, iter_max=2, eps=0.0, term="delta_e")
    xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    bdx = 1e-9
    if precision == 1:
        xq = x0 * (1.0 + 2.0 ** -24)
        xp, _, _ = pncg.step(P, xq, v0, sc.h, iter_max=2, eps=0.0, term="delta_e", fixed_targets=xq[sc.fixed])
        bdx = max(1e-3, 4.0 * rel(xp - xq, xo - x0))
    _say(f"  iters {sg['iters']}/{st.iters} active {sg['n_active']} cand {sg['n_candidates']} "
         f"rel_x={rx:.3e} rel_dx={rdx:.3e} (bar {bdx:.1e}) hits {sg['alpha_upper_hits']}/{st.alpha_upper_hits}")
    assert sg["iters"] == st.iters == 2
    assert sg["n_active"] > 1000
    assert sg["alpha_upper_hits"] == st.alpha_upper_hits
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= bdx
    dmin, jmin = ctx.pncg_min_distance(xg)
    assert dmin > 0 and jmin > 0


def test_stacked_bars_four_iterations_within_rounding_envelope():
    """With ~5,500 stiff barriers active, each further iteration amplifies
    rounding differences several hundred times (the oracle's own result
    after 4 iterations moves by ~1e-4 in the step displacement under a
    1e-15 relative perturbation of the start state).  The float64 GPU result
    after 4 iterations must lie within 20x that envelope."""
    from oracle import pncg
    _say("stacked bars, 4 iterations vs rounding envelope")
    sc, x0, v0 = _stacked()
    P = make_problem(sc)
    xo, _, st = pncg.step(P, x0, v0, sc.h, iter_max=4, eps=0.0, term="delta_e", fixed_targets=x0[sc.fixed])
    xq = x0 * (1.0 + 1e-15)
    xp, _, _ = pncg.step(P, xq, v0, sc.h, iter_max=4, eps=0.0, term="delta_e", fixed_targets=xq[sc.fixed])
    env = rel(xp - xq, xo - x0)
    ctx = make_ctx(sc, 0, iter_max=4, eps=0.0, term="delta_e")
    xg, _, sg = ctx.pncg_step(x0, v0, sc.h)
    rdx = rel(xg - x0, xo - x0)
    _say(f"  envelope rel_dx={env:.3e} gpu rel_dx={rdx:.3e}")
    assert sg["iters"] == 4
    assert rdx <= max(20.0 * env, 1e-9)
    dmin, jmin = ctx.pncg_min_distance(xg)
    assert dmin > 0 and jmin > 0


_PILE = {}


def _pile():
    """The pile scene and its oracle problem (built once: the rest-pose
    exclusion over 110k tets takes the oracle about 20 s)."""
    if not _PILE:
        sc = scenes.pile_scene()
        _PILE["sc"] = sc
        _PILE["P"] = make_problem(sc)
    return _PILE["sc"], _PILE["P"]


def test_pile_candidates_bit_exact_full_size():
    """The 110k-tet pile squashed to 40% of its height about the floor (the
    24 shapes' boxes overlap in many places; the state need not be
    feasible for the AABB test): the sorted point-triangle, edge-edge and
    vertex-plane lists equal the oracle's bit for bit."""
    _say("pile candidates (squashed)")
    sc, P = _pile()
    x = sc.x0.copy()
    x[:, 2] *= 0.4
    pt, ee, pg = P.candidate_lists(x)
    ctx = make_ctx(sc, 1)
    import paper_2405_08001_amd as L
    g_pt = ctx.pncg_candidates(x, L.KIND_PT)
    g_ee = ctx.pncg_candidates(x, L.KIND_EE)
    g_pg = ctx.pncg_candidates(x, L.KIND_PG)
    _say(f"  pt {len(g_pt)}/{len(pt)} ee {len(g_ee)}/{len(ee)} pg {len(g_pg)}/{len(pg)}")
    assert len(pt) > 1000 and len(ee) > 1000
    assert np.array_equal(g_pt, pt)
    assert np.array_equal(g_ee, ee)
    assert np.array_equal(g_pg, pg)


def test_pile_solver_list_matches_oracle_full_size():
    """The solver's own pair list (built by the step's kernels: candidates
    within dhat + skin kept by their closest distance) on the squashed
    110k-tet pile equals the oracle's at full size.  With a skin of 9 dhat
    the list holds about 73k point-triangle and 209k edge-edge pairs, many
    between neighbouring primitives of one surface, so the cell buckets are
    long."""
    _say("pile solver list (squashed)")
    sc, P = _pile()
    x = sc.x0.copy()
    x[:, 2] *= 0.4
    ctx = make_ctx(sc, 1)
    skin = 9.0 * sc.dhat
    ctx.pncg_set_tuning(skin=skin)
    n_pt, n_ee = check_solver_pairs(ctx, P, x, sc.dhat + skin)
    _say(f"  pt {n_pt} ee {n_ee}")
    assert n_pt > 10000 and n_ee > 10000


@pytest.mark.parametrize("precision", [1, 0])
def test_pile_two_iterations_match_oracle(precision):
    """The 110k-tet pile at its start state moving down at 0.1 m/s (the
    bottom shapes reach the floor barrier), 2 fixed iterations in the
    bench's configuration against the oracle."""
    from oracle import pncg
    _say(f"pile 2 iterations precision={precision}")
    sc, P = _pile()
    v0 = np.zeros_like(sc.x0)
    v0[:, 2] = -0.1
    if "step" not in _PILE:
        _PILE["step"] = pncg.step(P, sc.x0, v0, sc.h, iter_max=2, eps=0.0, term="delta_e")
    xo, vo, st = _PILE["step"]
    ctx = make_ctx(sc, precision, iter_max=2, eps=0.0, term="delta_e")
    xg, vg, sg = ctx.pncg_step(sc.x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - sc.x0, xo - sc.x0)
    _say(f"  iters {sg['iters']}/{st.iters} active {sg['n_active']} rel_x={rx:.3e} rel_dx={rdx:.3e} "
         f"hits {sg['alpha_upper_hits']}/{st.alpha_upper_hits}")
    assert sg["iters"] == st.iters == 2
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= (1e-9 if precision == 0 else 1e-3)
