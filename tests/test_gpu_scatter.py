"""Scatter of the contact-pair terms into their vertices (Sec. 3.2, equations
eq8-eq11; Sec. 4.2) and the explicit candidate list (Algorithm 1,
ComputeConstraintSet), on the GPU.

The segmented scatter writes one slot per (pair, corner) and sums each
vertex's slots in a fixed order, so whole steps with active pairs and list
rebuilds are bit-reproducible; the atomic scatter adds the same terms with
float64 atomics and agrees to the order of those additions.  Both are held
to the oracle."""
import sys

import numpy as np
import pytest

import scenes
from helpers import elem, make_ctx, make_problem, rel

pytestmark = pytest.mark.gpu

SEG, ATOM = 2, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _stack_drop():
    sc = scenes.small_contact_scene()
    v0 = np.zeros_like(sc.X)
    v0[sc.object_id == 1, 2] = -0.05
    return sc, sc.X.copy(), v0


def _stack_state():
    sc = scenes.small_contact_scene()
    x = sc.X.copy()
    top = sc.object_id == 1
    x[top, 2] -= 5.5e-4
    x[~top, 2] -= 3e-4
    rng = np.random.default_rng(3)
    xt = x + rng.uniform(-1e-4, 1e-4, x.shape)
    return sc, x, xt


def _steps(ctx, sc, x, v, n):
    out = []
    for _ in range(n):
        x, v, st = ctx.pncg_step(x, v, sc.h)
        out.append(st)
    return x, v, out


@pytest.mark.parametrize("precision", [0, 1])
def test_segmented_steps_are_bit_reproducible(precision):
    """Four steps of 12 fixed iterations from the falling stack (point-triangle,
    edge-edge and plane pairs active, candidate lists rebuilt within steps),
    on two fresh contexts and again on the first: identical bits."""
    _say(f"segmented reproducibility precision={precision}")
    sc, x0, v0 = _stack_drop()
    runs = []
    ca = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG)
    cb = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG)
    for ctx in (ca, cb, ca):
        runs.append(_steps(ctx, sc, x0, v0, 4))
    xa, va, sa = runs[0]
    _say(f"  active {[s['n_active'] for s in sa]} rebuilds {[s['rebuilds'] for s in sa]}")
    assert sum(s["rebuilds"] for s in sa) > 4 and min(s["n_active"] for s in sa) > 0
    for xb, vb, sb in runs[1:]:
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
        for s, t in zip(sa, sb):
            assert s == t


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_rebuilds_equal_eager_rebuilds(precision):
    """The candidate-list rebuild replayed from a captured HIP graph against
    the same kernels launched one by one: the falling stack for four steps
    of 12 iterations (several rebuilds per step, from both position
    buffers, with the step's own eager launches, host status reads and
    synchronisations between the replays), then four more steps through
    pncg_run_dev on the same contexts: identical bits and statistics after
    every step."""
    _say(f"graph vs eager rebuilds precision={precision}")
    import torch
    sc, x0, v0 = _stack_drop()
    cg = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG, graphs=True)
    ce = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG, graphs=False)
    xg, vg, xe, ve = x0, v0, x0, v0
    for i in range(4):
        xg, vg, sg = cg.pncg_step(xg, vg, sc.h)
        xe, ve, se = ce.pncg_step(xe, ve, sc.h)
        _say(f"  step {i}: rebuilds {sg['rebuilds']} active {sg['n_active']}")
        assert np.array_equal(xg, xe) and np.array_equal(vg, ve) and sg == se
    dev = torch.device("cuda:0")
    tg = [torch.tensor(a, device=dev) for a in (xg, vg)]
    te = [torch.tensor(a, device=dev) for a in (xe, ve)]
    sg, _ = cg.pncg_run_dev(tg[0], tg[1], sc.h, 4)
    se, _ = ce.pncg_run_dev(te[0], te[1], sc.h, 4)
    assert sum(s["rebuilds"] for s in sg) >= 4
    assert sg == se
    assert torch.equal(tg[0], te[0]) and torch.equal(tg[1], te[1])


@pytest.mark.parametrize("precision", [0, 1])
def test_carried_list_is_checked_at_the_step_start(precision):
    """A step may start on the previous step's candidate list.  (a) After
    steps from the falling stack, a step on the same context from a state
    far from the list's build positions (the stack back at its start) must
    pause at iteration 0, rebuild, and give the bits of a fresh context.
    (b) A one-iteration step that continues from where the context stopped
    keeps the list (no rebuild, where a fresh context builds one) and
    matches the fresh context's step to the rounding of the pair sums'
    grouping."""
    _say(f"carried list precision={precision}")
    sc, x0, v0 = _stack_drop()
    ctx = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG)
    x, v = x0, v0
    for _ in range(3):
        x, v, _ = ctx.pncg_step(x, v, sc.h)
    # (a) back to the start state: the carried list no longer covers x_0
    xa, va, sa = ctx.pncg_step(x0, v0, sc.h)
    fresh = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=SEG)
    xf, vf, sf = fresh.pncg_step(x0, v0, sc.h)
    _say(f"  restart from x0: rebuilds {sa['rebuilds']}/{sf['rebuilds']}")
    assert np.array_equal(xa, xf) and np.array_equal(va, vf) and sa == sf
    # (b) one-iteration steps of the resting stack move every vertex by at
    # most dhat / 2, under a quarter of the skin: the next step keeps the list
    rest = make_ctx(sc, precision, iter_max=1, eps=0.0, term="delta_e", scatter=SEG)
    xr, vr = sc.X.copy(), np.zeros_like(sc.X)
    xr, vr, s1 = rest.pncg_step(xr, vr, sc.h)
    x2, v2, s2 = rest.pncg_step(xr, vr, sc.h)
    fresh2 = make_ctx(sc, precision, iter_max=1, eps=0.0, term="delta_e", scatter=SEG)
    x3, v3, s3 = fresh2.pncg_step(xr, vr, sc.h)
    _say(f"  resting stack: rebuilds carried {s2['rebuilds']} fresh {s3['rebuilds']}, "
         f"rel_x {rel(x2, x3):.2e} rel_dx {rel(x2 - xr, x3 - xr):.2e}")
    assert s2["rebuilds"] < s3["rebuilds"]
    assert s2["iters"] == s3["iters"] and s2["n_active"] == s3["n_active"] > 0
    assert rel(x2, x3) <= (1e-12 if precision == 0 else 1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_atomic_and_segmented_scatter_agree(precision):
    """Queries at a pressed stack and 12 fixed iterations of a step: both
    scatter modes against the oracle at the parity bars, and against each
    other element by element."""
    _say(f"atomic vs segmented precision={precision}")
    from oracle import pncg
    sc, x, xt = _stack_state()
    P = make_problem(sc)
    h = sc.h
    a = P.active_set(x)
    assert np.sum(a.kind == 0) > 0 and np.sum(a.kind == 1) > 0
    g_o = P.gradient(x, xt, h, a)
    d_o = P.diag(x, h, a)
    p = np.random.default_rng(5).standard_normal(x.shape) * 1e-3
    Hp_o = P.hvp(x, p, h, a) if hasattr(P, "hvp") else None
    res = {}
    for mode in (ATOM, SEG):
        ctx = make_ctx(sc, precision, scatter=mode)
        g, d = ctx.pncg_gradient(x, xt, h)
        Hp, php = ctx.pncg_hvp(x, p, h)
        res[mode] = (g, d, Hp, php)
        tol = 1e-10 if precision == 0 else 1e-5
        _say(f"  mode {mode}: g {elem(g, g_o):.2e} diag {elem(d, d_o):.2e}")
        assert elem(g, g_o) <= tol and elem(d, d_o) <= tol
        if Hp_o is not None:
            assert elem(Hp, Hp_o) <= tol
    tol = 1e-13 if precision == 0 else 1e-6
    for i, name in enumerate(("g", "diag", "Hp")):
        e = elem(res[SEG][i], res[ATOM][i])
        _say(f"  seg vs atomic {name}: {e:.2e}")
        assert e <= tol, name
    assert abs(res[SEG][3] - res[ATOM][3]) <= tol * abs(res[ATOM][3])
    # whole step, fixed iterations
    sc, x0, v0 = _stack_drop()
    xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=12, eps=0.0, term="delta_e")
    xs = {}
    for mode in (ATOM, SEG):
        ctx = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=mode)
        xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
        xs[mode] = xg
        rdx = rel(xg - x0, xo - x0)
        _say(f"  step mode {mode}: rel_dx {rdx:.3e} elem_dx {elem(xg - x0, xo - x0):.3e} iters {sg['iters']}")
        assert sg["iters"] == st.iters == 12
        assert rel(xg, xo) <= (1e-12 if precision == 0 else 1e-6)
        assert rdx <= (1e-9 if precision == 0 else 1e-3)
    e = elem(xs[SEG] - x0, xs[ATOM] - x0)
    _say(f"  step seg vs atomic elem_dx {e:.2e}")
    assert e <= (1e-9 if precision == 0 else 1e-3)


def _override_lists(P, x, r):
    from oracle import candidates
    pt = candidates.pt_brute(x, P.tris, P.surf_verts, r, P.excl_pt)
    ee = candidates.ee_brute(x, P.edges, r, P.excl_ee)
    return pt, ee


@pytest.mark.parametrize("scatter", [SEG, ATOM])
@pytest.mark.parametrize("precision", [0, 1])
def test_candidates_override_matches_oracle(precision, scatter):
    """An explicit candidate list on both sides: the full list within 4 dhat
    of the start state, then the point-triangle pairs alone.  Steps of 12
    fixed iterations and the gradient query match the oracle under the same
    lists, and dropping the edge-edge pairs changes the result."""
    _say(f"candidates override precision={precision} scatter={scatter}")
    import paper_2405_08001_amd as L
    from oracle import pncg
    sc, x0, v0 = _stack_drop()
    P = make_problem(sc)
    pt, ee = _override_lists(P, x0, 4 * sc.dhat)
    assert len(pt) > 0 and len(ee) > 0
    ctx = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", scatter=scatter)
    outs = {}
    for name, lists in (("full", (pt, ee)), ("pt", (pt, np.zeros((0, 2), np.int64)))):
        ctx.pncg_set_candidates_override(L.KIND_PT, lists[0])
        ctx.pncg_set_candidates_override(L.KIND_EE, lists[1])
        P.set_candidates_override(*lists)
        xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=12, eps=0.0, term="delta_e")
        xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
        _say(f"  {name}: pairs {len(lists[0]) + len(lists[1])} cand {sg['n_candidates']} active {sg['n_active']} "
             f"rel_dx {rel(xg - x0, xo - x0):.3e}")
        assert sg["iters"] == st.iters == 12
        assert sg["n_candidates"] == len(lists[0]) + len(lists[1])
        assert rel(xg, xo) <= (1e-12 if precision == 0 else 1e-6)
        assert rel(xg - x0, xo - x0) <= (1e-9 if precision == 0 else 1e-3)
        # the gradient query at the step's result uses the same list
        xt = P.predictor(x0, v0, sc.h)
        g, _ = ctx.pncg_gradient(xg, xt, sc.h)
        assert elem(g, P.gradient(xg, xt, sc.h)) <= (1e-10 if precision == 0 else 1e-5)
        outs[name] = xg
    assert rel(outs["pt"] - x0, outs["full"] - x0) > 1e-6
    # removing the override returns to the hash
    ctx.pncg_set_candidates_override(L.KIND_PT, None)
    P.set_candidates_override(None, None)
    xo, _, _ = pncg.step(P, x0, v0, sc.h, iter_max=12, eps=0.0, term="delta_e")
    xg, _, _ = ctx.pncg_step(x0, v0, sc.h)
    assert rel(xg - x0, xo - x0) <= (1e-9 if precision == 0 else 1e-3)


def test_candidates_override_rejects_bad_pairs():
    import paper_2405_08001_amd as L
    sc, x0, v0 = _stack_drop()
    ctx = make_ctx(sc, 0)
    t0 = sc.tris[0]
    bad = [
        (L.KIND_PT, [[int(t0[0]), 0]]),                  # vertex of its own triangle
        (L.KIND_PT, [[sc.nV, 0]]),                       # vertex out of range
        (L.KIND_PT, [[0, len(sc.tris)]]),                # triangle out of range
        (L.KIND_EE, [[0, 0]]),                           # an edge with itself
        (7, [[0, 1]]),                                   # unknown kind
    ]
    e0 = sc.edges[0]
    share = [i for i, e in enumerate(sc.edges) if i > 0 and (set(e) & set(e0))]
    bad.append((L.KIND_EE, [[0, share[0]]]))             # shared vertex
    far = [i for i, e in enumerate(sc.edges) if not (set(e) & set(e0))]
    bad.append((L.KIND_EE, [[0, far[0]], [far[0], 0]]))   # the same pair twice
    for kind, pairs in bad:
        with pytest.raises(L.PncgError) as e:
            ctx.pncg_set_candidates_override(kind, np.array(pairs))
        assert e.value.code == L.E_INVAL, (kind, pairs)
