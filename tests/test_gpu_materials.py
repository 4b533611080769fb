"""GPU parity of the material models (SNH, ARAP, FCR beside Neo-Hookean)
against the oracle: queries on deformed, twisted and inverted states, whole
iterations, the batched kernel, the adjoint, and the undefined-I1 error."""
import sys

import numpy as np
import pytest

import scenes
from helpers import make_ctx, make_problem, rel

pytestmark = pytest.mark.gpu

MODELS = ["snh", "arap", "fcr"]
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


def _twisted_state():
    """The cube twisted about its vertical axis (0.9 rad top to bottom) and
    turned by 0.5 rad: rotations far from the identity, the floor barrier
    still active."""
    sc, x, xt = _cube_state()
    c = x[:, :2].mean(axis=0)
    z = x[:, 2]
    ang = 0.5 + 0.9 * (z - z.min()) / (z.max() - z.min())
    d = x[:, :2] - c
    x = x.copy()
    x[:, 0] = c[0] + np.cos(ang) * d[:, 0] - np.sin(ang) * d[:, 1]
    x[:, 1] = c[1] + np.sin(ang) * d[:, 0] + np.cos(ang) * d[:, 1]
    return sc, x, xt


def _inverted_state():
    """One interior vertex pushed through its neighbours: several tets with
    det F < 0 (defined for SNH, ARAP and FCR)."""
    sc, x, xt = _cube_state()
    ctr = x.mean(axis=0)
    v = int(np.argmin(np.linalg.norm(x - ctr, axis=1)))
    x = x.copy()
    x[v, 0] += 1.3 * 0.1 / 6
    return sc, x, xt


STATES = {"cube": _cube_state, "twisted": _twisted_state, "inverted": _inverted_state}


def _lifted(x):
    """The same shape 2 cm higher: no plane within dhat."""
    x = x.copy()
    x[:, 2] += 0.02
    return x


# elastic parts alone (inertia and mass removed): mixed-form elements are
# float32, so a few hundred float32 roundings of a relative size 2^-24
# bound them
TOL_EL = {0: 1e-9, 1: 2e-4}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["cube", "twisted", "inverted"])
@pytest.mark.parametrize("model", MODELS)
def test_material_queries_match_oracle(model, which, precision):
    _say(f"material queries {model} {which} precision={precision}")
    from oracle import elastic
    sc, x, xt = STATES[which]()
    P = make_problem(sc, model=model)
    if which == "inverted":
        F = elastic.deformation_gradient(x, P.tets, P.Bmat)
        assert np.sum(np.linalg.det(F) < 0) >= 2
    ctx = make_ctx(sc, precision, model=model)
    t = TOL[precision]
    h = sc.h
    a = P.active_set(x)
    assert len(a.pd) > 0
    E_ref = P.energy(x, xt, h, a)
    E = ctx.pncg_energy(x, xt, h)
    g, d = ctx.pncg_gradient(x, xt, h)
    p = np.random.default_rng(5).standard_normal(x.shape) * 1e-3
    hp, php = ctx.pncg_hvp(x, p, h)
    ref_php = P.pHp(x, p, h, a)
    errs = dict(e=abs(E - E_ref) / abs(E_ref), g=rel(g, P.gradient(x, xt, h, a)), d=rel(d, P.diag(x, h, a)),
                hp=rel(hp, P.hvp(x, p, h, a)), php=abs(php - ref_php) / abs(ref_php))
    _say("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= t[k], (k, v)
    # elastic parts alone: the state lifted clear of the floor (no barrier),
    # xt = x (no inertia), and the mass part taken out of diag, H p, p^T H p
    xl = _lifted(x)
    al = P.active_set(xl)
    assert len(al.pd) == 0
    m = P.mass[:, None]
    g0, d0 = ctx.pncg_gradient(xl, xl, h)
    hp0, php0 = ctx.pncg_hvp(xl, p, h)
    ref_php0 = P.pHp(xl, p, h, al) - np.sum(m * p * p)
    el = dict(g=rel(g0, P.gradient(xl, xl, h, al)), d=rel(d0 - m, P.diag(xl, h, al) - m),
              hp=rel(hp0 - m * p, P.hvp(xl, p, h, al) - m * p),
              php=abs((php0 - np.sum(m * p * p)) - ref_php0) / abs(ref_php0))
    _say("  elastic parts: " + " ".join(f"{k}={v:.2e}" for k, v in el.items()))
    for k, v in el.items():
        assert v <= TOL_EL[precision], (k, v)


@pytest.mark.parametrize("model", MODELS + ["nh"])
def test_material_elastic_terms_differ_between_models(model):
    """The twisted state separates the models: each model's gradient is its
    own (a model silently running another's kernels fails here)."""
    sc, x, _ = _twisted_state()
    x = _lifted(x)
    ctx = make_ctx(sc, 0, model=model)
    g, _ = ctx.pncg_gradient(x, x, sc.h)
    for other in MODELS + ["nh"]:
        ref = make_problem(sc, model=other).gradient(x, x, sc.h)
        if other == model:
            assert rel(g, ref) <= 1e-10
        else:
            assert rel(g, ref) > 1e-3, other


def _cube_drop():
    sc = scenes.cube_scene()
    x0 = sc.X.copy()
    x0[:, 2] -= 0.05 - 1.2e-3
    # turned rigidly by 0.7 rad about the vertical axis, so that every tet's
    # rotation is far from the identity
    c = x0[:, :2].mean(axis=0)
    d = x0[:, :2] - c
    ca, sa = np.cos(0.7), np.sin(0.7)
    x0[:, 0] = c[0] + ca * d[:, 0] - sa * d[:, 1]
    x0[:, 1] = c[1] + sa * d[:, 0] + ca * d[:, 1]
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
@pytest.mark.parametrize("which", ["cube", "stack"])
@pytest.mark.parametrize("model", MODELS)
def test_material_fixed_iterations_match_oracle(model, which, precision):
    _say(f"material fixed-iteration step {model} {which} precision={precision}")
    from oracle import pncg
    sc, x0, v0 = DROPS[which]()
    K = 12
    P = make_problem(sc, model=model)
    ctx = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e", model=model)
    xo, vo, st = pncg.step(P, x0, v0, sc.h, iter_max=K, eps=0.0, term="delta_e")
    xg, vg, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} rel_x={rx:.3e} rel_dx={rdx:.3e} "
         f"hits {st.alpha_upper_hits}/{sg['alpha_upper_hits']}")
    assert sg["iters"] == st.iters == K
    assert sg["alpha_upper_hits"] == st.alpha_upper_hits
    if precision == 0:
        assert rx <= 1e-12 and rdx <= 1e-9 and rel(vg, vo) <= 1e-9
        return
    # mixed form: within 20x the oracle's own spread when its input carries
    # float32-sized rounding (relative 2^-24), or the Neo-Hookean bars
    u = np.random.default_rng(17).uniform(-1.0, 1.0, x0.shape)
    xp, _, _ = pncg.step(P, x0 * (1.0 + 2.0 ** -24 * u), v0, sc.h, iter_max=K, eps=0.0, term="delta_e")
    env_x, env_dx = rel(xp, xo), rel(xp - x0, xo - x0)
    _say(f"  float32 envelope rel_x={env_x:.3e} rel_dx={env_dx:.3e}")
    assert rx <= max(1e-6, 20 * env_x)
    assert rdx <= max(1e-3, 20 * env_dx)
    assert rel(vg, vo) <= max(1e-3, 20 * env_dx)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("model", ["fcr", "arap"])
def test_material_twisted_bar_first_step_matches_oracle(model, precision):
    """The 15,360-tet bar with its end faces turned 3 degrees each way: the
    corotated terms at large rotations over a mesh of many tiles."""
    from oracle import pncg
    _say(f"twisted bar {model} precision={precision}")
    sc = scenes.twisted_bar_scene()
    tgt = scenes.twist_targets(sc, 1)
    P = make_problem(sc, model=model)
    v0 = np.zeros_like(sc.X)
    xo, vo, st = pncg.step(P, sc.X, v0, sc.h, iter_max=12, eps=0.0, term="delta_e", fixed_targets=tgt)
    ctx = make_ctx(sc, precision, iter_max=12, eps=0.0, term="delta_e", model=model)
    ctx.pncg_set_dirichlet(sc.fixed, tgt)
    xg, vg, sg = ctx.pncg_step(sc.X, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - sc.X, xo - sc.X)
    _say(f"  iters {sg['iters']}/{st.iters} rel_x={rx:.3e} rel_dx={rdx:.3e}")
    assert sg["iters"] == st.iters == 12
    assert rx <= (1e-12 if precision == 0 else 1e-6)
    assert rdx <= (1e-9 if precision == 0 else 1e-3)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("model", MODELS)
def test_material_batch_matches_single_scene_path(model, precision):
    """Fixed 6 iterations per scene: the batched kernel under a model and one
    context per scene under the same model agree to rounding; the setting
    can be changed on a live batch."""
    import torch
    import paper_2405_08001_amd as L
    scs = scenes.batched_scenes(seed=5, n_scenes=4, t_lo=30, t_hi=2000)
    _say(f"batch {model} precision={precision}")
    rng = np.random.default_rng(3)
    xs, vs = [], []
    for s in scs:
        x = s.x0.copy()
        x[:, 2] -= x[:, 2].min() - 1.2e-3
        x += rng.uniform(-5e-5, 5e-5, x.shape)
        v = s.v0.copy()
        v[:, 2] = -0.1
        xs.append(x)
        vs.append(v)
    b = scenes.pack_batch(scs)
    bt = L.Batch(b["vert_off"], b["X"], b["tet_off"], b["tets"], b["tri_off"], b["tris"], b["E"], b["nu"],
                 b["rho"], b["planes"], precision=precision)
    s0 = scs[0]
    bt.pncg_batch_set_params(s0.dhat, s0.kappa, 6, 0.0, L.TERM_DELTA_E, s0.gravity, 0)
    dev = torch.device("cuda:0")

    def step():
        xd = torch.tensor(np.concatenate(xs), dtype=torch.float64, device=dev)
        vd = torch.tensor(np.concatenate(vs), dtype=torch.float64, device=dev)
        xo, vo = torch.empty_like(xd), torch.empty_like(vd)
        bt.pncg_batch_step(xd, vd, s0.h, xo, vo)
        return xo.cpu().numpy()
    x_nh = step()
    bt.pncg_batch_set_model(model)
    xg = step()
    off = b["vert_off"]
    for i, s in enumerate(scs):
        ctx = make_ctx(s, precision, iter_max=6, eps=0.0, term="delta_e", model=model)
        xc, _, st = ctx.pncg_step(xs[i], vs[i], s.h)
        sl = slice(off[i], off[i + 1])
        rdx = rel(xg[sl] - xs[i], xc - xs[i])
        _say(f"  scene {i}: rel_dx={rdx:.3e} (vs NH {rel(x_nh[sl] - xs[i], xc - xs[i]):.2e})")
        assert st["iters"] == 6
        assert rdx <= (1e-9 if precision == 0 else 1e-3)


@pytest.mark.parametrize("model", ["snh", "arap", "fcr"])
def test_material_adjoint_step_matches_oracle(model):
    """lambda and the parameter adjoint under a model: device CG against the
    oracle's sparse direct solve at the oracle's converged x^{t+1}."""
    from oracle import adjoint
    sc = scenes.diff_bar_scene(seed=4, nx=8, ny=3, nz=3, dx=0.01, lift=0.0012)
    P = make_problem(sc, model=model)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    v0[:, 1] = 0.3 * (sc.X[:, 0] - sc.X[:, 0].mean())     # a turn, so that R matters
    x1, _ = adjoint.newton_solve(P, sc.X, v0, sc.h, tol=1e-12)
    rng = np.random.default_rng(8)
    xbar = rng.standard_normal(x1.shape)
    vbar = rng.standard_normal(x1.shape)
    xo, vo, Eo, _ = adjoint.step_adjoint(P, x1, sc.h, xbar, vbar)
    ctx = make_ctx(sc, 0, model=model)
    xg, vg, Eg, st = ctx.pncg_adjoint_step(x1, sc.h, xbar, vbar, cg_tol=1e-13, cg_max=20000)
    _say(f"adjoint {model}: cg {st['cg_iters']} rel xbar {rel(xg, xo):.2e} vbar {rel(vg, vo):.2e} "
         f"Ebar {rel(Eg, Eo):.2e}")
    assert st["reason"] == 0
    assert rel(xg, xo) <= 1e-9 and rel(vg, vo) <= 1e-9 and rel(Eg, Eo) <= 1e-9


@pytest.mark.parametrize("model", ["arap", "fcr"])
def test_material_collapsed_tets_report_inverted(model):
    """Every vertex at one point (F = 0): the rotation of the polar
    decomposition, and with it the I1 Hessian, is undefined; the stable
    Neo-Hookean density is defined there and matches the oracle."""
    import paper_2405_08001_amd as L
    from oracle import elastic
    sc = scenes.tiny_scene()
    x = np.zeros_like(sc.X) + sc.X.mean(axis=0)
    ctx = make_ctx(sc, 0, model=model)
    with pytest.raises(L.PncgError) as ei:
        ctx.pncg_gradient(x, x, sc.h)
    assert ei.value.code == L.E_INVERTED
    with pytest.raises(elastic.InvertedElement):
        make_problem(sc, model=model).diag(x, sc.h)
    ctx = make_ctx(sc, 0, model="snh")
    P = make_problem(sc, model="snh")
    g, _ = ctx.pncg_gradient(x, x, sc.h)
    assert rel(g, P.gradient(x, x, sc.h)) <= 1e-12 or np.abs(g - P.gradient(x, x, sc.h)).max() < 1e-12
    assert abs(ctx.pncg_energy(x, x, sc.h) - P.energy(x, x, sc.h)) <= 1e-11 * abs(P.energy(x, x, sc.h))


def test_unknown_model_is_rejected():
    import paper_2405_08001_amd as L
    sc = scenes.tiny_scene()
    ctx = make_ctx(sc, 0)
    with pytest.raises(L.PncgError) as ei:
        ctx.pncg_set_model(7)
    assert ei.value.code == L.E_INVAL
    scs = scenes.batched_scenes(seed=5, n_scenes=2, t_lo=30, t_hi=200)
    b = scenes.pack_batch(scs)
    bt = L.Batch(b["vert_off"], b["X"], b["tet_off"], b["tets"], b["tri_off"], b["tris"], b["E"], b["nu"],
                 b["rho"], b["planes"], precision=L.MIXED)
    with pytest.raises(L.PncgError) as ei:
        bt.pncg_batch_set_model(-1)
    assert ei.value.code == L.E_INVAL
    bt.pncg_batch_set_model("arap")          # a known model is accepted


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("model", ["snh", "fcr"])
def test_material_split_step_matches_oracle(model, precision):
    """The per-object step (splitting computation) under a model: 10 fixed
    iterations on the stacked cubes against the oracle's split step."""
    from oracle import pncg
    _say(f"material split step {model} precision={precision}")
    sc, x0, v0 = _stack_drop()
    K = 10
    prob = make_problem(sc, model=model)
    xo, _, st = pncg.step(prob, x0, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", split=True)
    ctx = make_ctx(sc, precision, iter_max=K, eps=0.0, term="delta_e", split=True, model=model)
    xg, _, sg = ctx.pncg_step(x0, v0, sc.h)
    rx, rdx = rel(xg, xo), rel(xg - x0, xo - x0)
    bx, bdx = (1e-12, 1e-9) if precision == 0 else (1e-6, 1e-3)
    if precision == 1:
        u = np.random.default_rng(17).uniform(-1.0, 1.0, x0.shape)
        xq = x0 * (1.0 + 2.0 ** -24 * u)
        xp, _, _ = pncg.step(prob, xq, v0, sc.h, iter_max=K, eps=0.0, term="delta_e", split=True)
        bx = max(bx, 20.0 * rel(xp, xo))
        bdx = max(bdx, 20.0 * rel(xp - xq, xo - x0))
    _say(f"  iters oracle={st.iters} gpu={sg['iters']} rel_x={rx:.3e} (bar {bx:.1e}) rel_dx={rdx:.3e} (bar {bdx:.1e})")
    assert sg["iters"] == st.iters == K
    assert sg["alpha_upper_hits"] == st.alpha_upper_hits
    assert rx <= bx and rdx <= bdx


@pytest.mark.parametrize("model", ["snh", "fcr"])
def test_material_trajectory_gradient_matches_oracle(model):
    """The differentiable rollout under a model (the moduli are re-uploaded
    on every pass): 4 steps of the small bar onto the floor, dL/dE against
    the oracle's Newton trajectory and direct-solve adjoint recursion."""
    import torch
    import paper_2405_08001_amd as L
    from oracle import adjoint, problem
    sc = scenes.diff_bar_scene(seed=4, nx=4, ny=2, nz=2, dx=0.01, lift=0.0012)
    v0 = np.zeros_like(sc.X)
    v0[:, 2] = -0.04
    steps = 4
    rng = np.random.default_rng(5)
    E_tgt = 1e5 * np.exp(0.5 * rng.standard_normal(sc.nT))
    P2 = problem.Problem.from_scene(sc, model=model)
    P2.set_material(E_tgt, sc.nu)
    x_tgt = adjoint.trajectory(P2, sc.X, v0, sc.h, steps)[0][-1]
    P = make_problem(sc, model=model)
    Lo, Eo, _ = adjoint.loss_and_gradient(P, sc.X, v0, sc.h, steps, x_tgt)
    ctx = make_ctx(sc, 0, model=model)
    sim = L.Simulation(ctx, sc.nu, sc.rho, sc.h, steps, checkpoint=2, cg_tol=1e-12, cg_max=20000)
    dev = torch.device("cuda:0")
    Et = torch.tensor(sc.E, dtype=torch.float64, requires_grad=True)
    xT, _ = L.simulate(Et, torch.tensor(sc.X, device=dev), torch.tensor(v0, device=dev), sim)
    loss = ((xT - torch.tensor(x_tgt, device=dev)) ** 2).sum()
    loss.backward()
    Lg, Eg = float(loss.detach()), Et.grad.numpy()
    _say(f"trajectory {model}: L {Lg:.6e}/{Lo:.6e} rel dL/dE {rel(Eg, Eo):.2e}")
    assert abs(Lg - Lo) <= 1e-8 * Lo
    assert rel(Eg, Eo) <= 1e-5
