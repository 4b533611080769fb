"""Pins for the oracle's Algorithm 1 driver (Sec. 4)."""
import numpy as np
import pytest
from scipy.optimize import brentq

import scenes
from oracle import barrier, pncg, problem


class _Quadratic:
    """E(x) = 1/2 x^T A x - b^T x in the Problem interface (no contact)."""

    def __init__(self, A, b):
        self.A, self.bv = A, b
        n = b.size // 3
        self.fixed = np.zeros(0, np.int64)
        self.free = np.ones(n, bool)
        self.has_collision_primitives = False
        self.dhat = 1.0

    def predictor(self, x_t, v_t, h):
        return x_t

    def active_set(self, x):
        return None

    def gradient(self, x, xt, h, aset=None):
        return (self.A @ x.ravel() - self.bv).reshape(-1, 3)

    def diag(self, x, h, aset=None):
        return np.diag(self.A).reshape(-1, 3).copy()

    def pHp(self, x, p, h, aset=None):
        return float(p.ravel() @ self.A @ p.ravel())

    def energy(self, x, xt, h, aset=None):
        return 0.5 * x.ravel() @ self.A @ x.ravel() - self.bv @ x.ravel()


def _textbook_pcg(A, b, x0, iters):
    """Jacobi-preconditioned linear conjugate gradient (Hestenes-Stiefel form)."""
    Minv = 1.0 / np.diag(A)
    x = x0.copy()
    r = b - A @ x
    z = Minv * r
    p = z.copy()
    xs = []
    for _ in range(iters):
        Ap = A @ p
        a = (r @ z) / (p @ Ap)
        x = x + a * p
        xs.append(x.copy())
        r_new = r - a * Ap
        z_new = Minv * r_new
        beta = (r_new @ z_new) / (r @ z)
        p = z_new + beta * p
        r, z = r_new, z_new
    return xs


def test_dk_with_newton_step_is_jacobi_pcg_on_quadratics():
    # With an exact line search p_k^T g_{k+1} = 0, so the preconditioned
    # Dai-Kou beta reduces to preconditioned Hestenes-Stiefel, i.e. linear PCG.
    rng = np.random.default_rng(0)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(0.5, 5, n))
    b = rng.standard_normal(n)
    qp = _Quadratic(A, b)
    ref = _textbook_pcg(A, b, np.zeros(n), 12)
    for k in range(1, 13):
        x, _, st = pncg.step(qp, np.zeros((n // 3, 3)), np.zeros((n // 3, 3)), 1.0,
                             iter_max=k, eps=0.0, term="delta_e")
        assert st.iters == k
        np.testing.assert_allclose(x.ravel(), ref[k - 1], rtol=1e-9, atol=1e-12)
    # and it converges to the solution of A x = b
    x, _, st = pncg.step(qp, np.zeros((n // 3, 3)), np.zeros((n // 3, 3)), 1.0,
                         iter_max=200, eps=1e-13, term="grad_rel")
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b), rtol=1e-10)


@pytest.mark.parametrize("rule", pncg.BETA_RULES)
def test_every_beta_rule_is_jacobi_pcg_on_quadratics(rule):
    # With an exact line search (the Newton step on a quadratic) and a fixed
    # preconditioner, FR, PRP, CD, HZ and DK all reduce to linear PCG: the
    # terms that tell them apart (g^T P g_k, d^T g) vanish by conjugacy.
    rng = np.random.default_rng(1)
    n = 24
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(0.5, 5, n))
    b = rng.standard_normal(n)
    qp = _Quadratic(A, b)
    ref = _textbook_pcg(A, b, np.zeros(n), 10)
    for k in (1, 2, 5, 10):
        x, _, st = pncg.step(qp, np.zeros((n // 3, 3)), np.zeros((n // 3, 3)), 1.0,
                             iter_max=k, eps=0.0, term="delta_e", beta_rule=rule)
        assert st.iters == k
        np.testing.assert_allclose(x.ravel(), ref[k - 1], rtol=1e-9, atol=1e-12)


def test_hz_and_dk_sufficient_descent_bounds():
    # The Hager-Zhang family beta = g^T P y / d^T y - c (y^T P y / d^T y)(d^T g / d^T y)
    # gives d_new^T g <= -(1 - 1/(4c)) g^T P g for ANY line search (Hager and
    # Zhang 2005, Thm 1.1, in the P metric): 7/8 for HZ (c = 2), 3/4 for DK
    # (c = 1).  Random inexact states: both bounds hold, and DK breaks the HZ
    # bound somewhere (so the two factors are told apart).
    rng = np.random.default_rng(2)
    dk_breaks_hz = 0
    for _ in range(4000):
        n = 6
        g, gp, d = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
        P = rng.uniform(0.1, 3.0, n)
        gPg = float(g @ (P * g))
        for rule, bound in (("dk", 0.75), ("hz", 0.875)):
            b = pncg.beta_value(rule, g, P, gp, P, d)
            r = float((-P * g + b * d) @ g) / gPg
            assert r <= -bound + 1e-12
            if rule == "dk" and r > -0.875:
                dk_breaks_hz += 1
    assert dk_breaks_hz > 0


def test_beta_rules_special_cases():
    # unchanged gradient (y = 0): PRP, HZ and DK give 0, FR gives 1; CD gives
    # -g^T P g / (d^T g_k), which is 1 when d = -P g_k (a steepest-descent
    # previous direction)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(9)
    P = rng.uniform(0.5, 2.0, 9)
    d = rng.standard_normal(9)
    assert pncg.beta_value("prp", g, P, g, P, d) == 0.0
    assert pncg.beta_value("hz", g, P, g, P, d) == 0.0
    assert pncg.beta_value("dk", g, P, g, P, d) == 0.0
    assert pncg.beta_value("fr", g, P, g, P, d) == pytest.approx(1.0, rel=1e-15)
    assert pncg.beta_value("cd", g, P, g, P, -P * g) == pytest.approx(1.0, rel=1e-15)
    with pytest.raises(ValueError):
        pncg.beta_value("xx", g, P, g, P, d)


def test_beta_rules_differ_on_a_contact_step():
    # on a real (non-quadratic) step the rules take different paths
    sc = scenes.cube_scene()
    P_ = problem.Problem.from_scene(sc)
    x0 = sc.X.copy()
    x0[:, 2] -= 0.05 - 1.2e-3
    v0 = np.zeros_like(x0)
    v0[:, 2] = -0.1
    xs = {r: pncg.step(P_, x0, v0, sc.h, iter_max=6, eps=0.0, beta_rule=r)[0] for r in pncg.BETA_RULES}
    for r in pncg.BETA_RULES:
        if r != "dk":
            assert not np.array_equal(xs[r], xs["dk"]), r


def test_free_fall_converges_to_predictor():
    # no contact: the minimiser of the incremental potential is the rigidly
    # translated predictor x^t + h v + h^2 g (zero elastic energy there)
    sc = scenes.tiny_scene()
    P = problem.Problem.from_scene(sc)
    v0 = np.tile([0.1, -0.2, 0.05], (sc.nV, 1))
    x, v, st = pncg.step(P, sc.X, v0, sc.h, iter_max=2000, eps=1e-12, term="grad_rel")
    xt = sc.X + sc.h * v0 + sc.h ** 2 * np.array([0, 0, -9.8])
    np.testing.assert_allclose(x, xt, atol=1e-12)
    np.testing.assert_allclose(v, (xt - sc.X) / sc.h, atol=1e-9)


def test_vertices_resting_on_floor_match_scalar_root():
    # a single tet with a negligible modulus over z = 0: each vertex solves
    # m (z - zt) + kappa b'(z) = 0 on its own (lumped mass, plane barrier)
    X = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0], [0, 0, 0.01]]) + np.array([0, 0, 8e-4])
    tets = np.array([[0, 1, 2, 3]])
    tris, edges, _ = scenes.surface_of(tets)
    dhat, kappa, h = 1e-3, 1e-2, 1.0 / 60
    P = problem.Problem(X, tets, tris, edges, E=1e-9, nu=0.3, rho=1000.0,
                        planes=[[0, 0, 1, 0.0]], dhat=dhat, kappa=kappa)
    v0 = np.zeros((4, 3))
    v0[:, 2] = -0.05
    x, _, st = pncg.step(P, X, v0, h, iter_max=5000, eps=1e-11, term="grad_rel")
    zt = X[:, 2] + h * v0[:, 2] - h * h * 9.8
    for i in range(4):
        m = P.mass[i]
        if zt[i] >= dhat:
            ref = zt[i]
        else:
            f = lambda z: m * (z - zt[i]) + kappa * barrier.db(np.array([z]), dhat)[0]
            ref = brentq(f, 1e-12, dhat, xtol=1e-16, rtol=1e-15)
        assert np.isclose(x[i, 2], ref, rtol=1e-7), (i, x[i, 2], ref)
        assert x[i, 2] > 0


def test_cube_drop_invariants():
    sc = scenes.cube_scene()
    P = problem.Problem.from_scene(sc)
    x, v = sc.x0.copy(), sc.v0.copy()
    for s in range(2):
        x, v, st = pncg.step(P, x, v, sc.h, iter_max=sc.iter_max, eps=sc.eps, term=sc.term,
                             track_energy=True)
        assert st.energy_increase == 0
        dmin, jmin = P.min_distance(x)
        assert dmin > 0 and jmin > 0


def test_energy_decrease_matches_prediction_on_contact_scene():
    # dE = -alpha g^T p - alpha^2/2 p^T H p is the exact decrease of the
    # quadratic model; for small steps it tracks the true energy decrease
    sc = scenes.small_contact_scene()
    P = problem.Problem.from_scene(sc)
    v0 = np.zeros_like(sc.X)
    v0[sc.object_id == 1, 2] = -0.05
    x, v, st = pncg.step(P, sc.X, v0, sc.h, iter_max=60, eps=1e-6, record=True, track_energy=True)
    assert st.iters > 5
    dmin, jmin = P.min_distance(x)
    assert dmin > 0 and jmin > 0
    assert st.energy_increase == 0
    hist = st.history
    assert all(hh["alpha"] > 0 and hh["dE"] > 0 for hh in hist)


def test_alpha_upper_caps_vertex_displacement():
    sc = scenes.small_contact_scene()
    P = problem.Problem.from_scene(sc)
    v0 = np.zeros_like(sc.X)
    v0[sc.object_id == 1, 2] = -0.5
    x_prev = sc.X.copy()
    xt = P.predictor(sc.X, v0, sc.h)
    x, _, st = pncg.step(P, sc.X, v0, sc.h, iter_max=1, eps=0.0)
    assert st.alpha_upper_hits == 1
    disp = np.linalg.norm(x - x_prev, axis=1).max()
    assert disp <= 0.5 * sc.dhat * (1 + 1e-12)


def test_grad_abs_rule_is_grad_rel_scaled_by_g0():
    """The absolute gradient rule with eps * ||g_0|| stops exactly where the
    relative rule with eps does; with eps >= ||g_0|| it stops before any
    update."""
    from helpers import make_problem
    sc = scenes.tiny_scene()
    P = make_problem(sc)
    v0 = np.zeros_like(sc.X)
    v0[:, 0] = 0.3
    xr, _, sr = pncg.step(P, sc.X, v0, sc.h, iter_max=500, eps=1e-6, term="grad_rel")
    xa, _, sa = pncg.step(P, sc.X, v0, sc.h, iter_max=500, eps=1e-6 * sr.g0, term="grad_abs")
    assert sr.reason == "grad_rel" and sa.reason == "grad_abs"
    assert sa.iters == sr.iters and np.array_equal(xa, xr)
    x0, _, s0 = pncg.step(P, sc.X, v0, sc.h, iter_max=500, eps=2.0 * sr.g0, term="grad_abs")
    assert s0.iters == 0 and np.array_equal(x0, sc.X)


# ------------------------------------------------ splitting computation (Sec. 5.2)
def _two_apart_scene():
    """Two cubes 0.2 m apart above a floor (no pair between them ever comes
    near dhat), different stiffness, one dropping onto the floor."""
    Xa, Ta = scenes.hex_grid(3, 3, 3, 0.01, origin=(0.0, 0.0, 5e-4))
    Xb, Tb = scenes.hex_grid(3, 3, 3, 0.01, origin=(0.2, 0.0, 0.02))
    X, tets, oid = scenes.merge_meshes([(Xa, Ta), (Xb, Tb)])
    rng = np.random.default_rng(12)
    X = X + rng.uniform(-2e-4, 2e-4, X.shape)
    E = np.where(np.arange(len(tets)) < len(Ta), 1e5, 1e6)
    sc = scenes.configs._scene(X, tets, E=E, nu=0.4, rho=1000.0, planes=[[0.0, 0.0, 1.0, 0.0]], dhat=1e-3,
                               kappa=1e4, h=1.0 / 60.0, object_id=oid, self_contact=True, cell=4e-3)
    v0 = np.zeros_like(X)
    v0[oid == 0, 2] = -0.1
    return sc, v0, oid


def test_split_with_one_object_is_the_unsplit_step():
    sc = scenes.cube_scene()
    P_ = problem.Problem.from_scene(sc)
    x0 = sc.X.copy()
    x0[:, 2] -= 0.05 - 1.2e-3
    v0 = np.zeros_like(x0)
    v0[:, 2] = -0.1
    for rule in ("dk", "fr"):
        xa, _, sa = pncg.step(P_, x0, v0, sc.h, iter_max=8, eps=0.0, beta_rule=rule)
        xb, _, sb = pncg.step(P_, x0, v0, sc.h, iter_max=8, eps=0.0, beta_rule=rule, split=True)
        assert sa.iters == sb.iters == 8
        assert np.array_equal(xa, xb)
        assert sa.alpha_upper_hits == sb.alpha_upper_hits


def test_split_on_separate_objects_equals_stepping_each_alone():
    # no term couples the two objects, so per-object beta, p and alpha make
    # the union's step exactly the two single-object steps (up to the order
    # of the sums)
    sc, v0, oid = _two_apart_scene()
    P_ = problem.Problem.from_scene(sc)
    xs, _, st = pncg.step(P_, sc.X, v0, sc.h, iter_max=10, eps=0.0, split=True)
    assert st.iters == 10
    xu, _, _ = pncg.step(P_, sc.X, v0, sc.h, iter_max=10, eps=0.0)
    for o in (0, 1):
        m = oid == o
        vmap = -np.ones(len(oid), np.int64)
        vmap[m] = np.arange(m.sum())
        tm = np.all(m[sc.tets], axis=1)
        sub = scenes.configs._scene(sc.X[m], vmap[sc.tets[tm]], E=sc.E[tm], nu=0.4, rho=1000.0,
                                    planes=sc.planes, dhat=sc.dhat, kappa=sc.kappa, h=sc.h,
                                    self_contact=True, cell=4e-3)
        xo, _, so = pncg.step(problem.Problem.from_scene(sub), sub.X, v0[m], sc.h, iter_max=10, eps=0.0)
        assert so.iters == 10
        np.testing.assert_allclose(xs[m], xo, rtol=0, atol=1e-13)
    # while the unsplit step (one alpha for both) moves the free-falling cube
    # differently from its own single-object step
    assert not np.allclose(xu[oid == 1], xs[oid == 1], rtol=0, atol=1e-12)


def test_split_keeps_every_vertex_within_half_dhat_per_iteration():
    sc = scenes.small_contact_scene()
    P_ = problem.Problem.from_scene(sc)
    v0 = np.zeros_like(sc.X)
    v0[sc.object_id == 1, 2] = -0.05
    x_prev = sc.X.copy()
    for k in range(1, 7):
        x, _, st = pncg.step(P_, sc.X, v0, sc.h, iter_max=k, eps=0.0, split=True)
        assert st.iters == k
        assert np.max(np.linalg.norm(x - x_prev, axis=1)) <= 0.5 * sc.dhat * (1 + 1e-12)
        x_prev = x

