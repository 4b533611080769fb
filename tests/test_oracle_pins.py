"""Pins for three oracle pieces that every other test takes as given: the
Lame parameters (reading S3), the lumped mass (reading S1) and the predicted
energy decrease that drives the stop rule dE < eps dE_0 (Sec. 4.4).

Each pin rests on something other than the formula it checks: hand values,
the definitions of Young's modulus and Poisson's ratio through the small-strain
response of the material law, exact mass conservation, and the exact energy
change of a quadratic objective along a line.
"""
import numpy as np
import pytest

import scenes
from oracle import elastic, pncg, problem


# ----------------------------------------------------------------- Lame (S3)
def test_lame_hand_values():
    # E = 1e5, nu = 0.25: mu = 1e5 / 2.5 = 4e4, lam = 2.5e4 / (1.25 * 0.5) = 4e4
    mu, lam = elastic.lame(1e5, 0.25)
    assert mu == pytest.approx(4e4, rel=1e-15) and lam == pytest.approx(4e4, rel=1e-15)
    # nu = 0: no lateral coupling, mu = E / 2
    mu, lam = elastic.lame(3e5, 0.0)
    assert mu == pytest.approx(1.5e5, rel=1e-15) and lam == 0.0
    # nu = 1/3: mu = 3E/8, lam = 3E/4
    mu, lam = elastic.lame(8e4, 1.0 / 3.0)
    assert mu == pytest.approx(3e4, rel=1e-14) and lam == pytest.approx(6e4, rel=1e-14)


def test_lame_bulk_and_shear_moduli():
    # textbook relations of isotropic linear elasticity: shear modulus
    # G = E / (2 (1 + nu)) and bulk modulus K = lam + 2 mu / 3 = E / (3 (1 - 2 nu))
    rng = np.random.default_rng(0)
    E = np.exp(rng.uniform(np.log(1e3), np.log(1e7), 50))
    nu = rng.uniform(0.0, 0.49, 50)
    mu, lam = elastic.lame(E, nu)
    np.testing.assert_allclose(mu, E / (2 * (1 + nu)), rtol=1e-14)
    np.testing.assert_allclose(lam + 2 * mu / 3, E / (3 * (1 - 2 * nu)), rtol=1e-12)


@pytest.mark.parametrize("model", ["nh", "snh", "fcr"])
def test_uniaxial_small_strain_response_gives_E_and_nu(model):
    # E and nu are defined by uniaxial stress: stretching by eps with lateral
    # strain -nu eps leaves the lateral faces traction-free and needs axial
    # stress E eps.  Feed lame(E, nu) to the material law and check both to
    # first order (the O(eps^2) terms are below the tolerance).
    E, nu = 2.3e5, 0.37
    mu, lam = elastic.lame(E, nu)
    for eps in (1e-6, -1e-6):
        F = np.diag([1 + eps, 1 - nu * eps, 1 - nu * eps])[None]
        P = elastic.vec_inv(elastic.dPsi_dF(F, np.array([mu]), np.array([lam]), model)[0])
        assert P[0, 0] / eps == pytest.approx(E, rel=1e-5)
        assert abs(P[1, 1]) <= 1e-5 * E * abs(eps)
        assert abs(P[2, 2]) <= 1e-5 * E * abs(eps)


# ------------------------------------------------------------ lumped mass (S1)
def test_lumped_mass_single_tet_quarter_each():
    X = np.array([[0, 0, 0], [0.02, 0, 0], [0, 0.03, 0], [0, 0, 0.05]], float)
    tets = np.array([[0, 1, 2, 3]])
    _, vol = elastic.rest_setup(X, tets)
    assert vol[0] == pytest.approx(0.02 * 0.03 * 0.05 / 6, rel=1e-14)   # right-corner tet
    m = elastic.lumped_mass(vol, np.array([1200.0]), tets, 4)
    np.testing.assert_allclose(m, 1200.0 * vol[0] / 4, rtol=1e-15)


def test_lumped_mass_conserves_total_and_counts_shared_vertices():
    sc = scenes.cube_scene()
    _, vol = elastic.rest_setup(sc.X, sc.tets)
    rho = np.random.default_rng(3).uniform(500, 2000, sc.nT)
    m = elastic.lumped_mass(vol, rho, sc.tets, sc.nV)
    # total mass is exact; a cube of side 0.1 m (jittered) has volume near 1e-3 m^3
    assert m.sum() == pytest.approx(float(np.sum(rho * vol)), rel=1e-13)
    assert vol.sum() == pytest.approx(1e-3, rel=1e-2)
    # each vertex: a quarter of every incident tet, by an explicit loop
    ref = np.zeros(sc.nV)
    for e, t in enumerate(sc.tets):
        for a in t:
            ref[a] += rho[e] * vol[e] * 0.25
    np.testing.assert_allclose(m, ref, rtol=1e-13)
    # the problem's masses are these
    P = problem.Problem(sc.X, sc.tets, sc.tris, sc.edges, E=sc.E, nu=sc.nu, rho=rho,
                        planes=sc.planes, dhat=sc.dhat, kappa=sc.kappa)
    np.testing.assert_allclose(P.mass, ref, rtol=1e-13)


# ------------------------------------------------ predicted dE (Sec. 4.4)
class _BoundedQuadratic:
    """E(x) = 1/2 x^T A x - b^T x with a nominal collision primitive, so the
    step bound dhat / (2 max_v |p_v|) applies (no barrier is ever active)."""

    def __init__(self, A, b, dhat):
        self.A, self.bv = A, b
        n = b.size // 3
        self.fixed = np.zeros(0, np.int64)
        self.free = np.ones(n, bool)
        self.has_collision_primitives = True
        self.dhat = dhat

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

    def energy(self, x, xt=None, h=None, aset=None):
        xv = x.ravel()
        return 0.5 * xv @ self.A @ xv - self.bv @ xv


@pytest.mark.parametrize("dhat", [1e3, 5e-2])
def test_predicted_dE_is_the_exact_decrease_on_a_quadratic(dhat):
    # On a quadratic, E(x + alpha p) = E(x) + alpha g^T p + alpha^2/2 p^T A p
    # exactly, so the recorded dE of every iteration must equal the measured
    # E(x_k) - E(x_{k+1}).  dhat = 1e3 never binds (every alpha is the Newton
    # step -g^T p / p^T A p); dhat = 5e-2 makes the step bound win on the first
    # four iterations and the Newton step win on the rest.
    rng = np.random.default_rng(7)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(0.5, 5, n))
    b = rng.standard_normal(n) * 3.0
    qp = _BoundedQuadratic(A, b, dhat)
    x0 = np.zeros((n // 3, 3))
    K = 12
    _, _, st = pncg.step(qp, x0, x0, 1.0, iter_max=K, eps=0.0, term="delta_e", record=True)
    assert st.iters == K
    E_prev = qp.energy(x0)
    n_up = n_bar = 0
    for k in range(1, K + 1):
        xk, _, sk = pncg.step(qp, x0, x0, 1.0, iter_max=k, eps=0.0, term="delta_e")
        E_k = qp.energy(xk)
        rec = st.history[k - 1]
        scale = max(abs(E_prev), abs(E_k), 1.0)
        assert rec["dE"] == pytest.approx(E_prev - E_k, rel=1e-9, abs=1e-12 * scale), k
        if rec["a_up"] < rec["a_bar"]:
            n_up += 1
        else:
            n_bar += 1
        E_prev = E_k
    if dhat > 1.0:
        assert n_up == 0 and n_bar == K
    else:
        assert n_up >= 2 and n_bar >= 2, (n_up, n_bar)


def test_stop_rule_uses_the_first_dE():
    # dE_0 is the first iteration's decrease and the step stops at the first
    # update with dE < eps dE_0; with eps just above dE_k / dE_0 for some k the
    # step must end exactly at that k.
    rng = np.random.default_rng(8)
    n = 24
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(0.5, 5, n))
    b = rng.standard_normal(n)
    qp = _BoundedQuadratic(A, b, 1e3)
    x0 = np.zeros((n // 3, 3))
    _, _, st = pncg.step(qp, x0, x0, 1.0, iter_max=20, eps=0.0, term="delta_e", record=True)
    dE = np.array([hh["dE"] for hh in st.history])
    ratios = dE / dE[0]
    k_stop = 5
    eps = float(ratios[k_stop - 1]) * (1 + 1e-9)
    assert np.all(ratios[: k_stop - 1] >= eps), "ratios must not reach eps earlier for this pin"
    _, _, st2 = pncg.step(qp, x0, x0, 1.0, iter_max=20, eps=eps, term="delta_e")
    assert st2.iters == k_stop and st2.reason == "delta_e"
    assert st2.dE0 == pytest.approx(dE[0], rel=1e-15)
