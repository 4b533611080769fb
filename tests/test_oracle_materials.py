"""Pins for the oracle's material models (Sec. 3.1 invariants; the SNH,
ARAP and FCR materials of Table 1)."""
import numpy as np
import pytest

from oracle import elastic

MU, LAM = 3.5e4, 1.4e5
MODELS = elastic.MODELS


def _rand_F(rng, n, s=0.2):
    F = np.eye(3)[None] + s * rng.standard_normal((n, 3, 3))
    F[np.linalg.det(F) < 0.2] = np.eye(3)
    return F


def _rand_rotation(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def _arr(v, n=1):
    return np.full(n, float(v))


def _tet(rng):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]) * 0.01
    X = X + 1e-3 * rng.standard_normal((4, 3))
    if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) < 0:
        X[[1, 2]] = X[[2, 1]]
    return X


def _F_of(x, X):
    T = np.array([[0, 1, 2, 3]])
    B, vol = elastic.rest_setup(X, T)
    return elastic.deformation_gradient(x.reshape(4, 3), T, B), elastic.shape_vectors(B), vol


def _energy(x, X, model):
    F, _, vol = _F_of(x, X)
    return elastic.element_energy(F, vol, _arr(MU), _arr(LAM), model)[0]


def _grad(x, X, model):
    F, b, vol = _F_of(x, X)
    return elastic.element_gradient(F, b, vol, _arr(MU), _arr(LAM), model)[0].ravel()


def test_polar_rv_is_a_rotation_variant_svd():
    rng = np.random.default_rng(30)
    F = rng.standard_normal((40, 3, 3))          # about half inverted
    U, s, V = elastic.polar_rv(F)
    np.testing.assert_allclose(U @ (s[:, :, None] * np.transpose(V, (0, 2, 1))), F, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(U), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(V), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.prod(s, axis=1), np.linalg.det(F), rtol=1e-10, atol=1e-12)
    # I1 = max over rotations of tr(Q^T F) (the rotation-variant trace):
    # no random rotation does better
    I1 = s.sum(axis=1)
    for _ in range(200):
        Q = _rand_rotation(rng)
        assert np.all(np.einsum("ij,tij->t", Q, F) <= I1 + 1e-12)


@pytest.mark.parametrize("model", MODELS)
def test_rest_energy_and_stress_vanish(model):
    F = np.eye(3)[None]
    assert abs(elastic.psi(F, _arr(MU), _arr(LAM), model)[0]) < 1e-9
    assert np.abs(elastic.dPsi_dF(F, _arr(MU), _arr(LAM), model)).max() < 1e-9


@pytest.mark.parametrize("model", MODELS)
def test_small_strain_limit_is_linear_elasticity(model):
    # at F = I every model's Hessian is the linear-elastic one with (mu, lam)
    # (ARAP has no volume term: lam = 0):
    # dF : C : dF = mu |dF|^2 + mu tr(dF dF) + lam (tr dF)^2
    rng = np.random.default_rng(31)
    K = elastic.d2Psi_dF2(np.eye(3)[None], _arr(MU), _arr(LAM), model)[0]
    lam = 0.0 if model == "arap" else LAM
    for _ in range(10):
        dF = rng.standard_normal((3, 3))
        v = elastic.vec(dF[None])[0]
        ref = MU * np.sum(dF * dF) + MU * np.trace(dF @ dF) + lam * np.trace(dF) ** 2
        assert np.isclose(v @ K @ v, ref, rtol=1e-11)


def test_corotated_closed_forms():
    rng = np.random.default_rng(32)
    Q = _rand_rotation(rng)
    for s in (0.6, 1.0, 1.4):
        F = (s * Q)[None]
        arap = elastic.psi(F, _arr(MU), _arr(LAM), "arap")[0]
        fcr = elastic.psi(F, _arr(MU), _arr(LAM), "fcr")[0]
        assert np.isclose(arap, 3 * MU * (s - 1) ** 2, rtol=1e-11, atol=1e-6)
        assert np.isclose(fcr, 3 * MU * (s - 1) ** 2 + 0.5 * LAM * (s ** 3 - 1) ** 2, rtol=1e-11, atol=1e-6)
        # stress 2 mu (F - R) + lam (J - 1) cof F with R = Q
        P = 2 * MU * (s - 1) * Q + LAM * (s ** 3 - 1) * s * s * Q
        np.testing.assert_allclose(elastic.dPsi_dF(F, _arr(MU), _arr(LAM), "fcr")[0], elastic.vec(P[None])[0],
                                   rtol=1e-10, atol=1e-6)
    # inverted: F = diag(2, 1, -0.5) keeps R = I and S = F, so
    # |F - R|^2 = 1 + 0 + 2.25
    F = np.diag([2.0, 1.0, -0.5])[None]
    assert np.isclose(elastic.psi(F, _arr(MU), _arr(LAM), "arap")[0], 3.25 * MU, rtol=1e-12)
    np.testing.assert_allclose(elastic.dPsi_dF(F, _arr(MU), _arr(LAM), "arap")[0],
                               elastic.vec((2 * MU * (F[0] - np.eye(3)))[None])[0], atol=1e-8)
    # stable Neo-Hookean on an inverted F: defined, closed form
    J = -0.5 * 2.0
    ref = 0.5 * MU * (4 + 1 + 0.25 - 3) - MU * (J - 1) + 0.5 * (LAM + MU) * (J - 1) ** 2
    assert np.isclose(elastic.psi(F, _arr(MU), _arr(LAM), "snh")[0], ref, rtol=1e-12)


def test_I1_hessian_undefined_raises():
    # singular values (1, 1, -1): the last pair sums to zero
    F = np.diag([1.0, 1.0, -1.0])[None]
    with pytest.raises(elastic.InvertedElement):
        elastic.d2Psi_dF2(F, _arr(MU), _arr(LAM), "arap")
    with pytest.raises(elastic.InvertedElement):
        elastic.psi(F, _arr(MU), _arr(LAM), "nh")


@pytest.mark.parametrize("model", ["arap", "fcr"])
def test_I1_gradient_is_the_derivative_of_the_rotation_variant_trace(model):
    rng = np.random.default_rng(33)
    F = _rand_F(rng, 1, 0.4)
    g1, H1 = elastic.I1_grad_hess(F)
    e = 1e-6

    def I1(G):
        return elastic.polar_rv(G)[1].sum(axis=1)[0]
    fd = np.array([(I1(F + e * elastic.vec_inv(u)) - I1(F - e * elastic.vec_inv(u))) / (2 * e)
                   for u in np.eye(9)])
    np.testing.assert_allclose(g1[0], fd, atol=1e-8)
    # H1 is the Jacobian of vec R
    fdH = np.stack([(elastic.I1_grad_hess(F + e * elastic.vec_inv(u))[0][0]
                     - elastic.I1_grad_hess(F - e * elastic.vec_inv(u))[0][0]) / (2 * e) for u in np.eye(9)], 1)
    np.testing.assert_allclose(H1[0], fdH, atol=1e-7)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("seed", range(3))
def test_gradient_and_hessian_match_finite_differences(model, seed):
    rng = np.random.default_rng(40 + seed)
    X = _tet(rng)
    x = (X + 1.5e-3 * rng.standard_normal((4, 3))).ravel()
    F, b, vol = _F_of(x, X)
    g = _grad(x, X, model)
    H = elastic.element_hessian(F, b, vol, _arr(MU), _arr(LAM), model)[0]
    e = 1e-7
    fd_g = np.array([(_energy(x + e * u, X, model) - _energy(x - e * u, X, model)) / (2 * e) for u in np.eye(12)])
    np.testing.assert_allclose(g, fd_g, rtol=1e-6, atol=1e-6 * np.abs(g).max())
    fd_H = np.stack([(_grad(x + e * u, X, model) - _grad(x - e * u, X, model)) / (2 * e) for u in np.eye(12)], 1)
    np.testing.assert_allclose(H, fd_H, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    np.testing.assert_allclose(H, H.T, atol=1e-9 * np.abs(H).max())


@pytest.mark.parametrize("model", ["snh", "arap", "fcr"])
def test_inverted_tet_finite_differences(model):
    # these models are defined through inversion (the rotation-variant
    # decomposition carries the sign of det F)
    rng = np.random.default_rng(50)
    X = _tet(rng)
    x = X.copy()
    x[3] = X[0] - 0.3 * (X[3] - X[0]) + 1e-3 * rng.standard_normal(3)   # through the base
    x = x.ravel()
    F, b, vol = _F_of(x, X)
    assert np.linalg.det(F[0]) < 0
    g = _grad(x, X, model)
    H = elastic.element_hessian(F, b, vol, _arr(MU), _arr(LAM), model)[0]
    e = 1e-8
    fd_g = np.array([(_energy(x + e * u, X, model) - _energy(x - e * u, X, model)) / (2 * e) for u in np.eye(12)])
    np.testing.assert_allclose(g, fd_g, rtol=1e-5, atol=1e-5 * np.abs(g).max())
    fd_H = np.stack([(_grad(x + e * u, X, model) - _grad(x - e * u, X, model)) / (2 * e) for u in np.eye(12)], 1)
    np.testing.assert_allclose(H, fd_H, rtol=1e-5, atol=1e-5 * np.abs(H).max())


@pytest.mark.parametrize("model", MODELS)
def test_invariance(model):
    rng = np.random.default_rng(34)
    F = _rand_F(rng, 20)
    Q = _rand_rotation(rng)
    p = elastic.psi(F, _arr(MU, 20), _arr(LAM, 20), model)
    np.testing.assert_allclose(elastic.psi(Q[None] @ F, _arr(MU, 20), _arr(LAM, 20), model), p, rtol=1e-10, atol=1e-6)
    np.testing.assert_allclose(elastic.psi(F @ Q[None], _arr(MU, 20), _arr(LAM, 20), model), p, rtol=1e-10, atol=1e-6)
    # element gradient: no net force or torque
    X = _tet(rng)
    x = X + 2e-3 * rng.standard_normal((4, 3))
    g = _grad(x.ravel(), X, model).reshape(4, 3)
    scale = np.abs(g).max()
    assert np.abs(g.sum(axis=0)).max() < 1e-11 * scale
    assert np.abs(np.cross(x, g).sum(axis=0)).max() < 1e-11 * scale * np.abs(x).max()


@pytest.mark.parametrize("model", MODELS)
def test_param_gradient_matches_finite_difference(model):
    rng = np.random.default_rng(35)
    X = _tet(rng)
    x = X + 2e-3 * rng.standard_normal((4, 3))
    F, b, vol = _F_of(x.ravel(), X)
    nu = 0.4
    dmu, dlam = elastic.lame(1.0, nu)
    an = elastic.element_param_gradient(F, b, vol, np.array([dmu]), np.array([dlam]), model)[0]

    def g(E):
        mu, lam = elastic.lame(E, nu)
        return elastic.element_gradient(F, b, vol, np.array([mu]), np.array([lam]), model)[0]
    fd = (g(1e5 + 1.0) - g(1e5 - 1.0)) / 2.0
    np.testing.assert_allclose(an, fd, rtol=1e-7, atol=1e-9 * np.abs(an).max())
