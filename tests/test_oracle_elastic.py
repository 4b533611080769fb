"""Pins for the oracle's Neo-Hookean element terms (Sec. 3.1)."""
import numpy as np
import pytest

from oracle import elastic

MU, LAM = 3.5e4, 1.4e5


def _rand_F(rng, n, s=0.2):
    F = np.eye(3)[None] + s * rng.standard_normal((n, 3, 3))
    F[np.linalg.det(F) < 0.2] = np.eye(3)
    return F


def _rand_tet(rng):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]) * 0.01
    X = X + 1e-3 * rng.standard_normal((4, 3))
    if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) < 0:
        X[[1, 2]] = X[[2, 1]]
    return X


def test_rest_energy_and_stress_vanish():
    F = np.eye(3)[None]
    assert abs(elastic.psi(F, MU, LAM)[0]) < 1e-12
    assert np.abs(elastic.dPsi_dF(F, np.array([MU]), np.array([LAM]))).max() < 1e-9


def test_uniform_scaling_closed_form():
    for s in (0.7, 0.95, 1.0, 1.3, 2.0):
        F = s * np.eye(3)[None]
        ref = 1.5 * MU * (s * s - 1) - 3 * MU * np.log(s) + 4.5 * LAM * np.log(s) ** 2
        assert np.isclose(elastic.psi(F, MU, LAM)[0], ref, rtol=1e-12, atol=1e-9)


def test_first_piola_matches_textbook_formula():
    # Neo-Hookean first Piola-Kirchhoff stress mu (F - F^-T) + lam log J F^-T
    rng = np.random.default_rng(1)
    F = _rand_F(rng, 50)
    mu = np.full(50, MU)
    lam = np.full(50, LAM)
    vecP = elastic.dPsi_dF(F, mu, lam)
    FinvT = np.transpose(np.linalg.inv(F), (0, 2, 1))
    J = np.linalg.det(F)
    P = MU * (F - FinvT) + LAM * np.log(J)[:, None, None] * FinvT
    np.testing.assert_allclose(vecP, elastic.vec(P), rtol=1e-10, atol=1e-6)


def test_rotation_invariance_and_isotropy():
    rng = np.random.default_rng(2)
    F = _rand_F(rng, 20)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    p = elastic.psi(F, MU, LAM)
    np.testing.assert_allclose(elastic.psi(Q[None] @ F, MU, LAM), p, rtol=1e-11)
    np.testing.assert_allclose(elastic.psi(F @ Q[None], MU, LAM), p, rtol=1e-11)


def test_small_strain_limit_is_linear_elasticity():
    # at F = I: dF : C : dF = mu |dF|^2 + mu tr(dF dF) + lam (tr dF)^2
    rng = np.random.default_rng(3)
    K = elastic.d2Psi_dF2(np.eye(3)[None], np.array([MU]), np.array([LAM]))[0]
    for _ in range(10):
        dF = rng.standard_normal((3, 3))
        v = elastic.vec(dF[None])[0]
        ref = MU * np.sum(dF * dF) + MU * np.trace(dF @ dF) + LAM * np.trace(dF) ** 2
        assert np.isclose(v @ K @ v, ref, rtol=1e-12)


def test_dFdx_reproduces_F():
    rng = np.random.default_rng(4)
    X = _rand_tet(rng)
    x = X + 2e-3 * rng.standard_normal((4, 3))
    B, vol = elastic.rest_setup(X, np.array([[0, 1, 2, 3]]))
    b = elastic.shape_vectors(B)
    A = elastic.dF_dx(b)[0]
    F = elastic.deformation_gradient(x, np.array([[0, 1, 2, 3]]), B)
    np.testing.assert_allclose(A @ x.ravel(), elastic.vec(F)[0], rtol=1e-12, atol=1e-14)
    assert np.isclose(vol[0], np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) / 6)


def _elem_energy(x, X):
    T = np.array([[0, 1, 2, 3]])
    B, vol = elastic.rest_setup(X, T)
    F = elastic.deformation_gradient(x.reshape(4, 3), T, B)
    return elastic.element_energy(F, vol, np.array([MU]), np.array([LAM]))[0]


def _elem_grad(x, X):
    T = np.array([[0, 1, 2, 3]])
    B, vol = elastic.rest_setup(X, T)
    F = elastic.deformation_gradient(x.reshape(4, 3), T, B)
    return elastic.element_gradient(F, elastic.shape_vectors(B), vol, np.array([MU]), np.array([LAM]))[0].ravel()


@pytest.mark.parametrize("seed", range(5))
def test_gradient_and_hessian_match_finite_differences(seed):
    rng = np.random.default_rng(10 + seed)
    X = _rand_tet(rng)
    x = (X + 1.5e-3 * rng.standard_normal((4, 3))).ravel()
    T = np.array([[0, 1, 2, 3]])
    B, vol = elastic.rest_setup(X, T)
    F = elastic.deformation_gradient(x.reshape(4, 3), T, B)
    g = _elem_grad(x, X)
    H = elastic.element_hessian(F, elastic.shape_vectors(B), vol, np.array([MU]), np.array([LAM]))[0]
    e = 1e-7
    fd_g = np.array([(_elem_energy(x + e * u, X) - _elem_energy(x - e * u, X)) / (2 * e)
                     for u in np.eye(12)])
    np.testing.assert_allclose(g, fd_g, rtol=1e-6, atol=1e-6 * np.abs(g).max())
    fd_H = np.stack([(_elem_grad(x + e * u, X) - _elem_grad(x - e * u, X)) / (2 * e)
                     for u in np.eye(12)], axis=1)
    np.testing.assert_allclose(H, fd_H, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    np.testing.assert_allclose(H, H.T, rtol=1e-12, atol=1e-9 * np.abs(H).max())


def test_gradient_translation_and_rotation_invariance():
    rng = np.random.default_rng(20)
    X = _rand_tet(rng)
    x = X + 2e-3 * rng.standard_normal((4, 3))
    g = _elem_grad(x.ravel(), X).reshape(4, 3)
    scale = np.abs(g).max()
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * scale
    assert np.abs(np.cross(x, g).sum(axis=0)).max() < 1e-12 * scale * np.abs(x).max()


def test_param_gradient_matches_finite_difference():
    rng = np.random.default_rng(21)
    X = _rand_tet(rng)
    x = X + 2e-3 * rng.standard_normal((4, 3))
    T = np.array([[0, 1, 2, 3]])
    B, vol = elastic.rest_setup(X, T)
    F = elastic.deformation_gradient(x, T, B)
    b = elastic.shape_vectors(B)
    nu = 0.4
    dmu, dlam = elastic.lame(1.0, nu)
    E0 = 1e5
    an = elastic.element_param_gradient(F, b, vol, np.array([dmu]), np.array([dlam]))[0]
    e = 1.0

    def g(E):
        mu, lam = elastic.lame(E, nu)
        return elastic.element_gradient(F, b, vol, np.array([mu]), np.array([lam]))[0]
    fd = (g(E0 + e) - g(E0 - e)) / (2 * e)
    np.testing.assert_allclose(an, fd, rtol=1e-7, atol=1e-9 * np.abs(an).max())
