"""Hyperelasticity on linear tetrahedra (Sec. 3.1, and the materials of
Table 1).

The energy density is written with the invariants I1 = tr S (polar
decomposition F = R S), I2 = tr(F^T F) and I3 = det F (Sec. 3.1).  Models
(`model` argument):
    "nh"   Neo-Hookean (Sec. 3.1):
           Psi = mu/2 (I2 - 3) - mu log I3 + lam/2 (log I3)^2
    "snh"  stable Neo-Hookean (Smith et al. 2018, in the invariant form of
           Kim and Eberle's course that Sec. 3.1 cites):
           Psi = mu/2 (I2 - 3) - mu (I3 - 1) + lam'/2 (I3 - 1)^2,
           lam' = lam + mu so that its small-strain limit is linear
           elasticity with the same (mu, lam)
    "arap" as-rigid-as-possible: Psi = mu |F - R|^2 = mu (I2 - 2 I1 + 3)
    "fcr"  fixed corotated (Stomakhin et al. 2012):
           Psi = mu |F - R|^2 + lam/2 (I3 - 1)^2
R and S are those of the rotation-variant polar decomposition (R a proper
rotation; an inverted F gives S a negative eigenvalue), so I1 is defined for
every F.
The Hessian with respect to F is assembled exactly as the paper's chain rule
states it (Sec. 3.1):
    d2Psi/dF2 = sum_i (Psi_ii g_i g_i^T + Psi_i H_i),
with g1 = vec R, H1 = sum_i lambda_i q_i q_i^T (the twist eigenpairs of
Kim and Eberle's course: q_i = vec(U T_i V^T) / sqrt 2 with T_i the unit
skew matrices, lambda_i = 2 / (s_j + s_k) over the two singular values that
T_i couples), g2 = 2 vec F, H2 = 2 I9, g3 = vec[f1 x f2, f2 x f0, f0 x f1]
and H3 the block cross-product matrix, and mapped to the 12 vertex
coordinates through vec(dF/dx) (9 x 12).  diag(H) and p^T H p are then taken
from that explicit matrix (the "two matrix-matrix products" route the paper
compares against), so this file contains none of the compact per-term
formulas.  No model's Hessian is projected to be positive semi-definite.

Discretisation readings: constant-strain tets, F = D_s D_m^{-1}; the element
energy is V_e Psi(F_e) with V_e the rest volume; lumped mass m_v = sum over
incident tets of rho V_e / 4; Lame parameters from (E, nu) by
mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu)).
"""
import numpy as np


MODELS = ("nh", "snh", "arap", "fcr")


class InvertedElement(ValueError):
    """A tet with det F <= 0 under the Neo-Hookean model (log I3 undefined),
    a tet whose I1 Hessian is undefined (two singular values of the
    rotation-variant decomposition summing to <= 0), or a degenerate rest
    tet."""


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def rest_setup(X, tets):
    """Returns (Bmat, vol): Bmat[e] = D_m^{-1} (3x3), vol[e] = det(D_m)/6.

    D_m has columns X1-X0, X2-X0, X3-X0.  A tet with det D_m <= 0 raises
    InvertedElement (tets must be given positively oriented).
    """
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(tets, dtype=np.int64)
    Dm = np.stack([X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]],
                   X[T[:, 3]] - X[T[:, 0]]], axis=2)          # (T,3,3), columns
    det = np.linalg.det(Dm)
    if np.any(det <= 0):
        raise InvertedElement(f"{int(np.sum(det <= 0))} rest tets with det <= 0")
    return np.linalg.inv(Dm), det / 6.0


def shape_vectors(Bmat):
    """b_a (T,4,3) with F = sum_a x_a b_a^T: b_1..b_3 are the rows of D_m^{-1}
    and b_0 = -(b_1 + b_2 + b_3)."""
    b = np.empty((Bmat.shape[0], 4, 3))
    b[:, 1:, :] = Bmat
    b[:, 0, :] = -Bmat.sum(axis=1)
    return b


def lumped_mass(vol, rho, tets, nV):
    m = np.zeros(nV)
    share = np.asarray(rho, dtype=np.float64) * vol / 4.0
    for a in range(4):
        m += np.bincount(np.asarray(tets)[:, a], weights=share, minlength=nV)
    return m


def deformation_gradient(x, tets, Bmat):
    """F = D_s D_m^{-1}, D_s columns x1-x0, x2-x0, x3-x0 (T,3,3)."""
    T = np.asarray(tets, dtype=np.int64)
    Ds = np.stack([x[T[:, 1]] - x[T[:, 0]], x[T[:, 2]] - x[T[:, 0]],
                   x[T[:, 3]] - x[T[:, 0]]], axis=2)
    return Ds @ Bmat


def invariants(F):
    I2 = np.einsum("tij,tij->t", F, F)
    I3 = np.linalg.det(F)
    return I2, I3


def _check_model(model):
    if model not in MODELS:
        raise ValueError(f"unknown material model {model!r}")


def polar_rv(F):
    """Rotation-variant SVD F = U diag(s) V^T with det U = det V = +1: the
    sign of det F is carried by the last (smallest) singular value.  Returns
    (U, s, V); R = U V^T, S = V diag(s) V^T, I1 = s0 + s1 + s2."""
    U, s, Vt = np.linalg.svd(F)
    U = U.copy()
    s = s.copy()
    V = np.transpose(Vt, (0, 2, 1)).copy()
    fu = np.linalg.det(U) < 0
    U[fu, :, 2] *= -1.0
    s[fu, 2] *= -1.0
    fv = np.linalg.det(V) < 0
    V[fv, :, 2] *= -1.0
    s[fv, 2] *= -1.0
    return U, s, V


def psi(F, mu, lam, model="nh"):
    """Energy density of `model` (Sec. 3.1, Table 1)."""
    _check_model(model)
    I2, I3 = invariants(F)
    if model == "nh":
        if np.any(I3 <= 0):
            raise InvertedElement("det F <= 0")
        L = np.log(I3)
        return 0.5 * mu * (I2 - 3.0) - mu * L + 0.5 * lam * L * L
    if model == "snh":
        lamp = lam + mu
        return 0.5 * mu * (I2 - 3.0) - mu * (I3 - 1.0) + 0.5 * lamp * (I3 - 1.0) ** 2
    _, s, _ = polar_rv(F)
    I1 = s.sum(axis=1)
    out = mu * (I2 - 2.0 * I1 + 3.0)
    if model == "fcr":
        out = out + 0.5 * lam * (I3 - 1.0) ** 2
    return out


def _psi_derivs(I3, mu, lam, model="nh"):
    """Psi_1, Psi_2, Psi_3, Psi_33 of `model` (no density here has a
    Psi_11, Psi_22 or mixed term)."""
    if model == "nh":
        L = np.log(I3)
        return 0.0 * I3, 0.5 * mu + 0.0 * I3, -mu / I3 + lam * L / I3, mu / I3 ** 2 + lam * (1.0 - L) / I3 ** 2
    if model == "snh":
        lamp = lam + mu
        return 0.0 * I3, 0.5 * mu + 0.0 * I3, lamp * (I3 - 1.0) - mu, lamp + 0.0 * I3
    psi1 = -2.0 * mu + 0.0 * I3
    psi2 = mu + 0.0 * I3
    if model == "arap":
        return psi1, psi2, 0.0 * I3, 0.0 * I3
    return psi1, psi2, lam * (I3 - 1.0), lam + 0.0 * I3


def _uses_I1(model):
    return model in ("arap", "fcr")


def _checked_I3(F, model):
    _, I3 = invariants(F)
    if model == "nh" and np.any(I3 <= 0):
        raise InvertedElement("det F <= 0")
    return I3


def vec(M):
    """Column-wise flattening of (T,3,3) into (T,9): [col0; col1; col2]."""
    return np.transpose(M, (0, 2, 1)).reshape(M.shape[0], 9)


def vec_inv(v):
    """Inverse of vec for one (9,) vector: the 3x3 matrix with columns
    v[0:3], v[3:6], v[6:9]."""
    return np.asarray(v, dtype=np.float64).reshape(3, 3).T


def _cross_matrix(f):
    """(T,3) -> (T,3,3) with hat(f) v = f x v."""
    z = np.zeros(f.shape[0])
    return np.stack([np.stack([z, -f[:, 2], f[:, 1]], -1),
                     np.stack([f[:, 2], z, -f[:, 0]], -1),
                     np.stack([-f[:, 1], f[:, 0], z], -1)], axis=1)


def invariant_grads(F):
    """g2 = 2 vec F, g3 = vec[f1 x f2, f2 x f0, f0 x f1], H3 (9x9 blocks)."""
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    g2 = 2.0 * vec(F)
    g3 = np.concatenate([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=1)
    Z = np.zeros((F.shape[0], 3, 3))
    h0, h1, h2 = _cross_matrix(f0), _cross_matrix(f1), _cross_matrix(f2)
    H3 = np.concatenate([
        np.concatenate([Z, -h2, h1], axis=2),
        np.concatenate([h2, Z, -h0], axis=2),
        np.concatenate([-h1, h0, Z], axis=2)], axis=1)
    return g2, g3, H3


# unit skew matrices of the twist modes and the singular-value pair each
# couples: T couples (i, j) with T[i, j] = -1, T[j, i] = +1
_TWIST = [((0, 1), np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])),
          ((1, 2), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])),
          ((0, 2), np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [-1.0, 0.0, 0.0]]))]


def I1_grad_hess(F):
    """g1 = vec R (T,9) and H1 = sum_i lambda_i q_i q_i^T (T,9,9) from the
    rotation-variant SVD; raises InvertedElement where a lambda_i is
    undefined (s_j + s_k <= 0)."""
    U, s, V = polar_rv(F)
    Vt = np.transpose(V, (0, 2, 1))
    g1 = vec(U @ Vt)
    H1 = np.zeros((F.shape[0], 9, 9))
    for (i, j), T in _TWIST:
        den = s[:, i] + s[:, j]
        if np.any(den <= 0):
            raise InvertedElement("singular values summing to <= 0: I1 Hessian undefined")
        q = vec(U @ T[None] @ Vt) / np.sqrt(2.0)
        H1 += (2.0 / den)[:, None, None] * np.einsum("ti,tj->tij", q, q)
    return g1, H1


def dPsi_dF(F, mu, lam, model="nh"):
    """vec(dPsi/dF) = Psi_1 g1 + Psi_2 g2 + Psi_3 g3  (T,9)."""
    _check_model(model)
    I3 = _checked_I3(F, model)
    psi1, psi2, psi3, _ = _psi_derivs(I3, mu, lam, model)
    g2, g3, _ = invariant_grads(F)
    out = psi2[:, None] * g2 + psi3[:, None] * g3
    if _uses_I1(model):
        g1, _ = I1_grad_hess(F)
        out = out + psi1[:, None] * g1
    return out


def d2Psi_dF2(F, mu, lam, model="nh"):
    """9x9 Hessian: Psi_1 H1 + Psi_2 H2 + Psi_33 g3 g3^T + Psi_3 H3."""
    _check_model(model)
    I3 = _checked_I3(F, model)
    psi1, psi2, psi3, psi33 = _psi_derivs(I3, mu, lam, model)
    _, g3, H3 = invariant_grads(F)
    H2 = 2.0 * np.eye(9)[None]
    out = (psi2[:, None, None] * H2 + psi33[:, None, None] * np.einsum("ti,tj->tij", g3, g3)
           + psi3[:, None, None] * H3)
    if _uses_I1(model):
        _, H1 = I1_grad_hess(F)
        out = out + psi1[:, None, None] * H1
    return out


def dF_dx(b):
    """vec(dF/dx) (T,9,12): entry [3j+i, 3a+k] = delta_ik b_a[j]."""
    T = b.shape[0]
    A = np.zeros((T, 9, 12))
    for a in range(4):
        for j in range(3):
            for i in range(3):
                A[:, 3 * j + i, 3 * a + i] = b[:, a, j]
    return A


def element_energy(F, vol, mu, lam, model="nh"):
    return vol * psi(F, mu, lam, model)


def element_gradient(F, b, vol, mu, lam, model="nh"):
    """(T,4,3): V_e * vec(dF/dx)^T vec(dPsi/dF)."""
    A = dF_dx(b)
    g = np.einsum("tmn,tm->tn", A, dPsi_dF(F, mu, lam, model))
    return (vol[:, None] * g).reshape(-1, 4, 3)


def element_hessian(F, b, vol, mu, lam, model="nh"):
    """(T,12,12): V_e * vec(dF/dx)^T d2Psi/dF2 vec(dF/dx)  (Sec. 3.1)."""
    A = dF_dx(b)
    K = d2Psi_dF2(F, mu, lam, model)
    return vol[:, None, None] * (np.transpose(A, (0, 2, 1)) @ (K @ A))


def element_param_gradient(F, b, vol, dmu, dlam, model="nh"):
    """d(element gradient)/d(parameter) for mu = dmu * s, lam = dlam * s,
    shape (T,4,3).  Every density here has a stress that is linear in
    (mu, lam) jointly, so this is the element gradient evaluated with
    (mu, lam) = (dmu, dlam)."""
    return element_gradient(F, b, vol, np.broadcast_to(dmu, vol.shape), np.broadcast_to(dlam, vol.shape), model)
