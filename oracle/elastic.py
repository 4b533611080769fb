"""Neo-Hookean hyperelasticity on linear tetrahedra (Sec. 3.1).

The energy density is written with the invariants I2 = tr(F^T F) and
I3 = det F (Sec. 3.1); Neo-Hookean:
    Psi = mu/2 (I2 - 3) - mu log I3 + lam/2 (log I3)^2.
Its Hessian with respect to F is assembled exactly as the paper's chain rule
states it (Sec. 3.1):
    d2Psi/dF2 = sum_i (Psi_ii g_i g_i^T + Psi_i H_i),
with g2 = 2 vec F, H2 = 2 I9, g3 = vec[f1 x f2, f2 x f0, f0 x f1] and H3 the
block cross-product matrix, and mapped to the 12 vertex coordinates through
vec(dF/dx) (9 x 12).  diag(H) and p^T H p are then taken from that explicit
matrix (the "two matrix-matrix products" route the paper compares against),
so this file contains none of the compact per-term formulas.

Discretisation readings: constant-strain tets, F = D_s D_m^{-1}; the element
energy is V_e Psi(F_e) with V_e the rest volume; lumped mass m_v = sum over
incident tets of rho V_e / 4; Lame parameters from (E, nu) by
mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu)).
"""
import numpy as np


class InvertedElement(ValueError):
    """A tet with det F <= 0 (log I3 undefined), or a degenerate rest tet."""


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


def psi(F, mu, lam):
    """Neo-Hookean energy density (Sec. 3.1)."""
    I2, I3 = invariants(F)
    if np.any(I3 <= 0):
        raise InvertedElement("det F <= 0")
    L = np.log(I3)
    return 0.5 * mu * (I2 - 3.0) - mu * L + 0.5 * lam * L * L


def _psi_derivs(I3, mu, lam):
    """Psi_2, Psi_3, Psi_33 of the Neo-Hookean density (Psi_22 = Psi_23 = 0)."""
    L = np.log(I3)
    psi2 = 0.5 * mu
    psi3 = -mu / I3 + lam * L / I3
    psi33 = mu / I3 ** 2 + lam * (1.0 - L) / I3 ** 2
    return psi2, psi3, psi33


def vec(M):
    """Column-wise flattening of (T,3,3) into (T,9): [col0; col1; col2]."""
    return np.transpose(M, (0, 2, 1)).reshape(M.shape[0], 9)


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


def dPsi_dF(F, mu, lam):
    """vec(dPsi/dF) = Psi_2 g2 + Psi_3 g3  (T,9)."""
    _, I3 = invariants(F)
    if np.any(I3 <= 0):
        raise InvertedElement("det F <= 0")
    psi2, psi3, _ = _psi_derivs(I3, mu, lam)
    psi2 = np.broadcast_to(psi2, I3.shape)
    g2, g3, _ = invariant_grads(F)
    return psi2[:, None] * g2 + psi3[:, None] * g3


def d2Psi_dF2(F, mu, lam):
    """9x9 Hessian: Psi_2 H2 + Psi_33 g3 g3^T + Psi_3 H3 (Psi_22 = 0)."""
    _, I3 = invariants(F)
    if np.any(I3 <= 0):
        raise InvertedElement("det F <= 0")
    psi2, psi3, psi33 = _psi_derivs(I3, mu, lam)
    _, g3, H3 = invariant_grads(F)
    H2 = 2.0 * np.eye(9)[None]
    psi2 = np.broadcast_to(psi2, I3.shape)
    return (psi2[:, None, None] * H2 + psi33[:, None, None] * np.einsum("ti,tj->tij", g3, g3)
            + psi3[:, None, None] * H3)


def dF_dx(b):
    """vec(dF/dx) (T,9,12): entry [3j+i, 3a+k] = delta_ik b_a[j]."""
    T = b.shape[0]
    A = np.zeros((T, 9, 12))
    for a in range(4):
        for j in range(3):
            for i in range(3):
                A[:, 3 * j + i, 3 * a + i] = b[:, a, j]
    return A


def element_energy(F, vol, mu, lam):
    return vol * psi(F, mu, lam)


def element_gradient(F, b, vol, mu, lam):
    """(T,4,3): V_e * vec(dF/dx)^T vec(dPsi/dF)."""
    A = dF_dx(b)
    g = np.einsum("tmn,tm->tn", A, dPsi_dF(F, mu, lam))
    return (vol[:, None] * g).reshape(-1, 4, 3)


def element_hessian(F, b, vol, mu, lam):
    """(T,12,12): V_e * vec(dF/dx)^T d2Psi/dF2 vec(dF/dx)  (Sec. 3.1)."""
    A = dF_dx(b)
    K = d2Psi_dF2(F, mu, lam)
    return vol[:, None, None] * (np.transpose(A, (0, 2, 1)) @ (K @ A))


def element_param_gradient(F, b, vol, dmu, dlam):
    """d(element gradient)/d(parameter) for mu = dmu * s, lam = dlam * s
    (the gradient is linear in (mu, lam)); shape (T,4,3)."""
    _, I3 = invariants(F)
    L = np.log(I3)
    g2, g3, _ = invariant_grads(F)
    # dPsi/dF = (mu/2) g2 + ((lam L - mu)/I3) g3, differentiated in s
    dvecP = 0.5 * dmu[:, None] * g2 + ((dlam * L - dmu) / I3)[:, None] * g3
    A = dF_dx(b)
    return (vol[:, None] * np.einsum("tmn,tm->tn", A, dvecP)).reshape(-1, 4, 3)
