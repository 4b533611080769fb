"""Pins for the oracle's assembled incremental potential (Sec. 3): gradient,
diag(H), p^T H p and H v against finite differences and against each other."""
import numpy as np
import pytest

import scenes
from oracle import barrier, problem


def _contact_state():
    """Two stacked blocks over a floor, pressed together so that PT, EE and
    plane barriers are all active."""
    sc = scenes.small_contact_scene()
    P = problem.Problem.from_scene(sc)
    x = sc.X.copy()
    top = sc.object_id == 1
    x[top, 2] -= 5.5e-4            # close the 0.4 mm gap to ~0.15 mm
    x[~top, 2] -= 3e-4              # bottom block within dhat of the floor
    xt = P.predictor(x, np.zeros_like(x), sc.h)
    xt += np.random.default_rng(3).uniform(-1e-4, 1e-4, x.shape)
    return sc, P, x, xt


def test_contact_state_has_all_kinds():
    sc, P, x, _ = _contact_state()
    a = P.active_set(x)
    assert np.sum(a.kind == 0) > 0 and np.sum(a.kind == 1) > 0 and len(a.pd) > 0
    assert np.all((a.d > 0) & (a.d < sc.dhat))


def test_gradient_matches_energy_fd():
    sc, P, x, xt = _contact_state()
    g = P.gradient(x, xt, sc.h, project=False)
    rng = np.random.default_rng(0)
    for _ in range(4):
        u = rng.standard_normal(x.shape)
        e = 1e-9
        fd = (P.energy(x + e * u, xt, sc.h) - P.energy(x - e * u, xt, sc.h)) / (2 * e)
        assert np.isclose(np.sum(g * u), fd, rtol=1e-6)


class _FrozenC:
    """Gradient of the contact model with c held at the base point's values
    (Sec. 3.2: dt/dx = [c_i I], d2t/dx2 = 0), used to finite-difference the
    Hessian model."""

    def __init__(self, P, x, xt, h):
        self.P, self.xt, self.h = P, xt, h
        self.a = P.active_set(x)

    def grad(self, x):
        P, a = self.P, self.a
        g = P.mass[:, None] * (x - self.xt)
        from oracle import elastic
        ge = elastic.element_gradient(elastic.deformation_gradient(x, P.tets, P.Bmat), P.b, P.vol, P.mu, P.lam)
        g += self.h ** 2 * P._scatter(ge, P.tets)
        t = np.einsum("na,naj->nj", a.c, x[a.idx])
        d = np.linalg.norm(t, axis=1)
        coef = P.kappa * barrier.db(d, P.dhat) / d
        g += P._scatter(coef[:, None, None] * a.c[:, :, None] * t[:, None, :], a.idx)
        n = P.planes[a.pk, :3]
        dp = np.einsum("ni,ni->n", x[a.pv], n) - P.planes[a.pk, 3]
        g += P._scatter((P.kappa * barrier.db(dp, P.dhat))[:, None, None] * n[:, None, :], a.pv[:, None])
        return g


def test_full_hessian_model_matches_fd_of_frozen_c_gradient():
    sc, P, x, xt = _contact_state()
    fz = _FrozenC(P, x, xt, sc.h)
    np.testing.assert_allclose(fz.grad(x), P.gradient(x, xt, sc.h, project=False), rtol=1e-10,
                               atol=1e-12 * np.abs(fz.grad(x)).max())
    rng = np.random.default_rng(1)
    for _ in range(3):
        p = rng.standard_normal(x.shape)
        e = 1e-10
        fd = (fz.grad(x + e * p) - fz.grad(x - e * p)) / (2 * e)
        Hp = P.hvp(x, p, sc.h, mode="full")
        np.testing.assert_allclose(Hp, fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max())
        assert np.isclose(P.pHp(x, p, sc.h, mode="full"), np.sum(p * fd), rtol=1e-5)


def test_diag_and_pHp_agree_with_assembled_matrix():
    sc, P, x, xt = _contact_state()
    for mode in ("psd", "full"):
        H = P.hessian_matrix(x, sc.h, mode=mode).toarray()
        np.testing.assert_allclose(P.diag(x, sc.h, mode=mode).ravel(), np.diag(H), rtol=1e-12)
        p = np.random.default_rng(2).standard_normal(x.shape)
        assert np.isclose(P.pHp(x, p, sc.h, mode=mode), p.ravel() @ H @ p.ravel(), rtol=1e-11)
        np.testing.assert_allclose(P.hvp(x, p, sc.h, mode=mode).ravel(), H @ p.ravel(),
                                   rtol=1e-10, atol=1e-12 * np.abs(H @ p.ravel()).max())


def test_psd_contact_block_is_projection_of_full():
    # per pair: psd block = full block with its negative t-space eigen-part removed
    sc, P, x, _ = _contact_state()
    a = P.active_set(x)
    full = P._contact_blocks(a, "full")
    psd = P._contact_blocks(a, "psd")
    for k in range(min(len(a.d), 20)):
        w, V = np.linalg.eigh(full[k])
        proj = (V * np.maximum(w, 0)) @ V.T
        np.testing.assert_allclose(psd[k], proj, rtol=1e-8, atol=1e-8 * np.abs(full[k]).max())
        assert np.linalg.eigvalsh(psd[k]).min() > -1e-8 * np.abs(psd[k]).max()


def test_diag_positive_near_contact_with_psd_but_not_full():
    sc, P, x, xt = _contact_state()
    x2 = x.copy()
    top = sc.object_id == 1
    x2[top, 2] -= 1.3e-4     # ~0.02 mm gap: deep in the barrier
    a = P.active_set(x2)
    assert a.d.min() < 0.1 * sc.dhat
    assert P.diag(x2, sc.h, a, "psd").min() > 0
    assert P.diag(x2, sc.h, a, "full").min() < 0


def test_rigid_motion_has_zero_elastic_gradient():
    sc = scenes.tiny_scene()
    P = problem.Problem.from_scene(sc)
    from scenes.mesh import rotation_matrix
    R = rotation_matrix([0.3, -0.5, 0.8], 0.7)
    x = sc.X @ R.T + np.array([0.01, -0.02, 0.03])
    g = P.gradient(x, x, sc.h)             # x = xt: inertia term vanishes too
    assert np.abs(g).max() < 1e-12
    assert abs(P.energy(x, x, sc.h)) < 1e-14


def test_candidates_override_with_the_full_lists_changes_nothing():
    # an explicit list holding every pair within dhat (the brute-force AABB
    # lists) gives the same active set; a subset drops exactly its complement
    sc, P, x, xt = _contact_state()
    a = P.active_set(x)
    from oracle import candidates
    pt = candidates.pt_brute(x, P.tris, P.surf_verts, P.dhat, P.excl_pt)
    ee = candidates.ee_brute(x, P.edges, P.dhat, P.excl_ee)
    P.set_candidates_override(pt, ee[:, ::-1])      # edge order inside a pair does not matter
    b = P.active_set(x)
    order_a = np.lexsort(a.idx.T[::-1])
    order_b = np.lexsort(b.idx.T[::-1])
    np.testing.assert_array_equal(a.idx[order_a], b.idx[order_b])
    np.testing.assert_array_equal(a.d[order_a], b.d[order_b])
    g_full = P.gradient(x, xt, 1.0 / 60, b)
    P.set_candidates_override(pt, None)              # point-triangle pairs only
    c = P.active_set(x)
    assert np.all(c.kind == 0) and np.sum(c.kind == 0) == np.sum(a.kind == 0)
    assert not np.allclose(P.gradient(x, xt, 1.0 / 60, c), g_full)
    P.set_candidates_override(None, None)
    d = P.active_set(x)
    np.testing.assert_array_equal(np.sort(d.d), np.sort(a.d))
