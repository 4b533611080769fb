"""Pins for the oracle's closest-point routines (Sec. 3.2, equations PT, EE)."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import distance


def _brute_pt(x0, x1, x2, x3):
    """Minimum over a dense barycentric grid, refined by a bounded local solve."""
    n = 120
    a, b = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1), indexing="ij")
    m = a + b <= 1
    a, b = a[m], b[m]
    pts = x1[None] + a[:, None] * (x2 - x1)[None] + b[:, None] * (x3 - x1)[None]
    dd = np.linalg.norm(pts - x0[None], axis=1)
    i = np.argmin(dd)
    f = lambda z: np.sum((x1 + z[0] * (x2 - x1) + z[1] * (x3 - x1) - x0) ** 2)
    cons = ({"type": "ineq", "fun": lambda z: 1 - z[0] - z[1]},)
    r = minimize(f, [a[i], b[i]], bounds=[(0, 1), (0, 1)], constraints=cons, method="SLSQP",
                 options={"ftol": 1e-30, "maxiter": 500})
    return min(np.sqrt(max(r.fun, 0.0)), dd[i])


def _brute_ee(x0, x1, x2, x3):
    n = 300
    s, u = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1), indexing="ij")
    s, u = s.ravel(), u.ravel()
    pa = x0[None] + s[:, None] * (x1 - x0)[None]
    pb = x2[None] + u[:, None] * (x3 - x2)[None]
    dd = np.linalg.norm(pa - pb, axis=1)
    i = np.argmin(dd)
    f = lambda z: np.sum((x0 + z[0] * (x1 - x0) - x2 - z[1] * (x3 - x2)) ** 2)
    r = minimize(f, [s[i], u[i]], bounds=[(0, 1), (0, 1)], method="L-BFGS-B",
                 options={"ftol": 1e-30, "gtol": 1e-30, "maxiter": 1000})
    return min(np.sqrt(max(r.fun, 0.0)), dd[i])


@pytest.mark.parametrize("seed", range(12))
def test_point_triangle_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((4, 3))
    c, t, d = distance.point_triangle(*(x[i:i + 1] for i in range(4)))
    ref = _brute_pt(*x)
    assert d[0] <= ref + 1e-12
    assert np.isclose(d[0], ref, rtol=1e-6, atol=1e-9)
    # structure of c (Sec. 3.2): c0 = 1, c1..c3 <= 0, sum -1; t = sum c_i x_i
    assert c[0, 0] == 1.0 and np.all(c[0, 1:] <= 0) and np.isclose(c[0, 1:].sum(), -1.0)
    np.testing.assert_allclose(t[0], c[0] @ x, atol=1e-12)


@pytest.mark.parametrize("seed", range(12))
def test_edge_edge_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    x = rng.standard_normal((4, 3))
    c, t, d = distance.edge_edge(*(x[i:i + 1] for i in range(4)))
    ref = _brute_ee(*x)
    assert d[0] <= ref + 1e-12
    assert np.isclose(d[0], ref, rtol=1e-6, atol=1e-9)
    assert np.all(c[0, :2] >= 0) and np.all(c[0, 2:] <= 0)
    assert np.isclose(c[0, :2].sum(), 1.0) and np.isclose(c[0, 2:].sum(), -1.0)
    np.testing.assert_allclose(t[0], c[0] @ x, atol=1e-12)


def test_point_over_face_interior():
    x1, x2, x3 = np.array([0, 0, 0.0]), np.array([1, 0, 0.0]), np.array([0, 1, 0.0])
    x0 = np.array([0.2, 0.3, 0.37])
    c, t, d = distance.point_triangle(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], 0.37, rtol=1e-14)
    np.testing.assert_allclose(c[0], [1, -0.5, -0.2, -0.3], atol=1e-14)


def test_point_edge_and_point_point_regions():
    x1, x2, x3 = np.array([0, 0, 0.0]), np.array([1, 0, 0.0]), np.array([0, 1, 0.0])
    # beyond edge x1-x2 (y < 0): point-edge, c3 = 0
    x0 = np.array([0.4, -0.3, 0.4])
    c, t, d = distance.point_triangle(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], 0.5) and c[0, 3] == 0.0
    # beyond vertex x2: point-point, exactly one nonzero weight
    x0 = np.array([1.5, -0.2, 0.0])
    c, t, d = distance.point_triangle(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], np.hypot(0.5, 0.2)) and np.isclose(c[0, 2], -1.0)


def test_skew_perpendicular_edges():
    x0, x1 = np.array([-1, 0, 0.0]), np.array([1, 0, 0.0])
    x2, x3 = np.array([0.3, -1, 0.25]), np.array([0.3, 1, 0.25])
    c, t, d = distance.edge_edge(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], 0.25, rtol=1e-14)
    np.testing.assert_allclose(c[0], [0.35, 0.65, -0.5, -0.5], atol=1e-14)


def test_parallel_edges():
    # overlapping parallel edges: distance is the separation
    x0, x1 = np.array([0, 0, 0.0]), np.array([1, 0, 0.0])
    x2, x3 = np.array([0.5, 0.2, 0.0]), np.array([1.5, 0.2, 0.0])
    c, t, d = distance.edge_edge(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], 0.2)
    # disjoint collinear edges: endpoint to endpoint
    x2, x3 = np.array([1.5, 0.0, 0.0]), np.array([2.5, 0.0, 0.0])
    c, t, d = distance.edge_edge(x0[None], x1[None], x2[None], x3[None])
    assert np.isclose(d[0], 0.5)
    np.testing.assert_allclose(c[0], [0, 1, -1, 0], atol=1e-14)


def test_ties_pick_another_valid_closest_pair():
    # overlapping parallel edges have a segment of closest-point pairs: both
    # tie rules return the separation as distance and a valid pair (c in
    # range, t = sum c_i x_i), but not the same pair
    x0, x1 = np.array([0, 0, 0.0]), np.array([1, 0, 0.0])
    x2, x3 = np.array([0.5, 0.2, 0.0]), np.array([1.5, 0.2, 0.0])
    X = [v[None] for v in (x0, x1, x2, x3)]
    c1, t1, d1 = distance.edge_edge(*X, ties="first")
    c2, t2, d2 = distance.edge_edge(*X, ties="last")
    assert d1[0] == pytest.approx(0.2, rel=1e-15) and d2[0] == pytest.approx(0.2, rel=1e-15)
    for c, t in ((c1, t1), (c2, t2)):
        assert 0 <= c[0, 1] <= 1 and -1 <= c[0, 3] <= 0
        np.testing.assert_allclose(t[0], c[0, 0] * x0 + c[0, 1] * x1 + c[0, 2] * x2 + c[0, 3] * x3, atol=1e-15)
    assert not np.allclose(c1, c2)
    # the tied sides are s = 1 (x1 against edge 2, at its middle) and u = 0
    # (x2 against edge 1, at its middle): first takes s = 1, last u = 0
    np.testing.assert_allclose(c1[0], [0, 1, -0.5, -0.5], atol=1e-15)
    np.testing.assert_allclose(c2[0], [0.5, 0.5, -1, 0], atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_ties_agree_where_the_closest_point_is_unique(seed):
    # random pairs: the closest point is unique, so both rules give the same
    # distance and coefficients (a vertex closest point reached from two
    # sides may differ in t by rounding only)
    rng = np.random.default_rng(seed)
    X = [rng.standard_normal((200, 3)) for _ in range(4)]
    for fn in (distance.edge_edge, distance.point_triangle):
        ca, ta, da = fn(*X, ties="first")
        cb, tb, db = fn(*X, ties="last")
        assert np.array_equal(da, db)
        assert np.array_equal(ca, cb)
        np.testing.assert_allclose(ta, tb, rtol=0, atol=1e-14)


def test_degenerate_triangle_raises():
    x = np.array([[0, 0, 1.0], [0, 0, 0], [1, 0, 0], [2, 0, 0]])
    with pytest.raises(distance.DegenerateTriangle):
        distance.point_triangle(*(x[i:i + 1] for i in range(4)))


def test_distance_gradient_is_ct_over_d():
    # Danskin: dd/dx_i = c_i t / d, checked by central differences with c re-solved
    rng = np.random.default_rng(7)
    for fn in (distance.point_triangle, distance.edge_edge):
        for _ in range(5):
            x = rng.standard_normal((4, 3))
            c, t, d = fn(*(x[i:i + 1] for i in range(4)))
            g = (c[0][:, None] * t[0][None, :]) / d[0]
            e = 1e-7
            fd = np.zeros((4, 3))
            for i in range(4):
                for j in range(3):
                    xp = x.copy(); xp[i, j] += e
                    xm = x.copy(); xm[i, j] -= e
                    fd[i, j] = (fn(*(xp[k:k + 1] for k in range(4)))[2][0]
                                - fn(*(xm[k:k + 1] for k in range(4)))[2][0]) / (2 * e)
            np.testing.assert_allclose(g, fd, atol=1e-6)
