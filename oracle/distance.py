"""Closest points of point-triangle and edge-edge primitives (Sec. 3.2).

Both distances are written as d = ||t||, t = sum_i c_i x_i (Sec. 3.2):
  PT: c0 = 1, c1, c2, c3 <= 0, c1 + c2 + c3 = -1  (x0 the point, x1..x3 the
      triangle): t = x0 - (alpha x1 + beta x2 + gamma x3).
  EE: c0, c1 >= 0, c2, c3 <= 0, c0 + c1 = 1, c2 + c3 = -1  (x0-x1 and x2-x3
      the edges): t = (a0 x0 + a1 x1) - (b0 x2 + b1 x3).
The minimisation is done by plain enumeration, which is correct because the
squared distance is a convex quadratic over a convex domain: if the
unconstrained stationary point lies in the domain it is the minimiser,
otherwise the minimum lies on the boundary, i.e. on one of the triangle's
three edges (PT) or on one of the four sides s=0, s=1, u=0, u=1 of the
parameter square (EE), each a clamped point-segment projection.  On exact
ties the first case in that order wins (ties="first"); ties="last" takes the
last, an equally valid choice.  Ties occur where the closest points are not
unique (parallel overlapping edges, a point equidistant from two triangle
edges): there the distance is the same either way but the coefficients c,
and so the barrier gradient's split over the four vertices, are not, and a
test can measure how far that choice alone moves a result.

Readings: a zero-area triangle is an input error; two edges count as parallel
(no interior stationary point) when (d1.d1)(d2.d2) - (d1.d2)^2 <=
1e-12 (d1.d1)(d2.d2).
"""
import numpy as np

PARALLEL_TOL = 1e-12


class DegenerateTriangle(ValueError):
    pass


def _dot(a, b):
    return np.einsum("ni,ni->n", a, b)


def point_segment(p, a, b):
    """Clamped projection of p onto segment a-b.  Returns (tau, t = p - q)."""
    ab = b - a
    den = _dot(ab, ab)
    tau = np.clip(_dot(p - a, ab) / den, 0.0, 1.0)
    t = (p - a) - tau[:, None] * ab
    return tau, t


def _pick(d2, ties):
    """Index of the smallest candidate per pair: the first of equal ones, or
    the last (ties="last")."""
    if ties == "first":
        return np.argmin(d2, axis=0)
    if ties == "last":
        return d2.shape[0] - 1 - np.argmin(d2[::-1], axis=0)
    raise ValueError(f"ties must be 'first' or 'last', not {ties!r}")


def point_triangle(x0, x1, x2, x3, ties="first"):
    """Vectorised over n pairs (arrays (n,3)).  Returns c (n,4), t (n,3), d (n,)."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (x0, x1, x2, x3))
    n = x0.shape[0]
    e1, e2, w = x2 - x1, x3 - x1, x0 - x1
    a11, a12, a22 = _dot(e1, e1), _dot(e1, e2), _dot(e2, e2)
    r1, r2 = _dot(e1, w), _dot(e2, w)
    det = a11 * a22 - a12 * a12
    if np.any(det <= 0):
        raise DegenerateTriangle("zero-area triangle")
    s = (a22 * r1 - a12 * r2) / det        # weight of x2
    u = (a11 * r2 - a12 * r1) / det        # weight of x3
    inside = (s >= 0) & (u >= 0) & (s + u <= 1)
    # candidate 0: interior projection; 1..3: edges x1-x2, x2-x3, x3-x1
    C = np.zeros((4, n, 4))
    Tt = np.zeros((4, n, 3))
    C[0, :, 0] = 1.0
    C[0, :, 1] = -(1.0 - s - u)
    C[0, :, 2] = -s
    C[0, :, 3] = -u
    Tt[0] = w - s[:, None] * e1 - u[:, None] * e2
    for k, (ia, ib, pa, pb) in enumerate(((1, 2, x1, x2), (2, 3, x2, x3), (3, 1, x3, x1)), start=1):
        tau, t = point_segment(x0, pa, pb)
        C[k, :, 0] = 1.0
        C[k, :, ia] = -(1.0 - tau)
        C[k, :, ib] = -tau
        Tt[k] = t
    d2 = np.einsum("kni,kni->kn", Tt, Tt)
    d2[0, ~inside] = np.inf
    pick = _pick(d2, ties)
    idx = np.arange(n)
    c = C[pick, idx]
    t = Tt[pick, idx]
    return c, t, np.sqrt(_dot(t, t))


def edge_edge(x0, x1, x2, x3, ties="first"):
    """Vectorised over n pairs.  Returns c (n,4), t (n,3), d (n,)."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (x0, x1, x2, x3))
    n = x0.shape[0]
    d1, d2, r = x1 - x0, x3 - x2, x0 - x2
    a, bb, cc = _dot(d1, d1), _dot(d1, d2), _dot(d2, d2)
    e, f = _dot(d1, r), _dot(d2, r)
    det = a * cc - bb * bb
    nonpar = det > PARALLEL_TOL * a * cc
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (bb * f - cc * e) / det
        u = (a * f - bb * e) / det
    inside = nonpar & (s >= 0) & (s <= 1) & (u >= 0) & (u <= 1)
    s = np.where(inside, s, 0.0)
    u = np.where(inside, u, 0.0)
    S = np.zeros((5, n))
    U = np.zeros((5, n))
    S[0], U[0] = s, u
    # s = 0: point x0 against edge 2;  s = 1: point x1 against edge 2
    U[1], _ = point_segment(x0, x2, x3)
    S[2] = 1.0
    U[2], _ = point_segment(x1, x2, x3)
    # u = 0: point x2 against edge 1;  u = 1: point x3 against edge 1
    S[3], _ = point_segment(x2, x0, x1)
    S[4], _ = point_segment(x3, x0, x1)
    U[4] = 1.0
    Tt = r[None] + S[..., None] * d1[None] - U[..., None] * d2[None]
    dd = np.einsum("kni,kni->kn", Tt, Tt)
    dd[0, ~inside] = np.inf
    pick = _pick(dd, ties)
    idx = np.arange(n)
    s, u = S[pick, idx], U[pick, idx]
    t = Tt[pick, idx]
    c = np.stack([1.0 - s, s, -(1.0 - u), -u], axis=1)
    return c, t, np.sqrt(_dot(t, t))


def point_plane(x, n, o):
    """Signed distance n.x - o of points x (n,3) to the plane (n, o)."""
    return np.asarray(x) @ np.asarray(n, dtype=np.float64) - o
