"""Candidate contact pairs and the rest-pose exclusion set.

The paper culls pairs with a grid spatial hash (Sec. 6) and builds the active
set each iteration (Algorithm 1, ComputeConstraintSet).  The hash only
changes speed, so the candidate set is defined here without it, as an
inflated axis-aligned bounding-box test evaluated in float64 (no fused
multiply-add), which makes it reproducible bit for bit:

  PT (v, f), v a surface vertex not in triangle f: for every axis,
      min_f - r <= x_v  and  x_v <= max_f + r
  EE (e1, e2), e1 < e2 surface edges with no common vertex: for every axis,
      min_e1 - r <= max_e2  and  min_e2 <= max_e1 + r
  PG (v, k), v a surface vertex, plane k = (n, o):
      ((n0 x0 + n1 x1) + n2 x2) - o <= r

Each list is returned sorted lexicographically.  Pairs in the rest-pose
exclusion set (pairs closer than 1.5 dhat in the rest shape, Sec. 5.1) are
removed.  ``*_brute`` test every pair; the default routines prune with a
sort along x first and return the same sets (the tests compare them).
"""
import numpy as np

from . import distance


def _keys(a, b):
    return (np.asarray(a, dtype=np.int64) << 32) | np.asarray(b, dtype=np.int64)


def _drop_excluded(pairs, excl_keys):
    if excl_keys is None or len(excl_keys) == 0 or len(pairs) == 0:
        return pairs
    k = _keys(pairs[:, 0], pairs[:, 1])
    return pairs[~np.isin(k, excl_keys)]


def _sorted_pairs(a, b):
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    order = np.lexsort((b, a))
    return np.stack([a[order], b[order]], axis=1).astype(np.int32) if len(a) else np.zeros((0, 2), np.int32)


def pt_brute(x, tris, surf_verts, r, excl_keys=None):
    x = np.asarray(x, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    lo = x[tris].min(axis=1) - r
    hi = x[tris].max(axis=1) + r
    A, B = [], []
    for chunk in np.array_split(np.asarray(surf_verts, dtype=np.int64), max(1, len(surf_verts) // 256)):
        p = x[chunk]
        ok = np.all((lo[None] <= p[:, None]) & (p[:, None] <= hi[None]), axis=2)
        ok &= ~np.any(tris[None, :, :] == chunk[:, None, None], axis=2)
        vi, fi = np.nonzero(ok)
        A.append(chunk[vi])
        B.append(fi)
    pairs = _sorted_pairs(np.concatenate(A) if A else [], np.concatenate(B) if B else [])
    return _drop_excluded(pairs, excl_keys)


def ee_brute(x, edges, r, excl_keys=None):
    x = np.asarray(x, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    mn = x[edges].min(axis=1)
    mx = x[edges].max(axis=1)
    A, B = [], []
    n = len(edges)
    for chunk in np.array_split(np.arange(n), max(1, n // 256)):
        ok = np.all(((mn[chunk, None] - r) <= mx[None]) & (mn[None] <= (mx[chunk, None] + r)), axis=2)
        ok &= chunk[:, None] < np.arange(n)[None]
        sh = (edges[chunk, None, 0:1] == edges[None, :, :]).any(axis=2) | \
             (edges[chunk, None, 1:2] == edges[None, :, :]).any(axis=2)
        ok &= ~sh
        i, j = np.nonzero(ok)
        A.append(chunk[i])
        B.append(j)
    pairs = _sorted_pairs(np.concatenate(A) if A else [], np.concatenate(B) if B else [])
    return _drop_excluded(pairs, excl_keys)


def plane_signed(x, plane):
    """((n0 x0 + n1 x1) + n2 x2) - o, each operation rounded separately."""
    n0, n1, n2, o = (float(v) for v in plane)
    return ((n0 * x[:, 0] + n1 * x[:, 1]) + n2 * x[:, 2]) - o


def pg_candidates(x, surf_verts, planes, r):
    x = np.asarray(x, dtype=np.float64)
    sv = np.asarray(surf_verts, dtype=np.int64)
    A, B = [], []
    for k, pl in enumerate(np.asarray(planes, dtype=np.float64).reshape(-1, 4)):
        ok = plane_signed(x[sv], pl) <= r
        A.append(sv[ok])
        B.append(np.full(int(ok.sum()), k))
    return _sorted_pairs(np.concatenate(A) if A else [], np.concatenate(B) if B else [])


def _sweep_pairs(lo_a, hi_a, lo_b, hi_b):
    """All (i, j) with box a_i overlapping box b_j on every axis (closed
    intervals), found by sorting b along x.  Same set as the double loop."""
    if len(lo_a) == 0 or len(lo_b) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    order = np.argsort(lo_b[:, 0], kind="stable")
    sl = lo_b[order, 0]
    ext = float(np.max(hi_b[:, 0] - lo_b[:, 0]))
    # b_j can overlap a_i on x only if lo_b_x in [lo_a_x - ext', hi_a_x]; the
    # window is widened by one ulp-scale margin and every axis is re-tested
    # exactly below, so the window only has to be a superset.
    start = np.searchsorted(sl, lo_a[:, 0] - ext - 1e-9 * (1 + abs(ext)), side="left")
    stop = np.searchsorted(sl, hi_a[:, 0], side="right")
    cnt = np.maximum(stop - start, 0)
    I = np.repeat(np.arange(len(lo_a)), cnt)
    off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    J = order[np.repeat(start, cnt) + off]
    ok = np.all((lo_a[I] <= hi_b[J]) & (lo_b[J] <= hi_a[I]), axis=1)
    return I[ok], J[ok]


def pt_candidates(x, tris, surf_verts, r, excl_keys=None):
    x = np.asarray(x, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    sv = np.asarray(surf_verts, dtype=np.int64)
    lo_f = x[tris].min(axis=1) - r
    hi_f = x[tris].max(axis=1) + r
    p = x[sv]
    I, J = _sweep_pairs(p, p, lo_f, hi_f)
    v = sv[I]
    keep = ~np.any(tris[J] == v[:, None], axis=1)
    pairs = _sorted_pairs(v[keep], J[keep])
    return _drop_excluded(pairs, excl_keys)


def ee_candidates(x, edges, r, excl_keys=None):
    x = np.asarray(x, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    mn = x[edges].min(axis=1)
    mx = x[edges].max(axis=1)
    I, J = _sweep_pairs(mn - r, mx + r, mn, mx)
    # the exact test is min_i - r <= max_j and min_j <= max_i + r (as above)
    keep = I < J
    I, J = I[keep], J[keep]
    ea, eb = edges[I], edges[J]
    shared = (ea[:, :1] == eb).any(axis=1) | (ea[:, 1:] == eb).any(axis=1)
    pairs = _sorted_pairs(I[~shared], J[~shared])
    return _drop_excluded(pairs, excl_keys)


def rest_exclusion(X, tris, edges, surf_verts, dhat, object_id=None):
    """Keys (a << 32 | b) of self-collision PT and EE pairs (both primitives
    on the same object) closer than 1.5 dhat in the rest shape (Sec. 5.1);
    PT keys use (v, f), EE keys (e1, e2).  Returned as two sorted int64 arrays
    (pt_keys, ee_keys).  ``object_id`` (per vertex) defaults to one object."""
    r = 1.5 * dhat
    pt = pt_candidates(X, tris, surf_verts, r)
    ee = ee_candidates(X, edges, r)
    tris = np.asarray(tris, dtype=np.int64)
    edges = np.asarray(edges, dtype=np.int64)
    if object_id is not None:
        oid = np.asarray(object_id)
        pt = pt[oid[pt[:, 0]] == oid[tris[pt[:, 1], 0]]]
        ee = ee[oid[edges[ee[:, 0], 0]] == oid[edges[ee[:, 1], 0]]]
    pt_keys = np.zeros(0, np.int64)
    ee_keys = np.zeros(0, np.int64)
    if len(pt):
        f = tris[pt[:, 1]]
        _, _, d = distance.point_triangle(X[pt[:, 0]], X[f[:, 0]], X[f[:, 1]], X[f[:, 2]])
        sel = pt[d < r]
        pt_keys = np.sort(_keys(sel[:, 0], sel[:, 1]))
    if len(ee):
        ea, eb = edges[ee[:, 0]], edges[ee[:, 1]]
        _, _, d = distance.edge_edge(X[ea[:, 0]], X[ea[:, 1]], X[eb[:, 0]], X[eb[:, 1]])
        sel = ee[d < r]
        ee_keys = np.sort(_keys(sel[:, 0], sel[:, 1]))
    return pt_keys, ee_keys
