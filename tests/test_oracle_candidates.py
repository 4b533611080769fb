"""Pins for the oracle's candidate sets (inflated-AABB definition)."""
import numpy as np
import pytest

import scenes
from oracle import candidates, distance


def _deformed_bar(seed, n=(6, 3, 3), amp=4e-3):
    X, T = scenes.hex_grid(*n, 0.01)
    tris, edges, sv = scenes.surface_of(T)
    rng = np.random.default_rng(seed)
    # fold the bar so that its two halves come close, then jitter
    x = X.copy()
    L = n[0] * 0.01
    sel = x[:, 0] > L / 2
    x[sel, 0] = L - x[sel, 0] + 0.002
    x[sel, 2] = x[sel, 2] + n[2] * 0.01 + 0.0015
    x += rng.uniform(-amp, amp, size=x.shape) * 0.1
    return X, x, T, tris, edges, sv


@pytest.mark.parametrize("seed", range(3))
def test_sweep_equals_brute_force(seed):
    X, x, T, tris, edges, sv = _deformed_bar(seed)
    for r in (1e-3, 3e-3, 1e-2):
        a = candidates.pt_candidates(x, tris, sv, r)
        b = candidates.pt_brute(x, tris, sv, r)
        assert np.array_equal(a, b)
        a = candidates.ee_candidates(x, edges, r)
        b = candidates.ee_brute(x, edges, r)
        assert np.array_equal(a, b)


def test_candidates_contain_every_close_pair():
    # completeness against exact distances over all pairs
    X, x, T, tris, edges, sv = _deformed_bar(5)
    r = 2.5e-3
    pt = {tuple(p) for p in candidates.pt_candidates(x, tris, sv, r)}
    V, F = np.meshgrid(sv, np.arange(len(tris)), indexing="ij")
    V, F = V.ravel(), F.ravel()
    keep = ~np.any(tris[F] == V[:, None], axis=1)
    V, F = V[keep], F[keep]
    f = tris[F]
    _, _, d = distance.point_triangle(x[V], x[f[:, 0]], x[f[:, 1]], x[f[:, 2]])
    close = {(int(v), int(k)) for v, k in zip(V[d < r], F[d < r])}
    assert len(close) > 0 and close <= pt
    ee = {tuple(p) for p in candidates.ee_candidates(x, edges, r)}
    I, J = np.triu_indices(len(edges), 1)
    ea, eb = edges[I], edges[J]
    ok = ~((ea[:, :1] == eb).any(1) | (ea[:, 1:] == eb).any(1))
    I, J, ea, eb = I[ok], J[ok], ea[ok], eb[ok]
    _, _, d = distance.edge_edge(x[ea[:, 0]], x[ea[:, 1]], x[eb[:, 0]], x[eb[:, 1]])
    close = {(int(i), int(j)) for i, j in zip(I[d < r], J[d < r])}
    assert len(close) > 0 and close <= ee


def test_candidate_lists_sorted_and_topology_free():
    X, x, T, tris, edges, sv = _deformed_bar(1)
    pt = candidates.pt_candidates(x, tris, sv, 3e-3)
    ee = candidates.ee_candidates(x, edges, 3e-3)
    for lst in (pt, ee):
        keys = lst[:, 0].astype(np.int64) * 10 ** 7 + lst[:, 1]
        assert np.all(np.diff(keys) > 0)
    assert not np.any(tris[pt[:, 1]] == pt[:, :1])
    assert np.all(ee[:, 0] < ee[:, 1])
    assert not np.any((edges[ee[:, 0]][:, :, None] == edges[ee[:, 1]][:, None, :]).any((1, 2)))


def test_plane_candidates():
    x = np.array([[0, 0, 1e-3], [0, 0, 2e-3], [0, 0, 0.5e-3], [1, 1, 1.0]])
    pg = candidates.pg_candidates(x, np.arange(4), [[0, 0, 1, 0.0], [0, 0, -1, -1.0005]], 1e-3)
    assert [tuple(p) for p in pg] == [(0, 0), (2, 0), (3, 1)]


def test_rest_exclusion_empty_on_coarse_meshes():
    # edges of 1 cm are far longer than 1.5 dhat = 1.5 mm: nothing but
    # topology is close in the rest shape
    X, T = scenes.hex_grid(8, 2, 2, 0.01)
    tris, edges, sv = scenes.surface_of(T)
    pk, ek = candidates.rest_exclusion(X, tris, edges, sv, 1e-3)
    assert len(pk) == 0 and len(ek) == 0


def test_rest_exclusion_catches_close_rest_pairs():
    # two blocks 1 mm apart at rest: pairs across the gap are excluded at 1.5 dhat
    Xa, Ta = scenes.hex_grid(2, 2, 1, 0.01)
    Xb, Tb = scenes.hex_grid(2, 2, 1, 0.01, origin=(0.0, 0.0, 0.011))
    X, T, oid = scenes.merge_meshes([(Xa, Ta), (Xb, Tb)])
    tris, edges, sv = scenes.surface_of(T)
    # as two objects the pairs across the gap are not self-collision pairs
    pk2, ek2 = candidates.rest_exclusion(X, tris, edges, sv, 1e-3, oid)
    assert len(pk2) == 0 and len(ek2) == 0
    pk, ek = candidates.rest_exclusion(X, tris, edges, sv, 1e-3)
    assert len(pk) > 0 and len(ek) > 0
    # what remains after exclusion is at least 1.5 dhat apart at rest
    pt = candidates.pt_candidates(X, tris, sv, 1e-3, pk)
    ee = candidates.ee_candidates(X, edges, 1e-3, ek)
    f = tris[pt[:, 1]]
    _, _, d = distance.point_triangle(X[pt[:, 0]], X[f[:, 0]], X[f[:, 1]], X[f[:, 2]])
    assert np.all(d >= 1.5e-3)
    ea, eb = edges[ee[:, 0]], edges[ee[:, 1]]
    _, _, d = distance.edge_edge(X[ea[:, 0]], X[ea[:, 1]], X[eb[:, 0]], X[eb[:, 1]])
    assert np.all(d >= 1.5e-3)
    # and every excluded pair was a candidate closer than that
    full = candidates.pt_candidates(X, tris, sv, 1e-3)
    keys = (full[:, 0].astype(np.int64) << 32) | full[:, 1]
    assert np.all(np.isin(pk[np.isin(pk, keys)], keys)) and len(full) - len(pt) == np.isin(keys, pk).sum()
