"""Mesh construction for the synthetic scenes (topology and rest geometry only)."""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# The six tetrahedra of a unit cube that all share the main diagonal
# (0,0,0)-(1,1,1): one per ordering of the three axes (Freudenthal / Kuhn
# split).  Using the same split in every cell gives a conforming mesh.
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_tets():
    """Corner bit-triples of the six tets, each oriented with positive volume."""
    out = []
    for perm in _PERMS:
        c = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] = 1
            c.append(cur)
        m = np.stack([c[1] - c[0], c[2] - c[0], c[3] - c[0]], axis=1)
        if np.linalg.det(m.astype(float)) < 0:
            c[1], c[2] = c[2], c[1]
        out.append(c)
    return out


_KUHN = _kuhn_tets()


@dataclasses.dataclass
class Scene:
    """One simulation input.

    X       float64 (V,3) rest positions
    tets    int32 (T,4) positively oriented
    tris    int32 (F,3) boundary triangles (outward normal by right-hand rule)
    edges   int32 (E,2) boundary edges, i<j, sorted lexicographically
    E, nu, rho   float64 (T,) per-tet Young's modulus, Poisson ratio, density
    x0, v0  float64 (V,3) initial state
    planes  float64 (P,4) half-spaces n.x >= o, rows (n0,n1,n2,o), |n| = 1
    dhat, kappa, h, gravity   contact/time parameters
    object_id int32 (V,) object index of each vertex
    fixed   int32 (n,) indices of prescribed vertices (may be empty)
    """
    X: np.ndarray
    tets: np.ndarray
    tris: np.ndarray
    edges: np.ndarray
    E: np.ndarray
    nu: np.ndarray
    rho: np.ndarray
    x0: np.ndarray
    v0: np.ndarray
    planes: np.ndarray
    dhat: float
    kappa: float
    h: float
    gravity: np.ndarray
    object_id: np.ndarray
    fixed: np.ndarray
    self_contact: bool = False
    name: str = ""
    iter_max: int = 100
    eps: float = 1e-3
    term: str = "delta_e"      # "delta_e" or "grad_rel"
    cell: float = 0.0          # spatial-hash cell size hint (0: library default)
    meta: Optional[dict] = None

    @property
    def nV(self):
        return int(self.X.shape[0])

    @property
    def nT(self):
        return int(self.tets.shape[0])


def rotation_matrix(axis, angle):
    """Rotation by ``angle`` about unit vector ``axis`` (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def random_rotation(rng):
    """Uniform random rotation (from a normalised Gaussian quaternion)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def voxel_mesh(mask, pitch, origin=(0.0, 0.0, 0.0)):
    """Tet mesh of the occupied cells of a boolean voxel grid ``mask[nx,ny,nz]``.

    Every occupied cell is split into six tets sharing its main diagonal.
    Only grid points used by some tet become vertices.  Returns (X, tets).
    """
    mask = np.asarray(mask, dtype=bool)
    nx, ny, nz = mask.shape
    cells = np.argwhere(mask)                       # (C,3)
    gid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    tets = []
    for corners in _KUHN:
        cols = []
        for c in corners:
            cols.append(gid(cells[:, 0] + c[0], cells[:, 1] + c[1], cells[:, 2] + c[2]))
        tets.append(np.stack(cols, axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4)    # cell-major order
    used, inv = np.unique(tets, return_inverse=True)
    tets = inv.reshape(-1, 4).astype(np.int32)
    k = used % (nz + 1)
    j = (used // (nz + 1)) % (ny + 1)
    i = used // ((nz + 1) * (ny + 1))
    X = np.stack([i, j, k], axis=1).astype(np.float64) * pitch + np.asarray(origin, dtype=np.float64)
    return X, tets


def hex_grid(nx, ny, nz, dx, origin=(0.0, 0.0, 0.0)):
    """Box of nx*ny*nz cubes of side dx, six tets per cube: (X, tets)."""
    return voxel_mesh(np.ones((nx, ny, nz), dtype=bool), dx, origin)


def surface_of(tets):
    """Boundary triangles (faces used by exactly one tet, outward oriented),
    boundary edges (unique, i<j, lexicographically sorted) and boundary
    vertices (sorted)."""
    tets = np.asarray(tets, dtype=np.int64)
    # faces opposite each local vertex, ordered so that the normal points
    # away from the opposite vertex for a positively oriented tet
    local = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
    faces = tets[:, local].reshape(-1, 3)
    key = np.sort(faces, axis=1)
    _, idx, cnt = np.unique(key, axis=0, return_index=True, return_counts=True)
    tris = faces[idx[cnt == 1]]
    order = np.lexsort((tris[:, 2], tris[:, 1], tris[:, 0]))
    tris = tris[order]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1)
    edges = np.unique(e, axis=0)
    verts = np.unique(tris.reshape(-1))
    return tris.astype(np.int32), edges.astype(np.int32), verts.astype(np.int32)


def merge_meshes(parts):
    """Concatenate (X, tets) parts into one mesh; returns X, tets, object_id."""
    Xs, Ts, ids = [], [], []
    off = 0
    for oid, (X, T) in enumerate(parts):
        Xs.append(X)
        Ts.append(np.asarray(T, dtype=np.int64) + off)
        ids.append(np.full(X.shape[0], oid, dtype=np.int32))
        off += X.shape[0]
    return (np.concatenate(Xs, 0), np.concatenate(Ts, 0).astype(np.int32),
            np.concatenate(ids, 0))
