"""The five benchmark scenes plus small test scenes (all seeded, synthetic).

Sizes and parameters:
  cube      6x6x6 cells of 1/60 m (0.1 m cube, 1296 tets, 343 vertices),
            E=1e5 Pa, nu=0.4, rho=1000, dropped from 0.05 m onto z=0,
            dhat=1e-3 m, kappa=1e4, h=1/60, vertex jitter 1e-4 m (seed 0)
  bar       40x8x8 cells of 0.01 m (15360 tets), E=5e5, nu=0.45, both end
            faces prescribed and counter-rotated (2*pi over 120 steps each),
            self contact (point-triangle + edge-edge), dhat=1e-3, h=1/30
  pile      24 voxelised shapes (12 spheres r~0.05, 12 tori R=0.06 r=0.02),
            ~110k tets, E log-uniform in [1e4,1e6], nu=0.4, dropped into a
            0.4 m box (5 half-spaces), dhat=5e-4, h=1/30 (seed 2)
  batched   256 cubes/bars with tet counts log-uniform in [500,8000]
            (seed 3), each over its own ground plane, h=1/60
  diff bar  50x10x10 cells of 0.01 m (30000 tets), per-tet log-normal E
            (median 1e5, sigma 0.5), ground contact, h=1/60 (seeds 4/5/6)
"""
from __future__ import annotations

import numpy as np

from .mesh import (Scene, hex_grid, surface_of, voxel_mesh, merge_meshes,
                   random_rotation, rotation_matrix)

GRAVITY = np.array([0.0, 0.0, -9.8])


def _scene(X, tets, *, E, nu, rho, x0=None, v0=None, planes=None, dhat, kappa,
           h, gravity=GRAVITY, object_id=None, fixed=None, self_contact=False,
           name="", iter_max=100, eps=1e-3, term="delta_e", cell=0.0, meta=None):
    T = tets.shape[0]
    V = X.shape[0]
    tris, edges, _ = surface_of(tets)
    bc = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), (T,)).copy()
    return Scene(
        X=np.ascontiguousarray(X, dtype=np.float64),
        tets=np.ascontiguousarray(tets, dtype=np.int32),
        tris=tris, edges=edges, E=bc(E), nu=bc(nu), rho=bc(rho),
        x0=np.ascontiguousarray(X if x0 is None else x0, dtype=np.float64).copy(),
        v0=np.zeros((V, 3)) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64),
        planes=np.zeros((0, 4)) if planes is None else np.asarray(planes, dtype=np.float64).reshape(-1, 4),
        dhat=float(dhat), kappa=float(kappa), h=float(h),
        gravity=np.asarray(gravity, dtype=np.float64),
        object_id=np.zeros(V, dtype=np.int32) if object_id is None else np.asarray(object_id, dtype=np.int32),
        fixed=np.zeros(0, dtype=np.int32) if fixed is None else np.asarray(fixed, dtype=np.int32),
        self_contact=self_contact, name=name, iter_max=iter_max, eps=eps,
        term=term, cell=cell, meta=meta or {})


def cube_scene(seed=0, n=6, side=0.1, drop=0.05):
    """Cube of n^3 cells x 6 tets, bottom at z=drop, over the plane z=0.

    Every vertex (rest and initial state alike) is jittered by U[-1e-4,1e-4]^3.
    """
    rng = np.random.default_rng(seed)
    X, tets = hex_grid(n, n, n, side / n, origin=(0.0, 0.0, drop))
    X = X + rng.uniform(-1e-4, 1e-4, size=X.shape)
    return _scene(X, tets, E=1e5, nu=0.4, rho=1000.0,
                  planes=[[0.0, 0.0, 1.0, 0.0]], dhat=1e-3, kappa=1e4,
                  h=1.0 / 60.0, name=f"cube{n}", iter_max=100, eps=1e-6,
                  term="grad_rel", cell=2e-3)


def twisted_bar_scene(nx=40, ny=8, nz=8, dx=0.01, steps_per_turn=120):
    """Bar along x with both end faces prescribed (twisted per ``twist_targets``)."""
    X, tets = hex_grid(nx, ny, nz, dx)
    L = nx * dx
    fixed = np.nonzero((X[:, 0] < 0.25 * dx) | (X[:, 0] > L - 0.25 * dx))[0].astype(np.int32)
    return _scene(X, tets, E=5e5, nu=0.45, rho=1000.0, dhat=1e-3, kappa=1e4,
                  h=1.0 / 30.0, gravity=np.zeros(3), fixed=fixed,
                  self_contact=True, name=f"bar{nx}x{ny}x{nz}", iter_max=150,
                  eps=1e-3, cell=2e-3,
                  meta={"center": np.array([0.0, ny * dx / 2, nz * dx / 2]),
                        "length": L, "steps_per_turn": steps_per_turn})


def stacked_bars_scene(gap=6e-4, angle=0.03, nx=40, ny=8, nz=8, dx=0.01):
    """Two copies of the twisted-bar mesh, the second one turned by ``angle``
    about the vertical axis and resting ``gap`` above the first: point-
    triangle and edge-edge barriers are active over the whole overlap (the
    self-contact state of the twist scene at its own scale, without the
    120 twist steps needed to reach it)."""
    Xa, Ta = hex_grid(nx, ny, nz, dx)
    Xb, Tb = hex_grid(nx, ny, nz, dx)
    c = np.array([nx * dx / 2, ny * dx / 2, 0.0])
    R = rotation_matrix([0.0, 0.0, 1.0], angle)
    Xb = (Xb - c) @ R.T + c + np.array([0.0, 0.0, nz * dx + gap])
    X, tets, oid = merge_meshes([(Xa, Ta), (Xb, Tb)])
    fixed = np.nonzero((oid == 0) & ((X[:, 0] < 0.25 * dx) | (X[:, 0] > nx * dx - 0.25 * dx)))[0].astype(np.int32)
    return _scene(X, tets, E=5e5, nu=0.45, rho=1000.0, dhat=1e-3, kappa=1e4,
                  h=1.0 / 30.0, fixed=fixed, object_id=oid, self_contact=True,
                  name="stackedbars", iter_max=150, eps=1e-3, cell=2e-3,
                  meta={"length": nx * dx})


def twist_targets(scene, step):
    """Prescribed positions of the bar's end faces at ``step`` (1-based):
    the end x=0 turns by +2*pi*step/steps_per_turn about the bar axis, the
    end x=L by the opposite angle."""
    c = scene.meta["center"]
    L = scene.meta["length"]
    ang = 2.0 * np.pi * step / scene.meta["steps_per_turn"]
    Xf = scene.X[scene.fixed]
    out = np.empty_like(Xf)
    for sgn, sel in ((+1.0, Xf[:, 0] < 0.5 * L), (-1.0, Xf[:, 0] >= 0.5 * L)):
        R = rotation_matrix([1.0, 0.0, 0.0], sgn * ang)
        r = Xf[sel] - c
        r[:, 0] = 0.0
        out[sel] = (r @ R.T) + c
        out[sel, 0] = Xf[sel, 0]
    return out


def _sphere_mask(r, pitch):
    n = int(np.ceil(2 * r / pitch)) + 1
    ctr = (np.arange(n) + 0.5) * pitch - n * pitch / 2
    gx, gy, gz = np.meshgrid(ctr, ctr, ctr, indexing="ij")
    return (gx ** 2 + gy ** 2 + gz ** 2) <= r * r, n * pitch / 2


def _torus_mask(R, r, pitch):
    nxy = int(np.ceil(2 * (R + r) / pitch)) + 1
    nz = int(np.ceil(2 * r / pitch)) + 1
    cxy = (np.arange(nxy) + 0.5) * pitch - nxy * pitch / 2
    cz = (np.arange(nz) + 0.5) * pitch - nz * pitch / 2
    gx, gy, gz = np.meshgrid(cxy, cxy, cz, indexing="ij")
    q = np.sqrt(gx ** 2 + gy ** 2) - R
    return (q ** 2 + gz ** 2) <= r * r, (nxy * pitch / 2, nxy * pitch / 2, nz * pitch / 2)


def _largest_component(mask):
    """Keep the face-connected component with most cells (voxelisation of a
    thin torus may leave stray cells)."""
    from scipy import ndimage
    lab, n = ndimage.label(mask)
    if n <= 1:
        return mask
    sizes = ndimage.sum(mask, lab, index=np.arange(1, n + 1))
    return lab == (1 + int(np.argmax(sizes)))


def _pile_masks(rng, pitch, n_shapes):
    masks = []
    for s in range(n_shapes):
        if s % 2 == 0:
            r = 0.05 * rng.uniform(0.9, 1.1)
            mask, half = _sphere_mask(r, pitch)
            half = np.array([half] * 3)
        else:
            mask, half = _torus_mask(0.06, 0.02, pitch)
            half = np.asarray(half)
        masks.append((_largest_component(mask), half))
    return masks


def _pile_pitch(seed, n_shapes, target_tets):
    """Voxel pitch at which the pile's shapes total target_tets (within 3 %),
    by bisection on the cell count."""
    def count(p):
        return 6 * sum(int(m.sum()) for m, _ in _pile_masks(np.random.default_rng(seed), p, n_shapes))
    lo, hi = 0.003, 0.02
    for _ in range(25):
        mid = 0.5 * (lo + hi)
        if count(mid) > target_tets:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def packed_pile_scene(seed=2, n_shapes=24, target_tets=110_000, box=0.4, gap_frac=0.3, dhat=5e-4):
    """A contact-rich state of the pile workload: the same 24 voxelised
    shapes (the pile's masks and pitch, so the same tet and vertex counts;
    interior vertices jittered by U[-0.1,0.1]*pitch), unrotated and stacked in
    four columns inside the 0.4 m box, each turned by a random angle about the
    vertical axis: spheres in two columns, tori (lying flat) in the other two.  Each shape rests on the one below, or on the
    floor, with a gap of gap_frac * dhat between the flat voxel facets that
    face each other, so every facing pair of facets has its vertices, edges
    and triangles within dhat: thousands of point-triangle and edge-edge
    pairs and the plane contacts of the bottom shapes are active in the rest
    state, which is also the start state (zero velocity).  E per shape is
    log-uniform in [1e4, 1e6], nu = 0.4; the other settings are the pile's."""
    pitch = _pile_pitch(seed, n_shapes, target_tets)
    masks = _pile_masks(np.random.default_rng(seed), pitch, n_shapes)
    rng = np.random.default_rng(seed + 1000)
    gap = gap_frac * dhat
    cols = {0: (0.1 * box / 0.4, 0.1 * box / 0.4), 1: (0.3 * box / 0.4, 0.1 * box / 0.4),
            2: (0.1 * box / 0.4, 0.3 * box / 0.4), 3: (0.3 * box / 0.4, 0.3 * box / 0.4)}
    top = {k: 0.0 for k in cols}
    parts, Es = [], []
    n_sph = n_tor = 0
    for s, (mask, half) in enumerate(masks):
        X, T = voxel_mesh(mask, pitch, origin=-np.asarray(half))
        _, _, sv = surface_of(T)
        interior = np.setdiff1d(np.arange(X.shape[0]), sv)
        X[interior] += rng.uniform(-0.1 * pitch, 0.1 * pitch, size=(interior.size, 3))
        # a random turn about the vertical axis: facets stay horizontal, but
        # the lattices of facing facets no longer line up vertex on vertex
        X = X @ rotation_matrix([0.0, 0.0, 1.0], rng.uniform(0.0, 0.5 * np.pi)).T
        if s % 2 == 0:          # spheres: columns 0 and 3
            col = 0 if n_sph % 2 == 0 else 3
            n_sph += 1
        else:                   # tori: columns 1 and 2
            col = 1 if n_tor % 2 == 0 else 2
            n_tor += 1
        cx, cy = cols[col]
        z0 = top[col] + gap
        X = X + np.array([cx, cy, z0 - X[:, 2].min()])
        top[col] = float(X[:, 2].max())
        parts.append((X, T))
        Es.append(float(np.exp(rng.uniform(np.log(1e4), np.log(1e6)))))
    X, tets, oid = merge_meshes(parts)
    E = np.concatenate([np.full(T.shape[0], e) for (_, T), e in zip(parts, Es)])
    planes = np.array([[0, 0, 1, 0.0], [1, 0, 0, 0.0], [-1, 0, 0, -box],
                       [0, 1, 0, 0.0], [0, -1, 0, -box]], dtype=np.float64)
    return _scene(X, tets, E=E, nu=0.4, rho=1000.0, planes=planes, dhat=dhat,
                  kappa=1e4, h=1.0 / 30.0, object_id=oid, self_contact=True,
                  name="pile-packed", iter_max=25, eps=1e-3, cell=0.0,
                  meta={"pitch": pitch, "n_shapes": n_shapes, "gap": gap})


def pile_scene(seed=2, n_shapes=24, target_tets=110_000, pitch=None, box=0.4,
               gap=2e-3):
    """Voxelised spheres and tori stacked in a box of side ``box``.

    The pitch is tuned (bisection on the cell count) so the total tet count
    is within 3% of ``target_tets``.  Interior vertices of each shape are
    jittered by U[-0.1,0.1]*pitch per axis; each shape gets a uniform random
    rotation and is dropped at the lowest height where a random footprint
    position keeps its bounding sphere ``gap`` away from the floor and from
    every shape already placed, so shapes meet the floor and each other within
    a few frames.  E per shape is log-uniform in [1e4, 1e6]; nu=0.4.
    """
    if pitch is None:
        pitch = _pile_pitch(seed, n_shapes, target_tets)
    rng = np.random.default_rng(seed)
    masks = _pile_masks(rng, pitch, n_shapes)
    placed = []
    out_parts = []
    Es = []
    for mask, half in masks:
        X, T = voxel_mesh(mask, pitch, origin=-half)
        X = X - X.mean(axis=0)
        _, _, sv = surface_of(T)
        interior = np.setdiff1d(np.arange(X.shape[0]), sv)
        X[interior] += rng.uniform(-0.1 * pitch, 0.1 * pitch, size=(interior.size, 3))
        X = X @ random_rotation(rng).T
        rad = float(np.max(np.linalg.norm(X, axis=1)))
        zc = rad + gap
        c = None
        while c is None:
            for _ in range(64):
                cand = np.array([rng.uniform(rad + gap, box - rad - gap),
                                 rng.uniform(rad + gap, box - rad - gap), zc])
                if all(np.linalg.norm(cand - pc) > rad + pr + gap for pc, pr in placed):
                    c = cand
                    break
            zc += 0.1 * rad
        placed.append((c, rad))
        out_parts.append((X + c, T))
        Es.append(float(np.exp(rng.uniform(np.log(1e4), np.log(1e6)))))
    X, tets, oid = merge_meshes(out_parts)
    E = np.concatenate([np.full(T.shape[0], e) for (_, T), e in zip(out_parts, Es)])
    planes = np.array([[0, 0, 1, 0.0], [1, 0, 0, 0.0], [-1, 0, 0, -box],
                       [0, 1, 0, 0.0], [0, -1, 0, -box]], dtype=np.float64)
    return _scene(X, tets, E=E, nu=0.4, rho=1000.0, planes=planes, dhat=5e-4,
                  kappa=1e4, h=1.0 / 30.0, object_id=oid, self_contact=True,
                  name="pile", iter_max=25, eps=1e-3, cell=0.0,
                  meta={"pitch": pitch, "n_shapes": n_shapes})


def batched_scenes(seed=3, n_scenes=256, t_lo=500, t_hi=8000, drop=0.05):
    """Independent cubes or bars (50/50) with log-uniform tet counts, each
    dropped ``drop`` metres onto its own plane z=0."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        T = float(np.exp(rng.uniform(np.log(t_lo), np.log(t_hi))))
        E = float(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
        if rng.uniform() < 0.5:
            n = max(2, int(round((T / 6.0) ** (1.0 / 3.0))))
            dims = (n, n, n)
        else:
            k = max(1, int(round((T / 24.0) ** (1.0 / 3.0))))
            dims = (4 * k, k, k)
        dx = 0.1 / max(dims)
        X, tets = hex_grid(*dims, dx, origin=(0.0, 0.0, drop))
        out.append(_scene(X, tets, E=E, nu=0.4, rho=1000.0,
                          planes=[[0.0, 0.0, 1.0, 0.0]], dhat=1e-3, kappa=1e4,
                          h=1.0 / 60.0, name=f"batch{s}", iter_max=100, eps=1e-3,
                          cell=2e-3))
    return out


def pack_batch(scs, x=None, v=None):
    """Concatenate scenes for the batched entry points: per-scene offsets,
    scene-local indices, one plane row per scene (zero normal if none).
    ``x``/``v`` (lists of per-scene states, default x0/v0) are stacked too."""
    nv = [s.nV for s in scs]
    nt = [s.nT for s in scs]
    nf = [len(s.tris) for s in scs]
    planes = np.zeros((len(scs), 4))
    for i, s in enumerate(scs):
        if len(s.planes) > 1:
            raise ValueError("a batched scene has at most one plane")
        if len(s.planes):
            planes[i] = s.planes[0]
    cat = lambda arrs, shape: (np.concatenate(arrs) if arrs else np.zeros(shape))
    return dict(
        vert_off=np.concatenate([[0], np.cumsum(nv)]).astype(np.int32),
        tet_off=np.concatenate([[0], np.cumsum(nt)]).astype(np.int32),
        tri_off=np.concatenate([[0], np.cumsum(nf)]).astype(np.int32),
        X=cat([s.X for s in scs], (0, 3)),
        tets=cat([s.tets for s in scs], (0, 4)).astype(np.int32),
        tris=cat([s.tris for s in scs], (0, 3)).astype(np.int32),
        E=cat([np.broadcast_to(s.E, (s.nT,)) for s in scs], (0,)),
        nu=cat([np.broadcast_to(s.nu, (s.nT,)) for s in scs], (0,)),
        rho=cat([np.broadcast_to(s.rho, (s.nT,)) for s in scs], (0,)),
        planes=planes,
        x=cat([s.x0 for s in scs] if x is None else list(x), (0, 3)),
        v=cat([s.v0 for s in scs] if v is None else list(v), (0, 3)),
    )


def diff_bar_scene(seed=4, nx=50, ny=10, nz=10, dx=0.01, lift=0.01, gtol=1e-10):
    """Bar whose per-tet Young's modulus is E = 1e5 * exp(0.5 z), z ~ N(0,1),
    starting ``lift`` metres above the ground plane.  Steps are converged to
    an absolute gradient norm of ``gtol`` times the gravity impulse scale
    h^2 |g| rho dx^3 sqrt(nV) (a node's weight impulse, 2-norm over the
    nodes): once the bar rests on the floor, ||g_0|| of a step is itself only
    a few orders above the gradient's rounding floor, so a rule relative to
    ||g_0|| cannot be met."""
    rng = np.random.default_rng(seed)
    X, tets = hex_grid(nx, ny, nz, dx, origin=(0.0, 0.0, lift))
    E = 1e5 * np.exp(0.5 * rng.standard_normal(tets.shape[0]))
    h = 1.0 / 60.0
    scale = h * h * 9.8 * 1000.0 * dx ** 3 * np.sqrt(X.shape[0])
    return _scene(X, tets, E=E, nu=0.4, rho=1000.0,
                  planes=[[0.0, 0.0, 1.0, 0.0]], dhat=1e-3, kappa=1e4,
                  h=h, name=f"diffbar{nx}x{ny}x{nz}", iter_max=20000,
                  eps=gtol * scale, term="grad_abs", cell=2e-3)


def small_contact_scene(seed=7, n=3, gap=4e-4, dhat=1e-3):
    """Two small cubes stacked with a sub-dhat gap and a twist, plus a ground
    plane: exercises point-triangle, edge-edge and plane barriers at once."""
    rng = np.random.default_rng(seed)
    side = 0.03
    Xa, Ta = hex_grid(n, n, n, side / n, origin=(0.0, 0.0, 5e-4))
    Xb, Tb = hex_grid(n, n, n, side / n)
    R = rotation_matrix([0.0, 0.0, 1.0], 0.3)
    ctr = np.array([side / 2, side / 2, 0.0])
    Xb = (Xb - ctr) @ R.T + ctr + np.array([0.004, -0.003, 5e-4 + side + gap])
    X, tets, oid = merge_meshes([(Xa, Ta), (Xb, Tb)])
    X = X + rng.uniform(-2e-5, 2e-5, size=X.shape)
    return _scene(X, tets, E=2e5, nu=0.4, rho=1000.0,
                  planes=[[0.0, 0.0, 1.0, 0.0]], dhat=dhat, kappa=1e4,
                  h=1.0 / 60.0, object_id=oid, self_contact=True,
                  name="stack2", iter_max=200, eps=1e-6, cell=4e-3)


def tiny_scene(seed=11, n=2, dx=0.02):
    """A single n^3-cell block with jittered rest shape, no contact."""
    rng = np.random.default_rng(seed)
    X, tets = hex_grid(n, n, n, dx, origin=(0.0, 0.0, 0.1))
    X = X + rng.uniform(-0.1 * dx, 0.1 * dx, size=X.shape)
    return _scene(X, tets, E=1e5, nu=0.4, rho=1000.0, dhat=1e-3, kappa=1e4,
                  h=1.0 / 60.0, name=f"tiny{n}", iter_max=100, eps=1e-8)
