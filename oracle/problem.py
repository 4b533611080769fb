"""The incremental potential and its derivatives (Sec. 3, equations E and
Hessian), assembled on the CPU in float64.

    E(x) = 1/2 (x - xt)^T M (x - xt) + h^2 Psi(x) + kappa sum_k b(d_k(x))

Contact terms (Sec. 3.2):
  * PT / EE pairs: t = sum_i c_i x_i with c held fixed (dt/dx = [c_i I3],
    d2t/dx2 = 0).  Gradient kappa b'(d)/d * c_i t (equation eq8).  Hessian
    (equation eq9):
        (b''/d^2 - b'/d^3) (J t)(J t)^T + (b'/d) J J^T,   J = dt/dx.
    Reading: because b' < 0 on (0, dhat) the second term is negative
    semidefinite and makes diagonal entries negative close to contact, which
    the Jacobi preconditioner cannot use; by default ("psd") the 3x3 Hessian
    in t-space, b'' n n^T + (b'/d)(I - n n^T), is projected onto the PSD cone,
    i.e. only (b''/d^2)(J t)(J t)^T is kept.  barrier_mode="full" keeps the
    equation verbatim (used for finite-difference tests).
  * Planes n.x >= o (not in the paper; the scenes need a floor and walls):
    d = n.x_v - o for surface vertices, gradient kappa b'(d) n, Hessian
    kappa b''(d) n n^T (exact).
  * Active iff 0 < d < dhat; d <= 0 on an active candidate is a penetration
    error.  kappa is not multiplied by h^2 (equation E as written).
Prescribed vertices: their rows of the gradient are zero and their diagonal
entries one; p^T H p and H v see p = 0 there.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import barrier, candidates, distance, elastic


class Penetration(ValueError):
    pass


@dataclasses.dataclass
class ActiveSet:
    kind: np.ndarray      # (A,) 0 = PT, 1 = EE
    idx: np.ndarray       # (A,4) vertex indices (x0..x3)
    c: np.ndarray         # (A,4)
    t: np.ndarray         # (A,3)
    d: np.ndarray         # (A,)
    pv: np.ndarray        # (P,) plane contacts: vertex
    pk: np.ndarray        # (P,) plane index
    pd: np.ndarray        # (P,) distance


class Problem:
    """Mesh, material and contact parameters of one scene (all float64)."""

    def __init__(self, X, tets, tris, edges, E, nu, rho, planes, dhat, kappa,
                 self_contact=False, fixed=None, barrier_mode="psd",
                 rest_exclude=True, gravity=(0.0, 0.0, -9.8), object_id=None, model="nh", ties="first"):
        self.X = np.asarray(X, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
        self.nV = self.X.shape[0]
        self.Bmat, self.vol = elastic.rest_setup(self.X, self.tets)
        self.b = elastic.shape_vectors(self.Bmat)
        self.rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), self.vol.shape).copy()
        self.set_material(E, nu)
        self.set_model(model)
        self.mass = elastic.lumped_mass(self.vol, self.rho, self.tets, self.nV)
        self.planes = np.asarray(planes, dtype=np.float64).reshape(-1, 4)
        self.dhat = float(dhat)
        self.kappa = float(kappa)
        self.self_contact = bool(self_contact)
        self.fixed = np.zeros(0, np.int64) if fixed is None else np.asarray(fixed, dtype=np.int64)
        self.free = np.ones(self.nV, dtype=bool)
        self.free[self.fixed] = False
        self.barrier_mode = barrier_mode
        self.ties = ties          # closest points on exact ties (see distance)
        self.gravity = np.asarray(gravity, dtype=np.float64)
        self.surf_verts = np.unique(self.tris.reshape(-1)) if len(self.tris) else np.zeros(0, np.int64)
        self.object_id = (np.zeros(self.nV, np.int64) if object_id is None
                          else np.asarray(object_id, dtype=np.int64).reshape(self.nV))
        self._override = None
        if self.self_contact and rest_exclude:
            self.excl_pt, self.excl_ee = candidates.rest_exclusion(
                self.X, self.tris, self.edges, self.surf_verts, self.dhat, object_id)
        else:
            self.excl_pt = self.excl_ee = np.zeros(0, np.int64)

    @classmethod
    def from_scene(cls, sc, **kw):
        args = dict(self_contact=sc.self_contact, fixed=sc.fixed, gravity=sc.gravity,
                    object_id=sc.object_id)
        args.update(kw)
        return cls(sc.X, sc.tets, sc.tris, sc.edges, sc.E, sc.nu, sc.rho,
                   sc.planes, sc.dhat, sc.kappa, **args)

    def set_material(self, E, nu):
        self.E = np.broadcast_to(np.asarray(E, dtype=np.float64), self.vol.shape).copy()
        self.nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), self.vol.shape).copy()
        self.mu, self.lam = elastic.lame(self.E, self.nu)

    def set_model(self, model):
        """Elastic density: one of elastic.MODELS (Sec. 3.1, Table 1)."""
        if model not in elastic.MODELS:
            raise ValueError(f"unknown material model {model!r}")
        self.model = model

    @property
    def has_collision_primitives(self):
        return len(self.planes) > 0 or (self.self_contact and len(self.tris) > 0)

    # ------------------------------------------------------------------ sets
    def candidate_lists(self, x, r=None):
        r = self.dhat if r is None else r
        pt = ee = np.zeros((0, 2), np.int32)
        if self.self_contact:
            pt = candidates.pt_candidates(x, self.tris, self.surf_verts, r, self.excl_pt)
            ee = candidates.ee_candidates(x, self.edges, r, self.excl_ee)
        pg = candidates.pg_candidates(x, self.surf_verts, self.planes, r)
        return pt, ee, pg

    def set_candidates_override(self, pt=None, ee=None):
        """Explicit point-triangle (v, f) and edge-edge (e1, e2) candidate
        lists for active_set in place of the AABB lists (the library's test
        hook for ComputeConstraintSet, Algorithm 1); a list left None is empty
        while the other is given, and both None restore the AABB lists.  The
        distance test 0 < d < dhat still selects the active pairs."""
        if pt is None and ee is None:
            self._override = None
            return
        pt = np.zeros((0, 2), np.int64) if pt is None else np.asarray(pt, dtype=np.int64).reshape(-1, 2)
        ee = np.zeros((0, 2), np.int64) if ee is None else np.sort(np.asarray(ee, dtype=np.int64).reshape(-1, 2), axis=1)
        self._override = (pt, ee)

    def active_set(self, x):
        """ComputeConstraintSet (Algorithm 1): candidates, closest points, and
        the pairs with 0 < d < dhat."""
        x = np.asarray(x, dtype=np.float64)
        pt, ee, pg = self.candidate_lists(x)
        if self._override is not None and self.self_contact:
            pt, ee = self._override
        kinds, idxs, cs, ts, ds = [], [], [], [], []
        if len(pt):
            f = self.tris[pt[:, 1]]
            idx = np.stack([pt[:, 0], f[:, 0], f[:, 1], f[:, 2]], axis=1).astype(np.int64)
            c, t, d = distance.point_triangle(*(x[idx[:, i]] for i in range(4)), ties=self.ties)
            kinds.append(np.zeros(len(d), np.int64)); idxs.append(idx); cs.append(c); ts.append(t); ds.append(d)
        if len(ee):
            ea, eb = self.edges[ee[:, 0]], self.edges[ee[:, 1]]
            idx = np.stack([ea[:, 0], ea[:, 1], eb[:, 0], eb[:, 1]], axis=1).astype(np.int64)
            c, t, d = distance.edge_edge(*(x[idx[:, i]] for i in range(4)), ties=self.ties)
            kinds.append(np.ones(len(d), np.int64)); idxs.append(idx); cs.append(c); ts.append(t); ds.append(d)
        if kinds:
            kind = np.concatenate(kinds); idx = np.concatenate(idxs); c = np.concatenate(cs)
            t = np.concatenate(ts); d = np.concatenate(ds)
        else:
            kind = np.zeros(0, np.int64); idx = np.zeros((0, 4), np.int64); c = np.zeros((0, 4))
            t = np.zeros((0, 3)); d = np.zeros(0)
        if np.any(d <= 0):
            raise Penetration(f"{int(np.sum(d <= 0))} pairs with d <= 0")
        act = d < self.dhat
        pv, pk = pg[:, 0].astype(np.int64), pg[:, 1].astype(np.int64)
        pd = np.zeros(len(pv))
        for k in range(len(self.planes)):
            sel = pk == k
            pd[sel] = candidates.plane_signed(x[pv[sel]], self.planes[k])
        if np.any(pd <= 0):
            raise Penetration(f"{int(np.sum(pd <= 0))} vertices on or behind a plane")
        pact = pd < self.dhat
        return ActiveSet(kind[act], idx[act], c[act], t[act], d[act], pv[pact], pk[pact], pd[pact])

    # --------------------------------------------------------------- pieces
    def _F(self, x):
        F = elastic.deformation_gradient(x, self.tets, self.Bmat)
        if self.model == "nh" and np.any(np.linalg.det(F) <= 0):
            raise elastic.InvertedElement("inverted element")
        return F

    def _scatter(self, per_elem, idx):
        """Sum (n,k,3) contributions into (V,3) by vertex index (n,k)."""
        out = np.zeros((self.nV, 3))
        for a in range(idx.shape[1]):
            for j in range(3):
                out[:, j] += np.bincount(idx[:, a], weights=per_elem[:, a, j], minlength=self.nV)
        return out

    def predictor(self, x_t, v_t, h):
        """xt = x^t + h v^t + h^2 M^{-1} f_ext with f_ext = m g (Sec. 3)."""
        return np.asarray(x_t) + h * np.asarray(v_t) + h * h * self.gravity[None, :]

    def energy(self, x, xt, h, aset=None):
        aset = self.active_set(x) if aset is None else aset
        dx = x - xt
        Ein = 0.5 * np.sum(self.mass[:, None] * dx * dx)
        Eel = h * h * np.sum(elastic.element_energy(self._F(x), self.vol, self.mu, self.lam, self.model))
        Eb = self.kappa * (np.sum(barrier.b(aset.d, self.dhat)) + np.sum(barrier.b(aset.pd, self.dhat)))
        return Ein + Eel + Eb

    def gradient(self, x, xt, h, aset=None, project=True):
        aset = self.active_set(x) if aset is None else aset
        g = self.mass[:, None] * (x - xt)
        ge = elastic.element_gradient(self._F(x), self.b, self.vol, self.mu, self.lam, self.model)
        g += h * h * self._scatter(ge, self.tets)
        if len(aset.d):
            coef = self.kappa * barrier.db(aset.d, self.dhat) / aset.d
            gc = coef[:, None, None] * aset.c[:, :, None] * aset.t[:, None, :]
            g += self._scatter(gc, aset.idx)
        if len(aset.pd):
            coef = self.kappa * barrier.db(aset.pd, self.dhat)
            gp = coef[:, None] * self.planes[aset.pk, :3]
            g += self._scatter(gp[:, None, :], aset.pv[:, None])
        if project:
            g[~self.free] = 0.0
        return g

    def _contact_blocks(self, aset, mode=None):
        """Per-pair 12x12 barrier Hessians kappa * d2b/dx2 (fixed c)."""
        mode = self.barrier_mode if mode is None else mode
        d = aset.d
        b1 = barrier.db(d, self.dhat)
        b2 = barrier.d2b(d, self.dhat)
        Jt = (aset.c[:, :, None] * aset.t[:, None, :]).reshape(-1, 12)
        JJ = np.einsum("na,nb->nab", aset.c, aset.c)
        JJ = np.einsum("nab,ij->naibj", JJ, np.eye(3)).reshape(-1, 12, 12)
        if mode == "psd":
            H = (b2 / d ** 2)[:, None, None] * np.einsum("ni,nj->nij", Jt, Jt)
        else:
            H = (b2 / d ** 2 - b1 / d ** 3)[:, None, None] * np.einsum("ni,nj->nij", Jt, Jt) \
                + (b1 / d)[:, None, None] * JJ
        return self.kappa * H

    def element_hessians(self, x, h):
        return h * h * elastic.element_hessian(self._F(x), self.b, self.vol, self.mu, self.lam, self.model)

    def diag(self, x, h, aset=None, mode=None):
        """diag(H) (V,3); prescribed rows are 1."""
        aset = self.active_set(x) if aset is None else aset
        D = np.repeat(self.mass[:, None], 3, axis=1).astype(np.float64)
        He = self.element_hessians(x, h)
        D += self._scatter(np.einsum("tii->ti", He).reshape(-1, 4, 3), self.tets)
        if len(aset.d):
            Hc = self._contact_blocks(aset, mode)
            D += self._scatter(np.einsum("nii->ni", Hc).reshape(-1, 4, 3), aset.idx)
        if len(aset.pd):
            n = self.planes[aset.pk, :3]
            dp = (self.kappa * barrier.d2b(aset.pd, self.dhat))[:, None] * n * n
            D += self._scatter(dp[:, None, :], aset.pv[:, None])
        D[~self.free] = 1.0
        return D

    def pHp(self, x, p, h, aset=None, mode=None):
        """p^T H p (p is zeroed on prescribed vertices first)."""
        return float(np.sum(self.hvp(x, p, h, aset, mode) * self._mask(p)))

    def _mask(self, p):
        p = np.array(p, dtype=np.float64, copy=True)
        p[~self.free] = 0.0
        return p

    def hvp(self, x, p, h, aset=None, mode=None):
        """H p (V,3) with p zeroed on prescribed vertices; prescribed rows of
        the result are zero."""
        aset = self.active_set(x) if aset is None else aset
        p = self._mask(p)
        out = self.mass[:, None] * p
        He = self.element_hessians(x, h)
        pe = p[self.tets].reshape(-1, 12)
        out += self._scatter(np.einsum("tij,tj->ti", He, pe).reshape(-1, 4, 3), self.tets)
        if len(aset.d):
            Hc = self._contact_blocks(aset, mode)
            pc = p[aset.idx].reshape(-1, 12)
            out += self._scatter(np.einsum("nij,nj->ni", Hc, pc).reshape(-1, 4, 3), aset.idx)
        if len(aset.pd):
            n = self.planes[aset.pk, :3]
            s = (self.kappa * barrier.d2b(aset.pd, self.dhat)) * np.einsum("ni,ni->n", n, p[aset.pv])
            out += self._scatter((s[:, None] * n)[:, None, :], aset.pv[:, None])
        out[~self.free] = 0.0
        return out

    def hessian_matrix(self, x, h, aset=None, mode=None):
        """Assembled sparse H (3V x 3V); prescribed rows/columns replaced by
        the identity."""
        aset = self.active_set(x) if aset is None else aset
        rows, cols, vals = [], [], []
        He = self.element_hessians(x, h)
        dof = (3 * self.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows.append(np.repeat(dof, 12, axis=1).ravel()); cols.append(np.tile(dof, (1, 12)).ravel())
        vals.append(He.ravel())
        if len(aset.d):
            Hc = self._contact_blocks(aset, mode)
            dofc = (3 * aset.idx[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
            rows.append(np.repeat(dofc, 12, axis=1).ravel()); cols.append(np.tile(dofc, (1, 12)).ravel())
            vals.append(Hc.ravel())
        if len(aset.pd):
            n = self.planes[aset.pk, :3]
            s = self.kappa * barrier.d2b(aset.pd, self.dhat)
            Hp = s[:, None, None] * np.einsum("ni,nj->nij", n, n)
            dofp = 3 * aset.pv[:, None] + np.arange(3)[None, :]
            rows.append(np.repeat(dofp, 3, axis=1).ravel()); cols.append(np.tile(dofp, (1, 3)).ravel())
            vals.append(Hp.ravel())
        m3 = np.repeat(self.mass, 3)
        rows.append(np.arange(3 * self.nV)); cols.append(np.arange(3 * self.nV)); vals.append(m3)
        H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(3 * self.nV, 3 * self.nV)).tocsr()
        if len(self.fixed):
            keep = np.repeat(self.free, 3).astype(np.float64)
            Dk = sp.diags(keep)
            H = Dk @ H @ Dk + sp.diags(1.0 - keep)
        return H

    def min_distance(self, x):
        """Smallest distance over all non-excluded PT/EE pairs within a wide
        radius and all surface-vertex/plane pairs, and the smallest det F
        (penetration audit, Sec. 6)."""
        x = np.asarray(x, dtype=np.float64)
        dmin = np.inf
        r = 10 * self.dhat
        pt, ee, _ = self.candidate_lists(x, r)
        if len(pt):
            f = self.tris[pt[:, 1]]
            _, _, d = distance.point_triangle(x[pt[:, 0]], x[f[:, 0]], x[f[:, 1]], x[f[:, 2]])
            dmin = min(dmin, float(d.min()))
        if len(ee):
            ea, eb = self.edges[ee[:, 0]], self.edges[ee[:, 1]]
            _, _, d = distance.edge_edge(x[ea[:, 0]], x[ea[:, 1]], x[eb[:, 0]], x[eb[:, 1]])
            dmin = min(dmin, float(d.min()))
        for pl in self.planes:
            if len(self.surf_verts):
                dmin = min(dmin, float(candidates.plane_signed(x[self.surf_verts], pl).min()))
        F = elastic.deformation_gradient(x, self.tets, self.Bmat)
        return dmin, float(np.linalg.det(F).min())
