"""ctypes binding of libpncg (include/pncg.h): argument marshalling only.

Every function here converts NumPy arrays (or torch CUDA tensors for the
``*_dev`` entry points) to the pointers and sizes of the C ABI and raises
``PncgError`` on a negative status.  All computation happens in the HIP
library; if it is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpncg.so")

OK, W_MAXITER = 0, 1
E_INVAL, E_NOMEM, E_HIP, E_STATE = -1, -2, -3, -4
E_PENETRATION, E_INVERTED, E_NONFINITE, E_CAPACITY, E_INDEFINITE = -5, -6, -7, -8, -9
FP64, MIXED = 0, 1
TERM_DELTA_E, TERM_GRAD_REL, TERM_GRAD_ABS = 0, 1, 2
BARRIER_FULL, ALPHA_INF_COMPONENT = 1, 2
BETA_DK, BETA_FR, BETA_PRP, BETA_CD, BETA_HZ = 0, 1 << 4, 2 << 4, 3 << 4, 4 << 4
BETA_RULES = {"dk": BETA_DK, "fr": BETA_FR, "prp": BETA_PRP, "cd": BETA_CD, "hz": BETA_HZ}
SPLIT_OBJECTS = 1 << 8
MODEL_NH, MODEL_SNH, MODEL_ARAP, MODEL_FCR = 0, 1, 2, 3
MODELS = {"nh": MODEL_NH, "snh": MODEL_SNH, "arap": MODEL_ARAP, "fcr": MODEL_FCR}
CONTACT_SELF, CONTACT_REST_EXCLUDE = 1, 2
KIND_PT, KIND_EE, KIND_PG = 0, 1, 2
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_SEGMENTED = 0, 1, 2
NOALLOC_ITER_MAX = 9566

CODE_NAMES = {0: "OK", 1: "W_MAXITER", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_HIP", -4: "E_STATE",
              -5: "E_PENETRATION", -6: "E_INVERTED", -7: "E_NONFINITE", -8: "E_CAPACITY", -9: "E_INDEFINITE"}
EXPORTS = ("pncg_create", "pncg_destroy", "pncg_last_error", "pncg_set_mesh", "pncg_set_material",
           "pncg_set_contact", "pncg_set_solver", "pncg_set_dirichlet", "pncg_step", "pncg_step_dev",
           "pncg_energy", "pncg_gradient", "pncg_hvp", "pncg_candidates", "pncg_solver_pairs", "pncg_min_distance",
           "pncg_set_profiling", "pncg_get_profile", "pncg_adjoint_step", "pncg_adjoint_step_dev",
           "pncg_set_tuning", "pncg_mean_boundary_edge", "pncg_set_adjoint_warm_start",
           "pncg_batch_create", "pncg_batch_destroy", "pncg_batch_last_error", "pncg_batch_set_params",
           "pncg_batch_set_block", "pncg_batch_step", "pncg_batch_run", "pncg_batch_stats",
           "pncg_batch_autotune", "pncg_batch_set_staging", "pncg_batch_get_config",
           "pncg_batch_set_split", "pncg_set_model", "pncg_batch_set_model", "pncg_run_dev",
           "pncg_set_candidates_override", "pncg_step_dev_noalloc")
PROF_KINDS = ("narrow", "grad", "dir", "rebuild", "predict")


class PncgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class pncg_opts(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32), ("stream", C.c_void_p),
                ("scatter", C.c_int32), ("chunk", C.c_int32), ("graphs", C.c_int32)]


class pncg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reason", C.c_int32), ("dE0", C.c_double), ("last_dE", C.c_double),
                ("g0_norm", C.c_double), ("g_norm", C.c_double), ("alpha_upper_hits", C.c_int32),
                ("rebuilds", C.c_int32), ("n_candidates", C.c_int64), ("n_active", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pncg_adjoint_stats(C.Structure):
    _fields_ = [("cg_iters", C.c_int32), ("reason", C.c_int32), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2405_08001_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32
    sig = {
        "pncg_create": (I32, [C.POINTER(P), C.POINTER(pncg_opts)]),
        "pncg_destroy": (None, [P]),
        "pncg_last_error": (C.c_char_p, [P]),
        "pncg_set_mesh": (I32, [P, I32, P, I32, P, I32, P, I32, P, P]),
        "pncg_set_material": (I32, [P, P, P, P]),
        "pncg_set_contact": (I32, [P, D, D, D, I32, P, U32]),
        "pncg_set_solver": (I32, [P, I32, D, I32, P, U32]),
        "pncg_set_dirichlet": (I32, [P, I32, P, P]),
        "pncg_set_tuning": (I32, [P, D, I32]),
        "pncg_set_candidates_override": (I32, [P, I32, C.c_int64, P]),
        "pncg_step_dev_noalloc": (I32, [P, P, P, D, P, P, C.POINTER(pncg_stats)]),
        "pncg_set_model": (I32, [P, I32]),
        "pncg_batch_set_model": (I32, [P, I32]),
        "pncg_mean_boundary_edge": (I32, [P, P]),
        "pncg_set_adjoint_warm_start": (I32, [P, I32]),
        "pncg_step": (I32, [P, P, P, D, P, P, C.POINTER(pncg_stats)]),
        "pncg_step_dev": (I32, [P, P, P, D, P, P, C.POINTER(pncg_stats)]),
        "pncg_run_dev": (I32, [P, P, P, D, I32, P]),
        "pncg_energy": (I32, [P, P, P, D, P]),
        "pncg_gradient": (I32, [P, P, P, D, P, P]),
        "pncg_hvp": (I32, [P, P, P, D, P, P]),
        "pncg_candidates": (I32, [P, P, I32, P, I64, C.POINTER(I64)]),
        "pncg_solver_pairs": (I32, [P, P, I32, P, I64, C.POINTER(I64)]),
        "pncg_min_distance": (I32, [P, P, P, P]),
        "pncg_set_profiling": (I32, [P, I32]),
        "pncg_get_profile": (I32, [P, P, P]),
        "pncg_adjoint_step": (I32, [P, P, D, P, P, D, I32, P, P, P, C.POINTER(pncg_adjoint_stats)]),
        "pncg_adjoint_step_dev": (I32, [P, P, D, P, P, D, I32, P, P, P, C.POINTER(pncg_adjoint_stats)]),
        "pncg_batch_create": (I32, [C.POINTER(P), C.POINTER(pncg_opts), I32, P, P, P, P, P, P, P, P, P, P]),
        "pncg_batch_destroy": (None, [P]),
        "pncg_batch_last_error": (C.c_char_p, [P]),
        "pncg_batch_set_params": (I32, [P, D, D, I32, D, I32, P, U32]),
        "pncg_batch_set_block": (I32, [P, I32]),
        "pncg_batch_step": (I32, [P, P, P, D, P, P]),
        "pncg_batch_run": (I32, [P, P, P, D, I32]),
        "pncg_batch_stats": (I32, [P, P, P, P]),
        "pncg_batch_autotune": (I32, [P, P, P, D, I32, P]),
        "pncg_batch_set_staging": (I32, [P, I32]),
        "pncg_batch_get_config": (I32, [P, P, P, P, P]),
        "pncg_batch_set_split": (I32, [P, I32, I32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_L = _load()


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """One libpncg context (a device, a precision, a mesh)."""

    def __init__(self, device=0, precision=FP64, stream=None, chunk=0, scatter=SCATTER_AUTO, graphs=True):
        opts = pncg_opts(device, precision, stream, scatter, chunk, 0 if graphs else 1)
        self._stream = int(stream or 0)
        h = C.c_void_p()
        rc = _L.pncg_create(C.byref(h), C.byref(opts))
        if rc < 0:
            raise PncgError(rc, _L.pncg_last_error(None).decode())
        self._h = h
        self.precision = precision
        self.nV = 0
        self.nT = 0

    def close(self):
        if getattr(self, "_h", None) and _L is not None:   # _L is None at interpreter exit
            _L.pncg_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise PncgError(rc, _L.pncg_last_error(self._h).decode())
        return rc

    # -------------------------------------------------------------- setup
    def pncg_set_mesh(self, X, tets, tris=None, edges=None, object_id=None):
        X = _f64(X)
        tets = _i32(tets)
        tris = _i32(np.zeros((0, 3)) if tris is None else tris)
        edges = _i32(np.zeros((0, 2)) if edges is None else edges)
        oid = None if object_id is None else _i32(object_id)
        self._check(_L.pncg_set_mesh(self._h, X.shape[0], _ptr(X), tets.shape[0], _ptr(tets),
                                     tris.shape[0], _ptr(tris), edges.shape[0], _ptr(edges), _ptr(oid)))
        self.nV = X.shape[0]
        self.nT = tets.shape[0]

    def pncg_set_material(self, E, nu, rho):
        n = max(self.nT, np.size(E))
        E, nu, rho = (_f64(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,))) for a in (E, nu, rho))
        self._check(_L.pncg_set_material(self._h, _ptr(E), _ptr(nu), _ptr(rho)))

    def pncg_set_model(self, model):
        """model: a MODEL_* value or one of the names in MODELS."""
        self._check(_L.pncg_set_model(self._h, _model_code(model)))

    def pncg_set_contact(self, dhat, kappa, cell=0.0, planes=None, flags=0):
        pl = _f64(np.zeros((0, 4)) if planes is None else np.asarray(planes, dtype=np.float64).reshape(-1, 4))
        self._check(_L.pncg_set_contact(self._h, float(dhat), float(kappa), float(cell), pl.shape[0], _ptr(pl),
                                        int(flags)))

    def pncg_set_solver(self, iter_max=100, eps=1e-3, term=TERM_DELTA_E, gravity=(0.0, 0.0, -9.8), flags=0):
        g = _f64(gravity)
        self._check(_L.pncg_set_solver(self._h, int(iter_max), float(eps), int(term), _ptr(g), int(flags)))

    def pncg_set_candidates_override(self, kind, pairs):
        """Install an explicit (n, 2) pair list of KIND_PT or KIND_EE in place of
        the hash candidates; pairs=None removes every override."""
        if pairs is None:
            self._check(_L.pncg_set_candidates_override(self._h, int(kind), -1, None))
            return
        pr = _i32(np.asarray(pairs).reshape(-1, 2))
        self._check(_L.pncg_set_candidates_override(self._h, int(kind), pr.shape[0], _ptr(pr)))

    def pncg_set_tuning(self, skin=0.0, chunk=0):
        self._check(_L.pncg_set_tuning(self._h, float(skin), int(chunk)))

    def pncg_set_adjoint_warm_start(self, on):
        self._check(_L.pncg_set_adjoint_warm_start(self._h, 1 if on else 0))

    def pncg_mean_boundary_edge(self):
        out = C.c_double()
        self._check(_L.pncg_mean_boundary_edge(self._h, C.byref(out)))
        return out.value

    def pncg_set_dirichlet(self, idx, target):
        idx = _i32(idx)
        target = _f64(target).reshape(-1, 3)
        self._check(_L.pncg_set_dirichlet(self._h, idx.shape[0], _ptr(idx), _ptr(target)))

    # -------------------------------------------------------------- steps
    def pncg_step(self, x, v, h):
        x = _f64(x, (self.nV, 3))
        v = _f64(v, (self.nV, 3))
        xo = np.empty_like(x)
        vo = np.empty_like(v)
        st = pncg_stats()
        rc = self._check(_L.pncg_step(self._h, _ptr(x), _ptr(v), float(h), _ptr(xo), _ptr(vo), C.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        return xo, vo, d

    def pncg_step_dev(self, x, v, h, x_out, v_out):
        """x, v, x_out, v_out: float64 CUDA tensors of shape (nV, 3), contiguous."""
        for t in (x, v, x_out, v_out):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
                    and tuple(t.shape) == (self.nV, 3)):
                raise ValueError("step_dev needs contiguous float64 CUDA tensors of shape (nV, 3)")
        _ready(x, self._stream)
        st = pncg_stats()
        rc = self._check(_L.pncg_step_dev(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()), float(h),
                                          C.c_void_p(x_out.data_ptr()), C.c_void_p(v_out.data_ptr()), C.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        return d

    def pncg_step_dev_noalloc(self, x, v, h, x_out, v_out):
        """pncg_step_dev through the allocation-free entry point (the step's
        reduction scratch in the library's static device array)."""
        for t in (x, v, x_out, v_out):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
                    and tuple(t.shape) == (self.nV, 3)):
                raise ValueError("step_dev_noalloc needs contiguous float64 CUDA tensors of shape (nV, 3)")
        _ready(x, self._stream)
        st = pncg_stats()
        rc = self._check(_L.pncg_step_dev_noalloc(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()),
                                                  float(h), C.c_void_p(x_out.data_ptr()),
                                                  C.c_void_p(v_out.data_ptr()), C.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        return d

    def pncg_run_dev(self, x, v, h, nsteps):
        """nsteps steps in place on the float64 CUDA tensors x, v (nV, 3);
        returns the per-step statistics (list of dicts) and the status."""
        for t in (x, v):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
                    and tuple(t.shape) == (self.nV, 3)):
                raise ValueError("run_dev needs contiguous float64 CUDA tensors of shape (nV, 3)")
        n = int(nsteps)
        if n < 1:
            raise ValueError("nsteps must be >= 1")
        _ready(x, self._stream)
        sts = (pncg_stats * n)()
        rc = self._check(_L.pncg_run_dev(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()), float(h), n,
                                         sts))
        return [s.as_dict() for s in sts], rc

    # ------------------------------------------------------------ queries
    def pncg_energy(self, x, xt, h):
        x = _f64(x, (self.nV, 3))
        xt = _f64(xt, (self.nV, 3))
        out = C.c_double()
        self._check(_L.pncg_energy(self._h, _ptr(x), _ptr(xt), float(h), C.byref(out)))
        return out.value

    def pncg_gradient(self, x, xt, h, want_diag=True):
        x = _f64(x, (self.nV, 3))
        xt = _f64(xt, (self.nV, 3))
        g = np.empty((self.nV, 3))
        d = np.empty((self.nV, 3)) if want_diag else None
        self._check(_L.pncg_gradient(self._h, _ptr(x), _ptr(xt), float(h), _ptr(g), _ptr(d)))
        return g, d

    def pncg_hvp(self, x, p, h, want_hp=True):
        x = _f64(x, (self.nV, 3))
        p = _f64(p, (self.nV, 3))
        hp = np.empty((self.nV, 3)) if want_hp else None
        out = C.c_double()
        self._check(_L.pncg_hvp(self._h, _ptr(x), _ptr(p), float(h), _ptr(hp), C.byref(out)))
        return hp, out.value

    def pncg_candidates(self, x, kind):
        x = _f64(x, (self.nV, 3))
        n = C.c_int64()
        rc = _L.pncg_candidates(self._h, _ptr(x), int(kind), None, 0, C.byref(n))
        if rc < 0 and rc != E_CAPACITY:
            self._check(rc)
        out = np.empty((max(n.value, 1), 2), dtype=np.int32)
        self._check(_L.pncg_candidates(self._h, _ptr(x), int(kind), _ptr(out), out.shape[0], C.byref(n)))
        return out[:n.value]

    def pncg_solver_pairs(self, x, kind):
        x = _f64(x, (self.nV, 3))
        n = C.c_int64()
        rc = _L.pncg_solver_pairs(self._h, _ptr(x), int(kind), None, 0, C.byref(n))
        if rc < 0 and rc != E_CAPACITY:
            self._check(rc)
        out = np.empty((max(n.value, 1), 2), dtype=np.int32)
        self._check(_L.pncg_solver_pairs(self._h, _ptr(x), int(kind), _ptr(out), out.shape[0], C.byref(n)))
        return out[:n.value]

    def pncg_min_distance(self, x):
        x = _f64(x, (self.nV, 3))
        d, j = C.c_double(), C.c_double()
        self._check(_L.pncg_min_distance(self._h, _ptr(x), C.byref(d), C.byref(j)))
        return d.value, j.value


    # ------------------------------------------------------------ adjoint
    def pncg_adjoint_step(self, x1, h, xbar, vbar, Ebar=None, cg_tol=1e-10, cg_max=10000):
        """Host arrays; returns (xbar_t, vbar_t, Ebar (accumulated copy), stats)."""
        x1 = _f64(x1, (self.nV, 3))
        xbar = _f64(xbar, (self.nV, 3))
        vbar = _f64(vbar, (self.nV, 3))
        Eb = np.zeros(self.nT) if Ebar is None else np.array(Ebar, dtype=np.float64).reshape(self.nT)
        xo = np.empty_like(x1)
        vo = np.empty_like(x1)
        st = pncg_adjoint_stats()
        rc = self._check(_L.pncg_adjoint_step(self._h, _ptr(x1), float(h), _ptr(xbar), _ptr(vbar), float(cg_tol),
                                              int(cg_max), _ptr(xo), _ptr(vo), _ptr(Eb), C.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        return xo, vo, Eb, d

    def pncg_adjoint_step_dev(self, x1, h, xbar, vbar, xbar_t, vbar_t, Ebar, cg_tol=1e-10, cg_max=10000):
        """float64 CUDA tensors: x1, xbar, vbar, xbar_t, vbar_t (nV, 3); Ebar (nT,) accumulated."""
        n = self.nV
        if not (Ebar.is_cuda and Ebar.element_size() == 8 and Ebar.is_contiguous() and Ebar.numel() == self.nT):
            raise ValueError(f"Ebar must be a contiguous float64 CUDA tensor of {self.nT} values")
        _ready(x1, self._stream)
        st = pncg_adjoint_stats()
        rc = self._check(_L.pncg_adjoint_step_dev(
            self._h, _dev_ptr(x1, n, "x1"), float(h), _dev_ptr(xbar, n, "xbar"), _dev_ptr(vbar, n, "vbar"),
            float(cg_tol), int(cg_max), _dev_ptr(xbar_t, n, "xbar_t"), _dev_ptr(vbar_t, n, "vbar_t"),
            C.c_void_p(Ebar.data_ptr()), C.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        return d

    # ---------------------------------------------------------- profiling
    def pncg_set_profiling(self, on):
        self._check(_L.pncg_set_profiling(self._h, 1 if on else 0))

    def pncg_get_profile(self):
        """{kind: (total_us, launches)} for the kinds in PROF_KINDS."""
        us = np.zeros(len(PROF_KINDS))
        n = np.zeros(len(PROF_KINDS), dtype=np.int64)
        self._check(_L.pncg_get_profile(self._h, _ptr(us), _ptr(n)))
        return {k: (float(us[i]), int(n[i])) for i, k in enumerate(PROF_KINDS)}


def _model_code(model):
    """A MODEL_* value from a name in MODELS or an integer (which the library
    validates)."""
    if isinstance(model, str):
        if model not in MODELS:
            raise ValueError(f"unknown material model {model!r}; one of {sorted(MODELS)}")
        return MODELS[model]
    return int(model)


def _ready(t, stream=0):
    """The library reads device inputs on its own stream, which does not wait
    for torch's: finish what torch has queued on the tensor's device (a
    clone of the state, say) before the library reads it.  Nothing to wait
    for when the library runs on torch's current stream (``stream``, the
    handle given at creation)."""
    import torch
    cur = torch.cuda.current_stream(t.device)
    if stream and cur.cuda_stream == stream:
        return
    cur.synchronize()


def _dev_ptr(t, n, what):
    if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()
            and tuple(t.shape) == (n, 3)):
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor of shape ({n}, 3)")
    return C.c_void_p(t.data_ptr())


class Batch:
    """A batch of independent scenes (pncg_batch_*): concatenated meshes
    with per-scene offsets and scene-local indices."""

    def __init__(self, vert_off, X, tet_off, tets, tri_off, tris, E, nu, rho, planes=None,
                 device=0, precision=FP64, stream=None):
        vert_off, tet_off, tri_off = _i32(vert_off), _i32(tet_off), _i32(tri_off)
        X, E, nu, rho = _f64(X), _f64(E), _f64(nu), _f64(rho)
        tets, tris = _i32(tets), _i32(tris)
        S = vert_off.shape[0] - 1
        if tet_off.shape[0] != S + 1 or tri_off.shape[0] != S + 1:
            raise ValueError("offset arrays must all have nScenes + 1 entries")
        nV, nT, nF = int(vert_off[-1]), int(tet_off[-1]), int(tri_off[-1])
        if X.shape != (nV, 3) or tets.shape != (nT, 4) or tris.reshape(-1, 3).shape[0] != nF:
            raise ValueError("array sizes do not match the offsets")
        if E.shape != (nT,) or nu.shape != (nT,) or rho.shape != (nT,):
            raise ValueError("E, nu, rho need one value per tet")
        pl = None if planes is None else _f64(planes).reshape(S, 4)
        opts = pncg_opts(device, precision, stream, 0, 0, 0)
        self._stream = int(stream or 0)
        h = C.c_void_p()
        rc = _L.pncg_batch_create(C.byref(h), C.byref(opts), S, _ptr(vert_off), _ptr(X), _ptr(tet_off), _ptr(tets),
                                  _ptr(tri_off), _ptr(tris), _ptr(E), _ptr(nu), _ptr(rho), _ptr(pl))
        if rc < 0:
            raise PncgError(rc, _L.pncg_batch_last_error(None).decode())
        self._h = h
        self.nScenes, self.nV, self.nT = S, nV, nT
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None) and _L is not None:   # _L is None at interpreter exit
            _L.pncg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise PncgError(rc, _L.pncg_batch_last_error(self._h).decode())
        return rc

    def pncg_batch_set_params(self, dhat, kappa, iter_max=100, eps=1e-3, term=TERM_DELTA_E,
                              gravity=(0.0, 0.0, -9.8), flags=0):
        g = _f64(gravity)
        self._check(_L.pncg_batch_set_params(self._h, float(dhat), float(kappa), int(iter_max), float(eps), int(term),
                                             _ptr(g), int(flags)))

    def pncg_batch_set_block(self, block):
        self._check(_L.pncg_batch_set_block(self._h, int(block)))

    def pncg_batch_set_model(self, model):
        """model: a MODEL_* value or one of the names in MODELS."""
        self._check(_L.pncg_batch_set_model(self._h, _model_code(model)))

    def pncg_batch_set_staging(self, lds):
        self._check(_L.pncg_batch_set_staging(self._h, int(lds)))

    def pncg_batch_set_split(self, max_team, max_polls=0):
        self._check(_L.pncg_batch_set_split(self._h, int(max_team), int(max_polls)))

    def pncg_batch_get_config(self):
        """dict(block, lds, max_team, teams) of the step kernel's schedule."""
        v = [C.c_int32() for _ in range(4)]
        self._check(_L.pncg_batch_get_config(self._h, *[C.byref(q) for q in v]))
        return dict(zip(("block", "lds", "max_team", "teams"), [q.value for q in v]))

    def pncg_batch_step(self, x, v, h, x_out, v_out):
        """float64 CUDA tensors (nV, 3); x_out/v_out must not alias x/v."""
        n = self.nV
        _ready(x, self._stream)
        self._check(_L.pncg_batch_step(self._h, _dev_ptr(x, n, "x"), _dev_ptr(v, n, "v"), float(h),
                                       _dev_ptr(x_out, n, "x_out"), _dev_ptr(v_out, n, "v_out")))

    def pncg_batch_run(self, x, v, h, nsteps):
        """nsteps steps in place on the float64 CUDA tensors x, v (nV, 3)."""
        n = self.nV
        _ready(x, self._stream)
        self._check(_L.pncg_batch_run(self._h, _dev_ptr(x, n, "x"), _dev_ptr(v, n, "v"), float(h), int(nsteps)))

    def pncg_batch_stats(self):
        it = np.zeros(self.nScenes, dtype=np.int32)
        rs = np.zeros(self.nScenes, dtype=np.int32)
        tot = np.zeros(self.nScenes, dtype=np.int64)
        self._check(_L.pncg_batch_stats(self._h, _ptr(it), _ptr(rs), _ptr(tot)))
        return it, rs, tot

    def pncg_batch_autotune(self, x, v, h, reps=3):
        n = self.nV
        _ready(x, self._stream)
        out = C.c_int32()
        self._check(_L.pncg_batch_autotune(self._h, _dev_ptr(x, n, "x"), _dev_ptr(v, n, "v"), float(h), int(reps),
                                           C.byref(out)))
        return out.value


def pncg_create(device=0, precision=FP64, stream=None, chunk=0, scatter=SCATTER_AUTO):
    return Context(device, precision, stream, chunk, scatter)
