"""The C-ABI library loads, exports every symbol include/pncg.h declares, and
rejects bad input on the host before any device call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pncg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pncg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2405_08001_amd as P
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTS)


def test_header_compiles_as_c():
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        open(src, "w").write('#include "pncg.h"\nint main(void){pncg_opts o={0,PNCG_MIXED,0,0,0};(void)o;return 0;}\n')
        r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), src, "-o",
                            os.path.join(d, "t")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def _ctx():
    import paper_2405_08001_amd as P
    return P.Context(0, P.FP64)


def test_create_rejects_bad_precision():
    import paper_2405_08001_amd as P
    with pytest.raises(P.PncgError) as e:
        P.Context(0, 7)
    assert e.value.code == P.E_INVAL


def test_create_rejects_bad_scatter_mode():
    import paper_2405_08001_amd as P
    for bad in (-1, 3):
        with pytest.raises(P.PncgError) as e:
            P.Context(0, P.FP64, scatter=bad)
        assert e.value.code == P.E_INVAL
    for ok in (P.SCATTER_AUTO, P.SCATTER_ATOMIC, P.SCATTER_SEGMENTED):
        P.Context(0, P.MIXED, scatter=ok).close()


def test_create_rejects_bad_graphs_flag():
    import ctypes as C
    import paper_2405_08001_amd as P
    from paper_2405_08001_amd import _lib
    h = C.c_void_p()
    for bad in (-1, 2):
        opts = _lib.pncg_opts(0, P.FP64, None, 0, 0, bad)
        assert _lib._L.pncg_create(C.byref(h), C.byref(opts)) == P.E_INVAL
    for graphs in (True, False):
        P.Context(0, P.MIXED, graphs=graphs).close()


def test_candidates_override_needs_a_mesh():
    import paper_2405_08001_amd as P
    c = _ctx()
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_candidates_override(P.KIND_PT, np.array([[0, 0]]))
    assert e.value.code == P.E_STATE
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_candidates_override(P.KIND_PT, None)
    assert e.value.code == P.E_STATE


def test_call_order_is_enforced():
    import paper_2405_08001_amd as P
    c = _ctx()
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_material([1e5], [0.3], [1e3])
    assert e.value.code == P.E_STATE
    c.nV = 4
    with pytest.raises(P.PncgError) as e:
        c.pncg_step(np.zeros((4, 3)), np.zeros((4, 3)), 0.01)
    assert e.value.code == P.E_STATE
    with pytest.raises(P.PncgError) as e:
        c.pncg_energy(np.zeros((4, 3)), np.zeros((4, 3)), 0.01)
    assert e.value.code == P.E_STATE


def test_set_mesh_validation():
    import paper_2405_08001_amd as P
    sc = scenes.tiny_scene()
    c = _ctx()
    bad = sc.tets.copy()
    bad[0, 0] = sc.nV            # index out of range
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(sc.X, bad, sc.tris, sc.edges)
    assert e.value.code == P.E_INVAL
    inv = sc.tets.copy()
    inv[3, [1, 2]] = inv[3, [2, 1]]   # negative orientation
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(sc.X, inv, sc.tris, sc.edges)
    assert e.value.code == P.E_INVERTED
    X = sc.X.copy()
    X[2, 1] = np.nan
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(X, sc.tets, sc.tris, sc.edges)
    assert e.value.code == P.E_NONFINITE
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(sc.X, sc.tets, sc.tris, np.array([[0, 0]]))
    assert e.value.code == P.E_INVAL


def test_vertex_degree_limit():
    import paper_2405_08001_amd as P
    # a fan of 65 tets around vertex 0
    n = 65
    ang = np.linspace(0, 2 * np.pi, n, endpoint=False)
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(n)], 1)
    X = np.concatenate([[[0, 0, 0.0]], [[0, 0, 1.0]], ring])
    tets = np.array([[0, 2 + i, 2 + (i + 1) % n, 1] for i in range(n)])
    c = _ctx()
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(X, tets)
    assert e.value.code == P.E_INVAL and "64" in str(e.value)


def test_valid_mesh_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2405_08001_amd as P
    sc = scenes.tiny_scene()
    c = _ctx()
    with pytest.raises(P.PncgError) as e:
        c.pncg_set_mesh(sc.X, sc.tets, sc.tris, sc.edges)
    assert e.value.code == P.E_HIP


def _batch_args(n=3):
    scs = scenes.batched_scenes(n_scenes=n, t_lo=30, t_hi=200)
    b = scenes.pack_batch(scs)
    return {k: b[k] for k in ("vert_off", "X", "tet_off", "tets", "tri_off", "tris", "E", "nu", "rho", "planes")}


def test_batch_create_validation():
    """Host-side checks of pncg_batch_create run before any device call."""
    import paper_2405_08001_amd as P
    a = _batch_args()
    bad = dict(a, tets=a["tets"].copy())
    bad["tets"][a["tet_off"][1], 0] = a["vert_off"][2] - a["vert_off"][1]   # local index past scene 1's vertices
    with pytest.raises(P.PncgError) as e:
        P.Batch(**bad)
    assert e.value.code == P.E_INVAL and "scene 1" in str(e.value)
    bad = dict(a, tets=a["tets"].copy())
    bad["tets"][0, [0, 1]] = bad["tets"][0, [1, 0]]                          # negative orientation
    with pytest.raises(P.PncgError) as e:
        P.Batch(**bad)
    assert e.value.code == P.E_INVERTED
    bad = dict(a, E=a["E"].copy())
    bad["E"][5] = -1.0
    with pytest.raises(P.PncgError) as e:
        P.Batch(**bad)
    assert e.value.code == P.E_INVAL
    bad = dict(a, planes=a["planes"] * 2.0)                                  # non-unit normal
    with pytest.raises(P.PncgError) as e:
        P.Batch(**bad)
    assert e.value.code == P.E_INVAL
    bad = dict(a, tet_off=a["tet_off"].copy())
    bad["tet_off"][2] = bad["tet_off"][1]                                    # a scene without tets
    with pytest.raises(P.PncgError) as e:
        P.Batch(**bad)
    assert e.value.code == P.E_INVAL


def test_batch_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2405_08001_amd as P
    with pytest.raises(P.PncgError) as e:
        P.Batch(**_batch_args())
    assert e.value.code == P.E_HIP


def _header_constants():
    """PNCG_* integer constants of the header, evaluated (plain integers,
    `u` suffixes and shifts only)."""
    out = {}
    for name, expr in re.findall(r"^#define\s+PNCG_([A-Z0-9_]+)\s+([^/\n]+)", open(HEADER).read(), flags=re.M):
        expr = re.sub(r"(\d+)u\b", r"\1", expr.strip())
        if re.fullmatch(r"[\d\s()<\-+]+", expr):
            out[name] = eval(expr)     # noqa: S307 - digits, parentheses and shifts only
    return out


def test_binding_constants_match_the_header():
    import paper_2405_08001_amd._lib as L
    consts = _header_constants()
    checked = 0
    for name, value in consts.items():
        if name == "PROF_KINDS":
            # the binding holds the kind names in index order
            assert len(L.PROF_KINDS) == value
            assert all(consts["PROF_" + k.upper()] == i for i, k in enumerate(L.PROF_KINDS))
            continue
        if hasattr(L, name):
            assert getattr(L, name) == value, name
            checked += 1
    for name in ("MODEL_NH", "MODEL_SNH", "MODEL_ARAP", "MODEL_FCR", "BETA_HZ", "SPLIT_OBJECTS", "E_INVERTED",
                 "TERM_GRAD_ABS", "CONTACT_REST_EXCLUDE", "MIXED"):
        assert name in consts and hasattr(L, name), name
    assert checked >= 30
    assert L.MODELS == {"nh": consts["MODEL_NH"], "snh": consts["MODEL_SNH"], "arap": consts["MODEL_ARAP"],
                        "fcr": consts["MODEL_FCR"]}
    assert L.BETA_RULES == {"dk": consts["BETA_DK"], "fr": consts["BETA_FR"], "prp": consts["BETA_PRP"],
                            "cd": consts["BETA_CD"], "hz": consts["BETA_HZ"]}
