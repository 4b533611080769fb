"""The allocation-free step (pncg_step_dev_noalloc) against pncg_step_dev:
the same kernels with the step's reduction scratch in the library's static
device array, so the results must be the same bits.  Calls come in a row on
one device with shrinking inputs (the twisted bar's first twist step, then
the falling cube stack, then a small cube), so each call runs on scratch the
previous one left behind.  A state that needs larger contact buffers than
the context holds gets E_CAPACITY and an in-place state is left as it was."""
import sys

import numpy as np
import pytest

import scenes
from helpers import make_ctx

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    bar = scenes.twisted_bar_scene()
    xb = bar.X.copy()
    stack = scenes.small_contact_scene()
    vs = np.zeros_like(stack.X)
    vs[stack.object_id == 1, 2] = -0.05
    tiny = scenes.tiny_scene()
    vt = np.tile([0.0, 0.0, -0.1], (tiny.nV, 1))
    return [("twisted bar", bar, xb, np.zeros_like(xb), {}),
            ("cube stack", stack, stack.X.copy(), vs, dict(iter_max=12, eps=0.0, term="delta_e")),
            ("tiny cube", tiny, tiny.X.copy(), vt, {})]


def _dev_step(ctx, x0, v0, h, fn):
    import torch
    dev = torch.device("cuda:0")
    x, v = torch.tensor(x0, device=dev), torch.tensor(v0, device=dev)
    xo, vo = torch.empty_like(x), torch.empty_like(v)
    st = getattr(ctx, fn)(x, v, h, xo, vo)
    return xo.cpu().numpy(), vo.cpu().numpy(), st


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_step_equals_step_dev(precision):
    for name, sc, x0, v0, kw in _cases():
        _say(f"no-alloc step: {name} ({sc.nV} vertices) precision={precision}")
        ctx = make_ctx(sc, precision, **kw)
        if len(sc.fixed):
            # the first twist step: the end faces turned by 2 pi / 120
            ctx.pncg_set_dirichlet(sc.fixed, scenes.twist_targets(sc, 1))
        # pncg_step_dev first: it sizes the context's contact buffers for this state
        xb, vb, sb = _dev_step(ctx, x0, v0, sc.h, "pncg_step_dev")
        xa, va, sa = _dev_step(ctx, x0, v0, sc.h, "pncg_step_dev_noalloc")
        xc, vc, sc2 = _dev_step(ctx, x0, v0, sc.h, "pncg_step_dev_noalloc")
        _say(f"  iters {sa['iters']}/{sb['iters']} active {sa['n_active']} rebuilds {sa['rebuilds']}")
        assert sa["iters"] > 0
        for xo, vo, so in ((xa, va, sa), (xc, vc, sc2)):
            assert np.array_equal(xo, xb) and np.array_equal(vo, vb)
            assert so == sb


def test_noalloc_step_rejects_what_would_allocate():
    import paper_2405_08001_amd as P
    import torch
    sc = scenes.small_contact_scene()
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.X, device=dev)
    v = torch.zeros_like(x)
    xo, vo = torch.empty_like(x), torch.empty_like(v)
    ctx = make_ctx(sc, 0, iter_max=P.NOALLOC_ITER_MAX + 1)
    with pytest.raises(P.PncgError) as e:
        ctx.pncg_step_dev_noalloc(x, v, sc.h, xo, vo)
    assert e.value.code == P.E_INVAL
    ctx = make_ctx(sc, 0, split=True)
    with pytest.raises(P.PncgError) as e:
        ctx.pncg_step_dev_noalloc(x, v, sc.h, xo, vo)
    assert e.value.code == P.E_INVAL
    ctx = make_ctx(sc, 0)
    ctx.pncg_set_profiling(1)
    with pytest.raises(P.PncgError) as e:
        ctx.pncg_step_dev_noalloc(x, v, sc.h, xo, vo)
    assert e.value.code == P.E_STATE


def test_noalloc_capacity_error_leaves_an_in_place_state():
    import paper_2405_08001_amd as P
    import torch
    sc = scenes.twisted_bar_scene()
    ctx = make_ctx(sc, 1)
    ctx.pncg_set_dirichlet(sc.fixed, scenes.twist_targets(sc, 1))
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.X, device=dev)
    v = torch.zeros_like(x)
    with pytest.raises(P.PncgError) as e:
        ctx.pncg_step_dev_noalloc(x, v, sc.h, x, v)
    assert e.value.code == P.E_CAPACITY
    assert np.array_equal(x.cpu().numpy(), sc.X) and not v.cpu().numpy().any()
    st = ctx.pncg_step_dev(x, v, sc.h, x, v)            # grows the buffers and steps
    x2, v2 = torch.tensor(sc.X, device=dev), torch.zeros_like(x)
    st2 = ctx.pncg_step_dev_noalloc(x2, v2, sc.h, x2, v2)
    assert st2 == st
    assert torch.equal(x2, x) and torch.equal(v2, v)
