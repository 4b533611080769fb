"""The twisted bar (40x8x8 cells, 15,360 tets, ends counter-rotated by 2 pi
per 120 steps) run on the GPU until it coils into itself: every step must
stay penetration-free with no inverted tet, the property the step bound of
Sec. 4.3 guarantees in place of continuous collision detection."""
import sys

import numpy as np
import pytest

import scenes
from helpers import make_ctx

pytestmark = pytest.mark.gpu


def test_twisted_bar_coils_without_penetration():
    sc = scenes.twisted_bar_scene()
    ctx = make_ctx(sc, 1)                        # mixed precision, IterMax 150, eps 1e-3
    x, v = sc.x0.copy(), sc.v0.copy()
    worst_d, worst_j, max_act = np.inf, np.inf, 0
    for t in range(1, 301):
        ctx.pncg_set_dirichlet(sc.fixed, scenes.twist_targets(sc, t))
        x, v, st = ctx.pncg_step(x, v, sc.h)
        d, j = ctx.pncg_min_distance(x)
        worst_d, worst_j = min(worst_d, d), min(worst_j, j)
        max_act = max(max_act, st["n_active"])
        if t % 50 == 0:
            print(f"step {t}: iters {st['iters']} active {st['n_active']} candidates {st['n_candidates']} "
                  f"dmin {d:.3e} jmin {j:.3f}", flush=True)
            sys.stdout.flush()
        assert d > 0.0 and j > 0.0, f"step {t}: dmin {d} jmin {j}"
    print(f"worst dmin {worst_d:.3e}, worst jmin {worst_j:.3f}, most active pairs {max_act}", flush=True)
    assert max_act > 100                          # the bar did coil into itself
