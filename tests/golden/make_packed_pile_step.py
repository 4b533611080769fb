"""Writes tests/golden/packed_pile_step.npz: the float64 oracle's time steps
of the contact-rich packed pile (scenes.packed_pile_scene: the pile's 110k
tets stacked with sub-dhat gaps, about 25k point-triangle and edge-edge
pairs active) from rest, which the GPU parity test compares against.  It
calls only the oracle and the scene generator.

  x      the configured step (Algorithm 1: at most 25 iterations, stop at
         dE < 1e-3 dE_0)
  x2     two fixed iterations
  x2_ties  the same with the other tie rule for closest points (the last
         of equally near candidates, see oracle.distance): the packed
         shapes have exactly parallel edges whose closest-point pair is not
         unique, and this measures how far that choice alone moves x2
  x_pert the configured step from the start state perturbed by a relative
         1e-15 (seeded), which measures how far rounding alone moves the
         oracle's own result after the configured iterations

    python tests/golden/make_packed_pile_step.py      (about 25 minutes)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scenes  # noqa: E402
from oracle import pncg, problem  # noqa: E402


def main():
    t0 = time.time()
    sc = scenes.packed_pile_scene()
    P = problem.Problem.from_scene(sc)
    a = P.active_set(sc.x0)
    x, v, st = pncg.step(P, sc.x0, sc.v0, sc.h, iter_max=sc.iter_max, eps=sc.eps, term=sc.term, record=True)
    dmin, jmin = P.min_distance(x)
    dE = np.array([h["dE"] for h in st.history])
    print(f"configured: {st.iters} iterations ({st.reason}), {time.time() - t0:.0f} s", flush=True)
    x2, _, st2 = pncg.step(P, sc.x0, sc.v0, sc.h, iter_max=2, eps=0.0, term="delta_e")
    print(f"two iterations: {st2.iters}, {time.time() - t0:.0f} s", flush=True)
    Pt = problem.Problem.from_scene(sc, ties="last")
    x2t, _, _ = pncg.step(Pt, sc.x0, sc.v0, sc.h, iter_max=2, eps=0.0, term="delta_e")
    print(f"two iterations, other tie rule: rel x {np.linalg.norm(x2t - x2) / np.linalg.norm(x2):.3e}, "
          f"{time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(12)
    xp0 = sc.x0 * (1.0 + 1e-15 * rng.choice([-1.0, 1.0], size=sc.x0.shape))
    xp, _, stp = pncg.step(P, xp0, sc.v0, sc.h, iter_max=sc.iter_max, eps=sc.eps, term=sc.term)
    out = os.path.join(HERE, "packed_pile_step.npz")
    np.savez_compressed(out, x=x, iters=st.iters, reason=st.reason, dE=dE, alpha_upper_hits=st.alpha_upper_hits,
                        n_pt0=int(np.sum(a.kind == 0)), n_ee0=int(np.sum(a.kind == 1)), n_plane0=len(a.pd),
                        n_active=st.n_active, n_plane=st.n_plane, dmin=dmin, jmin=jmin,
                        x2=x2, iters2=st2.iters, alpha_upper_hits2=st2.alpha_upper_hits, x2_ties=x2t,
                        x_pert=xp, iters_pert=stp.iters)
    dx, dxp = x - sc.x0, xp - sc.x0
    print(f"{out}: {st.iters} iterations ({st.reason}), dE/dE0 {dE[-1] / dE[0]:.3e}, "
          f"active at start PT {int(np.sum(a.kind == 0))} EE {int(np.sum(a.kind == 1))} plane {len(a.pd)}, "
          f"dmin {dmin:.3e}, jmin {jmin:.3f}; perturbed start: rel x "
          f"{np.linalg.norm(xp - x) / np.linalg.norm(x):.3e}, rel dx "
          f"{np.linalg.norm(dxp - dx) / np.linalg.norm(dx):.3e}; {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
