"""FP64 CPU oracle for the Jacobi-preconditioned Dai-Kou nonlinear conjugate
gradient (PNCG) method on the IPC incremental potential.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library: its only shared input is the seeded
scene generator module ``scenes``, which holds no solver arithmetic.

Modules (each function cites the passage of the paper it follows):
  barrier     IPC log barrier b(d) and its derivatives     (Sec. 3, eq. barrier)
  elastic     Neo-Hookean energy, gradient, Hessian diag,
              p^T H p, Hessian-vector product               (Sec. 3.1)
  distance    point-triangle / edge-edge closest points as
              t = sum_i c_i x_i                              (Sec. 3.2, eqs. PT, EE)
  candidates  inflated-AABB candidate sets, rest exclusion  (Sec. 5.1, Sec. 6)
  problem     incremental potential E, gradient, diag(H),
              p^T H p, H v                                   (Sec. 3, eqs. E, Hessian)
  pncg        Algorithm 1 (PNCG time step)                  (Sec. 4, Algorithm 1)
  adjoint     implicit-differentiation gradient of a loss
              over a trajectory (direct sparse solves)       (not in the paper)

Functions whose pin is weaker than the bar are marked "parity unpinned" in
their docstrings.
"""
from . import barrier, elastic, distance, candidates, problem, pncg, adjoint  # noqa: F401
