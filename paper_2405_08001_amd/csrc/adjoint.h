// Adjoint of one converged time step (implicit differentiation): device
// conjugate gradients on H lambda = xbar + vbar / h with the Hessian-vector
// product of the elastic, inertia, plane and pair terms, then the adjoints of
// x^t, v^t and the per-tet Young's moduli.
#pragma once

#include "internal.h"

namespace pncg {

// Scalars of CG iteration k (single writer per field: block 0 of the launch
// named beside it).
struct CgScal {
  double rz;     // r_k . z_k            (Hv launch of k)
  double beta;   // rz_k / rz_{k-1}      (Hv launch of k)
  double alpha;  // rz_k / p_k . H p_k   (update launch of k)
  double pq;     // p_k . H p_k          (update launch of k)
};

struct CgStatus {
  int stopped;   // CG has ended
  int iters;     // CG iterations made (updates of lambda)
  int reason;    // 0 residual rule, 1 iteration cap, 2 p^T H p <= 0 or not finite
  int pad;
  double bb;     // |b|^2 (= |r_0|^2)
  double rr;     // |r|^2 at the end
};

struct AdjArgs {
  double4* lam;
  double4* r;
  double4* z;
  double4* pbuf[2];       // p_k lives in pbuf[k & 1]
  double4* q;             // H p_k
  double4* zw[2];         // fused form: {z_k, diag^-1 q_k} per vertex (2 double4) in zw[k & 1]
  const double* diag;     // [nV][3] Jacobi diagonal (prescribed rows 1)
  double* part_rz;        // [kMaxGrid][2]  r.z, r.r of the last update
  double* part_pq;        // [kMaxGrid]     p.Hp of the last Hv
  double* part_f;         // [kMaxGrid][8]  fused form: p.q, r.z, r.r, r.w, q.z, q.w of the last launch
  CgScal* scal;           // [max_iter + 1]
  CgStatus* status;
  double tol2;            // relative residual tolerance, squared
  int max_iter;
};

// b = xbar + vbar / h, r = b, lambda = 0, z = r / diag, partial sums; warm
// (no pair terms): start from the lambda already in C.lam, r = b - H lambda.
// The caller clears status->stopped before a warm start (the Hv sweep
// checks it).
void launch_adj_init(const Args<double>& A, const AdjArgs& C, const double* xbar, const double* vbar, bool warm,
                     hipStream_t s);
// CG iteration k.  fused (no pair terms): one launch that finishes update
// k-1 and forms z_k and p_k on the fly wherever the Hv sweep needs them;
// launches 0 .. max_iter+1.
// Otherwise a direction launch, the pair H p into acc, the Hv sweep and the
// update launch; launches 0 .. max_iter.
void launch_cg_iteration(const Args<double>& A, const AdjArgs& C, int k, bool fused, hipStream_t s);
// xbar_t = M lambda - vbar / h, vbar_t = h M lambda; Ebar[e] -= lambda . dG/dE_e.
void launch_adj_out(const Args<double>& A, const AdjArgs& C, const double* vbar, const double* E, double* xbar_t,
                    double* vbar_t, double* Ebar, hipStream_t s);

}  // namespace pncg
