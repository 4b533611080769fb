// Adjoint of one converged time step by implicit differentiation (not in
// the paper; the paper only notes that the IPC formulation is
// differentiable, Sec. 1).
//
// x^{t+1} solves G(x) = grad E(x) = 0 (Sec. 3, equation E) with
// xt = x^t + h v^t + h^2 g and v^{t+1} = (x^{t+1} - x^t) / h.  For adjoints
// xbar = dL/dx^{t+1}, vbar = dL/dv^{t+1}:
//     H lambda = xbar + vbar / h          (H = dG/dx at x^{t+1})
//     dL/dx^t  = M lambda - vbar / h,    dL/dv^t = h M lambda,
//     dL/dE_e -= lambda . dG/dE_e.
// H is applied matrix-free: the element term is the exact Neo-Hookean
// Hessian-vector product h^2 V dP(dF) b_a (Sec. 3.1), inertia M, the plane
// barrier kappa b''(d) n n^T (exact), and the pair terms as the solver's
// pair Hessian model (Sec. 3.2, equations eq9/eq12).  The system is solved by
// Jacobi-preconditioned linear CG.  Without pair terms an iteration is one
// launch (k_cg_fused): it finishes the previous update lazily, forms the new
// direction on the fly and applies H; with pair terms it is a direction
// launch, the pair H p, the Hv sweep and the update of lambda, r, z.  Global
// scalars are per-block partials re-reduced by the next launch in a fixed
// order, so every block takes the same decisions.
#include "adjoint.h"
#include "kernels.h"
#include "sweep_common.h"

namespace pncg {

namespace {

// threads per block of the fused CG iteration (512 measured slower: the
// register cap it needs makes the sweep spill)
constexpr int kCgBlock = 256;

__device__ __forceinline__ int read_stopped(const CgStatus* st) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = *reinterpret_cast<const volatile int*>(&st->stopped);
  __syncthreads();
  const int r = s_stop;
  __syncthreads();
  return r;
}

__device__ __forceinline__ V3<double> row3(const double* a, int v) {
  return mk3(a[3 * v], a[3 * v + 1], a[3 * v + 2]);
}

// Reduce the update partials of iteration k-1 (or of the initialisation),
// apply the stop rule and compute beta.  Returns false if CG has ended.
__device__ __forceinline__ bool cg_begin(const Args<double>& A, const AdjArgs& C, int k, double& beta, double* sh) {
  double red[2];
  const int kind[2] = {0, 0};
  reduce_partials<2>(C.part_rz, 2, A.grid, kind, red, sh);
  const double rz = red[0], rr = red[1];
  const double bb = (k == 0) ? rr : C.status->bb;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (k == 0 && lead) C.status->bb = rr;
  const bool conv = rr <= C.tol2 * bb;
  if (conv || k >= C.max_iter) {
    if (lead) {
      C.status->iters = k;
      C.status->reason = conv ? 0 : 1;
      C.status->rr = rr;
      C.status->stopped = 1;
    }
    return false;
  }
  beta = (k == 0) ? 0.0 : rz / C.scal[k - 1].rz;
  if (lead) {
    C.scal[k].rz = rz;
    C.scal[k].beta = beta;
  }
  return true;
}

}  // namespace

// warm: lambda holds a starting guess and q = H lambda (k_cg_hv on it), so
// r = b - q; otherwise lambda = 0 and r = b.  The stop rule's reference
// |b|^2 goes to slot 6 of the fused partials.
__global__ void __launch_bounds__(kSBlock) k_adj_init(Args<double> A, AdjArgs C, const double* xbar,
                                                      const double* vbar, int warm) {
  __shared__ double sh[kSWaves * 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    C.status->stopped = 0;
    C.status->iters = 0;
    C.status->reason = 0;
    C.status->bb = 0.0;
    C.status->rr = 0.0;
  }
  const double ih = 1.0 / A.h;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  const Slice sl = block_slice(A.nV);
  for (long long i = sl.begin + threadIdx.x; i < sl.end; i += kSBlock) {
    const int v = (int)i;
    const bool fixed = A.vflag[v] & kFixed;
    V3<double> b = mk3(0.0, 0.0, 0.0);
    if (!fixed) b = row3(xbar, v) + ih * row3(vbar, v);
    bb += dot(b, b);
    V3<double> r = b;
    if (warm) {
      const V3<double> q = ld3(C.q, v);
      r = mk3(b.x - q.x, b.y - q.y, b.z - q.z);
    } else {
      st3(C.lam, v, mk3(0.0, 0.0, 0.0));
    }
    const V3<double> d = row3(C.diag, v);
    const V3<double> z = mk3(r.x / d.x, r.y / d.y, r.z / d.z);
    st3(C.r, v, r);
    st3(C.z, v, z);
    st3(C.zw[1], 2 * v, z);                      // {z_0, w = 0} for the fused form
    st3(C.zw[1], 2 * v + 1, mk3(0.0, 0.0, 0.0));
    rz += dot(r, z);
    rr += dot(r, r);
  }
  double red[3] = {rz, rr, bb};
  const int kind[3] = {0, 0, 0};
  block_reduce<3>(red, kind, sh);
  if (threadIdx.x == 0) {
    C.part_rz[2 * blockIdx.x] = red[0];
    C.part_rz[2 * blockIdx.x + 1] = red[1];
    double* f = C.part_f + 8 * blockIdx.x;
    f[0] = 0.0;
    f[1] = red[0];
    f[2] = red[1];
    f[3] = f[4] = f[5] = 0.0;
    f[6] = red[2];
  }
}

// One launch per CG iteration k (no pair terms).  With D = diag^-1, the
// preconditioned residual z and w = D q are kept per vertex as one 64 B
// record {z, w} (zw[k & 1]), so a corner needs two gathers ({z, w} and the
// previous direction) like a plain Hv sweep.  From the partials of launch
// k-1 (p.q, r.z, r.r, r.w, q.z, q.w of iteration k-1):
//   stop if |r_{k-1}|^2 <= tol^2 |b|^2 (lambda_{k-1} is the result), or if
//   k-1 reached the cap, or if p.q <= 0;
//   alpha = r.z / p.q;  z_k = z_{k-1} - alpha w_{k-1};
//   r_k.z_k = r.z - alpha (r.w + q.z) + alpha^2 q.w;
//   beta = r_k.z_k / r.z;  p_k = z_k + beta p_{k-1},
// z_k and p_k formed on the fly at every corner; each vertex's last lane
// applies H and stores p_k, {z_k, D q_k} and lambda_k = lambda_{k-1} + alpha
// p_{k-1} (lambda in place: only that lane touches it), and adds the partials
// of launch k, with r_k = diag z_k (the residual itself is not stored).
// k_adj_init writes {z_0, 0} into zw[1] and the partials r_0.z_0, |r_0|^2.
template <int M>
__global__ void __launch_bounds__(kCgBlock) k_cg_fused(Args<double> A, AdjArgs C, int k) {
  constexpr int NW = kCgBlock / kWave;
  __shared__ double sh[NW * 7];
  if (read_stopped(C.status)) return;
  double red6[7];
  {
    const int kind[7] = {0, 0, 0, 0, 0, 0, 0};
    reduce_partials<7, kCgBlock>(C.part_f, 8, A.grid, kind, red6, sh);
  }
  const double pq = red6[0], rz = red6[1], rr = red6[2], rw = red6[3], qz = red6[4], qw = red6[5];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  // the stop rule's reference: |b|^2 from k_adj_init (slot 6)
  if (k == 0 && lead) C.status->bb = red6[6];
  const double bb = (k == 0) ? red6[6] : C.status->bb;
  auto stop = [&](int reason) {
    if (lead) {
      C.status->iters = k > 0 ? k - 1 : 0;
      C.status->reason = reason;
      C.status->rr = reason == 2 ? 0.0 : rr;
      C.status->stopped = 1;
    }
  };
  if (rr <= C.tol2 * bb) { stop(0); return; }
  if (k > 0 && k - 1 >= C.max_iter) { stop(1); return; }
  double alpha = 0.0, beta = 0.0;
  if (k > 0) {
    if (!(pq > 0.0) || !isfinite(pq)) { stop(2); return; }
    alpha = rz / pq;
    const double rz_new = rz - alpha * (rw + qz) + alpha * alpha * qw;
    beta = rz_new > 0.0 ? rz_new / rz : 0.0;
    if (lead) {
      C.scal[k - 1].alpha = alpha;
      C.scal[k - 1].pq = pq;
      C.scal[k].rz = rz_new;
      C.scal[k].beta = beta;
    }
  } else if (lead) {
    C.scal[0].rz = rz;
    C.scal[0].beta = 0.0;
  }
  const double4* zwprev = C.zw[(k + 1) & 1];
  double4* zwk = C.zw[k & 1];
  const double4* pprev = C.pbuf[(k + 1) & 1];
  double4* pk = C.pbuf[k & 1];
  auto zget = [&](int v) -> V3<double> {
    const V3<double> z = ld3(zwprev, 2 * v), w = ld3(zwprev, 2 * v + 1);
    return mk3(fma(-alpha, w.x, z.x), fma(-alpha, w.y, z.y), fma(-alpha, w.z, z.z));
  };
  auto pnext = [&](V3<double> z, V3<double> pp) -> V3<double> {
    if (k == 0) return z;
    return mk3(fma(beta, pp.x, z.x), fma(beta, pp.y, z.y), fma(beta, pp.z, z.z));
  };
  auto pget = [&](int v, V3<double> z) -> V3<double> {
    if (k == 0) return z;
    return pnext(z, ld3(pprev, v));
  };
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const Slice sl = block_slice(A.nWaves);
  double acc6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long w = sl.begin + wave; w < sl.end; w += NW) {
    const long long idx = w * kWave + lane;
    const int code = A.inc[idx];
    const int myv = A.inc_vert[idx];
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (code >= 0) {
      const ElemRec<double> rec = A.elem[code >> 2];
      Kin<double> kin = kinematics<double>(rec.B, ld3(A.x0, rec.v[0]), ld3(A.x0, rec.v[1]), ld3(A.x0, rec.v[2]),
                                           ld3(A.x0, rec.v[3]));
      V3<double> d[3];
      const int v0 = rec.v[0], v1 = rec.v[1], v2 = rec.v[2], v3 = rec.v[3];
      dF_cols(rec.B, pget(v0, zget(v0)), pget(v1, zget(v1)), pget(v2, zget(v2)), pget(v3, zget(v3)), d);
      V3<double> hp;
      if (el_Hp<double, M>(kin, rec.vmu, rec.vlam, d, shape_vec(rec.B, code & 3), hp)) {
        s[0] = hp.x;
        s[1] = hp.y;
        s[2] = hp.z;
      } else {
        raise_err(A.status, kErrInverted);
      }
    }
    if (!seg_sum(myv, s) || myv < 0) continue;
    const int v = myv;
    const V3<double> z = zget(v);
    const V3<double> pp = k > 0 ? ld3(pprev, v) : mk3(0.0, 0.0, 0.0);
    const V3<double> p = pnext(z, pp);
    const double m = A.mass[v];
    double hv[3] = {fma(A.h2, s[0], m * p.x), fma(A.h2, s[1], m * p.y), fma(A.h2, s[2], m * p.z)};
    const uint8_t fl = A.vflag[v];
    if (fl & kSurface) {
      const V3<double> x = ld3(A.x0, v);
      for (int j = 0; j < A.planes.n; ++j) {
        const double* pl = A.planes.p[j];
        const double d = plane_dist(pl, x);
        if (d > 0.0 && d < A.dhat) {
          const double c = A.kappa * barrier_d2b(d, A.dhat) * (pl[0] * p.x + pl[1] * p.y + pl[2] * p.z);
          hv[0] += c * pl[0];
          hv[1] += c * pl[1];
          hv[2] += c * pl[2];
        }
      }
    }
    if (fl & kFixed) hv[0] = hv[1] = hv[2] = 0.0;
    const V3<double> q = mk3(hv[0], hv[1], hv[2]);
    if (k > 0) {
      const V3<double> l = ld3(C.lam, v);
      st3(C.lam, v, mk3(fma(alpha, pp.x, l.x), fma(alpha, pp.y, l.y), fma(alpha, pp.z, l.z)));
    }
    const V3<double> dg = row3(C.diag, v);
    const V3<double> r = mk3(dg.x * z.x, dg.y * z.y, dg.z * z.z);
    const V3<double> wq = mk3(q.x / dg.x, q.y / dg.y, q.z / dg.z);
    st3(pk, v, p);
    st3(zwk, 2 * v, z);
    st3(zwk, 2 * v + 1, wq);
    acc6[0] += dot(p, q);
    acc6[1] += dot(r, z);
    acc6[2] += dot(r, r);
    acc6[3] += dot(r, wq);
    acc6[4] += dot(q, z);
    acc6[5] += dot(q, wq);
  }
  {
    const int kind[6] = {0, 0, 0, 0, 0, 0};
    block_reduce<6, kCgBlock>(acc6, kind, sh);
  }
  if (threadIdx.x == 0) {
    double* f = C.part_f + 8 * blockIdx.x;
    for (int i = 0; i < 6; ++i) f[i] = acc6[i];
    f[6] = 0.0;
  }
}

// Direction launch of the non-lazy form: p_k = z_k + beta p_{k-1}
// materialised, pair accumulators cleared for the pair H p launch.
__global__ void __launch_bounds__(kSBlock) k_cg_dir(Args<double> A, AdjArgs C, int k) {
  __shared__ double sh[kSWaves * 2];
  if (read_stopped(C.status)) return;
  double beta = 0.0;
  if (!cg_begin(A, C, k, beta, sh)) return;
  const double4* pprev = C.pbuf[(k + 1) & 1];
  double4* pk = C.pbuf[k & 1];
  const Slice sl = block_slice(A.nV);
  for (long long i = sl.begin + threadIdx.x; i < sl.end; i += kSBlock) {
    const int v = (int)i;
    V3<double> p = ld3(C.z, v);
    if (k > 0) {
      const V3<double> pp = ld3(pprev, v);
      p = mk3(fma(beta, pp.x, p.x), fma(beta, pp.y, p.y), fma(beta, pp.z, p.z));
    }
    st3(pk, v, p);
    A.acc[8 * v] = 0.0;
    A.acc[8 * v + 1] = 0.0;
    A.acc[8 * v + 2] = 0.0;
  }
}

// q = H p_k by the vertex-centric sweep (p_k materialised by k_cg_dir, the
// pair part already in acc); partials of p_k . q.
template <int M, bool SEG = false>
__global__ void __launch_bounds__(kSBlock) k_cg_hv(Args<double> A, AdjArgs C, int k) {
  __shared__ double sh[kSWaves * 2];
  if (read_stopped(C.status)) return;
  const double4* pk = C.pbuf[k & 1];
  auto pget = [&](int v) -> V3<double> { return ld3(pk, v); };
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const Slice sl = block_slice(A.nWaves);
  double pq = 0.0;
  for (long long w = sl.begin + wave; w < sl.end; w += kSWaves) {
    const long long idx = w * kWave + lane;
    const int code = A.inc[idx];
    const int myv = A.inc_vert[idx];
    int2 wr = make_int2(0, 0);
    if constexpr (SEG) wr = wave_range(A.wrange, (int)w);
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (code >= 0) {
      const ElemRec<double> rec = A.elem[code >> 2];
      Kin<double> kin = kinematics<double>(rec.B, ld3(A.x0, rec.v[0]), ld3(A.x0, rec.v[1]), ld3(A.x0, rec.v[2]),
                                           ld3(A.x0, rec.v[3]));
      V3<double> d[3];
      dF_cols(rec.B, pget(rec.v[0]), pget(rec.v[1]), pget(rec.v[2]), pget(rec.v[3]), d);
      V3<double> hp;
      bool ok;
      if constexpr (M == kModelNH) {
        // spelled out for Neo-Hookean: the generic helper costs registers here
        ok = kin.J > 0.0;
        if (ok) hp = nh_Hp(kin, rec.vmu, rec.vlam, d, shape_vec(rec.B, code & 3));
      } else {
        ok = el_Hp<double, M>(kin, rec.vmu, rec.vlam, d, shape_vec(rec.B, code & 3), hp);
      }
      if (ok) {
        s[0] = hp.x;
        s[1] = hp.y;
        s[2] = hp.z;
      } else {
        raise_err(A.status, kErrInverted);
      }
    }
    const bool vlane = seg_sum(myv, s) && myv >= 0;
    if (!vlane) continue;
    const int v = myv;
    double prs[3] = {0.0, 0.0, 0.0};
    if constexpr (SEG) {
      if (wr.x < wr.y) pair_partials_sum<3>(A.coff, A.rp, v, prs);
    }
    const V3<double> p = pget(v);
    const double m = A.mass[v];
    double hv[3] = {fma(A.h2, s[0], m * p.x), fma(A.h2, s[1], m * p.y), fma(A.h2, s[2], m * p.z)};
    const uint8_t fl = A.vflag[v];
    if (fl & kSurface) {
      const V3<double> x = ld3(A.x0, v);
      for (int j = 0; j < A.planes.n; ++j) {
        const double* pl = A.planes.p[j];
        const double d = plane_dist(pl, x);
        if (d > 0.0 && d < A.dhat) {
          const double c = A.kappa * barrier_d2b(d, A.dhat) * (pl[0] * p.x + pl[1] * p.y + pl[2] * p.z);
          hv[0] += c * pl[0];
          hv[1] += c * pl[1];
          hv[2] += c * pl[2];
        }
      }
    }
    if (A.self) {
      if constexpr (SEG) {
        hv[0] += prs[0];
        hv[1] += prs[1];
        hv[2] += prs[2];
      } else {
        hv[0] += A.acc[8 * v];
        hv[1] += A.acc[8 * v + 1];
        hv[2] += A.acc[8 * v + 2];
      }
    }
    if (fl & kFixed) hv[0] = hv[1] = hv[2] = 0.0;
    st3(C.q, v, mk3(hv[0], hv[1], hv[2]));
    pq += hv[0] * p.x + hv[1] * p.y + hv[2] * p.z;
  }
  double red[1] = {pq};
  const int kind[1] = {0};
  block_reduce<1>(red, kind, sh);
  if (threadIdx.x == 0) C.part_pq[blockIdx.x] = red[0];
}

// alpha = rz_k / p_k . H p_k; lambda += alpha p, r -= alpha q, z = r / diag.
__global__ void __launch_bounds__(kSBlock) k_cg_update(Args<double> A, AdjArgs C, int k) {
  __shared__ double sh[kSWaves * 2];
  if (read_stopped(C.status)) return;
  double red1[1];
  const int kind1[1] = {0};
  reduce_partials<1>(C.part_pq, 1, A.grid, kind1, red1, sh);
  const double pq = red1[0];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead) {
      C.status->iters = k;
      C.status->reason = 2;
      C.status->rr = 0.0;
      C.status->stopped = 1;
    }
    return;
  }
  const double alpha = C.scal[k].rz / pq;
  if (lead) {
    C.scal[k].alpha = alpha;
    C.scal[k].pq = pq;
  }
  const double4* pk = C.pbuf[k & 1];
  double rz = 0.0, rr = 0.0;
  const Slice sl = block_slice(A.nV);
  for (long long i = sl.begin + threadIdx.x; i < sl.end; i += kSBlock) {
    const int v = (int)i;
    const V3<double> p = ld3(pk, v), q = ld3(C.q, v), l = ld3(C.lam, v), r0 = ld3(C.r, v);
    const V3<double> d = row3(C.diag, v);
    st3(C.lam, v, mk3(fma(alpha, p.x, l.x), fma(alpha, p.y, l.y), fma(alpha, p.z, l.z)));
    const V3<double> r = mk3(fma(-alpha, q.x, r0.x), fma(-alpha, q.y, r0.y), fma(-alpha, q.z, r0.z));
    const V3<double> z = mk3(r.x / d.x, r.y / d.y, r.z / d.z);
    st3(C.r, v, r);
    st3(C.z, v, z);
    rz += dot(r, z);
    rr += dot(r, r);
  }
  double red[2] = {rz, rr};
  const int kind[2] = {0, 0};
  block_reduce<2>(red, kind, sh);
  if (threadIdx.x == 0) {
    C.part_rz[2 * blockIdx.x] = red[0];
    C.part_rz[2 * blockIdx.x + 1] = red[1];
  }
}

// Adjoints of x^t, v^t and the per-tet moduli (accumulated into Ebar).
template <int M>
__global__ void __launch_bounds__(kSBlock) k_adj_out(Args<double> A, AdjArgs C, const double* vbar, const double* E,
                                                     double* xbar_t, double* vbar_t, double* Ebar) {
  const int tid = blockIdx.x * kSBlock + threadIdx.x, stride = gridDim.x * kSBlock;
  const double ih = 1.0 / A.h;
  for (int v = tid; v < A.nV; v += stride) {
    const V3<double> l = ld3(C.lam, v), vb = row3(vbar, v);
    const double m = A.mass[v];
    const V3<double> ml = m * l;
    xbar_t[3 * v] = ml.x - vb.x * ih;
    xbar_t[3 * v + 1] = ml.y - vb.y * ih;
    xbar_t[3 * v + 2] = ml.z - vb.z * ih;
    vbar_t[3 * v] = A.h * ml.x;
    vbar_t[3 * v + 1] = A.h * ml.y;
    vbar_t[3 * v + 2] = A.h * ml.z;
  }
  for (int e = tid; e < A.nT; e += stride) {
    const ElemRec<double> rec = A.elem[e];
    Kin<double> kin = kinematics<double>(rec.B, ld3(A.x0, rec.v[0]), ld3(A.x0, rec.v[1]), ld3(A.x0, rec.v[2]),
                                         ld3(A.x0, rec.v[3]));
    // mu and lam are linear in E: d(V mu)/dE = V mu / E, likewise for lam
    const double iE = 1.0 / E[e];
    double s = 0.0;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      V3<double> dg;
      ok = ok && el_dgdE<double, M>(kin, rec.vmu * iE, rec.vlam * iE, shape_vec(rec.B, a), dg);
      if (ok) s += dot(ld3(C.lam, rec.v[a]), dg);
    }
    if (!ok) {
      raise_err(A.status, kErrInverted);
      continue;
    }
    Ebar[e] -= A.h2 * s;
  }
}

void launch_adj_init(const Args<double>& A, const AdjArgs& C, const double* xbar, const double* vbar, bool warm,
                     hipStream_t s) {
  if (warm) {
    // q = H lambda with the Hv sweep reading lambda as its direction
    AdjArgs W = C;
    W.pbuf[0] = C.lam;
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL(k_cg_hv<M_>, dim3(A.grid), dim3(kSBlock), 0, s, A, W, 0));
  }
  hipLaunchKernelGGL(k_adj_init, dim3(A.grid), dim3(kSBlock), 0, s, A, C, xbar, vbar, warm ? 1 : 0);
}

void launch_cg_iteration(const Args<double>& A, const AdjArgs& C, int k, bool fused, hipStream_t s) {
  if (fused) {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL(k_cg_fused<M_>, dim3(A.grid), dim3(kCgBlock), 0, s, A, C, k));
    return;
  }
  hipLaunchKernelGGL(k_cg_dir, dim3(A.grid), dim3(kSBlock), 0, s, A, C, k);
  if (A.self) {
    Args<double> B = A;
    B.p0 = C.pbuf[k & 1];
    launch_pairs_hvp<double>(B, s);
  }
  PNCG_BY_SCATTER(A.self && A.seg,
                  PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_cg_hv<M_, S_>), dim3(A.grid), dim3(kSBlock), 0, s, A, C, k)));
  hipLaunchKernelGGL(k_cg_update, dim3(A.grid), dim3(kSBlock), 0, s, A, C, k);
}

void launch_adj_out(const Args<double>& A, const AdjArgs& C, const double* vbar, const double* E, double* xbar_t,
                    double* vbar_t, double* Ebar, hipStream_t s) {
  PNCG_BY_MODEL(A.model,
                hipLaunchKernelGGL(k_adj_out<M_>, dim3(A.grid), dim3(kSBlock), 0, s, A, C, vbar, E, xbar_t, vbar_t, Ebar));
}

}  // namespace pncg
