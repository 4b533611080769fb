// Per-iteration kernels of the PNCG time step (Algorithm 1, Sec. 4) and the
// query kernels built from the same pieces.
//
// One iteration k is two launches (three with point-triangle / edge-edge
// contact under the atomic scatter or with one step size per object):
//   [narrow]  candidate pairs at x_k -> barrier gradient and diagonal, as
//             float64 atomics into per-vertex accumulators or as run
//             partials of the per-vertex entry index (segmented scatter);
//             with the segmented scatter and one step size the pass runs
//             inside the first grad launch, each block evaluating the
//             entries of its own vertices before its sweep
//   grad      vertex-centric element sweep: every lane evaluates one
//             (tet, corner) incidence, a wave-segmented sum gives each
//             vertex its complete gradient and diag(H) without atomics;
//             the vertex's lane adds inertia, planes and contact terms and
//             the dot products for beta (Sec. 4.1-4.2)
//   dir       beta from the grad partials; p_{k+1} = -P g + beta p_k is
//             recomputed on the fly wherever a tet or pair needs it, so the
//             element and pair parts of p^T H p run in the same launch as
//             the per-vertex update of p (Sec. 4.3)
// The first launch of iteration k + 1 reduces the dir partials into alpha
// (equations upper, alpha), applies x_{k+1} = x_k + alpha p while reading
// positions lazily, and evaluates the stop test (Sec. 4.4).
//
// Grid-wide reductions never use atomics on one address: each block writes
// its partial sums and the next launch's blocks re-reduce them in a fixed
// order, which is deterministic and costs no extra launch.
#include <cfloat>
#include <climits>

#include "internal.h"
#include "kernels.h"
#include "sweep_common.h"

namespace pncg {

// Threads per block of the vertex-centric sweep: it is latency bound and
// gains from more resident waves per compute unit than the 256-thread blocks
// of the other kernels give (the grid, and so the number of partials, stays
// the same).  Measured on the 110k-tet pile: float 448 (seven waves, about
// 115 VGPRs, so two blocks hold 14 waves of a compute unit: 24.2 us against
// 25.4 us at 384; 512 needs 131 VGPRs and drops to three waves per SIMD).
// Double 448 too (122 VGPRs, no spill; 512 with a four-wave cap spilled
// 16 B per lane): the 30,000-tet bar's forward step 13.6 -> 13.1 ms; except
// the corotated model (below).
template <typename R, int M>
struct GradBlock {
  static constexpr int value = 448, min_waves = 1;
};
// The float64 corotated sweep needs 134-156 VGPRs: at 448 threads one block
// fills a compute unit; 512 threads capped at four waves per SIMD keep two.
template <>
struct GradBlock<double, kModelCorot> {
  static constexpr int value = 512, min_waves = 4;
};

template <typename R>
__device__ __forceinline__ double4* xbuf(const Args<R>& A, int k) { return (k & 1) ? A.x1 : A.x0; }
template <typename R>
__device__ __forceinline__ R4<R>* pbuf(const Args<R>& A, int k) { return (k & 1) ? A.p1 : A.p0; }

// --------------------------------------------------------------- predict
// xt = x^t + h v^t + h^2 g (Sec. 3); x_0 = x^t with prescribed vertices at
// their targets (Algorithm 1, first line).  With A.carry, each block also
// leaves in part_dir[4 b + 3] the largest distance of its surface vertices
// from the positions the current candidate list was built at.
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_predict(Args<R> A, const double* x_in, const double* v_in, double3 grav) {
  __shared__ double sh[kSWaves];
  double dmax = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StepStatus* s = A.status;
    s->stopped = 0; s->final_k = 0; s->iters = 0; s->reason = 2; s->paused_at = -1; s->err = 0;
    s->a_up_hits = 0; s->g0 = 0; s->gk = 0; s->dE0 = 0; s->last_dE = 0; s->n_active = 0;
  }
  if (A.split && blockIdx.x == 0)
    for (int i = threadIdx.x; i < 2 * A.nObj; i += kSBlock) A.opair[i] = 0.0;
  for (int v = blockIdx.x * kSBlock + threadIdx.x; v < A.nV; v += gridDim.x * kSBlock) {
    V3<double> x = mk3(x_in[3 * v], x_in[3 * v + 1], x_in[3 * v + 2]);
    V3<double> vel = mk3(v_in[3 * v], v_in[3 * v + 1], v_in[3 * v + 2]);
    if (!(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(vel.x) && isfinite(vel.y) && isfinite(vel.z)))
      raise_err(A.status, kErrNonfinite);
    st3(A.xstart, v, x);
    V3<double> xt = x + A.h * vel;
    xt = xt + A.h2 * mk3(grav.x, grav.y, grav.z);
    st3(A.xt, v, xt);
    if (A.vflag[v] & kFixed) x = ld3(A.target, v);
    st3(A.x0, v, x);
    str<R>(A.g, v, mk3(R(0), R(0), R(0)));
    str<R>(A.p0, v, mk3(R(0), R(0), R(0)));
    if (A.self) {
#pragma unroll
      for (int j = 0; j < 6; ++j) A.acc[8 * v + j] = 0.0;
      if (A.carry && (A.vflag[v] & kSurface)) {
        const V3<double> xb = ld3(A.xbuild, v);
        const double ex = x.x - xb.x, ey = x.y - xb.y, ez = x.z - xb.z;
        dmax = fmax(dmax, sqrt(ex * ex + ey * ey + ez * ez));
      }
    }
  }
  if (A.self && A.carry) {
    dmax = wave_max(dmax);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = sh[0];
      for (int w = 1; w < kSWaves; ++w) m = fmax(m, sh[w]);
      A.part_dir[4 * blockIdx.x + 3] = m;
    }
  }
}

// ------------------------------------------------ first-launch prologue
enum FirstMode { kModeNormal = 0, kModeFinish = 1, kModeResume = 2 };

struct FirstPro {
  double alpha;
  int materialize;   // apply x_k = x_{k-1} + alpha p_k in this launch
  int work;          // evaluate the iteration's terms at x_k
};

// Sums (kind 0) or maxima (kind 1) of N per-object values over all objects,
// by the block's first wave (lane l takes objects l, l + 64, ...) in a fixed
// order, then handed to every thread through LDS.  Called by all threads.
template <int N, typename F>
__device__ __forceinline__ void over_objects(int nObj, const int (&kind)[N], F&& get, double (&out)[N],
                                             double* sh) {
  if (threadIdx.x < kWave) {
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0.0;
    for (int o = threadIdx.x; o < nObj; o += kWave) {
      double val[N];
      get(o, val);
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = kind[i] ? fmax(acc[i], val[i]) : acc[i] + val[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      acc[i] = kind[i] ? wave_max(acc[i]) : wave_sum(acc[i]);
      if (threadIdx.x == 0) sh[i] = acc[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = sh[i];
  __syncthreads();
}

// SPLIT: one step size per object (Sec. 5.2), taken from the per-object
// scalars of iteration k - 1; dE is their sum and the displacement bound
// grows by the largest alpha_o max_{v in o} |p_v|.
template <typename R, bool SPLIT, int BS = kSBlock>
__device__ FirstPro first_prologue(const Args<R>& A, int k, int mode, double* sh) {
  FirstPro fp{0.0, 0, 1};
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  if (k == 0 || mode == kModeResume) {
    // a step that starts on an earlier step's list first checks that x_0 is
    // within half the skin of the list's build positions, else it pauses
    // here for a rebuild at x_0 (and resumes at iteration 0)
    double D0 = 0.0;
    int pause = 0;
    if (k == 0 && mode == kModeNormal && A.self && A.carry) {
      const int kind[1] = {1};
      double r[1];
      reduce_partials<1, BS>(A.part_dir + 3, 4, A.grid, kind, r, sh);
      D0 = r[0];
      pause = D0 > 0.5 * A.skin ? 1 : 0;
    }
    if (leader) {
      IterScal& s = A.scal[k];
      if (k == 0) {
        s.alpha = 0; s.dE = 0; s.dE0 = 0; s.a_up = 0;
      }
      s.D = 0; s.stop = 0; s.pause = pause;
      A.status->paused_at = pause ? 0 : -1;
      A.status->D = D0;
    }
    if (pause) fp.work = 0;
    return fp;
  }
  const IterScal prev = A.scal[k - 1];
  if (prev.stop || prev.dir_stop || prev.pause) {
    if (leader) { A.scal[k].stop = 1; A.scal[k].pause = 0; }
    fp.work = 0;
    return fp;
  }
  double alpha = 0.0, dE = 0.0, dmove = 0.0;
  int hits = 0;
  bool unbounded = false;
  if (!SPLIT) {
    const int kind[3] = {0, 1, 1};
    double r[3];
    reduce_partials<3, BS>(A.part_dir, 4, A.grid, kind, r, sh);
    const double pHp = r[0], pmv = r[1], pmc = r[2];
    const double gTp = prev.gTp;
    const double abar = pHp > 0.0 ? -gTp / pHp : HUGE_VAL;
    const double pm = (A.flags & 2u) ? pmc : pmv;
    const double aup = (A.has_prims && pm > 0.0) ? A.dhat / (2.0 * pm) : HUGE_VAL;
    alpha = fmin(aup, abar);
    hits = aup < abar ? 1 : 0;
    unbounded = !isfinite(alpha);
    dE = -alpha * gTp - 0.5 * alpha * alpha * pHp;
    dmove = alpha * pmv;
  } else {
    const ObjScal* os = A.oscal + (size_t)(k - 1) * A.nObj;
    const int kind[4] = {0, 0, 1, 1};
    double r[4];
    over_objects<4>(A.nObj, kind, [&](int o, double (&val)[4]) {
      const ObjScal q = os[o];
      val[0] = q.moving ? q.dE : 0.0;
      val[1] = q.moving ? double(q.a_up) : 0.0;
      val[2] = q.moving ? q.alpha * q.pmv : 0.0;
      val[3] = (q.moving && !isfinite(q.alpha)) ? 1.0 : 0.0;
    }, r, sh);
    dE = r[0];
    hits = int(r[1]);
    dmove = r[2];
    unbounded = r[3] > 0.0;
  }
  IterScal s{};
  s.a_up = prev.a_up + hits;
  if (unbounded) {
    if (leader) {
      s.alpha = 0; s.dE = 0; s.dE0 = prev.dE0; s.D = prev.D; s.stop = 1; s.pause = 0;
      A.scal[k].alpha = s.alpha; A.scal[k].dE = 0; A.scal[k].dE0 = s.dE0; A.scal[k].D = s.D;
      A.scal[k].stop = 1; A.scal[k].pause = 0; A.scal[k].a_up = s.a_up;
      StepStatus* st = A.status;
      st->stopped = 1; st->final_k = k - 1; st->iters = k - 1; st->reason = 3;
      st->gk = prev.gnorm; st->dE0 = prev.dE0; st->last_dE = prev.dE; st->a_up_hits = prev.a_up;
      st->n_active = prev.n_active;
    }
    fp.work = 0;
    return fp;
  }
  const double dE0 = (k == 1) ? dE : prev.dE0;
  // displacement of any surface vertex since the list build: exact at x_{k-1}
  // (measured by the gradient sweep) plus at most alpha |p|_max this update
  const double D = (A.self ? prev.Dx : prev.D) + dmove;
  int stop = 0, reason = 0;
  if (A.term == 0 && dE < A.eps * dE0) { stop = 1; reason = 0; }
  else if (mode == kModeFinish) { stop = 1; reason = 2; }
  const int pause = (!stop && A.self && D > 0.5 * A.skin) ? 1 : 0;
  if (leader) {
    IterScal& o = A.scal[k];
    o.alpha = alpha; o.dE = dE; o.dE0 = dE0; o.D = D; o.stop = stop; o.pause = pause; o.a_up = s.a_up;
    o.dir_stop = 0;
    if (stop) {
      StepStatus* st = A.status;
      st->stopped = 1; st->final_k = k; st->iters = k; st->reason = reason;
      st->gk = prev.gnorm; st->dE0 = dE0; st->last_dE = dE; st->a_up_hits = s.a_up;
      st->n_active = prev.n_active;
    }
    if (pause) A.status->paused_at = k;
    A.status->D = D;
  }
  fp.alpha = alpha;
  fp.materialize = 1;
  fp.work = (stop || pause) ? 0 : 1;
  return fp;
}

// Reader of the positions of iteration k in the first launch (lazy when the
// launch also applies the update) and the update itself.
template <typename R, bool SPLIT>
struct FirstPos {
  using type = PosReader<R>;
};
template <typename R>
struct FirstPos<R, true> {
  using type = PosReaderSplit<R>;
};

template <typename R, bool SPLIT>
__device__ __forceinline__ typename FirstPos<R, SPLIT>::type first_pos(const Args<R>& A, int k, const FirstPro& fp,
                                                                       const double4* xsrc, const R4<R>* pk) {
  if constexpr (SPLIT)
    return PosReaderSplit<R>{xsrc, pk, A.oscal + (size_t)(k > 0 ? k - 1 : 0) * A.nObj, A.vobj, fp.materialize};
  else
    return PosReader<R>{xsrc, pk, fp.alpha, fp.materialize};
}

// x_k = x_{k-1} + alpha p_k on this block's vertex slice.
template <typename R, bool SPLIT, int BS = kSBlock>
__device__ __forceinline__ void apply_update(const Args<R>& A, int k, const FirstPro& fp, double4* xcur,
                                             const double4* xprev, const R4<R>* pk) {
  const auto pos = first_pos<R, SPLIT>(A, k, fp, xprev, pk);
  const Slice sv = block_slice(A.nV);
  for (int v = (int)sv.begin + threadIdx.x; v < sv.end; v += BS) st3(xcur, v, pos(v));
}

// ----------------------------------------------------------- narrow phase
// One candidate pair at positions from `pos`: closest points (Sec. 3.2),
// returns false if inactive.  Penetration raises the error bit.
template <typename R, typename Pos>
__device__ __forceinline__ bool pair_closest(const Args<R>& A, int q, const Pos& pos, int (&iv)[4], Closest& c,
                                             long long npt) {
  V3<double> X[4];
  if (A.pv) {
    // the pair index holds the corner vertices: one load fewer on the way
    // to the positions
    const int4 w = A.pv[q];
    iv[0] = w.x; iv[1] = w.y; iv[2] = w.z; iv[3] = w.w >= 0 ? w.w : ~w.w;
#pragma unroll
    for (int i = 0; i < 4; ++i) X[i] = pos(iv[i]);
    c = w.w >= 0 ? closest_pt(X[0], X[1], X[2], X[3]) : closest_ee(X[0], X[1], X[2], X[3]);
    if (!(c.d > 0.0)) {
      raise_err(A.status, kErrPenetration);
      return false;
    }
    return c.d < A.dhat;
  }
  int2 pr = A.cand[q];
  // kind: by position in a sorted list (npt >= 0), or in the pair itself
  // (npt < 0: edge-edge pairs are stored as (e1, ~e2))
  if (npt >= 0 ? q < npt : pr.y >= 0) {
    iv[0] = pr.x;
    iv[1] = A.tris[3 * pr.y]; iv[2] = A.tris[3 * pr.y + 1]; iv[3] = A.tris[3 * pr.y + 2];
#pragma unroll
    for (int i = 0; i < 4; ++i) X[i] = pos(iv[i]);
    c = closest_pt(X[0], X[1], X[2], X[3]);
  } else {
    const int e2 = pr.y >= 0 ? pr.y : ~pr.y;
    iv[0] = A.edges[2 * pr.x]; iv[1] = A.edges[2 * pr.x + 1];
    iv[2] = A.edges[2 * e2]; iv[3] = A.edges[2 * e2 + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) X[i] = pos(iv[i]);
    c = closest_ee(X[0], X[1], X[2], X[3]);
  }
  if (!(c.d > 0.0)) {
    raise_err(A.status, kErrPenetration);
    return false;
  }
  return c.d < A.dhat;
}

// coefficient of (J t)(J t)^T and of J J^T in kappa * d2b/dx2 (eq9, or its
// PSD projection (b''/d^2)(J t)(J t)^T when not BARRIER_FULL)
template <typename R>
__device__ __forceinline__ void pair_hess_coefs(const Args<R>& A, double d, double& ca, double& cb) {
  const double b1 = barrier_db(d, A.dhat), b2 = barrier_d2b(d, A.dhat);
  if (A.flags & 1u) {
    ca = A.kappa * (b2 / (d * d) - b1 / (d * d * d));
    cb = A.kappa * b1 / d;
  } else {
    ca = A.kappa * b2 / (d * d);
    cb = 0.0;
  }
}

// Calls f(q) for the candidate pairs of this block: a contiguous slice of
// the list (atomic scatter), or, with the segmented scatter, the pairs named
// by the corner-0 entries of a slice of the per-vertex entry index, whose
// order does not depend on the list's order (so sums over pairs are
// reproducible).
template <typename R, int BS, typename F>
__device__ __forceinline__ void for_each_pair(const Args<R>& A, F&& f) {
  const long long nq = min(A.ncand[0], A.cand_cap);
  if (A.seg) {
    const Slice se = block_slice(4 * nq);
    for (long long j = se.begin + threadIdx.x; j < se.end; j += BS) {
      const int sl = A.cent[j];
      if ((sl & 3) == 0) f(sl >> 2);
    }
  } else {
    const Slice sq = block_slice(nq);
    for (long long q = sq.begin + threadIdx.x; q < sq.end; q += BS) f((int)q);
  }
}

// Barrier gradient and diagonal at corner i of an active pair (eq8, eq10,
// eq11): val = {g xyz, diag xyz}.
template <typename R>
__device__ __forceinline__ void pair_grad_diag_corner(const Args<R>& A, const Closest& c, int i, double (&val)[6]) {
  const double d = c.d;
  const double cg = A.kappa * barrier_db(d, A.dhat) / d;
  double ca, cb;
  pair_hess_coefs(A, d, ca, cb);
  const double ci = c.c[i];
  const double tx = ci * c.t.x, ty = ci * c.t.y, tz = ci * c.t.z;
  const double dj = cb * ci * ci;
  val[0] = cg * tx; val[1] = cg * ty; val[2] = cg * tz;
  val[3] = ca * tx * tx + dj; val[4] = ca * ty * ty + dj; val[5] = ca * tz * tz + dj;
}

// (H p) at corner i of an active pair and the pair's p^T H p (eq12, eq13):
// (H p)_i = c_i [ca (t . sp) t + cb sp] with sp = sum_k c_k p_k.
template <typename R>
__device__ __forceinline__ double pair_hp_corner(const Args<R>& A, const Closest& c, const int (&iv)[4], int i,
                                                 double (&val)[3]) {
  double ca, cb;
  pair_hess_coefs(A, c.d, ca, cb);
  V3<double> sp = mk3(0.0, 0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) sp = sp + c.c[k] * cast3<double>(ldr<R>(A.p0, iv[k]));
  const double st = dot(sp, c.t);
  const double ci = c.c[i];
  val[0] = ci * (ca * st * c.t.x + cb * sp.x);
  val[1] = ci * (ca * st * c.t.y + cb * sp.y);
  val[2] = ci * (ca * st * c.t.z + cb * sp.z);
  return ca * st * st + cb * dot(sp, sp);
}

// Atomic scatter: the gradient and diagonal of an active pair added to its
// corners' accumulators.
template <typename R>
__device__ __forceinline__ void pair_grad_diag_atomic(const Args<R>& A, const int (&iv)[4], const Closest& c) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double val[6];
    pair_grad_diag_corner(A, c, i, val);
    double* a = A.acc + 8 * (size_t)iv[i];
#pragma unroll
    for (int j = 0; j < 6; ++j) atomicAdd(a + j, val[j]);
  }
}

// Segmented scatter: the corner entries (grouped by vertex) of this block's
// 64-entry chunks, one per lane; each lane evaluates its pair at `pos` (the
// four entries of a pair evaluate it alike) and its corner's terms, a
// wave-segmented sum reduces each vertex run and the run's last lane
// stores the run partial in A.rp.  WHAT 0: gradient and diagonal (6 values);
// WHAT 2: H p (3 values, p in A.p0) and p^T H p counted once per pair.
// Returns this thread's count of active pairs (WHAT 0) or its p^T H p sum
// (WHAT 2).
template <typename R, int WHAT, int BS, typename Pos>
__device__ __forceinline__ double pair_entries(const Args<R>& A, const Pos& pos) {
  constexpr int N = WHAT == 0 ? 6 : 3;
  const int lane = threadIdx.x & (kWave - 1);
  const long long nq = min(A.ncand[0], A.cand_cap), npt = A.ncand[1];
  const long long nent = 4 * nq;
  const Slice sc = block_slice((nent + kWave - 1) / kWave);
  double acc = 0.0;
  for (long long m = sc.begin + (threadIdx.x >> 6); m < sc.end; m += BS / kWave) {
    const long long j = m * kWave + lane;
    double val[N];
#pragma unroll
    for (int i = 0; i < N; ++i) val[i] = 0.0;
    int key = -1 - lane;   // distinct keys for lanes past the end
    if (j < nent) {
      const int sl = A.cent[j];
      const int q = sl >> 2, ci = sl & 3;
      int iv[4];
      Closest c;
      const bool act = pair_closest(A, q, pos, iv, c, npt);
      key = iv[ci];
      if (act) {
        if constexpr (WHAT == 0) {
          pair_grad_diag_corner(A, c, ci, val);
          if (ci == 0) acc += 1.0;
        } else {
          const double php = pair_hp_corner(A, c, iv, ci, val);
          if (ci == 0) acc += php;
        }
      }
    }
    const bool last = seg_sum(key, val);
    if (j < nent && last) {
      double* o = A.rp + 6 * (size_t)j;
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] = val[i];
    }
  }
  return acc;
}

// First launch of an iteration with self contact: apply the pending update,
// then barrier gradient + diagonal of every active pair into acc (eq8,
// eq10, eq11).
template <typename R, bool SPLIT>
__global__ void __launch_bounds__(kSBlock) k_narrow(Args<R> A, int k, int mode) {
  __shared__ double sh[kSWaves * 8];
  FirstPro fp = first_prologue<R, SPLIT>(A, k, mode, sh);
  double4* xcur = xbuf(A, k);
  const double4* xprev = xbuf(A, k - 1);
  const R4<R>* pk = pbuf(A, k);
  if (fp.materialize) apply_update<R, SPLIT>(A, k, fp, xcur, xprev, pk);
  if (!fp.work) return;
  const auto pos = first_pos<R, SPLIT>(A, k, fp, fp.materialize ? xprev : xcur, pk);
  double nact = 0.0;
  if (A.seg) {
    nact = pair_entries<R, 0, kSBlock>(A, pos);
  } else {
    const long long nq = min(A.ncand[0], A.cand_cap), npt = A.ncand[1];
    const Slice sq = block_slice(nq);
    for (long long q = sq.begin + threadIdx.x; q < sq.end; q += kSBlock) {
      int iv[4];
      Closest c;
      if (!pair_closest(A, (int)q, pos, iv, c, npt)) continue;
      nact += 1.0;
      pair_grad_diag_atomic(A, iv, c);
    }
  }
  double v[1] = {nact};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) A.part_narrow[blockIdx.x] = v[0];
}

// The pair pass folded into the first launch of the sweep (segmented
// scatter, unsplit step): the corner entries of this block's vertices,
// [wrange[first wave].x, wrange[last wave].y), evaluated at `pos` 64 to a
// wave in the 64-entry chunks of the global entry index that pair_entries
// uses, so every run partial is the same number it computes.  Entries of
// another block's vertices in a shared chunk are left out: their runs are
// that block's.  Returns this thread's count of active pairs (each pair
// counted at its corner-0 entry, which lies in exactly one block).
template <typename R, int BS, typename Pos>
__device__ __forceinline__ double block_pair_entries(const Args<R>& A, const Pos& pos, const Slice& swv) {
  if (swv.begin >= swv.end) return 0.0;
  const int lane = threadIdx.x & (kWave - 1);
  const long long npt = A.ncand[1];
  const int e0 = A.wrange[swv.begin].x, e1 = A.wrange[swv.end - 1].y;
  double acc = 0.0;
  if (e0 >= e1) return 0.0;
  for (int m = (e0 >> 6) + (int)(threadIdx.x >> 6); m <= ((e1 - 1) >> 6); m += BS / kWave) {
    const int j = m * kWave + lane;
    const bool mine = j >= e0 && j < e1;
    double val[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int key = -1 - lane;   // distinct keys for lanes outside the range
    if (mine) {
      const int sl = A.cent[j];
      const int q = sl >> 2, ci = sl & 3;
      int iv[4];
      Closest c;
      const bool act = pair_closest(A, q, pos, iv, c, npt);
      key = iv[ci];
      if (act) {
        pair_grad_diag_corner(A, c, ci, val);
        if (ci == 0) acc += 1.0;
      }
    }
    const bool last = seg_sum(key, val);
    if (mine && last) {
      double* o = A.rp + 6 * (size_t)j;
#pragma unroll
      for (int i = 0; i < 6; ++i) o[i] = val[i];
    }
  }
  return acc;
}

// ---------------------------------------------------- vertex-centric sweep
enum GradMode { kGradFirst = 0, kGradDirect = 1, kGradQuery = 2 };

// Element gradient and diagonal of one (tet, corner) lane under model M;
// false if the lane holds no tet.  Without the h^2 factor.
template <typename R, int M, typename Pos>
__device__ __forceinline__ bool lane_elem(const Args<R>& A, int code, const Pos& pos, V3<R>& g, V3<R>& dg) {
  if (code < 0) return false;
  const int e = code >> 2, a = code & 3;
  const ElemRec<R> rec = A.elem[e];
  Kin<R> kin = kinematics<R>(rec.B, pos(rec.v[0]), pos(rec.v[1]), pos(rec.v[2]), pos(rec.v[3]));
  if (!el_grad_diag<R, M>(kin, rec.vmu, rec.vlam, shape_vec(rec.B, a), g, dg)) {
    raise_err(A.status, kErrInverted);
    g = mk3(R(0), R(0), R(0));
    dg = g;
  }
  return true;
}

// Vertex terms at x_v: inertia m (x - xt), plane barriers (surface
// vertices), contact-pair sums (`pairs`: the segmented sums of the vertex's
// slots, or NULL for the atomic accumulators); returns g and diag in float64.
template <typename R>
__device__ __forceinline__ void vertex_terms(const Args<R>& A, int v, V3<double> x, double (&gd)[3], double (&dd)[3],
                                             double& nplane, bool zero_acc, const double* pairs = nullptr) {
  const double m = A.mass[v];
  V3<double> xt = ld3(A.xt, v);
  gd[0] += m * (x.x - xt.x); gd[1] += m * (x.y - xt.y); gd[2] += m * (x.z - xt.z);
  dd[0] += m; dd[1] += m; dd[2] += m;
  const uint8_t fl = A.vflag[v];
  if (fl & kSurface) {
    for (int j = 0; j < A.planes.n; ++j) {
      const double* pl = A.planes.p[j];
      const double d = plane_dist(pl, x);
      if (d < A.dhat) {
        if (!(d > 0.0)) { raise_err(A.status, kErrPenetration); continue; }
        const double b1 = A.kappa * barrier_db(d, A.dhat), b2 = A.kappa * barrier_d2b(d, A.dhat);
        gd[0] += b1 * pl[0]; gd[1] += b1 * pl[1]; gd[2] += b1 * pl[2];
        dd[0] += b2 * pl[0] * pl[0]; dd[1] += b2 * pl[1] * pl[1]; dd[2] += b2 * pl[2] * pl[2];
        nplane += 1.0;
      }
    }
  }
  if (A.self) {
    if (pairs) {
#pragma unroll
      for (int j = 0; j < 3; ++j) { gd[j] += pairs[j]; dd[j] += pairs[3 + j]; }
    } else {
      double* a = A.acc + 8 * v;
#pragma unroll
      for (int j = 0; j < 3; ++j) { gd[j] += a[j]; dd[j] += a[3 + j]; }
      if (zero_acc) {
#pragma unroll
        for (int j = 0; j < 6; ++j) a[j] = 0.0;
      }
    }
  }
}

// Gradient, diag(H) and the dot products for beta (Sec. 4.1-4.2).
// Mode kGradFirst: first launch of the iteration (no self contact): applies
// the pending update lazily.  kGradDirect: x_k already materialised.
// kGradQuery: writes g and diag to out_g / out_d (float64, [nV][3]).
// SPLIT: the beta dot products go per vertex to vdots (reduced per object
// by k_objred_grad) instead of into the block partials.
// SEG: the contact-pair terms come from the run partials of the segmented
// scatter instead of the atomic accumulators.  With kGradFirst (self
// contact, unsplit) the launch also computes those partials for its own
// vertices first (block_pair_entries), so an iteration is two launches.
template <typename R, int MODE, bool SPLIT = false, int M = kModelNH, bool SEG = false, int BS = GradBlock<R, M>::value>
__global__ void __launch_bounds__(BS, (GradBlock<R, M>::min_waves)) k_grad(Args<R> A, int k, int mode, double* out_g, double* out_d) {
  constexpr int NW = BS / kWave;
  constexpr bool FUSED = MODE == kGradFirst && SEG;
  __shared__ double sh[NW * 8];
  FirstPro fp{0.0, 0, 1};
  if (MODE == kGradFirst) {
    fp = first_prologue<R, SPLIT, BS>(A, k, mode, sh);
  } else if (MODE == kGradDirect) {
    const IterScal s = A.scal[k];
    if (s.stop || s.pause) return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const Slice swv = block_slice(A.nWaves);
  double4* xcur = MODE == kGradQuery ? A.x0 : xbuf(A, k);
  const double4* xprev = xbuf(A, k - 1);
  const R4<R>* pk = pbuf(A, k);
  if (MODE == kGradFirst && fp.materialize && !fp.work) {
    // stop test passed: only apply the last update
    apply_update<R, SPLIT, BS>(A, k, fp, xcur, xprev, pk);
    return;
  }
  if (!fp.work) return;
  const auto pos = first_pos<R, SPLIT>(A, k, fp, fp.materialize ? xprev : xcur, pk);
  double nact = 0.0;
  if constexpr (FUSED) {
    nact = block_pair_entries<R, BS>(A, pos, swv);
    __syncthreads();   // the block's run partials are in A.rp before its vertex lanes read them
  }
  double dots[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = (int)swv.begin + (threadIdx.x >> 6); w < swv.end; w += NW) {
    const int idx = w * kWave + lane;
    const int code = A.inc[idx];
    const int myv = A.inc_vert[idx];
    int2 wr = make_int2(0, 0);
    if constexpr (SEG) wr = wave_range(A.wrange, w);
    V3<R> g, dg;
    R s[6];
    if (lane_elem<R, M>(A, code, pos, g, dg)) {
      s[0] = g.x; s[1] = g.y; s[2] = g.z; s[3] = dg.x; s[4] = dg.y; s[5] = dg.z;
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) s[i] = R(0);
    }
    const bool vlane = seg_sum(myv, s) && myv >= 0;
    if (!vlane) continue;
    // this lane is the vertex's last lane
    const int v = myv;
    double prs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (SEG) {
      if (wr.x < wr.y) pair_partials_sum<6>(A.coff, A.rp, v, prs);
    }
    const V3<double> x = pos(v);
    if (MODE == kGradFirst && fp.materialize) st3(xcur, v, x);
    double gd[3] = {A.h2 * double(s[0]), A.h2 * double(s[1]), A.h2 * double(s[2])};
    double dd[3] = {A.h2 * double(s[3]), A.h2 * double(s[4]), A.h2 * double(s[5])};
    vertex_terms(A, v, x, gd, dd, dots[6], MODE != kGradQuery, SEG ? prs : nullptr);
    if ((MODE == kGradDirect || FUSED) && A.self && (A.vflag[v] & kSurface)) {
      const V3<double> xb = ld3(A.xbuild, v);
      const double ex = x.x - xb.x, ey = x.y - xb.y, ez = x.z - xb.z;
      dots[7] = fmax(dots[7], sqrt(ex * ex + ey * ey + ez * ez));
    }
    if (A.vflag[v] & kFixed) {
      gd[0] = gd[1] = gd[2] = 0.0;
      dd[0] = dd[1] = dd[2] = 1.0;
    }
    if (MODE == kGradQuery) {
#pragma unroll
      for (int j = 0; j < 3; ++j) { out_g[3 * v + j] = gd[j]; if (out_d) out_d[3 * v + j] = dd[j]; }
      continue;
    }
    V3<R> gR = mk3(R(gd[0]), R(gd[1]), R(gd[2]));
    V3<R> pgR = mk3(R(gd[0] / dd[0]), R(gd[1] / dd[1]), R(gd[2] / dd[2]));
    V3<R> gpR = ldr<R>(A.g, v);
    V3<R> ppR = ldr<R>(pk, v);
    str<R>(A.g, v, gR);
    str<R>(A.pg, v, pgR);
    const double g3[3] = {double(gR.x), double(gR.y), double(gR.z)};
    const double pg3[3] = {double(pgR.x), double(pgR.y), double(pgR.z)};
    const double gp3[3] = {double(gpR.x), double(gpR.y), double(gpR.z)};
    const double pp3[3] = {double(ppR.x), double(ppR.y), double(ppR.z)};
    if constexpr (SPLIT) {
      double vd[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double P = 1.0 / dd[j];
        const double y = g3[j] - gp3[j];
        vd[0] += g3[j] * g3[j];
        vd[1] += g3[j] * pg3[j];
        vd[2] += g3[j] * P * y;
        vd[3] += y * pp3[j];
        vd[4] += y * P * y;
        vd[5] += pp3[j] * g3[j];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) A.vdots[6 * (size_t)v + i] = vd[i];
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double P = 1.0 / dd[j];
        const double y = g3[j] - gp3[j];
        dots[0] += g3[j] * g3[j];
        dots[1] += g3[j] * pg3[j];
        dots[2] += g3[j] * P * y;
        dots[3] += y * pp3[j];
        dots[4] += y * P * y;
        dots[5] += pp3[j] * g3[j];
      }
    }
  }
  if (MODE == kGradQuery) return;
  const int kind[8] = {0, 0, 0, 0, 0, 0, 0, 1};
  block_reduce<8, BS>(dots, kind, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) A.part_grad[blockIdx.x * 8 + i] = dots[i];
  }
  if constexpr (FUSED) {
    double v[1] = {nact};
    const int kind1[1] = {0};
    block_reduce<1, BS>(v, kind1, sh);
    if (threadIdx.x == 0) A.part_narrow[blockIdx.x] = v[0];
  }
}

// ------------------------------------------------------ direction + pHp
// SPLIT: beta per object (from k_objred_grad), and the p^T H p terms go
// per tet, per vertex and per object (pairs) for k_objred_dir.
// Threads per block of the direction kernel.  With more than kSBlock, the
// first kSBlock threads take the tets while the waves beyond them take the
// vertices, so that the two passes' memory round trips overlap instead of
// adding up (pile: 12.6 -> 12.3 us float, 14.7 -> 14.3 us float64).  The
// float64 corotated instantiation keeps kSBlock threads doing both passes:
// with the split it measured 17.4 against 10.9 us on the 30,000-tet bar.
template <typename R, int M>
struct DirBlock {
  static constexpr int value = (sizeof(R) == sizeof(double) && M == kModelCorot) ? kSBlock : 384;
};

template <typename R, bool SPLIT = false, int M = kModelNH, int BS = DirBlock<R, M>::value>
__global__ void __launch_bounds__(BS) k_dir(Args<R> A, int k) {
  static_assert(BS >= kSBlock, "k_dir needs at least kSBlock threads");
  constexpr bool kSplitPasses = BS > kSBlock;
  __shared__ double sh[BS / kWave * 8];
  const IterScal s = A.scal[k];
  if (s.stop || s.pause) return;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  double r[8];
  {
    const int kind[8] = {0, 0, 0, 0, 0, 0, 0, 1};
    reduce_partials<8, BS>(A.part_grad, 8, A.grid, kind, r, sh);
  }
  double nact = r[6];
  if (A.self) {
    const int kind[1] = {0};
    double q[1];
    reduce_partials<1, BS>(A.part_narrow, 1, A.grid, kind, q, sh);
    nact += q[0];
  }
  const ObjScal* os = A.oscal + (size_t)k * A.nObj;
  double gg = r[0], gPg = r[1];
  int dir_stop = 0, reason = 0, restart = 0;
  double beta = 0.0, gTp = 0.0;
  bool any_dir = false;
  if constexpr (SPLIT) {
    const int kind[4] = {0, 0, 0, 1};
    double q[4];
    over_objects<4>(A.nObj, kind, [&](int o, double (&val)[4]) {
      const ObjScal w = os[o];
      val[0] = w.gg;
      val[1] = w.gPg;
      val[2] = w.gTp;
      val[3] = w.gTp != 0.0 ? 1.0 : 0.0;
    }, q, sh);
    gg = q[0]; gPg = q[1]; gTp = q[2];
    any_dir = q[3] > 0.0;
  }
  const double gnorm = sqrt(gg);
  const double g0 = k == 0 ? gnorm : A.status->g0;
  if ((A.term == 1 && gnorm <= A.eps * g0) || (A.term == 2 && gnorm <= A.eps)) { dir_stop = 1; reason = 1; }
  if constexpr (!SPLIT) {
    const double gPy = r[2], yp = r[3], yPy = r[4], pg = r[5];
    if (k > 0) {
      const IterScal sp = A.scal[k - 1];
      beta = beta_rule(A.flags, gPg, gPy, yp, yPy, pg, sp.gPg, sp.gTp);
    }
    gTp = -gPg + beta * pg;
    if (!(gTp < 0.0)) {
      restart = 1;
      beta = 0.0;
      gTp = -gPg;
    }
    any_dir = gTp != 0.0;
  }
  if (!dir_stop && !any_dir) { dir_stop = 1; reason = 3; }
  if (leader) {
    IterScal& o = A.scal[k];
    o.beta = beta; o.gTp = gTp; o.gnorm = gnorm; o.dir_stop = dir_stop; o.restart = restart; o.n_active = nact;
    o.gPg = gPg;
    o.Dx = r[7];
    if (k == 0) A.status->g0 = gnorm;
    if (dir_stop) {
      StepStatus* st = A.status;
      st->stopped = 1; st->final_k = k; st->iters = k; st->reason = reason;
      st->gk = gnorm; st->dE0 = s.dE0; st->last_dE = s.dE; st->a_up_hits = s.a_up; st->n_active = nact;
    }
  }
  if (dir_stop) return;
  auto beta_of = [&](int v) -> R {
    if constexpr (SPLIT) return R(os[A.vobj[v]].beta);
    else return R(beta);
  };
  const double4* xk = xbuf(A, k);
  const R4<R>* pk = pbuf(A, k);
  R4<R>* pn = pbuf(A, k + 1);
  double acc_pHp = 0.0, pmv = 0.0, pmc = 0.0;
  // tets: element p^T H p with p recomputed at the four corners
  double el = 0.0;
  const Slice st = block_slice(A.nT);
  const bool tet_thread = !kSplitPasses || threadIdx.x < kSBlock;
  for (int e = (int)st.begin + threadIdx.x; tet_thread && e < st.end; e += kSBlock) {
    const ElemRec<R> rec = A.elem[e];
    const R rb = beta_of(rec.v[0]);      // a tet lies in one object
    V3<R> P[4];
    V3<double> X[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = rec.v[i];
      X[i] = ld3(xk, v);
      P[i] = direction(ldr<R>(A.pg, v), ldr<R>(pk, v), rb);
    }
    Kin<R> kin = kinematics<R>(rec.B, X[0], X[1], X[2], X[3]);
    V3<R> d[3];
    dF_cols(rec.B, P[0], P[1], P[2], P[3], d);
    R ph = R(0);
    if (!el_pHp<R, M>(kin, rec.vmu, rec.vlam, d, ph)) raise_err(A.status, kErrInverted);
    if constexpr (SPLIT) A.tphp[e] = A.h2 * double(ph);
    else el += double(ph);
  }
  acc_pHp += A.h2 * el;
  // vertices: store p_{k+1}; inertia and plane parts of p^T H p; |p| maxima
  const Slice sv = block_slice(A.nV);
  const bool vert_thread = !kSplitPasses || !tet_thread;
  const int vt = kSplitPasses ? (int)threadIdx.x - kSBlock : (int)threadIdx.x;
  for (int v = (int)sv.begin + vt; vert_thread && v < sv.end; v += kSplitPasses ? BS - kSBlock : BS) {
    V3<R> p = direction(ldr<R>(A.pg, v), ldr<R>(pk, v), beta_of(v));
    str<R>(pn, v, p);
    const double px = p.x, py = p.y, pz = p.z;
    const double p2 = px * px + py * py + pz * pz;
    double vp = A.mass[v] * p2;
    if ((A.vflag[v] & kSurface) && A.planes.n > 0) {
      const V3<double> x = ld3(xk, v);
      for (int j = 0; j < A.planes.n; ++j) {
        const double* pl = A.planes.p[j];
        const double d = plane_dist(pl, x);
        if (d > 0.0 && d < A.dhat) {
          const double np = pl[0] * px + pl[1] * py + pl[2] * pz;
          vp += A.kappa * barrier_d2b(d, A.dhat) * np * np;
        }
      }
    }
    const double pabs = sqrt(p2), pcomp = fmax(fabs(px), fmax(fabs(py), fabs(pz)));
    if constexpr (SPLIT) {
      A.vphp[3 * (size_t)v] = vp;
      A.vphp[3 * (size_t)v + 1] = pabs;
      A.vphp[3 * (size_t)v + 2] = pcomp;
    } else {
      acc_pHp += vp;
      pmv = fmax(pmv, pabs);
      pmc = fmax(pmc, pcomp);
    }
  }
  // pairs: kappa [ca (sum_i c_i p_i . t)^2 + cb |sum_i c_i p_i|^2] (eq12, eq13);
  // split: each object's side of the pair with the other side's p left out
  if (A.self) {
    PosReader<R> pos{xk, pk, 0.0, 0};
    const long long npt = A.ncand[1];
    for_each_pair<R, BS>(A, [&](int q) {
      int iv[4];
      Closest c;
      if (!pair_closest(A, q, pos, iv, c, npt)) return;
      double ca, cb;
      pair_hess_coefs(A, c.d, ca, cb);
      if constexpr (SPLIT) {
        const int oa = A.vobj[iv[0]];
        int ob = -1;
        V3<double> sa = mk3(0.0, 0.0, 0.0), sb = mk3(0.0, 0.0, 0.0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int oi = A.vobj[iv[i]];
          const V3<double> cp = c.c[i] * cast3<double>(direction(ldr<R>(A.pg, iv[i]), ldr<R>(pk, iv[i]), beta_of(iv[i])));
          if (oi == oa) {
            sa = sa + cp;
          } else {
            sb = sb + cp;
            ob = oi;
          }
        }
        double* op = A.opair + (size_t)(k & 1) * A.nObj;
        const double ta = dot(sa, c.t);
        atomicAdd(op + oa, ca * ta * ta + cb * dot(sa, sa));
        if (ob >= 0) {
          const double tb = dot(sb, c.t);
          atomicAdd(op + ob, ca * tb * tb + cb * dot(sb, sb));
        }
      } else {
        V3<double> sp = mk3(0.0, 0.0, 0.0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          V3<R> p = direction(ldr<R>(A.pg, iv[i]), ldr<R>(pk, iv[i]), beta_of(iv[i]));
          sp = sp + c.c[i] * cast3<double>(p);
        }
        const double st = dot(sp, c.t);
        acc_pHp += ca * st * st + cb * dot(sp, sp);
      }
    });
  }
  if constexpr (SPLIT) return;
  double v[3] = {acc_pHp, pmv, pmc};
  const int kind[3] = {0, 1, 1};
  block_reduce<3, BS>(v, kind, sh);
  if (threadIdx.x == 0) {
    A.part_dir[blockIdx.x * 4 + 0] = v[0];
    A.part_dir[blockIdx.x * 4 + 1] = v[1];
    A.part_dir[blockIdx.x * 4 + 2] = v[2];
  }
}

// ------------------------------------------------- split: object reductions
// One block per object: the object's beta dot products (from vdots) give
// its beta by the solver's rule, the restart test and g_o^T p_o (Sec. 5.2).
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_objred_grad(Args<R> A, int k) {
  __shared__ double sh[kSWaves * 6];
  const IterScal s = A.scal[k];
  if (s.stop || s.pause) return;
  const int o = blockIdx.x;
  double d[6] = {0, 0, 0, 0, 0, 0};
  const int v0 = A.voff[o], v1 = A.voff[o + 1];
  int v = v0 + threadIdx.x;
  for (; v + 3 * kSBlock < v1; v += 4 * kSBlock) {   // four independent loads in flight
    double t[4][6];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < 6; ++i) t[u][i] = A.vdots[6 * (size_t)(v + u * kSBlock) + i];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < 6; ++i) d[i] += t[u][i];
  }
  for (; v < v1; v += kSBlock)
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] += A.vdots[6 * (size_t)v + i];
  const int kind[6] = {0, 0, 0, 0, 0, 0};
  block_reduce<6>(d, kind, sh);
  if (threadIdx.x != 0) return;
  const double gg = d[0], gPg = d[1], gPy = d[2], yp = d[3], yPy = d[4], pg = d[5];
  double beta = 0.0;
  if (k > 0) {
    const ObjScal q = A.oscal[(size_t)(k - 1) * A.nObj + o];
    beta = beta_rule(A.flags, gPg, gPy, yp, yPy, pg, q.gPg, q.gTp);
  }
  double gTp = -gPg + beta * pg;
  if (!(gTp < 0.0)) {
    beta = 0.0;
    gTp = -gPg;
  }
  ObjScal& w = A.oscal[(size_t)k * A.nObj + o];
  w.beta = beta; w.gTp = gTp; w.gPg = gPg; w.gg = gg;
}

// One block per object: its p^T H p (tets, vertices, pairs) and max |p_v|
// give its step size alpha_o = min(dhat / (2 max |p_v|), -g_o^T p_o / p_o^T H p_o)
// (equations upper, alpha) and its share of dE; an object whose direction is
// zero does not move.
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_objred_dir(Args<R> A, int k) {
  __shared__ double sh[kSWaves * 4];
  const IterScal s = A.scal[k];
  if (s.stop || s.pause || s.dir_stop) return;
  const int o = blockIdx.x;
  double r[4] = {0, 0, 0, 0};
  const int t0 = A.toff[o], t1 = A.toff[o + 1];
  int e = t0 + threadIdx.x;
  for (; e + 3 * kSBlock < t1; e += 4 * kSBlock) {   // four independent loads in flight
    const double a0 = A.tphp[e], a1 = A.tphp[e + kSBlock], a2 = A.tphp[e + 2 * kSBlock], a3 = A.tphp[e + 3 * kSBlock];
    r[0] += a0; r[0] += a1; r[0] += a2; r[0] += a3;
  }
  for (; e < t1; e += kSBlock) r[0] += A.tphp[e];
  const int v0 = A.voff[o], v1 = A.voff[o + 1];
  int v = v0 + threadIdx.x;
  for (; v + kSBlock < v1; v += 2 * kSBlock) {
    const double* a = A.vphp + 3 * (size_t)v;
    const double* b = A.vphp + 3 * (size_t)(v + kSBlock);
    const double a0 = a[0], a1 = a[1], a2 = a[2], b0 = b[0], b1 = b[1], b2 = b[2];
    r[1] += a0; r[1] += b0;
    r[2] = fmax(r[2], fmax(a1, b1));
    r[3] = fmax(r[3], fmax(a2, b2));
  }
  for (; v < v1; v += kSBlock) {
    r[1] += A.vphp[3 * (size_t)v];
    r[2] = fmax(r[2], A.vphp[3 * (size_t)v + 1]);
    r[3] = fmax(r[3], A.vphp[3 * (size_t)v + 2]);
  }
  const int kind[4] = {0, 0, 1, 1};
  block_reduce<4>(r, kind, sh);
  if (threadIdx.x != 0) return;
  double* op = A.opair + (size_t)(k & 1) * A.nObj + o;
  const double pHp = r[0] + r[1] + *op;
  *op = 0.0;   // ready for iteration k + 2
  ObjScal& w = A.oscal[(size_t)k * A.nObj + o];
  const double gTp = w.gTp, pmv = r[2], pm = (A.flags & 2u) ? r[3] : r[2];
  const int moving = pmv > 0.0 ? 1 : 0;
  const double abar = pHp > 0.0 ? -gTp / pHp : HUGE_VAL;
  const double aup = (A.has_prims && pm > 0.0) ? A.dhat / (2.0 * pm) : HUGE_VAL;
  const double alpha = moving ? fmin(aup, abar) : 0.0;
  w.alpha = alpha; w.pHp = pHp; w.pmv = pmv; w.moving = moving;
  w.a_up = (moving && aup < abar) ? 1 : 0;
  w.dE = moving ? -alpha * gTp - 0.5 * alpha * alpha * pHp : 0.0;
}

// --------------------------------------------------------------- finalize
// x^{t+1} and v^{t+1} (Sec. 3) from the final iteration, written only once
// the step has stopped without an error: the host may queue this launch
// behind the chunk that reaches the iteration cap before it knows whether
// the step pauses first or fails, and the outputs may be the step's own
// inputs, which a failed or paused step must leave untouched.
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_finalize(Args<R> A, double* x_out, double* v_out) {
  if (!A.status->stopped || A.status->err) return;
  const int fk = A.status->final_k;
  const double4* xf = xbuf(A, fk);
  const double ih = 1.0 / A.h;
  for (int v = blockIdx.x * kSBlock + threadIdx.x; v < A.nV; v += gridDim.x * kSBlock) {
    V3<double> x = ld3(xf, v), x0 = ld3(A.xstart, v);
    if (!(isfinite(x.x) && isfinite(x.y) && isfinite(x.z))) raise_err(A.status, kErrNonfinite);
    x_out[3 * v] = x.x; x_out[3 * v + 1] = x.y; x_out[3 * v + 2] = x.z;
    v_out[3 * v] = (x.x - x0.x) * ih; v_out[3 * v + 1] = (x.y - x0.y) * ih; v_out[3 * v + 2] = (x.z - x0.z) * ih;
  }
}

// ----------------------------------------------------------------- queries
// Load query positions (row-major [nV][3]) into x0 and the predictor into xt.
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_load_query(Args<R> A, const double* x, const double* xt, const double* p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) A.status->err = 0;
  for (int v = blockIdx.x * kSBlock + threadIdx.x; v < A.nV; v += gridDim.x * kSBlock) {
    V3<double> xv = mk3(x[3 * v], x[3 * v + 1], x[3 * v + 2]);
    if (!(isfinite(xv.x) && isfinite(xv.y) && isfinite(xv.z))) raise_err(A.status, kErrNonfinite);
    st3(A.x0, v, xv);
    if (xt) st3(A.xt, v, mk3(xt[3 * v], xt[3 * v + 1], xt[3 * v + 2]));
    if (p) {
      const bool fixed = A.vflag[v] & kFixed;
      str<R>(A.p0, v, fixed ? mk3(R(0), R(0), R(0)) : mk3(R(p[3 * v]), R(p[3 * v + 1]), R(p[3 * v + 2])));
    }
    if (A.self) {
#pragma unroll
      for (int j = 0; j < 8; ++j) A.acc[8 * v + j] = 0.0;
    }
  }
}

// Pair terms at x0 for queries: WHAT = 0 gradient + diag into acc, 1 energy
// partials, 2 H p into acc (acc[0..2]) and p^T H p partials (p in p0).
template <typename R, int WHAT>
__global__ void __launch_bounds__(kSBlock) k_pairs_query(Args<R> A, double* part) {
  __shared__ double sh[kSWaves * 2];
  PosReader<R> pos{A.x0, A.p0, 0.0, 0};
  const long long npt = A.ncand[1];
  double sum = 0.0;
  for_each_pair<R, kSBlock>(A, [&](int q) {
    int iv[4];
    Closest c;
    if (!pair_closest(A, q, pos, iv, c, npt)) return;
    const double d = c.d;
    if (WHAT == 1) {
      sum += A.kappa * barrier_b(d, A.dhat);
      return;
    }
    if (WHAT == 0) {
      pair_grad_diag_atomic(A, iv, c);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double val[3];
        const double php = pair_hp_corner(A, c, iv, i, val);
        if (i == 0) sum += php;
        double* a = A.acc + 8 * (size_t)iv[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) atomicAdd(a + j, val[j]);
      }
    }
  });
  double v[1] = {sum};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Segmented form of the gradient / H p pair queries at x0 (WHAT 0, 2):
// run partials into A.rp and per-block partials of the active-pair count or
// p^T H p.
template <typename R, int WHAT>
__global__ void __launch_bounds__(kSBlock) k_pairs_entries(Args<R> A, double* part) {
  __shared__ double sh[kSWaves * 2];
  PosReader<R> pos{A.x0, A.p0, 0.0, 0};
  double v[1] = {pair_entries<R, WHAT, kSBlock>(A, pos)};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Energy of elements, inertia and planes at x0 (partials per block).
template <typename R, int M>
__global__ void __launch_bounds__(kSBlock) k_energy(Args<R> A, double* part) {
  __shared__ double sh[kSWaves * 2];
  const int tid = blockIdx.x * kSBlock + threadIdx.x, stride = gridDim.x * kSBlock;
  double el = 0.0, vt = 0.0;
  for (int e = tid; e < A.nT; e += stride) {
    const ElemRec<R> rec = A.elem[e];
    Kin<R> kin = kinematics<R>(rec.B, ld3(A.x0, rec.v[0]), ld3(A.x0, rec.v[1]), ld3(A.x0, rec.v[2]), ld3(A.x0, rec.v[3]));
    R ee;
    if (!el_energy<R, M>(kin, rec.vmu, rec.vlam, ee)) { raise_err(A.status, kErrInverted); continue; }
    el += double(ee);
  }
  for (int v = tid; v < A.nV; v += stride) {
    V3<double> x = ld3(A.x0, v), xt = ld3(A.xt, v);
    V3<double> dx = x - xt;
    vt += 0.5 * A.mass[v] * dot(dx, dx);
    if (A.vflag[v] & kSurface) {
      for (int j = 0; j < A.planes.n; ++j) {
        const double d = plane_dist(A.planes.p[j], x);
        if (d < A.dhat) {
          if (!(d > 0.0)) { raise_err(A.status, kErrPenetration); continue; }
          vt += A.kappa * barrier_b(d, A.dhat);
        }
      }
    }
  }
  double v[1] = {A.h2 * el + vt};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// H p by the vertex-centric sweep (p in p0, prescribed rows zero) and the
// per-block partials of p^T H p.  Pair contributions must already be in acc.
template <typename R, int M, bool SEG = false>
__global__ void __launch_bounds__(kSBlock) k_hvp(Args<R> A, double* out_hp, double* part) {
  __shared__ double sh[kSWaves * 2];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = (blockIdx.x * kSBlock + threadIdx.x) >> 6;
  const int nw = (gridDim.x * kSBlock) >> 6;
  double php = 0.0;
  for (int w = wid; w < A.nWaves; w += nw) {
    const int idx = w * kWave + lane;
    const int code = A.inc[idx];
    const int myv = A.inc_vert[idx];
    int2 wr = make_int2(0, 0);
    if constexpr (SEG) wr = wave_range(A.wrange, w);
    R s[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if (code >= 0) {
      const int e = code >> 2, a = code & 3;
      const ElemRec<R> rec = A.elem[e];
      Kin<R> kin = kinematics<R>(rec.B, ld3(A.x0, rec.v[0]), ld3(A.x0, rec.v[1]), ld3(A.x0, rec.v[2]), ld3(A.x0, rec.v[3]));
      V3<R> d[3];
      dF_cols(rec.B, ldr<R>(A.p0, rec.v[0]), ldr<R>(A.p0, rec.v[1]), ldr<R>(A.p0, rec.v[2]), ldr<R>(A.p0, rec.v[3]), d);
      V3<R> hp;
      if (el_Hp<R, M>(kin, rec.vmu, rec.vlam, d, shape_vec(rec.B, a), hp)) {
        s[0] = hp.x; s[1] = hp.y; s[2] = hp.z;
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
    V3<R> pr = ldr<R>(A.p0, v);
    const double p3[3] = {double(pr.x), double(pr.y), double(pr.z)};
    double hv[3] = {A.h2 * double(s[0]), A.h2 * double(s[1]), A.h2 * double(s[2])};
    const double m = A.mass[v];
    for (int j = 0; j < 3; ++j) hv[j] += m * p3[j];
    if (A.vflag[v] & kSurface) {
      const V3<double> x = ld3(A.x0, v);
      for (int j = 0; j < A.planes.n; ++j) {
        const double* pl = A.planes.p[j];
        const double d = plane_dist(pl, x);
        if (d > 0.0 && d < A.dhat) {
          const double c = A.kappa * barrier_d2b(d, A.dhat) * (pl[0] * p3[0] + pl[1] * p3[1] + pl[2] * p3[2]);
          hv[0] += c * pl[0]; hv[1] += c * pl[1]; hv[2] += c * pl[2];
        }
      }
    }
    if (A.self) {
      if constexpr (SEG) {
        for (int j = 0; j < 3; ++j) hv[j] += prs[j];
      } else {
        for (int j = 0; j < 3; ++j) hv[j] += A.acc[8 * v + j];
      }
    }
    if (A.vflag[v] & kFixed) hv[0] = hv[1] = hv[2] = 0.0;
    php += hv[0] * p3[0] + hv[1] * p3[1] + hv[2] * p3[2];
    if (out_hp) {
      for (int j = 0; j < 3; ++j) out_hp[3 * v + j] = hv[j];
    }
  }
  double v[1] = {php};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Sum of n partials (one block), optionally plus `extra` partials.
__global__ void __launch_bounds__(kSBlock) k_sum_partials(const double* a, int na, const double* b, int nb, double* out) {
  __shared__ double sh[kSWaves * 1];
  double s = 0.0;
  for (int j = threadIdx.x; j < na; j += kSBlock) s += a[j];
  if (b)
    for (int j = threadIdx.x; j < nb; j += kSBlock) s += b[j];
  double v[1] = {s};
  const int kind[1] = {0};
  block_reduce<1>(v, kind, sh);
  if (threadIdx.x == 0) out[0] = v[0];
}

// ----------------------------------------------------------------- audit
// Minimum distance over candidate pairs (positions x0) and surface-vertex
// plane distances, and minimum det F; partials [grid][2] (min d, min J).
template <typename R>
__global__ void __launch_bounds__(kSBlock) k_audit(Args<R> A, double* part) {
  __shared__ double sh[kSWaves * 2];
  const int tid = blockIdx.x * kSBlock + threadIdx.x, stride = gridDim.x * kSBlock;
  double dmin = HUGE_VAL, jmin = HUGE_VAL;
  const long long nq = min(A.ncand[0], A.cand_cap), npt = A.ncand[1];
  for (long long q = tid; q < nq; q += stride) {
    int2 pr = A.cand[q];
    Closest c;
    if (q < npt) {
      c = closest_pt(ld3(A.x0, pr.x), ld3(A.x0, A.tris[3 * pr.y]), ld3(A.x0, A.tris[3 * pr.y + 1]),
                     ld3(A.x0, A.tris[3 * pr.y + 2]));
    } else {
      c = closest_ee(ld3(A.x0, A.edges[2 * pr.x]), ld3(A.x0, A.edges[2 * pr.x + 1]), ld3(A.x0, A.edges[2 * pr.y]),
                     ld3(A.x0, A.edges[2 * pr.y + 1]));
    }
    dmin = fmin(dmin, c.d);
  }
  for (int v = tid; v < A.nV; v += stride) {
    if (!(A.vflag[v] & kSurface)) continue;
    const V3<double> x = ld3(A.x0, v);
    for (int j = 0; j < A.planes.n; ++j) dmin = fmin(dmin, plane_dist(A.planes.p[j], x));
  }
  for (int e = tid; e < A.nT; e += stride) {
    const ElemRec<R> rec = A.elem[e];
    // det F in float64 regardless of R
    V3<double> X0 = ld3(A.x0, rec.v[0]);
    V3<double> e1 = ld3(A.x0, rec.v[1]) - X0, e2 = ld3(A.x0, rec.v[2]) - X0, e3 = ld3(A.x0, rec.v[3]) - X0;
    V3<double> f[3];
    for (int j = 0; j < 3; ++j) f[j] = double(rec.B[j]) * e1 + double(rec.B[3 + j]) * e2 + double(rec.B[6 + j]) * e3;
    jmin = fmin(jmin, dot(f[0], cross(f[1], f[2])));
  }
  double v[2] = {-dmin, -jmin};
  const int kind[2] = {1, 1};
  block_reduce<2>(v, kind, sh);
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = -v[0]; part[2 * blockIdx.x + 1] = -v[1]; }
}

// ============================================================== launchers

template <typename R>
void launch_predict(const Args<R>& A, const double* x, const double* v, double3 grav, hipStream_t s) {
  hipLaunchKernelGGL(k_predict<R>, dim3(A.grid), dim3(kSBlock), 0, s, A, x, v, grav);
}
// With splitting the gradient part of an iteration ends with the per-object
// beta reduction and the direction part with the per-object alpha reduction.
template <typename R>
void launch_iteration_first(const Args<R>& A, int k, int mode, hipStream_t s) {
  if (fused_pairs(A)) {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradFirst, false, M_, true>), dim3(A.grid),
                                              dim3(GradBlock<R, M_>::value), 0, s, A, k, mode, (double*)nullptr,
                                              (double*)nullptr));
  } else if (A.self) {
    if (A.split)
      hipLaunchKernelGGL((k_narrow<R, true>), dim3(A.grid), dim3(kSBlock), 0, s, A, k, mode);
    else
      hipLaunchKernelGGL((k_narrow<R, false>), dim3(A.grid), dim3(kSBlock), 0, s, A, k, mode);
  } else if (A.split) {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradFirst, true, M_>), dim3(A.grid),
                                              dim3(GradBlock<R, M_>::value), 0, s, A, k, mode, (double*)nullptr,
                                              (double*)nullptr));
    hipLaunchKernelGGL(k_objred_grad<R>, dim3(A.nObj), dim3(kSBlock), 0, s, A, k);
  } else {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradFirst, false, M_>), dim3(A.grid),
                                              dim3(GradBlock<R, M_>::value), 0, s, A, k, mode, (double*)nullptr,
                                              (double*)nullptr));
  }
}
template <typename R>
void launch_iteration_grad(const Args<R>& A, int k, hipStream_t s) {
  const bool seg = A.self && A.seg;
  if (A.split) {
    PNCG_BY_SCATTER(seg, PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradDirect, true, M_, S_>), dim3(A.grid),
                                              dim3(GradBlock<R, M_>::value), 0, s, A, k, 0, (double*)nullptr,
                                              (double*)nullptr)));
    hipLaunchKernelGGL(k_objred_grad<R>, dim3(A.nObj), dim3(kSBlock), 0, s, A, k);
  } else {
    PNCG_BY_SCATTER(seg, PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradDirect, false, M_, S_>), dim3(A.grid),
                                              dim3(GradBlock<R, M_>::value), 0, s, A, k, 0, (double*)nullptr,
                                              (double*)nullptr)));
  }
}
template <typename R>
void launch_iteration_dir(const Args<R>& A, int k, hipStream_t s) {
  if (A.split) {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_dir<R, true, M_>), dim3(A.grid), dim3(DirBlock<R, M_>::value), 0, s, A, k));
    hipLaunchKernelGGL(k_objred_dir<R>, dim3(A.nObj), dim3(kSBlock), 0, s, A, k);
  } else {
    PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_dir<R, false, M_>), dim3(A.grid), dim3(DirBlock<R, M_>::value), 0, s, A, k));
  }
}
template <typename R>
void launch_finalize(const Args<R>& A, double* x_out, double* v_out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize<R>, dim3(A.grid), dim3(kSBlock), 0, s, A, x_out, v_out);
}
template <typename R>
void launch_load_query(const Args<R>& A, const double* x, const double* xt, const double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_load_query<R>, dim3(A.grid), dim3(kSBlock), 0, s, A, x, xt, p);
}
template <typename R>
void launch_query_gradient(const Args<R>& A, double* g, double* d, hipStream_t s) {
  if (A.self && A.seg)
    hipLaunchKernelGGL((k_pairs_entries<R, 0>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_narrow);
  else if (A.self)
    hipLaunchKernelGGL((k_pairs_query<R, 0>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_narrow);
  PNCG_BY_SCATTER(A.self && A.seg, PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_grad<R, kGradQuery, false, M_, S_>), dim3(A.grid),
                                            dim3(GradBlock<R, M_>::value), 0, s, A, 0, 0, g, d)));
}
template <typename R>
void launch_query_energy(const Args<R>& A, double* out, hipStream_t s) {
  PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_energy<R, M_>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_dir));
  if (A.self) hipLaunchKernelGGL((k_pairs_query<R, 1>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_narrow);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSBlock), 0, s, A.part_dir, A.grid,
                     A.self ? A.part_narrow : (const double*)nullptr, A.grid, out);
}
template <typename R>
void launch_query_hvp(const Args<R>& A, double* hp, double* out, hipStream_t s) {
  if (A.self) launch_pairs_hvp<R>(A, s);
  PNCG_BY_SCATTER(A.self && A.seg, PNCG_BY_MODEL(A.model, hipLaunchKernelGGL((k_hvp<R, M_, S_>), dim3(A.grid), dim3(kSBlock), 0, s, A, hp, A.part_dir)));
  // pair p^T H p is already inside H p at the vertices, so only k_hvp's partials are summed
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSBlock), 0, s, A.part_dir, A.grid, (const double*)nullptr, 0, out);
}
template <typename R>
void launch_pairs_hvp(const Args<R>& A, hipStream_t s) {
  if (A.seg)
    hipLaunchKernelGGL((k_pairs_entries<R, 2>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_narrow);
  else
    hipLaunchKernelGGL((k_pairs_query<R, 2>), dim3(A.grid), dim3(kSBlock), 0, s, A, A.part_narrow);
}
template <typename R>
void launch_audit(const Args<R>& A, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_audit<R>, dim3(A.grid), dim3(kSBlock), 0, s, A, part);
}

#define PNCG_INSTANTIATE(R)                                                                          \
  template void launch_predict<R>(const Args<R>&, const double*, const double*, double3, hipStream_t); \
  template void launch_iteration_first<R>(const Args<R>&, int, int, hipStream_t);                     \
  template void launch_iteration_grad<R>(const Args<R>&, int, hipStream_t);                           \
  template void launch_iteration_dir<R>(const Args<R>&, int, hipStream_t);                            \
  template void launch_finalize<R>(const Args<R>&, double*, double*, hipStream_t);                    \
  template void launch_load_query<R>(const Args<R>&, const double*, const double*, const double*,     \
                                     hipStream_t);                                                    \
  template void launch_query_gradient<R>(const Args<R>&, double*, double*, hipStream_t);              \
  template void launch_query_energy<R>(const Args<R>&, double*, hipStream_t);                         \
  template void launch_query_hvp<R>(const Args<R>&, double*, double*, hipStream_t);                   \
  template void launch_pairs_hvp<R>(const Args<R>&, hipStream_t);                                    \
  template void launch_audit<R>(const Args<R>&, double*, hipStream_t);

PNCG_INSTANTIATE(float)
PNCG_INSTANTIATE(double)

}  // namespace pncg
