// Batched form: many independent scenes (concatenated meshes), each stepped
// by one workgroup, or by a team of workgroups for a large scene, that runs
// the whole time step of Algorithm 1 (Sec. 4) inside the launch: predictor,
// every PNCG iteration with its per-scene beta, alpha and stop test, and the
// end-of-step velocity.  The grid-wide reductions of the single-scene path
// become block (or team) reductions, so an iteration costs no kernel launch;
// the grid is persistent and the host-built schedule lists each team's
// scenes.  Scenes have plane contact only (one optional plane each); the
// per-scene scalars follow the separate-step-size-per-object idea of Sec. 5.2.
#include "batch.h"
#include "sweep_common.h"

namespace pncg {

// Barrier among the workgroups of one team, waited on by one thread with a
// bounded number of polls.  The agent-scope fences publish this workgroup's
// stores before it arrives and make the others' visible after.  A wait that
// runs out of polls raises kErrTeam, and once that bit is set every later
// team barrier of the launch passes at once, so the launch always ends.
__device__ __forceinline__ void team_sync(int* bar, int target, int* err, int limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1);
    int polls = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++polls > limit || (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTeam)) {
        atomicOr(err, kErrTeam);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}

// Position of a workgroup in its team and the team's barrier state.
struct Team {
  int G, r;          // team size, rank of this workgroup
  int nb;            // team barriers passed so far in this launch
  int* bar;
  double* part;      // [2][kMaxTeam][8]
  int* err;
  int limit;
  __device__ void sync() {
    if (G > 1) team_sync(bar, G * ++nb, err, limit);
  }
  // Block reduction, then (G > 1) the members' results combined in rank
  // order, so every member holds the same bits.
  template <int N, int BS>
  __device__ void reduce(double (&v)[N], const int (&kind)[N], double* sh) {
    block_reduce<N, BS>(v, kind, sh);
    if (G == 1) return;
    double* slot = part + ((nb + 1) & 1) * (kMaxTeam * 8);
    if (threadIdx.x == 0)
      for (int i = 0; i < N; ++i) slot[r * 8 + i] = v[i];
    sync();
    for (int i = 0; i < N; ++i) {
      double acc = slot[i];
      for (int j = 1; j < G; ++j) acc = kind[i] ? fmax(acc, slot[j * 8 + i]) : acc + slot[j * 8 + i];
      v[i] = acc;
    }
  }
};

// LDSX: the positions and directions of the scene being stepped live in
// LDS (A.vcap vertices at most; dynamic shared memory of vcap * (3 doubles +
// 3 R)), so the gathers of the element loops read LDS instead of memory;
// otherwise they live in the per-vertex arrays x and p.  A scene stepped by
// a team of G > 1 workgroups (LDSX only) is split as follows: the incidence
// waves and the tets are dealt out over the members, each member keeps a
// full copy of the scene's x and p in its own LDS and forms the direction
// and the update for every vertex, and the members meet twice per iteration
// to combine their partial sums (after the gradient sweep, which also
// publishes P g, and after the p^T H p pass).
template <typename R, int BS, bool LDSX, int M>
__global__ void __launch_bounds__(BS) k_batch_step(BatchArgs<R> A, const double* x_in, const double* v_in,
                                                   double* x_out, double* v_out) {
  constexpr int NW = BS / kWave;
  __shared__ double sh[NW * 8];
  extern __shared__ double dyn[];
  double* sx = dyn;                                  // [3][vcap]
  R* sp = reinterpret_cast<R*>(dyn + 3 * A.vcap);    // [3][vcap]
  const int vc = A.vcap;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
  const int tm = A.blk_team[blockIdx.x];
  Team T{A.team_size[tm], A.blk_rank[blockIdx.x], 0, A.bar + tm, A.tpart + (size_t)tm * 2 * kMaxTeam * 8, A.err,
         A.spin_limit};
  const int G = T.G, r = T.r;
  for (int j = A.team_off[tm]; j < A.team_off[tm + 1]; ++j) {
    const int s = A.team_scene[j];
    const int v0 = A.vert_off[s], v1 = A.vert_off[s + 1];
    const int t0 = A.tet_off[s], t1 = A.tet_off[s + 1];
    const int w0 = A.wave_off[s], w1 = A.wave_off[s + 1];
    const double* pl = A.planes + 4 * s;
    const bool has_plane = pl[0] != 0.0 || pl[1] != 0.0 || pl[2] != 0.0;
    auto X = [&](int v) -> V3<double> {
      if (!LDSX) return ld3(A.x, v);
      const int l = v - v0;
      return mk3(sx[l], sx[vc + l], sx[2 * vc + l]);
    };
    auto setX = [&](int v, V3<double> x) {
      if (!LDSX) { st3(A.x, v, x); return; }
      const int l = v - v0;
      sx[l] = x.x; sx[vc + l] = x.y; sx[2 * vc + l] = x.z;
    };
    auto Pd = [&](int v) -> V3<R> {
      if (!LDSX) return ldr<R>(A.p, v);
      const int l = v - v0;
      return mk3(sp[l], sp[vc + l], sp[2 * vc + l]);
    };
    auto setP = [&](int v, V3<R> p) {
      if (!LDSX) { str<R>(A.p, v, p); return; }
      const int l = v - v0;
      sp[l] = p.x; sp[vc + l] = p.y; sp[2 * vc + l] = p.z;
    };
    // predictor: xt = x + h v + h^2 g; x_0 = x^t (the team's members share
    // the writes of xt and g, then meet)
    for (int v = v0 + tid; v < v1; v += BS) {
      const V3<double> x = mk3(x_in[3 * v], x_in[3 * v + 1], x_in[3 * v + 2]);
      if (!LDSX) st3(A.xstart, v, x);
      setX(v, x);
      setP(v, mk3(R(0), R(0), R(0)));
      if ((v - v0) / BS % G != r) continue;
      const V3<double> u = mk3(v_in[3 * v], v_in[3 * v + 1], v_in[3 * v + 2]);
      V3<double> xt = x + A.h * u;
      xt = xt + A.h2 * A.grav;
      st3(A.xt, v, xt);
      str<R>(A.g, v, mk3(R(0), R(0), R(0)));
    }
    T.sync();
    __syncthreads();
    int k = 0, reason = 2;
    double g0 = 0.0, dE0 = 0.0, gPg_prev = 0.0, gTp_prev = 0.0;
    for (;;) {
      // ---- gradient, diag(H), dot products (vertex-centric sweep)
      double dots[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int w = w0 + r * NW + wave; w < w1; w += G * NW) {
        const int idx = w * kWave + lane;
        const int code = A.inc[idx];
        const int myv = A.inc_vert[idx];
        R sv[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
        if (code >= 0) {
          const ElemRec<R> rec = A.elem[code >> 2];
          Kin<R> kin = kinematics<R>(rec.B, X(rec.v[0]), X(rec.v[1]), X(rec.v[2]), X(rec.v[3]));
          V3<R> g, dg;
          bool ok;
          if constexpr (M == kModelNH) {
            // the Neo-Hookean form spelled out: the generic helper's checks
            // cost this register-bound kernel registers and spills
            ok = kin.J > R(0);
            if (ok) nh_grad_diag(kin, rec.vmu, rec.vlam, shape_vec(rec.B, code & 3), g, dg);
          } else {
            ok = el_grad_diag<R, M>(kin, rec.vmu, rec.vlam, shape_vec(rec.B, code & 3), g, dg);
          }
          if (ok) {
            sv[0] = g.x; sv[1] = g.y; sv[2] = g.z; sv[3] = dg.x; sv[4] = dg.y; sv[5] = dg.z;
          } else {
            atomicOr(A.err, kErrInverted);
          }
        }
        if (!seg_sum_shfl(myv, sv) || myv < 0) continue;
        const int v = myv;
        const V3<double> x = X(v), xt = ld3(A.xt, v);
        const double m = A.mass[v];
        double gd[3] = {A.h2 * double(sv[0]) + m * (x.x - xt.x), A.h2 * double(sv[1]) + m * (x.y - xt.y),
                        A.h2 * double(sv[2]) + m * (x.z - xt.z)};
        double dd[3] = {A.h2 * double(sv[3]) + m, A.h2 * double(sv[4]) + m, A.h2 * double(sv[5]) + m};
        if (has_plane && (A.vflag[v] & kSurface)) {
          const double d = plane_dist(pl, x);
          if (d < A.dhat) {
            if (!(d > 0.0)) {
              atomicOr(A.err, kErrPenetration);
            } else {
              const double b1 = A.kappa * barrier_db(d, A.dhat), b2 = A.kappa * barrier_d2b(d, A.dhat);
              for (int j = 0; j < 3; ++j) {
                gd[j] += b1 * pl[j];
                dd[j] += b2 * pl[j] * pl[j];
              }
            }
          }
        }
        const V3<R> gR = mk3(R(gd[0]), R(gd[1]), R(gd[2]));
        const V3<R> pgR = mk3(R(gd[0] / dd[0]), R(gd[1] / dd[1]), R(gd[2] / dd[2]));
        const V3<R> gpR = ldr<R>(A.g, v), ppR = Pd(v);
        str<R>(A.g, v, gR);
        str<R>(A.pg, v, pgR);
        const double g3[3] = {double(gR.x), double(gR.y), double(gR.z)};
        const double pg3[3] = {double(pgR.x), double(pgR.y), double(pgR.z)};
        const double gp3[3] = {double(gpR.x), double(gpR.y), double(gpR.z)};
        const double pp3[3] = {double(ppR.x), double(ppR.y), double(ppR.z)};
        for (int j = 0; j < 3; ++j) {
          const double P = 1.0 / dd[j], y = g3[j] - gp3[j];
          dots[0] += g3[j] * g3[j];
          dots[1] += g3[j] * pg3[j];
          dots[2] += g3[j] * P * y;
          dots[3] += y * pp3[j];
          dots[4] += y * P * y;
          dots[5] += pp3[j] * g3[j];
        }
      }
      {
        const int kind[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        T.reduce<8, BS>(dots, kind, sh);
      }
      const double gnorm = sqrt(dots[0]);
      if (k == 0) g0 = gnorm;
      if ((A.term == 1 && gnorm <= A.eps * g0) || (A.term == 2 && gnorm <= A.eps)) { reason = 1; break; }
      double beta = 0.0;
      if (k > 0) beta = beta_rule(A.flags, dots[1], dots[2], dots[3], dots[4], dots[5], gPg_prev, gTp_prev);
      double gTp = -dots[1] + beta * dots[5];
      if (!(gTp < 0.0)) {
        beta = 0.0;
        gTp = -dots[1];
      }
      gPg_prev = dots[1];
      gTp_prev = gTp;
      if (gTp == 0.0) { reason = 3; break; }
      // ---- direction p = -P g + beta p (in place; every member forms all of
      // it), inertia and plane parts of p^T H p (counted by rank 0)
      const R rb = R(beta);
      double php = 0.0, pmv = 0.0, pmc = 0.0;
      for (int v = v0 + tid; v < v1; v += BS) {
        const V3<R> p = direction(ldr<R>(A.pg, v), Pd(v), rb);
        setP(v, p);
        const double px = p.x, py = p.y, pz = p.z, p2 = px * px + py * py + pz * pz;
        php += A.mass[v] * p2;
        pmv = fmax(pmv, sqrt(p2));
        pmc = fmax(pmc, fmax(fabs(px), fmax(fabs(py), fabs(pz))));
        if (has_plane && (A.vflag[v] & kSurface)) {
          const double d = plane_dist(pl, X(v));
          if (d > 0.0 && d < A.dhat) {
            const double np = pl[0] * px + pl[1] * py + pl[2] * pz;
            php += A.kappa * barrier_d2b(d, A.dhat) * np * np;
          }
        }
      }
      if (r != 0) php = 0.0;
      __syncthreads();
      // ---- element p^T H p
      double el = 0.0;
      for (int e = t0 + r * BS + tid; e < t1; e += G * BS) {
        const ElemRec<R> rec = A.elem[e];
        Kin<R> kin = kinematics<R>(rec.B, X(rec.v[0]), X(rec.v[1]), X(rec.v[2]), X(rec.v[3]));
        V3<R> d[3];
        dF_cols(rec.B, Pd(rec.v[0]), Pd(rec.v[1]), Pd(rec.v[2]), Pd(rec.v[3]), d);
        if constexpr (M == kModelNH) {
          el += double(nh_pHp(kin, rec.vmu, rec.vlam, d));   // inversion is caught by the sweep
        } else {
          R ph = R(0);
          if (!el_pHp<R, M>(kin, rec.vmu, rec.vlam, d, ph)) atomicOr(A.err, kErrInverted);
          el += double(ph);
        }
      }
      double red[3] = {php + A.h2 * el, pmv, pmc};
      {
        const int kind[3] = {0, 1, 1};
        T.reduce<3, BS>(red, kind, sh);
      }
      const double pHp = red[0];
      const double pm = (A.flags & 2u) ? red[2] : red[1];
      const double abar = pHp > 0.0 ? -gTp / pHp : HUGE_VAL;
      const double aup = (has_plane && pm > 0.0) ? A.dhat / (2.0 * pm) : HUGE_VAL;
      const double alpha = fmin(aup, abar);
      if (!isfinite(alpha)) { reason = 3; break; }
      // ---- update
      for (int v = v0 + tid; v < v1; v += BS) {
        const V3<double> x = X(v);
        const V3<R> q = Pd(v);
        setX(v, mk3(fma(alpha, double(q.x), x.x), fma(alpha, double(q.y), x.y), fma(alpha, double(q.z), x.z)));
      }
      const double dE = -alpha * gTp - 0.5 * alpha * alpha * pHp;
      if (k == 0) dE0 = dE;
      ++k;
      __syncthreads();
      if (A.term == 0 && dE < A.eps * dE0) { reason = 0; break; }
      if (k >= A.iter_max) { reason = 2; break; }
    }
    // end of step: v = (x - x^t) / h (the members share the writes)
    const double ih = 1.0 / A.h;
    for (int v = v0 + r * BS + tid; v < v1; v += G * BS) {
      const V3<double> x = X(v);
      const V3<double> xs = LDSX ? mk3(x_in[3 * v], x_in[3 * v + 1], x_in[3 * v + 2]) : ld3(A.xstart, v);
      x_out[3 * v] = x.x; x_out[3 * v + 1] = x.y; x_out[3 * v + 2] = x.z;
      v_out[3 * v] = (x.x - xs.x) * ih; v_out[3 * v + 1] = (x.y - xs.y) * ih; v_out[3 * v + 2] = (x.z - xs.z) * ih;
    }
    if (tid == 0 && r == 0) {
      A.iters[s] = k;
      A.reason[s] = reason;
      A.iters_total[s] += k;
    }
    __syncthreads();
  }
}

__global__ void k_team_reset(int* bar, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bar[i] = 0;
}

void launch_team_reset(int* bar, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_team_reset, dim3((n + 255) / 256), dim3(256), 0, s, bar, n);
}

template <typename R, bool LDSX, int M>
void launch_bsm(const BatchArgs<R>& A, int block, int grid, size_t shmem, const double* x, const double* v,
                double* xo, double* vo, hipStream_t s) {
  switch (block) {
    case 256:
      hipLaunchKernelGGL((k_batch_step<R, 256, LDSX, M>), dim3(grid), dim3(256), shmem, s, A, x, v, xo, vo);
      break;
    case 512:
      hipLaunchKernelGGL((k_batch_step<R, 512, LDSX, M>), dim3(grid), dim3(512), shmem, s, A, x, v, xo, vo);
      break;
    default:
      hipLaunchKernelGGL((k_batch_step<R, 1024, LDSX, M>), dim3(grid), dim3(1024), shmem, s, A, x, v, xo, vo);
      break;
  }
}

template <typename R>
size_t batch_lds_bytes(int vcap) {
  return (size_t)vcap * 3 * (sizeof(double) + sizeof(R));
}

template <typename R>
void launch_batch_step(const BatchArgs<R>& A, int block, int grid, bool lds, const double* x, const double* v,
                       double* xo, double* vo, hipStream_t s) {
  if (lds)
    PNCG_BY_MODEL(A.model, (launch_bsm<R, true, M_>(A, block, grid, batch_lds_bytes<R>(A.vcap), x, v, xo, vo, s)));
  else
    PNCG_BY_MODEL(A.model, (launch_bsm<R, false, M_>(A, block, grid, 0, x, v, xo, vo, s)));
}

template <typename R, bool LDSX, int M>
hipError_t occ(int block, size_t shmem, int* per_cu) {
  switch (block) {
    case 256:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_step<R, 256, LDSX, M>, 256, shmem);
    case 512:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_step<R, 512, LDSX, M>, 512, shmem);
    default:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_step<R, 1024, LDSX, M>, 1024, shmem);
  }
}

template <typename R>
hipError_t batch_occupancy(int block, bool lds, int vcap, int model, int* per_cu) {
  hipError_t e = hipSuccess;
  if (lds)
    PNCG_BY_MODEL(model, (e = occ<R, true, M_>(block, batch_lds_bytes<R>(vcap), per_cu)));
  else
    PNCG_BY_MODEL(model, (e = occ<R, false, M_>(block, 0, per_cu)));
  return e;
}

template size_t batch_lds_bytes<float>(int);
template size_t batch_lds_bytes<double>(int);
template hipError_t batch_occupancy<float>(int, bool, int, int, int*);
template hipError_t batch_occupancy<double>(int, bool, int, int, int*);
template void launch_batch_step<float>(const BatchArgs<float>&, int, int, bool, const double*, const double*, double*,
                                       double*, hipStream_t);
template void launch_batch_step<double>(const BatchArgs<double>&, int, int, bool, const double*, const double*,
                                        double*, double*, hipStream_t);

}  // namespace pncg
