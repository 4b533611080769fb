// Internal layout shared by the kernels and the host runtime of libpncg.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device_math.h"
#include "../../include/pncg.h"

namespace pncg {

constexpr int kMaxPlanes = 8;
constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per block of the broad-phase kernels
constexpr int kSBlock = 256;         // threads per block of the solver kernels
constexpr int kXcds = 8;             // accelerator complex dies; workgroups are dealt round-robin over them
constexpr int kMaxGrid = 512;        // blocks of the solver kernels (= partial count)

// per-vertex flags
constexpr uint8_t kFixed = 1;
constexpr uint8_t kSurface = 2;

// error bits raised by kernels
constexpr int kErrInverted = 1;
constexpr int kErrPenetration = 2;
constexpr int kErrNonfinite = 4;
constexpr int kErrCapacity = 8;
constexpr int kErrTeam = 16;       // a team barrier of the batched kernel timed out

// beta of iteration k > 0 by the rule in bits 4..6 of the solver flags, from
// this iteration's g^T P g, g^T P y, y^T d, y^T P y, d^T g and the previous
// iteration's g^T P g and d^T g (d the previous direction, y = g - g_prev);
// 0 for a zero denominator or a non-finite value.
__host__ __device__ inline double beta_rule(unsigned flags, double gPg, double gPy, double yp, double yPy,
                                            double pg, double gPg_prev, double gTp_prev) {
  double b = 0.0;
  switch ((flags >> 4) & 7u) {
    case 1:  // Fletcher-Reeves
      b = gPg_prev != 0.0 ? gPg / gPg_prev : 0.0;
      break;
    case 2:  // Polak-Ribiere-Polyak
      b = gPg_prev != 0.0 ? gPy / gPg_prev : 0.0;
      break;
    case 3:  // conjugate descent
      b = gTp_prev != 0.0 ? -gPg / gTp_prev : 0.0;
      break;
    default: {  // Dai-Kou (0) and Hager-Zhang (4, twice the second term)
      if (yp == 0.0) return 0.0;
      const double c = ((flags >> 4) & 7u) == 4u ? 2.0 : 1.0;
      b = gPy / yp - c * (yPy / yp) * (pg / yp);
    }
  }
  return isfinite(b) ? b : 0.0;
}

template <typename R> struct R4T;
template <> struct R4T<float> { using type = float4; };
template <> struct R4T<double> { using type = double4; };
template <typename R> using R4 = typename R4T<R>::type;

struct Planes {
  int n;
  double p[kMaxPlanes][4];   // n0 n1 n2 o  (half-space n.x >= o)
};

// Scalars of iteration k.  Each field has one writer kernel (block 0 of it):
//   first kernel of k: alpha, dE, dE0, D, stop, pause, a_up
//   direction kernel of k: beta, gTp, gnorm, dir_stop, restart, n_active, Dx
// and is read only by kernels launched after its writer.
struct IterScal {
  double alpha, dE, dE0, D;
  double beta, gTp, gnorm;
  double gPg;        // g^T P g of this iteration (denominator of the FR / PRP rules at the next)
  double n_active;
  double Dx;         // max over surface vertices of |x_k - x at the last list build|
  int stop, pause, a_up, dir_stop, restart, pad;
};

// Per-object scalars of iteration k when the step is split by object
// (Sec. 5.2): [iteration][object].  beta, gTp, gPg, gg by the object's
// gradient reduction; alpha, pHp, pmv, dE, a_up, moving by its direction
// reduction.
struct ObjScal {
  double beta, gTp, gPg, gg;
  double alpha, pHp, pmv, dE;
  int a_up, moving, pad0, pad1;
};

// Step status, written when the step ends or pauses (one writer at a time).
struct StepStatus {
  int stopped;      // the step has ended
  int final_k;      // iteration whose x buffer (final_k & 1) holds x^{t+1}
  int iters;        // position updates made
  int reason;       // 0 dE rule, 1 gradient rule, 2 cap, 3 zero/unbounded
  int paused_at;    // -1, or iteration whose candidate list must be rebuilt
  int err;          // kErr* bits
  int a_up_hits;
  int pad;
  double g0, gk, dE0, last_dE;
  double n_active;
  double D;           // displacement bound since the last list build (first launch of each iteration)
  long long n_cand;   // candidates of the last list (written by the list builder)
  long long n_pt;     // of which point-triangle
};

// Everything a solver kernel touches.  Passed by value.
template <typename R>
struct Args {
  // mesh
  int nV, nT;
  const ElemRec<R>* elem;
  const int* inc;          // per lane: e * 4 + a, -1 padding, -2 vertex without tets
  const int* inc_vert;     // per lane: vertex, -1 padding
  int nWaves;
  const double* mass;
  const uint8_t* vflag;
  const double4* target;   // prescribed positions (valid where kFixed)
  const double4* xbuild;   // positions at the last candidate-list build
  // state
  double4* x0;             // x buffer of even iterations
  double4* x1;             // x buffer of odd iterations
  double4* xt;             // predictor
  double4* xstart;         // x^t
  R4<R>* g;                // gradient of the last evaluation
  R4<R>* pg;               // P g
  R4<R>* p0;               // direction buffers (p_k lives in p[k & 1])
  R4<R>* p1;
  double* acc;             // [nV][8] contact accumulators: g xyz, diag xyz (atomic scatter)
  // segmented scatter: the (pair, corner) entries grouped by vertex are
  // evaluated 64 to a wave and summed per vertex run into run partials
  int seg;                 // 1: segmented, 0: atomic
  int fuse;                // 1: the pair pass runs inside the first sweep launch (see fused_pairs)
  int carry;               // 1: the step starts on the list of an earlier step (k_predict measures
                           // how far x_0 is from its build positions; iteration 0 pauses for a
                           // rebuild if that exceeds half the skin)
  const int* coff;         // [nV + 1] corner entries of each vertex
  const int* cent;         // [4 cap] slot id 4 q + corner of each entry (per vertex in pair-key order)
  const int2* wrange;      // [nWaves] corner-entry range of each incidence wave's vertices
  double* rp;              // [4 cap][6] run partials: gradient xyz, diag xyz (or H p xyz)
  const int4* pv;          // [cap] corner vertices of each pair (segmented scatter; NULL otherwise),
                           // edge-edge pairs with ~v3 in w
  // contact
  int self;                // point-triangle / edge-edge barriers on
  const int2* cand;        // candidate pairs: (v, f) point-triangle then (e1, e2) edge-edge
  const long long* ncand;  // device: [0] total, [1] point-triangle count (-1: kind in the pair)
  long long cand_cap;      // capacity of cand (counts above it are clamped)
  const int* tris;         // [nF][3]
  const int* edges;        // [nE][2]
  Planes planes;
  double dhat, kappa, h, h2, skin;
  int has_prims;           // any collision primitive (planes or self contact)
  // solver
  int iter_max, term;
  double eps;
  unsigned flags;
  IterScal* scal;
  StepStatus* status;
  double* part_grad;       // [kMaxGrid][8]
  double* part_dir;        // [kMaxGrid][4]
  double* part_narrow;     // [kMaxGrid]
  int grid;
  // splitting computation (Sec. 5.2): objects are contiguous vertex and tet ranges
  int split, nObj;
  int model;               // Model of device_math.h (kernel template argument)
  const int* vobj;         // [nV] object of each vertex
  const int* voff;         // [nObj + 1] vertex ranges
  const int* toff;         // [nObj + 1] tet ranges
  ObjScal* oscal;          // [iter_max + 2][nObj]
  double* vdots;           // [nV][6] per-vertex beta dot products
  double* tphp;            // [nT] h^2 p^T H_e p of each tet
  double* vphp;            // [nV][3] inertia + plane p^T H p, |p_v|_2, max_i |p_v,i|
  double* opair;           // [2][nObj] pair p^T H p per object (float64 atomics)
};

// Runs CALL with the constexpr M_ set to the model the arguments carry.
#define PNCG_BY_MODEL(model, CALL)                                  \
  do {                                                              \
    if ((model) == kModelSNH) {                                     \
      constexpr int M_ = kModelSNH;                                 \
      CALL;                                                         \
    } else if ((model) == kModelCorot) {                            \
      constexpr int M_ = kModelCorot;                               \
      CALL;                                                         \
    } else {                                                        \
      constexpr int M_ = kModelNH;                                  \
      CALL;                                                         \
    }                                                               \
  } while (0)

// Runs CALL with the constexpr S_ set to whether the pair terms use the
// segmented slots.
// With the segmented scatter and one step size for the whole scene, the
// pair pass can run inside the first launch of the gradient sweep (two
// launches per iteration): each block evaluates the entries of its own
// vertices.  That pays while contact is sparse; where entries crowd onto a
// few blocks' vertices the separate, evenly split pass is faster, so the
// host sets A.fuse per chunk from the size of the last list.  Both forms
// give the same bits.
template <typename R>
inline bool fused_pairs(const Args<R>& A) {
  return A.self && A.seg && !A.split && A.fuse;
}

#define PNCG_BY_SCATTER(seg, CALL) \
  do {                             \
    if (seg) {                     \
      constexpr bool S_ = true;    \
      CALL;                        \
    } else {                       \
      constexpr bool S_ = false;   \
      CALL;                        \
    }                              \
  } while (0)

// Kernel model (device_math.h Model) of a PNCG_MODEL_* value: ARAP runs
// the fixed-corotated kernels with lam = 0.
inline int kernel_model(int model) {
  return model == PNCG_MODEL_SNH ? 1 : (model == PNCG_MODEL_ARAP || model == PNCG_MODEL_FCR) ? 2 : 0;
}
// The lam the element record holds: lam' = lam + mu for the stable
// Neo-Hookean density, 0 for ARAP, lam otherwise.
inline double record_lam(int model, double mu, double lam) {
  return model == PNCG_MODEL_SNH ? lam + mu : model == PNCG_MODEL_ARAP ? 0.0 : lam;
}
inline const char* inverted_message(int model) {
  return model == PNCG_MODEL_NH ? "a tet has det F <= 0"
                                : "a tet's I1 Hessian is undefined (two singular values summing to <= 0)";
}

}  // namespace pncg
