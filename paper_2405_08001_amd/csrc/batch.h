// Arguments of the batched step kernel.
#pragma once

#include "internal.h"

namespace pncg {

template <typename R>
struct BatchArgs {
  int nScenes;
  const int* order;        // [nScenes] processing order (largest scene first)
  const int* vert_off;     // [nScenes + 1] vertex offsets in the concatenation
  const int* tet_off;      // [nScenes + 1]
  const int* wave_off;     // [nScenes + 1] incidence waves of each scene
  const ElemRec<R>* elem;  // tet records (global vertex ids)
  const int* inc;          // per lane: e * 4 + a, -1 padding, -2 vertex without tets
  const int* inc_vert;     // per lane: global vertex, -1 padding
  const double* mass;
  const uint8_t* vflag;
  const double* planes;    // [nScenes][4]; a zero normal means no plane
  double4* x;
  double4* xt;
  double4* xstart;
  R4<R>* g;
  R4<R>* pg;
  R4<R>* p;
  int vcap;                // largest scene's vertex count (LDS staging)
  double dhat, kappa, h, h2, eps;
  V3<double> grav;
  int iter_max, term;
  unsigned flags;
  int* iters;              // [nScenes] iterations of the last step
  int* reason;             // [nScenes]
  long long* iters_total;  // [nScenes] accumulated over steps
  int* err;                // error bits
};

// LDS bytes that staging the positions and directions of a scene of vcap
// vertices takes.
template <typename R>
size_t batch_lds_bytes(int vcap);

// Resident workgroups per compute unit of the step kernel at this block size
// (lds: with the positions and directions of a scene in LDS).
template <typename R>
hipError_t batch_occupancy(int block, bool lds, int vcap, int* per_cu);

template <typename R>
void launch_batch_step(const BatchArgs<R>& A, int block, int grid, bool lds, const double* x, const double* v,
                       double* xo, double* vo, hipStream_t s);

}  // namespace pncg
