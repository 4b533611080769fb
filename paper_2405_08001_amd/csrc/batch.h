// Arguments of the batched step kernel.
#pragma once

#include "internal.h"

namespace pncg {

constexpr int kMaxTeam = 8;   // workgroups one scene may use

template <typename R>
struct BatchArgs {
  int nScenes;
  // Schedule: workgroup b belongs to team blk_team[b] as rank blk_rank[b];
  // team t has team_size[t] workgroups and steps the scenes
  // team_scene[team_off[t] .. team_off[t+1]) in that order.
  const int* blk_team;
  const int* blk_rank;
  const int* team_size;
  const int* team_off;
  const int* team_scene;
  int* bar;                // [teams] barrier arrivals (zeroed before each launch)
  double* tpart;           // [teams][2][kMaxTeam][8] reduction partials
  int spin_limit;          // polls before a team barrier gives up
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
  int model;               // device_math.h Model (kernel template argument)
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
// (lds: with the positions and directions of a scene in LDS) for the kernel
// model `model` (device_math.h Model).
template <typename R>
hipError_t batch_occupancy(int block, bool lds, int vcap, int model, int* per_cu);

// Zero the team barrier counters (a kernel, so that it can sit in a graph).
void launch_team_reset(int* bar, int n, hipStream_t s);

template <typename R>
void launch_batch_step(const BatchArgs<R>& A, int block, int grid, bool lds, const double* x, const double* v,
                       double* xo, double* vo, hipStream_t s);

}  // namespace pncg
