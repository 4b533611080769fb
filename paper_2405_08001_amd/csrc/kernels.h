// Host-side launchers of the libpncg kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace pncg {

template <typename R> void launch_predict(const Args<R>& A, const double* x, const double* v, double3 grav, hipStream_t s);
template <typename R> void launch_iteration_first(const Args<R>& A, int k, int mode, hipStream_t s);
template <typename R> void launch_iteration_grad(const Args<R>& A, int k, hipStream_t s);
template <typename R> void launch_iteration_dir(const Args<R>& A, int k, hipStream_t s);
template <typename R> void launch_finalize(const Args<R>& A, double* x_out, double* v_out, hipStream_t s);
template <typename R> void launch_load_query(const Args<R>& A, const double* x, const double* xt, const double* p, hipStream_t s);
template <typename R> void launch_query_gradient(const Args<R>& A, double* g, double* d, hipStream_t s);
template <typename R> void launch_query_energy(const Args<R>& A, double* out, hipStream_t s);
template <typename R> void launch_query_hvp(const Args<R>& A, double* hp, double* out, hipStream_t s);
template <typename R> void launch_audit(const Args<R>& A, double* part, hipStream_t s);

// ------------------------------------------------------------ broad phase
// Candidate lists by the inflated-AABB test (float64, no contraction) with a
// uniform-grid spatial hash.  Point items are the surface vertices; edge
// items are keyed by the cell of their lower box corner.
struct Broad {
  // static
  int nV, nSV, nF, nE;
  const int* surf;       // [nSV] surface vertices
  const int* tris;       // [nF][3]
  const int* edges;      // [nE][2]
  const int* oid;        // [nV] object id (rest exclusion)
  // rest-pose exclusion keys (sorted)
  const unsigned long long* excl_pt; int n_excl_pt;
  const unsigned long long* excl_ee; int n_excl_ee;
  // hash table: items 0..nSV-1 surface vertices, nSV.. edges
  int tsize;             // power of two
  int* count;            // [tsize]
  int* start;            // [tsize + 1]
  int* items;            // [nSV + nE]
  double* part_ext;      // [kMaxGrid][3] max edge extent per block
  long long* part_cnt;   // [kMaxGrid * kBlock] per-thread pair counts (pt, ee interleaved)
  long long* part_off;   // [kMaxGrid * kBlock * 2]
  int grid;
};

// Build the hash at positions x (double4 [nV]) with cell size `cell`.
void broad_build(const Broad& B, const double4* x, double cell, hipStream_t s);
// Count pairs (pass 1); writes per-thread counts.  filter_d >= 0 keeps only
// pairs closer than filter_d (exact distance) from the same object.
void broad_count(const Broad& B, const double4* x, double cell, double r, double filter_d, hipStream_t s);
// Exclusive scan of the per-thread counts; totals to n_out[0] (all), n_out[1] (PT).
void broad_scan(const Broad& B, long long* n_out, hipStream_t s);
// Emit pairs (pass 2) into out[cap] (PT first, then EE); cap checked on device.
void broad_fill(const Broad& B, const double4* x, double cell, double r, double filter_d, int2* out, long long cap,
                hipStream_t s);
// Plane candidates ((n0 x0 + n1 x1) + n2 x2) - o <= r for surface vertices.
void plane_candidates(const Broad& B, const double4* x, const Planes& planes, double r, int2* out, long long* n,
                      long long cap, hipStream_t s);

}  // namespace pncg
