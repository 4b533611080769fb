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
// H p of the active pairs into acc[0..2] (p in A.p0, acc zeroed beforehand)
template <typename R> void launch_pairs_hvp(const Args<R>& A, hipStream_t s);
template <typename R> void launch_audit(const Args<R>& A, double* part, hipStream_t s);

// ------------------------------------------------------------ broad phase
// Candidate lists by the inflated-AABB test (float64, no contraction) over a
// uniform grid.  Triangles (boxes inflated by r) and edges (boxes inflated by
// r/2) are inserted into every cell their box touches; a surface vertex
// visits its own cell, edge pairs are tested per shared cell.
struct Broad {
  // static
  int nV, nSV, nF, nE;
  const int* surf;       // [nSV] surface vertices (ascending)
  const int* tris;       // [nF][3]
  const int* edges;      // [nE][2]
  const int* oid;        // [nV] object id (rest exclusion)
  // rest-pose exclusion keys (sorted)
  const unsigned long long* excl_pt; int n_excl_pt;
  const unsigned long long* excl_ee; int n_excl_ee;
  // items 0..nF-1 triangles, nF.. edges
  double4* item_lo;      // [nF + nE] triangle: min - r; edge: min
  double4* item_hi;      // [nF + nE] triangle: max + r; edge: max
  long long* item_cnt;   // [nF + nE + nSV] cells touched (primitives, then vertices)
  long long* item_off;   // [nF + nE + nSV + 1]
  // cell entries (item, cell key), then grouped by hash bucket
  long long ent_cap;
  unsigned long long* ent_key;   // [ent_cap]
  int* ent_item;                 // [ent_cap]
  unsigned long long* bkt_key;   // [ent_cap] records grouped by bucket
  int* bkt_item;                 // [ent_cap]
  double4* bkt_lo;               // [ent_cap] vertex: position; triangle: inflated box (lo, hi); edge: its two end points (box = their min, max)
  double4* bkt_hi;               // [ent_cap]
  int4* bkt_ids;                 // [ent_cap] vertex ids of the item (-1 unused)
  int tsize;             // power of two
  int* count;            // [tsize]
  int* start;            // [tsize + 1]
  // pair counting: PT and EE counts per entry
  long long work_cap;    // = 2 * ent_cap
  long long* part_cnt;   // [work_cap]
  long long* part_off;   // [work_cap + 4096]
  long long* totals;     // device: [0] entries, [1] pairs, [2] point-triangle pairs
  int grid;
};

// Rebuild the grid at positions x with cell size `cell` and inflation r,
// count the pairs and scan the counts.  totals[0] receives the number of
// cell entries (the build is valid only if it is <= ent_cap), totals[1] and
// totals[2] the pair counts.  filter_d >= 0 keeps only pairs closer than
// filter_d (exact distance), and with filter_obj only pairs of one object.
void broad_build_count(const Broad& B, const double4* x, double cell, double r, double filter_d, int filter_obj,
                       hipStream_t s);
// Emit the pairs counted above into out[cap] (point-triangle first, sorted by
// (v, f); then edge-edge).
void broad_fill(const Broad& B, const double4* x, double cell, double r, double filter_d, int filter_obj, int2* out,
                long long cap, hipStream_t s);
// The solver's list without host synchronisation: grid build and one-pass
// pair emission (pairs within distance r, unordered, kind in the pair:
// (v, f) point-triangle, (e1, ~e2) edge-edge; ncand[0] = pairs found,
// ncand[1] = -1).  Sets kErrCapacity in *err if the grid entries or the
// pairs exceeded their capacity (the list is then incomplete), and copies
// the pair count to *n_out.
void broad_solver_list(const Broad& B, const double4* x, double cell, double r, int2* out, long long cap,
                       long long* ncand, int* err, long long* n_out, hipStream_t s);
// Canonical order of a candidate list and the per-vertex index of its
// (pair, corner) slots, for the segmented scatter of the pair terms.
struct PairIndex {
  int nV, nE;
  const int* tris;       // [nF][3]
  const int* edges;      // [nE][2]
  int* bcnt;             // [2 (nV + nE)] pairs per first index (v, or nV + e1), then fill counters
  int* boff;             // [nV + nE + 1] their offsets
  int* vcnt;             // [2 nV] corners per vertex, then fill counters
  int* coff;             // [nV + 1] their offsets
  int* cent;             // [4 cap] slot ids (4 q + corner) grouped by vertex, ascending per vertex
  int* scan_tmp;         // scan partials, (nV + nE) / 4096 + 2 ints
  int grid;
};
// Sort in[0, min(ncand[0], cap)) lexicographically into out: point-triangle
// (v, f) first, then edge-edge (e1, ~e2) (the kind is taken by position when
// ncand[1] >= 0, else from the sign of the second index); set ncand[1] = -1
// (kind in the pair) and build coff / cent for out.  No host
// synchronisation; deterministic.
void pairs_canonical(const PairIndex& P, const int2* in, int2* out, long long* ncand, long long cap, hipStream_t s);
// Copy n pairs (kind in the pair) into out, set ncand = {n, -1} and *n_out = n.
void pairs_install(const int2* src, long long n, int2* out, long long* ncand, long long* n_out, hipStream_t s);

// Plane candidates ((n0 x0 + n1 x1) + n2 x2) - o <= r for surface vertices.
void plane_candidates(const Broad& B, const double4* x, const Planes& planes, double r, int2* out, long long* n,
                      long long cap, hipStream_t s);

}  // namespace pncg
