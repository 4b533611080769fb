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
  int* ent_rank;                 // [ent_cap] place of the entry in its bucket (its bucket count before it)
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
// the pair count to *n_out.  With P its launch also zeroes the pair index's
// counters (pairs_index is then called with zeroed = true), and with xbuild
// it copies x there (the list's build positions).
struct PairIndex;
void broad_solver_list(const Broad& B, const double4* x, double cell, double r, int2* out, long long cap,
                       long long* ncand, int* err, long long* n_out, hipStream_t s, const PairIndex* P = nullptr,
                       double4* xbuild = nullptr);
// Per-vertex index of the (pair, corner) entries of a candidate list, for the
// segmented scatter of the pair terms.
struct PairIndex {
  int nV;
  const int* tris;       // [nF][3]
  const int* edges;      // [nE][2]
  int* vcnt;             // [2 nV] entries per vertex, then fill counters
  int* coff;             // [nV + 1] their offsets
  int* cent;             // [4 cap] slot ids (4 q + corner) grouped by vertex, each vertex's in the
                         // order of its pairs' (kind, first index, second index)
  int* cent_tmp;         // [4 cap] the same before the per-vertex ordering
  unsigned long long* ckey_tmp;  // [4 cap] the pair key of each entry of cent_tmp
  int4* pv;              // [cap] the four vertices of pair q in narrow-phase order; edge-edge
                         // pairs store ~v3 in w (the kind is the sign of w)
  int* big;              // [nV + 1] vertices with more entries than a thread orders ([0] = count)
  int* scan_tmp;         // scan partials, nV / 4096 + 2 ints
  // entry range [x, y) of each 64-lane wave of the vertex incidence (its
  // vertices' entries), so that waves without entries skip the pair sums
  const int2* wvert;     // [nWaves] first and last vertex of each incidence wave
  int2* wrange;          // [nWaves]
  int nWaves;
  int grid;
};
// Build coff / cent for list[0, min(ncand[0], cap)) (kind by position when
// ncand[1] >= 0, else in the pair) and set each incidence wave's entry
// range.  The entry order depends on the set of pairs only, not on their
// order in the list.  No host synchronisation; deterministic.
void pairs_index(const PairIndex& P, const int2* list, const long long* ncand, long long cap, hipStream_t s,
                 bool zeroed = false);
// Copy n pairs (kind in the pair) into out, set ncand = {n, -1} and *n_out = n.
// dst[v] = src[v] for v < n (the list's build positions).
void copy_positions(double4* dst, const double4* src, int n, hipStream_t s);
void pairs_install(const int2* src, long long n, int2* out, long long* ncand, long long* n_out, hipStream_t s);

// Plane candidates ((n0 x0 + n1 x1) + n2 x2) - o <= r for surface vertices.
void plane_candidates(const Broad& B, const double4* x, const Planes& planes, double r, int2* out, long long* n,
                      long long cap, hipStream_t s);

}  // namespace pncg
