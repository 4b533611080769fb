// Broad phase: candidate point-triangle and edge-edge pairs by an inflated
// axis-aligned box test in float64 over a uniform grid (the paper culls with
// a grid hash, Sec. 6; the grid changes speed, not the set).
//
//   PT (v, f): v a surface vertex not in f, and on every axis
//              min_f - r <= x_v <= max_f + r
//   EE (e1 < e2) without a shared vertex, on every axis
//              min_e1 - r <= max_e2  and  min_e2 <= max_e1 + r
//
// Grid entries (cell, item): every surface vertex in its cell, every
// triangle in each cell its r-inflated box touches, every edge in each cell
// its (r/2 + margin)-inflated box touches.  Entries are grouped by a hash of
// the cell; each entry's record (cell, item, exact float64 box, vertex ids)
// is stored contiguously per bucket.  One thread per entry scans its bucket
// for entries of the same cell with a larger item id, so each pair sharing a
// cell is seen once per shared cell, and lanes of a wave read the same bucket
// (broadcast loads).  A vertex lies in one cell, which is among the
// triangle's cells whenever the PT test holds; an edge pair is reported only
// in the cell holding the lower corner of the intersection of the two
// inflated boxes, which both edges touch.  So every pair is found exactly
// once, and the exact test above makes the final decision.
//
// Output is produced without any global counter: a counting pass stores the
// pair counts of every entry, an exclusive scan turns them into offsets
// (point-triangle counts of all entries first, then edge-edge), and a second
// pass writes the pairs.
#include <algorithm>
#include <climits>

#include "kernels.h"

namespace pncg {

namespace {

constexpr int kTile = kBlock * 16;
constexpr double kEdgeMargin = 1e-9;   // absolute slack of the edge culling boxes (m)

__device__ __forceinline__ int cell_coord(double p, double inv) {
  double c = floor(p * inv);
  c = fmin(fmax(c, -1048575.0), 1048575.0);
  return (int)c;
}
__device__ __forceinline__ int3 cell_of(V3<double> p, double inv) {
  return make_int3(cell_coord(p.x, inv), cell_coord(p.y, inv), cell_coord(p.z, inv));
}
__device__ __forceinline__ unsigned long long cell_key(int cx, int cy, int cz) {
  return ((unsigned long long)(cx + 1048576) << 42) | ((unsigned long long)(cy + 1048576) << 21) |
         (unsigned long long)(cz + 1048576);
}
// bucket of a cell in one half of the table: triangles use [0, tsize/2),
// edges [tsize/2, tsize)
__device__ __forceinline__ unsigned hash_key(unsigned long long k, int tsize, bool edge) {
  const unsigned cx = (unsigned)(k >> 42), cy = (unsigned)((k >> 21) & 0x1FFFFF), cz = (unsigned)(k & 0x1FFFFF);
  unsigned h = (cx * 73856093u) ^ (cy * 19349663u) ^ (cz * 83492791u);
  const unsigned half = (unsigned)tsize >> 1;
  return (h & (half - 1)) + (edge ? half : 0u);
}
__device__ __forceinline__ V3<double> ldx(const double4* x, int i) {
  double4 v = x[i];
  return mk3(v.x, v.y, v.z);
}
__device__ __forceinline__ V3<double> v4(double4 v) { return mk3(v.x, v.y, v.z); }
__device__ __forceinline__ V3<double> vmin3(V3<double> a, V3<double> b) { return mk3(fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)); }
__device__ __forceinline__ V3<double> vmax3(V3<double> a, V3<double> b) { return mk3(fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)); }

__device__ __forceinline__ bool in_sorted(const unsigned long long* keys, int n, unsigned long long k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo < n && keys[lo] == k;
}

// --------------------------------------------------------------- scan
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const T* in, long long n, T* bsum) {
  __shared__ T sh[kBlock / kWave];
  const long long base = (long long)blockIdx.x * kTile;
  T s = 0;
  for (int i = threadIdx.x; i < kTile; i += kBlock) {
    long long j = base + i;
    if (j < n) s += in[j];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, kWave);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w];
    bsum[blockIdx.x] = t;
  }
}

// out[j] = exclusive prefix of in[j]; *total = sum (written by the last
// block).  Each block first adds up the sums of the blocks before it (bsum,
// from k_scan_reduce) in a fixed order, which takes the place of a separate
// launch that scans bsum.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_down(const T* in, long long n, const T* bsum, T* out, T* total) {
  __shared__ T sh[kBlock];
  __shared__ T sw[kBlock / kWave];
  T pre = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) pre += bsum[b];
  for (int o = kWave / 2; o > 0; o >>= 1) pre += __shfl_down(pre, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) sw[threadIdx.x / kWave] = pre;
  const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * 16;
  T v[16];
  T s = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    long long j = base + i;
    v[i] = j < n ? in[j] : 0;
    s += v[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  T boff = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) boff += sw[w];
  for (int o = 1; o < kBlock; o <<= 1) {
    T u = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += u;
    __syncthreads();
  }
  T run = boff + sh[threadIdx.x] - s;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    long long j = base + i;
    if (j < n) out[j] = run;
    run += v[i];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) *total = run;
}

template <typename T>
void scan_exclusive(const T* in, long long n, T* out, T* total, T* scratch, hipStream_t s) {
  const int nb = (int)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kBlock), 0, s, in, n, scratch);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kBlock), 0, s, in, n, (const T*)scratch, out, total);
}

// ------------------------------------------------------------ grid build

// culling box of primitive i (0..nF-1 triangles, nF.. edges): what is
// inserted into the grid
__device__ __forceinline__ void cull_box(const Broad& B, int i, double r, V3<double>& lo, V3<double>& hi) {
  lo = v4(B.item_lo[i]);
  hi = v4(B.item_hi[i]);
  if (i >= B.nF) {
    const double q = 0.5 * r + kEdgeMargin;
    lo = mk3(lo.x - q, lo.y - q, lo.z - q);
    hi = mk3(hi.x + q, hi.y + q, hi.z + q);
  }
}

// Boxes and cell counts of the items; also zeroes the bucket counters (which
// k_emit bumps next) and, given a list counter, empties the list.
__global__ void __launch_bounds__(kBlock) k_items(Broad B, const double4* x, double inv, double r,
                                                  long long* ncand) {
  for (int h = blockIdx.x * kBlock + threadIdx.x; h < B.tsize; h += gridDim.x * kBlock) B.count[h] = 0;
  if (ncand && blockIdx.x == 0 && threadIdx.x == 0) {
    ncand[0] = 0;
    ncand[1] = -1;
  }
  const int n = B.nF + B.nE;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    V3<double> lo, hi;
    if (i < B.nF) {
      const V3<double> a = ldx(x, B.tris[3 * i]), b = ldx(x, B.tris[3 * i + 1]), c = ldx(x, B.tris[3 * i + 2]);
      const V3<double> mn = vmin3(vmin3(a, b), c), mx = vmax3(vmax3(a, b), c);
      lo = mk3(mn.x - r, mn.y - r, mn.z - r);
      hi = mk3(mx.x + r, mx.y + r, mx.z + r);
    } else {
      const int e = i - B.nF;
      const V3<double> a = ldx(x, B.edges[2 * e]), b = ldx(x, B.edges[2 * e + 1]);
      lo = vmin3(a, b);
      hi = vmax3(a, b);
    }
    B.item_lo[i] = make_double4(lo.x, lo.y, lo.z, 0.0);
    B.item_hi[i] = make_double4(hi.x, hi.y, hi.z, 0.0);
    V3<double> cl, ch;
    cull_box(B, i, r, cl, ch);
    const int3 c0 = cell_of(cl, inv), c1 = cell_of(ch, inv);
    B.item_cnt[i] = (long long)(c1.x - c0.x + 1) * (c1.y - c0.y + 1) * (c1.z - c0.z + 1);
  }
}

// Entries of item i, one per cell of its culling box (z fastest, then y,
// then x), at item_off[i] on.  The bucket counters are bumped eight cells at
// a time, so that a thread has eight atomics in flight instead of waiting
// for each rank before the next.
__global__ void __launch_bounds__(kBlock) k_emit(Broad B, const double4* x, double inv, double r) {
  constexpr int kBatch = 8;
  const int n = B.nF + B.nE;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    V3<double> cl, ch;
    cull_box(B, i, r, cl, ch);
    const int3 c0 = cell_of(cl, inv), c1 = cell_of(ch, inv);
    const int nz = c1.z - c0.z + 1, nyz = (c1.y - c0.y + 1) * nz;
    const long long ncell = (long long)(c1.x - c0.x + 1) * nyz;
    const long long o = B.item_off[i];
    const long long m = min(ncell, B.ent_cap - o);   // entries past the capacity are not written
    const bool edge = i >= B.nF;
    for (long long t0 = 0; t0 < m; t0 += kBatch) {
      int rank[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const long long t = t0 + j;
        if (t < m) {
          const int cx = c0.x + (int)(t / nyz), rem = (int)(t % nyz);
          const int cy = c0.y + rem / nz, cz = c0.z + rem % nz;
          const unsigned long long k = cell_key(cx, cy, cz);
          B.ent_key[o + t] = k;
          B.ent_item[o + t] = B.nSV + i;
          rank[j] = atomicAdd(&B.count[hash_key(k, B.tsize, edge)], 1);
        }
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if (t0 + j < m) B.ent_rank[o + t0 + j] = rank[j];
    }
  }
}

// Group the entries by bucket and store each entry's full record there: its
// slot is the bucket's start plus the rank k_emit's counter gave it.
__global__ void __launch_bounds__(kBlock) k_bucket_fill(Broad B, const double4* x) {
  const long long n = min(B.totals[0], B.ent_cap);
  const int vbase = B.nSV, ebase = B.nSV + B.nF;
  for (long long j = blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) {
    const unsigned long long k = B.ent_key[j];
    const int it = B.ent_item[j];
    const unsigned h = hash_key(k, B.tsize, it >= B.nSV + B.nF);
    const int slot = B.start[h] + B.ent_rank[j];
    double4 lo, hi;
    int4 ids = make_int4(-1, -1, -1, 0);
    if (it < vbase) {
      ids.x = B.surf[it];
      lo = hi = x[ids.x];
    } else if (it < ebase) {
      const int f = it - vbase;
      ids = make_int4(B.tris[3 * f], B.tris[3 * f + 1], B.tris[3 * f + 2], 0);
      lo = B.item_lo[f];
      hi = B.item_hi[f];
    } else {
      // an edge record holds its two end points (its box is their
      // component-wise min and max), so the exact distance of a pair reads
      // the staged records instead of gathering positions
      const int e = it - ebase;
      ids.x = B.edges[2 * e];
      ids.y = B.edges[2 * e + 1];
      lo = x[ids.x];
      hi = x[ids.y];
    }
    B.bkt_key[slot] = k;
    B.bkt_item[slot] = it;
    B.bkt_lo[slot] = lo;
    B.bkt_hi[slot] = hi;
    B.bkt_ids[slot] = ids;
  }
}

// ------------------------------------------------------------------ pairs
// item ids: [0, nSV) surface vertices (surf order), [nSV, nSV + nF)
// triangles, [nSV + nF, ...) edges.
struct PairCtx {
  const double4* x;
  double inv, r, filter_d;
  int filter_obj;
};

// Records of a contiguous run of edge bucket slots held in LDS (an edge has
// two vertex ids; 34 KB, so that four blocks fit a compute unit).
constexpr int kSpan = 512;
struct SlotSpan {
  unsigned long long key[kSpan];
  int item[kSpan];
  int2 ids[kSpan];
  double lo[3][kSpan];
  double hi[3][kSpan];
};

// Record accessors: all slots from the LDS span, or all from global memory.
struct LdsRec {
  const SlotSpan& L;
  int base;
  __device__ __forceinline__ unsigned long long key(int t) const { return L.key[t - base]; }
  __device__ __forceinline__ int item(int t) const { return L.item[t - base]; }
  __device__ __forceinline__ int4 ids(int t) const {
    const int2 i = L.ids[t - base];
    return make_int4(i.x, i.y, -1, 0);
  }
  __device__ __forceinline__ V3<double> lo(int t) const {
    return mk3(L.lo[0][t - base], L.lo[1][t - base], L.lo[2][t - base]);
  }
  __device__ __forceinline__ V3<double> hi(int t) const {
    return mk3(L.hi[0][t - base], L.hi[1][t - base], L.hi[2][t - base]);
  }
};
struct GlobalRec {
  const Broad& B;
  __device__ __forceinline__ unsigned long long key(int t) const { return B.bkt_key[t]; }
  __device__ __forceinline__ int item(int t) const { return B.bkt_item[t]; }
  __device__ __forceinline__ int4 ids(int t) const { return B.bkt_ids[t]; }
  __device__ __forceinline__ V3<double> lo(int t) const { return v4(B.bkt_lo[t]); }
  __device__ __forceinline__ V3<double> hi(int t) const { return v4(B.bkt_hi[t]); }
};

// Point-triangle test of surface vertex v (position p, cell key) against
// the triangle entry in slot t.
__device__ __forceinline__ bool vertex_slot_pair(const Broad& B, const PairCtx& P, int v, V3<double> p,
                                                 unsigned long long key, int t, int2& out) {
  if (B.bkt_key[t] != key) return false;
  const int4 idB = B.bkt_ids[t];
  if (v == idB.x || v == idB.y || v == idB.z) return false;
  const V3<double> lo = v4(B.bkt_lo[t]), hi = v4(B.bkt_hi[t]);
  if (!(lo.x <= p.x && p.x <= hi.x && lo.y <= p.y && p.y <= hi.y && lo.z <= p.z && p.z <= hi.z)) return false;
  const int f = B.bkt_item[t] - B.nSV;
  // the distance filter first: it rejects most pairs in one step, while the
  // exclusion lookup is a chain of dependent loads (the filters commute)
  if (P.filter_d >= 0.0) {
    if (P.filter_obj && B.oid[v] != B.oid[idB.x]) return false;
    if (!(closest_pt(p, ldx(P.x, idB.x), ldx(P.x, idB.y), ldx(P.x, idB.z)).d < P.filter_d)) return false;
  }
  const unsigned long long pk = ((unsigned long long)(unsigned)v << 32) | (unsigned)f;
  if (B.n_excl_pt && in_sorted(B.excl_pt, B.n_excl_pt, pk)) return false;
  out = make_int2(v, f);
  return true;
}

// Exclusive prefix sum over a full wave by DPP lane moves: an inclusive
// scan within each row of 16 lanes (shifts by 1, 2, 4, 8), then lane 15 of
// rows 0 and 2 added to rows 1 and 3, then lane 31 to rows 2 and 3; the
// total is lane 63's.
__device__ __forceinline__ int wave_excl_scan(int v, int& total) {
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
  total = __builtin_amdgcn_readlane(x, kWave - 1);
  return x - v;
}

// Point-triangle pairs of surface vertex w: one wave per vertex, one lane per
// slot of the vertex's triangle bucket.  FILL = false returns the count (in
// every lane); FILL = true writes the pairs from offset `o` in slot order.
template <bool FILL>
__device__ __forceinline__ int vertex_pairs_wave(const Broad& B, const PairCtx& P, int w, long long o, int2* out,
                                                 long long cap) {
  const int lane = threadIdx.x & (kWave - 1);
  const int v = B.surf[w];
  const V3<double> p = ldx(P.x, v);
  const int3 c = cell_of(p, P.inv);
  const unsigned long long key = cell_key(c.x, c.y, c.z);
  const unsigned h = hash_key(key, B.tsize, false);
  const int s0 = B.start[h], s1 = B.start[h + 1];
  int count = 0;
  for (int t0 = s0; t0 < s1; t0 += kWave) {
    const int t = t0 + lane;
    int2 pr;
    const int hit = (t < s1 && vertex_slot_pair(B, P, v, p, key, t, pr)) ? 1 : 0;
    int tot;
    const int before = wave_excl_scan(hit, tot);
    if (FILL && hit) {
      const long long k = o + count + before;
      if (k < cap) out[k] = pr;
    }
    count += tot;
  }
  return count;
}

// Edge-edge pairs of edge slot s with the later edges of its cell.
template <typename Rec, typename Emit>
__device__ __forceinline__ void edge_pairs(const Broad& B, const PairCtx& P, const Rec& R, int s, Emit&& emit) {
  const int ebase = B.nSV + B.nF;
  const int ia = R.item(s);
  const unsigned long long key = R.key(s);
  const unsigned h = hash_key(key, B.tsize, true);
  const int s0 = B.start[h], s1 = B.start[h + 1];
  const V3<double> a0 = R.lo(s), a1 = R.hi(s);   // end points
  const V3<double> loA = vmin3(a0, a1), hiA = vmax3(a0, a1);
  const int4 idA = R.ids(s);
  const double r = P.r, q = 0.5 * P.r + kEdgeMargin;
  for (int t = s0; t < s1; ++t) {
    const int ib = R.item(t);
    if (ib <= ia || R.key(t) != key) continue;
    const int4 idB = R.ids(t);
    if (idA.x == idB.x || idA.x == idB.y || idA.y == idB.x || idA.y == idB.y) continue;
    const V3<double> b0 = R.lo(t), b1 = R.hi(t);
    const V3<double> lo = vmin3(b0, b1), hi = vmax3(b0, b1);
    // exact test with e1 = this (smaller) edge
    if (!((loA.x - r) <= hi.x && (loA.y - r) <= hi.y && (loA.z - r) <= hi.z)) continue;
    if (!(lo.x <= (hiA.x + r) && lo.y <= (hiA.y + r) && lo.z <= (hiA.z + r))) continue;
    // report only in the cell of the lower corner of the culling-box intersection
    const V3<double> corner = mk3(fmax(loA.x - q, lo.x - q), fmax(loA.y - q, lo.y - q), fmax(loA.z - q, lo.z - q));
    const int3 cc = cell_of(corner, P.inv);
    if (cell_key(cc.x, cc.y, cc.z) != key) continue;
    const int e1 = ia - ebase, e2 = ib - ebase;
    // distance filter before the exclusion lookup (see vertex_slot_pair)
    if (P.filter_d >= 0.0) {
      if (P.filter_obj && B.oid[idA.x] != B.oid[idB.x]) continue;
      if (!(closest_ee(a0, a1, b0, b1).d < P.filter_d)) continue;
    }
    const unsigned long long pk = ((unsigned long long)(unsigned)e1 << 32) | (unsigned)e2;
    if (B.n_excl_ee && in_sorted(B.excl_ee, B.n_excl_ee, pk)) continue;
    emit(make_int2(e1, e2));
  }
}

// Edge-edge test of two slots of one bucket, the pair reported once: e1 is
// the edge with the smaller item id, whose record takes the first place in
// the exact box test, the reporting-cell test and the distance (the same
// evaluation as edge_pairs from e1's side).  Emits (e1, ~e2).
template <typename Rec>
__device__ __forceinline__ bool edge_slot_pair_test(const Broad& B, const PairCtx& P, const Rec& R, int s, int t,
                                                    int2& out) {
  const int ebase = B.nSV + B.nF;
  const unsigned long long key = R.key(s);
  if (R.key(t) != key) return false;
  int sa = s, sb = t;
  if (R.item(t) < R.item(s)) {
    sa = t;
    sb = s;
  }
  const int4 idA = R.ids(sa), idB = R.ids(sb);
  if (idA.x == idB.x || idA.x == idB.y || idA.y == idB.x || idA.y == idB.y) return false;
  const V3<double> a0 = R.lo(sa), a1 = R.hi(sa), b0 = R.lo(sb), b1 = R.hi(sb);
  const V3<double> loA = vmin3(a0, a1), hiA = vmax3(a0, a1), lo = vmin3(b0, b1), hi = vmax3(b0, b1);
  const double r = P.r, q = 0.5 * P.r + kEdgeMargin;
  if (!((loA.x - r) <= hi.x && (loA.y - r) <= hi.y && (loA.z - r) <= hi.z)) return false;
  if (!(lo.x <= (hiA.x + r) && lo.y <= (hiA.y + r) && lo.z <= (hiA.z + r))) return false;
  const V3<double> corner = mk3(fmax(loA.x - q, lo.x - q), fmax(loA.y - q, lo.y - q), fmax(loA.z - q, lo.z - q));
  const int3 cc = cell_of(corner, P.inv);
  if (cell_key(cc.x, cc.y, cc.z) != key) return false;
  const int e1 = R.item(sa) - ebase, e2 = R.item(sb) - ebase;
  if (P.filter_d >= 0.0) {
    if (P.filter_obj && B.oid[idA.x] != B.oid[idB.x]) return false;
    if (!(closest_ee(a0, a1, b0, b1).d < P.filter_d)) return false;
  }
  const unsigned long long pk = ((unsigned long long)(unsigned)e1 << 32) | (unsigned)e2;
  if (B.n_excl_ee && in_sorted(B.excl_ee, B.n_excl_ee, pk)) return false;
  out = make_int2(e1, ~e2);
  return true;
}

// Load the edge buckets covering slots [S, S + kBlock) into LDS; returns the
// first slot of the span, or -1 if the span does not fit.
__device__ __forceinline__ int load_span(const Broad& B, SlotSpan& L, long long S, long long E) {
  const int lo = B.start[hash_key(B.bkt_key[S], B.tsize, true)];
  const int hi = B.start[hash_key(B.bkt_key[E - 1], B.tsize, true) + 1];
  const bool fits = hi - lo <= kSpan;
  if (fits) {
    for (int t = threadIdx.x; t < hi - lo; t += kBlock) {
      L.key[t] = B.bkt_key[lo + t];
      L.item[t] = B.bkt_item[lo + t];
      const int4 id = B.bkt_ids[lo + t];
      L.ids[t] = make_int2(id.x, id.y);
      const double4 a = B.bkt_lo[lo + t], b = B.bkt_hi[lo + t];
      L.lo[0][t] = a.x; L.lo[1][t] = a.y; L.lo[2][t] = a.z;
      L.hi[0][t] = b.x; L.hi[1][t] = b.y; L.hi[2][t] = b.z;
    }
  }
  __syncthreads();
  return fits ? lo : -1;
}

template <typename Emit>
__device__ __forceinline__ void edge_slot_pairs(const Broad& B, const PairCtx& P, const SlotSpan& L, int base, int s,
                                                Emit&& emit) {
  if (base >= 0) edge_pairs(B, P, LdsRec{L, base}, s, emit);
  else edge_pairs(B, P, GlobalRec{B}, s, emit);
}

// Work items: [0, nSV) surface vertices (point-triangle), then the edge slots
// [start[tsize/2], start[tsize]) (edge-edge).  part_cnt[w] = pairs of item w;
// every slot below work_cap is written, so no stale count survives.
__global__ void __launch_bounds__(kBlock) k_pairs_count(Broad B, PairCtx P) {
  __shared__ SlotSpan L;
  const long long e0 = B.start[B.tsize >> 1], e1 = B.start[B.tsize];
  const long long nw = B.nSV + (e1 - e0);
  // vertices: one wave each
  {
    const long long wid = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const long long nwv = ((long long)gridDim.x * kBlock) >> 6;
    for (long long w = wid; w < B.nSV; w += nwv) {
      const int c = vertex_pairs_wave<false>(B, P, (int)w, 0, nullptr, 0);
      if ((threadIdx.x & (kWave - 1)) == 0) B.part_cnt[w] = c;
    }
  }
  // edge slots: a block takes kBlock consecutive slots and their buckets in LDS
  for (long long S = e0 + (long long)blockIdx.x * kBlock; S < e1; S += (long long)gridDim.x * kBlock) {
    const long long s = S + threadIdx.x;
    const int base = load_span(B, L, S, min(S + (long long)kBlock, e1));
    int c = 0;
    if (s < e1) edge_slot_pairs(B, P, L, base, (int)s, [&](int2) { ++c; });
    __syncthreads();
    if (s < e1) B.part_cnt[B.nSV + (s - e0)] = c;
  }
  for (long long w = nw + blockIdx.x * kBlock + threadIdx.x; w < B.work_cap; w += (long long)gridDim.x * kBlock)
    B.part_cnt[w] = 0;
}

__global__ void __launch_bounds__(kBlock) k_pairs_fill(Broad B, PairCtx P, int2* out, long long cap) {
  __shared__ SlotSpan L;
  const long long e0 = B.start[B.tsize >> 1], e1 = B.start[B.tsize];
  {
    const long long wid = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const long long nwv = ((long long)gridDim.x * kBlock) >> 6;
    for (long long w = wid; w < B.nSV; w += nwv) vertex_pairs_wave<true>(B, P, (int)w, B.part_off[w], out, cap);
  }
  for (long long S = e0 + (long long)blockIdx.x * kBlock; S < e1; S += (long long)gridDim.x * kBlock) {
    const long long s = S + threadIdx.x;
    const int base = load_span(B, L, S, min(S + (long long)kBlock, e1));
    if (s < e1) {
      long long o = B.part_off[B.nSV + (s - e0)];
      edge_slot_pairs(B, P, L, base, (int)s, [&](int2 pr) {
        if (o < cap) out[o] = pr;
        ++o;
      });
    }
    __syncthreads();
  }
}

// Single-pass emission for the solver's list: every pair found is appended
// at a position reserved with one atomic per wave (point-triangle) or per
// block (edge-edge), in no particular order; the kind is in the pair:
// (v, f) point-triangle, (e1, ~e2) edge-edge.  counter counts every pair
// found, also those past cap (the caller checks it against cap).
constexpr int kEbuf = 2 * kBlock;   // edge-edge pairs buffered per block before one counter update

__device__ __forceinline__ int block_excl_scan(int v, int& total, int* sh) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  int wt;
  const int x = wave_excl_scan(v, wt);
  if (lane == 0) sh[w] = wt;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int i = 0; i < kBlock / kWave; ++i) {
    if (i < w) before += sh[i];
    total += sh[i];
  }
  __syncthreads();
  return before + x;
}

__global__ void __launch_bounds__(kBlock) k_pairs_emit(Broad B, PairCtx P, int2* out, long long cap,
                                                      unsigned long long* counter) {
  __shared__ SlotSpan L;
  __shared__ int2 ebuf[kEbuf];
  __shared__ int soff[kBlock + 1];
  __shared__ int ssum[kBlock / kWave];
  __shared__ int ecount;
  __shared__ unsigned long long sbase;
  const int lane = threadIdx.x & (kWave - 1);
  const long long e0 = B.start[B.tsize >> 1], e1 = B.start[B.tsize];
  // point-triangle: one wave per surface vertex, one lane per bucket slot
  {
    const long long wid = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const long long nwv = ((long long)gridDim.x * kBlock) >> 6;
    for (long long w = wid; w < B.nSV; w += nwv) {
      const int v = B.surf[w];
      const V3<double> p = ldx(P.x, v);
      const int3 c = cell_of(p, P.inv);
      const unsigned long long key = cell_key(c.x, c.y, c.z);
      const unsigned h = hash_key(key, B.tsize, false);
      const int s0 = B.start[h], s1 = B.start[h + 1];
      for (int t0 = s0; t0 < s1; t0 += kWave) {
        const int t = t0 + lane;
        int2 pr;
        const int hit = (t < s1 && vertex_slot_pair(B, P, v, p, key, t, pr)) ? 1 : 0;
        int tot;
        const int before = wave_excl_scan(hit, tot);
        if (tot == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(counter, (unsigned long long)tot);
        base = __shfl(base, 0, kWave);
        if (hit && (long long)(base + before) < cap) out[base + before] = pr;
      }
    }
  }
  // edge-edge: a block takes kBlock consecutive edge slots with their
  // buckets in LDS and enumerates the pairs (s, t), t a later slot of s's
  // bucket, spread evenly over its threads (pair i of the block goes to
  // thread i mod kBlock), so that a long bucket does not hold up a wave
  for (long long S = e0 + (long long)blockIdx.x * kBlock; S < e1; S += (long long)gridDim.x * kBlock) {
    const long long s = S + threadIdx.x;
    const long long Send = min(S + (long long)kBlock, e1);
    const int base = load_span(B, L, S, Send);
    int c = 0;
    if (s < e1) c = B.start[hash_key(B.bkt_key[s], B.tsize, true) + 1] - (int)s - 1;
    int total;
    const int before = block_excl_scan(c, total, ssum);
    soff[threadIdx.x] = before;
    if (threadIdx.x == 0) {
      soff[kBlock] = total;
      ecount = 0;
    }
    __syncthreads();
    for (int r0 = 0; r0 < total; r0 += kBlock) {
      const int i = r0 + threadIdx.x;
      if (i < total) {
        // the slot whose pairs hold index i: largest j with soff[j] <= i
        int lo = 0, hi = kBlock;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (soff[mid] <= i) lo = mid; else hi = mid;
        }
        const int sa = (int)S + lo, sb = sa + 1 + (i - soff[lo]);
        int2 pr;
        const bool hit = base >= 0 ? edge_slot_pair_test(B, P, LdsRec{L, base}, sa, sb, pr)
                                   : edge_slot_pair_test(B, P, GlobalRec{B}, sa, sb, pr);
        if (hit) ebuf[atomicAdd(&ecount, 1)] = pr;
      }
      __syncthreads();
      // every thread reads the count before any thread changes it again, so
      // the flush decision is the same in the whole block
      const int n = ecount;
      __syncthreads();
      // flush when another round could overflow the buffer, and at the end
      if (n > kEbuf - kBlock || r0 + kBlock >= total) {
        if (threadIdx.x == 0) {
          sbase = n ? atomicAdd(counter, (unsigned long long)n) : 0ull;
          ecount = 0;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += kBlock)
          if ((long long)(sbase + j) < cap) out[sbase + j] = ebuf[j];
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// ncand[0] = 0 (the counter), ncand[1] = -1 (the kind is in the pair)

// Flags a grid or list that did not fit (the list is then incomplete) and
// records the list size; with a pair index (vcnt non-null) also zeroes its
// per-vertex counters, and with xbuild copies the build positions.
__global__ void __launch_bounds__(kBlock) k_list_check(Broad B, const long long* ncand, long long cap, int* err,
                                                       long long* n_out, int* vcnt, int* big, int nV,
                                                       double4* xbuild, const double4* x) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (B.totals[0] > B.ent_cap || ncand[0] > cap) atomicOr(err, kErrCapacity);
    *n_out = ncand[0];
    if (big) big[0] = 0;
  }
  const int stride = gridDim.x * kBlock;
  if (vcnt)
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < 2 * nV; i += stride) vcnt[i] = 0;
  if (xbuild)
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < nV; v += stride) xbuild[v] = x[v];
}

// totals[2] = number of point-triangle pairs = offset of the first edge-edge slot
__global__ void k_pt_total(Broad B) {
  if (threadIdx.x == 0 && blockIdx.x == 0) B.totals[2] = B.part_off[B.nSV];
}

__global__ void __launch_bounds__(kBlock) k_plane_cand(Broad B, const double4* x, Planes P, double r, int2* out,
                                                       long long* n, long long cap) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < B.nSV; i += gridDim.x * kBlock) {
    const int v = B.surf[i];
    const V3<double> p = ldx(x, v);
    for (int j = 0; j < P.n; ++j) {
      const double* pl = P.p[j];
      double s;
      {
#pragma clang fp contract(off)
        s = ((pl[0] * p.x + pl[1] * p.y) + pl[2] * p.z) - pl[3];
      }
      if (s <= r) {
        unsigned long long slot = atomicAdd((unsigned long long*)n, 1ull);
        if ((long long)slot < cap) out[slot] = make_int2(v, j);
      }
    }
  }
}

// --------------------------------------------- canonical order of a list
// kind (0 point-triangle, 1 edge-edge) and the two indices of pair q
__device__ __forceinline__ void pl_decode(int2 pr, long long q, long long npt, int& kind, int& a, int& b) {
  if (npt >= 0) {
    kind = q < npt ? 0 : 1;
    a = pr.x;
    b = pr.y;
  } else if (pr.y >= 0) {
    kind = 0;
    a = pr.x;
    b = pr.y;
  } else {
    kind = 1;
    a = pr.x;
    b = ~pr.y;
  }
}
// the four vertices in the order the narrow phase uses them
__device__ __forceinline__ void pl_corners(const PairIndex& P, int kind, int a, int b, int (&v)[4]) {
  if (kind == 0) {
    v[0] = a;
    v[1] = P.tris[3 * b];
    v[2] = P.tris[3 * b + 1];
    v[3] = P.tris[3 * b + 2];
  } else {
    v[0] = P.edges[2 * a];
    v[1] = P.edges[2 * a + 1];
    v[2] = P.edges[2 * b];
    v[3] = P.edges[2 * b + 1];
  }
}

__global__ void __launch_bounds__(kBlock) k_pl_zero(PairIndex P) {
  const int nv = 2 * P.nV;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nv; i += gridDim.x * kBlock) P.vcnt[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.big[0] = 0;
}

// corner entries per vertex
__global__ void __launch_bounds__(kBlock) k_pl_count(PairIndex P, const int2* list, const long long* ncand,
                                                     long long cap) {
  const long long n = min(ncand[0], cap), npt = ncand[1];
  for (long long q = blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
    int kind, a, b;
    pl_decode(list[q], q, npt, kind, a, b);
    int v[4];
    pl_corners(P, kind, a, b, v);
    P.pv[q] = make_int4(v[0], v[1], v[2], kind == 0 ? v[3] : ~v[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) atomicAdd(&P.vcnt[v[i]], 1);
  }
}

// Content key of pair q: kind, then its two indices.  A vertex belongs to a
// pair at most once, so the keys of one vertex's entries are distinct, and
// their order does not depend on the list order.
__device__ __forceinline__ unsigned long long pair_key(int kind, int a, int b) {
  return ((unsigned long long)kind << 62) | ((unsigned long long)(unsigned)a << 31) | (unsigned long long)(unsigned)b;
}

// entries grouped by vertex (slot ids 4 q + corner and their pairs' keys, in
// no particular order within a vertex) and the entry range of each
// incidence wave
__global__ void __launch_bounds__(kBlock) k_pl_corners(PairIndex P, const int2* list, const long long* ncand,
                                                       long long cap) {
  const long long n = min(ncand[0], cap), npt = ncand[1];
  for (long long q = blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
    int kind, a, b;
    pl_decode(list[q], q, npt, kind, a, b);
    const unsigned long long key = pair_key(kind, a, b);
    int v[4];
    pl_corners(P, kind, a, b, v);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pos = P.coff[v[i]] + atomicAdd(&P.vcnt[P.nV + v[i]], 1);
      P.cent_tmp[pos] = (int)(4 * q + i);
      P.ckey_tmp[pos] = key;
    }
  }
  for (int w = blockIdx.x * kBlock + threadIdx.x; w < P.nWaves; w += gridDim.x * kBlock) {
    const int2 fv = P.wvert[w];
    P.wrange[w] = make_int2(P.coff[fv.x], P.coff[fv.y + 1]);
  }
}

// Each vertex's entries [coff[v], coff[v + 1]) of cent_tmp go to the same
// range of cent in ascending key order: every entry is written at its rank
// (the number of smaller keys of the vertex), which depends on the pairs
// only.  One thread per vertex with at most kRankSmall entries (held in
// registers); vertices with more are listed in big (count in big[0]) for
// k_rank_big.
constexpr int kRankSmall = 16;
constexpr int kRankLds = 1024;   // keys of a vertex staged in LDS by k_rank_big

__global__ void __launch_bounds__(kBlock) k_rank_small(PairIndex P) {
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < P.nV; v += gridDim.x * kBlock) {
    const int s0 = P.coff[v], n = P.coff[v + 1] - s0;
    if (n <= 0) continue;
    if (n > kRankSmall) {
      P.big[1 + atomicAdd(&P.big[0], 1)] = v;
      continue;
    }
    int e[kRankSmall];
    unsigned long long k[kRankSmall];
#pragma unroll
    for (int i = 0; i < kRankSmall; ++i)
      if (i < n) {
        e[i] = P.cent_tmp[s0 + i];
        k[i] = P.ckey_tmp[s0 + i];
      }
#pragma unroll
    for (int i = 0; i < kRankSmall; ++i) {
      if (i >= n) break;
      int r = 0;
#pragma unroll
      for (int j = 0; j < kRankSmall; ++j)
        if (j < n && k[j] < k[i]) ++r;
      P.cent[s0 + r] = e[i];
    }
  }
}

// One block per listed vertex: its keys are staged in LDS (up to kRankLds;
// beyond that they are read from memory) and each thread ranks entries
// tid, tid + kBlock, ... against all of them.
__global__ void __launch_bounds__(kBlock) k_rank_big(PairIndex P) {
  __shared__ unsigned long long ks[kRankLds];
  const int nbig = P.big[0];
  for (int w = blockIdx.x; w < nbig; w += gridDim.x) {
    const int v = P.big[1 + w];
    const int s0 = P.coff[v], n = P.coff[v + 1] - s0;
    const bool lds = n <= kRankLds;
    if (lds)
      for (int i = threadIdx.x; i < n; i += kBlock) ks[i] = P.ckey_tmp[s0 + i];
    __syncthreads();
    const unsigned long long* kk = lds ? ks : P.ckey_tmp + s0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
      const unsigned long long ki = kk[i];
      int r = 0;
      for (int j = 0; j < n; ++j) r += kk[j] < ki ? 1 : 0;
      P.cent[s0 + r] = P.cent_tmp[s0 + i];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_pl_install(const int2* src, long long n, int2* out, long long* ncand,
                                                       long long* n_out) {
  for (long long q = blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) out[q] = src[q];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ncand[0] = n;
    ncand[1] = -1;
    *n_out = n;
  }
}

}  // namespace

void pairs_index(const PairIndex& P, const int2* list, const long long* ncand, long long cap, hipStream_t s,
                 bool zeroed) {
  if (!zeroed) hipLaunchKernelGGL(k_pl_zero, dim3(P.grid), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_pl_count, dim3(P.grid), dim3(kBlock), 0, s, P, list, ncand, cap);
  scan_exclusive<int>(P.vcnt, P.nV, P.coff, P.coff + P.nV, P.scan_tmp, s);
  hipLaunchKernelGGL(k_pl_corners, dim3(P.grid), dim3(kBlock), 0, s, P, list, ncand, cap);
  hipLaunchKernelGGL(k_rank_small, dim3(P.grid), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_rank_big, dim3(P.grid), dim3(kBlock), 0, s, P);
}

__global__ void __launch_bounds__(kBlock) k_copy_positions(double4* dst, const double4* src, int n) {
  for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) dst[v] = src[v];
}

void copy_positions(double4* dst, const double4* src, int n, hipStream_t s) {
  const int g = std::min((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_copy_positions, dim3(std::max(g, 1)), dim3(kBlock), 0, s, dst, src, n);
}

void pairs_install(const int2* src, long long n, int2* out, long long* ncand, long long* n_out, hipStream_t s) {
  const int g = (int)std::min<long long>(std::max<long long>((n + kBlock - 1) / kBlock, 1), 1024);
  hipLaunchKernelGGL(k_pl_install, dim3(g), dim3(kBlock), 0, s, src, n, out, ncand, n_out);
}

void broad_build_count(const Broad& B, const double4* x, double cell, double r, double filter_d, int filter_obj,
                       hipStream_t s) {
  const double inv = 1.0 / cell;
  const int n = B.nF + B.nE;
  hipLaunchKernelGGL(k_items, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv, r, (long long*)nullptr);
  scan_exclusive<long long>(B.item_cnt, n, B.item_off, B.totals, B.part_off + B.work_cap, s);
  hipLaunchKernelGGL(k_emit, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv, r);
  scan_exclusive<int>(B.count, B.tsize, B.start, B.start + B.tsize, (int*)(B.part_off + B.work_cap), s);
  hipLaunchKernelGGL(k_bucket_fill, dim3(B.grid), dim3(kBlock), 0, s, B, x);
  PairCtx P{x, inv, r, filter_d, filter_obj};
  const int nb = (int)std::min<long long>((B.ent_cap + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_pairs_count, dim3(nb), dim3(kBlock), 0, s, B, P);
  scan_exclusive<long long>(B.part_cnt, B.work_cap, B.part_off, B.totals + 1, B.part_off + B.work_cap, s);
  hipLaunchKernelGGL(k_pt_total, dim3(1), dim3(64), 0, s, B);
}

void broad_fill(const Broad& B, const double4* x, double cell, double r, double filter_d, int filter_obj, int2* out,
                long long cap, hipStream_t s) {
  PairCtx P{x, 1.0 / cell, r, filter_d, filter_obj};
  const int nb = (int)std::min<long long>((B.ent_cap + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_pairs_fill, dim3(nb), dim3(kBlock), 0, s, B, P, out, cap);
}

void broad_solver_list(const Broad& B, const double4* x, double cell, double r, int2* out, long long cap,
                       long long* ncand, int* err, long long* n_out, hipStream_t s, const PairIndex* P,
                       double4* xbuild) {
  const double inv = 1.0 / cell;
  const int n = B.nF + B.nE;
  hipLaunchKernelGGL(k_items, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv, r, ncand);
  scan_exclusive<long long>(B.item_cnt, n, B.item_off, B.totals, B.part_off + B.work_cap, s);
  hipLaunchKernelGGL(k_emit, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv, r);
  scan_exclusive<int>(B.count, B.tsize, B.start, B.start + B.tsize, (int*)(B.part_off + B.work_cap), s);
  hipLaunchKernelGGL(k_bucket_fill, dim3(B.grid), dim3(kBlock), 0, s, B, x);
  PairCtx PC{x, inv, r, r, 0};
  const int nb = (int)std::min<long long>((B.ent_cap + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_pairs_emit, dim3(nb), dim3(kBlock), 0, s, B, PC, out, cap, (unsigned long long*)ncand);
  hipLaunchKernelGGL(k_list_check, dim3((P || xbuild) ? B.grid : 1), dim3(kBlock), 0, s, B, (const long long*)ncand,
                     cap, err, n_out, P ? P->vcnt : nullptr, P ? P->big : nullptr, B.nV, xbuild, x);
}

void plane_candidates(const Broad& B, const double4* x, const Planes& planes, double r, int2* out, long long* n,
                      long long cap, hipStream_t s) {
  (void)hipMemsetAsync(n, 0, sizeof(long long), s);
  hipLaunchKernelGGL(k_plane_cand, dim3(B.grid), dim3(kBlock), 0, s, B, x, planes, r, out, n, cap);
}

}  // namespace pncg
