// Broad phase: candidate point-triangle and edge-edge pairs by an inflated
// axis-aligned box test in float64 over a uniform-grid spatial hash (the
// paper culls with a grid hash, Sec. 6; the hash changes speed, not the set).
//
//   PT (v, f): v a surface vertex not in f, and on every axis
//              min_f - r <= x_v <= max_f + r
//   EE (e1 < e2) without a shared vertex, on every axis
//              min_e1 - r <= max_e2  and  min_e2 <= max_e1 + r
//
// Surface vertices are hashed by their cell; edges by the cell of their
// lower box corner.  A triangle visits the cells its inflated box covers; an
// edge e2 visits the cells where the lower corner of a qualifying e1 can lie
// (widened by the largest edge extent).  Each pair is found exactly once:
// a vertex or edge lives in one cell, and a visit only accepts items whose
// own cell is the visited cell (hash collisions are filtered).
//
// Output is produced without any global counter: a counting pass stores the
// number of pairs of every thread, an exclusive scan turns the counts into
// offsets (point-triangle counts first, then edge-edge), and a second pass
// writes the pairs.  Buckets are sorted by item index, so the list order is
// deterministic.
#include <climits>

#include "kernels.h"

namespace pncg {

namespace {

constexpr int kTile = kBlock * 16;

__device__ __forceinline__ int cell_coord(double p, double inv) {
  double c = floor(p * inv);
  c = fmin(fmax(c, -1048576.0), 1048576.0);
  return (int)c;
}
__device__ __forceinline__ int3 cell_of(V3<double> p, double inv) {
  return make_int3(cell_coord(p.x, inv), cell_coord(p.y, inv), cell_coord(p.z, inv));
}
__device__ __forceinline__ unsigned hash_cell(int cx, int cy, int cz, int tsize) {
  unsigned h = ((unsigned)cx * 73856093u) ^ ((unsigned)cy * 19349663u) ^ ((unsigned)cz * 83492791u);
  return h & (unsigned)(tsize - 1);
}
__device__ __forceinline__ V3<double> ldx(const double4* x, int i) {
  double4 v = x[i];
  return mk3(v.x, v.y, v.z);
}
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

// exclusive scan of nb block sums in place (one block, nb <= kBlock * 16)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_top(T* bsum, int nb) {
  __shared__ T sh[kBlock];
  const int per = (nb + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per;
  T s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += bsum[b0 + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    T v = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  T run = sh[threadIdx.x] - s;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      T v = bsum[b0 + i];
      bsum[b0 + i] = run;
      run += v;
    }
}

// out[j] = exclusive prefix of in[j]; *total = sum (written by the last block)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_down(const T* in, long long n, const T* boff, T* out, T* total) {
  __shared__ T sh[kBlock];
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
  for (int o = 1; o < kBlock; o <<= 1) {
    T u = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += u;
    __syncthreads();
  }
  T run = boff[blockIdx.x] + sh[threadIdx.x] - s;
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
  hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kBlock), 0, s, scratch, nb);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kBlock), 0, s, in, n, (const T*)scratch, out, total);
}

// ------------------------------------------------------------ hash build
__global__ void __launch_bounds__(kBlock) k_zero_int(int* a, int n) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) a[i] = 0;
}

__device__ __forceinline__ V3<double> item_key_point(const Broad& B, const double4* x, int it) {
  if (it < B.nSV) return ldx(x, B.surf[it]);
  const int e = it - B.nSV;
  return vmin3(ldx(x, B.edges[2 * e]), ldx(x, B.edges[2 * e + 1]));
}

__global__ void __launch_bounds__(kBlock) k_hash_count(Broad B, const double4* x, double inv) {
  __shared__ double sh[3][kBlock / kWave];
  const int n = B.nSV + B.nE;
  double ext[3] = {0.0, 0.0, 0.0};
  for (int it = blockIdx.x * kBlock + threadIdx.x; it < n; it += gridDim.x * kBlock) {
    V3<double> k = item_key_point(B, x, it);
    int3 c = cell_of(k, inv);
    atomicAdd(&B.count[hash_cell(c.x, c.y, c.z, B.tsize)], 1);
    if (it >= B.nSV) {
      const int e = it - B.nSV;
      V3<double> a = ldx(x, B.edges[2 * e]), b = ldx(x, B.edges[2 * e + 1]);
      V3<double> mx = vmax3(a, b);
      ext[0] = fmax(ext[0], mx.x - k.x);
      ext[1] = fmax(ext[1], mx.y - k.y);
      ext[2] = fmax(ext[2], mx.z - k.z);
    }
  }
  for (int j = 0; j < 3; ++j) {
    double v = ext[j];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
    if ((threadIdx.x & 63) == 0) sh[j][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < 3; ++j) {
      double m = 0.0;
      for (int w = 0; w < kBlock / kWave; ++w) m = fmax(m, sh[j][w]);
      B.part_ext[3 * blockIdx.x + j] = m;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_hash_fill(Broad B, const double4* x, double inv) {
  const int n = B.nSV + B.nE;
  for (int it = blockIdx.x * kBlock + threadIdx.x; it < n; it += gridDim.x * kBlock) {
    int3 c = cell_of(item_key_point(B, x, it), inv);
    const unsigned h = hash_cell(c.x, c.y, c.z, B.tsize);
    const int slot = atomicAdd(&B.count[h], 1);
    B.items[B.start[h] + slot] = it;
  }
}

// insertion sort of every bucket by item index
__global__ void __launch_bounds__(kBlock) k_hash_sort(Broad B) {
  for (int h = blockIdx.x * kBlock + threadIdx.x; h < B.tsize; h += gridDim.x * kBlock) {
    const int s0 = B.start[h], s1 = B.start[h + 1];
    for (int i = s0 + 1; i < s1; ++i) {
      const int v = B.items[i];
      int j = i - 1;
      while (j >= s0 && B.items[j] > v) {
        B.items[j + 1] = B.items[j];
        --j;
      }
      B.items[j + 1] = v;
    }
  }
}

// --------------------------------------------------------------- queries
// Visit every candidate of query `q` (a triangle when q < nF, else an edge
// e2 = q - nF) and call emit(a, b) for each pair in a fixed order.
template <typename Emit>
__device__ __forceinline__ void visit_query(const Broad& B, const double4* x, double inv, double r, double filter_d,
                                            const double ext[3], int q, Emit&& emit) {
  const int tsize = B.tsize;
  if (q < B.nF) {
    const int f = q;
    const int a = B.tris[3 * f], b = B.tris[3 * f + 1], c = B.tris[3 * f + 2];
    const V3<double> pa = ldx(x, a), pb = ldx(x, b), pc = ldx(x, c);
    const V3<double> mn = vmin3(vmin3(pa, pb), pc), mx = vmax3(vmax3(pa, pb), pc);
    const V3<double> lo = mk3(mn.x - r, mn.y - r, mn.z - r);
    const V3<double> hi = mk3(mx.x + r, mx.y + r, mx.z + r);
    const int3 c0 = cell_of(lo, inv), c1 = cell_of(hi, inv);
    for (int cx = c0.x; cx <= c1.x; ++cx)
      for (int cy = c0.y; cy <= c1.y; ++cy)
        for (int cz = c0.z; cz <= c1.z; ++cz) {
          const unsigned h = hash_cell(cx, cy, cz, tsize);
          const int s1 = B.start[h + 1];
          for (int s = B.start[h]; s < s1; ++s) {
            const int it = B.items[s];
            if (it >= B.nSV) break;   // buckets are sorted: edge items follow vertex items
            const int v = B.surf[it];
            if (v == a || v == b || v == c) continue;
            const V3<double> p = ldx(x, v);
            const int3 pc3 = cell_of(p, inv);
            if (pc3.x != cx || pc3.y != cy || pc3.z != cz) continue;
            if (!(lo.x <= p.x && p.x <= hi.x && lo.y <= p.y && p.y <= hi.y && lo.z <= p.z && p.z <= hi.z)) continue;
            const unsigned long long key = ((unsigned long long)(unsigned)v << 32) | (unsigned)f;
            if (B.n_excl_pt && in_sorted(B.excl_pt, B.n_excl_pt, key)) continue;
            if (filter_d >= 0.0) {
              if (B.oid[v] != B.oid[a]) continue;
              if (!(closest_pt(p, pa, pb, pc).d < filter_d)) continue;
            }
            emit(0, v, f);
          }
        }
  } else {
    const int e2 = q - B.nF;
    const int a2 = B.edges[2 * e2], b2 = B.edges[2 * e2 + 1];
    const V3<double> pa2 = ldx(x, a2), pb2 = ldx(x, b2);
    const V3<double> mn2 = vmin3(pa2, pb2), mx2 = vmax3(pa2, pb2);
    // the lower corner of a qualifying e1 lies in [mn2 - r - ext, mx2 + r]
    const double marg = 1e-9;
    const V3<double> lo = mk3(mn2.x - r - ext[0] - marg, mn2.y - r - ext[1] - marg, mn2.z - r - ext[2] - marg);
    const V3<double> hi = mk3(mx2.x + r + marg, mx2.y + r + marg, mx2.z + r + marg);
    const int3 c0 = cell_of(lo, inv), c1 = cell_of(hi, inv);
    for (int cx = c0.x; cx <= c1.x; ++cx)
      for (int cy = c0.y; cy <= c1.y; ++cy)
        for (int cz = c0.z; cz <= c1.z; ++cz) {
          const unsigned h = hash_cell(cx, cy, cz, tsize);
          const int s1 = B.start[h + 1];
          for (int s = B.start[h]; s < s1; ++s) {
            const int it = B.items[s];
            if (it < B.nSV) continue;
            const int e1 = it - B.nSV;
            if (e1 >= e2) break;      // sorted bucket: no smaller edge index follows
            const int a1 = B.edges[2 * e1], b1 = B.edges[2 * e1 + 1];
            if (a1 == a2 || a1 == b2 || b1 == a2 || b1 == b2) continue;
            const V3<double> pa1 = ldx(x, a1), pb1 = ldx(x, b1);
            const V3<double> mn1 = vmin3(pa1, pb1), mx1 = vmax3(pa1, pb1);
            const int3 k3 = cell_of(mn1, inv);
            if (k3.x != cx || k3.y != cy || k3.z != cz) continue;
            if (!((mn1.x - r) <= mx2.x && (mn1.y - r) <= mx2.y && (mn1.z - r) <= mx2.z)) continue;
            if (!(mn2.x <= (mx1.x + r) && mn2.y <= (mx1.y + r) && mn2.z <= (mx1.z + r))) continue;
            const unsigned long long key = ((unsigned long long)(unsigned)e1 << 32) | (unsigned)e2;
            if (B.n_excl_ee && in_sorted(B.excl_ee, B.n_excl_ee, key)) continue;
            if (filter_d >= 0.0) {
              if (B.oid[a1] != B.oid[a2]) continue;
              if (!(closest_ee(pa1, pb1, pa2, pb2).d < filter_d)) continue;
            }
            emit(1, e1, e2);
          }
        }
  }
}

__device__ __forceinline__ void reduce_ext(const Broad& B, double ext[3]) {
  ext[0] = ext[1] = ext[2] = 0.0;
  for (int j = 0; j < B.grid; ++j) {
    ext[0] = fmax(ext[0], B.part_ext[3 * j]);
    ext[1] = fmax(ext[1], B.part_ext[3 * j + 1]);
    ext[2] = fmax(ext[2], B.part_ext[3 * j + 2]);
  }
}

__global__ void __launch_bounds__(kBlock) k_query_count(Broad B, const double4* x, double inv, double r, double filter_d) {
  double ext[3];
  reduce_ext(B, ext);
  const int tid = blockIdx.x * kBlock + threadIdx.x, nth = gridDim.x * kBlock;
  long long cpt = 0, cee = 0;
  const int nq = B.nF + B.nE;
  for (int q = tid; q < nq; q += nth)
    visit_query(B, x, inv, r, filter_d, ext, q, [&](int kind, int, int) {
      if (kind == 0) ++cpt; else ++cee;
    });
  B.part_cnt[tid] = cpt;
  B.part_cnt[nth + tid] = cee;
}

__global__ void __launch_bounds__(kBlock) k_query_fill(Broad B, const double4* x, double inv, double r, double filter_d,
                                                       int2* out, long long cap) {
  double ext[3];
  reduce_ext(B, ext);
  const int tid = blockIdx.x * kBlock + threadIdx.x, nth = gridDim.x * kBlock;
  long long opt = B.part_off[tid], oee = B.part_off[nth + tid];
  const int nq = B.nF + B.nE;
  for (int q = tid; q < nq; q += nth)
    visit_query(B, x, inv, r, filter_d, ext, q, [&](int kind, int a, int b) {
      long long& o = kind == 0 ? opt : oee;
      if (o < cap) out[o] = make_int2(a, b);
      ++o;
    });
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

}  // namespace

void broad_build(const Broad& B, const double4* x, double cell, hipStream_t s) {
  const double inv = 1.0 / cell;
  hipLaunchKernelGGL(k_zero_int, dim3(B.grid), dim3(kBlock), 0, s, B.count, B.tsize);
  hipLaunchKernelGGL(k_hash_count, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv);
  // start = exclusive scan of count (start[tsize] = total); part_off serves as scratch
  scan_exclusive<int>(B.count, B.tsize, B.start, B.start + B.tsize, (int*)B.part_off, s);
  hipLaunchKernelGGL(k_zero_int, dim3(B.grid), dim3(kBlock), 0, s, B.count, B.tsize);
  hipLaunchKernelGGL(k_hash_fill, dim3(B.grid), dim3(kBlock), 0, s, B, x, inv);
  hipLaunchKernelGGL(k_hash_sort, dim3(B.grid), dim3(kBlock), 0, s, B);
}

void broad_count(const Broad& B, const double4* x, double cell, double r, double filter_d, hipStream_t s) {
  hipLaunchKernelGGL(k_query_count, dim3(B.grid), dim3(kBlock), 0, s, B, x, 1.0 / cell, r, filter_d);
}

void broad_scan(const Broad& B, long long* n_out, hipStream_t s) {
  const long long n = 2LL * B.grid * kBlock;
  // scratch for block sums: the tail of part_off beyond the 2n offsets
  scan_exclusive<long long>(B.part_cnt, n, B.part_off, n_out, B.part_off + n, s);
  // n_out[1] = offset of the first edge-edge pair = number of point-triangle pairs
  (void)hipMemcpyAsync(n_out + 1, B.part_off + (long long)B.grid * kBlock, sizeof(long long), hipMemcpyDeviceToDevice, s);
}

void broad_fill(const Broad& B, const double4* x, double cell, double r, double filter_d, int2* out, long long cap,
                hipStream_t s) {
  hipLaunchKernelGGL(k_query_fill, dim3(B.grid), dim3(kBlock), 0, s, B, x, 1.0 / cell, r, filter_d, out, cap);
}

void plane_candidates(const Broad& B, const double4* x, const Planes& planes, double r, int2* out, long long* n,
                      long long cap, hipStream_t s) {
  (void)hipMemsetAsync(n, 0, sizeof(long long), s);
  hipLaunchKernelGGL(k_plane_cand, dim3(B.grid), dim3(kBlock), 0, s, B, x, planes, r, out, n, cap);
}

}  // namespace pncg
