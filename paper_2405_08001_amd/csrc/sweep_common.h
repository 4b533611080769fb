// Helpers shared by the per-iteration kernels and the batched step kernel:
// wave / block reductions, wave-segmented sums, padded-vector loads and
// stores, the direction update, plane distances and lazy position reads.
#pragma once

#include "internal.h"

namespace pncg {

constexpr int kSWaves = kSBlock / kWave;

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
  return v;
}

// Sum (kind 0) or max (kind 1) of N per-thread values over a block of BS
// threads; the result is returned to every thread.  sh must hold
// (BS / 64) * N doubles.  The order of the additions is fixed.
template <int N, int BS = kSBlock>
__device__ __forceinline__ void block_reduce(double (&v)[N], const int (&kind)[N], double* sh) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = kind[i] ? wave_max(v[i]) : wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[w * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double r = sh[i];
    for (int j = 1; j < BS / kWave; ++j) r = kind[i] ? fmax(r, sh[j * N + i]) : r + sh[j * N + i];
    v[i] = r;
  }
  __syncthreads();
}

// Re-reduce the per-block partials [n][stride] of the previous launch.
template <int N, int BS = kSBlock>
__device__ __forceinline__ void reduce_partials(const double* part, int stride, int n, const int (&kind)[N],
                                                double (&out)[N], double* sh) {
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = kind[i] ? 0.0 : 0.0;
  for (int j = threadIdx.x; j < n; j += BS) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double v = part[j * stride + i];
      out[i] = kind[i] ? fmax(out[i], v) : out[i] + v;
    }
  }
  block_reduce<N, BS>(out, kind, sh);
}

// ------------------------------------------------------- work partitioning
// Workgroups are dispatched round-robin over the XCDs, each with its own L2.
// The logical block index below gives every XCD a contiguous range of
// logical blocks (the grid is a multiple of kXcds), and every logical block
// a contiguous slice of each work range, so an XCD touches one contiguous
// eighth of the mesh and its L2 holds that eighth's tets and vertices.
__device__ __forceinline__ int logical_block() {
  const int per = gridDim.x / kXcds;
  return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}
struct Slice {
  long long begin, end;
};
// slice of [0, n) for this block, in units of `unit` items
__device__ __forceinline__ Slice block_slice(long long n) {
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long b = (long long)logical_block() * per;
  return Slice{b, b + per < n ? b + per : n};
}

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ V3<double> ld3(const double4* a, int i) {
  double4 v = a[i];
  return mk3(v.x, v.y, v.z);
}
__device__ __forceinline__ void st3(double4* a, int i, V3<double> v) { a[i] = make_double4(v.x, v.y, v.z, 0.0); }

template <typename R>
__device__ __forceinline__ V3<R> ldr(const R4<R>* a, int i) {
  R4<R> v = a[i];
  return mk3(v.x, v.y, v.z);
}
template <typename R>
__device__ __forceinline__ void str(R4<R>* a, int i, V3<R> v) {
  R4<R> o;
  o.x = v.x; o.y = v.y; o.z = v.z; o.w = R(0);
  a[i] = o;
}

// the direction p_{k+1} = -P g + beta p_k, one rounding per component
template <typename R>
__device__ __forceinline__ V3<R> direction(V3<R> pg, V3<R> pprev, R beta) {
  return mk3(fma(beta, pprev.x, -pg.x), fma(beta, pprev.y, -pg.y), fma(beta, pprev.z, -pg.z));
}

__device__ __forceinline__ double plane_dist(const double* pl, V3<double> x) {
#pragma clang fp contract(off)
  return ((pl[0] * x.x + pl[1] * x.y) + pl[2] * x.z) - pl[3];
}

__device__ __forceinline__ void raise_err(StepStatus* st, int bit) { atomicOr(&st->err, bit); }

// x of iteration k, either materialised in x[k & 1] or, inside the launch
// that applies the update, lazily as x_{k-1} + alpha p_k.
// Same with one step size per object (the split step): x_{k-1} + alpha_o p_k.
template <typename R>
struct PosReaderSplit {
  const double4* xsrc;
  const R4<R>* p;
  const ObjScal* os;     // the previous iteration's per-object scalars
  const int* vobj;
  int lazy;
  __device__ __forceinline__ V3<double> operator()(int v) const {
    V3<double> x = ld3(xsrc, v);
    if (lazy) {
      const double alpha = os[vobj[v]].alpha;
      R4<R> q = p[v];
      x = mk3(fma(alpha, double(q.x), x.x), fma(alpha, double(q.y), x.y), fma(alpha, double(q.z), x.z));
    }
    return x;
  }
};

template <typename R>
struct PosReader {
  const double4* xsrc;   // x_{k-1} (lazy) or x_k (direct)
  const R4<R>* p;        // p_k (lazy only)
  double alpha;
  int lazy;
  __device__ __forceinline__ V3<double> operator()(int v) const {
    V3<double> x = ld3(xsrc, v);
    if (lazy) {
      R4<R> q = p[v];
      x = mk3(fma(alpha, double(q.x), x.x), fma(alpha, double(q.y), x.y), fma(alpha, double(q.z), x.z));
    }
    return x;
  }
};


// Wave-segmented suffix sum: lanes of one vertex are contiguous inside a
// wave; afterwards the vertex's first lane holds the segment total.
template <typename R>
__device__ __forceinline__ void seg_sum(int myv, R (&s)[6]) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int off = 1; off < kWave; off <<= 1) {
    int ov = __shfl_down(myv, off, kWave);
    R o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = __shfl_down(s[i], off, kWave);
    if (lane + off < kWave && ov == myv) {
#pragma unroll
      for (int i = 0; i < 6; ++i) s[i] += o[i];
    }
  }
}

// ------------------------------------------------- segmented pair gather
// Sum of the first N values of the (pair, corner) slots of the active pairs
// that touch this lane's vertex, in the fixed order of the vertex's corner
// entries.  Called by every lane of a wave of the vertex-centric incidence
// (vertices in increasing order, none straddling a wave, padding at the end);
// `vlane` marks the lane that owns its vertex's total.  The wave's vertices
// own one contiguous entry range, which the wave reads 64 entries at a time
// (one per lane) into its LDS block `lds` ([N][64] doubles); each owning lane
// then adds its own entries in order.
template <int N>
__device__ __forceinline__ void pair_gather(const int* coff, const int* cent, const uint8_t* cact,
                                            const double* cslot, int myv, bool vlane, double (&out)[N],
                                            double* lds) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = 0.0;
  const unsigned long long valid = __ballot(myv >= 0);
  if (!valid) return;
  const int last = 63 - __clzll(valid);
  const int vfirst = __shfl(myv, 0, kWave), vlast = __shfl(myv, last, kWave);
  const int j0 = coff[vfirst], j1 = coff[vlast + 1];
  if (j0 >= j1) return;
  int my0 = 0, my1 = 0;
  if (vlane) {
    my0 = coff[myv];
    my1 = coff[myv + 1];
  }
  for (int base = j0; base < j1; base += kWave) {
    const int j = base + lane;
    double e[N];
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = 0.0;
    if (j < j1) {
      const int s = cent[j];
      if (cact[s >> 2]) {
        const double* sl = cslot + 6 * (size_t)s;
#pragma unroll
        for (int i = 0; i < N; ++i) e[i] = sl[i];
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) lds[i * kWave + lane] = e[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (vlane) {
      const int t0 = max(my0, base) - base, t1 = min(my1, base + kWave) - base;
      for (int t = t0; t < t1; ++t) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] += lds[i * kWave + t];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Slot values of one active pair corner (segmented scatter) or atomic adds
// into the vertex's accumulator (atomic scatter): N values.
template <int N>
__device__ __forceinline__ void pair_corner_out(int seg, double* cslot, double* acc, long long slot, int v,
                                                const double (&val)[N]) {
  if (seg) {
    double* sl = cslot + 6 * (size_t)slot;
#pragma unroll
    for (int i = 0; i < N; ++i) sl[i] = val[i];
  } else {
    double* a = acc + 8 * (size_t)v;
#pragma unroll
    for (int i = 0; i < N; ++i) atomicAdd(a + i, val[i]);
  }
}

}  // namespace pncg
