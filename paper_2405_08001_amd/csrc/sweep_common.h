// Helpers shared by the per-iteration kernels and the batched step kernel:
// wave / block reductions, wave-segmented sums, padded-vector loads and
// stores, the direction update, plane distances and lazy position reads.
#pragma once
#include <climits>

#include "internal.h"

namespace pncg {

constexpr int kSWaves = kSBlock / kWave;

// ------------------------------------------------------------- reductions
// Lane moves by DPP (data-parallel primitives: the VALU reads another
// lane's register).  CTRL: 0x111 + s - 1 shifts right by s within each row
// of 16 lanes; 0x142 / 0x143 broadcast lane 15 / 31 into the next row(s).
// Lanes that ROW_MASK leaves out, or whose source lies outside the row,
// receive `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double old, double v) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum and maximum over the 64 lanes of a full wave, in a fixed order (a
// prefix scan within each row of 16, then the row totals carried upward);
// every lane receives the result.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111, 0xf>(0.0, v);
  v += dpp_move<0x112, 0xf>(0.0, v);
  v += dpp_move<0x114, 0xf>(0.0, v);
  v += dpp_move<0x118, 0xf>(0.0, v);
  v += dpp_move<0x142, 0xa>(0.0, v);
  v += dpp_move<0x143, 0xc>(0.0, v);
  return from_lane63(v);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<0x111, 0xf>(v, v));
  v = fmax(v, dpp_move<0x112, 0xf>(v, v));
  v = fmax(v, dpp_move<0x114, 0xf>(v, v));
  v = fmax(v, dpp_move<0x118, 0xf>(v, v));
  v = fmax(v, dpp_move<0x142, 0xa>(v, v));
  v = fmax(v, dpp_move<0x143, 0xc>(v, v));
  return from_lane63(v);
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

// Re-reduce the per-block partials [n][stride] of the previous launch.  The
// first kSBlock threads take partials j, j + kSBlock, ... whatever the
// block size, so launches of any block size reach the same bits.
template <int N, int BS = kSBlock>
__device__ __forceinline__ void reduce_partials(const double* part, int stride, int n, const int (&kind)[N],
                                                double (&out)[N], double* sh) {
  static_assert(BS >= kSBlock, "reduce_partials needs at least kSBlock threads");
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = 0.0;
  // Two partials per step, both loaded before either is added, so that the
  // usual grid (at most 2 kSBlock partials) costs one round trip; the
  // additions keep the order j, j + kSBlock, j + 2 kSBlock, ...
  for (int j = threadIdx.x; threadIdx.x < kSBlock && j < n; j += 2 * kSBlock) {
    const bool two = j + kSBlock < n;
    double a[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = part[j * stride + i];
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = two ? part[(j + kSBlock) * stride + i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = kind[i] ? fmax(out[i], a[i]) : out[i] + a[i];
    if (two) {
#pragma unroll
      for (int i = 0; i < N; ++i) out[i] = kind[i] ? fmax(out[i], b[i]) : out[i] + b[i];
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


// One step of the segmented sum: every lane adds the value that the DPP
// move brings from its source lane if that lane holds the same key (lanes
// without a source get a key no lane holds).
template <int CTRL, int ROW_MASK, typename T, int N>
__device__ __forceinline__ void seg_step(int key, T (&s)[N]) {
  const int ok = __builtin_amdgcn_update_dpp(INT_MIN, key, CTRL, ROW_MASK, 0xf, false);
  T o[N];
#pragma unroll
  for (int i = 0; i < N; ++i) o[i] = dpp_move<CTRL, ROW_MASK>(T(0), s[i]);
  if (ok == key) {
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] += o[i];
  }
}
// Wave-segmented sums over runs of equal `key` (each run contiguous within
// the wave; call with the whole wave active): an inclusive scan within each
// row of 16 lanes (shifts by 1, 2, 4, 8), then each row in turn adds the
// last lane of the row below it where the run continues.  Afterwards the
// last lane of every run holds the run's total, in a fixed order of
// additions; returns true on that lane.
template <typename T, int N>
__device__ __forceinline__ bool seg_sum(int key, T (&s)[N]) {
  seg_step<0x111, 0xf>(key, s);
  seg_step<0x112, 0xf>(key, s);
  seg_step<0x114, 0xf>(key, s);
  seg_step<0x118, 0xf>(key, s);
  seg_step<0x142, 0x2>(key, s);
  seg_step<0x142, 0x4>(key, s);
  seg_step<0x142, 0x8>(key, s);
  // the next lane's key (wave_shl:1); lane 63 has none
  const int next = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x130, 0xf, 0xf, false);
  return next != key;
}

// The same sums by shuffles (ds_bpermute, through the LDS crossbar) in a
// doubling pattern; afterwards the run's FIRST lane holds the total, and the
// function returns true on it.  Used by the batched step kernel: with 16
// waves per compute unit it is limited by vector ALU issue, and the
// shuffles move that work onto the LDS pipe (23.8k against 21.0k
// scene-steps/s on the 256-scene batch).
template <typename T, int N>
__device__ __forceinline__ bool seg_sum_shfl(int key, T (&s)[N]) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int off = 1; off < kWave; off <<= 1) {
    const int ok = __shfl_down(key, off, kWave);
    T o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = __shfl_down(s[i], off, kWave);
    if (lane + off < kWave && ok == key) {
#pragma unroll
      for (int i = 0; i < N; ++i) s[i] += o[i];
    }
  }
  const int up = __shfl_up(key, 1, kWave);
  return lane == 0 || up != key;
}

// Entry range of incidence wave w (wave-uniform) by a scalar load, so that
// waiting for it does not wait for the wave's outstanding vector memory
// operations.  The range is written by an earlier launch.
__device__ __forceinline__ int2 wave_range(const int2* wrange, int w) {
  typedef const __attribute__((address_space(4))) int* ConstIntPtr;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const ConstIntPtr p = (ConstIntPtr)(const void*)(wrange + wu);
  return make_int2(p[0], p[1]);
}

// ------------------------------------------------- segmented pair sums
// The corner entries of the candidate pairs are grouped by vertex (each
// vertex's entries in pair-key order) and evaluated 64 to a wave; a
// wave-segmented sum leaves, at the last entry of every run of one vertex
// inside a 64-entry chunk, the run's total (the run partial).  A vertex with
// entries [c0, c1) adds the partials of the chunks it touches, in chunk
// order: rp at min(c1, 64 (k + 1)) - 1 for k = c0 / 64 ... (c1 - 1) / 64.
template <int N>
__device__ __forceinline__ void pair_partials_sum(const int* coff, const double* rp, int v, double (&out)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = 0.0;
  const int c0 = coff[v], c1 = coff[v + 1];
  if (c0 >= c1) return;
  for (int k = c0 >> 6; k * kWave < c1; ++k) {
    const double* p = rp + 6 * (size_t)(min(c1, (k + 1) * kWave) - 1);
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] += p[i];
  }
}

}  // namespace pncg
