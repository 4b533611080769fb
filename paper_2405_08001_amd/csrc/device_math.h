// Device arithmetic of the PNCG hot path for gfx950: 3-vectors, the IPC
// barrier, point-triangle / edge-edge closest points, and the per-tet
// elastic terms (Neo-Hookean, stable Neo-Hookean, corotated) in compact
// closed forms.
//
// Real is the element/vector type (float in the mixed form, double in the
// plain form).  Distances, barrier terms and positions are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>
#include <limits>

namespace pncg {

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__host__ __device__ __forceinline__ V3<T> mk3(T a, T b, T c) { return V3<T>{a, b, c}; }
template <typename T>
__host__ __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__host__ __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__host__ __device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__host__ __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__host__ __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T, typename U>
__host__ __device__ __forceinline__ V3<T> cast3(V3<U> a) { return {T(a.x), T(a.y), T(a.z)}; }

// ---------------------------------------------------------------- barrier
// b(d) = -(d - dhat)^2 log(d / dhat) on (0, dhat), 0 beyond (Sec. 3,
// equation barrier); derivatives by differentiating that expression.
__device__ __forceinline__ double barrier_b(double d, double dhat) {
  if (d >= dhat) return 0.0;
  double e = d - dhat;
  return -e * e * log(d / dhat);
}
__device__ __forceinline__ double barrier_db(double d, double dhat) {
  if (d >= dhat) return 0.0;
  double e = d - dhat;
  return -2.0 * e * log(d / dhat) - e * e / d;
}
__device__ __forceinline__ double barrier_d2b(double d, double dhat) {
  if (d >= dhat) return 0.0;
  double e = d - dhat;
  double q = e / d;
  return -2.0 * log(d / dhat) - 4.0 * q + q * q;
}

// ------------------------------------------------------- closest points
// Result of a pair: t = sum_i c_i x_i, d = |t| (Sec. 3.2).
struct Closest {
  double c[4];
  V3<double> t;
  double d;
};

// Point x0 against triangle (x1, x2, x3): barycentric region tests on the
// dot products of the edge vectors with the point offsets (the Voronoi
// region method of Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5).
__device__ __forceinline__ Closest closest_pt(V3<double> x0, V3<double> x1, V3<double> x2, V3<double> x3) {
  V3<double> ab = x2 - x1, ac = x3 - x1, ap = x0 - x1;
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  double v, w;  // weights of x2 and x3; x1 gets 1 - v - w
  if (d1 <= 0.0 && d2 <= 0.0) {
    v = 0.0; w = 0.0;
  } else {
    V3<double> bp = x0 - x2;
    double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) {
      v = 1.0; w = 0.0;
    } else {
      double vc = d1 * d4 - d3 * d2;
      if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        v = d1 / (d1 - d3); w = 0.0;
      } else {
        V3<double> cp = x0 - x3;
        double d5 = dot(ab, cp), d6 = dot(ac, cp);
        if (d6 >= 0.0 && d5 <= d6) {
          v = 0.0; w = 1.0;
        } else {
          double vb = d5 * d2 - d1 * d6;
          if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
            v = 0.0; w = d2 / (d2 - d6);
          } else {
            double va = d3 * d6 - d5 * d4;
            if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
              w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
              v = 1.0 - w;
            } else {
              double den = 1.0 / (va + vb + vc);
              v = vb * den;
              w = vc * den;
            }
          }
        }
      }
    }
  }
  Closest r;
  r.c[0] = 1.0;
  r.c[1] = -(1.0 - v - w);
  r.c[2] = -v;
  r.c[3] = -w;
  r.t = ap - v * ab;
  r.t = r.t - w * ac;
  r.d = sqrt(dot(r.t, r.t));
  return r;
}

// Edges x0-x1 and x2-x3 with the clamped segment-segment solve (Ericson
// 2005, Sec. 5.1.9): s on the first edge from the unconstrained lines,
// clamped; u from s; if u leaves [0,1] it is clamped and s recomputed.
// Parallel edges ((d1.d1)(d2.d2) - (d1.d2)^2 <= 1e-12 (d1.d1)(d2.d2)) start
// from s = 0.
__device__ __forceinline__ Closest closest_ee(V3<double> x0, V3<double> x1, V3<double> x2, V3<double> x3) {
  V3<double> d1 = x1 - x0, d2 = x3 - x2, r = x0 - x2;
  double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  double c = dot(d1, r), b = dot(d1, d2);
  double den = a * e - b * b;
  double s = 0.0, u;
  if (den > 1e-12 * a * e) s = fmin(fmax((b * f - c * e) / den, 0.0), 1.0);
  u = (b * s + f) / e;
  if (u < 0.0) {
    u = 0.0;
    s = fmin(fmax(-c / a, 0.0), 1.0);
  } else if (u > 1.0) {
    u = 1.0;
    s = fmin(fmax((b - c) / a, 0.0), 1.0);
  }
  Closest out;
  out.c[0] = 1.0 - s;
  out.c[1] = s;
  out.c[2] = -(1.0 - u);
  out.c[3] = -u;
  out.t = r + s * d1;
  out.t = out.t - u * d2;
  out.d = sqrt(dot(out.t, out.t));
  return out;
}

// ------------------------------------------------------------ Neo-Hookean
// Per-tet record: vertex indices, the rows of D_m^{-1} and V_e mu_e,
// V_e lam_e (rest volume times Lame parameters).
template <typename R>
struct ElemRec {
  int v[4];
  R B[9];      // B[3*r + j]: row r of D_m^{-1}; shape vector b_{r+1} = row r
  R vmu, vlam;
};

// Columns f_j of F = sum_{a=1..3} (x_a - x_0) b_a^T, formed from float64
// position differences cast to R.
template <typename R>
struct Kin {
  V3<R> f[3];   // columns of F
  V3<R> c[3];   // columns of cof F: f1 x f2, f2 x f0, f0 x f1
  R J, lnJ;
};

template <typename R>
__device__ __forceinline__ Kin<R> kinematics(const R* B, V3<double> x0, V3<double> x1, V3<double> x2, V3<double> x3) {
  V3<R> e1 = cast3<R>(x1 - x0), e2 = cast3<R>(x2 - x0), e3 = cast3<R>(x3 - x0);
  Kin<R> k;
#pragma unroll
  for (int j = 0; j < 3; ++j) k.f[j] = B[j] * e1 + B[3 + j] * e2 + B[6 + j] * e3;
  k.c[0] = cross(k.f[1], k.f[2]);
  k.c[1] = cross(k.f[2], k.f[0]);
  k.c[2] = cross(k.f[0], k.f[1]);
  k.J = dot(k.f[0], k.c[0]);
  k.lnJ = k.J > R(0) ? log(k.J) : R(0);
  return k;
}

// shape vector b_a (a = 0..3) from the three stored rows; selected without
// indexing the register array by a runtime value
template <typename R>
__device__ __forceinline__ V3<R> shape_vec(const R* B, int a) {
  const V3<R> b1 = mk3(B[0], B[1], B[2]), b2 = mk3(B[3], B[4], B[5]), b3 = mk3(B[6], B[7], B[8]);
  const V3<R> b0 = mk3(-(B[0] + B[3] + B[6]), -(B[1] + B[4] + B[7]), -(B[2] + B[5] + B[8]));
  const V3<R> lo = a == 0 ? b0 : b1;
  const V3<R> hi = a == 2 ? b2 : b3;
  return a < 2 ? lo : hi;
}

// Psi_3 and Psi_33 of the Neo-Hookean density times V_e:
//   V Psi_3  = (V lam log J - V mu) / J
//   V Psi_33 = (V mu + V lam (1 - log J)) / J^2
template <typename R>
__device__ __forceinline__ void nh_coeffs(const Kin<R>& k, R vmu, R vlam, R& vpsi3, R& vpsi33) {
  R iJ = R(1) / k.J;
  vpsi3 = (vlam * k.lnJ - vmu) * iJ;
  vpsi33 = (vmu + vlam * (R(1) - k.lnJ)) * iJ * iJ;
}

// The I2 and I3 parts of a density with constant Psi_2 and a function of
// I3 alone, given a2 = 2 V Psi_2, V Psi_3 and V Psi_33.
// Gradient block g_a = V P(F) b_a with P = 2 Psi_2 F + Psi_3 cof F, and the
// diagonal block diag_a = V [2 Psi_2 |b_a|^2 + Psi_33 (cof F b_a)^2] (the H3
// term contributes nothing to the diagonal since hat(f) has a zero
// diagonal).  All without the h^2 factor.
template <typename R>
__device__ __forceinline__ void i23_grad_diag(const Kin<R>& k, R a2, R vpsi3, R vpsi33, V3<R> ba, V3<R>& g,
                                              V3<R>& dg) {
  V3<R> Fb = ba.x * k.f[0] + ba.y * k.f[1] + ba.z * k.f[2];
  V3<R> Cb = ba.x * k.c[0] + ba.y * k.c[1] + ba.z * k.c[2];
  g = a2 * Fb + vpsi3 * Cb;
  R bb = a2 * dot(ba, ba);
  dg = mk3(bb + vpsi33 * Cb.x * Cb.x, bb + vpsi33 * Cb.y * Cb.y, bb + vpsi33 * Cb.z * Cb.z);
}

// dF columns for per-vertex directions p_a: d_j = sum_{a=1..3} (p_a - p_0) B[a-1][j]
template <typename R>
__device__ __forceinline__ void dF_cols(const R* B, V3<R> p0, V3<R> p1, V3<R> p2, V3<R> p3, V3<R> d[3]) {
  V3<R> q1 = p1 - p0, q2 = p2 - p0, q3 = p3 - p0;
#pragma unroll
  for (int j = 0; j < 3; ++j) d[j] = B[j] * q1 + B[3 + j] * q2 + B[6 + j] * q3;
}

// p^T (d2 Psi/dx2) p / (without h^2), I2 and I3 parts:
//   V [2 Psi_2 |dF|^2 + Psi_33 (cof F : dF)^2
//      + 2 Psi_3 (f0.(d1 x d2) + f1.(d2 x d0) + f2.(d0 x d1))]
template <typename R>
__device__ __forceinline__ R i23_pHp(const Kin<R>& k, R a2, R vpsi3, R vpsi33, const V3<R> d[3]) {
  R dd = dot(d[0], d[0]) + dot(d[1], d[1]) + dot(d[2], d[2]);
  R cd = dot(k.c[0], d[0]) + dot(k.c[1], d[1]) + dot(k.c[2], d[2]);
  R mix = dot(k.f[0], cross(d[1], d[2])) + dot(k.f[1], cross(d[2], d[0])) + dot(k.f[2], cross(d[0], d[1]));
  return a2 * dd + vpsi33 * cd * cd + R(2) * vpsi3 * mix;
}

// (H p)_a / h^2, I2 and I3 parts: V dP b_a with
//   dP = 2 Psi_2 dF + Psi_33 (cof F : dF) cof F + Psi_3 dcof,
//   dcof = [d1 x f2 + f1 x d2, d2 x f0 + f2 x d0, d0 x f1 + f0 x d1]
template <typename R>
__device__ __forceinline__ V3<R> i23_Hp(const Kin<R>& k, R a2, R vpsi3, R vpsi33, const V3<R> d[3], V3<R> ba) {
  R cd = dot(k.c[0], d[0]) + dot(k.c[1], d[1]) + dot(k.c[2], d[2]);
  V3<R> dc0 = cross(d[1], k.f[2]) + cross(k.f[1], d[2]);
  V3<R> dc1 = cross(d[2], k.f[0]) + cross(k.f[2], d[0]);
  V3<R> dc2 = cross(d[0], k.f[1]) + cross(k.f[0], d[1]);
  V3<R> db = ba.x * d[0] + ba.y * d[1] + ba.z * d[2];
  V3<R> cb = ba.x * k.c[0] + ba.y * k.c[1] + ba.z * k.c[2];
  V3<R> dcb = ba.x * dc0 + ba.y * dc1 + ba.z * dc2;
  return a2 * db + (vpsi33 * cd) * cb + vpsi3 * dcb;
}

// Neo-Hookean (Sec. 3.1): 2 Psi_2 = mu.
template <typename R>
__device__ __forceinline__ void nh_grad_diag(const Kin<R>& k, R vmu, R vlam, V3<R> ba, V3<R>& g, V3<R>& dg) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  i23_grad_diag(k, vmu, vpsi3, vpsi33, ba, g, dg);
}
template <typename R>
__device__ __forceinline__ R nh_pHp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3]) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  return i23_pHp(k, vmu, vpsi3, vpsi33, d);
}
template <typename R>
__device__ __forceinline__ V3<R> nh_Hp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3], V3<R> ba) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  return i23_Hp(k, vmu, vpsi3, vpsi33, d, ba);
}

// V Psi(F) = V mu/2 (I2 - 3) - V mu log J + V lam/2 (log J)^2
template <typename R>
__device__ __forceinline__ R nh_energy(const Kin<R>& k, R vmu, R vlam) {
  R I2 = dot(k.f[0], k.f[0]) + dot(k.f[1], k.f[1]) + dot(k.f[2], k.f[2]);
  return R(0.5) * vmu * (I2 - R(3)) - vmu * k.lnJ + R(0.5) * vlam * k.lnJ * k.lnJ;
}

// d(g_a)/dE for mu = E mu', lam = E lam' (gradient is linear in mu, lam):
// V (mu' (F - F^{-T}) + lam' log J F^{-T}) b_a, with F^{-T} = cof F / J.
template <typename R>
__device__ __forceinline__ V3<R> nh_dgdE(const Kin<R>& k, R vol_mup, R vol_lamp, V3<R> ba) {
  R iJ = R(1) / k.J;
  V3<R> Fb = ba.x * k.f[0] + ba.y * k.f[1] + ba.z * k.f[2];
  V3<R> Cb = ba.x * k.c[0] + ba.y * k.c[1] + ba.z * k.c[2];
  return vol_mup * Fb + ((vol_lamp * k.lnJ - vol_mup) * iJ) * Cb;
}


// ------------------------------------------------------------- materials
// Densities by template argument (Sec. 3.1 invariants; the materials of
// Table 1), each Psi = Psi_1 I1 + Psi_2 I2 + f(I3) with constant Psi_1, Psi_2:
//   kModelNH     Neo-Hookean: Psi_2 = mu/2, f = -mu log J + lam/2 log^2 J
//   kModelSNH    stable Neo-Hookean: Psi_2 = mu/2,
//                f = -mu (J - 1) + lam'/2 (J - 1)^2; the element record's
//                vlam holds V lam' with lam' = lam + mu
//   kModelCorot  fixed corotated: Psi_1 = -2 mu, Psi_2 = mu,
//                f = lam/2 (J - 1)^2; as-rigid-as-possible is the same with
//                lam = 0 in the element record
enum Model { kModelNH = 0, kModelSNH = 1, kModelCorot = 2 };

// Rotation-variant polar decomposition F = R S, R = U V^T with U and V
// proper rotations, from the eigen-decomposition of C = F^T F by cyclic
// Jacobi rotations: v_i are C's eigenvectors by decreasing eigenvalue,
// v_2 = v_0 x v_1; u_0 = F v_0 / |F v_0|, u_1 the unit part of F v_1
// orthogonal to u_0, u_2 = u_0 x u_1; s_i = u_i . F v_i, so s_2 carries the
// sign of det F and I1 = s_0 + s_1 + s_2.  With A = U^T dF V and
// w = axial(A - A^T) = (A_21 - A_12, A_02 - A_20, A_10 - A_01), the I1
// Hessian's quadratic form is dF : H1 : dF = sum_i w_i^2 / kappa_i and its
// product dR = H1 dF = U [omega]x V^T with omega_i = w_i / kappa_i, where
// kappa_0 = s_1 + s_2, kappa_1 = s_0 + s_2, kappa_2 = s_0 + s_1 (the twist
// eigenvalues 2 / kappa_i of Kim and Eberle's course, written without the
// SVD's sign bookkeeping).
template <typename R>
struct Polar {
  V3<R> u[3], v[3];   // columns of U and V
  R s[3];
  R ik[3];            // 1 / kappa_i
};

// Reciprocal, square root and reciprocal square root inside the polar
// decomposition: the hardware's approximate (1 ulp) instructions in float,
// whose result is accurate to float rounding either way; IEEE operations in
// double.
__device__ __forceinline__ float pol_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double pol_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float pol_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double pol_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float pol_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double pol_rsq(double x) { return 1.0 / sqrt(x); }

template <typename R>
__device__ __forceinline__ void jacobi_rot(R& app, R& aqq, R& apq, R& arp, R& arq, V3<R>& vp, V3<R>& vq) {
  // skip zero and subnormal off-diagonals: the float reciprocal flushes a
  // subnormal input to zero, and (aqq - app) * inf is NaN when aqq == app
  if (!(std::fabs(apq) >= std::numeric_limits<R>::min())) return;
  const R th = (aqq - app) * pol_rcp(R(2) * apq);
  // |th| large: th^2 overflows, the reciprocal gives t = 0 (no rotation)
  const R t = std::copysign(pol_rcp(std::fabs(th) + pol_sqrt(std::fma(th, th, R(1)))), th);
  const R c = pol_rsq(std::fma(t, t, R(1)));
  const R sn = t * c;
  app -= t * apq;
  aqq += t * apq;
  apq = R(0);
  const R rp = arp, rq = arq;
  arp = c * rp - sn * rq;
  arq = sn * rp + c * rq;
  const V3<R> p = vp, q = vq;
  vp = mk3(c * p.x - sn * q.x, c * p.y - sn * q.y, c * p.z - sn * q.z);
  vq = mk3(sn * p.x + c * q.x, sn * p.y + c * q.y, sn * p.z + c * q.z);
}

// Jacobi sweeps: enough for rounding-level off-diagonals from any start.
template <typename R>
struct PolarSweeps {
  static constexpr int value = 4;
};
template <>
struct PolarSweeps<double> {
  static constexpr int value = 5;
};

// False where a kappa_i is not positive (the I1 Hessian is undefined there)
// or the decomposition is not finite (F of rank < 2).
template <typename R>
__device__ __forceinline__ bool polar_rv(const V3<R> f[3], Polar<R>& P) {
  R a00 = dot(f[0], f[0]), a11 = dot(f[1], f[1]), a22 = dot(f[2], f[2]);
  R a01 = dot(f[0], f[1]), a02 = dot(f[0], f[2]), a12 = dot(f[1], f[2]);
  V3<R> v0 = mk3(R(1), R(0), R(0)), v1 = mk3(R(0), R(1), R(0)), v2 = mk3(R(0), R(0), R(1));
  for (int it = 0; it < PolarSweeps<R>::value; ++it) {
    jacobi_rot(a00, a11, a01, a02, a12, v0, v1);
    jacobi_rot(a00, a22, a02, a01, a12, v0, v2);
    jacobi_rot(a11, a22, a12, a01, a02, v1, v2);
    // stop once the off-diagonal is at rounding level in every active lane
    // of the wave (a wave-wide vote keeps the loop uniform)
    const R off = std::fabs(a01) + std::fabs(a02) + std::fabs(a12);
    if (__all(off <= std::numeric_limits<R>::epsilon() * (a00 + a11 + a22))) break;
  }
  // order by decreasing eigenvalue
  if (a00 < a11) { R t = a00; a00 = a11; a11 = t; V3<R> w = v0; v0 = v1; v1 = w; }
  if (a00 < a22) { R t = a00; a00 = a22; a22 = t; V3<R> w = v0; v0 = v2; v2 = w; }
  if (a11 < a22) { R t = a11; a11 = a22; a22 = t; V3<R> w = v1; v1 = v2; v2 = w; }
  v2 = cross(v0, v1);
  const V3<R> Fv0 = v0.x * f[0] + v0.y * f[1] + v0.z * f[2];
  const V3<R> Fv1 = v1.x * f[0] + v1.y * f[1] + v1.z * f[2];
  const V3<R> Fv2 = v2.x * f[0] + v2.y * f[1] + v2.z * f[2];
  const V3<R> u0 = pol_rsq(dot(Fv0, Fv0)) * Fv0;
  const V3<R> w1 = Fv1 - dot(u0, Fv1) * u0;
  const V3<R> u1 = pol_rsq(dot(w1, w1)) * w1;
  const V3<R> u2 = cross(u0, u1);
  P.u[0] = u0; P.u[1] = u1; P.u[2] = u2;
  P.v[0] = v0; P.v[1] = v1; P.v[2] = v2;
  P.s[0] = dot(u0, Fv0);
  P.s[1] = dot(u1, Fv1);
  P.s[2] = dot(u2, Fv2);
  const R k0 = P.s[1] + P.s[2], k1 = P.s[0] + P.s[2], k2 = P.s[0] + P.s[1];
  P.ik[0] = pol_rcp(k0);
  P.ik[1] = pol_rcp(k1);
  P.ik[2] = pol_rcp(k2);
  return k0 > R(0) && k1 > R(0) && k2 > R(0) && P.ik[0] < R(INFINITY) && P.ik[1] < R(INFINITY) &&
         P.ik[2] < R(INFINITY);
}

// V^T b and U (omega x y)
template <typename R>
__device__ __forceinline__ V3<R> vt_mul(const Polar<R>& P, V3<R> b) { return mk3(dot(P.v[0], b), dot(P.v[1], b), dot(P.v[2], b)); }
template <typename R>
__device__ __forceinline__ V3<R> u_mul(const Polar<R>& P, V3<R> y) { return y.x * P.u[0] + y.y * P.u[1] + y.z * P.u[2]; }

// w = axial(A - A^T), A = U^T dF V, for dF with columns d_j
template <typename R>
__device__ __forceinline__ V3<R> twist_w(const Polar<R>& P, const V3<R> d[3]) {
  V3<R> dv[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) dv[j] = P.v[j].x * d[0] + P.v[j].y * d[1] + P.v[j].z * d[2];
  // A_ij = u_i . (dF v_j)
  return mk3(dot(P.u[2], dv[1]) - dot(P.u[1], dv[2]), dot(P.u[0], dv[2]) - dot(P.u[2], dv[0]),
             dot(P.u[1], dv[0]) - dot(P.u[0], dv[1]));
}

// Coefficients of the I2 and I3 parts: a2 = 2 V Psi_2, V Psi_3, V Psi_33.
template <typename R, int M>
__device__ __forceinline__ void i23_coeffs(const Kin<R>& k, R vmu, R vlam, R& a2, R& vpsi3, R& vpsi33) {
  if constexpr (M == kModelNH) {
    a2 = vmu;
    nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  } else if constexpr (M == kModelSNH) {
    a2 = vmu;
    vpsi3 = vlam * (k.J - R(1)) - vmu;
    vpsi33 = vlam;
  } else {
    a2 = R(2) * vmu;
    vpsi3 = vlam * (k.J - R(1));
    vpsi33 = vlam;
  }
}

// Whether F lies in the model's domain without the polar decomposition:
// Neo-Hookean needs det F > 0; the corotated model is checked by polar_rv.
template <typename R, int M>
__device__ __forceinline__ bool i23_ok(const Kin<R>& k) {
  if constexpr (M == kModelNH) return k.J > R(0);
  return true;
}

// Element gradient block and diagonal block (without h^2); false outside
// the model's domain.
template <typename R, int M>
__device__ __forceinline__ bool el_grad_diag(const Kin<R>& k, R vmu, R vlam, V3<R> ba, V3<R>& g, V3<R>& dg) {
  if (!i23_ok<R, M>(k)) return false;
  R a2, vpsi3, vpsi33;
  i23_coeffs<R, M>(k, vmu, vlam, a2, vpsi3, vpsi33);
  i23_grad_diag(k, a2, vpsi3, vpsi33, ba, g, dg);
  if constexpr (M == kModelCorot) {
    Polar<R> P;
    if (!polar_rv(k.f, P)) return false;
    const R a1 = R(-2) * vmu;
    const V3<R> y = vt_mul(P, ba);
    g = g + a1 * u_mul(P, y);             // Psi_1 R b_a
    // diagonal of H1 for coordinate c: w = (U^T e_c) x y
    const V3<R> r0 = mk3(P.u[0].x, P.u[1].x, P.u[2].x);
    const V3<R> r1 = mk3(P.u[0].y, P.u[1].y, P.u[2].y);
    const V3<R> r2 = mk3(P.u[0].z, P.u[1].z, P.u[2].z);
    const V3<R> z0 = cross(r0, y), z1 = cross(r1, y), z2 = cross(r2, y);
    dg.x += a1 * (z0.x * z0.x * P.ik[0] + z0.y * z0.y * P.ik[1] + z0.z * z0.z * P.ik[2]);
    dg.y += a1 * (z1.x * z1.x * P.ik[0] + z1.y * z1.y * P.ik[1] + z1.z * z1.z * P.ik[2]);
    dg.z += a1 * (z2.x * z2.x * P.ik[0] + z2.y * z2.y * P.ik[1] + z2.z * z2.z * P.ik[2]);
  }
  return true;
}

// p^T H_e p without h^2; false outside the model's domain.
template <typename R, int M>
__device__ __forceinline__ bool el_pHp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3], R& out) {
  if (!i23_ok<R, M>(k)) return false;
  R a2, vpsi3, vpsi33;
  i23_coeffs<R, M>(k, vmu, vlam, a2, vpsi3, vpsi33);
  out = i23_pHp(k, a2, vpsi3, vpsi33, d);
  if constexpr (M == kModelCorot) {
    Polar<R> P;
    if (!polar_rv(k.f, P)) return false;
    const V3<R> w = twist_w(P, d);
    out += R(-2) * vmu * (w.x * w.x * P.ik[0] + w.y * w.y * P.ik[1] + w.z * w.z * P.ik[2]);
  }
  return true;
}

// (H_e p)_a without h^2; false outside the model's domain.
template <typename R, int M>
__device__ __forceinline__ bool el_Hp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3], V3<R> ba, V3<R>& out) {
  if (!i23_ok<R, M>(k)) return false;
  R a2, vpsi3, vpsi33;
  i23_coeffs<R, M>(k, vmu, vlam, a2, vpsi3, vpsi33);
  out = i23_Hp(k, a2, vpsi3, vpsi33, d, ba);
  if constexpr (M == kModelCorot) {
    Polar<R> P;
    if (!polar_rv(k.f, P)) return false;
    const V3<R> w = twist_w(P, d);
    const V3<R> om = mk3(w.x * P.ik[0], w.y * P.ik[1], w.z * P.ik[2]);
    out = out + (R(-2) * vmu) * u_mul(P, cross(om, vt_mul(P, ba)));
  }
  return true;
}

// V Psi(F); false outside the model's domain.  The corotated |F - R|^2 is
// formed as sum_i (s_i - 1)^2.
template <typename R, int M>
__device__ __forceinline__ bool el_energy(const Kin<R>& k, R vmu, R vlam, R& out) {
  if constexpr (M == kModelNH) {
    if (!(k.J > R(0))) return false;
    out = nh_energy(k, vmu, vlam);
  } else if constexpr (M == kModelSNH) {
    const R I2 = dot(k.f[0], k.f[0]) + dot(k.f[1], k.f[1]) + dot(k.f[2], k.f[2]);
    const R e = k.J - R(1);
    out = R(0.5) * vmu * (I2 - R(3)) - vmu * e + R(0.5) * vlam * e * e;
  } else {
    Polar<R> P;
    if (!polar_rv(k.f, P)) return false;
    const R e = k.J - R(1);
    const R t0 = P.s[0] - R(1), t1 = P.s[1] - R(1), t2 = P.s[2] - R(1);
    out = vmu * (t0 * t0 + t1 * t1 + t2 * t2) + R(0.5) * vlam * e * e;
  }
  return true;
}

// d(g_a)/dE for mu = E mu', lam = E lam': every density's stress is linear
// in (mu, lam), so this is the gradient block with (V mu', V lam').
template <typename R, int M>
__device__ __forceinline__ bool el_dgdE(const Kin<R>& k, R vol_mup, R vol_lamp, V3<R> ba, V3<R>& out) {
  if constexpr (M == kModelNH) {
    if (!(k.J > R(0))) return false;
    out = nh_dgdE(k, vol_mup, vol_lamp, ba);
    return true;
  } else {
    V3<R> dg;
    return el_grad_diag<R, M>(k, vol_mup, vol_lamp, ba, out, dg);
  }
}

}  // namespace pncg
