// Device arithmetic of the PNCG hot path for gfx950: 3-vectors, the IPC
// barrier, point-triangle / edge-edge closest points, and the per-tet
// Neo-Hookean terms in their compact closed forms.
//
// Real is the element/vector type (float in the mixed form, double in the
// plain form).  Distances, barrier terms and positions are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

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

// Gradient block g_a = V P(F) b_a with P = mu F + Psi_3 cof F, and the
// diagonal block diag_a = V [mu |b_a|^2 + Psi_33 (cof F b_a)^2] (the H3 term
// contributes nothing to the diagonal since hat(f) has a zero diagonal).
// Both without the h^2 factor.
template <typename R>
__device__ __forceinline__ void nh_grad_diag(const Kin<R>& k, R vmu, R vlam, V3<R> ba, V3<R>& g, V3<R>& dg) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  V3<R> Fb = ba.x * k.f[0] + ba.y * k.f[1] + ba.z * k.f[2];
  V3<R> Cb = ba.x * k.c[0] + ba.y * k.c[1] + ba.z * k.c[2];
  g = vmu * Fb + vpsi3 * Cb;
  R bb = vmu * dot(ba, ba);
  dg = mk3(bb + vpsi33 * Cb.x * Cb.x, bb + vpsi33 * Cb.y * Cb.y, bb + vpsi33 * Cb.z * Cb.z);
}

// dF columns for per-vertex directions p_a: d_j = sum_{a=1..3} (p_a - p_0) B[a-1][j]
template <typename R>
__device__ __forceinline__ void dF_cols(const R* B, V3<R> p0, V3<R> p1, V3<R> p2, V3<R> p3, V3<R> d[3]) {
  V3<R> q1 = p1 - p0, q2 = p2 - p0, q3 = p3 - p0;
#pragma unroll
  for (int j = 0; j < 3; ++j) d[j] = B[j] * q1 + B[3 + j] * q2 + B[6 + j] * q3;
}

// p^T (d2 Psi/dx2) p / (without h^2) = V [mu |dF|^2 + Psi_33 (cof F : dF)^2
//   + 2 Psi_3 (f0.(d1 x d2) + f1.(d2 x d0) + f2.(d0 x d1))]
template <typename R>
__device__ __forceinline__ R nh_pHp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3]) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  R dd = dot(d[0], d[0]) + dot(d[1], d[1]) + dot(d[2], d[2]);
  R cd = dot(k.c[0], d[0]) + dot(k.c[1], d[1]) + dot(k.c[2], d[2]);
  R mix = dot(k.f[0], cross(d[1], d[2])) + dot(k.f[1], cross(d[2], d[0])) + dot(k.f[2], cross(d[0], d[1]));
  return vmu * dd + vpsi33 * cd * cd + R(2) * vpsi3 * mix;
}

// (H p)_a / h^2 = V dP b_a with dP = mu dF + Psi_33 (cof F : dF) cof F
//   + Psi_3 dcof, dcof = [d1 x f2 + f1 x d2, d2 x f0 + f2 x d0, d0 x f1 + f0 x d1]
template <typename R>
__device__ __forceinline__ V3<R> nh_Hp(const Kin<R>& k, R vmu, R vlam, const V3<R> d[3], V3<R> ba) {
  R vpsi3, vpsi33;
  nh_coeffs(k, vmu, vlam, vpsi3, vpsi33);
  R cd = dot(k.c[0], d[0]) + dot(k.c[1], d[1]) + dot(k.c[2], d[2]);
  V3<R> dc0 = cross(d[1], k.f[2]) + cross(k.f[1], d[2]);
  V3<R> dc1 = cross(d[2], k.f[0]) + cross(k.f[2], d[0]);
  V3<R> dc2 = cross(d[0], k.f[1]) + cross(k.f[0], d[1]);
  V3<R> db = ba.x * d[0] + ba.y * d[1] + ba.z * d[2];
  V3<R> cb = ba.x * k.c[0] + ba.y * k.c[1] + ba.z * k.c[2];
  V3<R> dcb = ba.x * dc0 + ba.y * dc1 + ba.z * dc2;
  return vmu * db + (vpsi33 * cd) * cb + vpsi3 * dcb;
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

}  // namespace pncg
