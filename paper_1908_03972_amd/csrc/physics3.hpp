// Device-side gas physics in three dimensions: primitive variables q_p = (p, u, v, w, T)
// (Sec. 2.2), the Weiss-Smith preconditioner of eq. (9) with the extra momentum row, and the
// common inviscid flux of eq. (21). Templates on the scalar type (double, or Dual<N> for the
// element Jacobian), as the two-dimensional routines.
#pragma once

#include "physics.hpp"

namespace pmg {

template <class T>
struct State3 {
  T p, u, v, w, t;
  T rho, rho_p, rho_t, inv_rho, q2, h, c2, inv_c2;
  T ur2, theta;
};

template <class T>
__device__ __forceinline__ State3<T> make_state3(const T q[5], const GasParams& g) {
  State3<T> s;
  s.p = q[0];
  s.u = q[1];
  s.v = q[2];
  s.w = q[3];
  s.t = q[4];
  s.rho_p = 1.0 / (g.rgas * s.t);
  s.rho = s.p * s.rho_p;
  s.inv_rho = 1.0 / s.rho;
  const T inv_t = g.rgas * s.rho_p;
  s.rho_t = -s.rho * inv_t;
  s.q2 = s.u * s.u + s.v * s.v + s.w * s.w;
  s.h = g.cp * s.t + 0.5 * s.q2;
  s.c2 = g.gamma * g.rgas * s.t;
  s.inv_c2 = s.rho_p * (1.0 / g.gamma);
  const T eps2 = epsilon2_from(s.q2 * s.inv_c2, g);
  s.ur2 = eps2 * s.c2;
  s.theta = 1.0 / s.ur2 + inv_t * (1.0 / g.cp);
  return s;
}

// conservative variables (rho, rho u, rho v, rho w, rho E)
template <class T>
__device__ __forceinline__ void conservative3(const T q[5], const GasParams& g, T out[5]) {
  T rho = q[0] / (g.rgas * q[4]);
  out[0] = rho;
  out[1] = rho * q[1];
  out[2] = rho * q[2];
  out[3] = rho * q[3];
  out[4] = q[0] * (1.0 / (g.gamma - 1.0)) + 0.5 * rho * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

// inviscid flux along a (not necessarily unit) vector s, density given
template <class T>
__device__ __forceinline__ void normal_flux3_rho(const T q[5], const T& rho, double sx, double sy, double sz,
                                                 const GasParams& g, T out[5]) {
  T un = q[1] * sx + q[2] * sy + q[3] * sz;
  T mflux = rho * un;
  T h = g.cp * q[4] + 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  out[0] = mflux;
  out[1] = mflux * q[1] + q[0] * sx;
  out[2] = mflux * q[2] + q[0] * sy;
  out[3] = mflux * q[3] + q[0] * sz;
  out[4] = mflux * h;
}

template <class T>
__device__ __forceinline__ void normal_flux3(const T q[5], double sx, double sy, double sz, const GasParams& g,
                                             T out[5]) {
  T rho = q[0] / (g.rgas * q[4]);
  normal_flux3_rho(q, rho, sx, sy, sz, g, out);
}

// y = Gamma x, eq. (9) in 3-D
template <class T, class X>
__device__ __forceinline__ void gamma_mul3(const State3<T>& s, const GasParams& g, const X x[5], T y[5]) {
  T y0 = s.theta * x[0] + s.rho_t * x[4];
  y[0] = y0;
  y[1] = s.u * y0 + s.rho * x[1];
  y[2] = s.v * y0 + s.rho * x[2];
  y[3] = s.w * y0 + s.rho * x[3];
  y[4] = s.h * y0 - x[0] + s.rho * (s.u * x[1] + s.v * x[2] + s.w * x[3]) + s.rho * g.cp * x[4];
}

// x = Gamma^{-1} y: the momentum rows give the velocity components; the remaining 2x2 system for
// (p, T) has determinant rho C_p / U_r^2
template <class T>
__device__ __forceinline__ void gamma_solve3(const State3<T>& s, const GasParams& g, const T y[5], T x[5]) {
  T z = y[4] - (s.h - s.q2) * y[0] - s.u * y[1] - s.v * y[2] - s.w * y[3];
  T rcp = s.rho * g.cp;
  T b = s.ur2 * (y[0] + s.theta * z) * (s.inv_rho * (1.0 / g.cp));
  x[0] = rcp * b - z;
  x[1] = (y[1] - s.u * y[0]) * s.inv_rho;
  x[2] = (y[2] - s.v * y[0]) * s.inv_rho;
  x[3] = (y[3] - s.w * y[0]) * s.inv_rho;
  x[4] = b;
}

// y = A_n x with A_n = d(f.n)/dq_p for a unit normal n
template <class T>
__device__ __forceinline__ void flux_jac_mul3(const State3<T>& s, const GasParams& g, double nx, double ny,
                                              double nz, const T& un, const T x[5], T y[5]) {
  T m = s.rho_p * x[0] + s.rho_t * x[4];
  T dun = nx * x[1] + ny * x[2] + nz * x[3];
  T r0 = un * m + s.rho * dun;
  T rhoun = s.rho * un;
  y[0] = r0;
  y[1] = s.u * r0 + rhoun * x[1] + nx * x[0];
  y[2] = s.v * r0 + rhoun * x[2] + ny * x[0];
  y[3] = s.w * r0 + rhoun * x[3] + nz * x[0];
  y[4] = s.h * r0 + rhoun * (s.u * x[1] + s.v * x[2] + s.w * x[3]) + rhoun * g.cp * x[4];
}

// Common inviscid flux of eq. (21) times |S|, as common_flux2: mean primitive state, the matrix
// function |Gamma^{-1} A_n| applied as the quadratic interpolating |lambda| at the three distinct
// eigenvalues of eq. (13) (u_n has multiplicity 3 in three dimensions).
template <class T>
__device__ __forceinline__ void common_flux3(const T qm[5], const T qp[5], const T dq[5], double nx, double ny,
                                             double nz, double smag, const GasParams& g, T out[5]) {
  T qa[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) qa[k] = 0.5 * (qm[k] + qp[k]);
  const State3<T> s = make_state3(qa, g);
  T un = s.u * nx + s.v * ny + s.w * nz;
  T alpha = 0.5 * (1.0 - s.ur2 * s.inv_c2);
  T cpr = dsqrt(alpha * alpha * un * un + s.ur2);
  T l1 = un;
  T l2 = un * (1.0 - alpha) + cpr;
  T l3 = un * (1.0 - alpha) - cpr;
  T a1 = rabs(l1), a2 = rabs(l2), a3 = rabs(l3);
  T d21 = l2 - l1, d31 = l3 - l1, d32 = l3 - l2;
  T inv = 1.0 / (d21 * d31 * d32);
  T f12 = (a2 - a1) * (d31 * d32) * inv;
  T f123 = ((a3 - a1) * d21 - (a2 - a1) * d31) * inv;

  T gd[5], ad[5], w[5], y[5], ay[5];
  gamma_mul3(s, g, dq, gd);
  flux_jac_mul3(s, g, nx, ny, nz, un, dq, ad);
#pragma unroll
  for (int k = 0; k < 5; ++k) w[k] = ad[k] - l2 * gd[k];
  gamma_solve3(s, g, w, y);
  flux_jac_mul3(s, g, nx, ny, nz, un, y, ay);

  T fm[5], fp[5];
  normal_flux3(qm, nx, ny, nz, g, fm);
  normal_flux3(qp, nx, ny, nz, g, fp);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    T diss = a1 * gd[k] + f12 * (ad[k] - l1 * gd[k]) + f123 * (ay[k] - l1 * w[k]);
    out[k] = smag * (0.5 * (fm[k] + fp[k]) - 0.5 * diss);
  }
}

}  // namespace pmg
