// Device-side gas physics for the preconditioned FR/CPR residual and its Jacobian.
//
// Working variables are the primitive q_p = (p, u, v, T) (Sec. 2.2). Every routine is a
// template on the scalar type so that the same code gives values (double) and exact
// forward-mode derivatives (Dual<N>) for the element Jacobian.
#pragma once

#include <hip/hip_runtime.h>

namespace pmg {

struct GasParams {
  double gamma;
  double rgas;
  double cp;        // gamma R / (gamma - 1)
  double ma_inf;
  double kappa;
  int eps_mode;     // 0: eps = min(1, Ma) (cut-off off); 1: eps = min(1, max(kappa Ma_inf, Ma)), eq. (11)
  double mu;        // dynamic viscosity (0: inviscid)
  double kcond;     // mu C_p / Pr
  double br2_eta;   // penalty of the BR2 common gradient
};

// ---- forward-mode dual numbers ------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
};

template <int N>
__device__ __forceinline__ Dual<N> dconst(double x) {
  Dual<N> r;
  r.v = x;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = 0.0;
  return r;
}

template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  const double inv = 1.0 / b.v;
  r.v = a.v * inv;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double b) {
  Dual<N> r = a;
  r.v += b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double b, const Dual<N>& a) { return a + b; }
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double b) {
  Dual<N> r = a;
  r.v -= b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(double b, const Dual<N>& a) {
  Dual<N> r;
  r.v = b - a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N>
__device__ __forceinline__ Dual<N> operator/(double b, const Dual<N>& a) {
  Dual<N> r;
  const double inv = 1.0 / a.v;
  r.v = b * inv;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -r.v * a.d[k] * inv;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a) {
  Dual<N> r;
  r.v = sqrt(a.v);
  const double h = 0.5 / r.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * h;
  return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

__device__ __forceinline__ double val(double x) { return x; }
template <int N>
__device__ __forceinline__ double val(const Dual<N>& x) { return x.v; }

// |x|, min and max continued from the branch the value selects
template <class T>
__device__ __forceinline__ T rabs(const T& x) { return val(x) < 0.0 ? -x : x; }
template <class T>
__device__ __forceinline__ T rmin(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }
template <class T>
__device__ __forceinline__ T rmax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }

template <class T>
__device__ __forceinline__ T lift(double x) { return T(x); }
template <>
__device__ __forceinline__ Dual<1> lift<Dual<1>>(double x) { return dconst<1>(x); }
template <>
__device__ __forceinline__ Dual<2> lift<Dual<2>>(double x) { return dconst<2>(x); }
template <>
__device__ __forceinline__ Dual<4> lift<Dual<4>>(double x) { return dconst<4>(x); }

// ---- thermodynamic state at one point ----------------------------------------------
// Quantities of the preconditioned system at a primitive state (2-D). Reciprocals are formed
// once (1/(R T), 1/U_r^2, 1/rho) and the ideal-gas identities 1/T = R rho_p, 1/c^2 = rho_p/gamma
// replace further divisions.
template <class T>
struct State2 {
  T p, u, v, t;      // primitive variables
  T rho, rho_p, rho_t, inv_rho, q2, h, c2, inv_c2;
  T ur2, theta;      // U_r^2 and Theta of eq. (10)
};

// eps^2 with eps of eq. (11): min(1, Ma)^2 = min(1, Ma^2) and the cut-off likewise, so no square
// root is needed
template <class T>
__device__ __forceinline__ T epsilon2_from(const T& ma2, const GasParams& g) {
  T one = lift<T>(1.0);
  if (g.eps_mode == 0) return rmin(one, ma2);
  const double km = g.kappa * g.ma_inf;
  return rmin(one, rmax(lift<T>(km * km), ma2));
}

template <class T>
__device__ __forceinline__ State2<T> make_state(const T q[4], const GasParams& g) {
  State2<T> s;
  s.p = q[0];
  s.u = q[1];
  s.v = q[2];
  s.t = q[3];
  s.rho_p = 1.0 / (g.rgas * s.t);
  s.rho = s.p * s.rho_p;
  s.inv_rho = 1.0 / s.rho;
  const T inv_t = g.rgas * s.rho_p;
  s.rho_t = -s.rho * inv_t;
  s.q2 = s.u * s.u + s.v * s.v;
  s.h = g.cp * s.t + 0.5 * s.q2;          // H = E + p/rho for an ideal gas
  s.c2 = g.gamma * g.rgas * s.t;
  s.inv_c2 = s.rho_p * (1.0 / g.gamma);
  const T eps2 = epsilon2_from(s.q2 * s.inv_c2, g);
  s.ur2 = eps2 * s.c2;
  s.theta = 1.0 / s.ur2 + inv_t * (1.0 / g.cp);   // 1/U_r^2 - rho_T/(rho C_p), eq. (10)
  return s;
}

// conservative variables (rho, rho u, rho v, rho E)
template <class T>
__device__ __forceinline__ void conservative2(const T q[4], const GasParams& g, T out[4]) {
  T rho = q[0] / (g.rgas * q[3]);
  out[0] = rho;
  out[1] = rho * q[1];
  out[2] = rho * q[2];
  out[3] = q[0] * (1.0 / (g.gamma - 1.0)) + 0.5 * rho * (q[1] * q[1] + q[2] * q[2]);
}

// inviscid flux along a (not necessarily unit) vector (sx, sy), density given
template <class T>
__device__ __forceinline__ void normal_flux2_rho(const T q[4], const T& rho, double sx, double sy,
                                                 const GasParams& g, T out[4]) {
  T un = q[1] * sx + q[2] * sy;
  T mflux = rho * un;
  T h = g.cp * q[3] + 0.5 * (q[1] * q[1] + q[2] * q[2]);
  out[0] = mflux;
  out[1] = mflux * q[1] + q[0] * sx;
  out[2] = mflux * q[2] + q[0] * sy;
  out[3] = mflux * h;
}

// inviscid flux along a (not necessarily unit) vector (sx, sy)
template <class T>
__device__ __forceinline__ void normal_flux2(const T q[4], double sx, double sy, const GasParams& g,
                                             T out[4]) {
  T rho = q[0] / (g.rgas * q[3]);
  T un = q[1] * sx + q[2] * sy;
  T mflux = rho * un;
  T h = g.cp * q[3] + 0.5 * (q[1] * q[1] + q[2] * q[2]);
  out[0] = mflux;
  out[1] = mflux * q[1] + q[0] * sx;
  out[2] = mflux * q[2] + q[0] * sy;
  out[3] = mflux * h;
}

// y = Gamma x, eq. (9) in 2-D
template <class T, class X>
__device__ __forceinline__ void gamma_mul(const State2<T>& s, const GasParams& g, const X x[4], T y[4]) {
  T y0 = s.theta * x[0] + s.rho_t * x[3];
  y[0] = y0;
  y[1] = s.u * y0 + s.rho * x[1];
  y[2] = s.v * y0 + s.rho * x[2];
  y[3] = s.h * y0 - x[0] + s.rho * (s.u * x[1] + s.v * x[2]) + s.rho * g.cp * x[3];
}

// x = Gamma^{-1} y, from the block structure of Gamma: the momentum rows give the
// velocity components, the remaining 2x2 system has determinant rho C_p / U_r^2
template <class T>
__device__ __forceinline__ void gamma_solve(const State2<T>& s, const GasParams& g, const T y[4], T x[4]) {
  T z = y[3] - (s.h - s.q2) * y[0] - s.u * y[1] - s.v * y[2];
  T rcp = s.rho * g.cp;
  T b = s.ur2 * (y[0] + s.theta * z) * (s.inv_rho * (1.0 / g.cp));
  x[0] = rcp * b - z;
  x[1] = (y[1] - s.u * y[0]) * s.inv_rho;
  x[2] = (y[2] - s.v * y[0]) * s.inv_rho;
  x[3] = b;
}

// y = A_n x with A_n = d(f.n)/dq_p for a unit normal (nx, ny)
template <class T>
__device__ __forceinline__ void flux_jac_mul(const State2<T>& s, const GasParams& g, double nx, double ny,
                                             const T& un, const T x[4], T y[4]) {
  T m = s.rho_p * x[0] + s.rho_t * x[3];
  T dun = nx * x[1] + ny * x[2];
  T r0 = un * m + s.rho * dun;
  T rhoun = s.rho * un;
  y[0] = r0;
  y[1] = s.u * r0 + rhoun * x[1] + nx * x[0];
  y[2] = s.v * r0 + rhoun * x[2] + ny * x[0];
  y[3] = s.h * r0 + rhoun * (s.u * x[1] + s.v * x[2]) + rhoun * g.cp * x[3];
}

// Common inviscid flux of eq. (21), multiplied by |S|:
//   |S| [ (f_n(q-) + f_n(q+))/2 - Gamma |Gamma^{-1} A_n| (q+ - q-)/2 ]
// The jump dq = q+ - q- is passed in: callers form it from the stored offsets q - q_ref, which
// keeps it exact to the size of the disturbance where q+ and q- are large and nearly equal.
// at the arithmetic mean of the primitive states. The matrix function is applied as the
// quadratic that interpolates |lambda| at the three distinct eigenvalues of eq. (13)
// (Newton divided differences), so that
//   Gamma |X| dq = |l1| G dq + f12 (A - l1 G) dq + f123 (A - l1 G) G^{-1} (A - l2 G) dq.
template <class T>
__device__ __forceinline__ void common_flux2(const T qm[4], const T qp[4], const T dq[4], double nx, double ny,
                                             double smag, const GasParams& g, T out[4]) {
  T qa[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) qa[k] = 0.5 * (qm[k] + qp[k]);
  const State2<T> s = make_state(qa, g);
  T un = s.u * nx + s.v * ny;
  T alpha = 0.5 * (1.0 - s.ur2 * s.inv_c2);     // beta = 1/c^2 for an ideal gas
  T cpr = dsqrt(alpha * alpha * un * un + s.ur2);
  T l1 = un;
  T l2 = un * (1.0 - alpha) + cpr;
  T l3 = un * (1.0 - alpha) - cpr;
  T a1 = rabs(l1), a2 = rabs(l2), a3 = rabs(l3);
  // divided differences of |x| at (l1, l2, l3) over one reciprocal
  T d21 = l2 - l1, d31 = l3 - l1, d32 = l3 - l2;
  T inv = 1.0 / (d21 * d31 * d32);
  T f12 = (a2 - a1) * (d31 * d32) * inv;
  T f123 = ((a3 - a1) * d21 - (a2 - a1) * d31) * inv;

  T gd[4], ad[4], w[4], y[4], ay[4];
  gamma_mul(s, g, dq, gd);
  flux_jac_mul(s, g, nx, ny, un, dq, ad);
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = ad[k] - l2 * gd[k];
  gamma_solve(s, g, w, y);
  flux_jac_mul(s, g, nx, ny, un, y, ay);

  T fm[4], fp[4];
  normal_flux2(qm, nx, ny, g, fm);
  normal_flux2(qp, nx, ny, g, fp);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T diss = a1 * gd[k] + f12 * (ad[k] - l1 * gd[k]) + f123 * (ay[k] - l1 * w[k]);
    out[k] = smag * (0.5 * (fm[k] + fp[k]) - 0.5 * diss);
  }
}

}  // namespace pmg

namespace pmg {

// ---- viscous terms (Sec. 2.1 fluxes, Sec. 2.3 BR2 common gradient) ----------------------
// Viscous flux of Sec. 2.1 in 2-D from the absolute velocity (u, v) and the gradients g[v][d] of
// the primitive variables (d = x, y): tau = 2 mu (S - div u / 3 I), K = -(mu C_p / Pr) grad T,
// f_vis,j = (0, tau_1j, tau_2j, u_i tau_ij - K_j).
template <class T>
__device__ __forceinline__ void visc_flux2(const T& u, const T& v, const T g[4][2], const GasParams& gp, T fx[4],
                                           T fy[4]) {
  const T div = g[1][0] + g[2][1];
  const T txx = 2.0 * gp.mu * (g[1][0] - div * (1.0 / 3.0));
  const T tyy = 2.0 * gp.mu * (g[2][1] - div * (1.0 / 3.0));
  const T txy = gp.mu * (g[1][1] + g[2][0]);
  fx[0] = lift<T>(0.0);
  fx[1] = txx;
  fx[2] = txy;
  fx[3] = u * txx + v * txy + gp.kcond * g[3][0];
  fy[0] = lift<T>(0.0);
  fy[1] = txy;
  fy[2] = tyy;
  fy[3] = u * txy + v * tyy + gp.kcond * g[3][1];
}

// Common viscous flux at one flux point of a face, N . f_vis(q_com, grad q_com), with
// q_com = (q- + q+)/2 and the BR2 common gradient of eq. (23): each side contributes its local
// gradient trace plus eta times its lifting of this face, (q_com - q_side) N_side lambda_side,
// lambda = sum_m l_m(face) g'(x_m) / |J_m| along the side's line. kind 0: interior face (mean of
// both sides); 1: wall face (q_com = mean with the ghost, which is the wall state; own side
// only); 2: no-slip adiabatic wall (as 1, and the wall-normal component of grad T removed);
// 3: far field (q_com = the free stream out; own side only). States are stored offsets, qref turns
// them into absolute values. Also returns jn = (q_com - own) N, the jump the own side lifts into
// its volume gradient.
template <class T>
__device__ __forceinline__ void visc_face2(const T own[4], const T out[4], const double qref[4], const T gown[4][2],
                                           const T gout[4][2], double nx, double ny, double sm, double lam,
                                           double nbx, double nby, double nbsm, double nblam, int kind,
                                           const GasParams& gp, T jn[4][2], T fhv[4]) {
  const double Nx = nx * sm, Ny = ny * sm;
  T qc[4], gc[4][2];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T half = (kind == 3) ? (out[v] - own[v]) : 0.5 * (out[v] - own[v]);   // q_com - own
    qc[v] = own[v] + half + qref[v];
    jn[v][0] = half * Nx;
    jn[v][1] = half * Ny;
    const T lo0 = gown[v][0] + gp.br2_eta * lam * jn[v][0];
    const T lo1 = gown[v][1] + gp.br2_eta * lam * jn[v][1];
    if (kind == 0) {
      const double fb = -gp.br2_eta * nblam * nbsm;   // q_com - out = -half
      gc[v][0] = 0.5 * (lo0 + gout[v][0] + fb * nbx * half);
      gc[v][1] = 0.5 * (lo1 + gout[v][1] + fb * nby * half);
    } else {
      gc[v][0] = lo0;
      gc[v][1] = lo1;
    }
  }
  if (kind == 2) {
    const T gn = gc[3][0] * nx + gc[3][1] * ny;
    gc[3][0] = gc[3][0] - gn * nx;
    gc[3][1] = gc[3][1] - gn * ny;
  }
  T fx[4], fy[4];
  visc_flux2(qc[1], qc[2], gc, gp, fx, fy);
#pragma unroll
  for (int v = 0; v < 4; ++v) fhv[v] = Nx * fx[v] + Ny * fy[v];
}

}  // namespace pmg
