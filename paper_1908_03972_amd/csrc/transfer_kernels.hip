// Level transfers (Sec. 3), pointwise helpers and the deterministic norm reduction.
//
// Restriction and prolongation apply a 1-D (P_c+1) x (P_f+1) matrix along xi and along eta
// (sum factorisation), one thread per output value, element index fastest so that every
// load and store is coalesced. They are bandwidth-bound: one read of the input level and one
// write of the output level per call.
#include "internal.hpp"
#include "vcycle.hpp"

namespace pmg {

struct Mat1D {
  double m[kMaxN1 * kMaxN1];   // row-major [rows][cols]
};

// x_c[v][a + nc b][e] = sum_{j,i} R[b][j] R[a][i] x_f[v][i + nf j][e]
__global__ void __launch_bounds__(256) k_restrict(int ne, int nvar, int nf1, int nc1, Mat1D R,
                                                  const double* __restrict__ xf, double* __restrict__ xc,
                                                  double* __restrict__ xc2) {
  const size_t npc = (size_t)nc1 * nc1, npf = (size_t)nf1 * nf1;
  const size_t total = (size_t)nvar * npc * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int pc = (int)(rest % npc);
  const int v = (int)(rest / npc);
  const int a = pc % nc1, b = pc / nc1;
  const double* base = xf + (size_t)v * npf * ne + e;
  double acc = 0.0;
  for (int j = 0; j < nf1; ++j) {
    double row = 0.0;
    for (int i = 0; i < nf1; ++i) row += R.m[a * nf1 + i] * base[(size_t)(i + nf1 * j) * ne];
    acc += R.m[b * nf1 + j] * row;
  }
  xc[idx] = acc;
  if (xc2) xc2[idx] = acc;
}

// Both restrictions of a V-cycle level transition in one pass (eqs. (39), (42) and (40), (43)):
// xc = xc2 = R xf (the state) and xd = R xg (the defect), the same index map as k_restrict.
__global__ void __launch_bounds__(256) k_restrict_pair(int ne, int nvar, int nf1, int nc1, Mat1D R,
                                                       const double* __restrict__ xf, double* __restrict__ xc,
                                                       double* __restrict__ xc2, const double* __restrict__ xg,
                                                       double* __restrict__ xd) {
  const size_t npc = (size_t)nc1 * nc1, npf = (size_t)nf1 * nf1;
  const size_t total = (size_t)nvar * npc * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int pc = (int)(rest % npc);
  const int v = (int)(rest / npc);
  const int a = pc % nc1, b = pc / nc1;
  const size_t off = (size_t)v * npf * ne + e;
  double acc = 0.0, accd = 0.0;
  for (int j = 0; j < nf1; ++j) {
    double row = 0.0, rowd = 0.0;
    for (int i = 0; i < nf1; ++i) {
      const size_t o = off + (size_t)(i + nf1 * j) * ne;
      row += R.m[a * nf1 + i] * xf[o];
      rowd += R.m[a * nf1 + i] * xg[o];
    }
    acc += R.m[b * nf1 + j] * row;
    accd += R.m[b * nf1 + j] * rowd;
  }
  xc[idx] = acc;
  xc2[idx] = acc;
  xd[idx] = accd;
}

__global__ void __launch_bounds__(256) k_copy(size_t n, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) dst[idx] = src[idx];
}

// x_f[v][i + nf j][e] += sum_{b,a} I[j][b] I[i][a] (xa - xb)[v][a + nc b][e]
__global__ void __launch_bounds__(256) k_prolong(int ne, int nvar, int nc1, int nf1, Mat1D I,
                                                 const double* __restrict__ xa, const double* __restrict__ xb,
                                                 double* __restrict__ xf) {
  const size_t npc = (size_t)nc1 * nc1, npf = (size_t)nf1 * nf1;
  const size_t total = (size_t)nvar * npf * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int pf = (int)(rest % npf);
  const int v = (int)(rest / npf);
  const int i = pf % nf1, j = pf / nf1;
  const size_t off = (size_t)v * npc * ne + e;
  double acc = 0.0;
  for (int b = 0; b < nc1; ++b) {
    double row = 0.0;
    for (int a = 0; a < nc1; ++a) {
      const size_t o = off + (size_t)(a + nc1 * b) * ne;
      const double d = xb ? (xa[o] - xb[o]) : xa[o];
      row += I.m[i * nc1 + a] * d;
    }
    acc += I.m[j * nc1 + b] * row;
  }
  xf[idx] += acc;
}

struct Ref4 {
  double v[4];
};
struct Ref5 {
  double v[5];
};

__global__ void __launch_bounds__(256) k_conservative(int n_points, GasParams g, Ref4 ref,
                                                      const double* __restrict__ q, double* __restrict__ qc) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n_points) return;
  double qv[4], out[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) qv[v] = ref.v[v] + q[(size_t)v * n_points + idx];
  conservative2(qv, g, out);
#pragma unroll
  for (int v = 0; v < 4; ++v) qc[(size_t)v * n_points + idx] = out[v];
}

constexpr int kMaxStages = 8;
struct StageSrc {
  const double* R[kMaxStages];
  double a[kMaxStages];
  int n;
};

// src = c_mass (q_c^n + dt sum_j a_j R_j), the source of eq. (26)
__global__ void __launch_bounds__(256) k_stage_source(size_t n, StageSrc s, double dt, double c_mass,
                                                      const double* __restrict__ qc_n, double* __restrict__ src) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  double acc = 0.0;
  for (int k = 0; k < s.n; ++k) acc += s.a[k] * s.R[k][idx];
  src[idx] = c_mass * (qc_n[idx] + dt * acc);
}

// Explicit predictor of an ESDIRK stage: q_c = q_c^n + dt sum_j a_j R_j (the coefficient of the
// previous stage's residual carries the extra omega), converted to primitive variables
// (p, u_i, T) with p = (gamma - 1)(rho E - rho |u|^2 / 2), T = p / (rho R), stored as offsets from
// q_ref. One thread per solution point; nv = 4 (2-D) or 5 (3-D), layout [nv][npts].
__global__ void __launch_bounds__(256) k_stage_predict(int npts, int nv, StageSrc s, double dt, GasParams gas,
                                                       Ref5 ref, const double* __restrict__ qc_n,
                                                       double* __restrict__ q) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npts) return;
  double c[5];
  for (int v = 0; v < nv; ++v) {
    const size_t o = (size_t)v * npts + idx;
    double acc = 0.0;
    for (int k = 0; k < s.n; ++k) acc += s.a[k] * s.R[k][o];
    c[v] = qc_n[o] + dt * acc;
  }
  const double rho = c[0];
  double ke = 0.0;
  for (int v = 1; v < nv - 1; ++v) {
    const double u = c[v] / rho;
    ke += u * c[v];
    q[(size_t)v * npts + idx] = u - ref.v[v];
  }
  const double p = (gas.gamma - 1.0) * (c[nv - 1] - 0.5 * ke);
  q[idx] = p - ref.v[0];
  q[(size_t)(nv - 1) * npts + idx] = p / (rho * gas.rgas) - ref.v[nv - 1];
}

// norms[v] = sqrt(sum_b part[b][v]); norms[Nv] = sqrt(sum_v sum_b part[b][v]). One workgroup,
// fixed summation order (strided per thread, then a tree), so the result is bitwise repeatable.
__global__ void __launch_bounds__(256) k_norm_finalize(const double* __restrict__ part, int nblk, int nv,
                                                       double* __restrict__ norms) {
  __shared__ double red[256];
  double total = 0.0;
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[(size_t)b * nv + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      norms[v] = sqrt(red[0]);
      total += red[0];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[nv] = sqrt(total);
}

static unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

// Pseudo-time scale of eq. (33), inviscid part: per solution point h_e / (c + |v|) with
// h_e = dx_e / (P+1); a point with T <= 0 or a non-finite value yields -1 so the minimum flags it.
__global__ void __launch_bounds__(256) k_dtau_partial(int ne, int np, const double* __restrict__ q,
                                                      const double* __restrict__ hdx, Ref4 ref, double gr,
                                                      double rgas, double mu, double* __restrict__ part) {
  __shared__ double red[256];
  const size_t total = (size_t)np * ne, st = total;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  double val = 1.0e300;
  if (i < total) {
    const int e = (int)(i % (size_t)ne);
    const double u = q[st + i] + ref.v[1], v = q[2 * st + i] + ref.v[2], t = q[3 * st + i] + ref.v[3];
    const double speed = sqrt(gr * t) + sqrt(u * u + v * v);
    double h = hdx[e] / speed;
    if (mu > 0.0) {                       // viscous limit (dx/(P+1))^2 rho / mu
      const double rho = (q[i] + ref.v[0]) / (rgas * t);
      h = fmin(h, hdx[e] * hdx[e] * rho / mu);
    }
    val = (t > 0.0 && h > 0.0 && h < 1.0e300) ? h : -1.0;
  }
  red[threadIdx.x] = val;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_dtau_final(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[256];
  double m = 1.0e300;
  for (int b = threadIdx.x; b < nblk; b += 256) m = fmin(m, part[b]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_restrict(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                           double* xc, int nvar, hipStream_t st, double* xc2) {
  if (Lf.dim == 3) return launch_restrict3(Lf, Lc, R1, xf, xc, nvar, st, xc2);
  Mat1D R{};
  for (int k = 0; k < Lc.n1 * Lf.n1; ++k) R.m[k] = R1[k];
  const size_t total = (size_t)nvar * Lc.np * Lc.ne;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3(blocks_for(total)), dim3(256), 0, st, Lf.ne, nvar, Lf.n1, Lc.n1, R, xf, xc,
                     xc2);
  return hipGetLastError();
}

hipError_t launch_restrict_pair(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                                double* xc, double* xc2, const double* xg, double* xd, int nvar, hipStream_t st) {
  if (Lf.dim == 3) {
    const hipError_t e = launch_restrict3(Lf, Lc, R1, xf, xc, nvar, st, xc2);
    return e != hipSuccess ? e : launch_restrict3(Lf, Lc, R1, xg, xd, nvar, st, nullptr);
  }
  Mat1D R{};
  for (int k = 0; k < Lc.n1 * Lf.n1; ++k) R.m[k] = R1[k];
  const size_t total = (size_t)nvar * Lc.np * Lc.ne;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict_pair, dim3(blocks_for(total)), dim3(256), 0, st, Lf.ne, nvar, Lf.n1, Lc.n1, R, xf,
                     xc, xc2, xg, xd);
  return hipGetLastError();
}

hipError_t launch_copy(size_t n, const double* src, double* dst, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(256), 0, st, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_prolong(const pmg_level_s& Lc, const pmg_level_s& Lf, const double* I1, const double* xa,
                          const double* xb, double* xf, int nvar, hipStream_t st) {
  if (Lf.dim == 3) return launch_prolong3(Lc, Lf, I1, xa, xb, xf, nvar, st);
  Mat1D I{};
  for (int k = 0; k < Lc.n1 * Lf.n1; ++k) I.m[k] = I1[k];
  const size_t total = (size_t)nvar * Lf.np * Lf.ne;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(total)), dim3(256), 0, st, Lf.ne, nvar, Lc.n1, Lf.n1, I, xa, xb,
                     xf);
  return hipGetLastError();
}

hipError_t launch_conservative(const pmg_level_s& L, const double* q, double* qc, hipStream_t st) {
  if (L.dim == 3) return launch_conservative3(L, q, qc, st);
  const int npts = L.np * L.ne;
  if (npts == 0) return hipSuccess;
  Ref4 ref{};
  for (int k = 0; k < 4; ++k) ref.v[k] = L.q_ref[k];
  hipLaunchKernelGGL(k_conservative, dim3(blocks_for(npts)), dim3(256), 0, st, npts, L.gas, ref, q, qc);
  return hipGetLastError();
}

hipError_t launch_stage_source(const pmg_level_s& L, const double* qc_n, const double* const* R, const double* a,
                               int n_prev, double dt, double c_mass, double* src, hipStream_t st) {
  if (n_prev > kMaxStages) return hipErrorInvalidValue;
  StageSrc s{};
  s.n = n_prev;
  for (int k = 0; k < n_prev; ++k) {
    s.R[k] = R[k];
    s.a[k] = a[k];
  }
  const size_t n = L.state_elems();
  hipLaunchKernelGGL(k_stage_source, dim3(blocks_for(n)), dim3(256), 0, st, n, s, dt, c_mass, qc_n, src);
  return hipGetLastError();
}

hipError_t launch_stage_predict(const pmg_level_s& L, const double* qc_n, const double* const* R, const double* a,
                                int n_prev, double dt, double omega, double* q, hipStream_t st) {
  if (n_prev < 1 || n_prev > kMaxStages) return hipErrorInvalidValue;
  StageSrc s{};
  s.n = n_prev;
  for (int k = 0; k < n_prev; ++k) {
    s.R[k] = R[k];
    s.a[k] = a[k] + (k == n_prev - 1 ? omega : 0.0);
  }
  Ref5 ref{};
  for (int k = 0; k < 5; ++k) ref.v[k] = L.q_ref[k];
  const int npts = L.np * L.ne;
  if (npts == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stage_predict, dim3(blocks_for((size_t)npts)), dim3(256), 0, st, npts, L.nv, s, dt, L.gas,
                     ref, qc_n, q);
  return hipGetLastError();
}

hipError_t launch_norm_finalize(const pmg_level_s& L, hipStream_t st) {
  return launch_norm_finalize_to(L.part, residual_blocks(L), L.nv, L.norms, st);
}

hipError_t launch_norm_finalize_to(const double* part, int nblk, int nv, double* norms, hipStream_t st) {
  hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, st, part, nblk, nv, norms);
  return hipGetLastError();
}

int dtau_blocks(const pmg_level_s& L) { return (int)blocks_for((size_t)L.np * L.ne); }

hipError_t launch_dtau_min(const pmg_level_s& L, const double* q, hipStream_t st) {
  Ref4 ref{};
  for (int k = 0; k < 4; ++k) ref.v[k] = L.q_ref[k];
  const int nblk = dtau_blocks(L);
  if (L.dim == 3) {
    const hipError_t e = launch_dtau_partial3(L, q, nblk, st);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_dtau_partial, dim3(nblk), dim3(256), 0, st, L.ne, L.np, q, L.hdx, ref,
                       L.gas.gamma * L.gas.rgas, L.gas.rgas, L.gas.mu, L.dtpart);
  }
  hipLaunchKernelGGL(k_dtau_final, dim3(1), dim3(256), 0, st, L.dtpart, nblk, L.dtmin);
  return hipGetLastError();
}

}  // namespace pmg
