// Vector kernels of the Newton-Krylov stage solve: linear combinations of states, blocks of dot
// products with a fixed reduction order (per-workgroup partials over a fixed grid, then one
// workgroup), and the pseudo-transient Newton operator Gamma(q) z / dtau - (F(q + h z) - F(q)) / h
// of eqs. (27)-(28) from two residuals.
#include "krylov.hpp"
#include "physics.hpp"
#include "physics3.hpp"

namespace pmg {

struct Terms {
  const double* x[kNkMaxTerms];
  double c[kNkMaxTerms];
  int n;
};


// y = beta y + sum_k c_k x_k, element by element (y may be one of the x_k); beta = 0 ignores y
__global__ void __launch_bounds__(256) k_lincomb(size_t n, Terms t, double beta, double* y) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    double acc = (beta == 0.0) ? 0.0 : beta * y[i];
    for (int k = 0; k < t.n; ++k) acc = fma(t.c[k], t.x[k][i], acc);
    y[i] = acc;
  }
}

// part[k][block] = sum over this workgroup's indices of w[i] x_k[i]
__global__ void __launch_bounds__(256) k_multidot(size_t n, Terms t, const double* w, double* part) {
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int k = 0; k < t.n; ++k) {
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + tid; i < n; i += (size_t)gridDim.x * 256) s = fma(w[i], t.x[k][i], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (tid == 0) part[(size_t)k * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

// out[k] = sum of part[k][0 .. nblk), in a fixed order
__global__ void __launch_bounds__(256) k_multidot_final(int nk, int nblk, const double* part, double* out) {
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int k = 0; k < nk; ++k) {
    double s = 0.0;
    for (int b = tid; b < nblk; b += 256) s += part[(size_t)k * nblk + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (tid == 0) out[k] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

struct RefState {
  double v[5];
};

// out = Gamma(q) z * inv_dtau - (Fh - F0) * inv_h at every solution point (states [Nv][Np][Ne],
// q stored as the offset from ref)
template <int NV>
__global__ void __launch_bounds__(256) k_newton_op(size_t npts, GasParams g, RefState ref, const double* q,
                                                   const double* z, const double* Fh, const double* F0,
                                                   double inv_dtau, double inv_h, double* out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npts) return;
  double qa[NV], x[NV], y[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    qa[v] = ref.v[v] + q[v * npts + i];
    x[v] = z[v * npts + i];
  }
  if constexpr (NV == 4) {
    const State2<double> s = make_state(qa, g);
    gamma_mul(s, g, x, y);
  } else {
    const State3<double> s = make_state3(qa, g);
    gamma_mul3(s, g, x, y);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v * npts + i] = y[v] * inv_dtau - (Fh[v * npts + i] - F0[v * npts + i]) * inv_h;
}

static unsigned grid_for(size_t n) {
  const size_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_lincomb(size_t n, int nt, const double* const* x, const double* c, double beta, double* y,
                          hipStream_t st) {
  if (nt < 0 || nt > kNkMaxTerms) return hipErrorInvalidValue;
  Terms t{};
  t.n = nt;
  for (int k = 0; k < nt; ++k) {
    t.x[k] = x[k];
    t.c[k] = c[k];
  }
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, st, n, t, beta, y);
  return hipGetLastError();
}

hipError_t launch_multidot(size_t n, int nt, const double* const* x, const double* w, double* part, double* out,
                           hipStream_t st) {
  if (nt < 1 || nt > kNkMaxTerms) return hipErrorInvalidValue;
  Terms t{};
  t.n = nt;
  for (int k = 0; k < nt; ++k) t.x[k] = x[k];
  hipLaunchKernelGGL(k_multidot, dim3(kNkDotBlocks), dim3(256), 0, st, n, t, w, part);
  hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(256), 0, st, nt, kNkDotBlocks, (const double*)part, out);
  return hipGetLastError();
}

hipError_t launch_newton_op(const pmg_level_s& L, const double* q, const double* z, const double* Fh,
                            const double* F0, double inv_dtau, double inv_h, double* out, hipStream_t st) {
  const size_t npts = (size_t)L.np * L.ne;
  if (npts == 0) return hipSuccess;
  RefState ref{};
  for (int k = 0; k < 5; ++k) ref.v[k] = L.q_ref[k];
  const unsigned blocks = (unsigned)((npts + 255) / 256);
  if (L.nv == 4)
    hipLaunchKernelGGL(k_newton_op<4>, dim3(blocks), dim3(256), 0, st, npts, L.gas, ref, q, z, Fh, F0, inv_dtau,
                       inv_h, out);
  else
    hipLaunchKernelGGL(k_newton_op<5>, dim3(blocks), dim3(256), 0, st, npts, L.gas, ref, q, z, Fh, F0, inv_dtau,
                       inv_h, out);
  return hipGetLastError();
}

}  // namespace pmg
