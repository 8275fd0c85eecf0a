// Element-line Jacobi on quadrilateral levels: block-tridiagonal solves along lines of elements.
//
// A line's matrix carries the element blocks D_e of eqs. (28)-(30) on its diagonal. Beside them
// are the blocks that couple an element to its predecessor and successor on the line,
// A_{e,e'} = -dR_e/dq_{e'}. The neighbour enters R_e only through the common flux of eq. (21) on
// the shared face, so such a block factors as A = P K E:
//   E  extrapolates the neighbour's state along its lines to the face's P+1 flux points
//      (weights l_m(-1) or l_m(+1));
//   K  holds, at each flux point, the 4 x 4 derivative of |S| f_com with respect to the neighbour's
//      trace;
//   P  spreads the result onto the element's points on the lines through those flux points, with
//      weights g'(xi)/|J|.
// Only K is stored: 16 (P+1) doubles per side and element.
//
// Kernels:
//   k_line_coupling  K of both sides of every element. Forward-mode duals are seeded in the
//                    neighbour's trace; the own trace is held fixed.
//   k_line_thomas    One workgroup per line runs the block-Thomas elimination
//                    D'_k = D_k - A_{k,k-1} W_{k-1} A_{k-1,k}, W_k = D'_k^{-1}. The Schur term has rank
//                    4(P+1). It is formed from H = W_{k-1} P K (n x 4(P+1), kept in LDS between steps),
//                    its face trace T = E H and Z = K T. D'_k is inverted by Gauss-Jordan with partial
//                    pivoting in LDS.
//   k_line_sweep     One workgroup per line. Forward: y_k = W_k (r_k - A_{k,k-1} y_{k-1}). Backward:
//                    x_k = y_k - W_k A_{k,k+1} x_{k+1}, then q += alpha x.
//   k_line_dense     The coupling blocks written out dense (for tests).
#include "lines.hpp"

namespace pmg {
namespace {

struct LineArgs {
  LevelView lv;
  Ops1D ops;
  GasParams gas;
  const int* elems;      // [n_lines][K]
  const int* fside;      // [2][Ne]
  int K;
  double* Kc;            // [2][Ne][n1][4][4]
};

template <int P>
struct LineCfg {
  static constexpr int N1 = P + 1, NP = N1 * N1, NV = 4, N = NV * NP;
  static constexpr int NJ = NV * N1;     // rank of a coupling block: 4 variables x (P+1) flux points
  static constexpr int LD = N + 1;       // LDS row stride of the n x n block
  static constexpr int NT = 256;
  static_assert(N <= NT / 2, "the matrix-vector products give each row two threads");
};

// Face geometry of a quad (faces 0/1: xi = -1/+1, 2/3: eta = -1/+1). Flux point k of face f sits on
// the solution-point line that runs normal to the face at tangential index k; m is the position
// along that line.
__device__ __forceinline__ int face_line_point(int f, int k, int m, int n1) { return f < 2 ? m + n1 * k : k + n1 * m; }
__device__ __forceinline__ int point_line(int f, int pp, int n1) { return f < 2 ? pp / n1 : pp % n1; }
__device__ __forceinline__ int point_normal(int f, int pp, int n1) { return f < 2 ? pp % n1 : pp / n1; }
__device__ __forceinline__ const double* trace_weights(const Ops1D& o, int f) { return (f % 2 == 0) ? o.lm : o.lp; }
__device__ __forceinline__ double corr_deriv(const Ops1D& o, int f, int m) { return (f % 2 == 0) ? o.gL[m] : o.gR[m]; }

// Task t = k * 4 + w: column w of K at flux point k on the face towards side `side`'s neighbour.
template <int P>
__global__ void __launch_bounds__(64) k_line_coupling(LineArgs a, const double* q) {
  using C = LineCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, NJ = C::NJ;
  static_assert(NJ <= 64, "one thread per task");
  const int ne = a.lv.ne, e = blockIdx.x, side = blockIdx.y, t = threadIdx.x;
  if (t >= NJ) return;
  double* Kout = a.Kc + ((size_t)side * ne + e) * (NJ * NV);
  const int k = t / NV, w = t % NV;
  const int f = a.fside[side * ne + e];
  if (f < 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Kout[(k * NV + v) * NV + w] = 0.0;
    return;
  }
  const Ops1D& o = a.ops;
  const size_t sstride = (size_t)NP * ne;
  const double* wt = trace_weights(o, f);
  double ownv[NV] = {0.0, 0.0, 0.0, 0.0};
  for (int m = 0; m < N1; ++m) {
    const size_t gp = (size_t)face_line_point(f, k, m, N1) * ne + e;
#pragma unroll
    for (int v = 0; v < NV; ++v) ownv[v] += wt[m] * q[v * sstride + gp];
  }
  const int nb = a.lv.nbr[f * ne + e], nf = a.lv.nbf[f * ne + e];
  const int kk = a.lv.ori[f * ne + e] ? (N1 - 1 - k) : k;
  const double* wn = trace_weights(o, nf);
  double ov[NV] = {0.0, 0.0, 0.0, 0.0};
  for (int m = 0; m < N1; ++m) {
    const size_t gp = (size_t)face_line_point(nf, kk, m, N1) * ne + nb;
#pragma unroll
    for (int v = 0; v < NV; ++v) ov[v] += wn[m] * q[v * sstride + gp];
  }
  Dual<1> own[NV], out[NV];              // stored offsets; the neighbour's trace seeded in component w
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    own[v] = dconst<1>(ownv[v]);
    out[v] = dconst<1>(ov[v]);
    out[v].d[0] = (v == w) ? 1.0 : 0.0;
  }
  const size_t fo = ((size_t)(f * N1 + k) * 3) * ne + e;
  const double nx = a.lv.fvec[fo], ny = a.lv.fvec[fo + ne], sm = a.lv.fvec[fo + 2 * ne];
  Dual<1> own_a[NV], out_a[NV], dq[NV], fh[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    own_a[v] = own[v] + a.lv.q_ref[v];
    out_a[v] = out[v] + a.lv.q_ref[v];
  }
  if (f == 0 || f == 2) {                // the neighbour is on the left of the +xi / +eta normal
#pragma unroll
    for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
    common_flux2(out_a, own_a, dq, nx, ny, sm, a.gas, fh);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
    common_flux2(own_a, out_a, dq, nx, ny, sm, a.gas, fh);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Kout[(k * NV + v) * NV + w] = fh[v].d[0];
}

// A[r][c] = (1/|J|)(pp) g'_f(normal index of pp) K[k(pp)][v][w] l_m(face of the neighbour) where the
// neighbour's point pn lies on the line through the matching flux point, else 0.
template <int P>
__global__ void __launch_bounds__(256) k_line_dense(LineArgs a, double* Am, double* Ap) {
  using C = LineCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ;
  const int ne = a.lv.ne, e = blockIdx.x, side = blockIdx.y;
  double* A = side ? Ap : Am;
  if (!A) return;
  A += (size_t)e * N * N;
  const int f = a.fside[side * ne + e];
  const Ops1D& o = a.ops;
  const double* Kf = a.Kc + ((size_t)side * ne + e) * (NJ * NV);
  const double* ijac = a.lv.met + 4 * (size_t)NP * ne;
  const int nf = f >= 0 ? a.lv.nbf[f * ne + e] : 0, ori = f >= 0 ? a.lv.ori[f * ne + e] : 0;
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    double val = 0.0;
    if (f >= 0) {
      const int r = t / N, c = t % N;
      const int pp = r / NV, v = r % NV, pn = c / NV, w = c % NV;
      const int kf = point_line(f, pp, N1), ni = point_normal(f, pp, N1);
      const int kk = point_line(nf, pn, N1), mm = point_normal(nf, pn, N1);
      if (kk == (ori ? N1 - 1 - kf : kf))
        val = ijac[(size_t)pp * ne + e] * corr_deriv(o, f, ni) * Kf[(kf * NV + v) * NV + w] * trace_weights(o, nf)[mm];
    }
    A[t] = val;
  }
}

template <int P, class T>
__global__ void __launch_bounds__(256) k_line_thomas(LineArgs a, const double* D, T* Winv, int* flag) {
  using C = LineCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ, LD = C::LD, NT = C::NT;
  __shared__ double sM[N * LD];          // D'_k, inverted in place
  __shared__ double sH[N * NJ];          // H = W_{k-1} P K of the previous element
  __shared__ double sT[NJ * NJ], sZ[NJ * NJ];
  __shared__ double sf[N];               // column k of the eliminated matrix (0 at the pivot row)
  __shared__ int sperm[N];               // row exchanged with row k at step k
  __shared__ double spiv;
  const int ne = a.lv.ne, line = blockIdx.x, tid = threadIdx.x;
  const Ops1D& o = a.ops;
  const double* ijac = a.lv.met + 4 * (size_t)NP * ne;
  bool bad = false;
  for (int k = 0; k < a.K; ++k) {
    const int e = a.elems[(size_t)line * a.K + k];
    const double* De = D + (size_t)e * N * N;
    for (int t = tid; t < N * N; t += NT) sM[(t / N) * LD + t % N] = De[t];
    if (k > 0) {
      // D'_k = D_k - P_m K_m (E_m H) with E_m taking the previous element's trace at this
      // element's flux points, and H's columns expanded onto this element's points by E_p
      const int ep = a.elems[(size_t)line * a.K + k - 1];
      const int fm = a.fside[e];
      const int nfm = a.lv.nbf[fm * ne + e], om = a.lv.ori[fm * ne + e];
      const int fpp = a.fside[ne + ep];
      const int nfp = a.lv.nbf[fpp * ne + ep], op = a.lv.ori[fpp * ne + ep];
      const double* wnm = trace_weights(o, nfm);
      for (int t = tid; t < NJ * NJ; t += NT) {
        const int i = t / NJ, j = t % NJ, kf = i / NV, w = i % NV;
        const int kk = om ? N1 - 1 - kf : kf;
        double s = 0.0;
        for (int m = 0; m < N1; ++m) s += wnm[m] * sH[(face_line_point(nfm, kk, m, N1) * NV + w) * NJ + j];
        sT[t] = s;
      }
      __syncthreads();
      const double* Km = a.Kc + (size_t)e * (NJ * NV);
      for (int t = tid; t < NJ * NJ; t += NT) {
        const int i = t / NJ, j = t % NJ, kf = i / NV, v = i % NV;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NV; ++w) s += Km[(kf * NV + v) * NV + w] * sT[(kf * NV + w) * NJ + j];
        sZ[t] = s;
      }
      __syncthreads();
      const double* wnp = trace_weights(o, nfp);
      for (int t = tid; t < N * N; t += NT) {
        const int r = t / N, c = t % N;
        const int pp = r / NV, v = r % NV, pn = c / NV, w = c % NV;
        const int kf = point_line(fm, pp, N1), ni = point_normal(fm, pp, N1);
        const int kkp = point_line(nfp, pn, N1), mm = point_normal(nfp, pn, N1);
        const int kfp = op ? N1 - 1 - kkp : kkp;
        sM[r * LD + c] -= ijac[(size_t)pp * ne + e] * corr_deriv(o, fm, ni) *
                          sZ[(kf * NV + v) * NJ + kfp * NV + w] * wnp[mm];
      }
    }
    __syncthreads();
    // Gauss-Jordan inversion in place with partial pivoting by row exchanges: step kk moves the
    // largest remaining entry of column kk to row kk, scales that row and eliminates column kk from
    // every other row, storing the inverse's column kk in its place; the exchanges are undone on
    // the columns at the end.
    for (int kk = 0; kk < N; ++kk) {
      if (tid < 64) {
        double best = -1.0;
        int bi = N;
        for (int i = kk + tid; i < N; i += 64) {
          const double av = fabs(sM[i * LD + kk]);
          if (av > best) {
            best = av;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {     // largest magnitude, ties to the lower row
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        const int p = bi < N ? bi : kk;               // only non-finite columns leave no candidate
        for (int i = tid; i < N; i += 64) sf[i] = (i == kk) ? 0.0 : (i == p ? sM[kk * LD + kk] : sM[i * LD + kk]);
        if (tid == 0) {
          sperm[kk] = p;
          spiv = sM[p * LD + kk];
        }
      }
      __syncthreads();
      const int p = sperm[kk];
      double piv = spiv;
      if (piv == 0.0 || !isfinite(piv)) {
        bad = true;
        piv = 1.0;
      }
      const double ip = 1.0 / piv;
      for (int j = tid; j < N; j += NT) {
        const double pv = sM[p * LD + j], kv = sM[kk * LD + j];
        if (p != kk) sM[p * LD + j] = kv;
        sM[kk * LD + j] = (j == kk ? 1.0 : pv) * ip;
      }
      __syncthreads();
      for (int t = tid; t < N * N; t += NT) {
        const int i = t / N, j = t % N;
        if (i == kk) continue;
        const double cur = (j == kk) ? 0.0 : sM[i * LD + j];
        sM[i * LD + j] = cur - sf[i] * sM[kk * LD + j];
      }
      __syncthreads();
    }
    for (int i = tid; i < N; i += NT) {
      for (int kk = N - 1; kk >= 0; --kk) {
        const int p = sperm[kk];
        if (p != kk) {
          const double x = sM[i * LD + kk];
          sM[i * LD + kk] = sM[i * LD + p];
          sM[i * LD + p] = x;
        }
      }
    }
    __syncthreads();
    T* We = Winv + (size_t)e * N * N;
    for (int t = tid; t < N * N; t += NT) We[t] = (T)sM[(t % N) * LD + t / N];
    if (k + 1 < a.K) {
      // H[r][kf, w] = sum over the points pp on line kf of the face towards the next element and
      // over v of W[r][pp, v] (1/|J|)(pp) g'(pp) K_p[kf][v][w]
      const int fpf = a.fside[ne + e];
      const double* Kp = a.Kc + ((size_t)ne + e) * (NJ * NV);
      for (int t = tid; t < N * NJ; t += NT) {
        const int r = t / NJ, j = t % NJ, kf = j / NV, w = j % NV;
        double s = 0.0;
        for (int m = 0; m < N1; ++m) {
          const int pp = face_line_point(fpf, kf, m, N1);
          const double cm = ijac[(size_t)pp * ne + e] * corr_deriv(o, fpf, m);
#pragma unroll
          for (int v = 0; v < NV; ++v) s += sM[r * LD + pp * NV + v] * cm * Kp[(kf * NV + v) * NV + w];
        }
        sH[t] = s;
      }
    }
    __syncthreads();
  }
  if (bad) *flag = 1;
}

// out = A_side x_nb (assign) or out -= A_side x_nb, for element e and its neighbour on side `side`
// (x_nb in LDS, n values). Every thread of the block must call it.
template <int P>
__device__ __forceinline__ void apply_coupling(const LineArgs& a, int e, int side, const double* x_nb, double* st,
                                               double* su, double* out, bool subtract) {
  using C = LineCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ, NT = C::NT;
  const int ne = a.lv.ne, tid = threadIdx.x;
  const Ops1D& o = a.ops;
  const int f = a.fside[side * ne + e];
  const int nf = a.lv.nbf[f * ne + e], ori = a.lv.ori[f * ne + e];
  const double* wn = trace_weights(o, nf);
  for (int t = tid; t < NJ; t += NT) {
    const int kf = t / NV, w = t % NV;
    const int kk = ori ? N1 - 1 - kf : kf;
    double s = 0.0;
    for (int m = 0; m < N1; ++m) s += wn[m] * x_nb[face_line_point(nf, kk, m, N1) * NV + w];
    st[t] = s;
  }
  __syncthreads();
  const double* Kf = a.Kc + ((size_t)side * ne + e) * (NJ * NV);
  for (int t = tid; t < NJ; t += NT) {
    const int kf = t / NV, v = t % NV;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NV; ++w) s += Kf[(kf * NV + v) * NV + w] * st[kf * NV + w];
    su[t] = s;
  }
  __syncthreads();
  const double* ijac = a.lv.met + 4 * (size_t)NP * ne;
  for (int t = tid; t < N; t += NT) {
    const int pp = t / NV, v = t % NV;
    const int kf = point_line(f, pp, N1), ni = point_normal(f, pp, N1);
    const double val = ijac[(size_t)pp * ne + e] * corr_deriv(o, f, ni) * su[kf * NV + v];
    out[t] = subtract ? out[t] - val : val;
  }
}

// y = W_e b with two threads per row (each half of the columns), the halves summed by the caller
// from part[0][r] + part[1][r]; W_e column-major, so a column's rows are contiguous.
template <int P, class T>
__device__ __forceinline__ void line_matvec(const T* We, const double* b, double (*part)[LineCfg<P>::NT / 2]) {
  using C = LineCfg<P>;
  constexpr int N = C::N, HALF = C::NT / 2;
  const int h = threadIdx.x / HALF, rr = threadIdx.x % HALF;
  double acc = 0.0;
  if (rr < N) {
    const int c0 = h ? N / 2 : 0, c1 = h ? N : N / 2;
    for (int c = c0; c < c1; ++c) acc += (double)We[(size_t)c * N + rr] * b[c];
  }
  part[h][rr] = acc;
}

template <int P, class T>
__global__ void __launch_bounds__(256) k_line_sweep(LineArgs a, const T* Winv, double* r, double* q, double alpha) {
  using C = LineCfg<P>;
  constexpr int NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ, NT = C::NT, HALF = NT / 2;
  __shared__ double sb[N], sx[N], st[NJ], su[NJ];
  __shared__ double part[2][HALF];
  const int ne = a.lv.ne, line = blockIdx.x, tid = threadIdx.x, K = a.K;
  const int* el = a.elems + (size_t)line * K;
  // forward: y_k = W_k (r_k - A_{k,k-1} y_{k-1}); y_k replaces r_k and stays in sx for the next step
  for (int k = 0; k < K; ++k) {
    const int e = el[k];
    for (int t = tid; t < N; t += NT) sb[t] = r[((size_t)(t % NV) * NP + t / NV) * ne + e];
    if (k > 0) apply_coupling<P>(a, e, 0, sx, st, su, sb, true);
    __syncthreads();
    line_matvec<P, T>(Winv + (size_t)e * N * N, sb, part);
    __syncthreads();
    for (int t = tid; t < N; t += NT) {
      const double y = part[0][t] + part[1][t];
      sx[t] = y;
      r[((size_t)(t % NV) * NP + t / NV) * ne + e] = y;
    }
    __syncthreads();
  }
  // backward: x_{K-1} = y_{K-1}; x_k = y_k - W_k A_{k,k+1} x_{k+1}; q += alpha x
  {
    const int e = el[K - 1];
    for (int t = tid; t < N; t += NT) q[((size_t)(t % NV) * NP + t / NV) * ne + e] += alpha * sx[t];
  }
  for (int k = K - 2; k >= 0; --k) {
    const int e = el[k];
    apply_coupling<P>(a, e, 1, sx, st, su, sb, false);
    __syncthreads();
    line_matvec<P, T>(Winv + (size_t)e * N * N, sb, part);
    __syncthreads();
    for (int t = tid; t < N; t += NT) {
      const size_t gi = ((size_t)(t % NV) * NP + t / NV) * ne + e;
      const double x = r[gi] - (part[0][t] + part[1][t]);
      sx[t] = x;
      q[gi] += alpha * x;
    }
    __syncthreads();
  }
}

LineArgs make_args(const pmg_level_s& L, const LineFactors& lf) {
  LineArgs a{};
  a.lv = L.view();
  a.ops = L.ops;
  a.gas = L.gas;
  a.elems = lf.elems;
  a.fside = lf.fside;
  a.K = lf.K;
  a.Kc = lf.Kc;
  return a;
}

template <int P>
hipError_t line_factor_p(const pmg_level_s& L, const LineArgs& a, const double* q, pmg_factors_s& fac, hipStream_t st) {
  const LineFactors& lf = *fac.lines;
  hipLaunchKernelGGL(k_line_coupling<P>, dim3(L.ne, 2), dim3(64), 0, st, a, q);
  if (fac.precision == 32)
    hipLaunchKernelGGL((k_line_thomas<P, float>), dim3(lf.n_lines), dim3(LineCfg<P>::NT), 0, st, a, lf.D,
                       (float*)lf.Winv, L.flag);
  else
    hipLaunchKernelGGL((k_line_thomas<P, double>), dim3(lf.n_lines), dim3(LineCfg<P>::NT), 0, st, a, lf.D,
                       (double*)lf.Winv, L.flag);
  return hipGetLastError();
}

template <int P>
hipError_t line_sweep_p(const LineArgs& a, const pmg_factors_s& fac, double* q, double alpha, hipStream_t st) {
  const LineFactors& lf = *fac.lines;
  if (fac.precision == 32)
    hipLaunchKernelGGL((k_line_sweep<P, float>), dim3(lf.n_lines), dim3(LineCfg<P>::NT), 0, st, a,
                       (const float*)lf.Winv, lf.r, q, alpha);
  else
    hipLaunchKernelGGL((k_line_sweep<P, double>), dim3(lf.n_lines), dim3(LineCfg<P>::NT), 0, st, a,
                       (const double*)lf.Winv, lf.r, q, alpha);
  return hipGetLastError();
}

template <int P>
hipError_t line_dense_p(const pmg_level_s& L, const LineArgs& a, double* Am, double* Ap, hipStream_t st) {
  hipLaunchKernelGGL(k_line_dense<P>, dim3(L.ne, 2), dim3(256), 0, st, a, Am, Ap);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_line_factor(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                              pmg_factors_s& fac, hipStream_t st) {
  if (!fac.lines || L.dim != 2 || L.P > kLineMaxP) return hipErrorInvalidValue;
  const LineFactors& lf = *fac.lines;
  pmg_factors_s blocks = fac;            // D_e only: no element inverses are written
  blocks.W = nullptr;
  blocks.lines = nullptr;
  hipError_t err = launch_jacobian(L, q, dtau, c_mass, lf.D, blocks, st);
  if (err != hipSuccess) return err;
  if (D_out) {
    err = hipMemcpyAsync(D_out, lf.D, (size_t)L.ne * L.n * L.n * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (err != hipSuccess) return err;
  }
  const LineArgs a = make_args(L, lf);
  switch (L.P) {
    case 0: return line_factor_p<0>(L, a, q, fac, st);
    case 1: return line_factor_p<1>(L, a, q, fac, st);
    case 2: return line_factor_p<2>(L, a, q, fac, st);
    case 3: return line_factor_p<3>(L, a, q, fac, st);
    case 4: return line_factor_p<4>(L, a, q, fac, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_line_sweep(const pmg_level_s& L, const pmg_factors_s& fac, double* q, const double* src,
                             const double* S, double c_mass, double alpha, bool want_norms, hipStream_t st) {
  if (!fac.lines || L.dim != 2 || L.P > kLineMaxP) return hipErrorInvalidValue;
  const LineFactors& lf = *fac.lines;
  hipError_t err = launch_residual(L, q, src, S, c_mass, lf.r, want_norms, st);
  if (err != hipSuccess) return err;
  const LineArgs a = make_args(L, lf);
  switch (L.P) {
    case 0: return line_sweep_p<0>(a, fac, q, alpha, st);
    case 1: return line_sweep_p<1>(a, fac, q, alpha, st);
    case 2: return line_sweep_p<2>(a, fac, q, alpha, st);
    case 3: return line_sweep_p<3>(a, fac, q, alpha, st);
    case 4: return line_sweep_p<4>(a, fac, q, alpha, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_line_dense(const pmg_level_s& L, const pmg_factors_s& fac, double* Am, double* Ap,
                             hipStream_t st) {
  if (!fac.lines || L.dim != 2 || L.P > kLineMaxP) return hipErrorInvalidValue;
  const LineArgs a = make_args(L, *fac.lines);
  switch (L.P) {
    case 0: return line_dense_p<0>(L, a, Am, Ap, st);
    case 1: return line_dense_p<1>(L, a, Am, Ap, st);
    case 2: return line_dense_p<2>(L, a, Am, Ap, st);
    case 3: return line_dense_p<3>(L, a, Am, Ap, st);
    case 4: return line_dense_p<4>(L, a, Am, Ap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmg
