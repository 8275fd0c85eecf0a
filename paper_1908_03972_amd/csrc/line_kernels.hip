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
//                    It also stores, for the substitutions, C_k = W_k P_m K_m and B_k = W_k P_p K_p
//                    (n x 4(P+1) each) and their face traces M_k = E_{k+1} C_k, N_k = E_{k-1} B_k.
//   line sweep       The block-tridiagonal solve y_k = W_k (r_k - A_{k,k-1} y_{k-1}),
//                    x_k = y_k - W_k A_{k,k+1} x_{k+1}. A coupling block reads its neighbour only
//                    through the 4(P+1) trace values on the shared face, so only those travel along
//                    the line: with z_k = W_k r_k, y_k = z_k - C_k t_k where t_k = E_k y_{k-1} obeys
//                    t_{k+1} = E_{k+1} z_k - M_k t_k; likewise x_k = y_k - B_k s_k with
//                    s_{k-1} = E_{k-1} y_k - N_k s_k. Three element-parallel kernels (k_line_zu,
//                    k_line_yv, k_line_x: the n x n and the two n x 4(P+1) matrix-vector products) and
//                    two line-sequential ones (k_line_rec: 4(P+1)-square products per step) replace
//                    a chain of K dependent n x n products per line.
//   k_line_dense     The coupling blocks written out dense (for tests).
#include "lines.hpp"
#include "wave_ops.hpp"

namespace pmg {
namespace {

struct LineArgs {
  LevelView lv;
  Ops1D ops;
  GasParams gas;
  const int* elems;      // [n_lines][K]
  const int* fside;      // [2][Ne]
  const int* pos;        // [Ne]: line * K + position of the element in its line
  int K;
  double* Kc;            // [2][Ne][n1][4][4]
  void* C;               // [Ne][NJ][n] at the factor precision
  void* B;               // [Ne][NJ][n] at the factor precision
  double* M;             // [Ne][NJ][NJ]
  double* N;             // [Ne][NJ][NJ]
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
  __shared__ double sH[NJ * N];          // B_{k-1} = W_{k-1} P_p K_p of the previous element, [j][r]
  __shared__ double sC[NJ * N];          // C_k = W_k P_m K_m, [j][r]
  __shared__ double sT[NJ * NJ], sZ[NJ * NJ];
  __shared__ double sf[N];               // column k of the eliminated matrix (0 at the pivot row)
  __shared__ int sperm[N];               // row exchanged with row k at step k
  __shared__ int scol[N];                // column of sM that holds column c of the inverse
  __shared__ double spiv;
  __shared__ double sIJ[NP];             // 1/|J| at the element's points
  __shared__ double sK[2][NJ * NV];      // its coupling derivatives towards the previous / next element
  const int ne = a.lv.ne, line = blockIdx.x, tid = threadIdx.x;
  const Ops1D& o = a.ops;
  const double* ijac = a.lv.met + 4 * (size_t)NP * ne;
  bool bad = false;
  for (int k = 0; k < a.K; ++k) {
    const int e = a.elems[(size_t)line * a.K + k];
    const double* De = D + (size_t)e * N * N;
    for (int t = tid; t < N * N; t += NT) sM[(t / N) * LD + t % N] = De[t];
    for (int t = tid; t < NP; t += NT) sIJ[t] = ijac[(size_t)t * ne + e];
    for (int t = tid; t < 2 * NJ * NV; t += NT)
      sK[t / (NJ * NV)][t % (NJ * NV)] = a.Kc[((size_t)(t / (NJ * NV)) * ne + e) * (NJ * NV) + t % (NJ * NV)];
    __syncthreads();
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
        for (int m = 0; m < N1; ++m) s += wnm[m] * sH[j * N + face_line_point(nfm, kk, m, N1) * NV + w];
        sT[t] = s;
      }
      __syncthreads();
      const double* Km = sK[0];
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
        sM[r * LD + c] -= sIJ[pp] * corr_deriv(o, fm, ni) *
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
        // pivot key: the upper word of |entry| (sign 0, exponent, 20 mantissa bits) with its low 7
        // bits replaced by 127 - row; the largest key wins, so the pivot is within a factor
        // 1 + 2^-13 of the largest candidate and ties go to the lowest row
        static_assert(N <= 128, "row index in 7 bits");
        unsigned key = 0u;
        for (int i = kk + tid; i < N; i += 64)
          key = max(key, (((unsigned)__double2hiint(fabs(sM[i * LD + kk]))) & ~0x7Fu) | (unsigned)(127 - i));
        const unsigned wkey = wave_max_u32(key);
        const int p = 127 - (int)(wkey & 0x7Fu);      // every row kk..N-1 is a candidate, so wkey != 0
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
      {
        // one column per thread, rows in RG interleaved groups; the row loop has a fixed trip count
        // so that its LDS loads can be issued ahead of the stores
        constexpr int CW = N <= 64 ? 64 : 128, RG = NT / CW;
        static_assert(N <= CW && NT % CW == 0, "a thread column per matrix column");
        constexpr int NR = (N + RG - 1) / RG;
        const int j = tid % CW, rg = tid / CW;
        if (j < N) {
          const double pr = sM[kk * LD + j];
          const bool colk = (j == kk);
          double col[NR], fac[NR];        // the whole column first, then the updates
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            const int i = rg + q * RG;
            col[q] = (i < N && !colk) ? sM[i * LD + j] : 0.0;
            fac[q] = i < N ? sf[i] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < NR; ++q) {
            const int i = rg + q * RG;
            if (i < N && i != kk) sM[i * LD + j] = col[q] - fac[q] * pr;
          }
        }
      }
      __syncthreads();
    }
    // the row exchanges act on the inverse's columns in reverse order; follow where each column
    // ends up instead of moving the data: W[r][c] = sM[r][scol[c]]
    for (int c = tid; c < N; c += NT) {
      int pc = c;
      for (int kk = N - 1; kk >= 0; --kk) {
        const int p = sperm[kk];
        pc = (pc == kk) ? p : (pc == p ? kk : pc);
      }
      scol[pc] = c;
    }
    __syncthreads();
    T* We = Winv + (size_t)e * N * N;
    for (int t = tid; t < N * N; t += NT) We[t] = (T)sM[(t % N) * LD + scol[t / N]];
    // B_k = W_k P_p K_p (towards the next element) and C_k = W_k P_m K_m (towards the previous one):
    // X[r][kf, w] = sum over the points pp on line kf of the face and over v of
    // W[r][pp, v] (1/|J|)(pp) g'(pp) K[kf][v][w]. B_k stays in LDS for the next step's update.
    for (int side = 1; side >= 0; --side) {
      if (side == 1 ? k + 1 >= a.K : k == 0) continue;
      const int fs = a.fside[side * ne + e];
      const double* Ks = sK[side];
      double* sX = side ? sH : sC;
      T* gX = static_cast<T*>(side ? a.B : a.C) + (size_t)e * NJ * N;
      for (int t = tid; t < N * NJ; t += NT) {
        const int j = t / N, r = t % N, kf = j / NV, w = j % NV;
        double s = 0.0;
        for (int m = 0; m < N1; ++m) {
          const int pp = face_line_point(fs, kf, m, N1);
          const double cm = sIJ[pp] * corr_deriv(o, fs, m);
#pragma unroll
          for (int v = 0; v < NV; ++v) s += sM[r * LD + scol[pp * NV + v]] * cm * Ks[(kf * NV + v) * NV + w];
        }
        sX[t] = s;
        gX[t] = (T)s;
      }
    }
    __syncthreads();
    if (k > 0 && k + 1 < a.K) {
      // M_k = E_{k+1} C_k and N_k = E_{k-1} B_k: the columns' traces on the faces shared with the
      // next and the previous element, in that element's flux-point order
      for (int side = 0; side < 2; ++side) {
        const int en = a.elems[(size_t)line * a.K + (side ? k - 1 : k + 1)];
        const int fn = a.fside[(side ? ne : 0) + en];            // the neighbour's face towards e
        const int fe = a.lv.nbf[fn * ne + en], on = a.lv.ori[fn * ne + en];
        const double* we = trace_weights(o, fe);
        const double* sX = side ? sH : sC;
        double* gX = (side ? a.N : a.M) + ((size_t)line * a.K + k) * NJ * NJ;
        for (int t = tid; t < NJ * NJ; t += NT) {
          const int jc = t / NJ, i = t % NJ, kf = i / NV, w = i % NV;
          const int kk = on ? N1 - 1 - kf : kf;
          double s = 0.0;
          for (int m = 0; m < N1; ++m) s += we[m] * sX[jc * N + face_line_point(fe, kk, m, N1) * NV + w];
          gX[t] = s;
        }
      }
    }
    __syncthreads();
  }
  if (bad) *flag = 1;
}

// Sixteen bytes of a column at a time: four FP32 or two FP64 rows per thread.
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

// part[g][r] = sum over the columns c = g, g + G, ... of X[c][r] x[c] for an NR x NC matrix stored
// column-major (a column's NR rows contiguous and 16-byte aligned); the caller sums over g < G.
template <int NR, int NC, class T, int NT>
struct ColMatvec {
  // at most 8 column groups on small blocks, so that a workgroup holds several elements (EPB)
  static constexpr int RV = Vec16<T>::n, RT = NR / RV, G0 = NT / RT, G1 = G0 < NC ? G0 : NC,
                       G = (NR <= 64 && G1 > 8) ? 8 : G1, TPE = RT * G, EPB = NT / TPE;
  static_assert(NR % RV == 0, "rows come in whole vectors");
  // lt: the thread's index among the TPE threads of its element
  __device__ static void run(const T* __restrict__ X, const double* x, double* part, int lt) {
    using V = typename Vec16<T>::type;
    const int rt = lt % RT, g = lt / RT;
    if (g >= G) return;
    double acc[RV];
#pragma unroll
    for (int i = 0; i < RV; ++i) acc[i] = 0.0;
#pragma unroll 4
    for (int c = g; c < NC; c += G) {
      V v = *reinterpret_cast<const V*>(X + (size_t)c * NR + rt * RV);
      T vv[RV];
      __builtin_memcpy(vv, &v, sizeof(V));
      const double xc = x[c];
#pragma unroll
      for (int i = 0; i < RV; ++i) acc[i] += (double)vv[i] * xc;
    }
#pragma unroll
    for (int i = 0; i < RV; ++i) part[g * NR + rt * RV + i] = acc[i];
  }
};

// The trace of an element's values x ([pp * NV + v]) on its face fe, at flux point kf of the
// neighbour across it (whose view of the face has orientation flag on), variable w.
template <int P>
__device__ __forceinline__ double face_trace(const Ops1D& o, int fe, int on, const double* x, int kf, int w) {
  constexpr int N1 = P + 1, NV = 4;
  const int kk = on ? N1 - 1 - kf : kf;
  const double* we = trace_weights(o, fe);
  double s = 0.0;
  for (int m = 0; m < N1; ++m) s += we[m] * x[face_line_point(fe, kk, m, N1) * NV + w];
  return s;
}

// The neighbour across element e's face towards side `side` of its line (-1 at a line end) and
// that neighbour's orientation flag for the shared face.
__device__ __forceinline__ int line_nbr(const LineArgs& a, int e, int side, int& fe, int& on) {
  const int ne = a.lv.ne;
  fe = a.fside[side * ne + e];
  if (fe < 0) return -1;
  const int en = a.lv.nbr[fe * ne + e];
  on = a.lv.ori[a.lv.nbf[fe * ne + e] * ne + en];
  return en;
}

// The substitution passes run EPB elements per workgroup (several on the small coarse-level blocks),
// TPE threads each; slot es of the workgroup holds element blockIdx.x * EPB + es.

// Substitution pass 1: z_k = W_k r_k, and u_k = E_{k+1} z_k, the trace of z_k on the face shared with
// the next element of the line in that element's flux-point order.
template <int P, class T>
__global__ void __launch_bounds__(256) k_line_zu(LineArgs a, const T* __restrict__ W, const double* __restrict__ r,
                                                 double* __restrict__ z, double* __restrict__ u) {
  using C = LineCfg<P>;
  constexpr int NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ, NT = C::NT;
  using MV = ColMatvec<N, N, T, NT>;
  constexpr int EPB = MV::EPB, TPE = MV::TPE;
  __shared__ double sx[EPB][N], sz[EPB][N];
  __shared__ double part[EPB][MV::G * N];
  const int ne = a.lv.ne, es = threadIdx.x / TPE, lt = threadIdx.x % TPE, e = blockIdx.x * EPB + es;
  const bool live = es < EPB && e < ne;
  if (live)
    for (int t = lt; t < N; t += TPE) sx[es][t] = r[((size_t)(t % NV) * NP + t / NV) * ne + e];
  __syncthreads();
  if (live) MV::run(W + (size_t)e * N * N, sx[es], part[es], lt);
  __syncthreads();
  if (live)
    for (int t = lt; t < N; t += TPE) {
      double v = 0.0;
#pragma unroll
      for (int g = 0; g < MV::G; ++g) v += part[es][g * N + t];
      sz[es][t] = v;
      z[(size_t)e * N + t] = v;
    }
  __syncthreads();
  int fe = -1, on = 0;
  if (live && line_nbr(a, e, 1, fe, on) >= 0)
    for (int t = lt; t < NJ; t += TPE)
      u[(size_t)a.pos[e] * NJ + t] = face_trace<P>(a.ops, fe, on, sz[es], t / NV, t % NV);
}

// Substitution pass 3: y_k = z_k - C_k t_k (in place of z), and v_k = E_{k-1} y_k, the trace of y_k on
// the face shared with the previous element in that element's order. A line's first element keeps
// y = z and needs no trace.
template <int P, class T>
__global__ void __launch_bounds__(256) k_line_yv(LineArgs a, double* __restrict__ z, const double* __restrict__ tt,
                                                 double* __restrict__ v) {
  using C = LineCfg<P>;
  constexpr int NV = C::NV, N = C::N, NJ = C::NJ, NT = C::NT;
  using MV = ColMatvec<N, NJ, T, NT>;
  constexpr int EPB = MV::EPB, TPE = MV::TPE;
  __shared__ double sx[EPB][NJ], sy[EPB][N];
  __shared__ double part[EPB][MV::G * N];
  const int es = threadIdx.x / TPE, lt = threadIdx.x % TPE, e = blockIdx.x * EPB + es;
  int fe = -1, on = 0;
  const bool live = es < EPB && e < a.lv.ne && line_nbr(a, e, 0, fe, on) >= 0;
  const size_t pe = live ? (size_t)a.pos[e] : 0;
  if (live)
    for (int t = lt; t < NJ; t += TPE) sx[es][t] = tt[pe * NJ + t];
  __syncthreads();
  if (live) MV::run(static_cast<const T*>(a.C) + (size_t)e * NJ * N, sx[es], part[es], lt);
  __syncthreads();
  if (live)
    for (int t = lt; t < N; t += TPE) {
      double y = z[(size_t)e * N + t];
#pragma unroll
      for (int g = 0; g < MV::G; ++g) y -= part[es][g * N + t];
      sy[es][t] = y;
      z[(size_t)e * N + t] = y;
    }
  __syncthreads();
  if (live)
    for (int t = lt; t < NJ; t += TPE) v[pe * NJ + t] = face_trace<P>(a.ops, fe, on, sy[es], t / NV, t % NV);
}

// Substitution pass 5: x_k = y_k - B_k s_k (y_k alone at a line's last element), q += alpha x_k.
template <int P, class T>
__global__ void __launch_bounds__(256) k_line_x(LineArgs a, const double* __restrict__ y, const double* __restrict__ ss,
                                                double* __restrict__ q, double alpha) {
  using C = LineCfg<P>;
  constexpr int NP = C::NP, NV = C::NV, N = C::N, NJ = C::NJ, NT = C::NT;
  using MV = ColMatvec<N, NJ, T, NT>;
  constexpr int EPB = MV::EPB, TPE = MV::TPE;
  __shared__ double sx[EPB][NJ];
  __shared__ double part[EPB][MV::G * N];
  const int ne = a.lv.ne, es = threadIdx.x / TPE, lt = threadIdx.x % TPE, e = blockIdx.x * EPB + es;
  const bool live = es < EPB && e < ne;
  const bool coupled = live && a.fside[ne + e] >= 0;
  if (coupled)
    for (int t = lt; t < NJ; t += TPE) sx[es][t] = ss[(size_t)a.pos[e] * NJ + t];
  __syncthreads();
  if (coupled) MV::run(static_cast<const T*>(a.B) + (size_t)e * NJ * N, sx[es], part[es], lt);
  __syncthreads();
  if (live)
    for (int t = lt; t < N; t += TPE) {
      double x = y[(size_t)e * N + t];
      if (coupled) {
#pragma unroll
        for (int g = 0; g < MV::G; ++g) x -= part[es][g * N + t];
      }
      q[((size_t)(t % NV) * NP + t / NV) * ne + e] += alpha * x;
    }
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Steps of the trace recursion staged in LDS at a time (two buffers of CH matrices, <= 112 KB).
template <int P>
struct RecChunk {
  static constexpr int NJ = 4 * (P + 1), MM = NJ * NJ, C0 = 112 * 1024 / (2 * MM * 8);
  static constexpr int CH = C0 < 64 ? C0 : 64;
};

// Substitution passes 2 and 4, one workgroup per line: the trace recursion
//   forward  t_0 = 0,     t_{k+1} = u_k - M_k t_k      (k = 0 .. K-2)
//   backward s_{K-1} = 0, s_{k-1} = v_k - N_k s_k      (k = K-1 .. 1)
// Matrices, vectors and results are stored by line position, so a chunk of steps is one contiguous
// range. The first wave runs the recursion, lane i holding entry i, from LDS; the other waves stage
// the next chunk meanwhile.
template <int P>
__global__ void __launch_bounds__(256) k_line_rec(LineArgs a, const double* __restrict__ Mat,
                                                  const double* __restrict__ vec, double* __restrict__ out,
                                                  int backward) {
  using C = LineCfg<P>;
  constexpr int NJ = C::NJ, NT = C::NT, CH = RecChunk<P>::CH, MM = NJ * NJ;
  static_assert(NJ <= 64 && NJ % 4 == 0, "one lane per trace entry, four partial sums");
  __shared__ double sMat[2][CH * MM];
  __shared__ double sVec[2][CH * NJ];
  const int line = blockIdx.x, tid = threadIdx.x, K = a.K;
  const size_t base = (size_t)line * K;
  const int nsteps = K - 1, nchunks = (nsteps + CH - 1) / CH;
  // chunk c: steps j0 .. j0 + ns - 1, whose source positions j (forward) or K-1-j (backward) form
  // the range lo .. lo + ns - 1
  auto stage = [&](int c, int b, int t0, int stride) {
    const int j0 = c * CH, ns = min(CH, nsteps - j0), lo = backward ? K - j0 - ns : j0;
    const double* gM = Mat + (base + lo) * MM;
    const double* gv = vec + (base + lo) * NJ;
#pragma unroll 8
    for (int t = t0; t < ns * MM; t += stride) sMat[b][t] = gM[t];
    for (int t = t0; t < ns * NJ; t += stride) sVec[b][t] = gv[t];
  };
  const int lane = tid, il = lane < NJ ? lane : NJ - 1;
  double cur = 0.0;
  if (tid < NJ) out[(base + (backward ? K - 1 : 0)) * NJ + tid] = 0.0;
  if (nchunks > 0) stage(0, 0, tid, NT);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int b = c & 1;
    if (tid >= 64) {
      if (c + 1 < nchunks) stage(c + 1, b ^ 1, tid - 64, NT - 64);
    } else {
      const int j0 = c * CH, ns = min(CH, nsteps - j0);
      for (int sidx = 0; sidx < ns; ++sidx) {
        const int off = backward ? ns - 1 - sidx : sidx;
        const double* Ms = sMat[b] + off * MM;
        double acc[4] = {sVec[b][off * NJ + il], 0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) acc[jj & 3] -= Ms[jj * NJ + il] * readlane_f64(cur, jj);
        cur = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        const int j = j0 + sidx, dst = backward ? K - 2 - j : j + 1;
        if (lane < NJ) out[(base + dst) * NJ + lane] = cur;
      }
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
  a.pos = lf.pos;
  a.K = lf.K;
  a.Kc = lf.Kc;
  a.C = lf.C;
  a.B = lf.B;
  a.M = lf.M;
  a.N = lf.N;
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

template <int P, class T>
hipError_t line_sweep_pt(const LineArgs& a, const LineFactors& lf, double* q, double alpha, hipStream_t st) {
  const int ne = a.lv.ne, NJ = LineCfg<P>::NJ, NT = LineCfg<P>::NT;
  double *u = lf.tr, *t = lf.tr + (size_t)ne * NJ, *v = lf.tr + (size_t)2 * ne * NJ, *s = lf.tr + (size_t)3 * ne * NJ;
  constexpr int N = LineCfg<P>::N, NJc = LineCfg<P>::NJ;
  constexpr int Ez = ColMatvec<N, N, T, 256>::EPB, Ec = ColMatvec<N, NJc, T, 256>::EPB;
  const int gz = (ne + Ez - 1) / Ez, gc = (ne + Ec - 1) / Ec;
  hipLaunchKernelGGL((k_line_zu<P, T>), dim3(gz), dim3(NT), 0, st, a, (const T*)lf.Winv, (const double*)lf.r, lf.z, u);
  hipLaunchKernelGGL(k_line_rec<P>, dim3(lf.n_lines), dim3(NT), 0, st, a, (const double*)lf.M, (const double*)u, t, 0);
  hipLaunchKernelGGL((k_line_yv<P, T>), dim3(gc), dim3(NT), 0, st, a, lf.z, (const double*)t, v);
  hipLaunchKernelGGL(k_line_rec<P>, dim3(lf.n_lines), dim3(NT), 0, st, a, (const double*)lf.N, (const double*)v, s, 1);
  hipLaunchKernelGGL((k_line_x<P, T>), dim3(gc), dim3(NT), 0, st, a, (const double*)lf.z, (const double*)s, q, alpha);
  return hipGetLastError();
}

template <int P>
hipError_t line_sweep_p(const LineArgs& a, const pmg_factors_s& fac, double* q, double alpha, hipStream_t st) {
  const LineFactors& lf = *fac.lines;
  if (fac.precision == 32) return line_sweep_pt<P, float>(a, lf, q, alpha, st);
  return line_sweep_pt<P, double>(a, lf, q, alpha, st);
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
