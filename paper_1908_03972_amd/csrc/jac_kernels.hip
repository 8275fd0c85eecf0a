// Element blocks of the pseudo-transient linearisation (eqs. (28)-(30)) and their inverses.
//
// One workgroup per element:
//   1. pointwise Jacobians of the transformed fluxes dF~/dq, dG~/dq (forward-mode duals, one
//      tangent per thread) and the diagonal term Gamma/dtau + c_mass M at every solution point;
//   2. the Jacobian of the common flux of eq. (21) with respect to the element's own trace at
//      every flux point, including the dependence of the mean state, eigenvalues and Gamma;
//   3. assembly of D_e = Gamma/dtau + c_mass M - dR_e/dq_e from the tensor-line structure: a
//      point couples only to points on its own xi- and eta-lines;
//   4. row equilibration by powers of two and in-place Gauss-Jordan inversion with partial
//      pivoting in FP64 LDS;
//   5. the inverse is written column-major per element ([c][e][r]) at the factor precision,
//      the layout the sweep kernel streams.
#include "internal.hpp"

namespace pmg {

struct JacArgs {
  LevelView lv;
  Ops1D ops;
  GasParams gas;
  const double* q;
  double inv_dtau;
  double c_mass;
  double* D_out;
  void* W;
  int precision;
  int* flag;
};

template <int P>
struct JCfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1;
  static constexpr int NV = 4;
  static constexpr int N = NV * NP;
  static constexpr int LD = N + 1;       // padded LDS row pitch
  static constexpr size_t lds_doubles() {
    return (size_t)N * LD + NV * NP + 3 * NP * 16 + 4 * N1 * 16 + 3 * N;
  }
  static constexpr size_t lds_bytes() { return lds_doubles() * 8 + (N + 4) * sizeof(int); }
};

template <int P>
__global__ void __launch_bounds__(256) k_jac(JacArgs a) {
  using C = JCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, LD = C::LD;
  extern __shared__ double smem[];
  double* sD = smem;                    // [N][LD]
  double* sq = sD + N * LD;             // [NV][NP]
  double* sAF = sq + NV * NP;           // [NP][NV][NV]  dF~/dq
  double* sAG = sAF + NP * 16;          // [NP][NV][NV]  dG~/dq
  double* sDg = sAG + NP * 16;          // [NP][NV][NV]  Gamma/dtau + c_mass M
  double* sB = sDg + NP * 16;           // [4][N1][NV][NV] dF^/dq_own
  double* scol = sB + 4 * N1 * 16;      // [N]
  double* srow = scol + N;              // [N]
  double* sscl = srow + N;              // [N]
  int* sperm = reinterpret_cast<int*>(sscl + N);  // [N]
  int* spiv = sperm + N;

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;

  for (int t = tid; t < NV * NP; t += blockDim.x) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  __syncthreads();

  // (1) pointwise flux Jacobians and the diagonal pseudo-time / mass term
  for (int t = tid; t < NP * NV; t += blockDim.x) {
    const int pp = t / NV, w = t % NV;
    Dual<1> qd[NV];
    double qv[NV];                       // absolute state: q_ref + stored offset
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qv[v] = a.lv.q_ref[v] + sq[v * NP + pp];
      qd[v] = dconst<1>(qv[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) qd[v].d[0] = (v == w) ? 1.0 : 0.0;   // seed without a dynamic index
    const size_t gp = (size_t)pp * ne + e;
    const double* m = a.lv.met;
    Dual<1> fs[NV], ft[NV], qc[NV];
    normal_flux2(qd, m[gp], m[sstride + gp], a.gas, fs);
    normal_flux2(qd, m[2 * sstride + gp], m[3 * sstride + gp], a.gas, ft);
    conservative2(qd, a.gas, qc);
    const State2<double> s = make_state(qv, a.gas);
    double ew[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ew[v] = (v == w) ? 1.0 : 0.0;
    double gcol[NV];
    gamma_mul(s, a.gas, ew, gcol);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      sAF[(pp * NV + v) * NV + w] = fs[v].d[0];
      sAG[(pp * NV + v) * NV + w] = ft[v].d[0];
      sDg[(pp * NV + v) * NV + w] = gcol[v] * a.inv_dtau + a.c_mass * qc[v].d[0];
    }
  }

  // (2) Jacobian of the common flux at every flux point w.r.t. the element's own trace
  for (int t = tid; t < 4 * N1 * NV; t += blockDim.x) {
    const int f = t / (N1 * NV), k = (t / NV) % N1, w = t % NV;
    const double* wt = (f == 0 || f == 2) ? o.lm : o.lp;
    double ownv[NV] = {0.0, 0.0, 0.0, 0.0};
    for (int mm = 0; mm < N1; ++mm) {
      const int pp = (f < 2) ? (mm + N1 * k) : (k + N1 * mm);
#pragma unroll
      for (int v = 0; v < NV; ++v) ownv[v] += wt[mm] * sq[v * NP + pp];
    }
    Dual<1> own[NV], out[NV];            // stored offsets; own seeded in component w
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v] = dconst<1>(ownv[v]);
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v].d[0] = (v == w) ? 1.0 : 0.0;
    const size_t fo = ((size_t)(f * N1 + k) * 3) * ne + e;
    const double nx = a.lv.fvec[fo], ny = a.lv.fvec[fo + ne], sm = a.lv.fvec[fo + 2 * ne];
    const int nb = a.lv.nbr[f * ne + e];
    if (nb >= 0) {
      const int nf = a.lv.nbf[f * ne + e];
      const int kk = a.lv.ori[f * ne + e] ? (N1 - 1 - k) : k;
      const double* wn = (nf == 0 || nf == 2) ? o.lm : o.lp;
      double ov[NV] = {0.0, 0.0, 0.0, 0.0};
      for (int mm = 0; mm < N1; ++mm) {
        const int pp = (nf < 2) ? (mm + N1 * kk) : (kk + N1 * mm);
#pragma unroll
        for (int v = 0; v < NV; ++v) ov[v] += wn[mm] * a.q[v * sstride + (size_t)pp * ne + nb];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = dconst<1>(ov[v]);
    } else if (nb == -1) {
      Dual<1> ua = own[1] + a.lv.q_ref[1], va = own[2] + a.lv.q_ref[2];
      Dual<1> un = ua * nx + va * ny;
      out[0] = own[0];
      out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
      out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
      out[3] = own[3];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = dconst<1>(a.lv.qinf_g[v]);
    }
    Dual<1> own_a[NV], out_a[NV], dq[NV], fh[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      own_a[v] = own[v] + a.lv.q_ref[v];
      out_a[v] = out[v] + a.lv.q_ref[v];
    }
    if (f == 0 || f == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
      common_flux2(out_a, own_a, dq, nx, ny, sm, a.gas, fh);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
      common_flux2(own_a, out_a, dq, nx, ny, sm, a.gas, fh);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sB[((f * N1 + k) * NV + v) * NV + w] = fh[v].d[0];
  }
  __syncthreads();

  // (3) assembly of D_e
  for (int idx = tid; idx < N * N; idx += blockDim.x) {
    const int r = idx / N, c = idx % N;
    const int pp = r / NV, v = r % NV, ss = c / NV, w = c % NV;
    const int i = pp % N1, j = pp / N1, k = ss % N1, l = ss / N1;
    double acc = 0.0;
    if (l == j) {   // xi-line of point (i, j)
      const double cx = o.D[i * N1 + k] - o.gL[i] * o.lm[k] - o.gR[i] * o.lp[k];
      acc += cx * sAF[(ss * NV + v) * NV + w] + o.gL[i] * o.lm[k] * sB[((0 * N1 + j) * NV + v) * NV + w] +
             o.gR[i] * o.lp[k] * sB[((1 * N1 + j) * NV + v) * NV + w];
    }
    if (k == i) {   // eta-line
      const double cy = o.D[j * N1 + l] - o.gL[j] * o.lm[l] - o.gR[j] * o.lp[l];
      acc += cy * sAG[(ss * NV + v) * NV + w] + o.gL[j] * o.lm[l] * sB[((2 * N1 + i) * NV + v) * NV + w] +
             o.gR[j] * o.lp[l] * sB[((3 * N1 + i) * NV + v) * NV + w];
    }
    const double ijac = a.lv.met[4 * sstride + (size_t)pp * ne + e];
    double dval = acc * ijac;             // -dR/dq, with R = -(1/|J|) div
    if (pp == ss) dval += sDg[(pp * NV + v) * NV + w];
    sD[r * LD + c] = dval;
    if (a.D_out) a.D_out[((size_t)e * N + r) * N + c] = dval;
  }
  __syncthreads();

  // (4) row equilibration by powers of two, then Gauss-Jordan with partial pivoting
  for (int r = tid; r < N; r += blockDim.x) {
    double mx = 0.0;
    for (int c = 0; c < N; ++c) mx = fmax(mx, fabs(sD[r * LD + c]));
    int ex = 0;
    frexp(mx, &ex);
    sscl[r] = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ex) : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < N * N; idx += blockDim.x) {
    const int r = idx / N, c = idx % N;
    sD[r * LD + c] *= sscl[r];
  }
  __syncthreads();

  for (int kk = 0; kk < N; ++kk) {
    if (tid < 64) {
      double best = -1.0;
      int bi = kk;
      for (int r = kk + tid; r < N; r += 64) {
        const double av = fabs(sD[r * LD + kk]);
        if (av > best) {
          best = av;
          bi = r;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        spiv[0] = bi;
        sperm[kk] = bi;
      }
    }
    __syncthreads();
    const int pr = spiv[0];
    if (pr != kk) {
      for (int c = tid; c < N; c += blockDim.x) {
        const double tmp = sD[kk * LD + c];
        sD[kk * LD + c] = sD[pr * LD + c];
        sD[pr * LD + c] = tmp;
      }
    }
    __syncthreads();
    for (int t = tid; t < N; t += blockDim.x) {
      scol[t] = sD[t * LD + kk];
      srow[t] = sD[kk * LD + t];
    }
    __syncthreads();
    double piv = scol[kk];
    if (piv == 0.0 || !isfinite(piv)) {
      if (tid == 0) *a.flag = 1;
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
    for (int idx = tid; idx < N * N; idx += blockDim.x) {
      const int r = idx / N, c = idx % N;
      double nv;
      if (r == kk)
        nv = (c == kk) ? ip : srow[c] * ip;
      else if (c == kk)
        nv = -scol[r] * ip;
      else
        nv = sD[r * LD + c] - scol[r] * (srow[c] * ip);
      sD[r * LD + c] = nv;
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int kk = N - 1; kk >= 0; --kk) {
    const int pr = sperm[kk];
    if (pr != kk) {
      for (int r = tid; r < N; r += blockDim.x) {
        const double tmp = sD[r * LD + kk];
        sD[r * LD + kk] = sD[r * LD + pr];
        sD[r * LD + pr] = tmp;
      }
    }
    __syncthreads();
  }

  // (5) D^{-1} = (S_r D)^{-1} S_r: scale column c by the row scale of row c; store [c][e][r]
  for (int idx = tid; idx < N * N; idx += blockDim.x) {
    const int c = idx / N, r = idx % N;
    const double val = sD[r * LD + c] * sscl[c];
    const size_t o_ = ((size_t)c * ne + e) * N + r;
    if (a.precision == 32)
      static_cast<float*>(a.W)[o_] = (float)val;
    else
      static_cast<double*>(a.W)[o_] = val;
  }
}

// Broadcast a double from a wave-uniform lane (two 32-bit lane reads into scalar registers).
__device__ __forceinline__ double read_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Same blocks for n = 4 (P+1)^2 <= 64 with one wavefront per element: lane r builds row r of
// D_e in registers and the Gauss-Jordan elimination runs with implicit partial pivoting (the
// pivot row is chosen among rows not yet used and broadcast by lane reads, no row swaps and no
// workgroup barriers); the inverse comes out with rows and columns permuted by the pivot order,
// which the final store undoes.
template <int P>
__global__ void __launch_bounds__(64) k_jac_wave(JacArgs a) {
  constexpr int N1 = P + 1, NP = N1 * N1, NV = 4, N = NV * NP;
  static_assert(N <= 64, "one row per lane");
  __shared__ double sq[NV * NP];
  __shared__ double sAF[NP * 16], sAG[NP * 16], sDg[NP * 16];
  __shared__ double sB[4 * N1 * 16];
  __shared__ double sscl[64];
  __shared__ int sperm[64];

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int lane = threadIdx.x;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;

  for (int t = lane; t < NV * NP; t += 64) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  __syncthreads();

  for (int t = lane; t < NP * NV; t += 64) {     // pointwise flux Jacobians and diagonal term
    const int pp = t / NV, w = t % NV;
    Dual<1> qd[NV];
    double qv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qv[v] = a.lv.q_ref[v] + sq[v * NP + pp];
      qd[v] = dconst<1>(qv[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) qd[v].d[0] = (v == w) ? 1.0 : 0.0;   // seed without a dynamic index
    const size_t gp = (size_t)pp * ne + e;
    const double* m = a.lv.met;
    Dual<1> fs[NV], ft[NV], qc[NV];
    normal_flux2(qd, m[gp], m[sstride + gp], a.gas, fs);
    normal_flux2(qd, m[2 * sstride + gp], m[3 * sstride + gp], a.gas, ft);
    conservative2(qd, a.gas, qc);
    const State2<double> s = make_state(qv, a.gas);
    double ew[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ew[v] = (v == w) ? 1.0 : 0.0;
    double gcol[NV];
    gamma_mul(s, a.gas, ew, gcol);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      sAF[(pp * NV + v) * NV + w] = fs[v].d[0];
      sAG[(pp * NV + v) * NV + w] = ft[v].d[0];
      sDg[(pp * NV + v) * NV + w] = gcol[v] * a.inv_dtau + a.c_mass * qc[v].d[0];
    }
  }
  for (int t = lane; t < 4 * N1 * NV; t += 64) {  // common-flux Jacobians w.r.t. the own trace
    const int f = t / (N1 * NV), k = (t / NV) % N1, w = t % NV;
    const double* wt = (f == 0 || f == 2) ? o.lm : o.lp;
    double ownv[NV] = {0.0, 0.0, 0.0, 0.0};
    for (int mm = 0; mm < N1; ++mm) {
      const int pp = (f < 2) ? (mm + N1 * k) : (k + N1 * mm);
#pragma unroll
      for (int v = 0; v < NV; ++v) ownv[v] += wt[mm] * sq[v * NP + pp];
    }
    Dual<1> own[NV], out[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v] = dconst<1>(ownv[v]);
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v].d[0] = (v == w) ? 1.0 : 0.0;
    const size_t fo = ((size_t)(f * N1 + k) * 3) * ne + e;
    const double nx = a.lv.fvec[fo], ny = a.lv.fvec[fo + ne], sm = a.lv.fvec[fo + 2 * ne];
    const int nb = a.lv.nbr[f * ne + e];
    if (nb >= 0) {
      const int nf = a.lv.nbf[f * ne + e];
      const int kk = a.lv.ori[f * ne + e] ? (N1 - 1 - k) : k;
      const double* wn = (nf == 0 || nf == 2) ? o.lm : o.lp;
      double ov[NV] = {0.0, 0.0, 0.0, 0.0};
      for (int mm = 0; mm < N1; ++mm) {
        const int pp = (nf < 2) ? (mm + N1 * kk) : (kk + N1 * mm);
#pragma unroll
        for (int v = 0; v < NV; ++v) ov[v] += wn[mm] * a.q[v * sstride + (size_t)pp * ne + nb];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = dconst<1>(ov[v]);
    } else if (nb == -1) {
      Dual<1> ua = own[1] + a.lv.q_ref[1], va = own[2] + a.lv.q_ref[2];
      Dual<1> un = ua * nx + va * ny;
      out[0] = own[0];
      out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
      out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
      out[3] = own[3];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = dconst<1>(a.lv.qinf_g[v]);
    }
    Dual<1> own_a[NV], out_a[NV], dq[NV], fh[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      own_a[v] = own[v] + a.lv.q_ref[v];
      out_a[v] = out[v] + a.lv.q_ref[v];
    }
    if (f == 0 || f == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
      common_flux2(out_a, own_a, dq, nx, ny, sm, a.gas, fh);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
      common_flux2(own_a, out_a, dq, nx, ny, sm, a.gas, fh);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sB[((f * N1 + k) * NV + v) * NV + w] = fh[v].d[0];
  }
  __syncthreads();

  // row r = lane of D_e (rows beyond n stay zero)
  const bool has_row = lane < N;
  const int r = has_row ? lane : 0;
  const int pp = r / NV, v = r % NV, i = pp % N1, jj = pp / N1;
  const double ijac = a.lv.met[4 * sstride + (size_t)pp * ne + e];
  double row[N];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const int ss = c / NV, w = c % NV, k = ss % N1, l = ss / N1;
    double acc = 0.0;
    if (l == jj) {
      const double cx = o.D[i * N1 + k] - o.gL[i] * o.lm[k] - o.gR[i] * o.lp[k];
      acc += cx * sAF[(ss * NV + v) * NV + w] + o.gL[i] * o.lm[k] * sB[((0 * N1 + jj) * NV + v) * NV + w] +
             o.gR[i] * o.lp[k] * sB[((1 * N1 + jj) * NV + v) * NV + w];
    }
    if (k == i) {
      const double cy = o.D[jj * N1 + l] - o.gL[jj] * o.lm[l] - o.gR[jj] * o.lp[l];
      acc += cy * sAG[(ss * NV + v) * NV + w] + o.gL[jj] * o.lm[l] * sB[((2 * N1 + i) * NV + v) * NV + w] +
             o.gR[jj] * o.lp[l] * sB[((3 * N1 + i) * NV + v) * NV + w];
    }
    double dval = acc * ijac;
    if (pp == ss) dval += sDg[(pp * NV + v) * NV + w];
    row[c] = has_row ? dval : 0.0;
  }
  if (a.D_out && has_row) {
#pragma unroll
    for (int c = 0; c < N; ++c) a.D_out[((size_t)e * N + r) * N + c] = row[c];
  }
  // row equilibration by a power of two
  double mx = 0.0;
#pragma unroll
  for (int c = 0; c < N; ++c) mx = fmax(mx, fabs(row[c]));
  int ex = 0;
  frexp(mx, &ex);
  const double scl = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ex) : 1.0;
#pragma unroll
  for (int c = 0; c < N; ++c) row[c] *= scl;
  sscl[lane] = scl;

  bool used = !has_row;
  int my_step = 0;
  bool bad = false;
  for (int k = 0; k < N; ++k) {
    double f = 0.0;                      // this row's entry in column k
#pragma unroll
    for (int c = 0; c < N; ++c) f = (c == k) ? row[c] : f;
    double best = used ? -1.0 : fabs(f);
    int bi = lane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    const int p = __builtin_amdgcn_readfirstlane(bi);
    double piv = read_lane(f, p);
    if (piv == 0.0 || !isfinite(piv)) {
      bad = true;
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
    const bool is_p = (lane == p);
    if (is_p) {
      used = true;
      my_step = k;
    }
    if (lane == 0) sperm[k] = p;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double pc = read_lane(row[c], p);
      double nv;
      if (is_p)
        nv = (c == k) ? ip : pc * ip;
      else
        nv = (c == k) ? -f * ip : row[c] - f * (pc * ip);
      row[c] = nv;
    }
  }
  if (bad && lane == 0) *a.flag = 1;
  __syncthreads();
  // lane L (pivot of step k_L) holds B[L][j] = (S_r D)^{-1}[k_L][perm[j]]; D^{-1} = (S_r D)^{-1} S_r
  if (has_row) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const int col = sperm[c];
      const double val = row[c] * sscl[col];
      const size_t o_ = ((size_t)col * ne + e) * N + my_step;
      if (a.precision == 32)
        static_cast<float*>(a.W)[o_] = (float)val;
      else
        static_cast<double*>(a.W)[o_] = val;
    }
  }
}

template <int P>
static hipError_t launch_jac_p(const JacArgs& a, int ne, hipStream_t st) {
  const size_t bytes = JCfg<P>::lds_bytes();
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jac<P>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_jac<P>), dim3(ne), dim3(256), bytes, st, a);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_jac_wave(const JacArgs& a, int ne, hipStream_t st) {
  hipLaunchKernelGGL((k_jac_wave<P>), dim3(ne), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_jacobian(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                           pmg_factors_s& fac, hipStream_t st) {
  JacArgs a{};
  a.lv = L.view();
  a.ops = L.ops;
  a.gas = L.gas;
  a.q = q;
  a.inv_dtau = 1.0 / dtau;
  a.c_mass = c_mass;
  a.D_out = D_out;
  a.W = fac.W;
  a.precision = fac.precision;
  a.flag = L.flag;
  switch (L.P) {
    case 0: return launch_jac_wave<0>(a, L.ne, st);
    case 1: return launch_jac_wave<1>(a, L.ne, st);
    case 2: return launch_jac_wave<2>(a, L.ne, st);
    case 3: return launch_jac_wave<3>(a, L.ne, st);
    case 4: return launch_jac_p<4>(a, L.ne, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmg
