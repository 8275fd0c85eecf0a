// Element blocks of the pseudo-transient linearisation (eqs. (28)-(30)) and their inverses.
//
// One workgroup of ceil(n / 64) wavefronts per element:
//   1. pointwise Jacobians of the transformed fluxes dF~/dq, dG~/dq (forward-mode duals, one
//      tangent per thread) and the diagonal term Gamma/dtau + c_mass M at every solution point;
//   2. the Jacobian of the common flux of eq. (21) with respect to the element's own trace at
//      every flux point, including the dependence of the mean state, eigenvalues and Gamma;
//   3. assembly of D_e = Gamma/dtau + c_mass M - dR_e/dq_e from the tensor-line structure (a
//      point couples only to points on its own xi- and eta-lines), one row per thread in
//      registers;
//   4. row equilibration by powers of two and Gauss-Jordan inversion in FP64 registers with
//      partial pivoting;
//   5. the inverse is written column-major per element ([c][e][r]) at the factor precision,
//      the layout the sweep kernel streams.
#include "internal.hpp"
#include "wave_ops.hpp"

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
  const double* Dv;     // [Ne][n][n] viscous part dR_vis/dq, or null
};

// Pointwise task t = pp * NV + w: column w of the flux Jacobians dF~/dq, dG~/dq at solution point
// pp (forward-mode duals seeded in component w) and of the diagonal term Gamma/dtau + c_mass M.
__device__ __forceinline__ void point_jacobian(const JacArgs& a, int e, const double* sq, int t, int NP, int ne,
                                               size_t sstride, double* sAF, double* sAG, double* sDg) {
  constexpr int NV = 4;
  const int pp = t / NV, w = t % NV;
  Dual<1> qd[NV];
  double qv[NV];                         // absolute state: q_ref + stored offset
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

// Face task t = (f * N1 + k) * NV + w: column w of the Jacobian of the common flux of eq. (21) at
// flux point k of face f with respect to the element's own trace (neighbour trace fixed; wall ghost
// and far-field state as in the residual), including the dependence of the mean state.
__device__ __forceinline__ void face_jacobian(const JacArgs& a, int e, const double* sq, int t, int N1, int NP,
                                              int ne, size_t sstride, double* sB) {
  constexpr int NV = 4;
  const Ops1D& o = a.ops;
  const int f = t / (N1 * NV), k = (t / NV) % N1, w = t % NV;
  const double* wt = (f == 0 || f == 2) ? o.lm : o.lp;
  double ownv[NV] = {0.0, 0.0, 0.0, 0.0};
  for (int mm = 0; mm < N1; ++mm) {
    const int pp = (f < 2) ? (mm + N1 * k) : (k + N1 * mm);
#pragma unroll
    for (int v = 0; v < NV; ++v) ownv[v] += wt[mm] * sq[v * NP + pp];
  }
  Dual<1> own[NV], out[NV];              // stored offsets; own seeded in component w
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
  } else if (nb == -1) {                 // slip wall: mirrored absolute velocity
    Dual<1> ua = own[1] + a.lv.q_ref[1], va = own[2] + a.lv.q_ref[2];
    Dual<1> un = ua * nx + va * ny;
    out[0] = own[0];
    out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
    out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
    out[3] = own[3];
  } else if (nb == -3) {                 // no-slip wall: reversed absolute velocity
    out[0] = own[0];
    out[1] = -(own[1] + a.lv.q_ref[1]) - a.lv.q_ref[1];
    out[2] = -(own[2] + a.lv.q_ref[2]) - a.lv.q_ref[2];
    out[3] = own[3];
  } else {                               // far field
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

// Same blocks for any P <= 5 with each row of D_e held in registers by S threads (S = 1; 2 for
// n = 100, thread 2r holding columns [0, n/2) of row r and thread 2r+1 columns [n/2, n); 4 for
// n = 144, a quarter of the row each), in ceil(S n / 64) wavefronts per element. The elimination is Gauss-Jordan with implicit partial
// pivoting (the pivot row is chosen among rows not yet used; no rows move) in the
// column-cycling form: step k always eliminates with the first stored column, every row shifts
// left by one and the new column of the inverse enters at the right end, so that after n steps
// the stored array is the in-place inverse and no register array is ever indexed by a run-time
// value. Each wavefront's pivot candidate publishes its row to LDS before the cross-wave choice,
// so one barrier per step suffices (two slot sets alternate between steps).
template <int P, int S>
struct RowsCfg {
  static constexpr int N1 = P + 1, NP = N1 * N1, NV = 4, N = NV * NP;
  static constexpr int H = N / S;                 // columns per thread
  static constexpr int NW = (S * N + 63) / 64;
  static constexpr int NT = 64 * NW;
  static_assert(N % S == 0 && (S == 1 || S == 2 || S == 4), "one, two or four threads per row");
  static_assert(S * N <= 1023, "pivot keys carry the thread index in 10 bits");
  // DPP quad permutations: every lane of a row's group takes the group's first lane (the row's
  // entry in the current column), or the next lane of the group (its first stored column)
  static constexpr int kFirst = S == 2 ? 0xA0 : 0x00;   // [0,0,2,2] or [0,0,0,0]
  static constexpr int kNext = S == 2 ? 0xF5 : 0xF9;    // [1,1,3,3] or [1,2,3,3]
};


// A double from another lane of the same quad, selected by a DPP quad permutation.
template <int CTRL>
__device__ __forceinline__ double pair_dpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int P, int S>
__global__ void __launch_bounds__((RowsCfg<P, S>::NT)) k_jac_rows(JacArgs a) {
  using C = RowsCfg<P, S>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, H = C::H, NW = C::NW, NT = C::NT;
  __shared__ double sq[NV * NP];
  __shared__ double sAF[NP * 16], sAG[NP * 16], sDg[NP * 16];
  __shared__ double sB[4 * N1 * 16];
  __shared__ double sscl[N];
  __shared__ int sperm[N];
  __shared__ double slot[2][NW][N];      // pivot candidates' rows, alternating between steps
  __shared__ unsigned skey[2][NW];

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;

  for (int t = tid; t < NV * NP; t += NT) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  __syncthreads();
  for (int t = tid; t < NP * NV; t += NT) point_jacobian(a, e, sq, t, NP, ne, sstride, sAF, sAG, sDg);
  for (int t = tid; t < 4 * N1 * NV; t += NT) face_jacobian(a, e, sq, t, N1, NP, ne, sstride, sB);
  __syncthreads();

  const bool has_row = tid < S * N;
  const int r = has_row ? tid / S : 0;
  const int h = (S > 1) ? (tid % S) : 0;          // which part of the row this thread holds
  const int pp = r / NV, v = r % NV, i = pp % N1, jj = pp / N1;
  const double ijac = a.lv.met[4 * sstride + (size_t)pp * ne + e];
  double row[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int c = h * H + j;
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
    if (a.Dv && has_row) dval -= a.Dv[((size_t)e * N + r) * N + c];
    row[j] = has_row ? dval : 0.0;
  }
  if (a.D_out && has_row) {
#pragma unroll
    for (int j = 0; j < H; ++j) a.D_out[((size_t)e * N + r) * N + h * H + j] = row[j];
  }
  if (!a.W) return;                       // blocks only (the line smoother factors them itself)
  double mx = 0.0;                        // row equilibration by a power of two
#pragma unroll
  for (int j = 0; j < H; ++j) mx = fmax(mx, fabs(row[j]));
  if (S >= 2) mx = fmax(mx, __shfl_xor(mx, 1, 64));
  if (S == 4) mx = fmax(mx, __shfl_xor(mx, 2, 64));
  int ex = 0;
  frexp(mx, &ex);
  const double scl = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ex) : 1.0;
#pragma unroll
  for (int j = 0; j < H; ++j) row[j] *= scl;
  if (has_row && h == 0) sscl[r] = scl;

  // Pivot rows are left unnormalised: a row keeps its scale d = pivot from the step it served
  // as pivot (it is never a pivot again), every later update of it is the same formula as for
  // any other row, and the scale is divided out once at the end. All threads therefore run one
  // fused multiply-add per column per step with no divergent branch.
  //
  // Pivot choice: a 32-bit key per row (on the thread holding its first column), the upper word
  // of |f| (sign 0, exponent, 20 mantissa bits) with its low 10 bits replaced by 1023 - thread,
  // and 0 for rows already used; the largest key wins. The pivot is therefore within a factor
  // 1 + 2^-10 of the largest candidate, and ties go to the lowest row.
  bool used = !has_row;
  int my_step = 0;
  double my_inv = 1.0;
  bool bad = false;
  for (int k = 0; k < N; ++k) {
    const int par = k & 1;
    const double f = (S > 1) ? pair_dpp<C::kFirst>(row[0]) : row[0];   // this row's entry in column k
    const unsigned key = (used || h != 0) ? 0u
                         : ((((unsigned)__double2hiint(fabs(f))) & ~0x3FFu) | (unsigned)(1023 - tid));
    const unsigned wkey = wave_max_u32(key);
    const int wtid = 1023 - (int)(wkey & 0x3FFu);
    if (wkey != 0u && tid >= wtid && tid < wtid + S) {   // publish the candidate row
#pragma unroll
      for (int j = 0; j < H; ++j) slot[par][wv][h * H + j] = row[j];
    }
    if (lane == 0) skey[par][wv] = wkey;
    __syncthreads();
    int win = 0;
    unsigned bk = skey[par][0];
#pragma unroll
    for (int w2 = 1; w2 < NW; ++w2) {
      const unsigned k2 = skey[par][w2];
      win = (k2 > bk) ? w2 : win;
      bk = (k2 > bk) ? k2 : bk;
    }
    int p = (1023 - (int)(bk & 0x3FFu)) / S;
    if (bk == 0u || p >= N) {             // no unused row left: only reachable with non-finite entries
      bad = true;
      p = (p < N && p >= 0) ? p : N - 1;
    }
    const double* pr = slot[par][win];
    double piv = pr[0];
    if (piv == 0.0 || !isfinite(piv)) {
      bad = true;
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
    const bool is_p = has_row && (r == p);
    if (tid == 0) sperm[k] = p;
    const double g = is_p ? 0.0 : f * ip;
    if (is_p) {
      used = true;
      my_step = k;
      my_inv = ip;
    }
    const double nb = (S > 1) ? pair_dpp<C::kNext>(row[0]) : 0.0;   // first column of the next part
    const double* prh = pr + h * H;
    // pivot-row values in batches, so that a batch of LDS reads is in flight at once
    constexpr int B = 16;
#pragma unroll
    for (int j0 = 0; j0 < H - 1; j0 += B) {
      double buf[B];
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j0 + j < H - 1) buf[j] = prh[j0 + j + 1];
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (j0 + j < H - 1) row[j0 + j] = fma(-g, buf[j], row[j0 + j + 1]);
    }
    if (S > 1 && h < S - 1)
      row[H - 1] = fma(-g, pr[(h + 1) * H], nb);
    else
      row[H - 1] = is_p ? 1.0 : -g;
  }
  if (bad) *a.flag = 1;
  __syncthreads();
  // row r (pivot of step k_r, scale 1/my_inv) holds B[r][c] = (S_r D)^{-1}[k_r][perm[c]] / my_inv;
  // D^{-1} = (S_r D)^{-1} S_r
  if (has_row) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int col = sperm[h * H + j];
      const double val = row[j] * my_inv * sscl[col];
      const size_t o_ = ((size_t)col * ne + e) * N + my_step;
      if (a.precision == 32)
        static_cast<float*>(a.W)[o_] = (float)val;
      else
        static_cast<double*>(a.W)[o_] = val;
    }
  }
}

template <int P, int S>
static hipError_t launch_jac_rows(const JacArgs& a, int ne, hipStream_t st) {
  hipLaunchKernelGGL((k_jac_rows<P, S>), dim3(ne), dim3(RowsCfg<P, S>::NT), 0, st, a);
  return hipGetLastError();
}

// Blocks with FP32 inverses at P = 4 (n = 100 padded to NR = 112 with identity rows and columns)
// held in LDS and inverted in FP32 by the panel Gauss-Jordan of the hexahedral kernels: panels of
// 16 columns whose steps run on the rows' panel entries in registers (one thread per row, column
// cycling, unnormalised pivot rows, the row's power-of-two equilibration in the pivot keys), then
// the rank-16 update of every other column on the FP32 matrix cores, accumulators and operands in
// LDS. The pointwise derivatives are computed as in k_jac_rows; viscous blocks subtract Dv.
template <int P>
struct LdsCfg {
  static constexpr int N1 = P + 1, NP = N1 * N1, NV = 4, N = NV * NP;
  static constexpr int NR = (N + 15) / 16 * 16, XS = NR + 4, B = 16, NW = 2, NT = 64 * NW;
  static constexpr int TILES = NR / 16, TPW = (TILES + NW - 1) / NW;
  static_assert(NR <= NT, "one thread per row");
};

template <int P>
__global__ void __launch_bounds__(LdsCfg<P>::NT) k_jac_lds(JacArgs a) {
  using C = LdsCfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, NR = C::NR, XS = C::XS, B = C::B, NW = C::NW,
                NT = C::NT, TILES = C::TILES, TPW = C::TPW;
  __shared__ float X[NR * XS];
  __shared__ float xp[B * XS];
  __shared__ double sq[NV * NP];
  __shared__ double sAF[NP * 16], sAG[NP * 16], sDg[NP * 16];
  __shared__ double sB[4 * N1 * 16];
  __shared__ float slot[2][NW][B];
  __shared__ int sperm[NR];
  __shared__ float sinv[NR];
  __shared__ unsigned skey[2][NW];

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int r = threadIdx.x;
  const int lane = r & 63, wv = r >> 6;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;

  for (int t = r; t < NV * NP; t += NT) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  for (int t = r; t < NR * XS; t += NT) X[t] = 0.f;
  __syncthreads();
  for (int t = r; t < NP * NV; t += NT) point_jacobian(a, e, sq, t, NP, ne, sstride, sAF, sAG, sDg);
  for (int t = r; t < 4 * N1 * NV; t += NT) face_jacobian(a, e, sq, t, N1, NP, ne, sstride, sB);
  __syncthreads();

  // row r of D_e (every column: viscous blocks couple beyond the two tensor lines), rounded to
  // FP32; its largest entry sets the power-of-two scale of the pivot keys. Padding rows: identity
  int e2 = 0;
  if (r < N) {
    const int pp = r / NV, v = r % NV, i = pp % N1, jj = pp / N1;
    const double ijac = a.lv.met[4 * sstride + (size_t)pp * ne + e];
    double mx = 0.0;
#pragma unroll 1
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
      if (a.Dv) dval -= a.Dv[((size_t)e * N + r) * N + c];
      if (a.D_out) a.D_out[((size_t)e * N + r) * N + c] = dval;
      mx = fmax(mx, fabs(dval));
      X[r * XS + c] = (float)dval;
    }
    int ex = 0;
    frexp(mx, &ex);
    e2 = (mx > 0.0 && isfinite(mx)) ? -ex : 0;
  } else if (r < NR) {
    X[r * XS + r] = 1.f;
  }
  __syncthreads();

  bool used = r >= NR;
  bool bad = false;
  const int lr = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < NR; k0 += B) {
    float row[B];
#pragma unroll
    for (int j = 0; j < B; ++j) row[j] = (r < NR) ? X[r * XS + k0 + j] : 0.f;
#pragma unroll 1
    for (int j = 0; j < B; ++j) {
      const int par = j & 1;
      const float fv = row[0];
      const unsigned key = used ? 0u : pivot_key(fv, r, e2);
      const unsigned wkey = wave_max_u32(key);
      if (wkey != 0u && r == 1023 - (int)(wkey & 0x3FFu)) {   // the row shifted by one, pivot last
#pragma unroll
        for (int c = 0; c < B - 1; ++c) slot[par][wv][c] = row[c + 1];
        slot[par][wv][B - 1] = row[0];
      }
      if (lane == 0) skey[par][wv] = wkey;
      __syncthreads();
      int win = 0;
      unsigned bk = skey[par][0];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) {
        const unsigned k2 = skey[par][w2];
        win = (k2 > bk) ? w2 : win;
        bk = (k2 > bk) ? k2 : bk;
      }
      int pr = 1023 - (int)(bk & 0x3FFu);
      if (bk == 0u || pr >= NR) {
        bad = true;
        pr = 0;
      }
      const float* prw = slot[par][win];
      float piv = prw[B - 1];
      if (piv == 0.f || !isfinite(piv)) {
        bad = true;
        piv = 1.f;
      }
      const float ip = 1.f / piv;
      const bool is_p = (r == pr);
      if (r == 0) sperm[k0 + j] = pr;
      if (is_p) {
        used = true;
        sinv[k0 + j] = ip;
      }
      const float g = is_p ? 0.f : fv * ip;
#pragma unroll
      for (int c = 0; c < B - 1; ++c) row[c] = fmaf(-g, prw[c], row[c + 1]);
      row[B - 1] = is_p ? 1.f : -g;
    }
    if (r < NR) {
#pragma unroll
      for (int j = 0; j < B; ++j) X[r * XS + k0 + j] = row[j];
    }
    __syncthreads();                      // the panel and sperm are complete
    for (int t = r; t < B * NR; t += NT) {
      const int k = t / NR, c = t % NR;
      xp[k * XS + c] = X[sperm[k0 + k] * XS + c];
    }
    float uop[TPW][B / 4];
#pragma unroll
    for (int TT = 0; TT < TPW; ++TT) {
      const int tile = TPW * wv + TT;
#pragma unroll
      for (int s4 = 0; s4 < B / 4; ++s4) {
        const int row_ = 16 * tile + lr, m = k0 + 4 * s4 + lk;
        const float u = tile < TILES ? X[row_ * XS + m] : 0.f;
        uop[TT][s4] = (tile < TILES && sperm[m] == row_) ? u - 1.f : u;
      }
    }
    __syncthreads();                      // xp complete, every panel value read
#pragma unroll 1
    for (int cg = 0; cg < NR; cg += 16) {
      if (cg == k0) continue;             // B == 16: the panel is one column group
      flt4 acc[TPW];
#pragma unroll
      for (int TT = 0; TT < TPW; ++TT) {
        const int tile = TPW * wv + TT;
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2)
          acc[TT][v2] = tile < TILES ? X[(16 * tile + 4 * lk + v2) * XS + cg + lr] : 0.f;
      }
#pragma unroll
      for (int s4 = 0; s4 < B / 4; ++s4) {
        const float xb = xp[(4 * s4 + lk) * XS + cg + lr];
#pragma unroll
        for (int TT = 0; TT < TPW; ++TT) acc[TT] = mfma16x16x4(uop[TT][s4], xb, acc[TT]);
      }
#pragma unroll
      for (int TT = 0; TT < TPW; ++TT) {
        const int tile = TPW * wv + TT;
        if (tile < TILES) {
#pragma unroll
          for (int v2 = 0; v2 < 4; ++v2) X[(16 * tile + 4 * lk + v2) * XS + cg + lr] = acc[TT][v2];
        }
      }
    }
    __syncthreads();                      // the updated columns are visible before the next panel
  }
  if (bad) *a.flag = 1;
  // row r of the inverse: slot row sperm[r] over its pivot, columns in pivot order
  if (r < N) {
    const int prow = sperm[r];
    const float pinv = sinv[r];
#pragma unroll 4
    for (int m = 0; m < N; ++m) {
      const int col = sperm[m];
      if (col >= N) continue;             // only a singular block (flagged) pivots on a padding row
      static_cast<float*>(a.W)[((size_t)col * ne + e) * N + r] = X[prow * XS + m] * pinv;
    }
  }
}

// Viscous part of the element blocks, dR_vis,e/dq_e (BR2, Sec. 2.3), by forward-mode duals: one
// workgroup per element, K columns of the block per pass. Each pass seeds K unknowns of the
// element, evaluates the element's viscous residual with the neighbours' states and gradient
// traces held fixed (as the inviscid blocks do), and writes the K tangent columns to Dv.
template <int P, int K>
__global__ void __launch_bounds__(64) k_visc_jac(JacArgs a, double* __restrict__ Dv) {
  constexpr int N1 = P + 1, NP = N1 * N1, NV = 4, N = NV * NP, NF = 4 * N1, KD = K + 1;
  static_assert(NP <= 64 && NF <= 64, "one point or face task per thread");
  using T = Dual<K>;
  __shared__ double sq[NV * NP];
  __shared__ double sgl[NV * 2 * NP * KD];      // local gradients
  __shared__ double sjn[NF * NV * 2 * KD];      // (q_com - q) N per flux point
  __shared__ double sfh[NF * NV * KD];          // common viscous flux N . f_vis
  __shared__ double sfv[NV * NP * KD];          // F~v
  __shared__ double sgv[NV * NP * KD];          // G~v
  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;
  auto st = [](double* dst, const T& x) {
    dst[0] = x.v;
#pragma unroll
    for (int k = 0; k < K; ++k) dst[1 + k] = x.d[k];
  };
  auto ld = [](const double* src) {
    T x;
    x.v = src[0];
#pragma unroll
    for (int k = 0; k < K; ++k) x.d[k] = src[1 + k];
    return x;
  };
  for (int t = tid; t < NV * NP; t += 64) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  // per point: metrics; per face task: geometry, neighbour data, the fixed outside state
  const bool pt = tid < NP;
  const int p = pt ? tid : 0, i = p % N1, j = p / N1;
  const size_t gp = (size_t)p * ne + e;
  const double sx = a.lv.met[gp], sy = a.lv.met[sstride + gp], tx = a.lv.met[2 * sstride + gp],
               ty = a.lv.met[3 * sstride + gp], ij = a.lv.met[4 * sstride + gp];
  const bool ft = tid < NF;
  const int f = ft ? tid / N1 : 0, kf = ft ? tid % N1 : 0;
  const size_t fo = ((size_t)(f * N1 + kf) * 3) * ne + e;
  const double nx = a.lv.fvec[fo], ny = a.lv.fvec[fo + ne], sm = a.lv.fvec[fo + 2 * ne];
  const double lam = a.lv.lam[(size_t)(f * N1 + kf) * ne + e];
  const int nb = a.lv.nbr[f * ne + e];
  double nbx = 0.0, nby = 0.0, nbsm = 0.0, nblam = 0.0, outv[NV] = {0.0, 0.0, 0.0, 0.0};
  double goutv[NV][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  int kind = (nb == -3) ? 2 : (nb == -2) ? 3 : 1;
  if (ft && nb >= 0) {
    kind = 0;
    const int nf = a.lv.nbf[f * ne + e];
    const int kk = a.lv.ori[f * ne + e] ? (N1 - 1 - kf) : kf;
    const size_t fn = ((size_t)(nf * N1 + kk) * 3) * ne + nb;
    nbx = a.lv.fvec[fn];
    nby = a.lv.fvec[fn + ne];
    nbsm = a.lv.fvec[fn + 2 * ne];
    nblam = a.lv.lam[(size_t)(nf * N1 + kk) * ne + nb];
    const double* wn = (nf == 0 || nf == 2) ? o.lm : o.lp;
    for (int m = 0; m < N1; ++m) {
      const int pp = (nf < 2) ? (m + N1 * kk) : (kk + N1 * m);
#pragma unroll
      for (int v = 0; v < NV; ++v) outv[v] += wn[m] * a.q[v * sstride + (size_t)pp * ne + nb];
    }
    const double* gf = a.lv.gface + (size_t)((nf * N1 + kk) * NV * 2) * ne + nb;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      goutv[v][0] = gf[(size_t)(v * 2) * ne];
      goutv[v][1] = gf[(size_t)(v * 2 + 1) * ne];
    }
  } else if (nb == -2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) outv[v] = a.lv.qinf_g[v];
  }
  __syncthreads();

  for (int c0 = 0; c0 < N; c0 += K) {
    // the element's state as duals: unknown (point m, variable v) carries tangent kk iff
    // m * NV + v == c0 + kk
    auto qd = [&](int v, int m) {
      T x = dconst<K>(sq[v * NP + m]);
#pragma unroll
      for (int kk = 0; kk < K; ++kk) x.d[kk] = (m * NV + v == c0 + kk) ? 1.0 : 0.0;
      return x;
    };
    if (pt) {                                         // local gradients
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T dxi = dconst<K>(0.0), deta = dconst<K>(0.0);
        for (int k = 0; k < N1; ++k) {
          dxi = dxi + o.D[i * N1 + k] * qd(v, k + N1 * j);
          deta = deta + o.D[j * N1 + k] * qd(v, i + N1 * k);
        }
        st(&sgl[((v * 2 + 0) * NP + p) * KD], ij * (sx * dxi + tx * deta));
        st(&sgl[((v * 2 + 1) * NP + p) * KD], ij * (sy * dxi + ty * deta));
      }
    }
    __syncthreads();
    if (ft) {                                         // common viscous flux and jumps
      const double* w = (f == 0 || f == 2) ? o.lm : o.lp;
      T own[NV], out[NV], gown[NV][2], gout[NV][2], jn[NV][2], fhv[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        own[v] = dconst<K>(0.0);
        gown[v][0] = gown[v][1] = dconst<K>(0.0);
        gout[v][0] = dconst<K>(goutv[v][0]);
        gout[v][1] = dconst<K>(goutv[v][1]);
      }
      for (int m = 0; m < N1; ++m) {
        const int pp = (f < 2) ? (m + N1 * kf) : (kf + N1 * m);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          own[v] = own[v] + w[m] * qd(v, pp);
          gown[v][0] = gown[v][0] + w[m] * ld(&sgl[((v * 2 + 0) * NP + pp) * KD]);
          gown[v][1] = gown[v][1] + w[m] * ld(&sgl[((v * 2 + 1) * NP + pp) * KD]);
        }
      }
      if (nb == -1) {                                 // slip wall ghost
        const T ua = own[1] + a.lv.q_ref[1], va = own[2] + a.lv.q_ref[2];
        const T un = ua * nx + va * ny;
        out[0] = own[0];
        out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
        out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
        out[3] = own[3];
      } else if (nb == -3) {                          // no-slip wall ghost
        out[0] = own[0];
        out[1] = -(own[1] + a.lv.q_ref[1]) - a.lv.q_ref[1];
        out[2] = -(own[2] + a.lv.q_ref[2]) - a.lv.q_ref[2];
        out[3] = own[3];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = dconst<K>(outv[v]);
      }
      visc_face2(own, out, a.lv.q_ref, gown, gout, nx, ny, sm, lam, nbx, nby, nbsm, nblam, kind, a.gas, jn, fhv);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        st(&sjn[((tid * NV + v) * 2 + 0) * KD], jn[v][0]);
        st(&sjn[((tid * NV + v) * 2 + 1) * KD], jn[v][1]);
        st(&sfh[(tid * NV + v) * KD], fhv[v]);
      }
    }
    __syncthreads();
    if (pt) {                                         // corrected gradient, viscous point fluxes
      T gc[NV][2];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const T lift = o.gL[i] * ld(&sjn[(((0 * N1 + j) * NV + v) * 2 + d) * KD]) +
                         o.gR[i] * ld(&sjn[(((1 * N1 + j) * NV + v) * 2 + d) * KD]) +
                         o.gL[j] * ld(&sjn[(((2 * N1 + i) * NV + v) * 2 + d) * KD]) +
                         o.gR[j] * ld(&sjn[(((3 * N1 + i) * NV + v) * 2 + d) * KD]);
          gc[v][d] = ld(&sgl[((v * 2 + d) * NP + p) * KD]) + ij * lift;
        }
      }
      const T u = qd(1, p) + a.lv.q_ref[1], vv = qd(2, p) + a.lv.q_ref[2];
      T fx[NV], fy[NV];
      visc_flux2(u, vv, gc, a.gas, fx, fy);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        st(&sfv[(v * NP + p) * KD], sx * fx[v] + sy * fy[v]);
        st(&sgv[(v * NP + p) * KD], tx * fx[v] + ty * fy[v]);
      }
    }
    __syncthreads();
    if (pt) {                                         // R_vis = (1/|J|)[div F~v + g'(F^v - F~v,f)]
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T d = dconst<K>(0.0), fl0 = dconst<K>(0.0), fl1 = dconst<K>(0.0), gl2 = dconst<K>(0.0),
          gl3 = dconst<K>(0.0);
        for (int k = 0; k < N1; ++k) {
          const T fvk = ld(&sfv[(v * NP + k + N1 * j) * KD]), gvk = ld(&sgv[(v * NP + i + N1 * k) * KD]);
          d = d + o.D[i * N1 + k] * fvk + o.D[j * N1 + k] * gvk;
          fl0 = fl0 + o.lm[k] * fvk;
          fl1 = fl1 + o.lp[k] * fvk;
          gl2 = gl2 + o.lm[k] * gvk;
          gl3 = gl3 + o.lp[k] * gvk;
        }
        d = d + o.gL[i] * (ld(&sfh[((0 * N1 + j) * NV + v) * KD]) - fl0) +
            o.gR[i] * (ld(&sfh[((1 * N1 + j) * NV + v) * KD]) - fl1) +
            o.gL[j] * (ld(&sfh[((2 * N1 + i) * NV + v) * KD]) - gl2) +
            o.gR[j] * (ld(&sfh[((3 * N1 + i) * NV + v) * KD]) - gl3);
        double* row = Dv + ((size_t)e * N + p * NV + v) * N;
#pragma unroll
        for (int kk = 0; kk < K; ++kk)
          if (c0 + kk < N) row[c0 + kk] = ij * d.d[kk];
      }
    }
    __syncthreads();
  }
}

template <int P>
static hipError_t launch_visc_jac_p(const JacArgs& a, double* Dv, int ne, hipStream_t st) {
  hipLaunchKernelGGL((k_visc_jac<P, 4>), dim3(ne), dim3(64), 0, st, a, Dv);
  return hipGetLastError();
}

hipError_t launch_jacobian(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                           pmg_factors_s& fac, hipStream_t st) {
  if (L.dim == 3) return launch_jacobian3(L, q, dtau, c_mass, D_out, fac, st);
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
  a.Dv = nullptr;
  if (L.visc) {                          // viscous blocks first: gradient traces, then the duals
    hipError_t err = launch_gradient_traces(L, q, st);
    if (err != hipSuccess) return err;
    switch (L.P) {
      case 0: err = launch_visc_jac_p<0>(a, L.Dv, L.ne, st); break;
      case 1: err = launch_visc_jac_p<1>(a, L.Dv, L.ne, st); break;
      case 2: err = launch_visc_jac_p<2>(a, L.Dv, L.ne, st); break;
      case 3: err = launch_visc_jac_p<3>(a, L.Dv, L.ne, st); break;
      case 4: err = launch_visc_jac_p<4>(a, L.Dv, L.ne, st); break;
      default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess) return err;
    a.Dv = L.Dv;
  }
  switch (L.P) {
    case 0: return launch_jac_rows<0, 1>(a, L.ne, st);
    case 1: return launch_jac_rows<1, 1>(a, L.ne, st);
    case 2: return launch_jac_rows<2, 1>(a, L.ne, st);
    case 3: return launch_jac_rows<3, 1>(a, L.ne, st);
    case 4:
      if (fac.precision == 32 && fac.W) {   // FP32 inverses: the block in LDS, matrix-core updates
        hipLaunchKernelGGL(k_jac_lds<4>, dim3(L.ne), dim3(LdsCfg<4>::NT), 0, st, a);
        return hipGetLastError();
      }
      return launch_jac_rows<4, 2>(a, L.ne, st);
    case 5: return launch_jac_rows<5, 4>(a, L.ne, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmg
