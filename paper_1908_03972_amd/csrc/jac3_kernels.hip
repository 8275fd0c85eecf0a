// Hexahedral element blocks of eqs. (28)-(30) and their inverses: pointwise derivatives by dual
// numbers, assembly along the three tensor lines, row equilibration by powers of two, and
// Gauss-Jordan elimination with partial pivoting, either on rows held in registers (n <= 135) or
// in panels over a global work slot per workgroup (n = 320).
//
// Inverse blocks are stored as [n][Ne][npad]: W[c][e][r] = D_e^{-1}[r][c], rows padded to
// npad = 4 ceil(n/4).
#include <type_traits>

#include "hex_points.hpp"
#include "internal.hpp"
#include "jac3.hpp"
#include "physics3.hpp"
#include "wave_ops.hpp"

namespace pmg {

// ---- element blocks (eqs. (28)-(30)) and their inverses ----------------------------------

typedef double dbl2 __attribute__((ext_vector_type(2)));

struct JacArgs3 {
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

// Rows of D_e in registers, S threads per row (S = 1, or 4 for n = 135 padded to 136 with an
// identity row and column), the Gauss-Jordan elimination of the 2-D kernel: column cycling,
// unnormalised pivot rows, a 32-bit pivot key (|f|'s upper word with the thread index in its low
// 10 bits) reduced over each wave with DPP and across waves through LDS.
template <int P, int S>
struct Rows3 {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5, N = NV * NP;
  static constexpr int NJ = (N + S - 1) / S * S;           // rows and columns including padding
  static constexpr int NPAD = (N + 3) / 4 * 4;             // row stride of the stored inverse
  static constexpr int H = NJ / S;
  static constexpr int NW = (S * NJ + 63) / 64;
  static constexpr int NT = 64 * NW;
  static_assert(S == 1 || S == 4, "one or four threads per row");
  static_assert(S * NJ <= 1023, "pivot keys carry the thread index in 10 bits");
};


// a double from a lane of the same quad selected by the DPP quad permutation CTRL
template <int CTRL>
__device__ __forceinline__ double quad_dpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
constexpr int kQuadFirst = 0x00;   // quad_perm [0,0,0,0]
constexpr int kQuadNext = 0xF9;    // quad_perm [1,2,3,3]: the next lane of the quad
template <int CTRL>
__device__ __forceinline__ float quad_dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}


// The element's state (sq, [Nv][Np]) and its pointwise derivatives into LDS, all threads of the
// workgroup taking part: sA[d] = dF~_d/dq at each solution point ([(pp Nv + v) Nv + w], three
// directions one after the other), sDg = Gamma/dtau + c_mass M at each point, and sB = d(common
// flux)/d(own trace) at each face point, the neighbour's trace fixed and the wall ghost and far-field
// state taken as in the residual. Columns w of the derivatives come from dual numbers seeded in w.
template <int P, int NT>
__device__ void element_point_jacobians3(const JacArgs3& a, int e, double* sq, double* sA, double* sDg,
                                         double* sB) {
  constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5;
  const int ne = a.lv.ne;
  const int tid = threadIdx.x;
  const size_t sstride = (size_t)NP * ne;
  const Ops1D& o = a.ops;
  for (int t = tid; t < NV * NP; t += NT) {
    const int v = t / NP, pp = t % NP;
    sq[t] = a.q[v * sstride + (size_t)pp * ne + e];
  }
  __syncthreads();
  for (int t = tid; t < NP * NV; t += NT) {
    const int pp = t / NV, w = t % NV;
    Dual<1> qd[NV];
    double qv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      qv[v] = a.lv.q_ref[v] + sq[v * NP + pp];
      qd[v] = dconst<1>(qv[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) qd[v].d[0] = (v == w) ? 1.0 : 0.0;
    const size_t gp = (size_t)pp * ne + e;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Dual<1> fl[NV];
      normal_flux3(qd, a.lv.met[(3 * d) * sstride + gp], a.lv.met[(3 * d + 1) * sstride + gp],
                   a.lv.met[(3 * d + 2) * sstride + gp], a.gas, fl);
#pragma unroll
      for (int v = 0; v < NV; ++v) sA[d * NP * NV * NV + (pp * NV + v) * NV + w] = fl[v].d[0];
    }
    Dual<1> qc[NV];
    conservative3(qd, a.gas, qc);
    const State3<double> s = make_state3(qv, a.gas);
    double ew[NV], gcol[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ew[v] = (v == w) ? 1.0 : 0.0;
    gamma_mul3(s, a.gas, ew, gcol);
#pragma unroll
    for (int v = 0; v < NV; ++v) sDg[(pp * NV + v) * NV + w] = gcol[v] * a.inv_dtau + a.c_mass * qc[v].d[0];
  }
  for (int t = tid; t < 6 * NF * NV; t += NT) {
    const int f = t / (NF * NV), kf = (t / NV) % NF, w = t % NV;
    const int k1 = kf % N1, k2 = kf / N1;
    const double* wt = (f % 2 == 0) ? o.lm : o.lp;
    double ownv[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m < N1; ++m) {
      const int pp = line_point3(f, k1, k2, m, N1);
#pragma unroll
      for (int v = 0; v < NV; ++v) ownv[v] += wt[m] * sq[v * NP + pp];
    }
    Dual<1> own[NV], out[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v] = dconst<1>(ownv[v]);
#pragma unroll
    for (int v = 0; v < NV; ++v) own[v].d[0] = (v == w) ? 1.0 : 0.0;
    const size_t fo = ((size_t)(f * NF + kf) * 4) * ne + e;
    const double nx = a.lv.fvec[fo], ny = a.lv.fvec[fo + ne], nz = a.lv.fvec[fo + 2 * ne],
                 sm = a.lv.fvec[fo + 3 * ne];
    const int nb = a.lv.nbr[f * ne + e];
    if (nb >= 0) {
      const int nfa = a.lv.nbf[f * ne + e];
      int na, nbb;
      orient3(a.lv.ori[f * ne + e], k1, k2, N1, na, nbb);
      const double* wn = (nfa % 2 == 0) ? o.lm : o.lp;
      double ov[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int m = 0; m < N1; ++m) {
        const int pp = line_point3(nfa, na, nbb, m, N1);
#pragma unroll
        for (int v = 0; v < NV; ++v) ov[v] += wn[m] * a.q[v * sstride + (size_t)pp * ne + nb];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = dconst<1>(ov[v]);
    } else if (nb == -1) {
      Dual<1> ua = own[1] + a.lv.q_ref[1], va = own[2] + a.lv.q_ref[2], wa = own[3] + a.lv.q_ref[3];
      Dual<1> un = ua * nx + va * ny + wa * nz;
      out[0] = own[0];
      out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
      out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
      out[3] = wa - 2.0 * un * nz - a.lv.q_ref[3];
      out[4] = own[4];
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
    if (f % 2 == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
      common_flux3(out_a, own_a, dq, nx, ny, nz, sm, a.gas, fh);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
      common_flux3(own_a, out_a, dq, nx, ny, nz, sm, a.gas, fh);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sB[((f * NF + kf) * NV + v) * NV + w] = fh[v].d[0];
  }
}

// Entry (row pp Nv + v, column ss Nv + w) of D_e from the pointwise derivatives: a point couples to
// the points of its three tensor lines through the divergence and the g_DG corrections of its own
// and the faces' fluxes (scaled by 1/|J| of the row's point), plus the diagonal term.
template <int P>
__device__ __forceinline__ double block_entry3(const Ops1D& o, const double* sA, const double* sDg,
                                               const double* sB, int pp, int v, int ss, int w, double ijac) {
  constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5;
  const int ii = pp % N1, jj = (pp / N1) % N1, kk = pp / (N1 * N1);
  const int ai = ss % N1, bj = (ss / N1) % N1, ck = ss / (N1 * N1);
  double acc = 0.0;
  if (bj == jj && ck == kk) {
    const double cx = o.D[ii * N1 + ai] - o.gL[ii] * o.lm[ai] - o.gR[ii] * o.lp[ai];
    const int kf = jj + N1 * kk;
    acc += cx * sA[(ss * NV + v) * NV + w] + o.gL[ii] * o.lm[ai] * sB[((0 * NF + kf) * NV + v) * NV + w] +
           o.gR[ii] * o.lp[ai] * sB[((1 * NF + kf) * NV + v) * NV + w];
  }
  if (ai == ii && ck == kk) {
    const double cy = o.D[jj * N1 + bj] - o.gL[jj] * o.lm[bj] - o.gR[jj] * o.lp[bj];
    const int kf = ii + N1 * kk;
    acc += cy * sA[NP * NV * NV + (ss * NV + v) * NV + w] +
           o.gL[jj] * o.lm[bj] * sB[((2 * NF + kf) * NV + v) * NV + w] +
           o.gR[jj] * o.lp[bj] * sB[((3 * NF + kf) * NV + v) * NV + w];
  }
  if (ai == ii && bj == jj) {
    const double cz = o.D[kk * N1 + ck] - o.gL[kk] * o.lm[ck] - o.gR[kk] * o.lp[ck];
    const int kf = ii + N1 * jj;
    acc += cz * sA[2 * NP * NV * NV + (ss * NV + v) * NV + w] +
           o.gL[kk] * o.lm[ck] * sB[((4 * NF + kf) * NV + v) * NV + w] +
           o.gR[kk] * o.lp[ck] * sB[((5 * NF + kf) * NV + v) * NV + w];
  }
  double dval = acc * ijac;
  if (pp == ss) dval += sDg[(pp * NV + v) * NV + w];
  return dval;
}

// Element blocks held in registers (n <= 135): S threads per row, Gauss-Jordan in FP64 (T); the
// pointwise derivatives are computed here with dual numbers.
template <int P, int S>
__global__ void __launch_bounds__((Rows3<P, S>::NT)) k_jac3_rows(JacArgs3 a) {
  using C = Rows3<P, S>;
  using T = double;
  constexpr int NP = C::NP, NF = C::NF, NV = C::NV, N = C::N, NJ = C::NJ, H = C::H, NW = C::NW, NT = C::NT,
                NPAD = C::NPAD;
  __shared__ double sq[NV * NP];
  __shared__ double sA[3 * NP * NV * NV];
  __shared__ double sDg[NP * NV * NV];
  __shared__ double sB[6 * NF * NV * NV];
  __shared__ int sperm[NJ];
  __shared__ T slot[2][NW][NJ];
  __shared__ unsigned skey[2][NW];

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const size_t sstride = (size_t)NP * ne;

  element_point_jacobians3<P, NT>(a, e, sq, sA, sDg, sB);
  __syncthreads();

  const bool has_row = tid < S * NJ;
  const int r = has_row ? tid / S : 0;
  const int h = (S > 1) ? (tid % S) : 0;
  const bool real_row = has_row && r < N;
  const int pp = real_row ? r / NV : 0, v = r % NV;
  const double ijac = a.lv.met[9 * sstride + (size_t)pp * ne + e];
  auto entry = [&](int c) {
    if (real_row && c < N) return block_entry3<P>(a.ops, sA, sDg, sB, pp, v, c / NV, c % NV, ijac);
    return (has_row && !real_row && c == r) ? 1.0 : 0.0;   // padding: identity row
  };
  // one pass: the row's entries rounded to T, unscaled, and its largest entry (in FP64), whose
  // power-of-two scale 2^e2 enters only the pivot keys (as in the large-block kernel: the
  // elimination of the row-equilibrated block, pivot for pivot, without the scaled copy)
  double mx = 0.0;
  T row[H];
#pragma unroll
  for (int jc = 0; jc < H; ++jc) {
    const double dval = entry(h * H + jc);
    if (a.D_out && real_row && h * H + jc < N) a.D_out[((size_t)e * N + r) * N + h * H + jc] = dval;
    mx = fmax(mx, fabs(dval));
    row[jc] = (T)dval;
    __builtin_amdgcn_sched_barrier(0);   // one entry at a time: keeps the assembly's registers few
  }
  if (S == 4) {
    mx = fmax(mx, __shfl_xor(mx, 1, 64));
    mx = fmax(mx, __shfl_xor(mx, 2, 64));
  }
  int ex = 0;
  frexp(mx, &ex);
  const int e2 = (mx > 0.0 && isfinite(mx)) ? -ex : 0;

  bool used = !has_row;
  int my_step = 0;
  T my_inv = (T)1;
  bool bad = false;
  for (int kstep = 0; kstep < NJ; ++kstep) {
    const int par = kstep & 1;
    const T fval = (S == 4) ? quad_dpp<kQuadFirst>(row[0]) : row[0];
    const unsigned key = (used || h != 0) ? 0u : pivot_key(fval, tid, e2);
    const unsigned wkey = wave_max_u32(key);
    const int wtid = 1023 - (int)(wkey & 0x3FFu);
    if (wkey != 0u && tid >= wtid && tid < wtid + S) {
#pragma unroll
      for (int jc = 0; jc < H; ++jc) slot[par][wv][h * H + jc] = row[jc];
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
    int pr_row = (1023 - (int)(bk & 0x3FFu)) / S;
    if (bk == 0u || pr_row >= NJ) {
      bad = true;
      pr_row = (pr_row < NJ && pr_row >= 0) ? pr_row : NJ - 1;
    }
    const T* prw = slot[par][win];
    T piv = prw[0];
    if (piv == (T)0 || !isfinite(piv)) {
      bad = true;
      piv = (T)1;
    }
    const T ip = (T)1 / piv;
    const bool is_p = has_row && (r == pr_row);
    if (tid == 0) sperm[kstep] = pr_row;
    const T g = is_p ? (T)0 : fval * ip;
    if (is_p) {
      used = true;
      my_step = kstep;
      my_inv = ip;
    }
    const T nxt = (S == 4) ? quad_dpp<kQuadNext>(row[0]) : (T)0;
    const T* prh = prw + h * H;
    constexpr int B = 16;
#pragma unroll
    for (int j0 = 0; j0 < H - 1; j0 += B) {
      T buf[B];
#pragma unroll
      for (int jb = 0; jb < B; ++jb)
        if (j0 + jb < H - 1) buf[jb] = prh[j0 + jb + 1];
#pragma unroll
      for (int jb = 0; jb < B; ++jb)
        if (j0 + jb < H - 1) row[j0 + jb] = fma(-g, buf[jb], row[j0 + jb + 1]);
    }
    if (S == 4 && h < S - 1)
      row[H - 1] = fma(-g, prw[(h + 1) * H], nxt);
    else
      row[H - 1] = is_p ? (T)1 : -g;
  }
  if (bad) *a.flag = 1;
  __syncthreads();
  if (has_row && my_step < N) {
#pragma unroll
    for (int jc = 0; jc < H; ++jc) {
      const int col = sperm[h * H + jc];
      if (col >= N) continue;
      const double val = (double)(row[jc] * my_inv);
      const size_t o_ = ((size_t)col * ne + e) * NPAD + my_step;
      if (a.precision == 32)
        static_cast<float*>(a.W)[o_] = (float)val;
      else
        static_cast<double*>(a.W)[o_] = val;
    }
  }
}

// The pointwise derivatives of every element into global memory (jac3_point_elems(P) doubles per
// element: sA, sDg, sB of element_point_jacobians3 one after the other), for the large-block
// elimination, which then needs none of the dual-number arithmetic and its registers.
template <int P>
__global__ void __launch_bounds__(256) k_point_jac3(JacArgs3 a, double* __restrict__ pj) {
  constexpr int NP = (P + 1) * (P + 1) * (P + 1), NV = 5;
  __shared__ double sq[NV * NP];
  const int e = blockIdx.x;
  double* base = pj + (size_t)e * jac3_point_elems(P);
  element_point_jacobians3<P, 256>(a, e, sq, base, base + 3 * NP * NV * NV, base + 4 * NP * NV * NV);
}

// Large element blocks (n = 320 at P = 3): the block is larger than a compute unit's LDS, so each
// workgroup owns a slot of a global work array (n x n row-major, X[r n + c], in the precision of
// the stored inverse, T = float or double) and takes elements in turn, one thread per row. The
// element's pointwise derivatives come from k_point_jac3 (global memory, read in place); the slot
// is cleared with whole-line stores, each thread assembles its row's non-zero entries in FP64 and
// writes them rounded to T, and the block is inverted by Gauss-Jordan elimination with partial
// pivoting in T arithmetic (pivots chosen on the rows equilibrated by powers of two), in panels of
// B columns:
//   * the panel's B steps run on each row's B panel entries held in registers; the pivot search and
//     the broadcast of the pivot row go through LDS as in the register kernel. Pivot rows stay
//     unnormalised (every row keeps the scale of its pivot, divided out once at the end), so a
//     step is one FMA per entry. Eliminating in place (the pivot column's slot receives the
//     transformed unit vector) leaves in the panel the columns e_p + u of T = I + U E^T, T the
//     product of the panel's elementary transforms, E the unit vectors of the panel's pivot rows;
//   * every other column c then takes x_c += U x_c[pivot rows] (U = panel minus the pivot unit
//     vectors), a rank-B update on the matrix cores (16x16x4 tiles, FP32 or FP64 with
//     accumulation in the same precision): the pivot rows' old values (contiguous in the
//     row-major slot) are gathered into LDS first, then every wave streams its own rows.
// Barriers order the slot's accesses across the lanes of a wave. At the end, physical row p_i of
// the slot is row i of the inverse times its pivot f_i, with its columns in pivot order:
// D_e^{-1}[i][p_m] = X[p_i n + m] / f_i.
template <int P, int B_>
struct Big3 {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5, N = NV * NP;
  static constexpr int NPAD = (N + 3) / 4 * 4;
  static constexpr int B = B_, G = 16;   // panel width; columns per matrix-core tile
  static constexpr int NT = N, NW = NT / 64;
  // columns per gathered chunk of pivot rows in the update: 32 x 320 FP32 values at most
  template <typename T>
  static constexpr int chunk() { return N * 32 * 4 / (B * (int)sizeof(T)); }
  // LDS pool in doubles: the pivot rows of the panel steps ([2][NW][B]), then the gathered pivot
  // rows of a chunk (B rows, stride padded by 64 bytes)
  static constexpr int GJ = 2 * NW * B;
  static constexpr int XPF = B * (chunk<float>() + 16) * 4 / 8, XPD = B * (chunk<double>() + 8);
  static constexpr int XP = XPF > XPD ? XPF : XPD;
  static constexpr int POOL = XP > GJ ? XP : GJ;
  static_assert(N % 64 == 0 && N % B == 0 && B % G == 0 && B % 4 == 0 && G == 16, "whole tiles and panels");
  static_assert(N % chunk<float>() == 0 && N % chunk<double>() == 0 && chunk<float>() % G == 0 &&
                chunk<double>() % G == 0, "whole 16-column groups per chunk");
  static_assert(B * (chunk<float>() + 16) * 4 <= POOL * 8 && B * (chunk<double>() + 8) * 8 <= POOL * 8,
                "gathered pivot rows fit the pool");
  static_assert(N <= 1023, "pivot keys carry the row in 10 bits");
};


// The FP32 instance is held to four waves per SIMD (at most 128 registers): two workgroups of five
// waves are then resident on each CU, and one's panel steps overlap the other's memory-bound
// phases (without the bound the compiler took 126 registers and only one workgroup per CU ran at a
// time, 1.3x slower). The FP64 instance needs more registers and runs one workgroup per CU.
template <int P, typename T, int BW>
__global__ void __launch_bounds__((Big3<P, BW>::NT)) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_jac3_big(JacArgs3 a, T* __restrict__ ws,
                                                             const double* __restrict__ pj) {
  using C = Big3<P, BW>;
  using T4 = typename std::conditional<sizeof(T) == 4, flt4, dbl4>::type;
  constexpr int NP = C::NP, NF = C::NF, NV = C::NV, N = C::N, NPAD = C::NPAD, B = C::B, G = C::G, NW = C::NW,
                NT = C::NT;
  __shared__ double pool[C::POOL];
  __shared__ int sperm[N];
  __shared__ unsigned skey[2][NW];
  __shared__ T sinv[N];                   // 1 / pivot of every step
  T* slot = reinterpret_cast<T*>(pool);   // [2][NW][B] pivot rows of the panel steps

  const int ne = a.lv.ne;
  const int r = threadIdx.x;
  const int lane = r & 63, wv = r >> 6;
  const size_t sstride = (size_t)NP * ne;
  T* X = ws + (size_t)blockIdx.x * N * N;
  const int pp = r / NV, v = r % NV;
  const int ii = pp % (P + 1), jj = (pp / (P + 1)) % (P + 1), kk = pp / ((P + 1) * (P + 1));
  bool bad = false;
  // the 1-D operators in LDS: D (row-major), then g_L', g_R', l(-1), l(+1)
  constexpr int kGL = (P + 1) * (P + 1), kGR = kGL + P + 1, kLM = kGR + P + 1, kLP = kLM + P + 1;
  __shared__ double sop[kLP + P + 1];
  if (r < (P + 1) * (P + 1)) sop[r] = a.ops.D[r];
  if (r <= P) {
    sop[kGL + r] = a.ops.gL[r];
    sop[kGR + r] = a.ops.gR[r];
    sop[kLM + r] = a.ops.lm[r];
    sop[kLP + r] = a.ops.lp[r];
  }

  for (int e = blockIdx.x; e < ne; e += gridDim.x) {
    __syncthreads();                        // the previous element is done with the pool and sperm
    // the element's pointwise derivatives, read in place (L2-resident once touched): the flux
    // Jacobians sA, the diagonal term sDg and the common-flux derivatives sB, one after the other
    const double* sA = pj + (size_t)e * jac3_point_elems(P);
    const double* sDg = sA + 3 * NP * NV * NV;
    const double* sB = sDg + NP * NV * NV;
    {   // clear the slot with 16-byte stores along its rows (whole lines per wave); the rows'
        // non-zero entries are written after the barrier that follows the row scales
      using V16 = typename std::conditional<sizeof(T) == 4, flt4, dbl2>::type;
      V16* xz = reinterpret_cast<V16*>(X);
      constexpr int NZ = N * N * (int)sizeof(T) / 16;
      for (int t = r; t < NZ; t += NT) xz[t] = V16{};
    }

    // row r of D_e: only the 10 points of the row point's three tensor lines couple to it, so
    // the row is cleared and those 50 entries (the point itself gathering all three lines and
    // the diagonal term, summed in the order x, y, z) are written over it; the largest entry sets
    // the row's power-of-two scale
    const double ijac = a.lv.met[9 * sstride + (size_t)pp * ne + e];
    const int ids[3] = {ii, jj, kk};
    auto line_val = [&](int d, int m, int w) {       // the line-d term of column (point on d at m, w)
      const int id = ids[d];
      const int ss = d == 0 ? m + (P + 1) * (jj + (P + 1) * kk)
                            : d == 1 ? ii + (P + 1) * (m + (P + 1) * kk) : ii + (P + 1) * (jj + (P + 1) * m);
      const int kf = d == 0 ? jj + (P + 1) * kk : d == 1 ? ii + (P + 1) * kk : ii + (P + 1) * jj;
      const double gl = sop[kGL + id] * sop[kLM + m], gr = sop[kGR + id] * sop[kLP + m];
      const double cv = sop[id * (P + 1) + m] - gl - gr;
      return cv * sA[d * NP * NV * NV + (ss * NV + v) * NV + w] +
             gl * sB[(((2 * d) * NF + kf) * NV + v) * NV + w] + gr * sB[(((2 * d + 1) * NF + kf) * NV + v) * NV + w];
    };
    auto diag_val = [&](int w) {
      double acc = 0.0;
#pragma unroll 1
      for (int d = 0; d < 3; ++d) acc += line_val(d, ids[d], w);
      return acc * ijac + sDg[(pp * NV + v) * NV + w];
    };
    // one pass: the entries are written unscaled (rounded to T) while the row's largest entry is
    // found; the row's power-of-two scale 2^e2 then enters only the pivot keys. Scaling a row by a
    // power of two commutes exactly with every operation of the elimination, so this is the
    // elimination of the row-equilibrated block, pivot for pivot, without the scaled copy, and
    // the result is the inverse of the block itself
    T* xr = X + (size_t)r * N;
    double* dr = a.D_out ? a.D_out + ((size_t)e * N + r) * N : nullptr;
    if (dr)
      for (int c = 0; c < N; ++c) dr[c] = 0.0;
    __syncthreads();                        // the slot is clear
    double mx = 0.0;
#pragma unroll 1
    for (int w = 0; w < NV; ++w) {
      const double dval = diag_val(w);
      mx = fmax(mx, fabs(dval));
      xr[pp * NV + w] = (T)dval;
      if (dr) dr[pp * NV + w] = dval;
    }
#pragma unroll 1
    for (int d = 0; d < 3; ++d)
#pragma unroll 1
      for (int m = 0; m <= P; ++m) {
        if (m == ids[d]) continue;
        const int ss = d == 0 ? m + (P + 1) * (jj + (P + 1) * kk)
                              : d == 1 ? ii + (P + 1) * (m + (P + 1) * kk) : ii + (P + 1) * (jj + (P + 1) * m);
        for (int w = 0; w < NV; ++w) {
          const double dval = line_val(d, m, w) * ijac;
          mx = fmax(mx, fabs(dval));
          xr[ss * NV + w] = (T)dval;
          if (dr) dr[ss * NV + w] = dval;
        }
      }
    int ex = 0;
    frexp(mx, &ex);
    const int e2 = (mx > 0.0 && isfinite(mx)) ? -ex : 0;
    __syncthreads();                        // every row of the slot is written

    bool used = false;
    for (int k0 = 0; k0 < N; k0 += B) {
      T row[B];
#pragma unroll
      for (int j = 0; j < B; ++j) row[j] = X[(size_t)r * N + k0 + j];
      // column cycling: before step j the row holds columns k0 + j .. k0 + B - 1, then the slots
      // of steps 0 .. j - 1; each step consumes entry 0 and appends its own slot, so after the
      // panel the row holds the B slots in step order
#pragma unroll 1
      for (int j = 0; j < B; ++j) {
        const int par = j & 1;
        const T fv = row[0];
        const unsigned key = used ? 0u : pivot_key(fv, r, e2);
        const unsigned wkey = wave_max_u32(key);
        if (wkey != 0u && r == 1023 - (int)(wkey & 0x3FFu)) {   // the row shifted by one, pivot last,
#pragma unroll                                                    // so that the reads below are aligned
          for (int c = 0; c < B - 1; ++c) slot[(par * NW + wv) * B + c] = row[c + 1];
          slot[(par * NW + wv) * B + B - 1] = row[0];
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
        if (bk == 0u || pr >= N) {
          bad = true;
          pr = 0;
        }
        const T* prw = slot + (par * NW + win) * B;
        T piv = prw[B - 1];
        if (piv == (T)0 || !isfinite(piv)) {
          bad = true;
          piv = (T)1;
        }
        const T ip = (T)1 / piv;
        const bool is_p = (r == pr);
        if (r == 0) sperm[k0 + j] = pr;
        if (is_p) {
          used = true;
          sinv[k0 + j] = ip;
        }
        const T g = is_p ? (T)0 : fv * ip;
#pragma unroll
        for (int c = 0; c < B - 1; ++c) row[c] = fma(-g, prw[c], row[c + 1]);
        row[B - 1] = is_p ? (T)1 : -g;
      }
#pragma unroll
      for (int j = 0; j < B; ++j) X[(size_t)r * N + k0 + j] = row[j];
      __syncthreads();                      // the panel is visible to the other lanes of each wave
      // Rank-B update of every other column on the matrix cores, wave wv taking rows
      // 64 wv .. 64 wv + 63 as four tiles of 16: per 16 columns cg.., D = U X_p + C with
      //   A[i][k] = U[r0 + i][4 s + k]: lane i + 16 k (U = panel minus the pivot unit vectors),
      //   B[k][j] = X_p[4 s + k][cg + j]: lane j + 16 k, the old value of column cg + j in the
      //             pivot row of step k0 + 4 s + k, from LDS,
      //   C, D[i][j] = X[r0 + i][cg + j]: lane j + 16 lk, register v with i = acc_row(lk, v),
      // so that the 16 lanes of a register cover 64 (FP32) or 128 (FP64) contiguous bytes of one
      // row. The pivot rows' old values of a chunk of CW columns are first gathered into LDS
      // (xp, row stride CWP), so that after one barrier every wave streams its own rows.
      const int lr = lane & 15, lk = lane >> 4;
      // slot offsets split into a per-lane part (one 32-bit register) and a uniform part, so that
      // every load and store addresses the slot as a scalar base plus that register
      const unsigned uoff = (unsigned)((64 * wv + lr) * N + lk);
      const unsigned aoff = (unsigned)((64 * wv + acc_row<T>(lk, 0)) * N + lr);
      constexpr int VS = sizeof(T) == 4 ? 1 : 4;   // row step of accumulator register v
      T uop[4][B / 4];
#pragma unroll
      for (int TT = 0; TT < 4; ++TT) {
#pragma unroll
        for (int s4 = 0; s4 < B / 4; ++s4) {
          const int row_ = 64 * wv + 16 * TT + lr, m = 4 * s4 + lk;
          const T u = (X + 16 * TT * N + k0 + 4 * s4)[uoff];
          uop[TT][s4] = (sperm[k0 + m] == row_) ? u - (T)1 : u;
        }
      }
      constexpr int CW = C::template chunk<T>(), CWP = CW + 64 / (int)sizeof(T);
      T* xp = reinterpret_cast<T*>(pool);   // [B][CWP]; the panel's pivot rows are done with
      for (int c0 = 0; c0 < N; c0 += CW) {
        __syncthreads();                    // LDS free (pivot slots, or the previous chunk)
        for (int t = r; t < B * CW; t += NT) {
          const int k = t / CW, c = t % CW;
          xp[k * CWP + c] = X[(size_t)sperm[k0 + k] * N + c0 + c];
        }
        __syncthreads();                    // every old pivot-row value is in LDS before any store
        // the chunk's 16-column groups outside the panel, in order
        const int ps = k0 > c0 ? k0 : c0, pe = (k0 + B < c0 + CW) ? k0 + B : c0 + CW;
        const int skip = pe > ps ? pe - ps : 0, ng = (CW - skip) / G;
        auto group = [&](int g) {
          const int cg = c0 + G * g;
          return (skip && cg >= ps) ? cg + skip : cg;
        };
        auto load_acc = [&](T4(&acc)[4], int cg) {
#pragma unroll
          for (int TT = 0; TT < 4; ++TT) {
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) acc[TT][v2] = (X + (16 * TT + VS * v2) * N + cg)[aoff];
          }
        };
        auto update_store = [&](T4(&acc)[4], int cg) {
#pragma unroll
          for (int s4 = 0; s4 < B / 4; ++s4) {
            const T xb = xp[(4 * s4 + lk) * CWP + (cg - c0) + lr];
#pragma unroll
            for (int TT = 0; TT < 4; ++TT) acc[TT] = mfma16x16x4(uop[TT][s4], xb, acc[TT]);
          }
#pragma unroll
          for (int TT = 0; TT < 4; ++TT) {
#pragma unroll
            for (int v2 = 0; v2 < 4; ++v2) (X + (16 * TT + VS * v2) * N + cg)[aoff] = acc[TT][v2];
          }
        };
        for (int g = 0; g < ng; ++g) {
          T4 acc_a[4];
          load_acc(acc_a, group(g));
          update_store(acc_a, group(g));
        }
      }
      __syncthreads();                      // the updated columns are visible before the next panel
    }
    __syncthreads();                        // sperm and sinv complete
    // thread r writes row r of the inverse (slot row p_r), so that for each column the lanes of
    // a wave store consecutive entries of W. The stores are non-temporal: the inverses (15 GB at
    // P3 on the 36864-element sphere) are not read again in this kernel, and cached they would
    // push the other workgroups' work slots out of the Infinity Cache (86 -> 76 ms per FP32
    // rebuild of that level)
    const int prow = sperm[r];
    const T pinv = sinv[r];
    for (int m0 = 0; m0 < N; m0 += 16) {    // sixteen loads in flight per thread, then the stores
      T xv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = X[(size_t)prow * N + m0 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int col = sperm[m0 + u];
        const double val = (double)(xv[u] * pinv);
        const size_t o_ = ((size_t)col * ne + e) * NPAD + r;
        if (a.precision == 32)
          __builtin_nontemporal_store((float)val, static_cast<float*>(a.W) + o_);
        else
          __builtin_nontemporal_store(val, static_cast<double*>(a.W) + o_);
      }
    }
  }
  if (bad) *a.flag = 1;
}

// Mid-size element blocks held in LDS (P = 2: n = 135 padded to NR = 144 with identity rows and
// columns), inverted in FP32 by the panel Gauss-Jordan of the large-block kernel, but with the whole
// block in LDS: one workgroup of three waves per element, the panels' B = 16 steps on the rows'
// panel entries in registers, every other column's rank-16 update on the FP32 matrix cores with
// its operands and accumulators read from and written back to LDS. The pointwise derivatives come
// from k_point_jac3; the row's power-of-two equilibration enters only the pivot keys.
template <int P>
struct Lds3 {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5, N = NV * NP;
  static constexpr int NR = (N + 15) / 16 * 16;     // rows and columns with the identity padding
  static constexpr int NPAD = (N + 3) / 4 * 4;      // row stride of the stored inverse
  static constexpr int XS = NR + 4;                 // LDS row stride (words)
  static constexpr int B = 16, NT = 192, NW = 3;
  static constexpr int TPW = NR / 16 / NW;          // 16-row tiles per wave in the update
  static constexpr int NPJ = (4 * NP + 6 * NF) * NV * NV;
  static_assert(NR % (16 * NW) == 0 && NR % B == 0 && NR <= NT, "whole tiles per wave, one thread per row");
  static_assert(NT <= 1023, "pivot keys carry the row in 10 bits");
};

template <int P>
__global__ void __launch_bounds__(Lds3<P>::NT) k_jac3_lds(JacArgs3 a, const double* __restrict__ pj) {
  using C = Lds3<P>;
  constexpr int NP = C::NP, NV = C::NV, N = C::N, NR = C::NR, NPAD = C::NPAD, XS = C::XS, B = C::B, NT = C::NT,
                NW = C::NW, TPW = C::TPW, NPJ = C::NPJ;
  __shared__ float X[NR * XS];
  __shared__ double sj[NPJ];                 // sA, sDg, sB one after the other
  __shared__ float xp[B * XS];               // old pivot-row values of a panel
  __shared__ float slot[2][NW][B];
  __shared__ int sperm[NR];
  __shared__ float sinv[NR];
  __shared__ unsigned skey[2][NW];

  const int ne = a.lv.ne;
  const int e = blockIdx.x;
  const int r = threadIdx.x;
  const int lane = r & 63, wv = r >> 6;
  const size_t sstride = (size_t)NP * ne;
  {
    const double* src = pj + (size_t)e * NPJ;
    constexpr int U = 4;
    for (int t0 = r; t0 < NPJ; t0 += U * NT) {   // U loads in flight per thread
      double vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) vv[u] = (t0 + u * NT < NPJ) ? src[t0 + u * NT] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (t0 + u * NT < NPJ) sj[t0 + u * NT] = vv[u];
    }
    for (int t = r; t < NR * XS; t += NT) X[t] = 0.f;
  }
  __syncthreads();
  const double* sA = sj;
  const double* sDg = sj + 3 * NP * NV * NV;
  const double* sB = sDg + NP * NV * NV;

  // row r: the 1 + 3P points of the row point's three tensor lines (the point itself once);
  // padding rows are identity rows
  int e2 = 0;
  if (r < N) {
    const int pp = r / NV, v = r % NV;
    const int ii = pp % (P + 1), jj = (pp / (P + 1)) % (P + 1), kk = pp / ((P + 1) * (P + 1));
    const double ijac = a.lv.met[9 * sstride + (size_t)pp * ne + e];
    double* dr = a.D_out ? a.D_out + ((size_t)e * N + r) * N : nullptr;
    if (dr)
      for (int c = 0; c < N; ++c) dr[c] = 0.0;
    double mx = 0.0;
#pragma unroll 1
    for (int t = 0; t < 1 + 3 * P; ++t) {
      int ss = pp;
      if (t > 0) {
        const int d = (t - 1) / P, mo = (t - 1) % P;
        const int own = d == 0 ? ii : d == 1 ? jj : kk;
        const int m = mo < own ? mo : mo + 1;   // the other points of line d
        ss = d == 0 ? m + (P + 1) * (jj + (P + 1) * kk)
                    : d == 1 ? ii + (P + 1) * (m + (P + 1) * kk) : ii + (P + 1) * (jj + (P + 1) * m);
      }
#pragma unroll 1
      for (int w = 0; w < NV; ++w) {
        const double dval = block_entry3<P>(a.ops, sA, sDg, sB, pp, v, ss, w, ijac);
        mx = fmax(mx, fabs(dval));
        X[r * XS + ss * NV + w] = (float)dval;
        if (dr) dr[ss * NV + w] = dval;
      }
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
    // column cycling as in the large-block kernel
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
    // the old values of the panel's pivot rows, then the rank-16 update of every other column
    for (int t = r; t < B * NR; t += NT) {
      const int k = t / NR, c = t % NR;
      xp[k * XS + c] = X[sperm[k0 + k] * XS + c];
    }
    float uop[TPW][B / 4];
#pragma unroll
    for (int TT = 0; TT < TPW; ++TT) {
#pragma unroll
      for (int s4 = 0; s4 < B / 4; ++s4) {
        const int row_ = 16 * (TPW * wv + TT) + lr, m = k0 + 4 * s4 + lk;
        const float u = X[row_ * XS + m];
        uop[TT][s4] = (sperm[m] == row_) ? u - 1.f : u;
      }
    }
    __syncthreads();                      // xp complete, every panel value read
#pragma unroll 1
    for (int cg = 0; cg < NR; cg += 16) {
      if (cg == k0) continue;             // B == 16: the panel is one column group
      flt4 acc[TPW];
#pragma unroll
      for (int TT = 0; TT < TPW; ++TT) {
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) acc[TT][v2] = X[(16 * (TPW * wv + TT) + 4 * lk + v2) * XS + cg + lr];
      }
#pragma unroll
      for (int s4 = 0; s4 < B / 4; ++s4) {
        const float xb = xp[(4 * s4 + lk) * XS + cg + lr];
#pragma unroll
        for (int TT = 0; TT < TPW; ++TT) acc[TT] = mfma16x16x4(uop[TT][s4], xb, acc[TT]);
      }
#pragma unroll
      for (int TT = 0; TT < TPW; ++TT) {
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) X[(16 * (TPW * wv + TT) + 4 * lk + v2) * XS + cg + lr] = acc[TT][v2];
      }
    }
    __syncthreads();                      // the updated columns are visible before the next panel
  }
  if (bad) *a.flag = 1;
  // row i of the inverse is slot row p_i = sperm[i] over 1/f_i, columns in pivot order
  if (r < N) {
    const int prow = sperm[r];
    const float pinv = sinv[r];
#pragma unroll 4
    for (int m = 0; m < N; ++m) {
      const int col = sperm[m];
      if (col >= N) continue;             // only a singular block (flagged) pivots on a padding row
      const double val = (double)(X[prow * XS + m] * pinv);
      static_cast<float*>(a.W)[((size_t)col * ne + e) * NPAD + r] = (float)val;
    }
  }
}

// ---- launchers -------------------------------------------------------------------------------

template <int P, int S>
static hipError_t launch_jac3_p(const JacArgs3& a, int ne, hipStream_t st) {
  hipLaunchKernelGGL((k_jac3_rows<P, S>), dim3(ne), dim3(Rows3<P, S>::NT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_jacobian3(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                            pmg_factors_s& fac, hipStream_t st) {
  JacArgs3 a{};
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
    case 0: return launch_jac3_p<0, 1>(a, L.ne, st);
    case 1: return launch_jac3_p<1, 1>(a, L.ne, st);
    case 2: {
      // FP64 inverses: the register-row kernel, pointwise derivatives computed in place (40 ms on
      // the 36 864-element sphere); FP32 inverses: the pointwise derivatives first, then the block
      // in LDS eliminated in FP32 with matrix-core updates (21 ms; the register-row elimination in
      // FP32 took 28 ms, split the same way in FP64 43.5 ms)
      if (fac.precision != 32 || !fac.ws) return launch_jac3_p<2, 4>(a, L.ne, st);
      hipLaunchKernelGGL(k_point_jac3<2>, dim3(L.ne), dim3(256), 0, st, a, fac.ws);
      hipLaunchKernelGGL(k_jac3_lds<2>, dim3(L.ne), dim3(Lds3<2>::NT), 0, st, a, (const double*)fac.ws);
      return hipGetLastError();
    }
    case 3: {
      if (!fac.ws || fac.ws_slots <= 0) return hipErrorInvalidValue;
      const int grid = fac.ws_slots < L.ne ? fac.ws_slots : L.ne;
      double* pj = fac.ws + (size_t)fac.ws_slots * L.n * L.n;   // after the work slots
      hipLaunchKernelGGL(k_point_jac3<3>, dim3(L.ne), dim3(256), 0, st, a, pj);
      // the mixed form (FP32 inverses) eliminates in FP32 on the FP32 matrix cores, the plain form in FP64
      // (panels of 32 columns)
      if (fac.precision == 32)
        hipLaunchKernelGGL((k_jac3_big<3, float, 32>), dim3(grid), dim3(Big3<3, 32>::NT), 0, st, a,
                           reinterpret_cast<float*>(fac.ws), (const double*)pj);
      else
        hipLaunchKernelGGL((k_jac3_big<3, double, 32>), dim3(grid), dim3(Big3<3, 32>::NT), 0, st, a, fac.ws,
                           (const double*)pj);
      return hipGetLastError();
    }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pmg
