// Hexahedral (3-D) kernels: FR/CPR residual and fused element-Jacobi sweep, P-level transfers and
// pointwise helpers (the element blocks and their inverses are in jac3_kernels.hip).
//
// Layouts (Ne elements, Np = (P+1)^3 points p = i + (P+1) j + (P+1)^2 k, Nv = 5 variables):
//   state            [Nv][Np][Ne]
//   metrics          [10][Np][Ne]: J grad xi^d (component n at 3 d + n), then 1/|J|
//   face data        [6][(P+1)^2][4][Ne]: unit +xi^(f/2) normal and its length |S|, face point
//                    k1 + (P+1) k2 along the face's tangential directions ((eta, zeta), (xi, zeta),
//                    (xi, eta))
//   inverse blocks   [n][Ne][npad]: W[c][e][r] = D_e^{-1}[r][c], rows padded to npad = 4 ceil(n/4)
//
// The fused sweep follows the 2-D kernel: one lane per solution point and per face point of its
// element; point and face loads first, then the neighbour gathers (branch-free), point fluxes
// F~_d = f . (J grad xi^d) to LDS, the common flux of eq. (21) per face point, the divergence with
// the g_DG corrections of eq. (20) along the three tensor lines, and for a sweep the matvec with
// the element's inverse block, float4 loads over four consecutive rows.
#include "internal.hpp"
#include "hex_points.hpp"
#include "physics3.hpp"
#include "block_loads.hpp"

namespace pmg {

constexpr int kPad3 = -100;   // neighbour tag of the padding elements of the last workgroup

// Elements per workgroup. Lanes are (point, element) with the element fastest, so that a load of
// one (variable, point) of the [Nv][Np][Ne] state by EPW consecutive lanes covers EPW consecutive
// elements: with one element per workgroup every such load would touch a cache line of its own.
constexpr int epw3_for(int P) { return P == 0 ? 32 : P == 1 ? 8 : P == 2 ? 8 : 4; }

// The tuner's candidates (pmg_level_autotune): the default and the groupings whose registers still
// fit the workgroup (twice the default would spill at P2 and P3).
constexpr bool epw3_candidate(int P, int epw) {
  return epw == epw3_for(P) || (P == 0 && (epw == 16 || epw == 64)) || (P == 1 && (epw == 4 || epw == 16)) ||
         (P == 2 && epw == 4) || (P == 3 && epw == 2);
}

template <int P, int EPW_ = epw3_for(P)>
struct Cfg3 {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, NF = N1 * N1, NV = 5, N = NV * NP;
  static constexpr int NPAD = (N + 3) / 4 * 4;
  static constexpr int EPW = EPW_;
  static constexpr int LPE = NP > 6 * NF ? NP : 6 * NF;   // lanes per element
  static constexpr int NACT = EPW * LPE;
  static constexpr int NT = ((NACT + 63) / 64) * 64;
  static constexpr int NW = NT / 64;
  static constexpr int MVL = NPAD / 4;                     // matvec lanes per element
};

struct ResArgs3 {
  LevelView lv;
  Ops1D ops;
  GasParams gas;
  const double* q;
  const double* src;
  const double* S;
  double c_mass;
  double* F;
  double* part;
  const void* W;
  double alpha;
  double* q_out;
  int w_stream;   // FP32 blocks larger than the Infinity Cache: non-temporal loads
};

template <int NT>
__device__ __forceinline__ void sync3() {
  if constexpr (NT == 64) {   // one wave: its LDS accesses complete in program order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// MODE 0: residual; 1: sweep with FP64 inverse blocks; 2: sweep with FP32 inverse blocks
template <int P, int MODE, int EPW_ = epw3_for(P)>
__global__ void __launch_bounds__((Cfg3<P, EPW_>::NT)) k_fr3(ResArgs3 a) {
  using C = Cfg3<P, EPW_>;
  constexpr int N1 = C::N1, NP = C::NP, NF = C::NF, NV = C::NV, N = C::N, NPAD = C::NPAD, EPW = C::EPW;
  __shared__ double s_q[NV * NP * EPW];
  // F~, G~, H~ per point; after the divergence the matvec's F and D^{-1} F reuse it
  constexpr int FGH = (3 * NV * NP > 2 * NPAD ? 3 * NV * NP : 2 * NPAD) * EPW;
  __shared__ double s_fgh[FGH];
  __shared__ double s_j[6 * NF * NV * EPW];
  __shared__ double s_ops[N1 * N1 + 4 * N1];
  __shared__ double s_red[C::NW * NV];

  const int ne = a.lv.ne;
  const int tid = threadIdx.x;
  const bool act = tid < C::NACT;
  const int el = tid % EPW;
  const int p = act ? tid / EPW : 0;
  const bool pt = act && p < NP;
  const int e = xcd_group(blockIdx.x, gridDim.x) * EPW + el;
  const bool valid = pt && e < ne;
  const int i = p % N1, j = (p / N1) % N1, k = p / (N1 * N1);
  const size_t sstride = (size_t)NP * ne;
  static_assert(N1 * N1 + 4 * N1 <= C::NT, "one lane per operator entry");
  double opv = 0.0;
  {
    const int r = tid - N1 * N1;
    const int idx = tid < N1 * N1 ? tid : kMaxN1 * kMaxN1 + (r / N1) * kMaxN1 + r % N1;
    const double* ops = reinterpret_cast<const double*>(reinterpret_cast<const char*>(&a.ops) + offsetof(Ops1D, D));
    if (tid < N1 * N1 + 4 * N1) opv = ops[idx];
  }
  struct {
    const double *D, *lm, *lp, *gL, *gR;
  } const o = {s_ops, s_ops + N1 * N1, s_ops + N1 * N1 + N1, s_ops + N1 * N1 + 2 * N1, s_ops + N1 * N1 + 3 * N1};

#define SQ(v, pp, ee) s_q[((v) * NP + (pp)) * EPW + (ee)]
#define SF(d, v, pp, ee) s_fgh[(((d) * NV + (v)) * NP + (pp)) * EPW + (ee)]
#define SJ(f, kf, v, ee) s_j[(((f) * NF + (kf)) * NV + (v)) * EPW + (ee)]

  // point operands (every lane loads a state; lanes without a point of a real element take a point
  // of the last element)
  const size_t gp = (size_t)p * ne + e;
  const size_t gpl = (size_t)(pt ? p : 0) * ne + (e < ne ? e : ne - 1);
  double qv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) qv[v] = a.q[v * sstride + gpl];
  double mt[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
  double ij = 0.0;
  double srcv[NV], sv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) srcv[v] = sv[v] = 0.0;
  if (valid) {
#pragma unroll
    for (int c = 0; c < 9; ++c) mt[c] = a.lv.met[c * sstride + gp];
    ij = a.lv.met[9 * sstride + gp];
    if (a.src) {
#pragma unroll
      for (int v = 0; v < NV; ++v) srcv[v] = a.src[v * sstride + gp];
    }
    if (a.S) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sv[v] = a.S[v * sstride + gp];
    }
  }
  // this lane's face point: face data, neighbour, and the neighbour's line of states
  const bool fpt = act && p < 6 * NF;
  const int f = p / NF, kf = p % NF, k1 = kf % N1, k2 = kf / N1;
  double nx = 1.0, ny = 0.0, nz = 0.0, sm = 1.0;
  int nb = kPad3, nf = 0, ori = 0;
  if (fpt && e < ne) {
    const size_t fo = ((size_t)(f * NF + kf) * 4) * ne + e;
    nx = a.lv.fvec[fo];
    ny = a.lv.fvec[fo + ne];
    nz = a.lv.fvec[fo + 2 * ne];
    sm = a.lv.fvec[fo + 3 * ne];
    nb = a.lv.nbr[f * ne + e];
    nf = a.lv.nbf[f * ne + e];
    ori = a.lv.ori[f * ne + e];
  }
  const bool hasn = nb >= 0;
  const int nbc = hasn ? nb : 0, nfc = hasn ? nf : 0;
  int na, nbb;
  orient3(hasn ? ori : 0, k1, k2, N1, na, nbb);
  double nq[N1][NV];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    const int pp = line_point3(nfc, na, nbb, m, N1);
#pragma unroll
    for (int v = 0; v < NV; ++v) nq[m][v] = a.q[v * sstride + (size_t)pp * ne + nbc];
  }

  double qa[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) qa[v] = a.lv.q_ref[v] + qv[v];
  const double rho = qa[0] / (a.gas.rgas * qa[4]);
  {
    double fl[3][NV];
#pragma unroll
    for (int d = 0; d < 3; ++d) normal_flux3_rho(qa, rho, mt[3 * d], mt[3 * d + 1], mt[3 * d + 2], a.gas, fl[d]);
    if (pt) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        SQ(v, p, el) = qv[v];
        SF(0, v, p, el) = fl[0][v];
        SF(1, v, p, el) = fl[1][v];
        SF(2, v, p, el) = fl[2][v];
      }
    }
  }
  if (tid < N1 * N1 + 4 * N1) s_ops[tid] = opv;
  sync3<C::NT>();

  // face phase: common flux minus the interpolated local flux at every face point
  {
    double out[NV];
    {
      const double* wn = o.lm + ((nfc % 2 == 0) ? 0 : N1);
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll
      for (int m = 0; m < N1; ++m) {
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] += wn[m] * nq[m][v];
      }
    }
    if (fpt) {
      const int d = f / 2;
      const double* w = o.lm + ((f % 2 == 0) ? 0 : N1);
      double own[NV], floc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) own[v] = floc[v] = 0.0;
#pragma unroll
      for (int m = 0; m < N1; ++m) {
        const int pp = line_point3(f, k1, k2, m, N1);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          own[v] += w[m] * SQ(v, pp, el);
          floc[v] += w[m] * s_fgh[((d * NV + v) * NP + pp) * EPW + el];
        }
      }
      if (nb >= 0) {
      } else if (nb == -1) {             // slip wall: reflect the normal velocity
        const double ua = a.lv.q_ref[1] + own[1], va = a.lv.q_ref[2] + own[2], wa = a.lv.q_ref[3] + own[3];
        const double un = ua * nx + va * ny + wa * nz;
        out[0] = own[0];
        out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
        out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
        out[3] = wa - 2.0 * un * nz - a.lv.q_ref[3];
        out[4] = own[4];
      } else if (nb == -2) {             // far field
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = a.lv.qinf_g[v];
      } else {                           // padding element of the last workgroup
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = own[v];
      }
      double own_a[NV], out_a[NV], dq[NV], fh[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        own_a[v] = a.lv.q_ref[v] + own[v];
        out_a[v] = a.lv.q_ref[v] + out[v];
      }
      if (f % 2 == 0) {                  // the neighbour is the '-' side
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
        common_flux3(out_a, own_a, dq, nx, ny, nz, sm, a.gas, fh);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
        common_flux3(own_a, out_a, dq, nx, ny, nz, sm, a.gas, fh);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) SJ(f, kf, v, el) = fh[v] - floc[v];
    }
  }
  sync3<C::NT>();

  double Fv[NV];
  {
    double qc[NV];
    conservative3(qa, a.gas, qc);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double dv = 0.0;
      if (pt) {
#pragma unroll
        for (int m = 0; m < N1; ++m) {
          dv += o.D[i * N1 + m] * SF(0, v, m + N1 * (j + N1 * k), el);
          dv += o.D[j * N1 + m] * SF(1, v, i + N1 * (m + N1 * k), el);
          dv += o.D[k * N1 + m] * SF(2, v, i + N1 * (j + N1 * m), el);
        }
        dv += o.gL[i] * SJ(0, j + N1 * k, v, el) + o.gR[i] * SJ(1, j + N1 * k, v, el);
        dv += o.gL[j] * SJ(2, i + N1 * k, v, el) + o.gR[j] * SJ(3, i + N1 * k, v, el);
        dv += o.gL[k] * SJ(4, i + N1 * j, v, el) + o.gR[k] * SJ(5, i + N1 * j, v, el);
      }
      const double fv = -dv * ij - a.c_mass * qc[v] + srcv[v] - sv[v];
      Fv[v] = valid ? fv : 0.0;
    }
  }

  if (a.part) {   // per-workgroup sums of F^2 per variable (fixed order, no atomics)
    double s2[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s2[v] = Fv[v] * Fv[v];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s2[v] += __shfl_xor(s2[v], off, 64);
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s_red[wave * NV + v] = s2[v];
    }
    sync3<C::NT>();
    if (tid == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double t = 0.0;
        for (int w = 0; w < C::NW; ++w) t += s_red[w * NV + v];
        a.part[(size_t)blockIdx.x * NV + v] = t;
      }
    }
  }

  if constexpr (MODE == 0) {
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.F[v * sstride + gp] = Fv[v];
    }
  } else {
    sync3<C::NT>();                       // every read of F~ is done: the matvec vectors reuse it
    double* s_fe = s_fgh;                 // [EPW][NPAD], index p Nv + v (padding rows zero)
    double* s_dq = s_fgh + NPAD * EPW;
    if (pt) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s_fe[el * NPAD + p * NV + v] = Fv[v];
    }
    if constexpr (NPAD > N) {
      if (tid < EPW * (NPAD - N)) s_fe[(tid / (NPAD - N)) * NPAD + N + tid % (NPAD - N)] = 0.0;
    }
    sync3<C::NT>();
    if (tid < EPW * C::MVL) {
      const int el2 = tid / C::MVL, l = tid % C::MVL;
      const int e2 = xcd_group(blockIdx.x, gridDim.x) * EPW + el2;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (e2 < ne) {
        const double* fe = s_fe + el2 * NPAD;
        const size_t cs = (size_t)ne * NPAD;
        if constexpr (MODE == 2) {
          const float* w0 = static_cast<const float*>(a.W) + (size_t)e2 * NPAD + 4 * l;
          float accf[4] = {0.f, 0.f, 0.f, 0.f};
          auto matvec = [&](auto nt) {
            // block columns requested before the first is waited for: all 40 at P1 and 24 at P2
            // (8 -> 16 made the sphere levels 9-10% faster, 16 -> 24 with non-temporal loads 3%:
            // more bytes in flight per CU), 8 at P3 (more gains nothing there)
#pragma unroll (N <= 40 ? 40 : N <= 135 ? 24 : 8)
            for (int c = 0; c < N; ++c) {
              const blk_f4 w = load_block4<decltype(nt)::value>(w0 + c * cs);
              const float fc = (float)fe[c];
              accf[0] = fmaf(w.x, fc, accf[0]);
              accf[1] = fmaf(w.y, fc, accf[1]);
              accf[2] = fmaf(w.z, fc, accf[2]);
              accf[3] = fmaf(w.w, fc, accf[3]);
            }
          };
          if (a.w_stream)
            matvec(std::true_type{});
          else
            matvec(std::false_type{});
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t] = (double)accf[t];
        } else {
          const double* w0 = static_cast<const double*>(a.W) + (size_t)e2 * NPAD + 4 * l;
#pragma unroll 4
          for (int c = 0; c < N; ++c) {
            const double2 wa = *reinterpret_cast<const double2*>(w0 + c * cs);
            const double2 wb = *reinterpret_cast<const double2*>(w0 + c * cs + 2);
            const double fc = fe[c];
            acc[0] = fma(wa.x, fc, acc[0]);
            acc[1] = fma(wa.y, fc, acc[1]);
            acc[2] = fma(wb.x, fc, acc[2]);
            acc[3] = fma(wb.y, fc, acc[3]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) s_dq[el2 * NPAD + 4 * l + t] = acc[t];
    }
    sync3<C::NT>();
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.q_out[v * sstride + gp] = qv[v] + a.alpha * s_dq[el * NPAD + p * NV + v];
    }
  }
#undef SQ
#undef SF
#undef SJ
}

// ---- transfers and pointwise helpers ----------------------------------------------------------

struct Mat1D3 {
  double m[kMaxN1 * kMaxN1];
};

// x_c[v][pc][e] = sum R[c][k] R[b][j] R[a][i] x_f[v][i + nf j + nf^2 k][e]
__global__ void __launch_bounds__(256) k_restrict3(int ne, int nvar, int nf1, int nc1, Mat1D3 R,
                                                   const double* __restrict__ xf, double* __restrict__ xc,
                                                   double* __restrict__ xc2) {
  const size_t npc = (size_t)nc1 * nc1 * nc1, npf = (size_t)nf1 * nf1 * nf1;
  const size_t total = (size_t)nvar * npc * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int pc = (int)(rest % npc);
  const int v = (int)(rest / npc);
  const int ca = pc % nc1, cb = (pc / nc1) % nc1, cc = pc / (nc1 * nc1);
  const double* base = xf + (size_t)v * npf * ne + e;
  double acc = 0.0;
  for (int k = 0; k < nf1; ++k) {
    double plane = 0.0;
    for (int j = 0; j < nf1; ++j) {
      double line = 0.0;
      for (int i = 0; i < nf1; ++i) line += R.m[ca * nf1 + i] * base[(size_t)(i + nf1 * (j + nf1 * k)) * ne];
      plane += R.m[cb * nf1 + j] * line;
    }
    acc += R.m[cc * nf1 + k] * plane;
  }
  xc[idx] = acc;
  if (xc2) xc2[idx] = acc;
}

// The same restriction sum-factorised for fixed sizes: one thread per (element, variable, coarse
// plane cc) contracts the element's fine values along k first (each fine value read once per
// plane), then along i and j in registers
template <int NF, int NC>
__global__ void __launch_bounds__(256) k_restrict3t(int ne, int nvar, Mat1D3 R, const double* __restrict__ xf,
                                                    double* __restrict__ xc, double* __restrict__ xc2) {
  const size_t total = (size_t)nvar * NC * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int cc = (int)(rest % NC), v = (int)(rest / NC);
  const double* base = xf + (size_t)v * NF * NF * NF * ne + e;
  double t[NF][NF];                 // t[j][i] = sum_k R[cc][k] x[i][j][k]
#pragma unroll
  for (int j = 0; j < NF; ++j)
#pragma unroll
    for (int i = 0; i < NF; ++i) t[j][i] = 0.0;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const double rk = R.m[cc * NF + k];
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int i = 0; i < NF; ++i) t[j][i] += rk * base[(size_t)(i + NF * (j + NF * k)) * ne];
  }
  double* out = xc + ((size_t)v * NC * NC * NC + (size_t)NC * NC * cc) * ne + e;
  double* out2 = xc2 ? xc2 + ((size_t)v * NC * NC * NC + (size_t)NC * NC * cc) * ne + e : nullptr;
#pragma unroll
  for (int ca = 0; ca < NC; ++ca) {
    double u[NF];                   // u[j] = sum_i R[ca][i] t[j][i]
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i) a += R.m[ca * NF + i] * t[j][i];
      u[j] = a;
    }
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < NF; ++j) a += R.m[cb * NF + j] * u[j];
      out[(size_t)(ca + NC * cb) * ne] = a;
      if (out2) out2[(size_t)(ca + NC * cb) * ne] = a;
    }
  }
}

// The same prolongation sum-factorised: one thread per (element, variable, fine plane fk)
template <int NC, int NF>
__global__ void __launch_bounds__(256) k_prolong3t(int ne, int nvar, Mat1D3 I, const double* __restrict__ xa,
                                                   const double* __restrict__ xb, double* __restrict__ xf) {
  const size_t total = (size_t)nvar * NF * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int fk = (int)(rest % NF), v = (int)(rest / NF);
  const size_t off = (size_t)v * NC * NC * NC * ne + e;
  double t[NC][NC];                 // t[b][a] = sum_c I[fk][c] d[a][b][c]
#pragma unroll
  for (int b = 0; b < NC; ++b)
#pragma unroll
    for (int a2 = 0; a2 < NC; ++a2) t[b][a2] = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double ic = I.m[fk * NC + c];
#pragma unroll
    for (int b = 0; b < NC; ++b)
#pragma unroll
      for (int a2 = 0; a2 < NC; ++a2) {
        const size_t o = off + (size_t)(a2 + NC * (b + NC * c)) * ne;
        const double d = xb ? (xa[o] - xb[o]) : xa[o];
        t[b][a2] += ic * d;
      }
  }
  double* out = xf + ((size_t)v * NF * NF * NF + (size_t)NF * NF * fk) * ne + e;
#pragma unroll
  for (int fi = 0; fi < NF; ++fi) {
    double u[NC];                   // u[b] = sum_a I[fi][a] t[b][a]
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      double a = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < NC; ++a2) a += I.m[fi * NC + a2] * t[b][a2];
      u[b] = a;
    }
#pragma unroll
    for (int fj = 0; fj < NF; ++fj) {
      double a = 0.0;
#pragma unroll
      for (int b = 0; b < NC; ++b) a += I.m[fj * NC + b] * u[b];
      out[(size_t)(fi + NF * fj) * ne] += a;
    }
  }
}

// x_f[v][pf][e] += sum I[k][c] I[j][b] I[i][a] (xa - xb)[v][a + nc b + nc^2 c][e]
__global__ void __launch_bounds__(256) k_prolong3(int ne, int nvar, int nc1, int nf1, Mat1D3 I,
                                                  const double* __restrict__ xa, const double* __restrict__ xb,
                                                  double* __restrict__ xf) {
  const size_t npc = (size_t)nc1 * nc1 * nc1, npf = (size_t)nf1 * nf1 * nf1;
  const size_t total = (size_t)nvar * npf * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int e = (int)(idx % ne);
  const size_t rest = idx / ne;
  const int pf = (int)(rest % npf);
  const int v = (int)(rest / npf);
  const int fi = pf % nf1, fj = (pf / nf1) % nf1, fk = pf / (nf1 * nf1);
  const size_t off = (size_t)v * npc * ne + e;
  double acc = 0.0;
  for (int c = 0; c < nc1; ++c) {
    double plane = 0.0;
    for (int b = 0; b < nc1; ++b) {
      double line = 0.0;
      for (int a2 = 0; a2 < nc1; ++a2) {
        const size_t o = off + (size_t)(a2 + nc1 * (b + nc1 * c)) * ne;
        const double d = xb ? (xa[o] - xb[o]) : xa[o];
        line += I.m[fi * nc1 + a2] * d;
      }
      plane += I.m[fj * nc1 + b] * line;
    }
    acc += I.m[fk * nc1 + c] * plane;
  }
  xf[idx] += acc;
}

struct Ref5 {
  double v[5];
};

__global__ void __launch_bounds__(256) k_conservative3(int n_points, GasParams g, Ref5 ref,
                                                       const double* __restrict__ q, double* __restrict__ qc) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n_points) return;
  double qv[5], out[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qv[v] = ref.v[v] + q[(size_t)v * n_points + idx];
  conservative3(qv, g, out);
#pragma unroll
  for (int v = 0; v < 5; ++v) qc[(size_t)v * n_points + idx] = out[v];
}

// pseudo-time scale of eq. (33) per solution point, h_e / (c + |v|), as the 2-D kernel
__global__ void __launch_bounds__(256) k_dtau_partial3(int ne, int np, const double* __restrict__ q,
                                                       const double* __restrict__ hdx, Ref5 ref, double gr,
                                                       double* __restrict__ part) {
  __shared__ double red[256];
  const size_t total = (size_t)np * ne, st = total;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  double val = 1.0e300;
  if (i < total) {
    const int e = (int)(i % (size_t)ne);
    const double u = q[st + i] + ref.v[1], v = q[2 * st + i] + ref.v[2], w = q[3 * st + i] + ref.v[3];
    const double t = q[4 * st + i] + ref.v[4];
    const double speed = sqrt(gr * t) + sqrt(u * u + v * v + w * w);
    const double h = hdx[e] / speed;
    val = (t > 0.0 && h > 0.0 && h < 1.0e300) ? h : -1.0;
  }
  red[threadIdx.x] = val;
  __syncthreads();
  for (int w2 = 128; w2 > 0; w2 >>= 1) {
    if ((int)threadIdx.x < w2) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- launchers -------------------------------------------------------------------------------

static unsigned blocks3(size_t n) { return (unsigned)((n + 255) / 256); }

int residual_blocks3(const pmg_level_s& L) {
  const int epw = L.epw > 0 ? L.epw : epw3_for(L.P);
  return (L.ne + epw - 1) / epw;
}

int default_epw3(int P) { return epw3_for(P); }

int epw3_candidates(int P, int* out) {
  int n = 0;
  out[n++] = epw3_for(P);
  const int all[6] = {2, 4, 8, 16, 32, 64};
  for (int c : all)
    if (c != epw3_for(P) && epw3_candidate(P, c)) out[n++] = c;
  return n;
}

template <int P, int MODE, int EPW>
static hipError_t launch_fr3_e(const ResArgs3& a, int ne, hipStream_t st) {
  using C = Cfg3<P, EPW>;
  const int blocks = (ne + EPW - 1) / EPW;
  hipLaunchKernelGGL((k_fr3<P, MODE, EPW>), dim3(blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int P, int MODE>
static hipError_t launch_fr3_p(const ResArgs3& a, int ne, int epw, hipStream_t st) {
  constexpr int DEF = epw3_for(P);
  if (epw <= 0 || epw == DEF) return launch_fr3_e<P, MODE, DEF>(a, ne, st);
  if constexpr (DEF != 2 && epw3_candidate(P, 2))
    if (epw == 2) return launch_fr3_e<P, MODE, 2>(a, ne, st);
  if constexpr (DEF != 4 && epw3_candidate(P, 4))
    if (epw == 4) return launch_fr3_e<P, MODE, 4>(a, ne, st);
  if constexpr (DEF != 16 && epw3_candidate(P, 16))
    if (epw == 16) return launch_fr3_e<P, MODE, 16>(a, ne, st);
  if constexpr (DEF != 64 && epw3_candidate(P, 64))
    if (epw == 64) return launch_fr3_e<P, MODE, 64>(a, ne, st);
  return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t launch_fr3(int P, const ResArgs3& a, int ne, int epw, hipStream_t st) {
  switch (P) {
    case 0: return launch_fr3_p<0, MODE>(a, ne, epw, st);
    case 1: return launch_fr3_p<1, MODE>(a, ne, epw, st);
    case 2: return launch_fr3_p<2, MODE>(a, ne, epw, st);
    case 3: return launch_fr3_p<3, MODE>(a, ne, epw, st);
    default: return hipErrorInvalidValue;
  }
}

static ResArgs3 base_args3(const pmg_level_s& L) {
  ResArgs3 a{};
  a.lv = L.view();
  a.ops = L.ops;
  a.gas = L.gas;
  return a;
}

hipError_t launch_residual3(const pmg_level_s& L, const double* q, const double* src, const double* S,
                            double c_mass, double* F, bool want_norms, hipStream_t st, double* part) {
  ResArgs3 a = base_args3(L);
  a.q = q;
  a.src = src;
  a.S = S;
  a.c_mass = c_mass;
  a.F = F;
  a.part = want_norms ? (part ? part : L.part) : nullptr;
  return launch_fr3<0>(L.P, a, L.ne, L.epw, st);
}

hipError_t launch_sweep3(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                         const double* src, const double* S, double c_mass, double alpha, bool want_norms,
                         hipStream_t st) {
  ResArgs3 a = base_args3(L);
  a.q = q_in;
  a.src = src;
  a.S = S;
  a.c_mass = c_mass;
  a.part = want_norms ? L.part : nullptr;
  a.W = fac.W;
  a.alpha = alpha;
  a.q_out = q_out;
  const size_t npad = (size_t)(L.n + 3) / 4 * 4;
  a.w_stream = fac.precision == 32 && (size_t)L.ne * L.n * npad * 4 > kStreamBlocksBytes;
  if (fac.precision == 32) return launch_fr3<2>(L.P, a, L.ne, L.epw, st);
  return launch_fr3<1>(L.P, a, L.ne, L.epw, st);
}

hipError_t launch_restrict3(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                            double* xc, int nvar, hipStream_t st, double* xc2) {
  Mat1D3 R{};
  for (int k = 0; k < Lc.n1 * Lf.n1; ++k) R.m[k] = R1[k];
  const size_t total = (size_t)nvar * Lc.np * Lc.ne;
  if (total == 0) return hipSuccess;
  const size_t tt = (size_t)nvar * Lc.n1 * Lc.ne;   // threads of the sum-factorised kernels
#define PMG_RESTRICT3(NF, NC)                                                                            \
  if (Lf.n1 == NF && Lc.n1 == NC) {                                                                      \
    hipLaunchKernelGGL((k_restrict3t<NF, NC>), dim3(blocks3(tt)), dim3(256), 0, st, Lf.ne, nvar, R, xf, xc, xc2); \
    return hipGetLastError();                                                                            \
  }
  PMG_RESTRICT3(4, 3) PMG_RESTRICT3(3, 2) PMG_RESTRICT3(2, 1) PMG_RESTRICT3(4, 2) PMG_RESTRICT3(4, 1)
  PMG_RESTRICT3(3, 1)
#undef PMG_RESTRICT3
  hipLaunchKernelGGL(k_restrict3, dim3(blocks3(total)), dim3(256), 0, st, Lf.ne, nvar, Lf.n1, Lc.n1, R, xf, xc,
                     xc2);
  return hipGetLastError();
}

hipError_t launch_prolong3(const pmg_level_s& Lc, const pmg_level_s& Lf, const double* I1, const double* xa,
                           const double* xb, double* xf, int nvar, hipStream_t st) {
  Mat1D3 I{};
  for (int k = 0; k < Lc.n1 * Lf.n1; ++k) I.m[k] = I1[k];
  const size_t total = (size_t)nvar * Lf.np * Lf.ne;
  if (total == 0) return hipSuccess;
  const size_t tt = (size_t)nvar * Lf.n1 * Lf.ne;   // threads of the sum-factorised kernels
#define PMG_PROLONG3(NC, NF)                                                                             \
  if (Lc.n1 == NC && Lf.n1 == NF) {                                                                      \
    hipLaunchKernelGGL((k_prolong3t<NC, NF>), dim3(blocks3(tt)), dim3(256), 0, st, Lf.ne, nvar, I, xa, xb, xf); \
    return hipGetLastError();                                                                            \
  }
  PMG_PROLONG3(3, 4) PMG_PROLONG3(2, 3) PMG_PROLONG3(1, 2) PMG_PROLONG3(2, 4) PMG_PROLONG3(1, 4)
  PMG_PROLONG3(1, 3)
#undef PMG_PROLONG3
  hipLaunchKernelGGL(k_prolong3, dim3(blocks3(total)), dim3(256), 0, st, Lf.ne, nvar, Lc.n1, Lf.n1, I, xa, xb,
                     xf);
  return hipGetLastError();
}

hipError_t launch_conservative3(const pmg_level_s& L, const double* q, double* qc, hipStream_t st) {
  const int npts = L.np * L.ne;
  if (npts == 0) return hipSuccess;
  Ref5 ref{};
  for (int k = 0; k < 5; ++k) ref.v[k] = L.q_ref[k];
  hipLaunchKernelGGL(k_conservative3, dim3(blocks3(npts)), dim3(256), 0, st, npts, L.gas, ref, q, qc);
  return hipGetLastError();
}

hipError_t launch_dtau_partial3(const pmg_level_s& L, const double* q, int nblk, hipStream_t st) {
  Ref5 ref{};
  for (int k = 0; k < 5; ++k) ref.v[k] = L.q_ref[k];
  hipLaunchKernelGGL(k_dtau_partial3, dim3(nblk), dim3(256), 0, st, L.ne, L.np, q, L.hdx, ref,
                     L.gas.gamma * L.gas.rgas, L.dtpart);
  return hipGetLastError();
}

}  // namespace pmg
