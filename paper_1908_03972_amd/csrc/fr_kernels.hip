// FR/CPR residual and fused element-Jacobi sweep kernels (2-D quadrilaterals).
//
// One workgroup owns EPW elements; thread (p, el) owns solution point p of element el (and flux
// point p of the element's faces), so that loads of the [Nv][Np][Ne] state are coalesced over
// consecutive elements. Per workgroup:
//   1. point states and transformed fluxes F~ = f.S, G~ = f.T go to LDS;
//   2. each element's 4(P+1) flux points: own trace (extrapolated along the tensor line), the
//      neighbour's trace (extrapolated from the neighbour's state) or a boundary ghost, the
//      common flux of eq. (21) and its jump against the interpolated local flux;
//   3. R = -(1/|J|)[line derivatives + g_L'/g_R' corrections] (eq. (20)), F = R - c q_c + src - S.
// With a viscosity (VISC) the BR2 terms of Sec. 2.3 join: local gradients at the points (chain
// rule), each face's jump (q_com - q) N, the common viscous flux from both sides' gradient traces
// and liftings (the neighbour's traces come from the pre-pass k_grad), the corrected gradient
// grad q + sum of the liftings, and the viscous fluxes are subtracted from F~, G~ and F^.
// The sweep variant then multiplies F by the element's stored inverse block (eq. (30)), with the
// workgroup re-mapped element-major so that the n x n block stream is read fully coalesced, and
// writes q + alpha D^{-1} F to a second buffer (synchronous Jacobi: neighbours are read from the
// input buffer only).
#include "internal.hpp"
#include "vcycle.hpp"
#include "block_loads.hpp"

namespace pmg {

constexpr int kPadding = -100;   // neighbour tag of the padding elements of the last workgroup
// LDS budget of a one-wave sweep workgroup that stages inverse-block columns ahead of its matvec:
// 8 such workgroups (the 2 waves per SIMD that ~200 VGPRs allow) share a CU's 160 KB
constexpr int kLdsTarget = 19968;

// Block columns (of n) that fit in `bytes` of LDS when staged 64 chunks of 16 B at a time, cl chunks
// per column.
constexpr int staged_columns(int n, int cl, int bytes) {
  int c = 0;
  while (c < n && ((c + 1) * cl + 63) / 64 * 1024 <= bytes) ++c;
  return c;
}

// Workgroup barrier. A one-wave workgroup needs none: the LDS accesses of a wave complete in
// program order, so wavefront-scope fences (which order the compiler, and wait for nothing) suffice;
// in particular they do not wait for the direct global->LDS loads still in flight.
template <int NT>
__device__ __forceinline__ void block_sync() {
  if constexpr (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Elements per workgroup. Lanes are (point, element) with the element fastest, so a load of one
// (variable, point) of the [Nv][Np][Ne] state by a wave covers EPW consecutive elements: 16-32
// elements fill whole cache lines, where 4-5 used a third of each (measured: P3 and P4 sweeps
// 10-25% faster at 16 and 20 than at 4 and 5; at P2 and P4, 16 beats 20 by 6-9%: 256 rather than
// 205 workgroups on a 4096-element level). Each element gets max((P+1)^2, 4(P+1)) lanes, so
// that every flux point of its four faces has a lane of its own (at P <= 2 the faces have more
// flux points than the element has solution points).
constexpr int epw_for(int P) {
  return P == 0 ? 32 : P == 1 ? 8 : P == 2 ? 16 : P == 3 ? 16 : P == 4 ? 16 : P == 5 ? 3 : 5;
}
constexpr int lanes_per_element(int P) { return (P + 1) * (P + 1) > 4 * (P + 1) ? (P + 1) * (P + 1) : 4 * (P + 1); }

// The tuner's candidates on inviscid levels (pmg_level_autotune): the default and the others whose
// registers still fit the workgroup (P4 at 32 elements would spill). Viscous levels and P >= 5
// keep the default.
constexpr bool epw_candidate(int P, int epw) {
  return epw == epw_for(P) || (P == 0 && (epw == 16 || epw == 64)) ||
         (P >= 1 && P <= 3 && (epw == 8 || epw == 16 || epw == 32)) || (P == 4 && epw == 8);
}

template <int P, int EPW_ = epw_for(P)>
struct Cfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1;
  static constexpr int NV = 4;
  static constexpr int N = NV * NP;
  static constexpr int EPW = EPW_;
  static constexpr int LPE = lanes_per_element(P);
  static constexpr int NACT = EPW * LPE;   // lanes with an element slot
  static constexpr int NPT = EPW * NP;     // lanes that own a solution point
  static constexpr int NT = ((NACT + 63) / 64) * 64;
  static constexpr int NW = NT / 64;
};

struct ResArgs {
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
  double* S_out;   // non-null: S held P w, the defect is P w and S_out receives F(q) - P w
  int w_stream;    // FP32 blocks larger than the Infinity Cache: non-temporal loads
};

// MODE 0: residual only; 1: sweep with FP64 inverse blocks; 2: sweep with FP32 inverse blocks
template <int P, int MODE, bool VISC, int EPW_ = epw_for(P)>
__global__ void __launch_bounds__((Cfg<P, EPW_>::NT)) k_fr(ResArgs a) {
  using C = Cfg<P, EPW_>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, N = C::N, EPW = C::EPW;
  constexpr int VS = VISC ? 1 : 0;          // viscous LDS arrays exist only when used
  __shared__ double s_q[NV * NP * EPW];
  // F~ then G~ in one array: LDS accesses index their variable directly (no selected pointers),
  // which lets them be told apart from the staged block columns
  __shared__ double s_fg[2 * NV * NP * EPW];
  __shared__ double s_j[4 * N1 * NV * EPW];
  __shared__ double s_red[C::NW * NV];
  // the 1-D operators: dynamically indexed, so they would otherwise be global loads from the
  // argument block in the middle of the kernel, queued behind any block columns being staged
  __shared__ double s_ops[N1 * N1 + 4 * N1];
  __shared__ double s_gl[VS * NV * 2 * NP * EPW + 1];      // local gradients
  __shared__ double s_jn[VS * 4 * N1 * NV * 2 * EPW + 1];  // (q_com - q) N per flux point
  __shared__ double s_fv[VS * NV * NP * EPW + 1];          // viscous F~v
  __shared__ double s_gv[VS * NV * NP * EPW + 1];          // viscous G~v
  // FP32 sweeps at P <= 3 stage the first CPF columns of the workgroup's inverse blocks in LDS
  // with direct global->LDS loads issued in the middle of the residual phase, so that part of
  // the block stream is in flight while the common fluxes and the divergence are computed
  constexpr bool PREF = (MODE == 2) && (P == 3) && !VISC && (C::NT == 64);
  constexpr int BASE_LDS = 8 * (3 * NV * NP * EPW + 4 * N1 * NV * EPW + C::NW * NV + N1 * N1 + 4 * N1) + 64;
  constexpr int SW_CL = EPW * N / 4;        // 16-B chunks per block column of the workgroup
  constexpr int CPF = PREF ? staged_columns(N, SW_CL, kLdsTarget - BASE_LDS) : 0;
  constexpr int SW_CHUNKS = CPF * SW_CL;
  constexpr int SW_INSTR = (SW_CHUNKS + 63) / 64;
  __shared__ __align__(16) float s_w[PREF ? SW_INSTR * 256 : 1];
  // block columns a lane requests before it waits for the first: enough 16-B loads in flight per
  // wave to cover the memory latency at the one or two waves per SIMD these kernels run at
  constexpr int MV_UNROLL = (N - CPF) <= 40 ? 40 : 8;
  constexpr int MV_UNROLL64 = N <= 20 ? 20 : 8;

  const int ne = a.lv.ne;
  const int tid = threadIdx.x;
  const bool act = tid < C::NACT;
  const int el = tid % EPW;
  const int p = act ? tid / EPW : 0;
  const bool pt = act && p < NP;            // this lane owns solution point p
  const int e = xcd_group(blockIdx.x, gridDim.x) * EPW + el;
  const bool valid = pt && e < ne;
  const int i = p % N1, j = p / N1;
  static_assert(N1 * N1 + 4 * N1 <= C::NT, "one lane per operator entry");
  double opv = 0.0;                         // this lane's operator entry, stored before the first barrier
  {
    // lm, lp, gL, gR follow D in the operator block, each kMaxN1 entries long
    static_assert(offsetof(Ops1D, lm) == offsetof(Ops1D, D) + 8 * kMaxN1 * kMaxN1 &&
                      offsetof(Ops1D, gR) == offsetof(Ops1D, lm) + 8 * 3 * kMaxN1,
                  "operator block layout");
    const int r = tid - N1 * N1;
    const int idx = tid < N1 * N1 ? tid : kMaxN1 * kMaxN1 + (r / N1) * kMaxN1 + r % N1;
    const double* ops = reinterpret_cast<const double*>(reinterpret_cast<const char*>(&a.ops) + offsetof(Ops1D, D));
    if (tid < N1 * N1 + 4 * N1) opv = ops[idx];
  }
  struct {
    const double *D, *lm, *lp, *gL, *gR;
  } const o = {s_ops, s_ops + N1 * N1, s_ops + N1 * N1 + N1, s_ops + N1 * N1 + 2 * N1, s_ops + N1 * N1 + 3 * N1};
  const size_t sstride = (size_t)NP * ne;   // stride between variables in the state layout

#define SQ(v, pp, ee) s_q[((v) * NP + (pp)) * EPW + (ee)]
#define SF(v, pp, ee) s_fg[((v) * NP + (pp)) * EPW + (ee)]
#define SG(v, pp, ee) s_fg[((NV + (v)) * NP + (pp)) * EPW + (ee)]
#define SJ(f, k, v, ee) s_j[(((f) * N1 + (k)) * NV + (v)) * EPW + (ee)]
#define SGL(v, d, pp, ee) s_gl[((((v) * 2 + (d)) * NP) + (pp)) * EPW + (ee)]
#define SJN(f, k, v, d, ee) s_jn[(((((f) * N1 + (k)) * NV + (v)) * 2) + (d)) * EPW + (ee)]
#define SFV(v, pp, ee) s_fv[((v) * NP + (pp)) * EPW + (ee)]
#define SGV(v, pp, ee) s_gv[((v) * NP + (pp)) * EPW + (ee)]

  const size_t gp = (size_t)p * ne + e;     // offset of (v=0, p, e)
  // every lane loads a state without a branch: lanes without a point of a real element take a
  // point of the last element (a physical state that keeps their discarded arithmetic finite)
  const size_t gpl = (size_t)(pt ? p : 0) * ne + (e < ne ? e : ne - 1);
  double qv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) qv[v] = a.q[v * sstride + gpl];
  double qa[NV];                            // absolute primitive state q_ref + stored offset
#pragma unroll
  for (int v = 0; v < NV; ++v) qa[v] = a.lv.q_ref[v] + qv[v];

  // every operand of this point is requested up front, before the first barrier
  double ij = 0.0, sx = 1.0, sy = 0.0, tx = 0.0, ty = 1.0;
  double srcv[NV], sv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    srcv[v] = 0.0;
    sv[v] = 0.0;
  }
  if (valid) {
    const double* m = a.lv.met;
    sx = m[gp];
    sy = m[sstride + gp];
    tx = m[2 * sstride + gp];
    ty = m[3 * sstride + gp];
    ij = m[4 * sstride + gp];
    if (a.src) {
#pragma unroll
      for (int v = 0; v < NV; ++v) srcv[v] = a.src[v * sstride + gp];
    }
    if (a.S) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sv[v] = a.S[v * sstride + gp];
    }
  }
  // this lane's flux point of its element's faces (each element has a lane for every one of its
  // 4 (P+1) flux points): face vector and neighbour, then the neighbour's state along the tensor
  // line through the point, in flight while the point fluxes are computed. The gathers and the
  // block-column staging are issued by every lane without a branch, so that the wait for the
  // gathers in the face phase is a count that leaves the staged columns in flight.
  static_assert(C::LPE >= 4 * N1, "one lane per flux point");
  const bool fpt = act && p < 4 * N1;
  const int f = p / N1, k = p % N1;
  double nx = (f < 2) ? 1.0 : 0.0, ny = (f < 2) ? 0.0 : 1.0, sm = 1.0;
  int nb = kPadding, nf = 0, ori = 0;
  if (fpt && e < ne) {
    const size_t fo = ((size_t)(f * N1 + k) * 3) * ne + e;
    nx = a.lv.fvec[fo];
    ny = a.lv.fvec[fo + ne];
    sm = a.lv.fvec[fo + 2 * ne];
    nb = a.lv.nbr[f * ne + e];
    nf = a.lv.nbf[f * ne + e];
    ori = a.lv.ori[f * ne + e];
  }
  const int kk = ori ? (N1 - 1 - k) : k;
  double nq[N1][NV];                        // the neighbour's states on the line through the flux point
  const bool hasn = nb >= 0;                // without a neighbour, any element's values (unused)
  const int nfc = hasn ? nf : 0;
  {
    const int nbc = hasn ? nb : 0, kkc = hasn ? kk : 0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      const int pp = (nfc < 2) ? (m + N1 * kkc) : (kkc + N1 * m);
#pragma unroll
      for (int v = 0; v < NV; ++v) nq[m][v] = a.q[v * sstride + (size_t)pp * ne + nbc];
    }
  }
  const double rho = qa[0] / (a.gas.rgas * qa[3]);
  {
    double fs[NV], ft[NV];
    normal_flux2_rho(qa, rho, sx, sy, a.gas, fs);
    normal_flux2_rho(qa, rho, tx, ty, a.gas, ft);
    if (pt) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        SQ(v, p, el) = qv[v];
        SF(v, p, el) = fs[v];
        SG(v, p, el) = ft[v];
      }
    }
  }
  if (tid < N1 * N1 + 4 * N1) s_ops[tid] = opv;
  block_sync<C::NT>();

  if constexpr (VISC) {                     // local gradient (chain rule) at this point
    if (pt) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double dxi = 0.0, deta = 0.0;
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          dxi += o.D[i * N1 + k] * SQ(v, k + N1 * j, el);
          deta += o.D[j * N1 + k] * SQ(v, i + N1 * k, el);
        }
        SGL(v, 0, p, el) = ij * (sx * dxi + tx * deta);
        SGL(v, 1, p, el) = ij * (sy * dxi + ty * deta);
      }
    }
    block_sync<C::NT>();
  }

  const double* w = o.lm + ((f == 0 || f == 2) ? 0 : N1);   // lm or lp along this face's lines
  double own[NV], floc[NV], out[NV];        // own trace, interpolated local flux, outside state
  {
    // the neighbour's trace, formed by every lane so that every path has consumed the gathers
    // before the direct-to-LDS loads below are issued
    const double* wn = o.lm + ((nfc == 0 || nfc == 2) ? 0 : N1);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] += wn[m] * nq[m][v];
    }
  }
  if (fpt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      own[v] = 0.0;
      floc[v] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      const int pp = (f < 2) ? (m + N1 * k) : (k + N1 * m);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        own[v] += w[m] * SQ(v, pp, el);
        floc[v] += w[m] * s_fg[(((f < 2 ? 0 : NV) + v) * NP + pp) * EPW + el];
      }
    }
    if (nb >= 0) {                     // interior face: the neighbour's trace formed above
    } else if (nb == -1) {             // slip wall: reflect the normal velocity
      const double ua = a.lv.q_ref[1] + own[1], va = a.lv.q_ref[2] + own[2];
      const double un = ua * nx + va * ny;
      out[0] = own[0];
      out[1] = ua - 2.0 * un * nx - a.lv.q_ref[1];
      out[2] = va - 2.0 * un * ny - a.lv.q_ref[2];
      out[3] = own[3];
    } else if (nb == -2) {             // far field
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = a.lv.qinf_g[v];
    } else if (nb == -3) {             // no-slip wall: reverse the velocity
      out[0] = own[0];
      out[1] = -(a.lv.q_ref[1] + own[1]) - a.lv.q_ref[1];
      out[2] = -(a.lv.q_ref[2] + own[2]) - a.lv.q_ref[2];
      out[3] = own[3];
    } else {                           // padding element of the last workgroup
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = own[v];
    }
  }
  if constexpr (PREF) {
    // The workgroup's part of the first CPF block columns is CPF x EPW N/4 chunks of 16 B,
    // contiguous per column; wave instruction it stages chunks 64 it .. 64 it + 63 (lane l writes
    // s_w[4 (64 it + l)], the layout [column][element][row]); lanes past the last chunk and chunks
    // of elements past the end re-read a valid chunk into the padding or an unused slot. Issued
    // once the neighbour gathers are consumed: the compiler's wait for any load issued before a
    // direct-to-LDS load also waits for the latter.
    const int e0 = xcd_group(blockIdx.x, gridDim.x) * EPW;
    const float* wb = static_cast<const float*>(a.W);
#pragma unroll
    for (int it = 0; it < SW_INSTR; ++it) {
      int g = it * 64 + tid;
      g = g < SW_CHUNKS ? g : SW_CHUNKS - 1;
      const int c = g / SW_CL, r4 = 4 * (g - c * SW_CL);
      int ee = e0 + r4 / N;
      ee = ee < ne ? ee : ne - 1;
      __builtin_amdgcn_global_load_lds((const void*)(wb + ((size_t)c * ne + ee) * N + r4 % N),
                                       (void*)(s_w + it * 256), 16, 0, 0);
    }
  }
  if (fpt) {
    {
      double own_a[NV], out_a[NV], dq[NV], fh[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        own_a[v] = a.lv.q_ref[v] + own[v];
        out_a[v] = a.lv.q_ref[v] + out[v];
      }
      if (f == 0 || f == 2) {            // the neighbour is the '-' side
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[v] = own[v] - out[v];
        common_flux2(out_a, own_a, dq, nx, ny, sm, a.gas, fh);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[v] = out[v] - own[v];
        common_flux2(own_a, out_a, dq, nx, ny, sm, a.gas, fh);
      }
      if constexpr (VISC) {
        double gown[NV][2], gout[NV][2], jn[NV][2], fhv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          gown[v][0] = gown[v][1] = gout[v][0] = gout[v][1] = 0.0;
        }
#pragma unroll
        for (int m = 0; m < N1; ++m) {
          const int pp = (f < 2) ? (m + N1 * k) : (k + N1 * m);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            gown[v][0] += w[m] * SGL(v, 0, pp, el);
            gown[v][1] += w[m] * SGL(v, 1, pp, el);
          }
        }
        double lam = 0.0, nbx = 0.0, nby = 0.0, nbsm = 0.0, nblam = 0.0;
        int kind = 1;
        if (e < ne) lam = a.lv.lam[(size_t)(f * N1 + k) * ne + e];
        if (nb >= 0) {
          kind = 0;
          const size_t fo = ((size_t)(nf * N1 + kk) * 3) * ne + nb;
          nbx = a.lv.fvec[fo];
          nby = a.lv.fvec[fo + ne];
          nbsm = a.lv.fvec[fo + 2 * ne];
          nblam = a.lv.lam[(size_t)(nf * N1 + kk) * ne + nb];
          const double* gf = a.lv.gface + (size_t)((nf * N1 + kk) * NV * 2) * ne + nb;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            gout[v][0] = gf[(size_t)(v * 2) * ne];
            gout[v][1] = gf[(size_t)(v * 2 + 1) * ne];
          }
        } else if (nb == -3) {
          kind = 2;
        } else if (nb == -2) {
          kind = 3;
        }
        visc_face2(own, out, a.lv.q_ref, gown, gout, nx, ny, sm, lam, nbx, nby, nbsm, nblam, kind, a.gas, jn,
                   fhv);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          SJ(f, k, v, el) = fh[v] - floc[v] - fhv[v];
          SJN(f, k, v, 0, el) = jn[v][0];
          SJN(f, k, v, 1, el) = jn[v][1];
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) SJ(f, k, v, el) = fh[v] - floc[v];
      }
    }
  }
  block_sync<C::NT>();

  if constexpr (VISC) {                     // corrected gradient and the viscous point fluxes
    if (pt) {
      double gc[NV][2];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const double lift = o.gL[i] * SJN(0, j, v, d, el) + o.gR[i] * SJN(1, j, v, d, el) +
                              o.gL[j] * SJN(2, i, v, d, el) + o.gR[j] * SJN(3, i, v, d, el);
          gc[v][d] = SGL(v, d, p, el) + ij * lift;
        }
      }
      double fx[NV], fy[NV];
      visc_flux2(qa[1], qa[2], gc, a.gas, fx, fy);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        SFV(v, p, el) = sx * fx[v] + sy * fy[v];
        SGV(v, p, el) = tx * fx[v] + ty * fy[v];
      }
    }
    block_sync<C::NT>();
  }

  double Fv[NV];
  {
    double qc[NV];
    qc[0] = rho;
    qc[1] = rho * qa[1];
    qc[2] = rho * qa[2];
    qc[3] = qa[0] * (1.0 / (a.gas.gamma - 1.0)) + 0.5 * rho * (qa[1] * qa[1] + qa[2] * qa[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double d = 0.0;
      if (pt) {
        if constexpr (VISC) {             // total flux f_inv - f_vis; the jumps gain the
          double fl0 = 0.0, fl1 = 0.0, gl2 = 0.0, gl3 = 0.0;   // interpolated local viscous flux
#pragma unroll
          for (int k = 0; k < N1; ++k) {
            const double fvk = SFV(v, k + N1 * j, el), gvk = SGV(v, i + N1 * k, el);
            d += o.D[i * N1 + k] * (SF(v, k + N1 * j, el) - fvk) + o.D[j * N1 + k] * (SG(v, i + N1 * k, el) - gvk);
            fl0 += o.lm[k] * fvk;
            fl1 += o.lp[k] * fvk;
            gl2 += o.lm[k] * gvk;
            gl3 += o.lp[k] * gvk;
          }
          d += o.gL[i] * (SJ(0, j, v, el) + fl0) + o.gR[i] * (SJ(1, j, v, el) + fl1);
          d += o.gL[j] * (SJ(2, i, v, el) + gl2) + o.gR[j] * (SJ(3, i, v, el) + gl3);
        } else {
#pragma unroll
          for (int k = 0; k < N1; ++k) d += o.D[i * N1 + k] * SF(v, k + N1 * j, el);
          d += o.gL[i] * SJ(0, j, v, el) + o.gR[i] * SJ(1, j, v, el);
#pragma unroll
          for (int k = 0; k < N1; ++k) d += o.D[j * N1 + k] * SG(v, i + N1 * k, el);
          d += o.gL[j] * SJ(2, i, v, el) + o.gR[j] * SJ(3, i, v, el);
        }
      }
      const double fraw = -d * ij - a.c_mass * qc[v] + srcv[v];
      const double fv = a.S_out ? sv[v] : fraw - sv[v];
      if (a.S_out && valid) a.S_out[v * sstride + gp] = fraw - sv[v];
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
    block_sync<C::NT>();
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
    if constexpr (PREF) __builtin_amdgcn_s_waitcnt(0);   // the staged block columns have landed
    block_sync<C::NT>();                  // all reads of F~ / G~ are done
    double* s_fe = s_fg + NV * NP * EPW;  // [EPW][N], index p*Nv + v
    double* s_dq = s_fg;                  // [EPW][N]
    if (pt) {
#pragma unroll
      for (int v = 0; v < NV; ++v) s_fe[el * N + p * NV + v] = Fv[v];
    }
    block_sync<C::NT>();
    if (tid < C::NPT) {
      const int el2 = tid / NP, p2 = tid % NP;
      const int e2 = xcd_group(blockIdx.x, gridDim.x) * EPW + el2;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (e2 < ne) {
        const double* fe = s_fe + el2 * N;
        const size_t cs = (size_t)ne * N;            // stride between block columns
        if constexpr (MODE == 2) {
          const float* w0 = static_cast<const float*>(a.W) + (size_t)e2 * N + 4 * p2;
          float accf[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
          for (int c = 0; c < CPF; ++c) {
            const float4 w = *reinterpret_cast<const float4*>(s_w + c * EPW * N + el2 * N + 4 * p2);
            const float fc = (float)fe[c];
            accf[0] = fmaf(w.x, fc, accf[0]);
            accf[1] = fmaf(w.y, fc, accf[1]);
            accf[2] = fmaf(w.z, fc, accf[2]);
            accf[3] = fmaf(w.w, fc, accf[3]);
          }
          auto matvec = [&](auto nt) {
#pragma unroll MV_UNROLL
            for (int c = CPF; c < N; ++c) {
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
          for (int v = 0; v < 4; ++v) acc[v] = (double)accf[v];
        } else {
          const double* w0 = static_cast<const double*>(a.W) + (size_t)e2 * N + 4 * p2;
#pragma unroll MV_UNROLL64
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
      for (int v = 0; v < 4; ++v) s_dq[el2 * N + p2 * NV + v] = acc[v];
    }
    block_sync<C::NT>();
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.q_out[v * sstride + gp] = qv[v] + a.alpha * s_dq[el * N + p * NV + v];
    }
  }
#undef SQ
#undef SF
#undef SG
#undef SJ
#undef SGL
#undef SJN
#undef SFV
#undef SGV
}

// Local gradients (chain rule on the solution polynomial) extrapolated to the flux points of
// every face, gface[f][k][v][d][e]: what the BR2 common gradient of a viscous residual needs from
// each neighbour. Same thread layout as k_fr.
template <int P>
__global__ void __launch_bounds__(Cfg<P>::NT) k_grad(LevelView lv, Ops1D o, const double* __restrict__ q,
                                                     double* __restrict__ gface) {
  using C = Cfg<P>;
  constexpr int N1 = C::N1, NP = C::NP, NV = C::NV, EPW = C::EPW;
  __shared__ double s_q[NV * NP * EPW];
  __shared__ double s_gl[NV * 2 * NP * EPW];
  const int ne = lv.ne;
  const int tid = threadIdx.x;
  const bool act = tid < C::NACT;
  const int el = tid % EPW;
  const int p = act ? tid / EPW : 0;
  const bool pt = act && p < NP;
  const int e = xcd_group(blockIdx.x, gridDim.x) * EPW + el;
  const bool valid = pt && e < ne;
  const int i = p % N1, j = p / N1;
  const size_t sstride = (size_t)NP * ne, gp = (size_t)p * ne + e;
  double sx = 1.0, sy = 0.0, tx = 0.0, ty = 1.0, ij = 0.0;
  if (valid) {
    sx = lv.met[gp];
    sy = lv.met[sstride + gp];
    tx = lv.met[2 * sstride + gp];
    ty = lv.met[3 * sstride + gp];
    ij = lv.met[4 * sstride + gp];
  }
  if (pt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) s_q[(v * NP + p) * EPW + el] = valid ? q[v * sstride + gp] : 0.0;
  }
  __syncthreads();
  if (pt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double dxi = 0.0, deta = 0.0;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        dxi += o.D[i * N1 + k] * s_q[(v * NP + k + N1 * j) * EPW + el];
        deta += o.D[j * N1 + k] * s_q[(v * NP + i + N1 * k) * EPW + el];
      }
      s_gl[((v * 2 + 0) * NP + p) * EPW + el] = ij * (sx * dxi + tx * deta);
      s_gl[((v * 2 + 1) * NP + p) * EPW + el] = ij * (sy * dxi + ty * deta);
    }
  }
  __syncthreads();
  if (act && e < ne) {
    for (int t = p; t < 4 * N1; t += C::LPE) {
      const int f = t / N1, k = t % N1;
      const double* w = (f == 0 || f == 2) ? o.lm : o.lp;
#pragma unroll
      for (int vd = 0; vd < NV * 2; ++vd) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
          const int pp = (f < 2) ? (m + N1 * k) : (k + N1 * m);
          acc += w[m] * s_gl[(vd * NP + pp) * EPW + el];
        }
        gface[((size_t)(f * N1 + k) * NV * 2 + vd) * ne + e] = acc;
      }
    }
  }
}

template <int P, int MODE, bool VISC, int EPW>
static hipError_t launch_fr_e(const ResArgs& a, int ne, hipStream_t st) {
  using C = Cfg<P, EPW>;
  const int blocks = (ne + EPW - 1) / EPW;
  hipLaunchKernelGGL((k_fr<P, MODE, VISC, EPW>), dim3(blocks), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int P, int MODE>
static hipError_t launch_fr_p(const ResArgs& a, int ne, bool visc, int epw, hipStream_t st) {
  constexpr int DEF = epw_for(P);
  if (visc) return launch_fr_e<P, MODE, true, DEF>(a, ne, st);
  if (epw <= 0 || epw == DEF) return launch_fr_e<P, MODE, false, DEF>(a, ne, st);
  if constexpr (DEF != 8 && epw_candidate(P, 8))
    if (epw == 8) return launch_fr_e<P, MODE, false, 8>(a, ne, st);
  if constexpr (DEF != 16 && epw_candidate(P, 16))
    if (epw == 16) return launch_fr_e<P, MODE, false, 16>(a, ne, st);
  if constexpr (DEF != 32 && epw_candidate(P, 32))
    if (epw == 32) return launch_fr_e<P, MODE, false, 32>(a, ne, st);
  if constexpr (DEF != 64 && epw_candidate(P, 64))
    if (epw == 64) return launch_fr_e<P, MODE, false, 64>(a, ne, st);
  return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t launch_fr(int P, const ResArgs& a, int ne, bool visc, int epw, hipStream_t st) {
  switch (P) {
    case 0: return launch_fr_p<0, MODE>(a, ne, visc, epw, st);
    case 1: return launch_fr_p<1, MODE>(a, ne, visc, epw, st);
    case 2: return launch_fr_p<2, MODE>(a, ne, visc, epw, st);
    case 3: return launch_fr_p<3, MODE>(a, ne, visc, epw, st);
    case 4: return launch_fr_p<4, MODE>(a, ne, visc, epw, st);
    case 5: return launch_fr_p<5, MODE>(a, ne, visc, epw, st);
    case 6: return launch_fr_p<6, MODE>(a, ne, visc, epw, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
static hipError_t launch_grad_p(const pmg_level_s& L, const double* q, hipStream_t st) {
  using C = Cfg<P>;
  const int blocks = (L.ne + C::EPW - 1) / C::EPW;
  hipLaunchKernelGGL((k_grad<P>), dim3(blocks), dim3(C::NT), 0, st, L.view(), L.ops, q, L.gface);
  return hipGetLastError();
}

hipError_t launch_gradient_traces(const pmg_level_s& L, const double* q, hipStream_t st) {
  switch (L.P) {
    case 0: return launch_grad_p<0>(L, q, st);
    case 1: return launch_grad_p<1>(L, q, st);
    case 2: return launch_grad_p<2>(L, q, st);
    case 3: return launch_grad_p<3>(L, q, st);
    case 4: return launch_grad_p<4>(L, q, st);
    case 5: return launch_grad_p<5>(L, q, st);
    case 6: return launch_grad_p<6>(L, q, st);
    default: return hipErrorInvalidValue;
  }
}

int residual_blocks(const pmg_level_s& L) {
  if (L.dim == 3) return residual_blocks3(L);
  const int epw = L.epw > 0 ? L.epw : epw_for(L.P);
  return (L.ne + epw - 1) / epw;
}

int default_epw(int P) { return epw_for(P); }

int epw_candidates(const pmg_level_s& L, int* out) {
  int n = 0;
  if (L.dim == 3) return epw3_candidates(L.P, out);
  out[n++] = epw_for(L.P);
  if (L.visc) return n;
  const int all[4] = {8, 16, 32, 64};
  for (int c : all)
    if (c != epw_for(L.P) && epw_candidate(L.P, c)) out[n++] = c;
  return n;
}

static ResArgs base_args(const pmg_level_s& L) {
  ResArgs a{};
  a.lv = L.view();
  a.ops = L.ops;
  a.gas = L.gas;
  return a;
}

hipError_t launch_residual(const pmg_level_s& L, const double* q, const double* src, const double* S,
                           double c_mass, double* F, bool want_norms, hipStream_t st, double* part) {
  if (L.dim == 3) return launch_residual3(L, q, src, S, c_mass, F, want_norms, st, part);
  ResArgs a = base_args(L);
  a.q = q;
  a.src = src;
  a.S = S;
  a.c_mass = c_mass;
  a.F = F;
  a.part = want_norms ? (part ? part : L.part) : nullptr;
  if (L.visc) {
    const hipError_t e = launch_gradient_traces(L, q, st);
    if (e != hipSuccess) return e;
  }
  return launch_fr<0>(L.P, a, L.ne, L.visc != 0, L.epw, st);
}

static hipError_t launch_sweep2(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                                const double* src, const double* S, double* S_out, double c_mass, double alpha,
                                bool want_norms, hipStream_t st) {
  ResArgs a = base_args(L);
  a.q = q_in;
  a.src = src;
  a.S = S;
  a.S_out = S_out;
  a.c_mass = c_mass;
  a.part = want_norms ? L.part : nullptr;
  a.W = fac.W;
  a.alpha = alpha;
  a.q_out = q_out;
  a.w_stream = fac.precision == 32 && (size_t)L.ne * L.n * L.n * 4 > kStreamBlocksBytes;
  if (L.visc) {
    const hipError_t e = launch_gradient_traces(L, q_in, st);
    if (e != hipSuccess) return e;
  }
  if (fac.precision == 32) return launch_fr<2>(L.P, a, L.ne, L.visc != 0, L.epw, st);
  return launch_fr<1>(L.P, a, L.ne, L.visc != 0, L.epw, st);
}

hipError_t launch_sweep(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                        const double* src, const double* S, double c_mass, double alpha, bool want_norms,
                        hipStream_t st) {
  if (L.dim == 3) return launch_sweep3(L, fac, q_in, q_out, src, S, c_mass, alpha, want_norms, st);
  return launch_sweep2(L, fac, q_in, q_out, src, S, nullptr, c_mass, alpha, want_norms, st);
}

hipError_t launch_sweep_forming_S(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                                  double* S, double c_mass, double alpha, hipStream_t st) {
  if (L.dim == 3) {
    const hipError_t e = launch_residual3(L, q_in, nullptr, S, c_mass, S, false, st);
    if (e != hipSuccess) return e;
    return launch_sweep3(L, fac, q_in, q_out, nullptr, S, c_mass, alpha, false, st);
  }
  return launch_sweep2(L, fac, q_in, q_out, nullptr, S, S, c_mass, alpha, false, st);
}

}  // namespace pmg
