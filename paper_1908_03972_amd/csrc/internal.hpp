// Library-internal types shared by the host orchestration and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "physics.hpp"

namespace pmg {

// Workgroups are dispatched to the device's eight XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has its own L2. A kernel whose workgroup b covers element group g reads the
// element-fastest arrays ([variable][point][element]) in runs of (elements per group) x 8 bytes;
// groups that share a 128-byte line must run on one XCD or every XCD fetches the whole line. The
// element group of workgroup b among nb: XCD x takes a contiguous range of groups (the first
// nb mod 8 XCDs one group more), in the order its workgroups are dispatched.
__device__ __forceinline__ int xcd_group(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd, x = b % kXcd, k = b / kXcd;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

constexpr int kMaxN1 = 7;   // P <= 6
constexpr int kNv2 = 4;     // 2-D primitive variables (p, u, v, T)

// 1-D operators of one polynomial degree on Gauss points, passed to kernels by value.
struct Ops1D {
  int n1;
  double D[kMaxN1 * kMaxN1];   // D[i*n1 + k] = l_k'(x_i)
  double lm[kMaxN1];           // l_k(-1)
  double lp[kMaxN1];           // l_k(+1)
  double gL[kMaxN1];           // g_L'(x_i)
  double gR[kMaxN1];           // g_R'(x_i)
};

// Device view of one level's geometry and connectivity.
struct LevelView {
  int ne;
  const double* met;    // 2-D [5][Np][Ne]: Sx, Sy (= y_eta, -x_eta), Tx, Ty (= -y_xi, x_xi), 1/|J|;
                        // 3-D [10][Np][Ne]: J grad xi^d (component n at 3 d + n), 1/|J|
  const double* fvec;   // 2-D [4][n1][3][Ne]: unit +xi (faces 0,1) or +eta (faces 2,3) normal and its
                        // length |S|; 3-D [6][n1^2][4][Ne]: unit +xi^(f/2) normal and |S|
  const int* nbr;       // [2 dim][Ne]
  const int* nbf;       // [4][Ne]
  const int* ori;       // [4][Ne]
  double q_ref[5];      // stored states are q - q_ref (4 variables in 2-D, 5 in 3-D)
  double qinf_g[5];     // far-field state in stored form, q_inf - q_ref
  const double* lam;    // [4][n1][Ne] BR2 lifting factor of each flux point (viscous levels)
  const double* gface;  // [4][n1][4][2][Ne] local gradient traces of the current state (viscous levels)
};

struct KernelStatus {
  int* flag;            // device int: bit 0 singular pivot, bit 1 non-finite value
};

}  // namespace pmg

struct pmg_level_s {
  int dim = 2, P = 0, n1 = 1, np = 1, nv = 4, n = 4, ne = 0, geom_order = 1, device = 0;
  int npad = 4;                     // row stride of the stored inverse blocks (n, or n rounded up to 4 in 3-D)
  pmg::GasParams gas{};
  double q_inf[5] = {0, 0, 0, 0, 0};
  double q_ref[5] = {0, 0, 0, 0, 0};
  pmg::Ops1D ops{};
  std::vector<double> x1, w1;       // 1-D Gauss points/weights
  std::vector<double> xy_host;      // [dim][Np][Ne] solution-point coordinates
  // device geometry
  double* met = nullptr;
  double* fvec = nullptr;
  int* nbr = nullptr;
  int* nbf = nullptr;
  int* ori = nullptr;
  // device workspace (allocated once at creation)
  double* wq = nullptr;      // sweep ping-pong state
  double* wF = nullptr;      // residual / defect
  double* wS = nullptr;      // FAS forcing S_l
  double* wqb = nullptr;     // restricted state q^b_l
  double* wql = nullptr;     // working state q_l of a coarse level
  double* wsrc = nullptr;    // ESDIRK source (finest level)
  double* part = nullptr;    // per-workgroup norm partials
  double* norms = nullptr;   // [Nv + 1]
  int* flag = nullptr;       // device error flags
  int part_blocks = 0;       // workgroups of the fused residual/sweep kernel (norm partials in use)
  int epw = 0;               // elements per workgroup of the fused kernel (0: the default for P)
  std::vector<double> dx_host;     // [Ne] element length scale of eqs. (32)-(33)
  double* hdx = nullptr;           // [Ne] device: dx_e / (P + 1)
  double* dtpart = nullptr;        // per-workgroup partial minima of the pseudo-time scale
  double* dtmin = nullptr;         // device scalar: dtau_min
  int visc = 0;                    // mu > 0: BR2 viscous terms
  double* lam = nullptr;           // [4][n1][Ne] lambda_f,k = sum_m l_m(face) g_f'(x_m) / |J_m|
  double* gface = nullptr;         // [4][n1][4][2][Ne] local gradient traces (pre-pass output)
  double* Dv = nullptr;            // [Ne][n][n] viscous part dR_vis/dq of the element blocks
  // replayable V-cycle of the stage solve (finest level only), keyed by its arguments
  hipGraphExec_t vc_exec = nullptr;
  hipStream_t capture_stream = nullptr;
  std::vector<uintptr_t> vc_key;
  // host side of the stage solve's lookahead (finest level only): two pinned copies of the norms
  // ([2][8]) and the events that mark their arrival
  double* hnorm = nullptr;
  hipEvent_t ev_norm[2] = {nullptr, nullptr};
  size_t state_elems() const { return (size_t)nv * np * ne; }
  pmg::LevelView view() const {
    pmg::LevelView v;
    v.ne = ne;
    v.met = met;
    v.fvec = fvec;
    v.nbr = nbr;
    v.nbf = nbf;
    v.ori = ori;
    for (int k = 0; k < 5; ++k) {
      v.q_ref[k] = q_ref[k];
      v.qinf_g[k] = q_inf[k] - q_ref[k];
    }
    v.lam = lam;
    v.gface = gface;
    return v;
  }
};

namespace pmg {
struct LineFactors;
}

struct pmg_factors_s {
  pmg_level_s* L = nullptr;
  int precision = 64;     // 64: FP64 inverse blocks; 32: FP32 inverse blocks
  void* W = nullptr;      // [n][Ne][npad] element inverse blocks, column-major per element
  size_t bytes = 0;
  double* ws = nullptr;   // 3-D P = 3 (and P = 2 with FP32 inverses): ws_slots x n x n FP64 work slots (P = 3), then every element's pointwise derivatives
  int ws_slots = 0;
  pmg::LineFactors* lines = nullptr;   // element-line Jacobi instead of element Jacobi (lines.hpp)
};

namespace pmg {

// kernel launchers (fr_kernels.hip, jac_kernels.hip, transfer_kernels.hip)
// with want_norms, the per-workgroup partial sums of F^2 go to `part` (residual_blocks(L) x Nv
// doubles) when given, else to the level's workspace
hipError_t launch_residual(const pmg_level_s& L, const double* q, const double* src, const double* S,
                           double c_mass, double* F, bool want_norms, hipStream_t st, double* part = nullptr);
hipError_t launch_sweep(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                        const double* src, const double* S, double c_mass, double alpha, bool want_norms,
                        hipStream_t st);
hipError_t launch_norm_finalize(const pmg_level_s& L, hipStream_t st);
// norms[v] and the composite norm from nblk x nv partial sums into a caller's device array
hipError_t launch_norm_finalize_to(const double* part, int nblk, int nv, double* norms, hipStream_t st);
// records the message pmg_last_error returns (for entry points outside api.cpp)
int32_t set_error(int32_t code, const char* msg);   // a pmg_status
hipError_t launch_jacobian(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                           pmg_factors_s& fac, hipStream_t st);
hipError_t launch_restrict(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                           double* xc, int nvar, hipStream_t st, double* xc2 = nullptr);
hipError_t launch_copy(size_t n, const double* src, double* dst, hipStream_t st);
hipError_t launch_prolong(const pmg_level_s& Lc, const pmg_level_s& Lf, const double* I1, const double* xa,
                          const double* xb, double* xf, int nvar, hipStream_t st);
hipError_t launch_conservative(const pmg_level_s& L, const double* q, double* qc, hipStream_t st);
// q = the explicit predictor of a stage, q_c^n + dt (sum_j a_j R_j + omega R_{n_prev - 1}), in
// primitive offsets
hipError_t launch_stage_predict(const pmg_level_s& L, const double* qc_n, const double* const* R, const double* a,
                                int n_prev, double dt, double omega, double* q, hipStream_t st);
hipError_t launch_stage_source(const pmg_level_s& L, const double* qc_n, const double* const* R, const double* a,
                               int n_prev, double dt, double c_mass, double* src, hipStream_t st);
int residual_blocks(const pmg_level_s& L);
// 2-D fused kernel: the default elements per workgroup at degree P; the tuner's candidates for a
// level, 2-D or 3-D (the default first; at most 4)
int default_epw(int P);
int epw_candidates(const pmg_level_s& L, int* out);
hipError_t launch_gradient_traces(const pmg_level_s& L, const double* q, hipStream_t st);
hipError_t launch_visc_jacobian(const pmg_level_s& L, const double* q, hipStream_t st);
int dtau_blocks(const pmg_level_s& L);
hipError_t launch_dtau_min(const pmg_level_s& L, const double* q, hipStream_t st);

// hexahedral levels (fr3_kernels.hip; element blocks in jac3_kernels.hip)
int residual_blocks3(const pmg_level_s& L);
int default_epw3(int P);
int epw3_candidates(int P, int* out);
hipError_t launch_residual3(const pmg_level_s& L, const double* q, const double* src, const double* S,
                            double c_mass, double* F, bool want_norms, hipStream_t st, double* part = nullptr);
hipError_t launch_sweep3(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                         const double* src, const double* S, double c_mass, double alpha, bool want_norms,
                         hipStream_t st);
hipError_t launch_jacobian3(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                            pmg_factors_s& fac, hipStream_t st);
hipError_t launch_restrict3(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                            double* xc, int nvar, hipStream_t st, double* xc2);
hipError_t launch_prolong3(const pmg_level_s& Lc, const pmg_level_s& Lf, const double* I1, const double* xa,
                           const double* xb, double* xf, int nvar, hipStream_t st);
hipError_t launch_conservative3(const pmg_level_s& L, const double* q, double* qc, hipStream_t st);
hipError_t launch_dtau_partial3(const pmg_level_s& L, const double* q, int nblk, hipStream_t st);

// hexahedral geometry (hex_geometry.cpp)
std::string build_hex_geometry(const double* nodes, int ne, int g, int P, const std::vector<double>& x1,
                               std::vector<double>& met, std::vector<double>& fvec, std::vector<double>& xyz,
                               std::vector<double>& dx);

}  // namespace pmg
