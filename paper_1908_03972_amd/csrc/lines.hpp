// Element-line Jacobi on quadrilateral levels: the state a line-smoother factor set keeps and its
// kernel launchers (line_kernels.hip).
#pragma once

#include "internal.hpp"

namespace pmg {

constexpr int kLineMaxP = 4;   // a line workgroup holds one n x n block in LDS (n = 100 at P = 4)

struct LineFactors {
  int n_lines = 0, K = 0;      // lines of K elements each; n_lines * K = Ne
  int* elems = nullptr;        // device [n_lines][K] element indices in line order
  int* pos = nullptr;          // device [Ne]: line * K + position of the element in its line
  int* fside = nullptr;        // device [2][Ne]: face of e towards the previous / next element of its
                               // line, -1 at the line's ends
  double* D = nullptr;         // device [Ne][n][n] row-major FP64: element blocks of the last factorisation
  void* Winv = nullptr;        // device [Ne][n][n] at the factor precision, column-major per element
                               // ([e][c][r]): W_k = D'_k^{-1} of the block-Thomas elimination
  double* Kc = nullptr;        // device [2][Ne][n1][4][4]: derivative of |S| f_com at each flux point of the
                               // face towards the previous / next element with respect to that
                               // neighbour's trace
  double* r = nullptr;         // device state-sized work array: F - S
  // The substitutions pass only face traces along a line (see line_kernels.hip):
  void* C = nullptr;           // device [Ne][NJ][n] at the factor precision: C_k = W_k P_m K_m (column-major)
  void* B = nullptr;           // device [Ne][NJ][n] at the factor precision: B_k = W_k P_p K_p
  double* M = nullptr;         // device [n_lines][K][NJ][NJ] by line position: M_k = E_{k+1} C_k
                               // (column-major), zero at the line ends
  double* N = nullptr;         // device [n_lines][K][NJ][NJ]: N_k = E_{k-1} B_k, zero at the line ends
  double* z = nullptr;         // device [Ne][n] element-major: W_k r_k, then y_k
  double* tr = nullptr;        // device [4][n_lines][K][NJ] by line position: u, t, v, s traces of the
                               // substitutions
};

// NJ = 4 (P + 1): the rank of a coupling block (4 variables at the P + 1 flux points of a face)
inline int line_rank(int P) { return 4 * (P + 1); }

// D_e (and D_out, if given), the coupling derivatives and the block-Thomas inverses of every line
hipError_t launch_line_factor(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                              pmg_factors_s& fac, hipStream_t st);
// one line-Jacobi sweep in place: q += alpha A_line^{-1} (F(q) - S), with the norms of F(q) - S
hipError_t launch_line_sweep(const pmg_level_s& L, const pmg_factors_s& fac, double* q, const double* src,
                             const double* S, double c_mass, double alpha, bool want_norms, hipStream_t st);
// the coupling blocks of the last factorisation written out dense, [Ne][n][n] row-major (null skips)
hipError_t launch_line_dense(const pmg_level_s& L, const pmg_factors_s& fac, double* Am, double* Ap,
                             hipStream_t st);

}  // namespace pmg
