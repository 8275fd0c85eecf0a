// Host side of the pmgfr C ABI: level setup (points, 1-D operators, metrics), argument checks,
// kernel sequencing for the smoother and transfers, and the pseudo-transient stage solve with
// FAS V-cycles (Secs. 2.4 and 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/pmgfr.h"
#include "internal.hpp"
#include "jac3.hpp"
#include "krylov.hpp"
#include "lines.hpp"
#include "vcycle.hpp"

using pmg::Ops1D;

namespace {

thread_local std::string g_error;

pmg_status fail(pmg_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

pmg_status hip_fail(hipError_t err, const char* what) {
  return fail(PMG_E_HIP, std::string(what) + ": " + hipGetErrorString(err));
}

#define PMG_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---- 1-D polynomial machinery --------------------------------------------------------------
// Legendre P_n(x) and P_n'(x) by the three-term recurrence and P'_{k+1} = P'_{k-1} + (2k+1) P_k.
void legendre(int n, double x, double& pn, double& dpn) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    pn = 1.0;
    dpn = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    const double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  pn = p1;
  dpn = d1;
}

// Gauss-Legendre points (ascending) and weights by Newton's method on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double xi = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    double pn = 0.0, dpn = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, pn, dpn);
      const double dx = pn / dpn;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre(n, xi, pn, dpn);
    x[n - 1 - k] = xi;
    w[n - 1 - k] = 2.0 / ((1.0 - xi * xi) * dpn * dpn);
  }
}

double lagrange(const std::vector<double>& nodes, int k, double x) {
  double r = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != k) r *= (x - nodes[m]) / (nodes[k] - nodes[m]);
  return r;
}

double lagrange_deriv(const std::vector<double>& nodes, int k, double x) {
  double s = 0.0;
  for (size_t a = 0; a < nodes.size(); ++a) {
    if ((int)a == k) continue;
    double t = 1.0 / (nodes[k] - nodes[a]);
    for (size_t m = 0; m < nodes.size(); ++m)
      if ((int)m != k && m != a) t *= (x - nodes[m]) / (nodes[k] - nodes[m]);
    s += t;
  }
  return s;
}

// Barycentric differentiation matrix D[i][k] = l_k'(x_i) on distinct nodes.
void diff_matrix(const std::vector<double>& x, double* D) {
  const int n = (int)x.size();
  std::vector<double> c(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m)
      if (m != i) c[i] *= (x[i] - x[m]);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int k = 0; k < n; ++k) {
      if (k == i) continue;
      D[i * n + k] = (c[i] / c[k]) / (x[i] - x[k]);
      diag += 1.0 / (x[i] - x[k]);
    }
    D[i * n + i] = diag;
  }
}

// FR correction derivatives with g_R = (L_{P+1} + L_P)/2 (g_DG) and g_L(x) = g_R(-x).
double radau_right_deriv(int P, double x) {
  double a, da, b, db;
  legendre(P + 1, x, a, da);
  legendre(P, x, b, db);
  return 0.5 * (da + db);
}

void build_ops(int P, Ops1D& o, std::vector<double>& x, std::vector<double>& w) {
  const int n1 = P + 1;
  gauss_legendre(n1, x, w);
  std::memset(&o, 0, sizeof(o));
  o.n1 = n1;
  diff_matrix(x, o.D);
  for (int k = 0; k < n1; ++k) {
    o.lm[k] = lagrange(x, k, -1.0);
    o.lp[k] = lagrange(x, k, 1.0);
    o.gR[k] = radau_right_deriv(P, x[k]);
    o.gL[k] = -radau_right_deriv(P, -x[k]);
  }
}

// Restriction (L2 projection onto degree Pc) and prolongation (interpolation) 1-D matrices.
void projection_matrix(const pmg_level_s& f, const pmg_level_s& c, std::vector<double>& R) {
  const int nf = f.n1, nc = c.n1;
  R.assign((size_t)nc * nf, 0.0);
  for (int a = 0; a < nc; ++a)
    for (int i = 0; i < nf; ++i) {
      double s = 0.0;
      for (int k = 0; k <= c.P; ++k) {
        double la, dla, li, dli;
        legendre(k, c.x1[a], la, dla);
        legendre(k, f.x1[i], li, dli);
        s += la * (2.0 * k + 1.0) * 0.5 * f.w1[i] * li;
      }
      R[a * nf + i] = s;
    }
}

void interpolation_matrix(const pmg_level_s& c, const pmg_level_s& f, std::vector<double>& I) {
  const int nf = f.n1, nc = c.n1;
  I.assign((size_t)nf * nc, 0.0);
  for (int i = 0; i < nf; ++i)
    for (int a = 0; a < nc; ++a) I[i * nc + a] = lagrange(c.x1, a, f.x1[i]);
}

// ---- geometry --------------------------------------------------------------------------------
struct MapEval {
  double x, y, x_xi, x_eta, y_xi, y_eta;
};

MapEval map_at(const double* nodes, int g, double xi, double eta) {
  std::vector<double> gn(g + 1);
  for (int a = 0; a <= g; ++a) gn[a] = -1.0 + 2.0 * a / g;
  MapEval m{0, 0, 0, 0, 0, 0};
  for (int b = 0; b <= g; ++b)
    for (int a = 0; a <= g; ++a) {
      const double na = lagrange(gn, a, xi), nb = lagrange(gn, b, eta);
      const double dna = lagrange_deriv(gn, a, xi), dnb = lagrange_deriv(gn, b, eta);
      const double X = nodes[2 * (a + (g + 1) * b)], Y = nodes[2 * (a + (g + 1) * b) + 1];
      m.x += na * nb * X;
      m.y += na * nb * Y;
      m.x_xi += dna * nb * X;
      m.y_xi += dna * nb * Y;
      m.x_eta += na * dnb * X;
      m.y_eta += na * dnb * Y;
    }
  return m;
}

// Twice the smallest distance from the element's area centroid to its faces (eqs. (32)-(33)); the
// centroid integrates the exact mapping with a 6x6 Gauss rule, a face is the segment joining its
// two corner nodes.
double element_length(const double* nodes, int g) {
  std::vector<double> xq, wq;
  gauss_legendre(6, xq, wq);
  double area = 0.0, cx = 0.0, cy = 0.0;
  for (int j = 0; j < 6; ++j)
    for (int i = 0; i < 6; ++i) {
      const MapEval m = map_at(nodes, g, xq[i], xq[j]);
      const double wj = wq[i] * wq[j] * (m.x_xi * m.y_eta - m.x_eta * m.y_xi);
      area += wj;
      cx += wj * m.x;
      cy += wj * m.y;
    }
  cx /= area;
  cy /= area;
  const int n1 = g + 1;
  const int corners[4][2] = {{0, n1 * g}, {g, g + n1 * g}, {0, g}, {n1 * g, g + n1 * g}};
  double dmin = std::numeric_limits<double>::infinity();
  for (const auto& c : corners) {
    const double ax = nodes[2 * c[0]], ay = nodes[2 * c[0] + 1];
    const double bx = nodes[2 * c[1]], by = nodes[2 * c[1] + 1];
    const double ex = bx - ax, ey = by - ay;
    double t = ((cx - ax) * ex + (cy - ay) * ey) / (ex * ex + ey * ey);
    t = std::min(1.0, std::max(0.0, t));
    const double dx = cx - (ax + t * ex), dy = cy - (ay + t * ey);
    dmin = std::min(dmin, std::sqrt(dx * dx + dy * dy));
  }
  return 2.0 * dmin;
}

template <class T>
pmg_status upload(T** dst, const std::vector<T>& src) {
  hipError_t e = hipMalloc(dst, src.size() * sizeof(T));
  if (e != hipSuccess) return fail(PMG_E_NOMEM, "hipMalloc failed for level data");
  e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy level data");
  return PMG_OK;
}

pmg_status alloc_zero(double** dst, size_t n) {
  hipError_t e = hipMalloc(dst, std::max<size_t>(n, 1) * sizeof(double));
  if (e != hipSuccess) return fail(PMG_E_NOMEM, "hipMalloc failed for level workspace");
  e = hipMemset(*dst, 0, std::max<size_t>(n, 1) * sizeof(double));
  if (e != hipSuccess) return hip_fail(e, "hipMemset workspace");
  return PMG_OK;
}

// Pinned norm copies and their events for the stage solve's lookahead.
pmg_status alloc_lookahead(pmg_level_s* L) {
  if (hipHostMalloc(reinterpret_cast<void**>(&L->hnorm), 16 * sizeof(double)) != hipSuccess) {
    L->hnorm = nullptr;
    return fail(PMG_E_NOMEM, "hipHostMalloc failed for the norm copies");
  }
  for (hipEvent_t& ev : L->ev_norm)
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
      return fail(PMG_E_HIP, "hipEventCreateWithFlags");
    }
  return PMG_OK;
}

void free_level(pmg_level_s* L) {
  if (!L) return;
  if (L->vc_exec) (void)hipGraphExecDestroy(L->vc_exec);
  if (L->capture_stream) (void)hipStreamDestroy(L->capture_stream);
  for (hipEvent_t ev : L->ev_norm)
    if (ev) (void)hipEventDestroy(ev);
  if (L->hnorm) (void)hipHostFree(L->hnorm);
  void* ptrs[] = {L->met,  L->fvec,   L->nbr,   L->nbf, L->ori, L->wq,    L->wF,     L->wS,  L->wqb, L->wql,
                  L->wsrc, L->part,   L->norms, L->flag, L->hdx, L->dtpart, L->dtmin, L->lam, L->gface, L->Dv};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete L;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// The smoother's blocks at state q: element inverses, or the block-Thomas factors of line factors.
hipError_t build_blocks(const pmg_level_s& L, const double* q, double dtau, double c_mass, double* D_out,
                        pmg_factors_s& fac, hipStream_t st) {
  if (fac.lines) return pmg::launch_line_factor(L, q, dtau, c_mass, D_out, fac, st);
  return pmg::launch_jacobian(L, q, dtau, c_mass, D_out, fac, st);
}

// n synchronous element-Jacobi sweeps ping-ponging between q and the level's workspace (kernels
// only, so the sequence can be captured in a graph); optional norms of the first sweep's F and
// F_after = F(q) - S at the final state. Line factors sweep in place instead (a residual, then
// the line solves).
// n sweeps; with form_S (a coarse level at its restricted state, S holding P w) the first sweep
// also turns S into the level's forcing (n must then be >= 1)
pmg_status run_sweeps(pmg_level_s& L, const pmg_factors_s& fac, double* q, const double* src, const double* S,
                      double c_mass, int n, double alpha, double* F_after, bool norms, hipStream_t st,
                      double* form_S = nullptr) {
  if (fac.lines) {
    if (form_S) {                         // S_{l+1} = F(q^b) - P w first, then ordinary sweeps
      PMG_HIP(pmg::launch_residual(L, q, nullptr, form_S, c_mass, form_S, false, st));
      S = form_S;
    }
    for (int k = 0; k < n; ++k) {
      const bool nrm = norms && k == 0;
      PMG_HIP(pmg::launch_line_sweep(L, fac, q, src, S, c_mass, alpha, nrm, st));
      if (nrm) PMG_HIP(pmg::launch_norm_finalize(L, st));
    }
    if (F_after) {
      const bool nrm = norms && n == 0;
      PMG_HIP(pmg::launch_residual(L, q, src, S, c_mass, F_after, nrm, st));
      if (nrm) PMG_HIP(pmg::launch_norm_finalize(L, st));
    }
    return PMG_OK;
  }
  double* in = q;
  double* out = L.wq;
  for (int k = 0; k < n; ++k) {
    const bool nrm = norms && k == 0;
    if (k == 0 && form_S)
      PMG_HIP(pmg::launch_sweep_forming_S(L, fac, in, out, form_S, c_mass, alpha, st));
    else
      PMG_HIP(pmg::launch_sweep(L, fac, in, out, src, S, c_mass, alpha, nrm, st));
    if (nrm) PMG_HIP(pmg::launch_norm_finalize(L, st));
    std::swap(in, out);
  }
  if (in != q) PMG_HIP(pmg::launch_copy(L.state_elems(), in, q, st));
  if (F_after) {
    const bool nrm = norms && n == 0;
    PMG_HIP(pmg::launch_residual(L, q, src, S, c_mass, F_after, nrm, st));
    if (nrm) PMG_HIP(pmg::launch_norm_finalize(L, st));
  }
  return PMG_OK;
}

pmg_status check_level(pmg_level L) {
  if (!L) return fail(PMG_E_ARG, "null level handle");
  return PMG_OK;
}

}  // namespace

pmg_status pmg::set_error(pmg_status code, const char* msg) { return fail(code, msg); }

// =============================================================================================
extern "C" {

const char* pmg_last_error(void) { return g_error.c_str(); }

int32_t pmg_abi_version(void) { return PMG_ABI_VERSION; }

// A hexahedral level (dim = 3): P <= 3, inviscid, slip-wall and far-field boundaries, face
// orientation codes 0..7 (see the header).
static pmg_status create_hex_level(const pmg_level_desc* d, pmg_level* out) {
  if (d->P < 0 || d->P > 3) return fail(PMG_E_ARG, "3-D levels support P in 0..3");
  if (d->geom_order != 1 && d->geom_order != 2) return fail(PMG_E_ARG, "geom_order must be 1 or 2");
  if (d->n_elements <= 0) return fail(PMG_E_ARG, "n_elements must be positive");
  if (!d->nodes || !d->face_nbr || !d->face_nbr_face || !d->face_orient) return fail(PMG_E_ARG, "null mesh array");
  if (!(d->gamma > 1.0) || !(d->rgas > 0.0)) return fail(PMG_E_ARG, "gamma must exceed 1 and rgas be positive");
  if (d->eps_mode != 0 && d->eps_mode != 1) return fail(PMG_E_ARG, "eps_mode must be 0 or 1");
  if (d->mu != 0.0) return fail(PMG_E_ARG, "3-D levels are inviscid (mu must be 0)");
  const int ne = d->n_elements;
  for (int k = 0; k < 6 * ne; ++k) {
    const int nb = d->face_nbr[k];
    if (nb >= ne || nb < PMG_BC_FAR_FIELD) return fail(PMG_E_ARG, "face_nbr entry out of range (3-D: >= -2)");
    if (nb >= 0 && (d->face_nbr_face[k] < 0 || d->face_nbr_face[k] > 5))
      return fail(PMG_E_ARG, "face_nbr_face entry out of range");
    if (d->face_orient[k] < 0 || d->face_orient[k] > 7) return fail(PMG_E_ARG, "face_orient must be in 0..7");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d->device < 0 || d->device >= ndev)
    return fail(PMG_E_ARG, "invalid HIP device ordinal");
  DeviceGuard guard(d->device);
  if (!guard.ok) return fail(PMG_E_HIP, "hipSetDevice failed");

  pmg_level_s* L = new pmg_level_s();
  L->dim = 3;
  L->P = d->P;
  L->n1 = d->P + 1;
  L->np = L->n1 * L->n1 * L->n1;
  L->nv = 5;
  L->n = L->nv * L->np;
  L->npad = (L->n + 3) / 4 * 4;
  L->ne = ne;
  L->geom_order = d->geom_order;
  L->device = d->device;
  L->gas.gamma = d->gamma;
  L->gas.rgas = d->rgas;
  L->gas.cp = d->gamma * d->rgas / (d->gamma - 1.0);
  L->gas.ma_inf = d->ma_inf;
  L->gas.kappa = d->kappa;
  L->gas.eps_mode = d->eps_mode;
  for (int k = 0; k < 5; ++k) {
    L->q_inf[k] = d->q_inf[k];
    L->q_ref[k] = d->q_ref[k];
  }
  build_ops(d->P, L->ops, L->x1, L->w1);
  std::vector<double> met, fvec, dx;
  const std::string why = pmg::build_hex_geometry(d->nodes, ne, d->geom_order, d->P, L->x1, met, fvec, L->xy_host, dx);
  if (!why.empty()) {
    free_level(L);
    return fail(PMG_E_ARG, why);
  }
  L->dx_host = dx;
  std::vector<double> hdx(ne);
  for (int e = 0; e < ne; ++e) hdx[e] = dx[e] / L->n1;
  std::vector<int> nbr((size_t)6 * ne), nbf((size_t)6 * ne), ori((size_t)6 * ne);
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < 6; ++f) {
      nbr[(size_t)f * ne + e] = d->face_nbr[6 * e + f];
      nbf[(size_t)f * ne + e] = d->face_nbr_face[6 * e + f];
      ori[(size_t)f * ne + e] = d->face_orient[6 * e + f];
    }
  pmg_status s = PMG_OK;
  if ((s = upload(&L->met, met)) || (s = upload(&L->fvec, fvec)) || (s = upload(&L->nbr, nbr)) ||
      (s = upload(&L->nbf, nbf)) || (s = upload(&L->ori, ori)) || (s = upload(&L->hdx, hdx))) {
    free_level(L);
    return s;
  }
  const size_t ns = L->state_elems();
  L->epw = pmg::default_epw3(L->P);
  L->part_blocks = pmg::residual_blocks(*L);
  int cand[4], min_epw = L->epw;
  for (int c = 0, nc = pmg::epw_candidates(*L, cand); c < nc; ++c) min_epw = std::min(min_epw, cand[c]);
  const size_t part_max = (size_t)(L->ne + min_epw - 1) / min_epw;   // room for every tuner candidate
  if ((s = alloc_zero(&L->wq, ns)) || (s = alloc_zero(&L->wF, ns)) || (s = alloc_zero(&L->wS, ns)) ||
      (s = alloc_zero(&L->wqb, ns)) || (s = alloc_zero(&L->wql, ns)) || (s = alloc_zero(&L->wsrc, ns)) ||
      (s = alloc_zero(&L->part, part_max * L->nv)) || (s = alloc_zero(&L->norms, L->nv + 1)) ||
      (s = alloc_zero(&L->dtpart, pmg::dtau_blocks(*L))) || (s = alloc_zero(&L->dtmin, 1))) {
    free_level(L);
    return s;
  }
  if (hipMalloc(&L->flag, sizeof(int)) != hipSuccess) {
    free_level(L);
    return fail(PMG_E_NOMEM, "hipMalloc failed for the fault flag");
  }
  if (hipMemset(L->flag, 0, sizeof(int)) != hipSuccess) {
    free_level(L);
    return fail(PMG_E_HIP, "hipMemset fault flag");
  }
  if ((s = alloc_lookahead(L))) {
    free_level(L);
    return s;
  }
  *out = L;
  return PMG_OK;
}

pmg_status pmg_level_create(const pmg_level_desc* d, pmg_level* out) {
  if (!d || !out) return fail(PMG_E_ARG, "null descriptor or output");
  *out = nullptr;
  if (d->dim == 3) return create_hex_level(d, out);
  if (d->dim != 2) return fail(PMG_E_ARG, "dim must be 2 (quadrilaterals) or 3 (hexahedra)");
  if (d->P < 0 || d->P > 6) return fail(PMG_E_ARG, "P must be in 0..6");
  if (d->geom_order != 1 && d->geom_order != 2) return fail(PMG_E_ARG, "geom_order must be 1 or 2");
  if (d->n_elements <= 0) return fail(PMG_E_ARG, "n_elements must be positive");
  if (!d->nodes || !d->face_nbr || !d->face_nbr_face || !d->face_orient)
    return fail(PMG_E_ARG, "null mesh array");
  if (!(d->gamma > 1.0) || !(d->rgas > 0.0)) return fail(PMG_E_ARG, "gamma must exceed 1 and rgas be positive");
  if (d->eps_mode != 0 && d->eps_mode != 1) return fail(PMG_E_ARG, "eps_mode must be 0 or 1");
  if (!(d->mu >= 0.0)) return fail(PMG_E_ARG, "mu must be non-negative");
  if (d->mu > 0.0 && (!(d->prandtl > 0.0) || !(d->br2_penalty > 0.0)))
    return fail(PMG_E_ARG, "a viscous level needs prandtl > 0 and br2_penalty > 0");
  if (d->mu > 0.0 && d->P > 4) return fail(PMG_E_ARG, "viscous levels support P <= 4");
  const int ne = d->n_elements;
  for (int k = 0; k < 4 * ne; ++k) {
    const int nb = d->face_nbr[k];
    if (nb >= ne || nb < PMG_BC_NOSLIP_WALL) return fail(PMG_E_ARG, "face_nbr entry out of range");
    if (nb >= 0 && (d->face_nbr_face[k] < 0 || d->face_nbr_face[k] > 3))
      return fail(PMG_E_ARG, "face_nbr_face entry out of range");
    if (d->face_orient[k] != 0 && d->face_orient[k] != 1) return fail(PMG_E_ARG, "face_orient must be 0 or 1");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d->device < 0 || d->device >= ndev)
    return fail(PMG_E_ARG, "invalid HIP device ordinal");
  DeviceGuard guard(d->device);
  if (!guard.ok) return fail(PMG_E_HIP, "hipSetDevice failed");

  pmg_level_s* L = new pmg_level_s();
  L->dim = 2;
  L->P = d->P;
  L->n1 = d->P + 1;
  L->np = L->n1 * L->n1;
  L->nv = 4;
  L->n = L->nv * L->np;
  L->npad = L->n;
  L->ne = ne;
  L->geom_order = d->geom_order;
  L->device = d->device;
  L->gas.gamma = d->gamma;
  L->gas.rgas = d->rgas;
  L->gas.cp = d->gamma * d->rgas / (d->gamma - 1.0);
  L->gas.ma_inf = d->ma_inf;
  L->gas.kappa = d->kappa;
  L->gas.eps_mode = d->eps_mode;
  L->gas.mu = d->mu;
  L->gas.kcond = d->mu > 0.0 ? d->mu * L->gas.cp / d->prandtl : 0.0;
  L->gas.br2_eta = d->mu > 0.0 ? d->br2_penalty : 0.0;
  L->visc = d->mu > 0.0 ? 1 : 0;
  for (int k = 0; k < 5; ++k) {
    L->q_inf[k] = d->q_inf[k];
    L->q_ref[k] = d->q_ref[k];
  }
  build_ops(d->P, L->ops, L->x1, L->w1);

  // metrics from the exact mapping at solution and flux points
  const int n1 = L->n1, np = L->np, g = d->geom_order, nn = (g + 1) * (g + 1);
  std::vector<double> met((size_t)5 * np * ne), fvec((size_t)4 * n1 * 3 * ne), jacp((size_t)np * ne);
  L->xy_host.assign((size_t)2 * np * ne, 0.0);
  for (int e = 0; e < ne; ++e) {
    const double* nodes = d->nodes + (size_t)e * nn * 2;
    for (int jj = 0; jj < n1; ++jj)
      for (int ii = 0; ii < n1; ++ii) {
        const int p = ii + n1 * jj;
        const MapEval m = map_at(nodes, g, L->x1[ii], L->x1[jj]);
        const double jac = m.x_xi * m.y_eta - m.x_eta * m.y_xi;
        if (!(jac > 0.0)) {
          free_level(L);
          return fail(PMG_E_ARG, "non-positive mapping Jacobian in element " + std::to_string(e));
        }
        const size_t o = (size_t)p * ne + e, st = (size_t)np * ne;
        met[o] = m.y_eta;
        met[st + o] = -m.x_eta;
        met[2 * st + o] = -m.y_xi;
        met[3 * st + o] = m.x_xi;
        met[4 * st + o] = 1.0 / jac;
        jacp[o] = jac;
        L->xy_host[o] = m.x;
        L->xy_host[st + o] = m.y;
      }
    for (int f = 0; f < 4; ++f)
      for (int k = 0; k < n1; ++k) {
        double xi, eta;
        if (f < 2) {
          xi = (f == 0) ? -1.0 : 1.0;
          eta = L->x1[k];
        } else {
          xi = L->x1[k];
          eta = (f == 2) ? -1.0 : 1.0;
        }
        const MapEval m = map_at(nodes, g, xi, eta);
        const double vx = (f < 2) ? m.y_eta : -m.y_xi;
        const double vy = (f < 2) ? -m.x_eta : m.x_xi;
        const double len = std::sqrt(vx * vx + vy * vy);
        const size_t o = ((size_t)(f * n1 + k) * 3) * ne + e;
        fvec[o] = vx / len;
        fvec[o + ne] = vy / len;
        fvec[o + 2 * ne] = len;
      }
  }
  // BR2 lifting factor of each flux point: lambda_f,k = sum_m l_m(face) g_f'(x_m) / |J_m| along the
  // tensor line through the point (viscous levels)
  std::vector<double> lam;
  if (L->visc) {
    lam.assign((size_t)4 * n1 * ne, 0.0);
    std::vector<double> lmv(n1), lpv(n1);
    for (int m = 0; m < n1; ++m) {
      lmv[m] = L->ops.lm[m];
      lpv[m] = L->ops.lp[m];
    }
    for (int e = 0; e < ne; ++e)
      for (int k = 0; k < n1; ++k)
        for (int m = 0; m < n1; ++m) {
          const double jx = jacp[(size_t)(m + n1 * k) * ne + e];     // point (m, k): line eta = x_k
          const double je = jacp[(size_t)(k + n1 * m) * ne + e];     // point (k, m): line xi = x_k
          lam[(size_t)(0 * n1 + k) * ne + e] += lmv[m] * L->ops.gL[m] / jx;
          lam[(size_t)(1 * n1 + k) * ne + e] += lpv[m] * L->ops.gR[m] / jx;
          lam[(size_t)(2 * n1 + k) * ne + e] += lmv[m] * L->ops.gL[m] / je;
          lam[(size_t)(3 * n1 + k) * ne + e] += lpv[m] * L->ops.gR[m] / je;
        }
  }
  L->dx_host.resize(ne);
  std::vector<double> hdx(ne);
  for (int e = 0; e < ne; ++e) {
    L->dx_host[e] = element_length(d->nodes + (size_t)e * nn * 2, g);
    hdx[e] = L->dx_host[e] / n1;
  }
  std::vector<int> nbr((size_t)4 * ne), nbf((size_t)4 * ne), ori((size_t)4 * ne);
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < 4; ++f) {
      nbr[(size_t)f * ne + e] = d->face_nbr[4 * e + f];
      nbf[(size_t)f * ne + e] = d->face_nbr_face[4 * e + f];
      ori[(size_t)f * ne + e] = d->face_orient[4 * e + f];
    }
  pmg_status s = PMG_OK;
  if ((s = upload(&L->met, met)) || (s = upload(&L->fvec, fvec)) || (s = upload(&L->nbr, nbr)) ||
      (s = upload(&L->nbf, nbf)) || (s = upload(&L->ori, ori)) || (s = upload(&L->hdx, hdx))) {
    free_level(L);
    return s;
  }
  const size_t ns = L->state_elems();
  L->epw = pmg::default_epw(L->P);
  L->part_blocks = pmg::residual_blocks(*L);
  int cand[4], min_epw = L->epw;
  for (int c = 0, nc = pmg::epw_candidates(*L, cand); c < nc; ++c) min_epw = std::min(min_epw, cand[c]);
  const size_t part_max = (size_t)(L->ne + min_epw - 1) / min_epw;   // room for every tuner candidate
  if ((s = alloc_zero(&L->wq, ns)) || (s = alloc_zero(&L->wF, ns)) || (s = alloc_zero(&L->wS, ns)) ||
      (s = alloc_zero(&L->wqb, ns)) || (s = alloc_zero(&L->wql, ns)) || (s = alloc_zero(&L->wsrc, ns)) ||
      (s = alloc_zero(&L->part, part_max * L->nv)) || (s = alloc_zero(&L->norms, L->nv + 1)) ||
      (s = alloc_zero(&L->dtpart, pmg::dtau_blocks(*L))) || (s = alloc_zero(&L->dtmin, 1))) {
    free_level(L);
    return s;
  }
  if (L->visc && ((s = upload(&L->lam, lam)) || (s = alloc_zero(&L->gface, (size_t)4 * n1 * 8 * ne)) ||
                  (s = alloc_zero(&L->Dv, (size_t)L->n * L->n * ne)))) {
    free_level(L);
    return s;
  }
  if (hipMalloc(&L->flag, sizeof(int)) != hipSuccess) {
    free_level(L);
    return fail(PMG_E_NOMEM, "hipMalloc failed for the fault flag");
  }
  if (hipMemset(L->flag, 0, sizeof(int)) != hipSuccess) {
    free_level(L);
    return fail(PMG_E_HIP, "hipMemset fault flag");
  }
  if ((s = alloc_lookahead(L))) {
    free_level(L);
    return s;
  }
  *out = L;
  return PMG_OK;
}

pmg_status pmg_level_destroy(pmg_level L) {
  if (!L) return PMG_OK;
  DeviceGuard guard(L->device);
  free_level(L);
  return PMG_OK;
}

pmg_status pmg_level_info(pmg_level L, int32_t* info) {
  if (pmg_status s = check_level(L)) return s;
  if (!info) return fail(PMG_E_ARG, "null info");
  info[0] = L->dim;
  info[1] = L->P;
  info[2] = L->np;
  info[3] = L->nv;
  info[4] = L->n;
  info[5] = L->ne;
  info[6] = L->device;
  info[7] = L->geom_order;
  return PMG_OK;
}

pmg_status pmg_level_points(pmg_level L, double* xy_host) {
  if (pmg_status s = check_level(L)) return s;
  if (!xy_host) return fail(PMG_E_ARG, "null output");
  std::memcpy(xy_host, L->xy_host.data(), L->xy_host.size() * sizeof(double));
  return PMG_OK;
}

pmg_status pmg_level_dx(pmg_level L, double* dx_host) {
  if (pmg_status e = check_level(L)) return e;
  if (!dx_host) return fail(PMG_E_ARG, "null output");
  std::memcpy(dx_host, L->dx_host.data(), L->dx_host.size() * sizeof(double));
  return PMG_OK;
}

pmg_status pmg_level_epw(pmg_level L, int32_t* epw, int32_t* cand, int32_t* n_cand) {
  if (pmg_status e = check_level(L)) return e;
  if (!epw) return fail(PMG_E_ARG, "null output");
  *epw = L->epw;
  int c[4];
  const int nc = pmg::epw_candidates(*L, c);
  if (n_cand) *n_cand = nc;
  if (cand)
    for (int i = 0; i < nc; ++i) cand[i] = c[i];
  return PMG_OK;
}

pmg_status pmg_level_set_epw(pmg_level L, int32_t epw) {
  if (pmg_status e = check_level(L)) return e;
  int c[4];
  const int nc = pmg::epw_candidates(*L, c);
  if (epw == 0) epw = c[0];
  if (std::find(c, c + nc, (int)epw) == c + nc) return fail(PMG_E_ARG, "not a compiled elements-per-workgroup variant");
  L->epw = epw;
  L->part_blocks = pmg::residual_blocks(*L);
  return PMG_OK;
}

pmg_status pmg_level_autotune(pmg_level L, int32_t precision, int32_t reps, int32_t* epw_out, double* us_out,
                              void* stream) {
  if (pmg_status e = check_level(L)) return e;
  if (precision != 32 && precision != 64) return fail(PMG_E_ARG, "precision must be 32 or 64");
  if (reps < 1) return fail(PMG_E_ARG, "reps must be >= 1");
  int c[4];
  const int nc = pmg::epw_candidates(*L, c);
  DeviceGuard guard(L->device);
  const hipStream_t st = as_stream(stream);
  // the free stream (zero offsets) and zero inverse blocks: the kernels' work does not depend on
  // the values, and alpha_r = 0 leaves the scratch state unchanged
  const size_t ns = L->state_elems();
  double *q = nullptr, *F = nullptr;
  pmg_factors_s fac{};
  fac.L = L;
  fac.precision = precision;
  fac.bytes = (size_t)L->n * L->npad * L->ne * (precision / 8);
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto release = [&]() {
    if (q) (void)hipFree(q);
    if (F) (void)hipFree(F);
    if (fac.W) (void)hipFree(fac.W);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (hipMalloc(&q, ns * sizeof(double)) != hipSuccess || hipMalloc(&F, ns * sizeof(double)) != hipSuccess ||
      hipMalloc(&fac.W, fac.bytes) != hipSuccess || hipMemsetAsync(q, 0, ns * sizeof(double), st) != hipSuccess ||
      hipMemsetAsync(fac.W, 0, fac.bytes, st) != hipSuccess || hipEventCreate(&ev[0]) != hipSuccess ||
      hipEventCreate(&ev[1]) != hipSuccess) {
    release();
    return fail(PMG_E_NOMEM, "could not allocate the tuner's scratch arrays");
  }
  const int keep = L->epw;
  int best = -1;
  double best_us = 0.0, us_def = 0.0;
  constexpr double kTuneMargin = 0.98;   // a candidate must beat the default by more than 2%
  pmg_status status = PMG_OK;
  for (int i = 0; i < nc && status == PMG_OK; ++i) {
    L->epw = c[i];
    L->part_blocks = pmg::residual_blocks(*L);
    float ms = 0.0f;
    hipError_t err = hipSuccess;
    for (int pass = 0; pass < 2 && err == hipSuccess; ++pass) {   // pass 0 warms up
      err = hipEventRecord(ev[0], st);
      for (int r = 0; r < reps && err == hipSuccess; ++r) {
        err = pmg::launch_residual(*L, q, nullptr, nullptr, 0.0, F, true, st);
        if (err == hipSuccess) err = pmg::launch_sweep(*L, fac, q, L->wq, nullptr, nullptr, 0.0, 0.0, true, st);
      }
      if (err == hipSuccess) err = hipEventRecord(ev[1], st);
      if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev[0], ev[1]);
    }
    if (err != hipSuccess) {
      status = fail(PMG_E_HIP, hipGetErrorString(err));
      break;
    }
    const double us = 1e3 * ms / reps;
    if (us_out) us_out[i] = us;
    if (i == 0) us_def = us;
    if (best < 0 || us < best_us) {
      best = i;
      best_us = us;
    }
  }
  release();
  // the default stays unless a candidate is clearly faster: timings within a few percent are noise
  // and would only make the configuration flip between runs
  if (status == PMG_OK && best != 0 && us_def * kTuneMargin <= best_us) best = 0;
  L->epw = (status == PMG_OK) ? c[best] : keep;
  L->part_blocks = pmg::residual_blocks(*L);
  if (status == PMG_OK && epw_out) *epw_out = L->epw;
  return status;
}

pmg_status pmg_dtau_min(pmg_level L, const double* q, double* dtau_min, void* stream) {
  if (pmg_status e = check_level(L)) return e;
  if (!q || !dtau_min) return fail(PMG_E_ARG, "null q or output");
  DeviceGuard guard(L->device);
  const hipStream_t st = as_stream(stream);
  PMG_HIP(pmg::launch_dtau_min(*L, q, st));
  double h = 0.0;
  PMG_HIP(hipMemcpyAsync(&h, L->dtmin, sizeof(double), hipMemcpyDeviceToHost, st));
  PMG_HIP(hipStreamSynchronize(st));
  if (!(h > 0.0) || !std::isfinite(h)) return fail(PMG_E_NONFINITE, "non-physical state in the pseudo-time scale");
  *dtau_min = h;
  return PMG_OK;
}

pmg_status pmg_level_status(pmg_level L, int32_t* flags) {
  if (pmg_status s = check_level(L)) return s;
  DeviceGuard guard(L->device);
  int h = 0;
  PMG_HIP(hipDeviceSynchronize());
  PMG_HIP(hipMemcpy(&h, L->flag, sizeof(int), hipMemcpyDeviceToHost));
  PMG_HIP(hipMemset(L->flag, 0, sizeof(int)));
  if (flags) *flags = h;
  if (h & 1) return fail(PMG_E_SINGULAR, "zero or non-finite pivot in an element block");
  return PMG_OK;
}

pmg_status pmg_factors_create(pmg_level L, int32_t precision, pmg_factors* out) {
  if (pmg_status s = check_level(L)) return s;
  if (!out) return fail(PMG_E_ARG, "null output");
  if (precision != 32 && precision != 64) return fail(PMG_E_ARG, "precision must be 32 or 64");
  if (L->P > 5) return fail(PMG_E_ARG, "element blocks are supported for P <= 5");
  if (L->dim == 3 && L->P > 3) return fail(PMG_E_ARG, "3-D element blocks are supported for P <= 3");
  DeviceGuard guard(L->device);
  pmg_factors_s* F = new pmg_factors_s();
  F->L = L;
  F->precision = precision;
  F->bytes = (size_t)L->n * L->npad * L->ne * (precision / 8);
  if (hipMalloc(&F->W, F->bytes) != hipSuccess) {
    delete F;
    return fail(PMG_E_NOMEM, "hipMalloc failed for element blocks");
  }
  if (hipMemset(F->W, 0, F->bytes) != hipSuccess) {
    (void)hipFree(F->W);
    delete F;
    return fail(PMG_E_HIP, "hipMemset element blocks");
  }
  if (L->dim == 3 && (L->P == 3 || (L->P == 2 && precision == 32))) {
    // every element's pointwise derivatives (P = 3, and P = 2 with FP32 inverses), after one FP64
    // work slot per resident workgroup of the large-block elimination (P = 3)
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, L->device) != hipSuccess || cus <= 0)
      cus = 256;
    F->ws_slots = L->P == 3 ? (2 * cus < L->ne ? 2 * cus : L->ne) : 0;
    // the slots, then every element's pointwise derivatives
    const size_t elems = (size_t)F->ws_slots * L->n * L->n + (size_t)L->ne * pmg::jac3_point_elems(L->P);
    if (hipMalloc(&F->ws, elems * sizeof(double)) != hipSuccess) {
      (void)hipFree(F->W);
      delete F;
      return fail(PMG_E_NOMEM, "hipMalloc failed for the elimination work array");
    }
  }
  *out = F;
  return PMG_OK;
}

pmg_status pmg_factors_destroy(pmg_factors F) {
  if (!F) return PMG_OK;
  DeviceGuard guard(F->L->device);
  if (F->W) (void)hipFree(F->W);
  if (F->ws) (void)hipFree(F->ws);
  if (pmg::LineFactors* lf = F->lines) {
    void* ptrs[] = {lf->elems, lf->pos, lf->fside, lf->D, lf->Winv, lf->Kc, lf->r, lf->C, lf->B, lf->M, lf->N, lf->z, lf->tr};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    delete lf;
  }
  delete F;
  return PMG_OK;
}

pmg_status pmg_line_factors_create(pmg_level L, int32_t precision, const int32_t* line_elems, int32_t n_lines,
                                   int32_t line_len, pmg_factors* out) {
  if (pmg_status s = check_level(L)) return s;
  if (!out || !line_elems) return fail(PMG_E_ARG, "null output or line list");
  if (precision != 32 && precision != 64) return fail(PMG_E_ARG, "precision must be 32 or 64");
  if (L->dim != 2) return fail(PMG_E_ARG, "element-line Jacobi is implemented for quadrilateral levels");
  if (L->P > pmg::kLineMaxP) return fail(PMG_E_ARG, "element-line Jacobi is implemented for P <= 4");
  if (L->visc) return fail(PMG_E_ARG, "element-line Jacobi is implemented for inviscid levels");
  if (n_lines < 1 || line_len < 1 || (int64_t)n_lines * line_len != L->ne)
    return fail(PMG_E_SHAPE, "the lines must hold every element exactly once (n_lines * line_len == Ne)");
  DeviceGuard guard(L->device);
  const int ne = L->ne;
  std::vector<int> nbr((size_t)4 * ne);
  PMG_HIP(hipMemcpy(nbr.data(), L->nbr, nbr.size() * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int> seen(ne, 0), fside((size_t)2 * ne, -1);
  for (int64_t i = 0; i < (int64_t)n_lines * line_len; ++i) {
    const int e = line_elems[i];
    if (e < 0 || e >= ne || seen[e]++) return fail(PMG_E_SHAPE, "an element is missing from the lines or repeated");
  }
  for (int l = 0; l < n_lines; ++l) {
    for (int k = 0; k + 1 < line_len; ++k) {
      const int e = line_elems[(size_t)l * line_len + k], e2 = line_elems[(size_t)l * line_len + k + 1];
      int f12 = -1, f21 = -1, n12 = 0, n21 = 0;
      for (int f = 0; f < 4; ++f) {
        if (nbr[(size_t)f * ne + e] == e2) f12 = f, ++n12;
        if (nbr[(size_t)f * ne + e2] == e) f21 = f, ++n21;
      }
      if (n12 != 1 || n21 != 1) return fail(PMG_E_SHAPE, "consecutive elements of a line must share exactly one face");
      fside[(size_t)ne + e] = f12;        // towards the next element
      fside[e2] = f21;                    // towards the previous element
    }
  }
  pmg_factors_s* F = new pmg_factors_s();
  F->L = L;
  F->precision = precision;
  F->lines = new pmg::LineFactors();
  pmg::LineFactors& lf = *F->lines;
  lf.n_lines = n_lines;
  lf.K = line_len;
  const size_t nn = (size_t)ne * L->n * L->n;
  F->bytes = nn * (precision / 8);
  std::vector<int> elems(line_elems, line_elems + (size_t)n_lines * line_len), pos(ne);
  for (size_t i = 0; i < elems.size(); ++i) pos[elems[i]] = (int)i;
  bool ok = upload(&lf.elems, elems) == PMG_OK && upload(&lf.pos, pos) == PMG_OK &&
            upload(&lf.fside, fside) == PMG_OK &&
            hipMalloc(&lf.D, nn * sizeof(double)) == hipSuccess && hipMalloc(&lf.Winv, F->bytes) == hipSuccess &&
            hipMalloc(&lf.Kc, (size_t)2 * ne * 16 * L->n1 * sizeof(double)) == hipSuccess &&
            hipMalloc(&lf.r, L->state_elems() * sizeof(double)) == hipSuccess;
  const size_t nj = (size_t)pmg::line_rank(L->P), cb = (size_t)ne * nj * L->n * (precision / 8),
               mn = (size_t)ne * nj * nj * sizeof(double);
  ok = ok && hipMalloc(&lf.C, cb) == hipSuccess && hipMalloc(&lf.B, cb) == hipSuccess &&
       hipMalloc(&lf.M, mn) == hipSuccess && hipMalloc(&lf.N, mn) == hipSuccess &&
       hipMalloc(&lf.z, (size_t)ne * L->n * sizeof(double)) == hipSuccess &&
       hipMalloc(&lf.tr, (size_t)4 * ne * nj * sizeof(double)) == hipSuccess;
  // a sweep before the first factorisation leaves q unchanged; M and N stay zero at the line ends
  ok = ok && hipMemset(lf.Winv, 0, F->bytes) == hipSuccess &&
       hipMemset(lf.Kc, 0, (size_t)2 * ne * 16 * L->n1 * sizeof(double)) == hipSuccess &&
       hipMemset(lf.C, 0, cb) == hipSuccess && hipMemset(lf.B, 0, cb) == hipSuccess &&
       hipMemset(lf.M, 0, mn) == hipSuccess && hipMemset(lf.N, 0, mn) == hipSuccess;
  if (!ok) {
    (void)pmg_factors_destroy(F);
    return fail(PMG_E_NOMEM, "device allocation failed for the line factors");
  }
  *out = F;
  return PMG_OK;
}

pmg_status pmg_line_blocks(pmg_factors F, const double* q, double dtau, double c_mass, double* D_out,
                           double* Am_out, double* Ap_out, void* stream) {
  if (!F || !F->lines) return fail(PMG_E_ARG, "not a line-factor handle");
  if (!q) return fail(PMG_E_ARG, "null q");
  if (!(dtau > 0.0)) return fail(PMG_E_ARG, "dtau must be positive");
  pmg_level L = F->L;
  DeviceGuard guard(L->device);
  hipStream_t st = as_stream(stream);
  PMG_HIP(pmg::launch_line_factor(*L, q, dtau, c_mass, D_out, *F, st));
  if (Am_out || Ap_out) PMG_HIP(pmg::launch_line_dense(*L, *F, Am_out, Ap_out, st));
  return PMG_OK;
}

pmg_status fr_residual(pmg_level L, const double* q, const double* src, const double* S, double c_mass, double* F,
                       double* norms, void* stream) {
  if (pmg_status s = check_level(L)) return s;
  if (!q || !F) return fail(PMG_E_ARG, "null q or F");
  if (F == q) return fail(PMG_E_ARG, "F must not alias q");
  DeviceGuard guard(L->device);
  hipStream_t st = as_stream(stream);
  PMG_HIP(pmg::launch_residual(*L, q, src, S, c_mass, F, norms != nullptr, st));
  if (norms) {
    PMG_HIP(pmg::launch_norm_finalize(*L, st));
    if (norms != L->norms)
      PMG_HIP(hipMemcpyAsync(norms, L->norms, (L->nv + 1) * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  return PMG_OK;
}

pmg_status fr_conservative(pmg_level L, const double* q, double* qc, void* stream) {
  if (pmg_status s = check_level(L)) return s;
  if (!q || !qc) return fail(PMG_E_ARG, "null pointer");
  DeviceGuard guard(L->device);
  PMG_HIP(pmg::launch_conservative(*L, q, qc, as_stream(stream)));
  return PMG_OK;
}

pmg_status fr_element_jacobian(pmg_level L, const double* q, double dtau, double c_mass, double* D_out,
                               pmg_factors fac, void* stream) {
  if (pmg_status s = check_level(L)) return s;
  if (!q || !fac) return fail(PMG_E_ARG, "null q or factors");
  if (fac->L != L) return fail(PMG_E_SHAPE, "factors belong to another level");
  if (!(dtau > 0.0)) return fail(PMG_E_ARG, "dtau must be positive");
  DeviceGuard guard(L->device);
  PMG_HIP(build_blocks(*L, q, dtau, c_mass, D_out, *fac, as_stream(stream)));
  return PMG_OK;
}

pmg_status ejacobi_sweep(pmg_level L, pmg_factors fac, double* q, const double* src, const double* S,
                         double c_mass, int32_t n_sweeps, double alpha_r, double* F_after, double* norms,
                         void* stream) {
  if (pmg_status s = check_level(L)) return s;
  if (!q || !fac) return fail(PMG_E_ARG, "null q or factors");
  if (fac->L != L) return fail(PMG_E_SHAPE, "factors belong to another level");
  if (n_sweeps < 0) return fail(PMG_E_ARG, "n_sweeps must be >= 0");
  if (F_after == q) return fail(PMG_E_ARG, "F_after must not alias q");
  DeviceGuard guard(L->device);
  hipStream_t st = as_stream(stream);
  if (pmg_status r = run_sweeps(*L, *fac, q, src, S, c_mass, n_sweeps, alpha_r, F_after, norms != nullptr, st))
    return r;
  if (norms && norms != L->norms) PMG_HIP(pmg::launch_copy(L->nv + 1, L->norms, norms, st));
  return PMG_OK;
}

static pmg_status check_pair(pmg_level fine, pmg_level coarse, int32_t nvar) {
  if (!fine || !coarse) return fail(PMG_E_ARG, "null level");
  if (fine->ne != coarse->ne || fine->dim != coarse->dim || fine->device != coarse->device)
    return fail(PMG_E_SHAPE, "levels are not on the same mesh and device");
  if (!(coarse->P < fine->P)) return fail(PMG_E_SHAPE, "coarse degree must be below the fine degree");
  for (int k = 0; k < 5; ++k)
    if (fine->q_ref[k] != coarse->q_ref[k]) return fail(PMG_E_SHAPE, "levels have different q_ref");
  if (nvar < 1 || nvar > fine->nv) return fail(PMG_E_ARG, "nvar out of range");
  return PMG_OK;
}

pmg_status pmg_restrict(pmg_level fine, pmg_level coarse, const double* x_f, double* x_c, int32_t nvar,
                        void* stream) {
  if (pmg_status s = check_pair(fine, coarse, nvar)) return s;
  if (!x_f || !x_c) return fail(PMG_E_ARG, "null pointer");
  DeviceGuard guard(fine->device);
  std::vector<double> R;
  projection_matrix(*fine, *coarse, R);
  PMG_HIP(pmg::launch_restrict(*fine, *coarse, R.data(), x_f, x_c, nvar, as_stream(stream)));
  return PMG_OK;
}

pmg_status pmg_prolong(pmg_level coarse, pmg_level fine, const double* dx_c, double* x_f, int32_t nvar,
                       void* stream) {
  if (pmg_status s = check_pair(fine, coarse, nvar)) return s;
  if (!dx_c || !x_f) return fail(PMG_E_ARG, "null pointer");
  DeviceGuard guard(fine->device);
  std::vector<double> I;
  interpolation_matrix(*coarse, *fine, I);
  PMG_HIP(pmg::launch_prolong(*coarse, *fine, I.data(), dx_c, nullptr, x_f, nvar, as_stream(stream)));
  return PMG_OK;
}

}  // extern "C"

// ---- stage solve -------------------------------------------------------------------------------
namespace {

struct Solve {
  const pmg_solve_opts* o;
  hipStream_t st;
  double c_mass;
  const double* src;       // finest-level source, or null
  double dtau;
  bool refresh;
  int n_refresh;
  std::vector<std::vector<double>> R1, I1;   // per level l: matrices between l and l+1
};

// One V-cycle from level l. With S_pending (coarse levels) S holds the restricted fine residual
// P w = P (F_l(q^a) - S_l) and q the restricted state q^b: the forcing S_{l+1} = F_{l+1}(q^b) - P w
// of eqs. (40), (43) is formed by the first pre-smoothing sweep, whose defect at q^b is P w.
pmg_status vcycle(Solve& s, int l, double* q, double* S, bool S_pending = false) {
  const pmg_solve_opts* o = s.o;
  pmg_level L = o->levels[l];
  pmg_factors fac = o->factors[l];
  const bool last = (l == o->n_levels - 1);
  const double* src = (l == 0) ? s.src : nullptr;
  if (s.refresh && l > 0) {
    PMG_HIP(build_blocks(*L, q, s.dtau, s.c_mass, nullptr, *fac, s.st));
    ++s.n_refresh;
  }
  if (S_pending && o->n_smooth[l] == 0) {   // no sweep to form it in
    PMG_HIP(pmg::launch_residual(*L, q, nullptr, S, s.c_mass, S, false, s.st));
    S_pending = false;
  }
  // pre-smoothing; F_after = F_l(q^a) - S_l = -d_l
  if (pmg_status r = run_sweeps(*L, *fac, q, src, S, s.c_mass, o->n_smooth[l], o->alpha_r, last ? nullptr : L->wF,
                                false, s.st, S_pending ? S : nullptr))
    return r;
  if (last) return PMG_OK;
  pmg_level Lc = o->levels[l + 1];
  // q^b_{l+1} = P q^a_l (eqs. (39), (42)), written also to the coarse working state, and
  // S_{l+1} = F_{l+1}(q^b) + P d_l = F_{l+1}(q^b) - P (F_l(q^a) - S_l)  (eqs. (40), (43))
  PMG_HIP(pmg::launch_restrict_pair(*L, *Lc, s.R1[l].data(), q, Lc->wqb, Lc->wql, L->wF, Lc->wS, Lc->nv, s.st));
  if (pmg_status r = vcycle(s, l + 1, Lc->wql, Lc->wS, true)) return r;
  // q^{c,b}_l = q^a_l + I (q^{(c,)a}_{l+1} - q^b_{l+1}) (eqs. (44), (45)), then post-smoothing
  PMG_HIP(pmg::launch_prolong(*Lc, *L, s.I1[l].data(), Lc->wql, Lc->wqb, q, L->nv, s.st));
  return run_sweeps(*L, *fac, q, src, S, s.c_mass, o->n_smooth[l], o->alpha_r, nullptr, false, s.st);
}

// One V-cycle followed by the finest-level residual norm of its result.
pmg_status vcycle_and_norm(Solve& s, double* q) {
  if (pmg_status e = vcycle(s, 0, q, nullptr)) return e;
  pmg_level L0 = s.o->levels[0];
  PMG_HIP(pmg::launch_residual(*L0, q, s.src, nullptr, s.c_mass, L0->wF, true, s.st));
  PMG_HIP(pmg::launch_norm_finalize(*L0, s.st));
  return PMG_OK;
}

// Everything a captured V-cycle depends on: replaying it is valid while this key is unchanged.
std::vector<uintptr_t> graph_key(const Solve& s, const double* q) {
  const pmg_solve_opts* o = s.o;
  std::vector<uintptr_t> k;
  k.push_back((uintptr_t)q);
  k.push_back((uintptr_t)s.src);
  uint64_t cm, ar;
  std::memcpy(&cm, &s.c_mass, 8);
  std::memcpy(&ar, &o->alpha_r, 8);
  k.push_back((uintptr_t)cm);
  k.push_back((uintptr_t)ar);
  k.push_back((uintptr_t)o->n_levels);
  for (int l = 0; l < o->n_levels; ++l) {
    k.push_back((uintptr_t)o->levels[l]);
    k.push_back((uintptr_t)o->factors[l]);
    k.push_back((uintptr_t)o->factors[l]->precision);
    k.push_back((uintptr_t)o->n_smooth[l]);
  }
  return k;
}

// Capture (or reuse) the graph of vcycle_and_norm for this solve and launch it on s.st.
pmg_status vcycle_graph(Solve& s, double* q) {
  pmg_level L0 = s.o->levels[0];
  const std::vector<uintptr_t> key = graph_key(s, q);
  if (!L0->vc_exec || L0->vc_key != key) {
    if (L0->vc_exec) {
      PMG_HIP(hipGraphExecDestroy(L0->vc_exec));
      L0->vc_exec = nullptr;
    }
    if (!L0->capture_stream) PMG_HIP(hipStreamCreateWithFlags(&L0->capture_stream, hipStreamNonBlocking));
    Solve sc = s;
    sc.st = L0->capture_stream;
    sc.refresh = false;
    PMG_HIP(hipStreamBeginCapture(sc.st, hipStreamCaptureModeRelaxed));
    const pmg_status e = vcycle_and_norm(sc, q);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(sc.st, &g);
    if (e != PMG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&L0->vc_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    L0->vc_key = key;
  }
  PMG_HIP(hipGraphLaunch(L0->vc_exec, s.st));
  return PMG_OK;
}

// ---- one stage solve as a state machine between V-cycles ----------------------------------------
// The single and the batched entry points share it: stage_begin enqueues the set-up and the norm of
// q^0, stage_advance consumes the latest norm (host copy), applies the SER law of eq. (31) and
// enqueues the next V-cycle with its norm, stage_finish checks the fault flags and fills the stats.
//
// Lookahead (single-case solves): between block rebuilds a V-cycle depends on the host only through
// the decision to run it (Delta tau enters through the blocks alone), so the V-cycle after the one
// in flight is enqueued before the host has read the in-flight one's norm, and the device does not
// wait for the host between V-cycles. The state before that speculative V-cycle is copied to the
// finest level's restriction buffer (unused on the finest level); when the norm then says stop,
// the copy is restored, so the result, the norm history and the V-cycle count are those of the
// plain loop. No speculation where the next V-cycle rebuilds blocks or would pass max_vcycles, or
// where the last rate of decrease predicts the tolerance within a factor of 8 (a stop there would
// cost a whole V-cycle, more than the host wait it saves).
struct StageRun {
  Solve s;
  pmg_solve_stats* stats = nullptr;
  double* q = nullptr;
  double* R_out = nullptr;
  double dtau_max = 0.0;
  double dtau_floor = 0.0;      // lower bound of the SER law (dtau_init with ser_floor, else 0)
  double r0 = 0.0, r = 0.0, r_prev = 0.0, dtau_last_refresh = -1.0;
  int m = 0;                    // V-cycles done
  bool active = false;          // a norm is in flight and more V-cycles may follow
  pmg_status result = PMG_E_NOT_CONVERGED;
  std::chrono::steady_clock::time_point t_start;
  double* host_norms = nullptr; // [Nv + 1] host copy of the finest-level norms
  // lookahead (null spec_norms: off)
  double* spec_norms = nullptr; // [Nv + 1] norm copy of the speculative V-cycle
  hipEvent_t ev_cur = nullptr;  // recorded after the copy into host_norms
  hipEvent_t ev_spec = nullptr; // recorded after the copy into spec_norms
  bool spec = false;            // a speculative V-cycle and its norm copy are in flight
  double rate = 1.0;            // r_m / r_{m-1} of the last two norms read
};

pmg_status check_opts(const pmg_solve_opts* o) {
  if (!o) return fail(PMG_E_ARG, "null options");
  if (o->n_levels < 1 || o->n_levels > 8 || !o->levels || !o->factors || !o->n_smooth)
    return fail(PMG_E_ARG, "bad level list");
  for (int l = 0; l < o->n_levels; ++l) {
    if (!o->levels[l] || !o->factors[l]) return fail(PMG_E_ARG, "null level or factors");
    if (o->factors[l]->L != o->levels[l]) return fail(PMG_E_SHAPE, "factors do not match their level");
    if (o->n_smooth[l] < 0) return fail(PMG_E_ARG, "negative smoothing count");
    if (l > 0 && (o->levels[l]->P >= o->levels[l - 1]->P || o->levels[l]->ne != o->levels[0]->ne ||
                  o->levels[l]->device != o->levels[0]->device))
      return fail(PMG_E_SHAPE, "levels must share the mesh with strictly decreasing P");
    for (int k = 0; k < 5; ++k)
      if (o->levels[l]->q_ref[k] != o->levels[0]->q_ref[k]) return fail(PMG_E_SHAPE, "levels have different q_ref");
  }
  if (o->use_cfl) {
    if (!(o->cfl_init > 0.0) || !(o->cfl_max >= o->cfl_init)) return fail(PMG_E_ARG, "bad CFL range");
  } else if (!(o->dtau_init > 0.0) || !(o->dtau_max >= o->dtau_init)) {
    return fail(PMG_E_ARG, "bad dtau range");
  }
  if (o->refresh_every < 1 || o->max_vcycles < 0) return fail(PMG_E_ARG, "bad refresh/max_vcycles");
  if (o->stage_guess != 0 && o->stage_guess != 1) return fail(PMG_E_ARG, "stage_guess must be 0 or 1");
  if (o->ser_floor != 0 && o->ser_floor != 1) return fail(PMG_E_ARG, "ser_floor must be 0 or 1");
  if (o->lookahead < 0 || o->lookahead > 2) return fail(PMG_E_ARG, "lookahead must be 0, 1 or 2");
  return PMG_OK;
}

pmg_status enqueue_norm_copy(StageRun& R, double* dst, hipEvent_t ev) {
  pmg_level L0 = R.s.o->levels[0];
  PMG_HIP(hipMemcpyAsync(dst, L0->norms, (L0->nv + 1) * sizeof(double), hipMemcpyDeviceToHost, R.s.st));
  if (ev) PMG_HIP(hipEventRecord(ev, R.s.st));
  return PMG_OK;
}

pmg_status enqueue_norm_copy(StageRun& R) { return enqueue_norm_copy(R, R.host_norms, R.ev_cur); }

// Whether the V-cycle that the stage_advance reading the norm of V-cycle m (after the one in flight)
// would enqueue rebuilds the finest blocks.
bool refresh_at(const StageRun& R, int m) {
  const pmg_solve_opts* o = R.s.o;
  const bool frozen = o->freeze_at_max && R.dtau_last_refresh >= R.dtau_max;
  return (m == 0) || (m % o->refresh_every == 0 && !frozen);
}

// Enqueue the V-cycle after the one in flight (R.m V-cycles done once it ends) if that is safe
// and likely to be kept.
pmg_status maybe_speculate(StageRun& R) {
  const pmg_solve_opts* o = R.s.o;
  if (!R.spec_norms || R.spec || !R.active) return PMG_OK;
  const int m = R.m;
  if (m >= o->max_vcycles || refresh_at(R, m)) return PMG_OK;
  if (o->lookahead == 1 && R.r0 > 0.0 && R.r * std::min(R.rate, 1.0) <= 8.0 * o->tol_rel * R.r0)
    return PMG_OK;   // r_m predicted within 8x of the tolerance
  pmg_level L0 = o->levels[0];
  Solve& s = R.s;
  PMG_HIP(hipMemcpyAsync(L0->wqb, R.q, L0->state_elems() * sizeof(double), hipMemcpyDeviceToDevice, s.st));
  s.refresh = false;
  if (o->use_graph) {
    if (pmg_status e = vcycle_graph(s, R.q)) return e;
  } else {
    if (pmg_status e = vcycle_and_norm(s, R.q)) return e;
  }
  if (pmg_status e = enqueue_norm_copy(R, R.spec_norms, R.ev_spec)) return e;
  R.spec = true;
  return PMG_OK;
}

// A stop while a speculative V-cycle is in flight: put back the state from before it.
pmg_status drop_speculation(StageRun& R) {
  if (!R.spec) return PMG_OK;
  pmg_level L0 = R.s.o->levels[0];
  PMG_HIP(hipMemcpyAsync(R.q, L0->wqb, L0->state_elems() * sizeof(double), hipMemcpyDeviceToDevice, R.s.st));
  R.spec = false;
  return PMG_OK;
}

pmg_status stage_begin(StageRun& R, const pmg_solve_opts* o, double omega, double dt, const double* qc_n,
                       const double* const* R_prev, const double* a_row, int32_t n_prev, double* q, double* R_out,
                       pmg_solve_stats* stats, hipStream_t st) {
  if (!q) return fail(PMG_E_ARG, "null q");
  if (pmg_status e = check_opts(o)) return e;
  const bool steady = !(dt > 0.0);
  if (!steady) {
    if (!(omega > 0.0)) return fail(PMG_E_ARG, "omega must be positive");
    if (!qc_n || n_prev < 1 || n_prev > 8 || !R_prev || !a_row) return fail(PMG_E_ARG, "bad ESDIRK history");
  }
  pmg_level L0 = o->levels[0];
  R.t_start = std::chrono::steady_clock::now();
  R.stats = stats;
  R.q = q;
  R.R_out = R_out;
  Solve& s = R.s;
  s.o = o;
  s.st = st;
  s.c_mass = steady ? 0.0 : 1.0 / (omega * dt);
  s.src = nullptr;
  s.refresh = false;
  s.n_refresh = 0;
  s.R1.assign(o->n_levels, {});
  s.I1.assign(o->n_levels, {});
  for (int l = 0; l + 1 < o->n_levels; ++l) {
    projection_matrix(*o->levels[l], *o->levels[l + 1], s.R1[l]);
    interpolation_matrix(*o->levels[l + 1], *o->levels[l], s.I1[l]);
  }
  if (!steady) {
    PMG_HIP(pmg::launch_stage_source(*L0, qc_n, R_prev, a_row, n_prev, dt, s.c_mass, L0->wsrc, st));
    s.src = L0->wsrc;
  }
  for (int l = 0; l < o->n_levels; ++l) PMG_HIP(hipMemsetAsync(o->levels[l]->flag, 0, sizeof(int), st));
  // pseudo-time range: given directly, or as CFL numbers times dtau_min of eq. (33) at q^0
  double dtau_init = o->dtau_init, dtmin = 0.0;
  R.dtau_max = o->dtau_max;
  if (o->use_cfl) {
    if (pmg_status e = pmg_dtau_min(L0, q, &dtmin, st)) return e;
    dtau_init = o->cfl_init * dtmin;
    R.dtau_max = o->cfl_max * dtmin;
  }
  if (stats) {
    stats->dtau_min = dtmin;
    stats->n_refresh = 0;
  }
  s.dtau = dtau_init;
  R.dtau_floor = o->ser_floor ? dtau_init : 0.0;
  R.m = 0;
  R.dtau_last_refresh = -1.0;
  R.result = PMG_E_NOT_CONVERGED;
  // r_0 = ||F(q^0)||; every V-cycle ends with the norm of its result, r_{m+1}
  PMG_HIP(pmg::launch_residual(*L0, q, s.src, nullptr, s.c_mass, L0->wF, true, st));
  PMG_HIP(pmg::launch_norm_finalize(*L0, st));
  if (pmg_status e = enqueue_norm_copy(R)) return e;
  R.active = true;
  return PMG_OK;
}

// The norm enqueued last must have arrived in R.host_norms (the caller synchronised R.s.st).
pmg_status stage_advance(StageRun& R) {
  const pmg_solve_opts* o = R.s.o;
  pmg_level L0 = o->levels[0];
  Solve& s = R.s;
  const int m = R.m;
  R.r = R.host_norms[L0->nv];
  if (R.stats && R.stats->history && m < R.stats->history_capacity) R.stats->history[m] = R.r;
  R.active = false;
  if (!std::isfinite(R.r)) {
    R.result = fail(PMG_E_NONFINITE, "non-finite residual norm");
    return drop_speculation(R);
  }
  if (m == 0) {
    R.r0 = R.r;
  } else {
    s.dtau = std::max(std::min(s.dtau * std::pow(R.r_prev / R.r, o->ser_exponent), R.dtau_max),   // eq. (31)
                      R.dtau_floor);
    R.rate = R.r_prev > 0.0 ? R.r / R.r_prev : 1.0;
  }
  if (R.r == 0.0 || R.r / R.r0 <= o->tol_rel) {
    R.result = PMG_OK;
    return drop_speculation(R);
  }
  if (m >= o->max_vcycles) {
    R.result = fail(PMG_E_NOT_CONVERGED, "stage solve reached max_vcycles");
    return drop_speculation(R);
  }
  if (R.spec) {   // the V-cycle this step would enqueue (no rebuild) is in flight: keep it
    R.spec = false;
    std::swap(R.host_norms, R.spec_norms);
    std::swap(R.ev_cur, R.ev_spec);
    R.r_prev = R.r;
    R.m = m + 1;
    R.active = true;
    return maybe_speculate(R);
  }
  s.refresh = refresh_at(R, m);
  if (s.refresh) {
    PMG_HIP(build_blocks(*L0, R.q, s.dtau, s.c_mass, nullptr, *o->factors[0], s.st));
    ++s.n_refresh;
    R.dtau_last_refresh = s.dtau;
    if (pmg_status e = vcycle_and_norm(s, R.q)) return e;
  } else if (o->use_graph) {
    if (pmg_status e = vcycle_graph(s, R.q)) return e;
  } else {
    if (pmg_status e = vcycle_and_norm(s, R.q)) return e;
  }
  R.r_prev = R.r;
  R.m = m + 1;
  if (pmg_status e = enqueue_norm_copy(R)) return e;
  R.active = true;
  return maybe_speculate(R);
}

pmg_status stage_finish(StageRun& R) {
  const pmg_solve_opts* o = R.s.o;
  pmg_level L0 = o->levels[0];
  hipStream_t st = R.s.st;
  pmg_status result = R.result;
  if (result != PMG_E_NONFINITE) {
    std::vector<int> h(o->n_levels, 0);
    for (int l = 0; l < o->n_levels; ++l)
      PMG_HIP(hipMemcpyAsync(&h[l], o->levels[l]->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PMG_HIP(hipStreamSynchronize(st));
    int any = 0;
    for (int v : h) any |= v;
    if (any & 1) result = fail(PMG_E_SINGULAR, "zero or non-finite pivot in an element block");
  }
  if (R.R_out && result == PMG_OK)
    PMG_HIP(pmg::launch_residual(*L0, R.q, nullptr, nullptr, 0.0, R.R_out, false, st));
  if (R.stats) {
    R.stats->n_vcycles = R.m;
    R.stats->n_refresh = R.s.n_refresh;
    R.stats->r0 = R.r0;
    R.stats->r_final = R.r;
    R.stats->status = result;
  }
  PMG_HIP(hipStreamSynchronize(st));
  if (R.stats) R.stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t_start).count();
  return result;
}

}  // namespace

extern "C" pmg_status esdirk_stage_solve(const pmg_solve_opts* o, double omega, double dt, const double* qc_n,
                                         const double* const* R_prev, const double* a_row, int32_t n_prev,
                                         double* q, double* R_out, pmg_solve_stats* stats, void* stream) {
  if (pmg_status e = check_opts(o)) return e;
  DeviceGuard guard(o->levels[0]->device);
  pmg_level L0 = o->levels[0];
  StageRun R;
  R.host_norms = L0->hnorm;
  R.spec_norms = o->lookahead ? L0->hnorm + 8 : nullptr;
  R.ev_cur = L0->ev_norm[0];
  R.ev_spec = L0->ev_norm[1];
  const hipStream_t st = as_stream(stream);
  pmg_status e = stage_begin(R, o, omega, dt, qc_n, R_prev, a_row, n_prev, q, R_out, stats, st);
  while (e == PMG_OK && R.active) {
    const hipError_t w = hipEventSynchronize(R.ev_cur);   // the latest kept norm (a speculative
    if (w != hipSuccess) {                                  // V-cycle may still run behind it)
      e = hip_fail(w, "hipEventSynchronize");
      break;
    }
    e = stage_advance(R);
  }
  if (e != PMG_OK) {   // leave nothing of this solve in flight
    (void)hipStreamSynchronize(st);
    return e;
  }
  return stage_finish(R);
}

// ---- Newton-Krylov stage solve (the V-cycle as a preconditioner) ------------------------------------
// Pseudo-transient Newton on the stage equation with the whole Jacobian: per Newton step one cycle
// of flexible GMRES on (Gamma(q_m)/dtau_m - dF/dq) delta = F(q_m), right-preconditioned by one FAS
// V-cycle from q_m with the finest forcing F(q_m) - e v, Jacobian products by forward differences
// of the residual kernel. The Hessenberg matrix and its Givens rotations live on the host; every
// vector operation runs on the device.
namespace {

struct NkWork {
  size_t N;
  int k;
  double* base;
  double* V(int j) const { return base + (size_t)j * N; }
  double* Z(int j) const { return base + (size_t)(k + 1 + j) * N; }
  double* F0() const { return base + (size_t)(2 * k + 1) * N; }
  double* W1() const { return base + (size_t)(2 * k + 2) * N; }
  double* W2() const { return base + (size_t)(2 * k + 3) * N; }
  double* part() const { return base + (size_t)(2 * k + 4) * N; }
  double* dots() const { return part() + (size_t)pmg::kNkMaxTerms * pmg::kNkDotBlocks; }
};

// host[i] = <x[i], v> for i < nx (synchronises the stream)
pmg_status nk_dots(const NkWork& w, const double* const* x, int nx, const double* v, double* host, hipStream_t st) {
  PMG_HIP(pmg::launch_multidot(w.N, nx, x, v, w.part(), w.dots(), st));
  PMG_HIP(hipMemcpyAsync(host, w.dots(), (size_t)nx * sizeof(double), hipMemcpyDeviceToHost, st));
  PMG_HIP(hipStreamSynchronize(st));
  return PMG_OK;
}

pmg_status nk_lincomb(const NkWork& w, int nt, const double* const* x, const double* c, double beta, double* y,
                      hipStream_t st) {
  PMG_HIP(pmg::launch_lincomb(w.N, nt, x, c, beta, y, st));
  return PMG_OK;
}

}  // namespace

extern "C" int64_t nk_work_elems(pmg_level L0, int32_t krylov_dim) {
  if (!L0 || krylov_dim < 1 || krylov_dim > pmg::kNkMaxDim) return -1;
  return (int64_t)(2 * krylov_dim + 4) * (int64_t)L0->state_elems() +
         (int64_t)pmg::kNkMaxTerms * (pmg::kNkDotBlocks + 1);
}

extern "C" pmg_status nk_stage_solve(const pmg_solve_opts* o, const pmg_nk_opts* nk, double omega, double dt,
                                     const double* qc_n, const double* const* R_prev, const double* a_row,
                                     int32_t n_prev, double* q, double* work, pmg_solve_stats* stats,
                                     int32_t* n_krylov, void* stream) {
  if (pmg_status e = check_opts(o)) return e;
  if (!nk || !work || !q) return fail(PMG_E_ARG, "null Newton-Krylov options, work array or state");
  const int k = nk->krylov_dim;
  if (k < 1 || k > pmg::kNkMaxDim) return fail(PMG_E_ARG, "krylov_dim must be in 1..32");
  if (nk->max_newton < 0 || !(nk->eta >= 0.0) || !(nk->fd_rel > 0.0) || !(nk->pc_rel > 0.0) ||
      (nk->precondition != 0 && nk->precondition != 1))
    return fail(PMG_E_ARG, "bad Newton-Krylov options");
  pmg_level L0 = o->levels[0];
  DeviceGuard guard(L0->device);
  const hipStream_t st = as_stream(stream);
  StageRun R;
  double hn[8];
  R.host_norms = hn;
  if (pmg_status e = stage_begin(R, o, omega, dt, qc_n, R_prev, a_row, n_prev, q, nullptr, stats, st)) return e;
  Solve& s = R.s;
  const NkWork w{L0->state_elems(), k, work};
  const size_t N = w.N;
  const double sqn = std::sqrt((double)N);
  int krylov = 0, newton = 0;
  double r0 = 0.0, r = 0.0, r_prev = 0.0, dtau_last_refresh = -1.0;
  pmg_status result = PMG_E_NOT_CONVERGED;
  std::vector<double> H((size_t)(k + 1) * k), cs(k), sn(k), g(k + 1), y(k), c(k + 1);
  std::vector<const double*> xs(k + 2);
  for (int m = 0;; ++m) {
    if (m > 0) {   // F(q_m) and its norm (stage_begin enqueued those of q_0)
      PMG_HIP(pmg::launch_residual(*L0, q, s.src, nullptr, s.c_mass, L0->wF, true, st));
      PMG_HIP(pmg::launch_norm_finalize(*L0, st));
      PMG_HIP(hipMemcpyAsync(hn, L0->norms, (L0->nv + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    PMG_HIP(pmg::launch_copy(N, L0->wF, w.F0(), st));
    PMG_HIP(hipStreamSynchronize(st));
    r = hn[L0->nv];
    if (stats && stats->history && m < stats->history_capacity) stats->history[m] = r;
    if (!std::isfinite(r)) {
      result = fail(PMG_E_NONFINITE, "non-finite residual norm");
      break;
    }
    if (m == 0)
      r0 = r;
    else
      s.dtau = std::max(std::min(s.dtau * std::pow(r_prev / r, o->ser_exponent), R.dtau_max),   // eq. (31)
                        R.dtau_floor);
    if (r == 0.0 || r / r0 <= o->tol_rel) {
      result = PMG_OK;
      break;
    }
    if (m >= nk->max_newton) {
      result = fail(PMG_E_NOT_CONVERGED, "Newton-Krylov stage solve reached max_newton");
      break;
    }
    const bool frozen = o->freeze_at_max && dtau_last_refresh >= R.dtau_max;
    bool refresh_coarse = false;
    if (m == 0 || (m % o->refresh_every == 0 && !frozen)) {
      PMG_HIP(build_blocks(*L0, q, s.dtau, s.c_mass, nullptr, *o->factors[0], st));
      ++s.n_refresh;
      dtau_last_refresh = s.dtau;
      refresh_coarse = true;
    }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = r;
    {
      const double* x0 = w.F0();
      const double c0 = 1.0 / r;
      if (pmg_status e = nk_lincomb(w, 1, &x0, &c0, 0.0, w.V(0), st)) return e;
    }
    int jj = 0;
    for (int j = 0; j < k; ++j) {
      double* v = w.V(j);
      double* z = w.Z(j);
      if (nk->precondition) {   // z = (V(q_m; S_0 = F(q_m) - e v) - q_m) / e, ||v|| = 1
        const double e = nk->pc_rel * sqn;
        PMG_HIP(pmg::launch_copy(N, q, w.W1(), st));
        const double* x2[2] = {w.F0(), v};
        const double c2[2] = {1.0, -e};
        if (pmg_status er = nk_lincomb(w, 2, x2, c2, 0.0, w.W2(), st)) return er;
        s.refresh = refresh_coarse;
        refresh_coarse = false;
        const pmg_status ve = vcycle(s, 0, w.W1(), w.W2());
        s.refresh = false;
        if (ve != PMG_OK) return ve;
        const double* x3[2] = {w.W1(), q};
        const double c3[2] = {1.0 / e, -1.0 / e};
        if (pmg_status er = nk_lincomb(w, 2, x3, c3, 0.0, z, st)) return er;
      } else {
        PMG_HIP(pmg::launch_copy(N, v, z, st));
      }
      double zz = 0.0;
      const double* xz = z;
      if (pmg_status e = nk_dots(w, &xz, 1, z, &zz, st)) return e;
      const double h = nk->fd_rel * sqn / std::sqrt(zz);
      const double* x4[2] = {q, z};
      const double c4[2] = {1.0, h};
      if (pmg_status e = nk_lincomb(w, 2, x4, c4, 0.0, w.W1(), st)) return e;
      PMG_HIP(pmg::launch_residual(*L0, w.W1(), s.src, nullptr, s.c_mass, w.W2(), false, st));
      double* wn = w.V(j + 1);
      PMG_HIP(pmg::launch_newton_op(*L0, q, z, w.W2(), w.F0(), 1.0 / s.dtau, 1.0 / h, wn, st));
      // classical Gram-Schmidt applied twice; the second pass's block of dots also gives ||w||^2,
      // and ||w - V c||^2 = ||w||^2 - ||c||^2 for orthonormal V
      for (int i = 0; i <= j; ++i) xs[i] = w.V(i);
      xs[j + 1] = wn;
      double ww = 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        if (pmg_status e = nk_dots(w, xs.data(), j + 1 + pass, wn, c.data(), st)) return e;
        if (pass == 1) ww = c[j + 1];
        for (int i = 0; i <= j; ++i) {
          H[(size_t)i * k + j] += c[i];
          if (pass == 1) ww -= c[i] * c[i];
          c[i] = -c[i];
        }
        if (pmg_status e = nk_lincomb(w, j + 1, xs.data(), c.data(), 1.0, wn, st)) return e;
      }
      const double hnorm = std::sqrt(std::max(ww, 0.0));
      H[(size_t)(j + 1) * k + j] = hnorm;
      for (int i = 0; i < j; ++i) {   // earlier rotations, then a new one
        const double a = H[(size_t)i * k + j], b = H[(size_t)(i + 1) * k + j];
        H[(size_t)i * k + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * k + j] = -sn[i] * a + cs[i] * b;
      }
      const double den = std::hypot(H[(size_t)j * k + j], H[(size_t)(j + 1) * k + j]);
      cs[j] = H[(size_t)j * k + j] / den;
      sn[j] = H[(size_t)(j + 1) * k + j] / den;
      H[(size_t)j * k + j] = den;
      H[(size_t)(j + 1) * k + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      jj = j + 1;
      if (std::fabs(g[j + 1]) <= nk->eta * r || hnorm == 0.0) break;
      if (pmg_status e = nk_lincomb(w, 0, nullptr, nullptr, 1.0 / hnorm, wn, st)) return e;
    }
    for (int i = jj - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < jj; ++l) t -= H[(size_t)i * k + l] * y[l];
      y[i] = t / H[(size_t)i * k + i];
    }
    for (int i = 0; i < jj; ++i) xs[i] = w.Z(i);
    if (pmg_status e = nk_lincomb(w, jj, xs.data(), y.data(), 1.0, q, st)) return e;
    krylov += jj;
    newton = m + 1;
    r_prev = r;
  }
  if (result != PMG_E_NONFINITE) {
    int any = 0;
    for (int l = 0; l < o->n_levels; ++l) {
      int fl = 0;
      PMG_HIP(hipMemcpyAsync(&fl, o->levels[l]->flag, sizeof(int), hipMemcpyDeviceToHost, st));
      PMG_HIP(hipStreamSynchronize(st));
      any |= fl;
    }
    if (any & 1) result = fail(PMG_E_SINGULAR, "zero or non-finite pivot in an element block");
  }
  if (stats) {
    stats->n_vcycles = newton;
    stats->n_refresh = s.n_refresh;
    stats->r0 = r0;
    stats->r_final = r;
    stats->status = result;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - R.t_start).count();
  }
  if (n_krylov) *n_krylov = krylov;
  return result;
}

// ---- ESDIRK time step ----------------------------------------------------------------------------
namespace {

// Butcher matrices (row-major s x s) of the stiffly accurate ESDIRK schemes named in Sec. 2.4.
int esdirk_tableau(int scheme, double* A) {
  if (scheme == 2) {            // three stages, gamma = 1 - sqrt(2)/2, c = (0, 2 gamma, 1)
    const double g = 1.0 - std::sqrt(2.0) / 2.0, b = std::sqrt(2.0) / 4.0;
    const double t[9] = {0, 0, 0, g, g, 0, b, b, g};
    std::memcpy(A, t, sizeof(t));
    return 3;
  }
  if (scheme == 3) {            // ESDIRK3(2)4L[2]SA, c = (0, 2 gamma, 3/5, 1)
    const double g = 1767732205903.0 / 4055673282236.0;
    const double t[16] = {0, 0, 0, 0,
                          g, g, 0, 0,
                          2746238789719.0 / 10658868560708.0, -640167445237.0 / 6845629431997.0, g, 0,
                          1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0,
                          11266239266428.0 / 11593286722821.0, g};
    std::memcpy(A, t, sizeof(t));
    return 4;
  }
  if (scheme == 4) {            // ESDIRK4(3)6L[2]SA, gamma = 1/4, c = (0, 1/2, 83/250, 31/50, 17/20, 1)
    const double g = 0.25;
    const double t[36] = {0, 0, 0, 0, 0, 0,
                          g, g, 0, 0, 0, 0,
                          8611.0 / 62500.0, -1743.0 / 31250.0, g, 0, 0, 0,
                          5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, g, 0, 0,
                          15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0,
                          2285395.0 / 8070912.0, g, 0,
                          82889.0 / 524892.0, 0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, g};
    std::memcpy(A, t, sizeof(t));
    return 6;
  }
  return 0;
}

}  // namespace

extern "C" int32_t esdirk_stages(int32_t scheme) {
  double A[64];
  return esdirk_tableau(scheme, A);
}

extern "C" int32_t esdirk_butcher(int32_t scheme, double* A_out) {
  double A[64];
  const int s = esdirk_tableau(scheme, A);
  if (A_out) std::memcpy(A_out, A, (size_t)s * s * sizeof(double));
  return s;
}

extern "C" pmg_status esdirk_step(const pmg_solve_opts* o, int32_t scheme, double dt, double* q, double* work,
                                  pmg_solve_stats* stats, int32_t n_stats, void* stream) {
  double A[64];
  const int s = esdirk_tableau(scheme, A);
  if (s == 0) return fail(PMG_E_ARG, "unknown ESDIRK scheme");
  if (!o || !q || !work || o->n_levels < 1 || !o->levels || !o->levels[0]) return fail(PMG_E_ARG, "null argument");
  if (o->stage_guess != 0 && o->stage_guess != 1) return fail(PMG_E_ARG, "stage_guess must be 0 or 1");
  if (o->ser_floor != 0 && o->ser_floor != 1) return fail(PMG_E_ARG, "ser_floor must be 0 or 1");
  if (o->lookahead < 0 || o->lookahead > 2) return fail(PMG_E_ARG, "lookahead must be 0, 1 or 2");
  if (!(dt > 0.0)) return fail(PMG_E_ARG, "dt must be positive");
  pmg_level L0 = o->levels[0];
  const size_t ns = L0->state_elems();
  double* qc_n = work;
  std::vector<const double*> R(s);
  for (int k = 0; k < s - 1; ++k) R[k] = work + (size_t)(k + 1) * ns;
  {
    DeviceGuard guard(L0->device);
    hipStream_t st = as_stream(stream);
    PMG_HIP(pmg::launch_conservative(*L0, q, qc_n, st));
    PMG_HIP(pmg::launch_residual(*L0, q, nullptr, nullptr, 0.0, const_cast<double*>(R[0]), false, st));
  }
  const double omega = A[1 * s + 1];
  pmg_status worst = PMG_OK;
  for (int i = 1; i < s; ++i) {
    double a_row[8];
    for (int j = 0; j < i; ++j) a_row[j] = A[i * s + j];
    pmg_solve_stats* sti = (stats && i - 1 < n_stats) ? &stats[i - 1] : nullptr;
    double* R_out = (i < s - 1) ? const_cast<double*>(R[i]) : nullptr;
    if (o->stage_guess == 1) {   // the explicit predictor; otherwise q holds the previous stage value
      DeviceGuard guard(L0->device);
      PMG_HIP(pmg::launch_stage_predict(*L0, qc_n, R.data(), a_row, i, dt, omega, q, as_stream(stream)));
    }
    const pmg_status r = esdirk_stage_solve(o, omega, dt, qc_n, R.data(), a_row, i, q, R_out, sti, stream);
    if (r == PMG_E_NOT_CONVERGED) {
      // the last iterate stands in for the stage value; later stages still run
      worst = r;
      if (R_out) {
        DeviceGuard guard(L0->device);
        PMG_HIP(pmg::launch_residual(*L0, q, nullptr, nullptr, 0.0, R_out, false, as_stream(stream)));
      }
    } else if (r != PMG_OK) {
      for (int k = i; k < s - 1 && stats && k < n_stats; ++k) stats[k].status = r;
      return r;
    }
  }
  if (worst != PMG_OK) return fail(worst, "a stage solve reached max_vcycles");
  return PMG_OK;
}

// ---- batches of independent cases -----------------------------------------------------------------
// Each case has its own levels (mesh, P) and factors; the batch owns one stream per case. A batched
// call forks the cases from the caller's stream, runs their stage solves concurrently (each on its
// stream, V-cycles replayed from each case's graph), synchronising case by case to read the norms
// the SER law needs, and joins them back into the caller's stream.
struct pmg_batch_s {
  int device = 0;
  std::vector<pmg_solve_opts> opts;
  std::vector<std::vector<pmg_level>> levels;
  std::vector<std::vector<pmg_factors>> factors;
  std::vector<std::vector<int32_t>> n_smooth;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  double* host_norms = nullptr;   // pinned, [cases][8]
};

namespace {

void free_batch(pmg_batch_s* B) {
  if (!B) return;
  for (hipStream_t s : B->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : B->done)
    if (e) (void)hipEventDestroy(e);
  if (B->fork) (void)hipEventDestroy(B->fork);
  if (B->host_norms) (void)hipHostFree(B->host_norms);
  delete B;
}

pmg_status batch_fork(pmg_batch B, hipStream_t caller) {
  PMG_HIP(hipEventRecord(B->fork, caller));
  for (hipStream_t s : B->streams) PMG_HIP(hipStreamWaitEvent(s, B->fork, 0));
  return PMG_OK;
}

pmg_status batch_join(pmg_batch B, hipStream_t caller) {
  for (size_t c = 0; c < B->streams.size(); ++c) {
    PMG_HIP(hipEventRecord(B->done[c], B->streams[c]));
    PMG_HIP(hipStreamWaitEvent(caller, B->done[c], 0));
  }
  return PMG_OK;
}

}  // namespace

extern "C" pmg_status pmg_batch_create(const pmg_solve_opts* cases, int32_t n_cases, pmg_batch* out) {
  if (!cases || !out) return fail(PMG_E_ARG, "null argument");
  *out = nullptr;
  if (n_cases < 1 || n_cases > 64) return fail(PMG_E_ARG, "n_cases must be in 1..64");
  for (int c = 0; c < n_cases; ++c) {
    if (pmg_status e = check_opts(&cases[c])) return e;
    if (cases[c].levels[0]->device != cases[0].levels[0]->device)
      return fail(PMG_E_SHAPE, "all cases of a batch must live on one device");
    for (int d = 0; d < c; ++d)
      for (int l = 0; l < cases[c].n_levels; ++l)
        for (int k = 0; k < cases[d].n_levels; ++k)
          if (cases[c].levels[l] == cases[d].levels[k])
            return fail(PMG_E_ARG, "cases of a batch must not share levels (their workspaces would race)");
  }
  pmg_batch_s* B = new pmg_batch_s();
  B->device = cases[0].levels[0]->device;
  DeviceGuard guard(B->device);
  B->opts.assign(cases, cases + n_cases);
  B->levels.resize(n_cases);
  B->factors.resize(n_cases);
  B->n_smooth.resize(n_cases);
  for (int c = 0; c < n_cases; ++c) {
    const pmg_solve_opts& o = cases[c];
    B->levels[c].assign(o.levels, o.levels + o.n_levels);
    B->factors[c].assign(o.factors, o.factors + o.n_levels);
    B->n_smooth[c].assign(o.n_smooth, o.n_smooth + o.n_levels);
    B->opts[c].levels = B->levels[c].data();
    B->opts[c].factors = B->factors[c].data();
    B->opts[c].n_smooth = B->n_smooth[c].data();
  }
  B->streams.assign(n_cases, nullptr);
  B->done.assign(n_cases, nullptr);
  for (int c = 0; c < n_cases; ++c) {
    if (hipStreamCreateWithFlags(&B->streams[c], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->done[c], hipEventDisableTiming) != hipSuccess) {
      free_batch(B);
      return fail(PMG_E_HIP, "stream or event creation failed");
    }
  }
  if (hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&B->host_norms), sizeof(double) * 8 * n_cases) != hipSuccess) {
    free_batch(B);
    return fail(PMG_E_NOMEM, "batch host buffers");
  }
  *out = B;
  return PMG_OK;
}

extern "C" pmg_status pmg_batch_destroy(pmg_batch B) {
  if (!B) return PMG_OK;
  DeviceGuard guard(B->device);
  for (hipStream_t s : B->streams)
    if (s) (void)hipStreamSynchronize(s);
  free_batch(B);
  return PMG_OK;
}

extern "C" int32_t pmg_batch_size(pmg_batch B) { return B ? (int32_t)B->opts.size() : 0; }

namespace {

// The cases with run[c] set, each solved as by esdirk_stage_solve; a case's own failure (a
// non-finite residual, a singular block, max_vcycles) ends only that case, and its status is
// left in status[c].
pmg_status stage_solve_cases(pmg_batch B, const std::vector<char>& run, const double* omega, const double* dt,
                             const double* const* qc_n, const double* const* const* R_prev,
                             const double* const* a_row, const int32_t* n_prev, double* const* q,
                             double* const* R_out, pmg_solve_stats* stats, std::vector<pmg_status>& status,
                             hipStream_t caller) {
  const int n = (int)B->opts.size();
  if (pmg_status e = batch_fork(B, caller)) return e;
  std::vector<StageRun> runs(n);
  std::vector<char> begun(n, 0);
  for (int c = 0; c < n; ++c) {
    status[c] = PMG_OK;
    if (!run[c]) continue;
    runs[c].host_norms = B->host_norms + 8 * c;
    const bool steady = !(dt[c] > 0.0);
    status[c] = stage_begin(runs[c], &B->opts[c], omega[c], dt[c], steady ? nullptr : qc_n[c],
                            steady ? nullptr : R_prev[c], steady ? nullptr : a_row[c], steady ? 0 : n_prev[c], q[c],
                            R_out ? R_out[c] : nullptr, stats ? &stats[c] : nullptr, B->streams[c]);
    begun[c] = status[c] == PMG_OK;
  }
  for (bool any = true; any;) {
    any = false;
    for (int c = 0; c < n; ++c) {
      if (!begun[c] || !runs[c].active) continue;
      PMG_HIP(hipStreamSynchronize(B->streams[c]));
      if (pmg_status e = stage_advance(runs[c])) {
        (void)batch_join(B, caller);
        return e;
      }
      any = any || runs[c].active;
    }
  }
  for (int c = 0; c < n; ++c)
    if (begun[c]) status[c] = stage_finish(runs[c]);
  return batch_join(B, caller);
}

pmg_status worst_of(const std::vector<pmg_status>& status) {
  pmg_status worst = PMG_OK;
  for (pmg_status r : status)
    if (r != PMG_OK && (worst == PMG_OK || worst == PMG_E_NOT_CONVERGED)) worst = r;
  return worst;
}

}  // namespace

extern "C" pmg_status esdirk_stage_solve_batched(pmg_batch B, const double* omega, const double* dt,
                                                 const double* const* qc_n, const double* const* const* R_prev,
                                                 const double* const* a_row, const int32_t* n_prev, double* const* q,
                                                 double* const* R_out, pmg_solve_stats* stats, void* stream) {
  if (!B || !omega || !dt || !q) return fail(PMG_E_ARG, "null argument");
  const int n = (int)B->opts.size();
  DeviceGuard guard(B->device);
  std::vector<char> run(n, 1);
  std::vector<pmg_status> status(n, PMG_OK);
  if (pmg_status e = stage_solve_cases(B, run, omega, dt, qc_n, R_prev, a_row, n_prev, q, R_out, stats, status,
                                       as_stream(stream)))
    return e;
  const pmg_status worst = worst_of(status);
  if (worst == PMG_E_NOT_CONVERGED) return fail(worst, "a stage solve of the batch reached max_vcycles");
  return worst;
}

extern "C" pmg_status esdirk_step_batched(pmg_batch B, int32_t scheme, const double* dt, double* const* q,
                                          double* const* work, pmg_solve_stats* stats, void* stream) {
  double A[64];
  const int s = esdirk_tableau(scheme, A);
  if (s == 0) return fail(PMG_E_ARG, "unknown ESDIRK scheme");
  if (!B || !dt || !q || !work) return fail(PMG_E_ARG, "null argument");
  const int n = (int)B->opts.size();
  for (int c = 0; c < n; ++c)
    if (!q[c] || !work[c] || !(dt[c] > 0.0)) return fail(PMG_E_ARG, "null state or non-positive dt");
  DeviceGuard guard(B->device);
  const hipStream_t caller = as_stream(stream);
  // per case: q_c^n and R(q^n) into the first two work slots (on the caller's stream)
  std::vector<std::vector<const double*>> R(n, std::vector<const double*>(s));
  std::vector<const double*> qc(n);
  for (int c = 0; c < n; ++c) {
    pmg_level L0 = B->opts[c].levels[0];
    const size_t ns = L0->state_elems();
    qc[c] = work[c];
    for (int k = 0; k < s - 1; ++k) R[c][k] = work[c] + (size_t)(k + 1) * ns;
    PMG_HIP(pmg::launch_conservative(*L0, q[c], work[c], caller));
    PMG_HIP(pmg::launch_residual(*L0, q[c], nullptr, nullptr, 0.0, const_cast<double*>(R[c][0]), false, caller));
  }
  const double omega = A[1 * s + 1];
  std::vector<double> om(n, omega);
  std::vector<const double* const*> Rp(n);
  std::vector<int32_t> np(n);
  std::vector<double*> Rout(n);
  std::vector<pmg_solve_stats> st_i(n);
  std::vector<char> run(n, 1);                   // cases still advancing (a hard failure stops one)
  std::vector<pmg_status> step_status(n, PMG_OK), status(n, PMG_OK);
  for (int i = 1; i < s; ++i) {
    double a_row[8];
    for (int j = 0; j < i; ++j) a_row[j] = A[i * s + j];
    std::vector<const double*> ar(n, a_row);
    for (int c = 0; c < n; ++c) {
      Rp[c] = R[c].data();
      np[c] = i;
      Rout[c] = (i < s - 1) ? const_cast<double*>(R[c][i]) : nullptr;
      st_i[c] = stats ? stats[c * (s - 1) + (i - 1)] : pmg_solve_stats{};
      if (!stats) st_i[c].history = nullptr;
      if (run[c] && B->opts[c].stage_guess == 1)   // the explicit predictor as the stage's guess
        PMG_HIP(pmg::launch_stage_predict(*B->opts[c].levels[0], qc[c], R[c].data(), a_row, i, dt[c], omega, q[c],
                                          caller));
    }
    if (pmg_status e = stage_solve_cases(B, run, om.data(), dt, qc.data(), Rp.data(), ar.data(), np.data(), q,
                                         Rout.data(), st_i.data(), status, caller))
      return e;
    for (int c = 0; c < n; ++c) {
      if (!run[c]) {
        st_i[c].status = step_status[c];          // a case stopped earlier in this step
        st_i[c].n_vcycles = 0;
      } else if (status[c] == PMG_E_NOT_CONVERGED) {
        // the last iterate stands in for the stage value; later stages still run
        if (step_status[c] == PMG_OK) step_status[c] = PMG_E_NOT_CONVERGED;
        if (Rout[c])
          PMG_HIP(pmg::launch_residual(*B->opts[c].levels[0], q[c], nullptr, nullptr, 0.0, Rout[c], false, caller));
      } else if (status[c] != PMG_OK) {
        step_status[c] = status[c];
        run[c] = 0;
      }
      if (stats) stats[c * (s - 1) + (i - 1)] = st_i[c];
    }
  }
  PMG_HIP(hipStreamSynchronize(caller));
  const pmg_status worst = worst_of(step_status);
  if (worst == PMG_E_NOT_CONVERGED) return fail(worst, "a stage solve of the batch reached max_vcycles");
  if (worst != PMG_OK) return fail(worst, "a case of the batch failed (see its stats)");
  return PMG_OK;
}
