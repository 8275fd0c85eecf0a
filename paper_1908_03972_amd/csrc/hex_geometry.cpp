// Host-side geometry of hexahedral levels: solution points, curl-form metric terms, face vectors
// and the element length scale of eqs. (32)-(33).
//
// The metric vectors J grad xi^i are taken in Kopriva's conservative curl form,
//   (J grad xi^i)_n = -[curl_xi I_Q(X_l grad_xi X_m)]_i,  (n, m, l) cyclic,
// with I_Q the interpolant at the (Q+1)^3 Gauss-Lobatto points (Q = max(P, 1)): for P >= 1 the
// result is a polynomial of degree <= P per direction whose discrete divergence vanishes at the
// Gauss points, and whose normal component on a face depends only on that face's geometry, so a
// uniform flow stays uniform and both elements of a face see the same face vector.
#include <cmath>
#include <string>
#include <vector>

namespace pmg {

namespace {

// Lagrange basis l_k(t) on nodes x and its derivative
double lag(const std::vector<double>& x, int k, double t) {
  double r = 1.0;
  for (size_t m = 0; m < x.size(); ++m)
    if ((int)m != k) r *= (t - x[m]) / (x[k] - x[m]);
  return r;
}

double dlag(const std::vector<double>& x, int k, double t) {
  double s = 0.0;
  for (size_t a = 0; a < x.size(); ++a) {
    if ((int)a == k) continue;
    double term = 1.0 / (x[k] - x[a]);
    for (size_t m = 0; m < x.size(); ++m)
      if ((int)m != k && m != a) term *= (t - x[m]) / (x[k] - x[m]);
    s += term;
  }
  return s;
}

// x(xi) and dx/dxi of the (g+1)^3-node Lagrange map of one element, node a + (g+1) b + (g+1)^2 c
void hex_map(const double* nodes, int g, const double ref[3], double X[3], double dX[3][3]) {
  std::vector<double> gn(g + 1);
  for (int a = 0; a <= g; ++a) gn[a] = -1.0 + 2.0 * a / g;
  double L[3][3], dL[3][3];
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a <= g; ++a) {
      L[d][a] = lag(gn, a, ref[d]);
      dL[d][a] = dlag(gn, a, ref[d]);
    }
  for (int n = 0; n < 3; ++n) {
    X[n] = 0.0;
    for (int k = 0; k < 3; ++k) dX[n][k] = 0.0;
  }
  const int n1 = g + 1;
  for (int c = 0; c <= g; ++c)
    for (int b = 0; b <= g; ++b)
      for (int a = 0; a <= g; ++a) {
        const double* x = nodes + 3 * (a + n1 * (b + n1 * c));
        const double s = L[0][a] * L[1][b] * L[2][c];
        const double s0 = dL[0][a] * L[1][b] * L[2][c];
        const double s1 = L[0][a] * dL[1][b] * L[2][c];
        const double s2 = L[0][a] * L[1][b] * dL[2][c];
        for (int n = 0; n < 3; ++n) {
          X[n] += s * x[n];
          dX[n][0] += s0 * x[n];
          dX[n][1] += s1 * x[n];
          dX[n][2] += s2 * x[n];
        }
      }
}

double det3(const double m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// Gauss-Legendre points (Newton on the three-term recurrence)
void gauss_points(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = (n == 0) ? 1.0 : p1, pm = (n == 0) ? 0.0 : p0;
      const double dp = n * (t * pn - pm) / (t * t - 1.0);
      const double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) {
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
        break;
      }
      w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    x[i] = -t;
  }
}

}  // namespace

// Fills, for Ne elements of geometry order g at degree P with Gauss points x1:
//   met  [10][Np][Ne]  J grad xi^d (component n at 3 d + n), then 1/|J|
//   fvec [6][(P+1)^2][4][Ne] unit +xi^(f/2) vector and its length at face points k1 + (P+1) k2
//   xyz  [3][Np][Ne]   solution-point coordinates
//   dx   [Ne]          twice the smallest distance from the volume centroid to a face plane
// Returns an empty string, or the reason the mesh is rejected.
std::string build_hex_geometry(const double* nodes, int ne, int g, int P, const std::vector<double>& x1,
                               std::vector<double>& met, std::vector<double>& fvec, std::vector<double>& xyz,
                               std::vector<double>& dx) {
  const int n1 = P + 1, np = n1 * n1 * n1, nf = n1 * n1, nn = (g + 1) * (g + 1) * (g + 1);
  const int Q = P > 1 ? P : 1, nq = Q + 1;
  std::vector<double> y;
  if (Q == 1) y = {-1.0, 1.0};
  else if (Q == 2) y = {-1.0, 0.0, 1.0};
  else if (Q == 3) y = {-1.0, -1.0 / std::sqrt(5.0), 1.0 / std::sqrt(5.0), 1.0};
  else return "3-D levels support P <= 3";
  // GL derivative matrix Dg[a][b] = l_b'(y_a) and GL -> Gauss interpolation Lv[i][a] = l_a(x_i)
  std::vector<double> Dg(nq * nq), Lv(n1 * nq);
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) Dg[a * nq + b] = dlag(y, b, y[a]);
  for (int i = 0; i < n1; ++i)
    for (int a = 0; a < nq; ++a) Lv[i * nq + a] = lag(y, a, x1[i]);
  met.assign((size_t)10 * np * ne, 0.0);
  fvec.assign((size_t)6 * nf * 4 * ne, 0.0);
  xyz.assign((size_t)3 * np * ne, 0.0);
  dx.assign(ne, 0.0);
  const size_t st = (size_t)np * ne;
  const int ng = nq * nq * nq;
  std::vector<double> Xg(3 * ng), dXg(9 * ng), V(3 * ng), Ja(9 * ng);   // Ja[(i*3 + n)*ng + grid]
  std::vector<double> xq, wq;
  gauss_points(5, xq, wq);
  for (int e = 0; e < ne; ++e) {
    const double* nd = nodes + (size_t)e * nn * 3;
    for (int c = 0; c < nq; ++c)
      for (int b = 0; b < nq; ++b)
        for (int a = 0; a < nq; ++a) {
          const int gi = a + nq * (b + nq * c);
          const double ref[3] = {y[a], y[b], y[c]};
          double X[3], dX[3][3];
          hex_map(nd, g, ref, X, dX);
          for (int n = 0; n < 3; ++n) {
            Xg[n * ng + gi] = X[n];
            for (int k = 0; k < 3; ++k) dXg[(n * 3 + k) * ng + gi] = dX[n][k];
          }
        }
    // derivative of grid values u along reference direction d at grid point (a, b, c)
    auto dref = [&](const double* u, int d, int a, int b, int c) {
      double s = 0.0;
      for (int m = 0; m < nq; ++m) {
        const int gi = (d == 0) ? m + nq * (b + nq * c) : (d == 1) ? a + nq * (m + nq * c) : a + nq * (b + nq * m);
        const int row = (d == 0) ? a : (d == 1) ? b : c;
        s += Dg[row * nq + m] * u[gi];
      }
      return s;
    };
    for (int n = 0; n < 3; ++n) {
      const int m = (n + 1) % 3, l = (n + 2) % 3;
      // V_k = X_l dX_m/dxi^k, stored as V[k*ng + grid]
      for (int gi = 0; gi < ng; ++gi)
        for (int k = 0; k < 3; ++k) V[k * ng + gi] = Xg[l * ng + gi] * dXg[(m * 3 + k) * ng + gi];
      for (int c = 0; c < nq; ++c)
        for (int b = 0; b < nq; ++b)
          for (int a = 0; a < nq; ++a) {
            const int gi = a + nq * (b + nq * c);
            const double c0 = dref(&V[2 * ng], 1, a, b, c) - dref(&V[1 * ng], 2, a, b, c);
            const double c1 = dref(&V[0 * ng], 2, a, b, c) - dref(&V[2 * ng], 0, a, b, c);
            const double c2 = dref(&V[1 * ng], 0, a, b, c) - dref(&V[0 * ng], 1, a, b, c);
            Ja[(0 * 3 + n) * ng + gi] = -c0;
            Ja[(1 * 3 + n) * ng + gi] = -c1;
            Ja[(2 * 3 + n) * ng + gi] = -c2;
          }
    }
    // solution points: interpolated metric polynomial, exact Jacobian and coordinates
    for (int k = 0; k < n1; ++k)
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
          const int p = i + n1 * (j + n1 * k);
          const size_t o = (size_t)p * ne + e;
          for (int in = 0; in < 9; ++in) {
            double s = 0.0;
            for (int c = 0; c < nq; ++c)
              for (int b = 0; b < nq; ++b)
                for (int a = 0; a < nq; ++a)
                  s += Lv[i * nq + a] * Lv[j * nq + b] * Lv[k * nq + c] * Ja[in * ng + a + nq * (b + nq * c)];
            met[in * st + o] = s;
          }
          const double ref[3] = {x1[i], x1[j], x1[k]};
          double X[3], dX[3][3];
          hex_map(nd, g, ref, X, dX);
          const double J = det3(dX);
          if (!(J > 0.0)) return "non-positive mapping Jacobian in element " + std::to_string(e);
          met[9 * st + o] = 1.0 / J;
          for (int n = 0; n < 3; ++n) xyz[n * st + o] = X[n];
        }
    // face points: the same polynomial on the face (a Gauss-Lobatto grid plane)
    for (int f = 0; f < 6; ++f) {
      const int d = f / 2, end = (f % 2 == 0) ? 0 : Q;
      for (int k2 = 0; k2 < n1; ++k2)
        for (int k1 = 0; k1 < n1; ++k1) {
          double v3[3] = {0.0, 0.0, 0.0};
          for (int t2 = 0; t2 < nq; ++t2)
            for (int t1 = 0; t1 < nq; ++t1) {
              const int gi = (d == 0) ? end + nq * (t1 + nq * t2) : (d == 1) ? t1 + nq * (end + nq * t2)
                                                                             : t1 + nq * (t2 + nq * end);
              const double wgt = Lv[k1 * nq + t1] * Lv[k2 * nq + t2];
              for (int n = 0; n < 3; ++n) v3[n] += wgt * Ja[(d * 3 + n) * ng + gi];
            }
          const double len = std::sqrt(v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2]);
          const size_t o = ((size_t)(f * nf + k1 + n1 * k2) * 4) * ne + e;
          for (int n = 0; n < 3; ++n) fvec[o + n * ne] = v3[n] / len;
          fvec[o + 3 * ne] = len;
        }
    }
    // element length: volume centroid (5^3 Gauss rule) to the nearest face plane, twice
    double vol = 0.0, cen[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 5; ++c)
      for (int b = 0; b < 5; ++b)
        for (int a = 0; a < 5; ++a) {
          const double ref[3] = {xq[a], xq[b], xq[c]};
          double X[3], dX[3][3];
          hex_map(nd, g, ref, X, dX);
          const double wj = wq[a] * wq[b] * wq[c] * det3(dX);
          vol += wj;
          for (int n = 0; n < 3; ++n) cen[n] += wj * X[n];
        }
    for (int n = 0; n < 3; ++n) cen[n] /= vol;
    const int gn1 = g + 1;
    auto nidx = [&](int a, int b, int c) { return a + gn1 * (b + gn1 * c); };
    double dmin = 1e300;
    for (int f = 0; f < 6; ++f) {
      const int end = (f % 2 == 0) ? 0 : g, h = g / 2;
      int cr[4], mid;
      if (f < 2) {
        cr[0] = nidx(end, 0, 0); cr[1] = nidx(end, g, 0); cr[2] = nidx(end, g, g); cr[3] = nidx(end, 0, g);
        mid = nidx(end, h, h);
      } else if (f < 4) {
        cr[0] = nidx(0, end, 0); cr[1] = nidx(g, end, 0); cr[2] = nidx(g, end, g); cr[3] = nidx(0, end, g);
        mid = nidx(h, end, h);
      } else {
        cr[0] = nidx(0, 0, end); cr[1] = nidx(g, 0, end); cr[2] = nidx(g, g, end); cr[3] = nidx(0, g, end);
        mid = nidx(h, h, end);
      }
      double d1[3], d2[3], nrm[3], p0[3];
      for (int n = 0; n < 3; ++n) {
        d1[n] = nd[3 * cr[2] + n] - nd[3 * cr[0] + n];
        d2[n] = nd[3 * cr[3] + n] - nd[3 * cr[1] + n];
      }
      nrm[0] = d1[1] * d2[2] - d1[2] * d2[1];
      nrm[1] = d1[2] * d2[0] - d1[0] * d2[2];
      nrm[2] = d1[0] * d2[1] - d1[1] * d2[0];
      const double ln = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      if (g % 2 == 0) {
        for (int n = 0; n < 3; ++n) p0[n] = nd[3 * mid + n];
      } else {
        for (int n = 0; n < 3; ++n) p0[n] = 0.25 * (nd[3 * cr[0] + n] + nd[3 * cr[1] + n] + nd[3 * cr[2] + n] +
                                                   nd[3 * cr[3] + n]);
      }
      const double dist = std::fabs((cen[0] - p0[0]) * nrm[0] + (cen[1] - p0[1]) * nrm[1] +
                                    (cen[2] - p0[2]) * nrm[2]) / ln;
      dmin = std::fmin(dmin, dist);
    }
    dx[e] = 2.0 * dmin;
  }
  return std::string();
}

}  // namespace pmg
