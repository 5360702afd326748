// Host-side setup of the bake-off operators: 1D rules, Lagrange matrices and
// the geometric factors (section 3: all geometric data are precomputed).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "bp_internal.h"

namespace bp {

namespace {

// P_n(x) and P_{n-1}(x) by the three-term recurrence (k+1)P_{k+1} =
// (2k+1) x P_k - k P_{k-1}.
void legendre_pair(int n, double x, double *pn, double *pnm1) {
  double a = 1.0, b = x;  // P_0, P_1
  if (n == 0) {
    *pn = 1.0;
    *pnm1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  *pn = b;
  *pnm1 = a;
}

double legendre(int n, double x) {
  double pn, pm;
  legendre_pair(n, x, &pn, &pm);
  return pn;
}

}  // namespace

// GLL points: the zeros of (1 - x^2) P_p'(x), which are the zeros of
// f = P_{p+1} - P_{p-1} (f' = (2p+1) P_p). Weights 2 / (p (p+1) P_p(x)^2).
void gll_rule(int n, double *x, double *w) {
  const int p = n - 1;
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    double t = -std::cos(pi * j / p);
    if (j > 0 && j < p) {
      for (int it = 0; it < 100; ++it) {
        double pp1 = legendre(p + 1, t), pm1 = legendre(p - 1, t);
        double dt = (pp1 - pm1) / ((2 * p + 1) * legendre(p, t));
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
    }
    x[j] = t;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  // exact symmetry
  for (int j = 0; j < n / 2; ++j) {
    double s = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -s;
    x[n - 1 - j] = s;
  }
  if (n % 2) x[n / 2] = 0.0;
  if (w)
    for (int j = 0; j < n; ++j) {
      double lp = legendre(p, x[j]);
      w[j] = 2.0 / (p * (p + 1) * lp * lp);
    }
}

// GL points: zeros of P_n; P_n' = n (x P_n - P_{n-1}) / (x^2 - 1).
// Weights 2 / ((1 - x^2) P_n'(x)^2).
void gl_rule(int n, double *x, double *w) {
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    double t = -std::cos(pi * (j + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre_pair(n, t, &pn, &pm);
      dp = n * (t * pn - pm) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, pm;
    legendre_pair(n, t, &pn, &pm);
    dp = n * (t * pn - pm) / (t * t - 1.0);
    x[j] = t;
    if (w) w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  for (int j = 0; j < n / 2; ++j) {
    double s = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -s;
    x[n - 1 - j] = s;
    if (w) {
      double ws = 0.5 * (w[j] + w[n - 1 - j]);
      w[j] = w[n - 1 - j] = ws;
    }
  }
  if (n % 2) x[n / 2] = 0.0;
}

// Barycentric weights lambda_j = 1 / prod_{m != j} (x_j - x_m).
static std::vector<double> bary_weights(int n, const double *nodes) {
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) lam[j] /= (nodes[j] - nodes[m]);
  return lam;
}

static int node_hit(int n, const double *nodes, double x) {
  for (int m = 0; m < n; ++m)
    if (x == nodes[m]) return m;
  return -1;
}

void lagrange_interp(int n, const double *nodes, int m, const double *pts, double *out) {
  auto lam = bary_weights(n, nodes);
  for (int a = 0; a < m; ++a) {
    double *row = out + (size_t)a * n;
    int hit = node_hit(n, nodes, pts[a]);
    if (hit >= 0) {
      for (int j = 0; j < n; ++j) row[j] = (j == hit) ? 1.0 : 0.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += lam[j] / (pts[a] - nodes[j]);
    for (int j = 0; j < n; ++j) row[j] = lam[j] / (pts[a] - nodes[j]) / den;
  }
}

// At a node x_a: D_aj = (lam_j / lam_a) / (x_a - x_j), D_aa = -sum_{j != a} D_aj.
// Elsewhere: h_j'(x) = h_j(x) * sum_{m != j} 1 / (x - x_m).
void lagrange_deriv(int n, const double *nodes, int m, const double *pts, double *out) {
  auto lam = bary_weights(n, nodes);
  std::vector<double> h(n);
  for (int a = 0; a < m; ++a) {
    double *row = out + (size_t)a * n;
    int hit = node_hit(n, nodes, pts[a]);
    if (hit >= 0) {
      double diag = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == hit) continue;
        row[j] = (lam[j] / lam[hit]) / (nodes[hit] - nodes[j]);
        diag -= row[j];
      }
      row[hit] = diag;
      continue;
    }
    lagrange_interp(n, nodes, 1, &pts[a], h.data());
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (k != j) s += 1.0 / (pts[a] - nodes[k]);
      row[j] = h[j] * s;
    }
  }
}

Basis make_basis(int p, int q, int quad) {
  Basis b;
  b.p1 = p + 1;
  b.q = q;
  b.xi.resize(b.p1);
  gll_rule(b.p1, b.xi.data(), nullptr);
  b.eta.resize(q);
  b.rho.resize(q);
  if (quad == BP_QUAD_GLL)
    gll_rule(q, b.eta.data(), b.rho.data());
  else
    gl_rule(q, b.eta.data(), b.rho.data());
  b.colloc = (quad == BP_QUAD_GLL && q == b.p1);
  b.J.assign((size_t)q * b.p1, 0.0);
  b.D.assign((size_t)q * b.p1, 0.0);
  b.Dq.assign((size_t)q * q, 0.0);
  if (b.colloc) {
    b.eta = b.xi;
    for (int a = 0; a < q; ++a) b.J[(size_t)a * b.p1 + a] = 1.0;
  } else {
    lagrange_interp(b.p1, b.xi.data(), q, b.eta.data(), b.J.data());
  }
  lagrange_deriv(b.p1, b.xi.data(), q, b.eta.data(), b.D.data());
  lagrange_deriv(q, b.eta.data(), q, b.eta.data(), b.Dq.data());
  return b;
}

// Geometric factors of one element. For collocated GLL the derivatives of the
// coordinates are taken with D^ directly at the nodes; otherwise the nodes are
// first interpolated to the quadrature points (J^ in each direction) and then
// differentiated there with the q x q matrix Dq (exact: x is a polynomial of
// degree p < q in each variable).
static bool element_factors(const Basis &b, const double *X, double *G, double *Bt,
                            std::vector<double> &s1, std::vector<double> &s2,
                            std::vector<double> &Xq) {
  const int p1 = b.p1, q = b.q;
  const int nq = q * q * q;
  // Xq[c][b][a][l]: coordinate l at quadrature point (a, b, c)
  if (b.colloc) {
    for (int n = 0; n < nq; ++n)
      for (int l = 0; l < 3; ++l) Xq[n * 3 + l] = X[n * 3 + l];
  } else {
    // along i: s1[k][j][a][l]
    for (int k = 0; k < p1; ++k)
      for (int j = 0; j < p1; ++j)
        for (int a = 0; a < q; ++a)
          for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int i = 0; i < p1; ++i)
              s += b.J[a * p1 + i] * X[((k * p1 + j) * p1 + i) * 3 + l];
            s1[((k * p1 + j) * q + a) * 3 + l] = s;
          }
    // along j: s2[k][bb][a][l]
    for (int k = 0; k < p1; ++k)
      for (int bb = 0; bb < q; ++bb)
        for (int a = 0; a < q; ++a)
          for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int j = 0; j < p1; ++j)
              s += b.J[bb * p1 + j] * s1[((k * p1 + j) * q + a) * 3 + l];
            s2[((k * q + bb) * q + a) * 3 + l] = s;
          }
    // along k
    for (int c = 0; c < q; ++c)
      for (int bb = 0; bb < q; ++bb)
        for (int a = 0; a < q; ++a)
          for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int k = 0; k < p1; ++k)
              s += b.J[c * p1 + k] * s2[((k * q + bb) * q + a) * 3 + l];
            Xq[((c * q + bb) * q + a) * 3 + l] = s;
          }
  }
  const double *Dm = b.colloc ? b.D.data() : b.Dq.data();  // q x q in both cases
  bool ok = true;
  for (int c = 0; c < q; ++c)
    for (int bb = 0; bb < q; ++bb)
      for (int a = 0; a < q; ++a) {
        double M[3][3];  // M[l][m] = dx_l / dr_m
        for (int l = 0; l < 3; ++l) {
          double dr = 0.0, ds = 0.0, dt = 0.0;
          for (int m = 0; m < q; ++m) {
            dr += Dm[a * q + m] * Xq[((c * q + bb) * q + m) * 3 + l];
            ds += Dm[bb * q + m] * Xq[((c * q + m) * q + a) * 3 + l];
            dt += Dm[c * q + m] * Xq[((m * q + bb) * q + a) * 3 + l];
          }
          M[l][0] = dr;
          M[l][1] = ds;
          M[l][2] = dt;
        }
        // cofactor matrix: inverse = cof^T / det, (dr_m/dx_l) = cof[l][m] / det
        double cof[3][3];
        cof[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        cof[0][1] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        cof[0][2] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        cof[1][0] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
        cof[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
        cof[1][2] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
        cof[2][0] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
        cof[2][1] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
        cof[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        const double det = M[0][0] * cof[0][0] + M[0][1] * cof[0][1] + M[0][2] * cof[0][2];
        if (!(det > 0.0) || !std::isfinite(det)) ok = false;
        const double wq = b.rho[a] * b.rho[bb] * b.rho[c];
        // G_mm' = sum_l (dr_m/dx_l)(dr_m'/dx_l) det w = sum_l cof[l][m] cof[l][m'] w / det
        const double s = wq / det;
        const int n = (c * q + bb) * q + a;
        int comp = 0;
        for (int m = 0; m < 3; ++m)
          for (int mp = m; mp < 3; ++mp) {
            double g = 0.0;
            for (int l = 0; l < 3; ++l) g += cof[l][m] * cof[l][mp];
            G[(size_t)comp * nq + n] = g * s;
            ++comp;
          }
        Bt[n] = det * wq;
      }
  return ok;
}

int64_t geometric_factors(const Basis &b, int64_t nelem, const double *node_xyz,
                          double *G, double *Bt, int nthreads) {
  const int p1 = b.p1, q = b.q;
  const int64_t n3 = (int64_t)p1 * p1 * p1, nq = (int64_t)q * q * q;
  std::atomic<int64_t> bad(INT64_MAX);
  std::atomic<int64_t> next(0);
  const int64_t chunk = 256;
  auto work = [&]() {
    std::vector<double> s1((size_t)p1 * p1 * q * 3), s2((size_t)p1 * q * q * 3),
        Xq((size_t)nq * 3);
    for (;;) {
      int64_t e0 = next.fetch_add(chunk);
      if (e0 >= nelem) break;
      int64_t e1 = std::min(nelem, e0 + chunk);
      for (int64_t e = e0; e < e1; ++e) {
        bool ok = element_factors(b, node_xyz + e * n3 * 3, G + e * 6 * nq, Bt + e * nq,
                                  s1, s2, Xq);
        if (!ok) {
          int64_t cur = bad.load();
          while (e < cur && !bad.compare_exchange_weak(cur, e)) {
          }
        }
      }
    }
  };
  nthreads = std::max(1, std::min<int>(nthreads, (int)((nelem + chunk - 1) / chunk)));
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  int64_t r = bad.load();
  return r == INT64_MAX ? -1 : r;
}

}  // namespace bp
