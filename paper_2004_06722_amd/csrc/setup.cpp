// Host-side setup of the bake-off operators: 1D rules and Lagrange matrices
// (the geometric factors of section 3 are computed on the device at set-up).
#include <algorithm>
#include <cmath>

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

}  // namespace bp

namespace bp {

// Internal node order of an operator (see bp_internal.h).
bool interior_first_order(int p1, int64_t nelem, int64_t nglobal, const int64_t *ed,
                          std::vector<int32_t> &new_of_old, std::vector<int32_t> &old_of_new,
                          int64_t *n_owned) {
  *n_owned = 0;
  if (p1 < 3) return false;  // no element-interior nodes
  const int64_t n3 = (int64_t)p1 * p1 * p1;
  std::vector<int32_t> inner;  // element-interior local ids, ascending
  for (int64_t l = 0; l < n3; ++l) {
    const int i = (int)(l % p1), j = (int)(l / p1 % p1), k = (int)(l / ((int64_t)p1 * p1));
    if (i > 0 && i < p1 - 1 && j > 0 && j < p1 - 1 && k > 0 && k < p1 - 1)
      inner.push_back((int32_t)l);
  }
  // references per node, saturated at 2
  std::vector<uint8_t> refs((size_t)nglobal, 0);
  for (int64_t k = 0; k < nelem * n3; ++k) {
    uint8_t &r = refs[(size_t)ed[k]];
    if (r < 2) ++r;
  }
  for (int64_t e = 0; e < nelem; ++e)
    for (int32_t l : inner)
      if (refs[(size_t)ed[e * n3 + l]] != 1) return false;
  new_of_old.assign((size_t)nglobal, -1);
  int32_t next = 0;
  for (int64_t e = 0; e < nelem; ++e)
    for (int32_t l : inner) new_of_old[(size_t)ed[e * n3 + l]] = next++;
  *n_owned = next;
  for (int64_t k = 0; k < nelem * n3; ++k) {
    int32_t &v = new_of_old[(size_t)ed[k]];
    if (v < 0) v = next++;
  }
  for (int64_t g = 0; g < nglobal; ++g)  // nodes no element references
    if (new_of_old[(size_t)g] < 0) new_of_old[(size_t)g] = next++;
  old_of_new.assign((size_t)nglobal, 0);
  for (int64_t g = 0; g < nglobal; ++g) old_of_new[(size_t)new_of_old[(size_t)g]] = (int32_t)g;
  return true;
}

}  // namespace bp
