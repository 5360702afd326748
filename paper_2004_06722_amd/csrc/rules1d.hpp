// 1D rules and Lagrange matrices of section 5 (the GLL nodes of the basis,
// Gauss-Legendre or GLL quadrature points, J^ and D^), written as constexpr
// functions so that the same code gives the host set-up its tables at run
// time and the kernels theirs at compile time, as immediates the compiler can
// rematerialise instead of holding them in scalar registers (the even-odd
// tables of two 9 x 8 matrices do not fit in the scalar register file).
//
// Methods: Newton iteration on the three-term Legendre recurrence for the
// points, barycentric Lagrange weights for the interpolation and derivative
// matrices. kMaxRule bounds the number of points.
#pragma once

namespace bp {

constexpr int kMaxRule = 64;

constexpr double cx_abs(double x) { return x < 0 ? -x : x; }

// cos(x) from its Taylor series after reduction to [-pi, pi]; used only for the
// starting points of the Newton iterations (accurate to rounding anyway).
constexpr double cx_cos(double x) {
  constexpr double pi = 3.14159265358979323846, two_pi = 2 * pi;
  while (x > pi) x -= two_pi;
  while (x < -pi) x += two_pi;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// P_n(x) and P_{n-1}(x) by the three-term recurrence (k+1)P_{k+1} =
// (2k+1) x P_k - k P_{k-1}.
constexpr void legendre_pair(int n, double x, double &pn, double &pnm1) {
  double a = 1.0, b = x;  // P_0, P_1
  if (n == 0) {
    pn = 1.0;
    pnm1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  pn = b;
  pnm1 = a;
}

constexpr double legendre(int n, double x) {
  double pn = 0, pm = 0;
  legendre_pair(n, x, pn, pm);
  return pn;
}

// GLL points: the zeros of (1 - x^2) P_p'(x), which are the zeros of
// f = P_{p+1} - P_{p-1} (f' = (2p+1) P_p). Weights 2 / (p (p+1) P_p(x)^2).
constexpr void gll_rule(int n, double *x, double *w) {
  const int p = n - 1;
  constexpr double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    double t = -cx_cos(pi * j / p);
    if (j > 0 && j < p) {
      for (int it = 0; it < 100; ++it) {
        const double pp1 = legendre(p + 1, t), pm1 = legendre(p - 1, t);
        const double dt = (pp1 - pm1) / ((2 * p + 1) * legendre(p, t));
        t -= dt;
        if (cx_abs(dt) < 1e-16) break;
      }
    }
    x[j] = t;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 0; j < n / 2; ++j) {  // exact symmetry
    const double s = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -s;
    x[n - 1 - j] = s;
  }
  if (n % 2) x[n / 2] = 0.0;
  if (w)
    for (int j = 0; j < n; ++j) {
      const double lp = legendre(p, x[j]);
      w[j] = 2.0 / (p * (p + 1) * lp * lp);
    }
}

// GL points: zeros of P_n; P_n' = n (x P_n - P_{n-1}) / (x^2 - 1).
// Weights 2 / ((1 - x^2) P_n'(x)^2).
constexpr void gl_rule(int n, double *x, double *w) {
  constexpr double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    double t = -cx_cos(pi * (j + 0.75) / (n + 0.5));
    double pn = 0, pm = 0, dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre_pair(n, t, pn, pm);
      dp = n * (t * pn - pm) / (t * t - 1.0);
      const double dt = pn / dp;
      t -= dt;
      if (cx_abs(dt) < 1e-16) break;
    }
    legendre_pair(n, t, pn, pm);
    dp = n * (t * pn - pm) / (t * t - 1.0);
    x[j] = t;
    if (w) w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  for (int j = 0; j < n / 2; ++j) {
    const double s = 0.5 * (x[n - 1 - j] - x[j]);
    x[j] = -s;
    x[n - 1 - j] = s;
    if (w) {
      const double ws = 0.5 * (w[j] + w[n - 1 - j]);
      w[j] = w[n - 1 - j] = ws;
    }
  }
  if (n % 2) x[n / 2] = 0.0;
}

// Barycentric weights lambda_j = 1 / prod_{m != j} (x_j - x_m).
constexpr void bary_weights(int n, const double *nodes, double *lam) {
  for (int j = 0; j < n; ++j) {
    lam[j] = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) lam[j] /= (nodes[j] - nodes[m]);
  }
}

constexpr int node_hit(int n, const double *nodes, double x) {
  for (int m = 0; m < n; ++m)
    if (x == nodes[m]) return m;
  return -1;
}

// out[a][j] = l_j(pts[a]), l_j the Lagrange polynomials on the n nodes.
constexpr void lagrange_interp(int n, const double *nodes, int m, const double *pts,
                               double *out) {
  double lam[kMaxRule] = {};
  bary_weights(n, nodes, lam);
  for (int a = 0; a < m; ++a) {
    double *row = out + a * n;
    const int hit = node_hit(n, nodes, pts[a]);
    if (hit >= 0) {
      for (int j = 0; j < n; ++j) row[j] = (j == hit) ? 1.0 : 0.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += lam[j] / (pts[a] - nodes[j]);
    for (int j = 0; j < n; ++j) row[j] = lam[j] / (pts[a] - nodes[j]) / den;
  }
}

// out[a][j] = l_j'(pts[a]). At a node x_a: D_aj = (lam_j / lam_a) / (x_a - x_j),
// D_aa = -sum_{j != a} D_aj. Elsewhere: l_j'(x) = l_j(x) sum_{m != j} 1 / (x - x_m).
constexpr void lagrange_deriv(int n, const double *nodes, int m, const double *pts,
                              double *out) {
  double lam[kMaxRule] = {}, h[kMaxRule] = {};
  bary_weights(n, nodes, lam);
  for (int a = 0; a < m; ++a) {
    double *row = out + a * n;
    const int hit = node_hit(n, nodes, pts[a]);
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
    lagrange_interp(n, nodes, 1, &pts[a], h);
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (k != j) s += 1.0 / (pts[a] - nodes[k]);
      row[j] = h[j] * s;
    }
  }
}

// Even-odd table of the nq x np matrix M with M[nq-1-a][np-1-i] = sign M[a][i]
// (symmetric point sets): for a < (nq+1)/2, (M[a][i] + M[a][np-1-i]) / 2 and
// (M[a][i] - M[a][np-1-i]) / 2 for i < np/2, then M[a][np/2] for odd np. M is
// first symmetrised, so that entries zero by symmetry are exactly zero.
// Returns the number of entries written, ((nq+1)/2) * np.
constexpr int even_odd_table(const double *M, int nq, int np, int sign, double *out) {
  int o = 0;
  for (int a = 0; a < (nq + 1) / 2; ++a) {
    double ms[kMaxRule] = {};
    for (int i = 0; i < np; ++i) ms[i] = 0.5 * (M[a * np + i] + sign * M[(nq - 1 - a) * np + (np - 1 - i)]);
    for (int i = 0; i < np / 2; ++i) out[o++] = 0.5 * (ms[i] + ms[np - 1 - i]);
    for (int i = 0; i < np / 2; ++i) out[o++] = 0.5 * (ms[i] - ms[np - 1 - i]);
    if (np & 1) out[o++] = ms[np / 2];
  }
  return o;
}

// Compile-time even-odd tables of J^ and D^ from the p1 GLL nodes to q
// Gauss-Legendre points, in the element type T of a kernel.
template <int P1, int Q, typename T>
struct GLTables {
  static constexpr int SIZE = ((Q + 1) / 2) * P1;
  T J[SIZE], D[SIZE];
  constexpr GLTables() : J(), D() {
    double xi[P1] = {}, eta[Q] = {}, M[Q * P1] = {}, t[SIZE] = {};
    gll_rule(P1, xi, nullptr);
    gl_rule(Q, eta, nullptr);
    lagrange_interp(P1, xi, Q, eta, M);
    even_odd_table(M, Q, P1, 1, t);
    for (int i = 0; i < SIZE; ++i) J[i] = static_cast<T>(t[i]);
    lagrange_deriv(P1, xi, Q, eta, M);
    even_odd_table(M, Q, P1, -1, t);
    for (int i = 0; i < SIZE; ++i) D[i] = static_cast<T>(t[i]);
  }
};

// Compile-time D^ on the p1 GLL nodes (collocated quadrature: the points
// are the nodes), row-major D[a * p1 + m] = l_m'(xi_a), in the type T.
template <int P1, typename T>
struct GLLDeriv {
  T D[P1 * P1];
  constexpr GLLDeriv() : D() {
    double xi[P1] = {}, M[P1 * P1] = {};
    gll_rule(P1, xi, nullptr);
    lagrange_deriv(P1, xi, P1, xi, M);
    for (int i = 0; i < P1 * P1; ++i) D[i] = static_cast<T>(M[i]);
  }
};

}  // namespace bp
