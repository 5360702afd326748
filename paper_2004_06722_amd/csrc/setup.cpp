// Host-side setup of the bake-off operators: the 1D basis of an operator
// (rules and Lagrange matrices from rules1d.hpp) and the internal node order
// (the geometric factors of section 3 are computed on the device at set-up).
#include <algorithm>
#include <cmath>

#include "bp_internal.h"

namespace bp {

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
