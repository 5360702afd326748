// Launchers of the operator kernels: dispatch on (p1, q, quadrature,
// components, precision) to the compiled template instances.
#include "bp_internal.h"
#include "kernels.hpp"
#include "launch.h"

namespace bp {

// Elements per work-group of the operator kernel for (p1, q, which); the
// Gauss-Legendre values mirror GLPlane, the GLL ones Plane.
int64_t plane_epb(int p1, int q, int which) {
  if (q > p1) return gl_epb(p1, q, which == BP_MASS ? kGLMass : kGLStiff);
  return plane_elements(p1 * p1);
}

int64_t apply_rows(const bp_op_s *op, int which) {
  // BP_HELM runs in one launch of the stiffness layout (GL and GLL)
  const int64_t epb = plane_epb(op->p1, op->q, which);
  return (op->nelem + epb - 1) / epb;
}

int64_t apply_blocks(const bp_op_s *op) {
  const int64_t a = apply_rows(op, BP_MASS), b = apply_rows(op, BP_STIFF);
  return a > b ? a : b;
}

int64_t max_partial_rows(const bp_op_s *op) {
  return apply_rows(op, BP_MASS) + apply_rows(op, BP_STIFF);
}

namespace {

// 1 when the internal node order gives the element-interior nodes to their
// element alone (plain stores in the scatter)
int owned(const bp_op_s *op) { return op->n_owned > 0 ? 1 : 0; }

// Component stride of the vectors a launch reads and writes: global vectors
// [ncomp][nglobal], or element-local vectors [ncomp][nelem][p1^3] (LOCAL).
template <bool LOCAL>
int64_t vec_stride(const bp_op_s *op) {
  return LOCAL ? op->nelem * op->p1 * op->p1 * op->p1 : op->nglobal;
}

// Several components up to p = 7 (p = 6 with the Helmholtz term): one launch
// of k_stiff_colloc_nc (G and the map read once per element for all of
// them). Beyond, G beside a component's working set no longer fits 256
// registers (the multi-component kernel spills), so each component gets its
// own launch.
template <int P1, typename T, bool LOCAL, bool HELM>
int stiff_colloc(const bp_op_s *op, const T *G, const T *basis, const T *Bb, const T *u, T *w,
                 int masked, double *part, const int *done, hipStream_t s) {
  using PL = Plane<P1, P1>;
  const int64_t cs = vec_stride<LOCAL>(op);
  if constexpr (P1 <= (HELM ? 7 : 8)) {
    if (op->ncomp > 1) {
      hipLaunchKernelGGL((k_stiff_colloc_nc<P1, T, LOCAL, HELM>), dim3(apply_blocks(op)),
                         dim3(PL::THREADS), 0, s, op->nelem, op->idx, G, Bb, u, w, cs,
                         op->ncomp, masked, part, done, owned(op));
      return BP_OK;
    }
  }
  for (int c = 0; c < op->ncomp; ++c)
    hipLaunchKernelGGL((k_stiff_colloc<P1, T, LOCAL, HELM>), dim3(apply_blocks(op)),
                       dim3(PL::THREADS), 0, s, op->nelem, op->idx, G, Bb, u + c * cs,
                       w + c * cs, op->ncomp, c, masked, part, done, owned(op));
  return BP_OK;
}

template <int P1, typename T, bool LOCAL>
int mass_colloc(const bp_op_s *op, const T *Bt, const T *u, T *w, int masked, double *part,
                const int *done, hipStream_t s) {
  using PL = Plane<P1, P1>;
  hipLaunchKernelGGL((k_mass_colloc<P1, T, LOCAL>), dim3(apply_blocks(op)), dim3(PL::THREADS), 0,
                     s, op->nelem, op->idx, Bt, u, w, vec_stride<LOCAL>(op), op->ncomp, masked,
                     part, done, owned(op));
  return BP_OK;
}

// Several Gauss-Legendre components in one launch of k_op_gl_nc (G and the
// map read once per element for all of them) where G beside a component's
// working set fits 256 registers: the mass operator, p1 <= 7, and the
// stiffness operator when the point values fit the pencil's LDS rows (p1
// even). Otherwise (p1 = 9, the Helmholtz form at p1 = 8) the multi-component
// kernel spills and each component gets its own launch.
constexpr bool gl_multi(int p1, int q, int mode) {
  return mode == kGLMass || p1 <= 7 || (mode == kGLStiff && gl_row_stride(p1) >= q);
}

// WL: u global, w element-local [ncomp][nelem][p1^3] (see k_op_gl)
template <int P1, int Q, typename T, int MODE, bool LOCAL, bool WL = false>
int gauss(const bp_op_s *op, const T *Gm, const T *Bb, const T *basis, const T *u, T *w,
          int masked, double *part, const int *done, hipStream_t s) {
  using PL = GLPlane<P1, Q, MODE>;
  static_assert(PL::EPB * Q * Q <= 256, "plane layout");
  const int64_t grid = (op->nelem + PL::EPB - 1) / PL::EPB;
  if (grid != apply_rows(op, MODE == kGLMass ? BP_MASS : BP_STIFF))
    return set_error(BP_ERR_ARG, "plane layout");
  const int64_t cs = vec_stride<LOCAL>(op), ws = WL ? vec_stride<true>(op) : cs;
  if constexpr (gl_multi(P1, Q, MODE)) {
    if (op->ncomp > 1) {
      hipLaunchKernelGGL((k_op_gl_nc<P1, Q, T, MODE, LOCAL, WL>), dim3(grid), dim3(PL::THREADS),
                         0, s, op->nelem, op->idx, Gm, Bb, basis, u, w, cs, ws, op->ncomp,
                         masked, part, done, owned(op));
      return BP_OK;
    }
  }
  for (int c = 0; c < op->ncomp; ++c)
    hipLaunchKernelGGL((k_op_gl<P1, Q, T, MODE, LOCAL, WL>), dim3(grid), dim3(PL::THREADS), 0,
                       s, op->nelem, op->idx, Gm, Bb, basis, u + c * cs, w + c * ws, op->ncomp,
                       c, masked, part, done, owned(op));
  return BP_OK;
}

template <typename T>
int dispatch_mass_wl(const bp_op_s *op, const T *Bt, const T *basis, const T *u, T *wl,
                     int masked, double *part, const int *done, hipStream_t s) {
  if (op->colloc || op->q != op->p1 + 1)
    return set_error(BP_ERR_ARG, "element-local mass output needs Gauss-Legendre q = p + 2");
#define BP_CASE(P) \
  case P:          \
    return gauss<P, P + 1, T, kGLMass, false, true>(op, Bt, nullptr, basis, u, wl, masked, part, \
                                                    done, s);
  switch (op->p1) {
    BP_CASE(2) BP_CASE(3) BP_CASE(4) BP_CASE(5) BP_CASE(6) BP_CASE(7) BP_CASE(8) BP_CASE(9)
  }
#undef BP_CASE
  return set_error(BP_ERR_ARG, "no compiled kernel for this (p, q, quadrature)");
}

// which = BP_HELM: H = A + B_beta (eq. (hm2)), the beta term fused into the
// stiffness kernel (GLL: diagonal mass; GL: one more J^ chain at the points).
template <typename T, bool LOCAL>
int dispatch(const bp_op_s *op, int which, const T *G, const T *Bt, const T *Bb,
             const T *basis, const T *u, T *w, int masked, double *part, const int *done,
             hipStream_t s) {
  const bool stiff = which != BP_MASS;
  const bool helm = which == BP_HELM && Bb != nullptr;
  if (op->colloc) {
#define BP_CASE(P)                                                                        \
  case P:                                                                                 \
    if (!stiff) return mass_colloc<P, T, LOCAL>(op, Bt, u, w, masked, part, done, s);     \
    return helm ? stiff_colloc<P, T, LOCAL, true>(op, G, basis, Bb, u, w, masked, part,   \
                                                  done, s)                                \
                : stiff_colloc<P, T, LOCAL, false>(op, G, basis, Bb, u, w, masked, part,  \
                                                   done, s);
    switch (op->p1) {
      BP_CASE(2) BP_CASE(3) BP_CASE(4) BP_CASE(5) BP_CASE(6) BP_CASE(7) BP_CASE(8) BP_CASE(9)
      BP_CASE(10) BP_CASE(11) BP_CASE(12) BP_CASE(13) BP_CASE(14) BP_CASE(15) BP_CASE(16)
    }
#undef BP_CASE
  } else if (op->q == op->p1 + 1) {
#define BP_CASE(P)                                                                         \
  case P:                                                                                  \
    if (!stiff)                                                                            \
      return gauss<P, P + 1, T, kGLMass, LOCAL>(op, Bt, Bb, basis, u, w, masked, part,     \
                                                done, s);                                  \
    return helm ? gauss<P, P + 1, T, kGLHelm, LOCAL>(op, G, Bb, basis, u, w, masked, part, \
                                                     done, s)                              \
                : gauss<P, P + 1, T, kGLStiff, LOCAL>(op, G, Bb, basis, u, w, masked,      \
                                                      part, done, s);
    switch (op->p1) {
      BP_CASE(2) BP_CASE(3) BP_CASE(4) BP_CASE(5) BP_CASE(6) BP_CASE(7) BP_CASE(8) BP_CASE(9)
    }
#undef BP_CASE
  }
  return set_error(BP_ERR_ARG, "no compiled kernel for this (p, q, quadrature)");
}

// The operator of the two-launch iteration (PZIter): collocated stiffness,
// one component.
template <int P1>
int stiff_colloc_pz(const bp_op_s *op, const double *G, const double *p, double *w, int masked,
                    double *part, const int *done, const PZIter &pz, hipStream_t s) {
  using PL = Plane<P1, P1>;
  hipLaunchKernelGGL((k_stiff_colloc_pz<P1>), dim3(apply_blocks(op)), dim3(PL::THREADS), 0, s,
                     op->nelem, op->idx, G, p, w, op->ncomp, 0, masked, part, done, owned(op),
                     pz);
  return BP_OK;
}

template <int P1>
void grad_colloc(const bp_op_s *op, const double *lam, const double *u, double *g,
                 hipStream_t s) {
  using PL = Plane<P1, P1>;
  hipLaunchKernelGGL((k_grad_kappa_colloc<P1>), dim3(apply_blocks(op)), dim3(PL::THREADS), 0, s,
                     op->nelem, op->idx, op->G, lam, u, g, op->nglobal, op->ncomp);
}

}  // namespace

bool kernels_cover(int p, int q, int quad) {
  if (p < 1) return false;
  if (quad == BP_QUAD_GLL) return p <= 15 && q == p + 1;
  return p <= 8 && q == p + 2;
}

template <bool LOCAL>
static int launch_apply_impl(const bp_op_s *op, int which, bool f32, const void *u, void *w,
                             bool masked, double *part, const int *done, hipStream_t s) {
  int rc;
  // work-group size: 256 for the Gauss-Legendre planes, whole waves of p1^2 else
  const int64_t tpb = op->q > op->p1 ? 256 : ((op->p1 * op->p1 + 63) / 64) * 64;
  if (apply_blocks(op) * tpb >= (int64_t(1) << 32))
    return set_error(BP_ERR_ARG, "mesh too large for one operator launch (work-items >= 2^32)");
  if (f32) {
    const float *G = op->kappa_set ? op->Gk32 : op->G32;
    rc = dispatch<float, LOCAL>(op, which, G, op->Bt32, op->Bb32, op->basis32,
                                (const float *)u, (float *)w, masked, part, done, s);
  } else {
    const double *G = op->kappa_set ? op->Gk : op->G;
    rc = dispatch<double, LOCAL>(op, which, G, op->Bt, op->Bb, op->basis_d,
                                 (const double *)u, (double *)w, masked, part, done, s);
  }
  if (rc != BP_OK) return rc;
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int launch_mass_wl(const bp_op_s *op, bool f32, const void *u, bool masked, double *part,
                   const int *done, hipStream_t s) {
  if (!op->tr_off) return set_error(BP_ERR_ARG, "no transposed gather map");
  int rc;
  if (f32)
    rc = dispatch_mass_wl<float>(op, op->Bt32, op->basis32, (const float *)u, op->wl32, masked,
                                 part, done, s);
  else
    rc = dispatch_mass_wl<double>(op, op->Bt, op->basis_d, (const double *)u, op->wl, masked,
                                  part, done, s);
  if (rc != BP_OK) return rc;
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int launch_apply(const bp_op_s *op, int which, bool f32, const void *u, void *w, bool masked,
                 double *part, const int *done, hipStream_t s) {
  if (which == BP_MASS && op->tr_off) {
    // element kernel into w_L, then w += Q^T w_L by the transposed gather
    const int rc = launch_mass_wl(op, f32, u, masked, part, done, s);
    if (rc != BP_OK) return rc;
    const int64_t nl = op->nelem * op->p1 * op->p1 * op->p1;
    if (f32)
      gather_local<float>(op->ncomp, op->nglobal, nl, op->tr_off, op->tr_pos, op->wl32,
                          (float *)w, done, s);
    else
      gather_local<double>(op->ncomp, op->nglobal, nl, op->tr_off, op->tr_pos, op->wl,
                           (double *)w, done, s);
    BP_HIP(hipGetLastError());
    return BP_OK;
  }
  return launch_apply_impl<false>(op, which, f32, u, w, masked, part, done, s);
}

bool apply_pz_supported(const bp_op_s *op, int which) {
  return op->colloc && which == BP_STIFF && op->ncomp == 1 && op->p1 >= 2 && op->p1 <= 9;
}

int launch_apply_pz(const bp_op_s *op, const double *p, double *w, bool masked, double *part,
                    const int *done, const PZIter &pz, hipStream_t s) {
  if (!apply_pz_supported(op, BP_STIFF))
    return set_error(BP_ERR_ARG,
                     "two-launch iteration: collocated stiffness, one component, p <= 8");
  const double *G = op->kappa_set ? op->Gk : op->G;
  const int m = masked ? 1 : 0;
  int rc = BP_OK;
  switch (op->p1) {
#define BP_CASE(P) \
  case P:          \
    rc = stiff_colloc_pz<P>(op, G, p, w, m, part, done, pz, s); \
    break;
    BP_CASE(2) BP_CASE(3) BP_CASE(4) BP_CASE(5) BP_CASE(6) BP_CASE(7) BP_CASE(8) BP_CASE(9)
#undef BP_CASE
  }
  if (rc != BP_OK) return rc;
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int launch_apply_local(const bp_op_s *op, int which, bool f32, const void *uL, void *wL,
                       hipStream_t s) {
  if (op->nelem * op->p1 * op->p1 * op->p1 >= (int64_t(1) << 31))
    return set_error(BP_ERR_ARG, "bp_apply_local: nelem * (p+1)^3 must be below 2^31");
  return launch_apply_impl<true>(op, which, f32, uL, wL, false, nullptr, nullptr, s);
}

int launch_diag(const bp_op_s *op, int which, double *d, bool masked, hipStream_t s) {
  const int p1 = op->p1, q = op->q;
  const size_t lds = sizeof(double) *
                     ((size_t)q * q * q + (size_t)q * q * p1 + (size_t)q * p1 * p1 +
                      (size_t)p1 * p1 * p1 + 2 * (size_t)q * p1);
  const int64_t grid = op->nelem < 65536 ? op->nelem : 65536;
  if (lds > 65536)  // high orders: more than the default dynamic LDS per work-group
    BP_HIP(hipFuncSetAttribute((const void *)k_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  // BP_HELM: diag(A) + diag(B_beta), both added into d
  const bool helm = which == BP_HELM && op->Bb != nullptr;
  for (int part = 0; part < (helm ? 2 : 1); ++part) {
    const bool stiff = part == 0 && which != BP_MASS;
    const double *Gm = stiff ? (op->kappa_set ? op->Gk : op->G) : (part == 1 ? op->Bb : op->Bt);
    hipLaunchKernelGGL(k_diag, dim3(grid), dim3(256), lds, s, op->nelem, p1, q, stiff ? 1 : 0,
                       op->idx, Gm, op->basis_d, d, masked ? 1 : 0, op->colloc ? 0 : 1);
    BP_HIP(hipGetLastError());
  }
  return BP_OK;
}

int launch_geometry(const bp_op_s *op, const double *X, double *G, double *Bt, int *bad,
                    hipStream_t s) {
  const int p1 = op->p1, q = op->q;
  const size_t n3 = (size_t)p1 * p1 * p1, nq = (size_t)q * q * q;
  const size_t ra = 3 * std::max(n3, (size_t)p1 * q * q), rb = 3 * std::max((size_t)p1 * p1 * q, nq);
  const size_t lds = op->colloc ? 0 : (ra + rb) * sizeof(double);
  const int64_t grid = op->nelem < 65536 ? op->nelem : 65536;
  hipLaunchKernelGGL(k_geometry, dim3(grid), dim3(256), lds, s, op->nelem,
                     p1, q, op->colloc ? 1 : 0, X, op->basis_d, G, Bt, bad);
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int launch_grad_kappa(const bp_op_s *op, const double *lam, const double *u, double *g,
                      hipStream_t s) {
  if (!op->colloc) return set_error(BP_ERR_ARG, "bp_grad_kappa: only collocated GLL operators");
  switch (op->p1) {
    case 2: grad_colloc<2>(op, lam, u, g, s); break;
    case 3: grad_colloc<3>(op, lam, u, g, s); break;
    case 4: grad_colloc<4>(op, lam, u, g, s); break;
    case 5: grad_colloc<5>(op, lam, u, g, s); break;
    case 6: grad_colloc<6>(op, lam, u, g, s); break;
    case 7: grad_colloc<7>(op, lam, u, g, s); break;
    case 8: grad_colloc<8>(op, lam, u, g, s); break;
    case 9: grad_colloc<9>(op, lam, u, g, s); break;
    default: return set_error(BP_ERR_ARG, "bp_grad_kappa: compiled for p <= 8");
  }
  BP_HIP(hipGetLastError());
  return BP_OK;
}

}  // namespace bp
