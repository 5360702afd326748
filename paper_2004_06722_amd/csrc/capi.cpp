// C ABI of the bake-off library: operator setup, application, diagonal and
// the Jacobi-PCG drivers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <climits>
#include <vector>

#include <mutex>

#include "bp_internal.h"
#include "launch.h"

namespace bp {

static thread_local std::string g_last_error;

// Workspace of bp_pcg_solve_static: a file-scope device array (one copy on
// every device the library runs on, held until the process ends). Host code
// never uses its name as an address: bp_setup resolves the device address
// once per device (hipGetSymbolAddress, with that device current) and the
// solve passes that address to the kernels.
constexpr size_t kStaticWsBytes = size_t(BP_STATIC_WS_MB) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxDevices] = {};

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

namespace {

template <typename T>
int dmalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(BP_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                     " bytes failed: " + hipGetErrorString(e));
  }
  return BP_OK;
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void release(bp_op op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  dfree(op->idx);
  dfree(op->G);
  dfree(op->Gk);
  dfree(op->Bt);
  dfree(op->basis_d);
  dfree(op->G32);
  dfree(op->Gk32);
  dfree(op->Bt32);
  dfree(op->basis32);
  dfree(op->Bb);
  dfree(op->Bb32);
  dfree(op->dinv[0]);
  dfree(op->dinv[1]);
  dfree(op->dinv[2]);
  dfree(op->r);
  dfree(op->pv);
  dfree(op->w);
  dfree(op->part);
  dfree(op->tmp);
  dfree(op->sv);
  dfree(op->tr_off);
  dfree(op->tr_pos);
  dfree(op->perm);
  dfree(op->iperm);
  dfree(op->bi);
  dfree(op->xi);
  dfree(op->wl);
  dfree(op->wl32);
  dfree(op->r32);
  dfree(op->p32);
  dfree(op->w32);
  dfree(op->x32);
  dfree(op->dinv32);
  dfree(op->b32);
  dfree(op->sc);
  if (op->sc_host) (void)hipHostFree(op->sc_host);
  if (op->ev0) (void)hipEventDestroy(op->ev0);
  if (op->ev1) (void)hipEventDestroy(op->ev1);
  if (op->evm0) (void)hipEventDestroy(op->evm0);
  if (op->evm1) (void)hipEventDestroy(op->evm1);
  for (auto ev : op->apply_ev)
    if (ev) (void)hipEventDestroy(ev);
  delete op;
}

// Appends the even-odd table (rules1d.hpp) of the q x p1 matrix M.
void append_even_odd(const std::vector<double> &M, int q, int p1, int sign,
                     std::vector<double> &out) {
  const size_t o = out.size();
  out.resize(o + (size_t)((q + 1) / 2) * p1);
  even_odd_table(M.data(), q, p1, sign, out.data() + o);
}

// Upload basis J | D | Dq | 1D quadrature weights | even-odd tables of J and D
// (FP64 and optional FP32 copies).
int upload_basis(bp_op op, hipStream_t s) {
  const Basis &b = op->basis;
  std::vector<double> all;
  all.insert(all.end(), b.J.begin(), b.J.end());
  all.insert(all.end(), b.D.begin(), b.D.end());
  all.insert(all.end(), b.Dq.begin(), b.Dq.end());
  all.insert(all.end(), b.rho.begin(), b.rho.end());
  append_even_odd(b.J, b.q, b.p1, 1, all);
  append_even_odd(b.D, b.q, b.p1, -1, all);
  int rc = dmalloc(&op->basis_d, all.size());
  if (rc) return rc;
  BP_HIP(hipMemcpyAsync(op->basis_d, all.data(), all.size() * sizeof(double),
                        hipMemcpyHostToDevice, s));
  BP_HIP(hipStreamSynchronize(s));
  if (op->fp32) {
    std::vector<float> f(all.begin(), all.end());
    rc = dmalloc(&op->basis32, f.size());
    if (rc) return rc;
    BP_HIP(hipMemcpyAsync(op->basis32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice,
                          s));
    BP_HIP(hipStreamSynchronize(s));
  }
  return BP_OK;
}

int check_op(bp_op op) {
  if (!op) return set_error(BP_ERR_ARG, "null operator");
  int dev = -1;
  BP_HIP(hipGetDevice(&dev));
  if (dev != op->device)
    return set_error(BP_ERR_ARG, "operator lives on device " + std::to_string(op->device) +
                                     ", current device is " + std::to_string(dev));
  return BP_OK;
}

// Inverse diagonal for `which` (cached; masked when the operator has Dirichlet nodes).
// Slots: 0 mass, 1 stiffness, 2 Helmholtz; without a beta term H = A uses
// slot 1. Slots 0 and 1 are allocated by bp_setup, slot 2 by
// bp_set_helmholtz, so the solves allocate nothing.
int dinv_slot(const bp_op_s *op, int which) {
  if (which == BP_MASS) return 0;
  return which == BP_HELM && op->Bb ? 2 : 1;
}

bool valid_which(int which) { return which == BP_MASS || which == BP_STIFF || which == BP_HELM; }

int ensure_dinv(bp_op op, int which, hipStream_t s) {
  const int slot = dinv_slot(op, which);
  if (op->dinv_valid[slot]) return BP_OK;
  if (!op->dinv[slot]) return set_error(BP_ERR_ARG, "inverse diagonal not allocated");
  fill_f64(op->tmp, op->nglobal, 0.0, s);
  int rc = launch_diag(op, which, op->tmp, op->has_dirichlet, s);
  if (rc) return rc;
  invert_diag(op->tmp, op->dinv[slot], (slot == 1 && op->fp32) ? op->dinv32 : nullptr,
              op->nglobal, s);
  BP_HIP(hipGetLastError());
  op->dinv_valid[slot] = true;
  return BP_OK;
}

// Partial-sum table and device scalars of one CG run: the operator's own
// (op->part, op->sc) or those in the static workspace of bp_pcg_solve_static.
struct CgWork {
  double *part;
  DevScalars *sc;
};

CgWork own_work(bp_op op) { return CgWork{op->part, op->sc}; }

// Flags of the library's timing events: without the system-scope release of
// a default event, whose cache writeback and invalidation would slow the
// timed kernels and those after them.
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

// Device address of `scratch` on device dev (current), looked up once.
int resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(BP_ERR_ARG, "device index " + std::to_string(dev) + " beyond the static table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev]) return BP_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_error(BP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  return BP_OK;
}

// Layout of the static workspace for an operator: device scalars, the
// partial-sum table (as op->part), then z, p, w ([ncomp][nglobal] each),
// every block 256-byte aligned. Returns the bytes needed.
size_t scratch_layout(const bp_op_s *op, unsigned char *base, CgWork *ws, double **z, double **p,
                      double **w) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t nv = (size_t)op->nglobal * op->ncomp;
  size_t off = 0;
  const size_t o_sc = off;
  off += up(sizeof(DevScalars));
  const size_t o_part = off;
  off += up((size_t)op->part_len * sizeof(double));
  size_t o_vec[3];
  for (int k = 0; k < 3; ++k) {
    o_vec[k] = off;
    off += up(nv * sizeof(double));
  }
  if (base) {
    ws->sc = reinterpret_cast<DevScalars *>(base + o_sc);
    ws->part = reinterpret_cast<double *>(base + o_part);
    *z = reinterpret_cast<double *>(base + o_vec[0]);
    *p = reinterpret_cast<double *>(base + o_vec[1]);
    *w = reinterpret_cast<double *>(base + o_vec[2]);
  }
  return off;
}

int upload_scalars(bp_op op, DevScalars *sc, double rtol, bool fixed, hipStream_t s) {
  std::memset(op->sc_host, 0, sizeof(DevScalars));
  op->sc_host->tol2 = rtol * rtol;
  op->sc_host->fixed = fixed ? 1 : 0;
  BP_HIP(hipMemcpyAsync(sc, op->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, s));
  return BP_OK;
}

int download_scalars(bp_op op, const DevScalars *sc, hipStream_t s) {
  BP_HIP(hipMemcpyAsync(op->sc_host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  BP_HIP(hipStreamSynchronize(s));
  return BP_OK;
}
int upload_scalars(bp_op op, double rtol, bool fixed, hipStream_t s) {
  return upload_scalars(op, op->sc, rtol, fixed, s);
}
int download_scalars(bp_op op, hipStream_t s) { return download_scalars(op, op->sc, s); }

// Nodes [0, n) whose w the operator for `which` overwrites with plain stores
// on every application (the element-interior block of the internal order),
// so the vector updates need not clear them. The Gauss-Legendre mass
// assembles w by adding Q^T w_L (gather_local) and needs w cleared.
int64_t stored_rows(const bp_op_s *op, int which) {
  return which == BP_MASS && op->tr_off ? 0 : op->n_owned;
}

// Jacobi-PCG on precision T. x0_zero: x is zero on entry (skips A x0).
// The buffer `r` holds the preconditioned residual z = dinv r during the
// iteration (ten vector words per DOF and iteration; see k_cg_init).
// resume: continue from the device scalars and the z, p, w (w zero) that a
// previous call or cg_restart left, without the set-up (b, rtol unused).
// ws: partial sums and device scalars of the run (own_work(op) unless the
// caller brings its own).
template <typename T>
int pcg_run(bp_op op, const CgWork &ws, int which, bool f32, const T *b, T *x, const T *dinv,
            T *r, T *p, T *w, double rtol, int maxit, bool fixed, bool x0_zero, hipStream_t s,
            int *iters_out, float *ms_out, double *apply_ms_out = nullptr,
            int *apply_count_out = nullptr, bool resume = false) {
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  const bool masked = op->has_dirichlet;
  const int64_t nb_apply = apply_rows(op, which), nb_vec = vec_blocks(n);
  double *const part = ws.part;
  DevScalars *const sc = ws.sc;
  int rc = BP_OK;
  if (!resume) {
    rc = upload_scalars(op, sc, rtol, fixed, s);
    if (rc) return rc;
    if constexpr (sizeof(T) == 8)
      fill_f64((double *)w, nv, 0.0, s);
    else
      fill_f32((float *)w, nv, 0.0f, s);
    if (!x0_zero) {
      rc = launch_apply(op, which, f32, x, w, masked, nullptr, nullptr, s);
      if (rc) return rc;
    }
    cg_init<T>(nc, n, b, r, w, p, dinv, part, sc, s);
    BP_HIP(hipGetLastError());
  }
  BP_HIP(hipEventRecord(op->ev0, s));
  const int poll = 8;
  int it = 0, timed = 0;
  // a fixed number of iterations has no stopping test to honour: the kernels
  // then skip the done flag (nothing waits on loading it)
  const bool check = !fixed;
  const int *done = check ? &sc->done : nullptr;
  // mass on Gauss-Legendre points: the kernel stores w_L and the residual
  // update gathers w = Q^T w_L itself (w stays zero)
  const bool mass_wl = which == BP_MASS && op->tr_off != nullptr;
  const int64_t nl = op->nelem * op->p1 * op->p1 * op->p1;
  const T *wl = reinterpret_cast<const T *>(sizeof(T) == 4 ? (const void *)op->wl32
                                                           : (const void *)op->wl);
  // small meshes (FP64): alpha and beta computed inside the two vector
  // updates, three launches per iteration; the operator's partials stay at
  // the start of `part`, the residual update's follow them
  const bool fused =
      op->cg_fuse > 0 && sizeof(T) == 8 && !mass_wl && !resume && cg_fused_fits(n, nb_apply);
  // two launches per iteration where the operator forms p itself (PZIter);
  // its shorter vector table lets it run on larger meshes than the three
  const bool fused2 = op->cg_fuse == 2 && sizeof(T) == 8 && !mass_wl && !resume &&
                      apply_pz_supported(op, which) && cg_fused2_fits(n, nb_apply);
  // above those bounds the same operator with beta from the finisher and one
  // vector pass for p, x and z: four launches instead of five, while the
  // vectors stay below the streaming size (measured at p = 7: 0.3-2% faster
  // at E = 2^12..2^14, 1.2% slower at E = 2^18, where the z gathered by the
  // operator costs more than the z the vector pass no longer reads)
  const bool fused4 = sizeof(T) == 8 && !mass_wl && !resume && apply_pz_supported(op, which) &&
                      !fused2 &&
                      (op->cg_fuse == 3 || (op->cg_fuse == 2 && !cg_streams(n)));
  double *const part_r = part + nb_apply * nc;
  while (it < maxit) {
    const int chunk = fixed ? maxit - it : std::min(poll, maxit - it);
    for (int c = 0; c < chunk; ++c) {
      const bool tm = op->time_apply && timed < kMaxTimedApplies;
      if constexpr (sizeof(T) == 8) {
        if (fused2) {
          const int k = it + c;
          const PZIter pz{r, part_r, rxp_rows(n), sc, k & 1, check ? 1 : 0, k == 0 ? 1 : 0, 1};
          if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed], s));
          rc = launch_apply_pz(op, p, w, masked, part, done, pz, s);
          if (rc) return rc;
          if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed++ + 1], s));
          cg_update_rxp_fused(nc, n, x, p, r, w, dinv, part, nb_apply, part_r, sc, k & 1, s,
                              check, k == 0, stored_rows(op, which));
          continue;
        }
        if (fused4) {
          const int k = it + c;
          const PZIter pz{r, nullptr, 0, sc, k & 1, check ? 1 : 0, k == 0 ? 1 : 0, 0};
          if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed], s));
          rc = launch_apply_pz(op, p, w, masked, part, done, pz, s);
          if (rc) return rc;
          if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed++ + 1], s));
          cg_fin_alpha(nc, part, nb_apply, sc, s, check);
          cg_update_rxp(n, x, p, r, w, dinv, part, sc, s, check, k == 0, stored_rows(op, which));
          cg_fin_beta(nc, nb_vec, part, sc, s, check);
          continue;
        }
      }
      if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed], s));
      rc = mass_wl ? launch_mass_wl(op, f32, p, masked, part, done, s)
                   : launch_apply(op, which, f32, p, w, masked, part, done, s);
      if (rc) return rc;
      if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed++ + 1], s));
      if constexpr (sizeof(T) == 8) {
        if (fused) {
          const int parity = (it + c) & 1;
          cg_update_r_fused(nc, n, r, w, dinv, part, nb_apply, part_r, sc, parity, s, check,
                            stored_rows(op, which));
          cg_update_xp_fused(nc, n, x, p, r, part_r, sc, parity, s, check);
          continue;
        }
      }
      cg_fin_alpha(nc, part, nb_apply, sc, s, check);
      if (mass_wl)
        cg_update_r_gather<T>(nc, n, nl, r, wl, op->tr_off, op->tr_pos, dinv, part, sc, s,
                              check);
      else
        cg_update_r<T>(nc, n, r, w, dinv, part, sc, s, check, stored_rows(op, which));
      cg_fin_beta(nc, nb_vec, part, sc, s, check);
      cg_update_xp<T>(nc, n, x, p, r, sc, s, check);
    }
    BP_HIP(hipGetLastError());
    it += chunk;
    if (!fixed) {
      rc = download_scalars(op, sc, s);
      if (rc) return rc;
      if (op->sc_host->done) break;
    }
  }
  BP_HIP(hipEventRecord(op->ev1, s));
  if constexpr (sizeof(T) == 8) {
    if (fused2 && it > 0) cg_fin_rxp_fused(nc, n, part_r, sc, s);  // r.z, r.r of the last x
  }
  rc = download_scalars(op, sc, s);
  if (rc) return rc;
  float ms = 0.0f;
  BP_HIP(hipEventElapsedTime(&ms, op->ev0, op->ev1));
  if (ms_out) *ms_out = ms;
  if (iters_out) *iters_out = op->sc_host->iters;
  if (apply_ms_out) {
    double sum = 0.0;
    for (int k = 0; k < timed; ++k) {
      float t = 0.0f;
      BP_HIP(hipEventElapsedTime(&t, op->apply_ev[2 * k], op->apply_ev[2 * k + 1]));
      sum += t;
    }
    *apply_ms_out = sum;
    if (apply_count_out) *apply_count_out = timed;
  }
  if (op->sc_host->nonfinite) return set_error(BP_ERR_NONFINITE, "non-finite value in CG reductions");
  if (op->sc_host->breakdown) return set_error(BP_ERR_BREAKDOWN, "CG breakdown: p.Ap <= 0 along a non-zero direction");
  return BP_OK;
}

// Single-reduction Jacobi-PCG (FP64): per iteration the fused vector update,
// the operator on u = dinv r (its energy partials give (u, A u)) and one
// finisher. u lives in op->tmp, s = A p in op->sv. Same timing and stopping
// conventions as pcg_run; x0_zero skips the operator on x0.
int pcg_run_sr(bp_op op, int which, const double *b, double *x, const double *dinv,
               double rtol, int maxit, bool fixed, bool x0_zero, hipStream_t s,
               int *iters_out, float *ms_out, double *apply_ms_out, int *apply_count_out) {
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  const bool masked = op->has_dirichlet;
  const int64_t nba = apply_rows(op, which), nbv = vec_blocks(n);
  double *pv = op->part;                                     // vector partials + stage 1
  double *pa = op->part + (nbv + kStage2Rows) * 3 * nc;      // operator partials + stage 1
  double *r = op->r, *u = op->tmp, *w = op->w, *p = op->pv, *sv = op->sv;
  int rc = upload_scalars(op, rtol, fixed, s);
  if (rc) return rc;
  fill_f64(w, nv, 0.0, s);
  if (!x0_zero) {
    rc = launch_apply(op, which, false, x, w, masked, nullptr, nullptr, s);
    if (rc) return rc;
  }
  sr_init<double>(nc, n, b, r, w, u, p, sv, dinv, pv, s);
  rc = launch_apply(op, which, false, u, w, masked, pa, nullptr, s);
  if (rc) return rc;
  sr_fin(true, nc, pv, nbv, pa, nba, op->sc, s);
  BP_HIP(hipGetLastError());
  BP_HIP(hipEventRecord(op->ev0, s));
  const int poll = 8;
  int it = 0, timed = 0;
  // a fixed number of iterations has no stopping test to honour: the kernels
  // then skip the done flag (nothing waits on loading it)
  const bool check = !fixed;
  const int *done = check ? &op->sc->done : nullptr;
  while (it < maxit) {
    const int chunk = fixed ? maxit - it : std::min(poll, maxit - it);
    for (int c = 0; c < chunk; ++c) {
      sr_update<double>(nc, n, x, u, w, p, sv, dinv, pv, op->sc, s, check,
                        stored_rows(op, which));
      // the operator and finisher of the last fixed iteration would only
      // prepare a step that is not taken
      if (fixed && it + c == maxit - 1) break;
      const bool tm = op->time_apply && timed < kMaxTimedApplies;
      if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed], s));
      rc = launch_apply(op, which, false, u, w, masked, pa, done, s);
      if (rc) return rc;
      if (tm) BP_HIP(hipEventRecord(op->apply_ev[2 * timed++ + 1], s));
      sr_fin(false, nc, pv, nbv, pa, nba, op->sc, s);
    }
    BP_HIP(hipGetLastError());
    it += chunk;
    if (!fixed) {
      rc = download_scalars(op, s);
      if (rc) return rc;
      if (op->sc_host->done) break;
    }
  }
  BP_HIP(hipEventRecord(op->ev1, s));
  rc = download_scalars(op, s);
  if (rc) return rc;
  float ms = 0.0f;
  BP_HIP(hipEventElapsedTime(&ms, op->ev0, op->ev1));
  if (ms_out) *ms_out = ms;
  // fixed mode skips the last finisher, which would have counted the last step
  if (iters_out) *iters_out = fixed ? maxit : op->sc_host->iters;
  if (apply_ms_out) {
    double sum = 0.0;
    for (int k = 0; k < timed; ++k) {
      float t = 0.0f;
      BP_HIP(hipEventElapsedTime(&t, op->apply_ev[2 * k], op->apply_ev[2 * k + 1]));
      sum += t;
    }
    *apply_ms_out = sum;
    if (apply_count_out) *apply_count_out = timed;
  }
  if (op->sc_host->nonfinite) return set_error(BP_ERR_NONFINITE, "non-finite value in CG reductions");
  if (op->sc_host->breakdown) return set_error(BP_ERR_BREAKDOWN, "CG breakdown: non-positive curvature");
  return BP_OK;
}

// FP64 residual r = b - A x into op->r and its norms into the device scalars
// (rr, bb); returns max_c ||r_c|| / ||b_c|| through *worst.
int true_residual(bp_op op, const double *b, const double *x, double *worst, hipStream_t s) {
  const int nc = op->ncomp;
  const int64_t n = op->nglobal;
  fill_f64(op->w, n * nc, 0.0, s);
  int rc = launch_apply(op, BP_STIFF, false, x, op->w, op->has_dirichlet, nullptr, nullptr, s);
  if (rc) return rc;
  dc_residual(nc, n, b, op->r, op->w, op->dinv[1], op->part, op->sc, s);
  rc = download_scalars(op, s);
  if (rc) return rc;
  double m = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double bb = op->sc_host->bb[c] > 0 ? op->sc_host->bb[c] : 1.0;
    const double rel = std::sqrt(op->sc_host->rr[c] / bb);
    if (!std::isfinite(rel)) return set_error(BP_ERR_NONFINITE, "mixed solve: non-finite residual");
    m = std::max(m, rel);
  }
  *worst = m;
  return BP_OK;
}

// FP32 Jacobi-PCG with reliable updates: one FP32 iteration whose search
// direction is kept for the whole solve; whenever the recursive FP32
// residual has dropped by `delta` since the last replacement, x += x32 in
// FP64, the FP64 residual b - A x replaces the FP32 one, and the pending
// direction update uses it. Stops at the FP64 tolerance, after max_updates
// replacements, or after max_iters FP32 iterations.
int mixed_reliable(bp_op op, const double *b, double *x, double rtol, double delta,
                   int max_updates, int max_iters, int *iters_out, int *updates_out,
                   hipStream_t s) {
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  int updates = 0, iters = 0;
  double worst = 0.0;
  int rc = true_residual(op, b, x, &worst, s);
  if (rc == BP_OK && worst > rtol && max_updates > 0) {
    // the first FP32 right-hand side is the FP64 residual (b and r of the
    // FP32 iteration are distinct buffers)
    to_f32(op->r, op->b32, nv, s);
    fill_f32(op->x32, nv, 0.0f, s);
    bool resume = false;
    for (;;) {
      rc = pcg_run<float>(op, own_work(op), BP_STIFF, true, op->b32, op->x32, op->dinv32,
                          op->r32, op->p32, op->w32, delta, max_iters - iters, false, true, s,
                          &iters, nullptr, nullptr, nullptr, resume);
      if (rc) break;
      const bool reached = op->sc_host->done != 0;
      dc_accumulate(nv, x, op->x32, s);
      fill_f32(op->x32, nv, 0.0f, s);
      ++updates;
      rc = true_residual(op, b, x, &worst, s);
      if (rc || worst <= rtol || updates >= max_updates || iters >= max_iters || !reached) break;
      to_f32(op->r, op->r32, nv, s);
      cg_restart<float>(nc, n, op->r32, op->p32, op->dinv32, op->part, op->sc, s);
      BP_HIP(hipGetLastError());
      resume = true;
    }
  }
  *iters_out = iters;
  *updates_out = updates;
  return rc;
}

// The b and x a solve iterates on: the caller's (caller order), or the
// internal copies bi, xi with b and x0 permuted into them.
struct SolveVectors {
  const double *b;
  double *x;
};

SolveVectors solve_in(bp_op op, const double *b, double *x, hipStream_t s) {
  if (!op->perm) return SolveVectors{b, x};
  permute_in<double>(op->ncomp, op->nglobal, op->perm, b, op->bi, s);
  permute_in<double>(op->ncomp, op->nglobal, op->perm, x, op->xi, s);
  return SolveVectors{op->bi, op->xi};
}

// the solution back into the caller's x (nothing to do in the caller's
// order); the stream is synchronised, as the solves promise
int solve_out(bp_op op, double *x, hipStream_t s) {
  if (!op->perm) return BP_OK;
  permute_out<double>(op->ncomp, op->nglobal, op->iperm, op->xi, x, s);
  BP_HIP(hipGetLastError());
  BP_HIP(hipStreamSynchronize(s));
  return BP_OK;
}

void fill_stats(bp_op op, double rtol, bp_pcg_stats *st) {
  if (!st) return;
  st->ncomp = op->ncomp;
  bool conv = true;
  for (int c = 0; c < kMaxComp; ++c) st->rel_res[c] = 0.0;
  for (int c = 0; c < op->ncomp; ++c) {
    const double bb = op->sc_host->bb[c] > 0 ? op->sc_host->bb[c] : 1.0;
    st->rel_res[c] = std::sqrt(std::max(0.0, op->sc_host->rr[c]) / bb);
    conv = conv && st->rel_res[c] <= rtol;
  }
  st->converged = conv ? 1 : 0;
}

}  // namespace
}  // namespace bp

using namespace bp;

extern "C" {

int bp_version(void) { return 100; }

const char *bp_last_error(void) { return g_last_error.c_str(); }

int bp_rule(int n, int quad, double *x, double *w) {
  if (!x) return set_error(BP_ERR_ARG, "bp_rule: x is NULL");
  if (quad == BP_QUAD_GLL) {
    if (n < 2 || n > 64) return set_error(BP_ERR_ARG, "bp_rule: GLL needs 2 <= n <= 64");
    gll_rule(n, x, w);
  } else if (quad == BP_QUAD_GL) {
    if (n < 1 || n > 64) return set_error(BP_ERR_ARG, "bp_rule: GL needs 1 <= n <= 64");
    gl_rule(n, x, w);
  } else {
    return set_error(BP_ERR_ARG, "bp_rule: unknown quadrature");
  }
  return BP_OK;
}

int bp_setup(bp_op *out, int p, int q, int quad, int ncomp, int64_t nelem, int64_t nglobal,
             const int64_t *elem_dofs, const double *node_xyz, const uint8_t *dirichlet,
             unsigned flags, void *stream) {
  if (!out) return set_error(BP_ERR_ARG, "bp_setup: out is NULL");
  *out = nullptr;
  if (p < 1 || p > 15) return set_error(BP_ERR_ARG, "bp_setup: p must be in [1, 15]");
  if (q < 2 || q > 16) return set_error(BP_ERR_ARG, "bp_setup: q must be in [2, 16]");
  if (quad != BP_QUAD_GL && quad != BP_QUAD_GLL)
    return set_error(BP_ERR_ARG, "bp_setup: unknown quadrature");
  if (quad == BP_QUAD_GLL && q != p + 1)
    return set_error(BP_ERR_ARG, "bp_setup: GLL quadrature must be collocated (q = p + 1)");
  if (ncomp < 1 || ncomp > kMaxComp) return set_error(BP_ERR_ARG, "bp_setup: ncomp must be in [1, 8]");
  if (nelem < 1) return set_error(BP_ERR_ARG, "bp_setup: nelem must be >= 1");
  if (nglobal < 1 || nglobal > 2147483647LL)
    return set_error(BP_ERR_ARG, "bp_setup: nglobal must be in [1, 2^31 - 1]");
  if (!elem_dofs || !node_xyz) return set_error(BP_ERR_ARG, "bp_setup: NULL mesh array");
  if (flags & ~(BP_SETUP_FP32 | BP_SETUP_CALLER_ORDER))
    return set_error(BP_ERR_ARG, "bp_setup: unknown flag");
  if (!kernels_cover(p, q, quad))
    return set_error(BP_ERR_ARG, "bp_setup: no compiled kernels for p=" + std::to_string(p) +
                                     ", q=" + std::to_string(q) +
                                     " (compiled: GLL q=p+1 with p <= 15, GL q=p+2 with p <= 8)");
  hipStream_t s = (hipStream_t)stream;
  const int p1 = p + 1;
  const int64_t n3 = (int64_t)p1 * p1 * p1, nq = (int64_t)q * q * q;

  for (int64_t k = 0; k < nelem * n3; ++k) {
    const int64_t g = elem_dofs[k];
    if (g < 0 || g >= nglobal)
      return set_error(BP_ERR_MESH, "bp_setup: elem_dofs entry " + std::to_string(k) + " = " +
                                        std::to_string(g) + " out of range (element " +
                                        std::to_string(k / n3) + ")");
  }
  // internal node order: element-interior nodes first, in per-element blocks
  std::vector<int32_t> new_of_old, old_of_new;
  int64_t n_owned = 0;
  const bool renum = !(flags & BP_SETUP_CALLER_ORDER) &&
                     interior_first_order(p1, nelem, nglobal, elem_dofs, new_of_old, old_of_new,
                                          &n_owned);
  // gather map in internal ids with the Dirichlet sign encoding
  std::vector<int32_t> idx((size_t)(nelem * n3));
  for (int64_t k = 0; k < nelem * n3; ++k) {
    const int64_t g = elem_dofs[k];
    const int32_t v = renum ? new_of_old[(size_t)g] : (int32_t)g;
    const bool dir = dirichlet && dirichlet[g];
    idx[k] = dir ? -1 - v : v;
  }

  bp_op op = new bp_op_s();
  op->p = p;
  op->p1 = p1;
  op->q = q;
  op->quad = quad;
  op->ncomp = ncomp;
  op->nelem = nelem;
  op->nglobal = nglobal;
  op->fp32 = (flags & BP_SETUP_FP32) != 0;
  op->has_dirichlet = dirichlet != nullptr;
  op->basis = make_basis(p, q, quad);
  op->colloc = op->basis.colloc;
  if (hipGetDevice(&op->device) != hipSuccess) {
    release(op);
    return set_error(BP_ERR_HIP, "bp_setup: no HIP device");
  }

  int rc = resolve_scratch(op->device);
  if (rc) {
    release(op);
    return rc;
  }
#define TRY(x)          \
  do {                  \
    rc = (x);           \
    if (rc) {           \
      release(op);      \
      return rc;        \
    }                   \
  } while (0)
#define TRYHIP(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      release(op);                                                                  \
      return set_error(BP_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    }                                                                               \
  } while (0)

  const int64_t nv = nglobal * ncomp;
  TRY(dmalloc(&op->idx, idx.size()));
  TRYHIP(hipMemcpyAsync(op->idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  TRYHIP(hipStreamSynchronize(s));
  if (renum) {
    op->n_owned = n_owned;
    TRY(dmalloc(&op->perm, old_of_new.size()));
    TRY(dmalloc(&op->iperm, new_of_old.size()));
    TRYHIP(hipMemcpyAsync(op->perm, old_of_new.data(), old_of_new.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    TRYHIP(hipMemcpyAsync(op->iperm, new_of_old.data(), new_of_old.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    TRYHIP(hipStreamSynchronize(s));
    TRY(dmalloc(&op->bi, nv));
    TRY(dmalloc(&op->xi, nv));
  }
  // Gauss-Legendre operators: the transposed gather map (counting sort of the
  // element-local slots by global node, ascending within a node) for the
  // mass operator's fixed-order assembly, and its element-local output
  const int64_t nl = nelem * n3;
  if (!op->colloc && nl < (int64_t(1) << 31)) {
    auto node = [&](int64_t k) -> size_t { return (size_t)(idx[k] >= 0 ? idx[k] : -1 - idx[k]); };
    std::vector<int32_t> off((size_t)nglobal + 1, 0), pos((size_t)nl);
    for (int64_t k = 0; k < nl; ++k) ++off[node(k) + 1];
    for (int64_t g = 0; g < nglobal; ++g) off[(size_t)g + 1] += off[(size_t)g];
    {
      std::vector<int32_t> cur(off.begin(), off.end() - 1);
      for (int64_t k = 0; k < nl; ++k) pos[(size_t)cur[node(k)]++] = (int32_t)k;
    }
    TRY(dmalloc(&op->tr_off, off.size()));
    TRY(dmalloc(&op->tr_pos, pos.size()));
    TRY(dmalloc(&op->wl, nl * ncomp));
    TRYHIP(hipMemcpyAsync(op->tr_off, off.data(), off.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    TRYHIP(hipMemcpyAsync(op->tr_pos, pos.data(), pos.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    TRYHIP(hipStreamSynchronize(s));
  }
  TRY(upload_basis(op, s));

  // geometric factors of eq. (gij) and B~ of eq. (mass), computed on the device
  // from the node coordinates (held only for this call)
  const int64_t ng = nelem * 6 * nq, nb = nelem * nq;
  TRY(dmalloc(&op->G, ng));
  TRY(dmalloc(&op->Bt, nb));
  {
    double *X = nullptr;
    int *bad = nullptr;
    const int big = INT_MAX;
    int bad_host = INT_MAX;
    rc = dmalloc(&X, nelem * n3 * 3);
    if (!rc) rc = dmalloc(&bad, 1);
    if (!rc && hipMemcpyAsync(X, node_xyz, (size_t)(nelem * n3 * 3) * sizeof(double),
                              hipMemcpyHostToDevice, s) != hipSuccess)
      rc = set_error(BP_ERR_HIP, "bp_setup: coordinate upload failed");
    if (!rc && hipMemcpyAsync(bad, &big, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess)
      rc = set_error(BP_ERR_HIP, "bp_setup: flag upload failed");
    if (!rc) rc = launch_geometry(op, X, op->G, op->Bt, bad, s);
    if (!rc && (hipMemcpyAsync(&bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
      rc = set_error(BP_ERR_HIP, "bp_setup: geometric factors failed");
    dfree(X);
    dfree(bad);
    if (!rc && bad_host != INT_MAX)
      rc = set_error(BP_ERR_MESH, "bp_setup: non-positive Jacobian in element " +
                                      std::to_string(bad_host));
    TRY(rc);
  }
  TRY(dmalloc(&op->dinv[0], nglobal));
  TRY(dmalloc(&op->dinv[1], nglobal));
  TRY(dmalloc(&op->r, nv));
  TRY(dmalloc(&op->pv, nv));
  TRY(dmalloc(&op->w, nv));
  TRY(dmalloc(&op->tmp, std::max<int64_t>(nv, nglobal)));
  // partial sums of the largest grid, followed by the stage-1 rows
  op->part_len =
      (vec_blocks(nglobal) + kStage2Rows) * 3 * ncomp + (max_partial_rows(op) + kStage2Rows) * ncomp;
  TRY(dmalloc(&op->part, op->part_len));
  TRY(dmalloc(&op->sc, 1));
  TRYHIP(hipHostMalloc((void **)&op->sc_host, sizeof(DevScalars), hipHostMallocDefault));
  // timing events: no system-scope fence on record (no cache writeback and
  // invalidation around the timed work; the solves synchronise the stream
  // themselves before reading them)
  TRYHIP(hipEventCreateWithFlags(&op->ev0, kTimingEvent));
  TRYHIP(hipEventCreateWithFlags(&op->ev1, kTimingEvent));
  if (op->fp32) {
    TRY(dmalloc(&op->G32, ng));
    TRY(dmalloc(&op->Bt32, nb));
    to_f32(op->G, op->G32, ng, s);
    to_f32(op->Bt, op->Bt32, nb, s);
    TRYHIP(hipGetLastError());
    TRYHIP(hipStreamSynchronize(s));
    TRY(dmalloc(&op->r32, nv));
    TRY(dmalloc(&op->p32, nv));
    TRY(dmalloc(&op->w32, nv));
    TRY(dmalloc(&op->x32, nv));
    TRY(dmalloc(&op->b32, nv));
    TRY(dmalloc(&op->dinv32, nglobal));
    if (op->tr_off) TRY(dmalloc(&op->wl32, nl * ncomp));
    TRYHIP(hipEventCreateWithFlags(&op->evm0, kTimingEvent));
    TRYHIP(hipEventCreateWithFlags(&op->evm1, kTimingEvent));
  }
#undef TRY
#undef TRYHIP
  *out = op;
  return BP_OK;
}

int bp_info(bp_op op, int64_t *nelem, int64_t *nglobal, int *p, int *q, int *ncomp) {
  if (!op) return set_error(BP_ERR_ARG, "null operator");
  if (nelem) *nelem = op->nelem;
  if (nglobal) *nglobal = op->nglobal;
  if (p) *p = op->p;
  if (q) *q = op->q;
  if (ncomp) *ncomp = op->ncomp;
  return BP_OK;
}

int bp_set_coeff(bp_op op, const double *kappa_q, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int nq = op->q * op->q * op->q;
  if (!kappa_q) {
    op->kappa_set = false;
  } else {
    if (!op->Gk) {
      rc = dmalloc(&op->Gk, (size_t)op->nelem * 6 * nq);
      if (rc) return rc;
      if (op->fp32) {
        rc = dmalloc(&op->Gk32, (size_t)op->nelem * 6 * nq);
        if (rc) return rc;
      }
    }
    scale_geometry(op->G, kappa_q, op->Gk, op->Gk32, op->colloc ? 0 : op->q, op->nelem, nq, s);
    BP_HIP(hipGetLastError());
    op->kappa_set = true;
  }
  op->dinv_valid[1] = op->dinv_valid[2] = false;
  return BP_OK;
}

int bp_set_helmholtz(bp_op op, double beta, const double *beta_q, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!std::isfinite(beta)) return set_error(BP_ERR_ARG, "bp_set_helmholtz: beta must be finite");
  hipStream_t s = (hipStream_t)stream;
  const int64_t count = op->nelem * op->q * op->q * op->q;
  if (!beta_q && beta == 0.0) {
    // no beta term: free the scaled mass factors (BP_HELM = BP_STIFF)
    BP_HIP(hipStreamSynchronize(s));
    dfree(op->Bb);
    dfree(op->Bb32);
  } else {
    if (!op->Bb) {
      rc = dmalloc(&op->Bb, count);
      if (rc) return rc;
      if (op->fp32) {
        rc = dmalloc(&op->Bb32, count);
        if (rc) return rc;
      }
    }
    if (!op->dinv[2]) {
      rc = dmalloc(&op->dinv[2], op->nglobal);
      if (rc) return rc;
    }
    scale_mass(op->Bt, beta_q, beta, op->Bb, op->Bb32, op->q * op->q * op->q,
               op->colloc ? 0 : op->q, count, s);
    BP_HIP(hipGetLastError());
  }
  op->dinv_valid[2] = false;
  return BP_OK;
}

int bp_apply(bp_op op, int which, int prec, const void *u, void *w, unsigned flags,
             void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!valid_which(which)) return set_error(BP_ERR_ARG, "bp_apply: which");
  if (prec != BP_FP64 && prec != BP_FP32) return set_error(BP_ERR_ARG, "bp_apply: prec");
  if (prec == BP_FP32 && !op->fp32)
    return set_error(BP_ERR_ARG, "bp_apply: FP32 needs BP_SETUP_FP32");
  if (!u || !w) return set_error(BP_ERR_ARG, "bp_apply: NULL vector");
  if (u == w) return set_error(BP_ERR_ARG, "bp_apply: w must not alias u");
  if (flags & ~BP_MASKED) return set_error(BP_ERR_ARG, "bp_apply: unknown flag");
  hipStream_t s = (hipStream_t)stream;
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  const bool f32 = prec == BP_FP32, masked = (flags & BP_MASKED) != 0;
  if (!op->perm) {
    if (f32)
      fill_f32((float *)w, nv, 0.0f, s);
    else
      fill_f64((double *)w, nv, 0.0, s);
    return launch_apply(op, which, f32, u, w, masked, nullptr, nullptr, s);
  }
  // internal order: u in, the operator on the operator's work vectors, w out
  if (f32) {
    permute_in<float>(nc, n, op->perm, (const float *)u, op->r32, s);
    fill_f32(op->w32, nv, 0.0f, s);
    rc = launch_apply(op, which, true, op->r32, op->w32, masked, nullptr, nullptr, s);
    if (rc) return rc;
    permute_out<float>(nc, n, op->iperm, op->w32, (float *)w, s);
  } else {
    permute_in<double>(nc, n, op->perm, (const double *)u, op->r, s);
    fill_f64(op->w, nv, 0.0, s);
    rc = launch_apply(op, which, false, op->r, op->w, masked, nullptr, nullptr, s);
    if (rc) return rc;
    permute_out<double>(nc, n, op->iperm, op->w, (double *)w, s);
  }
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int bp_apply_local(bp_op op, int which, int prec, const void *uL, void *wL, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!valid_which(which)) return set_error(BP_ERR_ARG, "bp_apply_local: which");
  if (prec != BP_FP64 && prec != BP_FP32) return set_error(BP_ERR_ARG, "bp_apply_local: prec");
  if (prec == BP_FP32 && !op->fp32)
    return set_error(BP_ERR_ARG, "bp_apply_local: FP32 needs BP_SETUP_FP32");
  if (!uL || !wL) return set_error(BP_ERR_ARG, "bp_apply_local: NULL vector");
  if (uL == wL) return set_error(BP_ERR_ARG, "bp_apply_local: wL must not alias uL");
  return launch_apply_local(op, which, prec == BP_FP32, uL, wL, (hipStream_t)stream);
}

int bp_diag(bp_op op, int which, double *d, unsigned flags, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!valid_which(which)) return set_error(BP_ERR_ARG, "bp_diag: which");
  if (!d) return set_error(BP_ERR_ARG, "bp_diag: NULL output");
  if (flags & ~BP_MASKED) return set_error(BP_ERR_ARG, "bp_diag: unknown flag");
  hipStream_t s = (hipStream_t)stream;
  double *dd = op->perm ? op->tmp : d;  // internal order: through op->tmp
  fill_f64(dd, op->nglobal, 0.0, s);
  rc = launch_diag(op, which, dd, (flags & BP_MASKED) != 0, s);
  if (rc || !op->perm) return rc;
  permute_out<double>(1, op->nglobal, op->iperm, dd, d, s);
  BP_HIP(hipGetLastError());
  return BP_OK;
}

int bp_pcg_solve(bp_op op, int which, const double *b, double *x, double rtol, int maxit,
                 int fixed_iters, bp_pcg_stats *st, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!valid_which(which)) return set_error(BP_ERR_ARG, "bp_pcg_solve: which");
  if (!b || !x) return set_error(BP_ERR_ARG, "bp_pcg_solve: NULL vector");
  if (maxit < 0 || !(rtol >= 0.0)) return set_error(BP_ERR_ARG, "bp_pcg_solve: maxit/rtol");
  hipStream_t s = (hipStream_t)stream;
  rc = ensure_dinv(op, which, s);
  if (rc) return rc;
  int iters = 0;
  float ms = 0.0f;
  double apply_ms = 0.0;
  int apply_count = 0;
  const SolveVectors v = solve_in(op, b, x, s);
  if (op->cg_variant == BP_CG_SINGLE_REDUCTION) {
    rc = pcg_run_sr(op, which, v.b, v.x, op->dinv[dinv_slot(op, which)], rtol, maxit,
                    fixed_iters != 0, false, s, &iters, &ms, &apply_ms, &apply_count);
  } else {
    rc = pcg_run<double>(op, own_work(op), which, false, v.b, v.x,
                         op->dinv[dinv_slot(op, which)], op->r, op->pv, op->w, rtol, maxit,
                         fixed_iters != 0, false, s, &iters, &ms, &apply_ms, &apply_count);
  }
  const int rc_out = solve_out(op, x, s);
  if (rc == BP_OK) rc = rc_out;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = iters;
    st->ms = ms;
    st->apply_ms = apply_ms;
    st->apply_count = apply_count;
    fill_stats(op, rtol, st);
  }
  return rc;
}

int bp_pcg_solve_static(bp_op op, int which, const double *b, double *x, double rtol,
                        int maxit, int fixed_iters, bp_pcg_stats *st, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!valid_which(which)) return set_error(BP_ERR_ARG, "bp_pcg_solve_static: which");
  if (!b || !x) return set_error(BP_ERR_ARG, "bp_pcg_solve_static: NULL vector");
  if (maxit < 0 || !(rtol >= 0.0)) return set_error(BP_ERR_ARG, "bp_pcg_solve_static: maxit/rtol");
  const size_t need = scratch_layout(op, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (need > kStaticWsBytes)
    return set_error(BP_ERR_ARG, "bp_pcg_solve_static: the operator needs " +
                                     std::to_string(need) + " bytes of workspace, the static "
                                     "workspace holds " + std::to_string(kStaticWsBytes) +
                                     " (nglobal * ncomp up to about 2.7e6); use bp_pcg_solve");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    base = g_scratch_ptr[op->device];
  }
  if (!base) return set_error(BP_ERR_HIP, "bp_pcg_solve_static: workspace not resolved");
  CgWork ws{};
  double *z = nullptr, *p = nullptr, *w = nullptr;
  scratch_layout(op, static_cast<unsigned char *>(base), &ws, &z, &p, &w);
  hipStream_t s = (hipStream_t)stream;
  rc = ensure_dinv(op, which, s);
  if (rc) return rc;
  int iters = 0;
  float ms = 0.0f;
  double apply_ms = 0.0;
  int apply_count = 0;
  // standard recurrences whatever BP_OPT_CG_VARIANT says; every workspace
  // word is written (w cleared, scalars uploaded) before it is read
  const SolveVectors v = solve_in(op, b, x, s);
  rc = pcg_run<double>(op, ws, which, false, v.b, v.x, op->dinv[dinv_slot(op, which)], z, p, w,
                       rtol, maxit, fixed_iters != 0, false, s, &iters, &ms, &apply_ms,
                       &apply_count);
  const int rc_out = solve_out(op, x, s);
  if (rc == BP_OK) rc = rc_out;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = iters;
    st->ms = ms;
    st->apply_ms = apply_ms;
    st->apply_count = apply_count;
    fill_stats(op, rtol, st);
  }
  return rc;
}

int bp_pcg_solve_mixed(bp_op op, const double *b, double *x_out, double outer_rtol,
                       double inner_rtol, int max_outer, int max_inner, bp_pcg_stats *st,
                       void *stream) {
  double *x = x_out;
  int rc = check_op(op);
  if (rc) return rc;
  if (!op->fp32) return set_error(BP_ERR_ARG, "bp_pcg_solve_mixed: needs BP_SETUP_FP32");
  if (!b || !x) return set_error(BP_ERR_ARG, "bp_pcg_solve_mixed: NULL vector");
  if (max_outer < 0 || max_inner < 1 || !(outer_rtol >= 0) || !(inner_rtol >= 0))
    return set_error(BP_ERR_ARG, "bp_pcg_solve_mixed: bad limits");
  hipStream_t s = (hipStream_t)stream;
  rc = ensure_dinv(op, BP_STIFF, s);
  if (rc) return rc;
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  const bool masked = op->has_dirichlet;
  // the events were created by bp_setup: the solve allocates nothing
  hipEvent_t t0 = op->evm0, t1 = op->evm1;
  const SolveVectors v = solve_in(op, b, x, s);
  b = v.b;
  x = v.x;
  BP_HIP(hipEventRecord(t0, s));
  int outer = 0, inner_total = 0;
  if (op->mixed_mode == BP_MIXED_RELIABLE) {
    rc = mixed_reliable(op, b, x, outer_rtol, inner_rtol, max_outer, max_inner, &inner_total,
                        &outer, s);
  } else for (;;) {
    fill_f64(op->w, nv, 0.0, s);
    rc = launch_apply(op, BP_STIFF, false, x, op->w, masked, nullptr, nullptr, s);
    if (rc) break;
    dc_residual(nc, n, b, op->r, op->w, op->dinv[1], op->part, op->sc, s);
    rc = download_scalars(op, s);
    if (rc) break;
    double worst = 0.0;
    bool bad = false;
    for (int c = 0; c < nc; ++c) {
      const double bb = op->sc_host->bb[c] > 0 ? op->sc_host->bb[c] : 1.0;
      const double rel = std::sqrt(op->sc_host->rr[c] / bb);
      bad = bad || !std::isfinite(rel);
      worst = std::max(worst, rel);
    }
    if (bad) {
      rc = set_error(BP_ERR_NONFINITE, "bp_pcg_solve_mixed: non-finite residual");
      break;
    }
    if (worst <= outer_rtol || outer >= max_outer) break;
    to_f32(op->r, op->b32, nv, s);
    fill_f32(op->x32, nv, 0.0f, s);
    int it = 0;
    rc = pcg_run<float>(op, own_work(op), BP_STIFF, true, op->b32, op->x32, op->dinv32,
                        op->r32, op->p32, op->w32, inner_rtol, max_inner, false, true, s, &it,
                        nullptr);
    if (rc) break;
    inner_total += it;
    dc_accumulate(nv, x, op->x32, s);
    ++outer;
  }
  BP_HIP(hipEventRecord(t1, s));
  const int rc_out = solve_out(op, x_out, s);
  if (rc == BP_OK) rc = rc_out;
  BP_HIP(hipEventSynchronize(t1));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->iters = inner_total;
    st->outer = outer;
    st->ms = ms;
    fill_stats(op, outer_rtol, st);
  }
  return rc;
}

int bp_grad_kappa(bp_op op, const double *lam, const double *u, double *g, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!lam || !u || !g) return set_error(BP_ERR_ARG, "bp_grad_kappa: NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  if (op->perm) {  // internal order: lam and u through the operator's work vectors
    permute_in<double>(op->ncomp, op->nglobal, op->perm, lam, op->r, s);
    permute_in<double>(op->ncomp, op->nglobal, op->perm, u, op->pv, s);
    lam = op->r;
    u = op->pv;
  }
  return launch_grad_kappa(op, lam, u, g, s);
}

int bp_mass_misfit(bp_op op, const double *u, const double *u_target, double *grad,
                   double *loss, void *stream) {
  int rc = check_op(op);
  if (rc) return rc;
  if (!u || !u_target || !loss) return set_error(BP_ERR_ARG, "bp_mass_misfit: NULL pointer");
  if (grad && (grad == u || grad == u_target))
    return set_error(BP_ERR_ARG, "bp_mass_misfit: grad must not alias an input");
  hipStream_t s = (hipStream_t)stream;
  const int nc = op->ncomp;
  const int64_t n = op->nglobal, nv = n * nc;
  // d = u - u_target in the internal order, in the operator's work vector r
  if (op->perm) {
    permute_in<double>(nc, n, op->perm, u, op->r, s);
    permute_in<double>(nc, n, op->perm, u_target, op->pv, s);
    difference(op->r, op->pv, op->r, nv, s);
  } else {
    difference(u, u_target, op->r, nv, s);
  }
  // M d (unmasked) with the element energies d_L^T B_L d_L per work-group
  // and component, whose sum is d^T M d
  double *pa = op->part + (vec_blocks(n) + kStage2Rows) * 3 * nc;
  fill_f64(op->w, nv, 0.0, s);
  rc = launch_apply(op, BP_MASS, false, op->r, op->w, false, pa, nullptr, s);
  if (rc) return rc;
  operator_energies(nc, pa, apply_rows(op, BP_MASS), op->sc, s);
  if (grad) {
    if (op->perm)
      permute_out<double>(nc, n, op->iperm, op->w, grad, s);
    else
      BP_HIP(hipMemcpyAsync(grad, op->w, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  BP_HIP(hipGetLastError());
  BP_HIP(hipMemcpyAsync(op->sc_host, op->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  BP_HIP(hipStreamSynchronize(s));
  double e = 0.0;
  for (int c = 0; c < nc; ++c) e += op->sc_host->pap[c];
  *loss = 0.5 * e;
  return BP_OK;
}

int bp_set_option(bp_op op, int option, int value) {
  if (!op) return set_error(BP_ERR_ARG, "null operator");
  // the resources an option needs are created here, so that the solves
  // themselves allocate nothing
  if (option == BP_OPT_TIME_APPLY) {
    if (value && op->apply_ev.empty()) {
      op->apply_ev.resize(2 * kMaxTimedApplies, nullptr);
      for (auto &ev : op->apply_ev) BP_HIP(hipEventCreateWithFlags(&ev, kTimingEvent));
    }
    op->time_apply = value != 0;
    return BP_OK;
  }
  if (option == BP_OPT_CG_VARIANT) {
    if (value != BP_CG_STANDARD && value != BP_CG_SINGLE_REDUCTION)
      return set_error(BP_ERR_ARG, "bp_set_option: unknown CG variant");
    if (value == BP_CG_SINGLE_REDUCTION && !op->sv) {
      const int rc = dmalloc(&op->sv, op->nglobal * op->ncomp);
      if (rc) return rc;
    }
    op->cg_variant = value;
    return BP_OK;
  }
  if (option == BP_OPT_CG_FUSE) {
    if (value < 0 || value > 3)
      return set_error(BP_ERR_ARG, "bp_set_option: CG fuse 0, 1, 2 or 3");
    op->cg_fuse = value;
    return BP_OK;
  }
  if (option == BP_OPT_MIXED_MODE) {
    if (value != BP_MIXED_RESTART && value != BP_MIXED_RELIABLE)
      return set_error(BP_ERR_ARG, "bp_set_option: unknown mixed-precision mode");
    op->mixed_mode = value;
    return BP_OK;
  }
  return set_error(BP_ERR_ARG, "bp_set_option: unknown option " + std::to_string(option));
}

int bp_destroy(bp_op op) {
  if (!op) return BP_OK;
  release(op);
  return BP_OK;
}

}  // extern "C"
