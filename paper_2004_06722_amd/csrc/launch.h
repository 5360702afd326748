// Host-callable launchers of the device kernels.
#pragma once

#include "bp_internal.h"

namespace bp {

// operator kernels (ops.hip)
bool kernels_cover(int p, int q, int quad);
int64_t plane_epb(int p1, int q, int which);
// work-groups (= energy partial rows) of one operator launch for `which`;
// apply_blocks is the largest over mass and stiffness (partial buffer size)
int64_t apply_rows(const bp_op_s *op, int which);
int64_t apply_blocks(const bp_op_s *op);
// partial rows that any one operator application may write (buffer sizing)
int64_t max_partial_rows(const bp_op_s *op);
int launch_apply(const bp_op_s *op, int which, bool f32, const void *u, void *w, bool masked,
                 double *part, const int *done, hipStream_t s);
// mass element kernel with element-local output: op->wl (op->wl32 if f32)
// [ncomp][nelem][p1^3] = B_L (Q u), zero at masked nodes; needs op->tr_off
// (Gauss-Legendre operators). launch_apply(BP_MASS) runs it and then
// gather_local; the PCG iteration fuses the gather into the residual update.
int launch_mass_wl(const bp_op_s *op, bool f32, const void *u, bool masked, double *part,
                   const int *done, hipStream_t s);
// w_L = A_L u_L (or B_L u_L) per element, no gather or scatter; uL and wL are
// [ncomp][nelem][p1^3] in the precision of f32
int launch_apply_local(const bp_op_s *op, int which, bool f32, const void *uL, void *wL,
                       hipStream_t s);
int launch_diag(const bp_op_s *op, int which, double *d, bool masked, hipStream_t s);
// G [E][6][q^3] and Bt [E][q^3] from the node coordinates X [E][p1^3][3] (device);
// *bad (device, preset to INT_MAX) gets the smallest element with det J <= 0
int launch_geometry(const bp_op_s *op, const double *X, double *G, double *Bt, int *bad,
                    hipStream_t s);
int launch_grad_kappa(const bp_op_s *op, const double *lam, const double *u, double *g,
                      hipStream_t s);

// vector kernels (vec.hip); sizes are global nodes n and components nc
// CG vector kernels give each work-group kVecThreads nodes (vec_blocks; FP32
// iteration kernels two per thread, FP64 one); fills and
// conversions use a capped grid-stride grid (grid_blocks). Up to
// kDirectRows block partial sums go straight to the final fixed-order
// single-work-group sum (one launch less per reduction on small meshes);
// more are first folded to at most kStage2Rows rows, stored right after
// the partials.
constexpr int kVecThreads = 256;
constexpr int64_t kVecMaxBlocks = 2048;
constexpr int64_t kStage2Rows = 256;
constexpr int64_t kDirectRows = 16384;
int64_t vec_blocks(int64_t n);
int64_t grid_blocks(int64_t n);
void fill_f64(double *x, int64_t n, double v, hipStream_t s);
void fill_f32(float *x, int64_t n, float v, hipStream_t s);
// Gk = kappa G per point (and its FP32 copy if Gk32); kappa is in the caller's
// [E][c][b][a] point order, G stored reversed when qrev = q (else qrev = 0)
void scale_geometry(const double *G, const double *kappa, double *Gk, float *Gk32, int qrev,
                    int64_t nelem, int nq, hipStream_t s);
// Bb = beta_q * Bt (beta_q NULL: the constant beta), and its FP32 copy if Bb32;
// point orders as for scale_geometry
void scale_mass(const double *Bt, const double *beta_q, double beta, double *Bb, float *Bb32,
                int nq, int qrev, int64_t count, hipStream_t s);
void to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void invert_diag(const double *d, double *dinv, float *dinv32, int64_t n, hipStream_t s);

// CG steps; part holds per-block partial sums, sc the device scalars.
template <typename T>
void cg_init(int nc, int64_t n, const T *b, T *r, T *w, T *p, const T *dinv, double *part,
             DevScalars *sc, hipStream_t s);
// check = false (a fixed number of iterations): the kernels do not stop on
// the done flag, so their loads need not wait for it
void cg_fin_alpha(int nc, const double *part, int64_t nb, DevScalars *sc, hipStream_t s,
                  bool check = true);
// n_own: nodes [0, n_own) are written whole by the operator (internal
// order), so w is cleared from n_own on
template <typename T>
void cg_update_r(int nc, int64_t n, T *r, T *w, const T *dinv, double *part, DevScalars *sc,
                 hipStream_t s, bool check = true, int64_t n_own = 0);
void cg_fin_beta(int nc, int64_t nb, const double *part, DevScalars *sc, hipStream_t s,
                 bool check = true);
template <typename T>
void cg_update_xp(int nc, int64_t n, T *x, T *p, const T *z, DevScalars *sc, hipStream_t s,
                  bool check = true);

// The fused iteration of small meshes (FP64): at most kFusedRows partial
// rows in both tables. The residual update computes alpha itself from the
// operator's partials pa[nba][nc] and writes its own partials into pr
// ([vec_blocks(n)][2 nc]); the direction update computes beta and the
// convergence test from pr. Three launches per iteration instead of five;
// parity = iteration index & 1 (selects the r.z slot, DevScalars::rzs).
constexpr int64_t kFusedRows = 1024;
bool cg_fused_fits(int64_t n, int64_t nb_apply);
void cg_update_r_fused(int nc, int64_t n, double *z, double *w, const double *dinv,
                       const double *pa, int64_t nba, double *pr, DevScalars *sc, int parity,
                       hipStream_t s, bool check, int64_t n_own);
void cg_update_xp_fused(int nc, int64_t n, double *x, double *p, const double *z,
                        const double *pr, DevScalars *sc, int parity, hipStream_t s,
                        bool check);

// The two-launch iteration of small and mid-size meshes (FP64, collocated
// stiffness, one component, p1 <= 9; PZIter; cg_fused2_fits): the operator
// launch forms p_k = z_k + beta p_{k-1} while gathering and takes the
// stopping test on r_k; cg_update_rxp_fused then
// stores p_k, updates x and z = dinv r and writes the partials of the next
// r.z and r.r into pr. cg_fin_rxp_fused, once after the last iteration,
// reduces pr into the scalars the host reads (r.z, r.r, and the stopping
// test of the last iterate).
// k_cg_update_rxp_fused: one node per thread up to kFusedRows groups,
// kRxpNodes beyond; the bounds of the two partial tables (measured at p = 7:
// the two-launch form gains 13-14% at E = 2^10, 2^11 and breaks even at 2^12)
constexpr int kRxpNodes = 4;
constexpr int64_t kFused2VecRows = 2048, kFused2ApplyRows = 8192;
constexpr int64_t kFused2Product = int64_t(4) << 20;
int64_t rxp_rows(int64_t n);  // partial rows of the vector kernel
bool cg_fused2_fits(int64_t n, int64_t nb_apply);
bool apply_pz_supported(const bp_op_s *op, int which);
int launch_apply_pz(const bp_op_s *op, const double *p, double *w, bool masked, double *part,
                    const int *done, const PZIter &pz, hipStream_t s);
void cg_update_rxp_fused(int nc, int64_t n, double *x, double *p, double *z, double *w,
                         const double *dinv, const double *pa, int64_t nba, double *pr,
                         DevScalars *sc, int parity, hipStream_t s, bool check, bool first,
                         int64_t n_own);
void cg_fin_rxp_fused(int nc, int64_t n, const double *pr, DevScalars *sc, hipStream_t s);
// The four-launch form (one component, above those bounds): the operator
// launch (PZIter with fused = 0: beta from k_fin_beta), cg_fin_alpha,
// cg_update_rxp (p, x and z in one pass; partials for cg_fin_beta),
// cg_fin_beta.
bool cg_streams(int64_t n);  // FP64 vectors of n entries take the streaming kernels
void cg_update_rxp(int64_t n, double *x, double *p, double *z, double *w, const double *dinv,
                   double *part, DevScalars *sc, hipStream_t s, bool check, bool first,
                   int64_t n_own);

// transposed gather Q^T w_L: w[c][g] += sum of wl[c][pos[k]] for k in
// [off[g], off[g+1]) in ascending order (wl is [nc][nl]); skipped while
// *done (done may be NULL)
template <typename T>
void gather_local(int nc, int64_t n, int64_t nl, const int32_t *off, const int32_t *pos,
                  const T *wl, T *w, const int *done, hipStream_t s);
// cg_update_r with w = Q^T w_L gathered per node (no w vector is read,
// written or cleared)
template <typename T>
void cg_update_r_gather(int nc, int64_t n, int64_t nl, T *r, const T *wl, const int32_t *off,
                        const int32_t *pos, const T *dinv, double *part, DevScalars *sc,
                        hipStream_t s, bool check = true);

// single-reduction PCG: init (r, u = dinv r, p = s = w = 0; partials r.u, r.r,
// b.b), the fused vector update (partials r.u, r.r), and the finisher that
// combines them with the operator's (u, A u) partials (alpha, beta, flags)
template <typename T>
void sr_init(int nc, int64_t n, const T *b, T *r, T *w, T *u, T *p, T *sv, const T *dinv,
             double *part, hipStream_t s);
template <typename T>
void sr_update(int nc, int64_t n, T *x, T *u, T *w, T *p, T *sv, const T *dinv, double *part,
               DevScalars *sc, hipStream_t s, bool check = true, int64_t n_own = 0);

// vectors [nc][n] between the caller's node order and the internal one,
// both as gathers: in, dst[c][v] = src[c][perm[v]] (perm[v] = the caller's
// id of internal node v); out, dst[c][g] = src[c][iperm[g]] (iperm[g] = the
// internal id of the caller's node g)
template <typename T>
void permute_in(int nc, int64_t n, const int32_t *perm, const T *src, T *dst, hipStream_t s);
template <typename T>
void permute_out(int nc, int64_t n, const int32_t *iperm, const T *src, T *dst, hipStream_t s);
void sr_fin(bool first, int nc, double *pv, int64_t nbv, double *pa, int64_t nba,
            DevScalars *sc, hipStream_t s);

// residual replacement after an iteration that stopped before its direction
// update: r holds the new residual and becomes z = dinv r (the form the
// iteration keeps); r.z and r.r of it, then the pending p = z + beta p with
// beta = (r.z)_new / (r.z)_old (the search direction is kept); r.r becomes
// the reference norm; clears done/halted
template <typename T>
void cg_restart(int nc, int64_t n, T *r, T *p, const T *dinv, double *part,
                DevScalars *sc, hipStream_t s);

// sc->pap[c] = sum over the rows of column c of the operator's energy table
// part[rows][nc] (fixed order); part + rows nc holds the stage-1 rows
void operator_energies(int nc, double *part, int64_t rows, DevScalars *sc, hipStream_t s);
// d = a - b over count entries (d may be a)
void difference(const double *a, const double *b, double *d, int64_t count, hipStream_t s);

// defect correction helpers (FP64 outer loop)
void dc_residual(int nc, int64_t n, const double *b, double *r, double *w, const double *dinv,
                 double *part, DevScalars *sc, hipStream_t s);
void dc_accumulate(int64_t n, double *x, const float *d, hipStream_t s);

}  // namespace bp
