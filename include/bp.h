/*
 * bp.h -- C ABI of the MI355X bake-off library (BP1-BP6 hot path).
 *
 * The library applies the assembled high-order hexahedral mass matrix B and
 * stiffness matrix A of the bake-off problems matrix-free (sum factorisation,
 * section 5, eq. (bk5x) and (mass)), with the element gather u_L = Q u and the
 * scatter-add w = Q^T w_L of section 4, and runs the diagonally (Jacobi)
 * preconditioned CG iteration of section 3 around them, on one HIP device.
 *
 * Conventions shared by every entry point
 *   - p is the polynomial order, p1 = p + 1 nodes per direction (GLL points),
 *     q quadrature points per direction (section 3, Table "bps": GL q = p+2
 *     for BP1-BP4, GLL q = p+1 for BP5-BP6).
 *   - Element-local node (i, j, k) has local id l = i + p1*(j + p1*k), i the
 *     fastest index (eq. (xijk)/(uijk)); quadrature point (a, b, c) likewise.
 *   - Global vectors are device arrays [ncomp][nglobal] (component-major:
 *     component c of node g at c * nglobal + g), FP64 unless stated.
 *   - Every call that takes a `stream` enqueues its device work on that HIP
 *     stream (hipStream_t passed as void*, NULL = the null stream) and returns
 *     without waiting, unless stated otherwise.
 *   - Return value: BP_OK (0) or a negative bp_status. bp_last_error()
 *     returns a message for the calling thread's last failure.
 *   - Device pointers are owned by the caller; the library never frees them.
 *     Everything the library allocates belongs to the bp_op and is freed by
 *     bp_destroy.
 *   - A bp_op's work vectors, partial-sum tables and device scalars are shared
 *     by its calls: calls on one bp_op must not overlap (one stream, or the
 *     caller orders them); different bp_op handles are independent.
 */
#ifndef BP_H
#define BP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bp_op_s *bp_op; /* opaque, owned by the library */

enum bp_status {
  BP_OK = 0,
  BP_ERR_ARG = -1,        /* invalid argument or unsupported combination   */
  BP_ERR_MESH = -2,       /* bad mesh: Jacobian <= 0, index out of range    */
  BP_ERR_HIP = -3,        /* a HIP runtime call failed                       */
  BP_ERR_NONFINITE = -4,  /* NaN or Inf in an input or a reduction           */
  BP_ERR_BREAKDOWN = -5,  /* CG breakdown: r.z != 0 and (r.z)/(p.Ap) not > 0  */
  BP_ERR_OOM = -6         /* device or host allocation failed                */
};

enum bp_quad { BP_QUAD_GL = 0, BP_QUAD_GLL = 1 };
enum bp_which { BP_MASS = 1, BP_STIFF = 3, BP_HELM = 4 };
enum bp_prec { BP_FP64 = 0, BP_FP32 = 1 };

/* flags of bp_apply / bp_diag */
#define BP_MASKED 1u          /* w = mask * A (mask * u), mask = 0 on Dirichlet nodes */
/* flags of bp_setup */
#define BP_SETUP_FP32 1u      /* also keep single-precision geometric factors and
                                 workspace for prec = BP_FP32 and the mixed solve   */
#define BP_SETUP_CALLER_ORDER 2u /* keep the caller's node numbering inside the
                                 library (see bp_setup)                             */

/* Version of this ABI (major*100 + minor). */
int bp_version(void);

/*
 * bp_rule -- host-only: the library's 1D rule with n points.
 * Section 3 / Table "bps": GLL (quad = BP_QUAD_GLL, n >= 2) or GL
 * (BP_QUAD_GL, n >= 1) points on [-1, 1], ascending, and their weights.
 * x, w: host arrays of n doubles (w may be NULL). No device work.
 * Callers use it to place mesh nodes at the library's own GLL points.
 */
int bp_rule(int n, int quad, double *x, double *w);

/*
 * bp_setup -- build an operator on the current HIP device.
 * Section 4 (isoparametric elements, eq. (xijk); global-to-local map Q,
 * eq. (dssum)) and section 5 (geometric factors G, eq. (gij); B~, eq. (mass)),
 * all precomputed as section 3 requires.
 *   p in [1, 15]; q in [2, 16]; quad = BP_QUAD_GL or BP_QUAD_GLL (GLL needs
 *   q = p + 1, collocated); ncomp in [1, 8] components per node.
 *   The compiled kernels cover (quad, q) = (GLL, p+1) for p <= 15 and
 *   (GL, p+2) for p <= 8; other combinations return BP_ERR_ARG.
 *   nelem >= 1; nglobal in [1, 2^31 - 1].
 *   elem_dofs: host int64 [nelem][p1^3], global node id of each local node,
 *     0 <= id < nglobal. The map is treated as arbitrary (no tensor layout).
 *   node_xyz: host double [nelem][p1^3][3], coordinates of the element nodes
 *     (placed at the GLL points of the reference element).
 *   dirichlet: host uint8 [nglobal] (nonzero = homogeneous Dirichlet node) or
 *     NULL (no Dirichlet nodes, e.g. BP1/BP2 with Neumann conditions).
 *   flags: 0 or a combination of BP_SETUP_FP32 and BP_SETUP_CALLER_ORDER.
 *   stream: stream for the uploads; bp_setup synchronises it before return.
 * Internal node order: in a conforming mesh every element-interior node
 * (local 0 < i, j, k < p) belongs to one element only. When the map shows
 * this (every interior slot names a node that no other slot names; p >= 2)
 * and BP_SETUP_CALLER_ORDER is not set, the library numbers its nodes
 * internally: the interior nodes element by element in contiguous blocks,
 * then the shared nodes in the order the elements first reach them. The
 * operator kernels then read and write the interior nodes as contiguous
 * blocks, with plain stores in place of atomic additions. Every entry point
 * still takes and returns vectors in the caller's numbering: the vectors
 * are permuted on entry and exit (one gather pass each, and a solve keeps
 * its iteration in the internal order), and the results are the same up to
 * the rounding order of the assembly sums.
 * With GL quadrature (and nelem p1^3 < 2^31) the operator also holds the
 * transposed gather map (int32, nglobal + 1 offsets and nelem p1^3 slots) and
 * an element-local output buffer of ncomp nelem p1^3 words (per precision):
 * the mass operator stores B_L u_L per element and assembles Q^T of it by a
 * fixed-order gather, so its results do not depend on scheduling.
 * Errors: BP_ERR_ARG (ranges), BP_ERR_MESH (Jacobian <= 0 at a quadrature
 * point -- the message names the element -- or an id out of range),
 * BP_ERR_OOM, BP_ERR_HIP. On error *out is set to NULL.
 */
int bp_setup(bp_op *out, int p, int q, int quad, int ncomp, int64_t nelem,
             int64_t nglobal, const int64_t *elem_dofs, const double *node_xyz,
             const uint8_t *dirichlet, unsigned flags, void *stream);

/* Sizes of an operator: nelem, nglobal, p, q, ncomp (any pointer may be NULL). */
int bp_info(bp_op op, int64_t *nelem, int64_t *nglobal, int *p, int *q, int *ncomp);

/*
 * bp_set_coeff -- variable coefficient of the stiffness operator.
 * Section 4, eq. (hm1)/(ip1): a(v,u) = int mu grad v . grad u with mu given at
 * the quadrature points: the element operator of eq. (bk5x) uses mu_q G_q.
 *   kappa_q: device double [nelem][q^3], read during the call (copied into a
 *   library buffer as mu_q G_q); NULL restores mu = 1.
 * Affects BP_STIFF in bp_apply, bp_diag and the solves; not bp_grad_kappa.
 */
int bp_set_coeff(bp_op op, const double *kappa_q, void *stream);

/*
 * bp_set_helmholtz -- beta of the Helmholtz operator H = A + B_beta used by
 * which = BP_HELM (bp_apply, bp_apply_local, bp_diag, bp_pcg_solve).
 * Section 4, eq. (hm1)-(hm2) with (ip1)-(ip2): -div(mu grad u) + beta u, where
 * (v, u)_beta integrates beta v u; B_beta is the mass matrix of eq. (mass)
 * with beta_q B~_q at the quadrature points. mu is the kappa of
 * bp_set_coeff (1 by default).
 *   beta_q: device double [nelem][q^3] (beta at the quadrature points, read
 *     during the call), or NULL for the constant `beta`.
 *   beta = 0 with beta_q = NULL removes the term (BP_HELM then equals
 *   BP_STIFF). The term is fused into the stiffness kernel: with GLL
 *   quadrature B_beta is diagonal; with GL points the kernel interpolates u
 *   to the points once more.
 * Errors: BP_ERR_ARG (non-finite beta), BP_ERR_OOM, BP_ERR_HIP.
 */
int bp_set_helmholtz(bp_op op, double beta, const double *beta_q, void *stream);

/*
 * bp_apply -- w = Q^T A_L Q u (BP_STIFF), Q^T B_L Q u (BP_MASS) or
 * Q^T (A_L + B_beta,L) Q u (BP_HELM, see bp_set_helmholtz).
 * Section 4 (w = Q^T A_L Q u), section 5 eq. (bk5x) / eq. (mass); with
 * BP_MASKED, w = mask * A (mask * u) as the Dirichlet restriction of
 * Appendix A1 (Nek5000 ax).
 *   prec = BP_FP64: u, w are double [ncomp][nglobal].
 *   prec = BP_FP32: u, w are float; requires BP_SETUP_FP32.
 *   w is overwritten (it must not alias u).
 */
int bp_apply(bp_op op, int which, int prec, const void *u, void *w,
             unsigned flags, void *stream);

/*
 * bp_apply_local -- the bake-off kernels on their own: w_L = A_L u_L
 * (BP_STIFF: BK3/BK5, and BK4/BK6 per component) or w_L = B_L u_L (BP_MASS:
 * BK1/BK2), with A_L = block-diag(A^e) the unassembled operator of section 4
 * and eq. (bk5x) / eq. (mass), evaluated element by element without the
 * gather Q, the scatter Q^T or the Dirichlet mask (section 3, the BK
 * definition; section 8, the single-GPU BK5 study).
 *   uL, wL: device arrays [ncomp][nelem][(p+1)^3], local node id
 *     i + p1 (j + p1 k); double for prec = BP_FP64, float for BP_FP32 (which
 *     requires BP_SETUP_FP32). Every entry of wL is written; wL must not
 *     alias uL. The κ of bp_set_coeff applies as in bp_apply.
 * Errors: BP_ERR_ARG (which, prec, NULL or aliased vectors, or
 * nelem (p+1)^3 >= 2^31), BP_ERR_HIP.
 */
int bp_apply_local(bp_op op, int which, int prec, const void *uL, void *wL,
                   void *stream);

/*
 * bp_diag -- d = diag(Q^T A_L Q) (or of B), the Jacobi preconditioner's
 * diagonal (section 3: diagonally preconditioned CG). d: device double
 * [nglobal] (the same for every component). With BP_MASKED, d = 0 on
 * Dirichlet nodes.
 */
int bp_diag(bp_op op, int which, double *d, unsigned flags, void *stream);

/* Statistics of a solve (host struct filled on return). */
typedef struct {
  int iters;          /* CG iterations done (inner iterations for the mixed solve) */
  int outer;          /* defect-correction steps (mixed solve), else 0               */
  int converged;      /* 1 if every component reached rtol                          */
  int ncomp;
  double rel_res[8];  /* final ||r||_2 / ||b||_2 per component                       */
  double ms;          /* device time of the iteration loop in milliseconds           */
  double apply_ms;    /* with BP_OPT_TIME_APPLY: summed device time of the operator
                         launches inside the loop (HIP events on the stream), else 0 */
  int apply_count;    /* number of operator launches timed                          */
  int pad_;
} bp_pcg_stats;

/*
 * bp_pcg_solve -- Jacobi-preconditioned CG for which x = b (section 3).
 * BP_STIFF solves the masked stiffness system (BP3-BP6; Dirichlet nodes stay
 * 0); BP_MASS solves the unmasked mass system (BP1, BP2) -- if the operator
 * was built with Dirichlet nodes the mass system is masked too.
 *   b: device double [ncomp][nglobal]; x: device double, in: x0, out: solution.
 *   fixed_iters != 0: exactly maxit iterations, no convergence test (the
 *     timing mode of section 2); otherwise stop at the first iteration with
 *     max_c ||r_c|| / ||b_c|| <= rtol, or at maxit (converged = 0, not an error).
 *   st: may be NULL. Components use independent CG scalars. Entries of b on
 *   Dirichlet nodes are ignored (read as 0).
 * The call synchronises the stream before it returns.
 * Errors: BP_ERR_NONFINITE if b holds NaN/Inf; BP_ERR_BREAKDOWN when a step
 * length alpha = (r.z) / (p.Ap) is not positive while r.z != 0 (an operator
 * or preconditioner that is not definite on the Krylov space). With a
 * stopping test the solve ends at that iteration and x keeps the last
 * iterate (stats give the iterations completed); in fixed-iteration mode all
 * maxit iterations run and the error is returned at the end.
 */
int bp_pcg_solve(bp_op op, int which, const double *b, double *x, double rtol,
                 int maxit, int fixed_iters, bp_pcg_stats *st, void *stream);

/*
 * bp_pcg_solve_static -- bp_pcg_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, results and errors
 * as bp_pcg_solve with the standard recurrences (BP_OPT_CG_VARIANT is not
 * consulted), but the iteration's workspace -- the vectors z = D^-1 r, p and
 * w = A p, the partial-sum tables and the device scalars -- lives in one
 * static device array of BP_STATIC_WS_MB MiB per device (resolved by
 * bp_setup), not in the operator's buffers. Nothing is allocated or freed.
 * Limits and sharing:
 *   - the operator must fit: 3 nglobal ncomp doubles plus the partial sums
 *     (nglobal ncomp up to about 2.7e6); larger operators return BP_ERR_ARG
 *     with the bytes needed (use bp_pcg_solve);
 *   - every call on a device shares that device's array and leaves its last
 *     contents there; each call writes what it reads (w is cleared, the
 *     scalars uploaded) before using it, but calls that overlap on one
 *     device (different streams or threads) race and must be serialised by
 *     the caller;
 *   - the Jacobi diagonal and, for Gauss-Legendre mass operators, the
 *     element-local output buffer are the operator's own (set up by
 *     bp_setup), as in bp_pcg_solve.
 */
#define BP_STATIC_WS_MB 64
int bp_pcg_solve_static(bp_op op, int which, const double *b, double *x, double rtol,
                        int maxit, int fixed_iters, bp_pcg_stats *st, void *stream);

/*
 * bp_pcg_solve_mixed -- FP64 defect correction around an FP32 Jacobi-PCG
 * (stiffness only; needs BP_SETUP_FP32). Two modes (bp_set_option
 * BP_OPT_MIXED_MODE):
 *   BP_MIXED_RESTART (default): outer step r = b - A x in FP64, stop when
 *     ||r||/||b|| <= outer_rtol; else solve A d = r in FP32 (vectors,
 *     geometric factors and operator in FP32, dot products accumulated in
 *     FP64) to inner_rtol or max_inner iterations, x += d in FP64.
 *   BP_MIXED_RELIABLE: one FP32 Jacobi-PCG whose search direction is kept;
 *     each time its recursive residual has dropped by the factor inner_rtol,
 *     x += x32 in FP64 and the FP64 residual b - A x replaces the FP32 one
 *     (at most max_outer replacements, max_inner FP32 iterations in all).
 * Stats: iters = FP32 iterations, outer = outer steps or replacements.
 * b, x: device double [ncomp][nglobal] (entries of b on Dirichlet nodes are
 * read as 0); synchronises the stream before return.
 */
int bp_pcg_solve_mixed(bp_op op, const double *b, double *x, double outer_rtol,
                       double inner_rtol, int max_outer, int max_inner,
                       bp_pcg_stats *st, void *stream);

/*
 * bp_grad_kappa -- g_q = - sum_c (D lam_c)_q^T G_q (D u_c)_q per element and
 * quadrature point: the derivative of lam^T A(kappa) u with respect to the
 * coefficient (section 4 eq. (ip1) with mu = kappa; section 5 eq. (bk5x)),
 * summed over the ncomp components. lam, u: device double [ncomp][nglobal]
 * (masked on Dirichlet nodes); g: device double [nelem][q^3], overwritten.
 * Collocated GLL operators with p <= 8; others return BP_ERR_ARG.
 */
int bp_grad_kappa(bp_op op, const double *lam, const double *u, double *g,
                  void *stream);

/*
 * bp_mass_misfit -- the data misfit of the variable-coefficient problem and
 * its gradient: L = 1/2 sum_c d_c^T M d_c and dL/du = M d, with d = u -
 * u_target and M = Q^T B_L Q the unmasked mass matrix of the operator's own
 * quadrature (section 5 eq. (mass); M is symmetric). With bp_pcg_solve and
 * bp_grad_kappa it gives the adjoint gradient of L with respect to the
 * coefficient of bp_set_coeff (A lam = mask * M d, then bp_grad_kappa).
 * d^T M d is summed from the element energies d_L^T B_L d_L in a fixed
 * order, so repeated calls give the same bits.
 *   u, u_target: device double [ncomp][nglobal], read only.
 *   grad: device double [ncomp][nglobal], overwritten with M d; NULL skips it.
 *   loss: host double, written on return (the call synchronises the stream).
 * Errors: BP_ERR_ARG (NULL u, u_target or loss; grad aliasing an input),
 * BP_ERR_HIP.
 */
int bp_mass_misfit(bp_op op, const double *u, const double *u_target, double *grad,
                   double *loss, void *stream);

/*
 * bp_set_option -- operator options (host state only, no device work).
 *   BP_OPT_TIME_APPLY (value 0/1): bp_pcg_solve records a HIP event pair on
 *   its stream around every operator launch of the iteration loop (at most
 *   4096 pairs per solve) and reports their summed duration in
 *   bp_pcg_stats.apply_ms. Costs two event records per iteration; the events
 *   are created when the option is first set (BP_ERR_HIP if that fails),
 *   without the system-scope fence of a default event
 *   (hipEventDisableSystemFence), so that recording them does not write back
 *   and invalidate the caches around the timed kernels.
 * Unknown options return BP_ERR_ARG.
 */
#define BP_OPT_TIME_APPLY 1
/*   BP_OPT_MIXED_MODE: BP_MIXED_RESTART (0, default) or BP_MIXED_RELIABLE (1),
 *   the algorithm of bp_pcg_solve_mixed. */
#define BP_OPT_MIXED_MODE 2
#define BP_MIXED_RESTART 0
#define BP_MIXED_RELIABLE 1
/*   BP_OPT_CG_VARIANT: the PCG recurrences of bp_pcg_solve.
 *     BP_CG_STANDARD (0, default): two reduction phases per iteration (alpha
 *       from p.Ap after the operator, beta from r.z after the residual update).
 *     BP_CG_SINGLE_REDUCTION (1): Chronopoulos-Gear recurrences -- s = A p
 *       by recurrence, one fused vector pass and one reduction phase per
 *       iteration (three launches instead of five for small meshes; the
 *       iterates are those of the standard form up to rounding, section 3's
 *       Jacobi-PCG in exact arithmetic). Selecting it allocates one more
 *       vector (BP_ERR_OOM if that fails); bp_pcg_solve allocates nothing. */
#define BP_OPT_CG_VARIANT 3
#define BP_CG_STANDARD 0
#define BP_CG_SINGLE_REDUCTION 1
/*   BP_OPT_CG_FUSE (2, default, 1 or 0): fewer launches per iteration with
 *     the standard recurrences in FP64, where the partial-sum tables are short
 *     enough for every work-group to reduce them itself, each in one fixed
 *     order (bit-identical in all work-groups):
 *     1: at most 1024 partial rows (about 2.6e5 nodes): every work-group of
 *     the residual update computes alpha from the operator's partial sums and
 *     every work-group of the direction update computes beta and the
 *     convergence test from the residual update's: three launches per
 *     iteration instead of five (the mass on Gauss-Legendre points, which
 *     assembles by a gather in the residual update, keeps five).
 *     2: in addition, for the collocated stiffness operator of one component
 *     up to p = 8, while (vector rows) x (operator work-groups) stays at
 *     most 4M (about 8e5 nodes at p = 7; rows of 256 nodes up to 1024
 *     rows, of 1024 nodes beyond): the
 *     operator launch forms the direction p_k = z_k + beta p_{k-1} at the
 *     nodes it gathers (beta and the stopping test from the vector kernel's
 *     partial sums) and one vector kernel stores p_k and updates x and the
 *     residual: two launches per iteration. Above those bounds, while a
 *     vector stays below 64 MiB, the same operator takes beta from the
 *     finisher of the previous iteration and the vector kernel sits between
 *     the two finishers: four launches.
 *     Other operators as 1.
 *     3: as 2 with the four-launch form at every size (for tests).
 *     The iterates are those of the standard recurrences. 0 always runs the
 *     five launches. */
#define BP_OPT_CG_FUSE 5
int bp_set_option(bp_op op, int option, int value);

/* Free every buffer of the operator (synchronises the device first). */
int bp_destroy(bp_op op);

/* Message of the calling thread's last error ("" if none). */
const char *bp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BP_H */
