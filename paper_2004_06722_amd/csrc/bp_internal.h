// Internal declarations of the bake-off library (host side).
#pragma once

#include "rules1d.hpp"
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bp.h"

namespace bp {

// ---- errors ---------------------------------------------------------------
int set_error(int code, const std::string &msg);
#define BP_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::bp::set_error(BP_ERR_HIP, std::string(#call) + ": " +         \
                                             hipGetErrorString(e_));         \
  } while (0)

// ---- host setup (setup.cpp) ----------------------------------------------
// 1D rules on [-1, 1], ascending, and the Lagrange matrices: rules1d.hpp.

// Per-operator 1D data: nodes, quadrature, J (q x p1), D (q x p1), Dq (q x q).
struct Basis {
  int p1 = 0, q = 0;
  bool colloc = false;
  std::vector<double> xi, eta, rho, J, D, Dq;
};
Basis make_basis(int p, int q, int quad);

// Internal node order. Every element-interior node (local (i, j, k) with
// 0 < i, j, k < p1 - 1) of a conforming mesh belongs to that one element
// alone, whatever the caller's numbering. If the map ed [nelem][p1^3] shows
// this (each interior slot names a node referenced exactly once), the
// interior nodes are numbered first, element by element in local order
// ([0, *n_owned)), then every other node in the order it is first met in
// ed, then the nodes no element references; returns true and the
// permutation both ways. Otherwise (p1 < 3, or an interior slot is shared)
// returns false and the caller's order is kept.
bool interior_first_order(int p1, int64_t nelem, int64_t nglobal, const int64_t *ed,
                          std::vector<int32_t> &new_of_old, std::vector<int32_t> &old_of_new,
                          int64_t *n_owned);

// ---- device-side scalars of the CG iteration --------------------------------
constexpr int kMaxComp = 8;
constexpr int kMaxTimedApplies = 4096;
struct DevScalars {
  double rz[kMaxComp], pap[kMaxComp], rr[kMaxComp], bb[kMaxComp];
  double rzp[kMaxComp];  // r.z before the last update (used after a residual replacement)
  // r.z by iteration parity for the fused small-mesh iterations: in the
  // three-launch form iteration k reads rzs[k & 1] and its direction update
  // writes rzs[(k + 1) & 1]; in the two-launch form (PZIter) the operator
  // launch of iteration k writes rzs[k & 1] and reads rzs[(k - 1) & 1]
  double rzs[2][kMaxComp];
  double alpha[kMaxComp], beta[kMaxComp];
  double tol2;
  int done;       // set when every component meets the tolerance
  int iters;      // iterations performed while not done
  int breakdown;  // p.Ap < 0 seen
  int nonfinite;  // NaN/Inf in a reduction
  int fixed;      // fixed-iteration mode: never set done
  int halted;     // set one iteration after done: the last x update has run
  int pad_[2];
};

// Operands of the two-launch iteration of small meshes (k_stiff_colloc_pz
// and the vector kernel k_cg_update_rxp_fused; one component): the operator
// applies A to p_k = z_k + beta_{k-1} p_{k-1}, formed at the gathered nodes
// from the stored z_k and p_{k-1}, with beta_{k-1} = (r_k.z_k) /
// (r_{k-1}.z_{k-1}) from the vector kernel's partial rows; the vector kernel
// then stores p_k (same expression, same beta). r.z by iteration parity:
// iteration k's operator launch writes rzs[k & 1].
struct PZIter {
  const double *z;   // z_k = dinv r_k, [n]
  const double *pr;  // partial rows [nbv][2]: r_k.z_k, r_k.r_k
  int64_t nbv;
  DevScalars *sc;
  int parity;  // k & 1
  int check;   // a stopping test is honoured (not fixed iterations)
  int first;   // k = 0: p_0 = z_0 is stored already; nothing to reduce
  int fused;   // 1: reduce pr here (two launches); 0: beta from sc->beta (four)
};

}  // namespace bp

// The operator object.
struct bp_op_s {
  int p = 0, p1 = 0, q = 0, quad = 0, ncomp = 1;
  int64_t nelem = 0, nglobal = 0;
  bool colloc = false, has_dirichlet = false, fp32 = false;
  int device = 0;
  bp::Basis basis;
  // device buffers (owned)
  int32_t *idx = nullptr;    // [E][p1^3]; Dirichlet node g stored as -1-g
  double *G = nullptr;       // [E][6][q^3] geometric factors
  double *Gk = nullptr;      // kappa_q * G (allocated by bp_set_coeff)
  double *Bt = nullptr;      // [E][q^3]
  double *basis_d = nullptr; // J | D | Dq on the device (FP64)
  double *Bb = nullptr;      // beta_q * B~ (allocated by bp_set_helmholtz; NULL: beta = 0)
  float *G32 = nullptr, *Gk32 = nullptr, *Bt32 = nullptr, *Bb32 = nullptr, *basis32 = nullptr;
  bool kappa_set = false;
  // inverse diagonals: [0] mass, [1] stiffness (masked), [2] Helmholtz (masked)
  double *dinv[3] = {nullptr, nullptr, nullptr};
  bool dinv_valid[3] = {false, false, false};
  // CG workspace
  double *r = nullptr, *pv = nullptr, *w = nullptr, *part = nullptr, *tmp = nullptr;
  float *r32 = nullptr, *p32 = nullptr, *w32 = nullptr, *x32 = nullptr, *b32 = nullptr;
  float *dinv32 = nullptr;
  int64_t part_len = 0;      // doubles in `part`
  bp::DevScalars *sc = nullptr;   // device
  bp::DevScalars *sc_host = nullptr;  // pinned host mirror
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evm0 = nullptr, evm1 = nullptr;  // around a mixed solve (BP_SETUP_FP32)
  bool time_apply = false;
  int mixed_mode = 0;  // BP_MIXED_RESTART or BP_MIXED_RELIABLE (bp_pcg_solve_mixed)
  int cg_variant = 0;  // BP_CG_STANDARD or BP_CG_SINGLE_REDUCTION (bp_pcg_solve)
  int cg_fuse = 2;  // BP_OPT_CG_FUSE: fewer launches per iteration (0 off, 1, 2, 3)
  double *sv = nullptr;  // s = A p of the single-reduction PCG (allocated when selected)
  // Gauss-Legendre operators: the gather map transposed (CSR over global
  // nodes: the element-local slots e p1^3 + l of node g are
  // tr_pos[tr_off[g] .. tr_off[g + 1]), ascending) and the element-local
  // output wl [ncomp][nelem][p1^3] of the mass kernel (wl32 in FP32)
  int32_t *tr_off = nullptr, *tr_pos = nullptr;
  // internal node order (interior_first_order): perm[v] = the caller's id of
  // internal node v (NULL: the caller's order); internal nodes [0, n_owned)
  // are element-interior, each written by its element with a plain store;
  // bi, xi: b and x of a solve in the internal order
  int32_t *perm = nullptr;
  int32_t *iperm = nullptr;  // iperm[g] = the internal id of the caller's node g
  int64_t n_owned = 0;
  double *bi = nullptr, *xi = nullptr;
  double *wl = nullptr;
  float *wl32 = nullptr;
  std::vector<hipEvent_t> apply_ev;  // pairs around operator launches
};
