// Device kernels of the bake-off operators (gfx950, wave64).
//
// Operator application w = Q^T A_L Q u (section 4) with the element operator
// of section 5: eq. (bk5x) for the stiffness matrix and eq. (mass) for the
// mass matrix, applied by sum factorisation (eq. (tens1)). One work-group
// owns one element (or, for small p, a slab of elements); each thread owns
// one (i, j) column of the element and walks the k direction in registers,
// so the k-derivatives never leave the thread while the i- and
// j-derivatives are taken through LDS tiles. The scatter w = Q^T w_L uses
// hardware FP64/FP32 atomic adds into a zeroed w; the local energy
// sum_e u_L^T w_L (Appendix A1: rho = w^T u before assembly) is reduced per
// work-group into a partial sum.
#pragma once
#include "bp_internal.h"
#include "rules1d.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bp {

// Elements per work-group for planes of n threads: the count up to 256
// threads that leaves the fewest idle lanes in the whole waves it occupies
// (the smaller count on ties), e.g. 5 planes of 7 x 7 in 256 threads.
constexpr int plane_elements(int n) {
  int best = 1, best_used = n, best_threads = ((n + 63) / 64) * 64;
  for (int e = 2; e * n <= 256; ++e) {
    const int used = e * n, threads = ((used + 63) / 64) * 64;
    if ((long)used * best_threads > (long)best_used * threads) {
      best = e;
      best_used = used;
      best_threads = threads;
    }
  }
  return best;
}

// Thread plane of an element: M x M threads, M = max(p1, q); EPB elements per
// work-group (plane_elements); THREADS rounded up to whole waves (idle lanes
// take part in barriers and reductions only).
template <int P1, int Q>
struct Plane {
  static constexpr int M = P1 > Q ? P1 : Q;
  static constexpr int N = M * M;
  static constexpr int EPB = plane_elements(N);
  static constexpr int USED = EPB * N;
  static constexpr int THREADS = ((USED + 63) / 64) * 64;
};

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Sum v over the work-group in a fixed order; thread 0 stores out[c * stride].
template <int NC, int THREADS>
__device__ __forceinline__ void block_sum_store(double (&v)[NC], double *out, int stride) {
  constexpr int NW = THREADS / 64;
  __shared__ double red[NW][NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[c] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NC; ++c) red[wid][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = 0.0;
      for (int k = 0; k < NW; ++k) s += red[k][c];
      out[c * stride] = s;
    }
}

// Column sums of a partial table part[nb][2] (r.z and r.r of one component)
// in one fixed order, split in two steps so that the loads of the first U
// rows per thread are in flight together with the operator's map and G:
// thread t adds rows t, t + THREADS, ... in turn; a fixed shuffle tree per
// wave; the waves' sums in order. Every work-group obtains bit-identical sums.
template <int THREADS>
struct RowPairSums {
  static constexpr int U = 8;
  double v[U][2];
  __device__ __forceinline__ void issue(const double *__restrict__ part, int64_t nb) {
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t r = threadIdx.x + (int64_t)q * THREADS;
      v[q][0] = r < nb ? part[2 * r] : 0.0;
      v[q][1] = r < nb ? part[2 * r + 1] : 0.0;
    }
  }
  __device__ __forceinline__ void finish(const double *__restrict__ part, int64_t nb,
                                         double *res) {
    constexpr int NW = THREADS / 64;
    __shared__ double red[NW][2];
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      a0 += v[q][0];
      a1 += v[q][1];
    }
    int64_t r = threadIdx.x + (int64_t)U * THREADS;
    for (; r + 3 * THREADS < nb; r += 4 * THREADS) {  // four rows' loads together
      double b[4][2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        b[q][0] = part[2 * (r + q * THREADS)];
        b[q][1] = part[2 * (r + q * THREADS) + 1];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a0 += b[q][0];
        a1 += b[q][1];
      }
    }
    for (; r < nb; r += THREADS) {
      a0 += part[2 * r];
      a1 += part[2 * r + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a0 += __shfl_down(a0, o, 64);
      a1 += __shfl_down(a1, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6][0] = a0;
      red[threadIdx.x >> 6][1] = a1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      double x = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) x += red[k][threadIdx.x];
      res[threadIdx.x] = x;
    }
    __syncthreads();
  }
};

// Element-interior local node (0 < i, j, k < P1 - 1): with the internal node
// order (own != 0) no other element touches it, so the scatter stores its
// value instead of adding it atomically (its internal id lies in a block of
// the element's own, on cache lines no atomic touches).
template <int P1>
__device__ __forceinline__ bool interior_node(int i, int j, int k) {
  return i > 0 && i < P1 - 1 && j > 0 && j < P1 - 1 && k > 0 && k < P1 - 1;
}

// Decoded gather index: global id, or -1 when the node is skipped
// (element slot not live, or a Dirichlet node under the mask).
__device__ __forceinline__ int decode_index(int v, bool live, int masked) {
  if (!live) return -1;
  if (v >= 0) return v;
  return masked ? -1 : -1 - v;
}

// Body of the collocated stiffness kernels (described below): with MULTI
// every component of u and w ([ncomp][cs]) runs through one work-group, G and
// the map loaded once; otherwise the one component that u and w point at
// (energy column c0).
template <int P1, typename T, bool LOCAL, bool HELM, bool MULTI, bool PZ = false>
__device__ __forceinline__ void stiff_colloc_body(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ G,
    const T *__restrict__ Bb, const T *__restrict__ u, T *__restrict__ w, int64_t cs, int ncomp,
    int c0, int masked, double *__restrict__ part, const int *__restrict__ done, int own,
    PZIter pz = {}) {
  constexpr int NC = 1;  // LDS tiles of one component at a time
  static constexpr GLLDeriv<P1, T> kD{};  // D^, compile-time constants
  const T *const Dg = kD.D;
  using PL = Plane<P1, P1>;
  constexpr int N3 = P1 * P1 * P1, PP = P1 * P1, PAD = P1 + 1;
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ij = t % PL::N;
  const int i = ij % P1, j = ij / P1;
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  if (PL::EPB == 1 && e >= nelem) return;  // uniform over the work-group
  const bool live = act && e < nelem;
  const int64_t ec = live ? e : nelem - 1;  // element whose data a lane reads

  __shared__ T sD[P1][PAD];   // sD[a][m]  = D^[a][m]
  __shared__ T sDt[P1][PAD];  // sDt[m][a] = D^[a][m]
  __shared__ T su[PL::EPB][NC][P1][P1][PAD];
  __shared__ T sr[PL::EPB][NC][P1][P1][PAD];
  __shared__ T ss[PL::EPB][NC][P1][P1][PAD];
  // two-launch iteration (PZIter, one component): the scalars and the
  // partial rows of r_k.z_k and r_k.r_k are requested first
  RowPairSums<PL::THREADS> pzs;
  double pz_rzo = 0.0, pz_bb = 1.0, pz_tol2 = 0.0;
  int pz_fixed = 1;
  double pz_beta = 0.0;
  if constexpr (PZ) {
    if (!pz.first) {
      const DevScalars *sc = pz.sc;
      if (pz.fused) {
        pz_rzo = sc->rzs[pz.parity ^ 1][0];
        pz_bb = sc->bb[0];
        pz_tol2 = sc->tol2;
        pz_fixed = sc->fixed;
        pzs.issue(pz.pr, pz.nbv);
      } else {
        pz_beta = sc->beta[0];  // from the finisher of the previous iteration
      }
    }
  }
  // one round trip: the column of the gather map and of G
  const int32_t *ie = idx + ec * N3 + ij;
  const T *Ge = G + ec * 6 * N3 + ij;
  int gk[P1];
  T g[6][P1];
#pragma unroll
  for (int k = 0; k < P1; ++k)
    gk[k] = LOCAL ? (int)(ec * N3) + ij + k * PP : __builtin_nontemporal_load(ie + k * PP);
#pragma unroll
  for (int k = 0; k < P1; ++k)
#pragma unroll
    for (int n = 0; n < 6; ++n) g[n][k] = __builtin_nontemporal_load(Ge + n * N3 + k * PP);
  // Helmholtz: beta B~ at the lane's nodes (B_beta is diagonal with GLL)
  T bb[HELM ? P1 : 1];
  if constexpr (HELM) {
#pragma unroll
    for (int k = 0; k < P1; ++k) bb[k] = __builtin_nontemporal_load(Bb + ec * N3 + ij + k * PP);
  }

  // decode: global id, and bit k of mb set when node k is gathered and
  // scattered (clear for dead slots and masked Dirichlet nodes)
  unsigned mb = 0;
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = gk[k];
    if (live && (LOCAL || v >= 0 || !masked)) mb |= 1u << k;
    if (!LOCAL) gk[k] = v >= 0 ? v : -1 - v;
  }

  // two-launch iteration (PZIter): z_k and p_{k-1} gathered before the
  // partial sums are finished (their loads in flight meanwhile); r_k.z_k and
  // r_k.r_k, the same in every work-group; the stopping test on r_k ends the
  // launch in all of them at once; p_k = z_k + beta p_{k-1} at the nodes
  T pzp[PZ ? P1 : 1], pzz[PZ ? P1 : 1];
  __shared__ double pzr[2];
  if constexpr (PZ) {
    static_assert(!MULTI, "the two-launch iteration runs one component");
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      pzp[k] = u[gk[k]];
      pzz[k] = pz.first ? T(0) : pz.z[gk[k]];
    }
    if (!pz.first && pz.fused) {
      pzs.finish(pz.pr, pz.nbv, pzr);
      const double bb = pz_bb > 0.0 ? pz_bb : 1.0;
      const bool conv = !pz_fixed && pzr[1] <= pz_tol2 * bb;
      const bool bad = !isfinite(pzr[0]) || !isfinite(pzr[1]);
      const bool stop = pz.check && (conv || bad);
      pz_beta = pz_rzo != 0.0 ? pzr[0] / pz_rzo : 0.0;
      if (blockIdx.x == 0 && t == 0) {
        DevScalars *sc = pz.sc;
        sc->rzs[pz.parity][0] = sc->rz[0] = pzr[0];
        sc->rzp[0] = pz_rzo;
        sc->rr[0] = pzr[1];
        sc->beta[0] = pz_beta;
        if (bad) sc->nonfinite = 1;
        if (stop) sc->done = sc->halted = 1;  // x_k is the answer
      }
      if (stop) return;
    }
    if (!pz.first)
#pragma unroll
      for (int k = 0; k < P1; ++k) pzp[k] = __builtin_fma(pz_beta, pzp[k], pzz[k]);
  }

  const int nrun = MULTI ? ncomp : 1;
#pragma unroll 1
  for (int cc = 0; cc < nrun; ++cc) {
    const T *uc = u + (MULTI ? cc * cs : 0);
    T *wc = w + (MULTI ? cc * cs : 0);
    // gather u (PZ: p_k, formed above as the vector kernel forms it)
    T ru[NC][P1];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        const T v = PZ ? pzp[PZ ? k : 0] : uc[gk[k]];
        ru[c][k] = (mb >> k & 1u) ? v : T(0);
      }
    if (cc == 0) {
      // D^ staged after the first gather is requested, so both wait together
      for (int x = t; x < PP; x += PL::THREADS) {
        sD[x / P1][x % P1] = Dg[x];
        sDt[x % P1][x / P1] = Dg[x];
      }
    } else {
      __syncthreads();  // the tiles of the previous component have been read
    }

    // u into LDS; derivative along t (k) in registers
    T rt[NC][P1];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        if (act) su[slot][c][k][j][i] = ru[c][k];
        T s = 0;
#pragma unroll
        for (int m = 0; m < P1; ++m) s += Dg[k * P1 + m] * ru[c][m];
        rt[c][k] = s;
      }
    }
    __syncthreads();

    // derivatives along r, s through LDS; apply G; energy at the points
    double en[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) en[c] = 0.0;
    if constexpr (HELM) {
      if (act)
#pragma unroll
        for (int k = 0; k < P1; ++k) en[0] += (double)ru[0][k] * (double)(bb[k] * ru[0][k]);
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T ur = 0, us = 0;
#pragma unroll
        for (int m = 0; m < P1; ++m) {
          ur += sD[i][m] * su[slot][c][k][j][m];
          us += sD[j][m] * su[slot][c][k][m][i];
        }
        const T ut = rt[c][k];
        const T vr = g[0][k] * ur + g[1][k] * us + g[2][k] * ut;
        const T vs = g[1][k] * ur + g[3][k] * us + g[4][k] * ut;
        const T vt = g[2][k] * ur + g[4][k] * us + g[5][k] * ut;
        // idle lanes of a partly used wave read another element's tile: no energy
        if (act)
          en[c] += (double)ur * (double)vr + (double)us * (double)vs + (double)ut * (double)vt;
        rt[c][k] = vt;
        if (act) {
          sr[slot][c][k][j][i] = vr;
          ss[slot][c][k][j][i] = vs;
        }
      }
    }
    __syncthreads();

    // transposed derivatives and scatter
#pragma unroll
    for (int k = 0; k < P1; ++k) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        T acc = 0;
        if constexpr (HELM) acc = bb[k] * su[slot][c][k][j][i];
#pragma unroll
        for (int m = 0; m < P1; ++m) {
          acc += Dg[m * P1 + k] * rt[c][m];
          acc += sDt[i][m] * sr[slot][c][k][j][m];
          acc += sDt[j][m] * ss[slot][c][k][m][i];
        }
        if (mb >> k & 1u) {
          if (LOCAL || (own && interior_node<P1>(i, j, k)))
            // element-local output, or a node of this element alone (streamed:
            // nothing reads it again in this launch)
            __builtin_nontemporal_store(acc, wc + gk[k]);
          else
            atomic_add(wc + gk[k], acc);
        }
      }
    }
    if (part)
      block_sum_store<NC, PL::THREADS>(en, part + (int64_t)blockIdx.x * ncomp +
                                               (MULTI ? cc : c0), 1);
  }
}

// ---------------------------------------------------------------------------
// BK5/BK6: stiffness with collocated GLL quadrature (J^ = I, q = p1).
// Vectors are component-major ([ncomp][nglobal]). k_stiff_colloc applies one
// component (u and w point at component c0; ncomp and c0 place the energy
// partial); k_stiff_colloc_nc applies all ncomp components of u and w
// (component stride cs) in one launch: each work-group loads its element's G
// column and map once and runs the components through the same LDS tiles
// one after the other (BK6 and the vector problems), with at most 256
// registers per lane so that two waves share each SIMD.
//
// Arithmetic is not the limit (HBM traffic and the rate of the atomic
// scatter are), so the kernel is laid out to need few dependent round trips:
// each lane requests its whole column of G (6 x p1 values) and of the gather
// map at entry, then gathers u, then computes from registers and LDS. The k direction stays in registers; the r and s contractions go
// through LDS tiles. Loads are branch-free: an element slot past the end
// reads the last element and a Dirichlet node reads its (valid) global
// entry, both masked. D^ is a compile-time table (rules1d.hpp): entries
// with compile-time indices are immediates, which the compiler rematerialises
// in each component of the loop instead of keeping them in scalar registers;
// the lane-dependent rows come from LDS. The local energy u_L^T A_L u_L is
// accumulated at the quadrature points as (D u)^T G (D u) = u_L^T w_L.
// HELM adds the Helmholtz term of eq. (hm2): with collocated GLL points the
// mass matrix is diagonal, so w_L += (beta B~) u_L node by node, with the
// beta-scaled B~ read beside G (one more word per point). With the internal
// node order (own) the element-interior nodes are stored, not added.
// ---------------------------------------------------------------------------
// Two waves per SIMD requested: it binds only from p1 = 11 in FP64 (the
// p1 <= 10 and FP32 instances compile to the same code with or without it),
// where the compiler otherwise let the register count pass 256 (p1 = 14) or
// scheduled the same 252 registers differently (p1 = 13) (BK5 alone, N = 12:
// 7.2 -> 10.0 TFLOP/s, N = 13: 7.3 -> 8.6;
// BP5 iteration at N = 11: 2.09 -> 1.69 ms, N = 12: 2.53 -> 2.46 ms, E = 2^15),
// at the cost of a few spilled registers at p1 = 13, 14.
template <int P1, typename T, bool LOCAL = false, bool HELM = false>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) __attribute__((amdgpu_waves_per_eu(2))) void k_stiff_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ G,
    const T *__restrict__ Bb, const T *__restrict__ u, T *__restrict__ w, int ncomp, int c0,
    int masked, double *__restrict__ part, const int *__restrict__ done, int own) {
  stiff_colloc_body<P1, T, LOCAL, HELM, false>(nelem, idx, G, Bb, u, w, 0, ncomp, c0, masked,
                                               part, done, own);
}

// The operator of the two-launch iteration (PZIter): p_k formed at the
// gathered nodes from z_k and p_{k-1}, FP64, assembled output.
// One component (ncomp = 1): u = p_{k-1} (p_0 at k = 0), pz.z = z_k.
template <int P1>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_stiff_colloc_pz(
    int64_t nelem, const int32_t *__restrict__ idx, const double *__restrict__ G,
    const double *__restrict__ u, double *__restrict__ w, int ncomp, int c0, int masked,
    double *__restrict__ part, const int *__restrict__ done, int own, PZIter pz) {
  stiff_colloc_body<P1, double, false, false, false, true>(
      nelem, idx, G, nullptr, u, w, 0, ncomp, c0, masked, part, done, own, pz);
}

template <int P1, typename T, bool LOCAL = false, bool HELM = false>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS), 2) void k_stiff_colloc_nc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ G,
    const T *__restrict__ Bb, const T *__restrict__ u, T *__restrict__ w, int64_t cs,
    int ncomp, int masked, double *__restrict__ part, const int *__restrict__ done, int own) {
  stiff_colloc_body<P1, T, LOCAL, HELM, true>(nelem, idx, G, Bb, u, w, cs, ncomp, 0, masked,
                                              part, done, own);
}

// ---------------------------------------------------------------------------
// Mass with collocated GLL quadrature: B_L is diagonal (section 5, remark
// after eq. (mass)); w = Q^T (B~ .* Q u).
// ---------------------------------------------------------------------------
template <int P1, typename T, bool LOCAL = false>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_mass_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Bt,
    const T *__restrict__ u, T *__restrict__ w, int64_t cstride, int ncomp, int masked,
    double *__restrict__ part, const int *__restrict__ done, int own) {
  using PL = Plane<P1, P1>;
  constexpr int N3 = P1 * P1 * P1;
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ij = t % PL::N;
  const int i = ij % P1, j = ij / P1;
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  const bool live = act && e < nelem;
  int gk[P1];
  T b[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    if constexpr (LOCAL) {
      gk[k] = live ? (int)(e * N3) + k * P1 * P1 + ij : -1;
    } else {
      const int v = live ? idx[e * N3 + k * P1 * P1 + ij] : -1;
      gk[k] = decode_index(v, live, masked);
    }
    b[k] = live ? Bt[e * N3 + k * P1 * P1 + ij] : T(0);
  }
  for (int cc = 0; cc < ncomp; ++cc) {
    double en[1] = {0.0};
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      if (gk[k] < 0) continue;
      const int64_t o = gk[k] + cc * cstride;
      const T uv = u[o];
      const T wv = b[k] * uv;
      en[0] += (double)uv * (double)wv;
      if (LOCAL || (own && interior_node<P1>(i, j, k)))
        w[o] = wv;
      else
        atomic_add(w + o, wv);
    }
    if (part) block_sum_store<1, PL::THREADS>(en, part + (int64_t)blockIdx.x * ncomp + cc, 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BK1-BK4: Gauss-Legendre quadrature with q = p1 + 1 points per direction.
// Every 1D contraction is done by a thread that owns a whole pencil of the
// element (all entries along one direction) in registers, so each value read
// from LDS feeds a full row of outputs, and the contraction uses the even-odd
// splitting of the appendix on even-odd decompositions: the GLL nodes and the
// Gauss points are both symmetric about 0, so J^ is centro-symmetric and D^
// centro-antisymmetric, and each pair of mirrored outputs costs one pass over
// half the (folded) inputs. Stages of the stiffness operator:
//   1 column (i, j) along t: A = J^_t u, A' = D^_t u       -> LDS [j][c][i]
//   2 pencil (i, c) along s: B = J^_s A, C = D^_s A, B' = J^_s A'
//                                                          -> LDS [b][c][i]
//   3 pencil (b, c) along r: u_r = D^_r B, u_s = J^_r C, u_t = J^_r B',
//     v = G (u_r, u_s, u_t) (eq. (gij)), then P = D^T_r v_r, R = J^T_r v_s,
//     T = J^T_r v_t, all in registers                      -> LDS (in place)
//   4 pencil (i, c) along s: S1 = J^T_s P + D^T_s R, S2 = J^T_s T
//                                                          -> LDS (in place)
//   5 column (i, j) along t: w = J^T_t S1 + D^T_t S2, scatter-added.
// The mass operator runs the J^ chains only with v = B~ x (eq. (mass)); the
// Helmholtz operator (eq. (hm2)) runs both, adding J^T_r (beta B~ x) to P.
// The quadrature data of these operators (G, B~) are stored with the point
// index reversed, [a][b][c] with c fastest, so that the stage-3 pencils,
// adjacent lanes along (b, c), read them coalesced; G and the gather map are
// requested at entry. k_op_gl applies one component (u and w point at
// component c0); k_op_gl_nc all of them, G and the map loaded once per
// element (the multi-component stiffness stages its point values through
// LDS and requests the next component's gather during stage 4). With LOCAL
// the input is read and the result stored per element. With
// WL the input is gathered from the global vector and the element result
// w_L is stored per element ([E][p1^3], zero at skipped nodes) instead of
// scatter-added: the mass operator moves little quadrature data, so FP64
// atomics bound it, and the assembly Q^T w_L is then done as a fixed-order
// gather over the transposed map (by the residual update of the PCG, or by
// a gather kernel after the launch).
// ---------------------------------------------------------------------------
enum GLMode { kGLMass = 0, kGLStiff = 1, kGLHelm = 2 };

// Even-odd tables of an NO x NI matrix M with M[NO-1-a][NI-1-i] = S M[a][i]:
// row a < (NO+1)/2 holds E[a][i] = (M[a][i] + M[a][NI-1-i]) / 2 and
// O[a][i] = (M[a][i] - M[a][NI-1-i]) / 2 for i < NI/2, then M[a][NI/2] when
// NI is odd. Then for a < NO/2, with e_i = x_i + x_{NI-1-i} and
// o_i = x_i - x_{NI-1-i}: y_a = E e + O o (+ middle term), and
// y_{NO-1-a} = S (E e - O o (+ middle term)).
template <int NO, int NI>
struct EvenOdd {
  static constexpr int H = NI / 2, HO = NO / 2, ROWS = (NO + 1) / 2, SIZE = ROWS * NI;
  static constexpr bool MI = (NI & 1) != 0, MO = (NO & 1) != 0;
};

// Folded input pencil: mirrored sums and differences, and the middle entry.
template <int NI, typename T>
struct Folded {
  T e[NI / 2 > 0 ? NI / 2 : 1], o[NI / 2 > 0 ? NI / 2 : 1], m;
};

template <int NI, typename T>
__device__ __forceinline__ Folded<NI, T> fold(const T (&x)[NI]) {
  Folded<NI, T> f;
#pragma unroll
  for (int i = 0; i < NI / 2; ++i) {
    f.e[i] = x[i] + x[NI - 1 - i];
    f.o[i] = x[i] - x[NI - 1 - i];
  }
  f.m = (NI & 1) ? x[NI / 2] : T(0);
  return f;
}

// Outputs a and NO-1-a of y = M x (only ya for the middle row of odd NO,
// where one half is zero by symmetry).
template <int NO, int NI, int S, typename T>
__device__ __forceinline__ void eo_row(const T *__restrict__ tab, int a, const Folded<NI, T> &x,
                                       T &ya, T &yb) {
  using E = EvenOdd<NO, NI>;
  const T *r = tab + a * NI;
  const bool mid = E::MO && a == E::HO;
  T ye = 0, yo = 0;
  if (!mid || S > 0) {
#pragma unroll
    for (int i = 0; i < E::H; ++i) ye += r[i] * x.e[i];
    if constexpr (E::MI) ye += r[2 * E::H] * x.m;
  }
  if (!mid || S < 0) {
#pragma unroll
    for (int i = 0; i < E::H; ++i) yo += r[E::H + i] * x.o[i];
  }
  ya = ye + yo;
  yb = S > 0 ? ye - yo : yo - ye;
}

// z = M^T v accumulated input pair by input pair: p[i] = (z_i + z_{NI-1-i})/2,
// m[i] = (z_i - z_{NI-1-i})/2, c = z_{NI/2} (odd NI).
template <int NI, typename T>
struct Unfold {
  T p[NI / 2 > 0 ? NI / 2 : 1], m[NI / 2 > 0 ? NI / 2 : 1], c;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) p[i] = m[i] = T(0);
    c = T(0);
  }
  // inputs a and NO-1-a (a < NO/2), or the middle input alone
  template <int NO, int S>
  __device__ __forceinline__ void add(const T *__restrict__ tab, int a, T va, T vb) {
    using E = EvenOdd<NO, NI>;
    const T *r = tab + a * NI;
    const bool mid = E::MO && a == E::HO;
    const T sp = mid ? va : (S > 0 ? va + vb : va - vb);
    const T sm = mid ? va : (S > 0 ? va - vb : va + vb);
    if (!mid || S > 0) {
#pragma unroll
      for (int i = 0; i < E::H; ++i) p[i] += r[i] * sp;
      if constexpr (E::MI) c += r[2 * E::H] * sp;
    }
    if (!mid || S < 0) {
#pragma unroll
      for (int i = 0; i < E::H; ++i) m[i] += r[E::H + i] * sm;
    }
  }
  __device__ __forceinline__ void get(T (&z)[NI]) const {
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
      z[i] = p[i] + m[i];
      z[NI - 1 - i] = p[i] - m[i];
    }
    if constexpr ((NI & 1) != 0) z[NI / 2] = c;
  }
};

// LDS layout and elements per work-group of the Gauss-Legendre kernels: up
// to 256 threads (q^2 per element) and at most 80 KB of LDS per work-group,
// so that two work-groups share a CU.
constexpr int gl_row_stride(int p1) { return p1 | 1; }
constexpr int gl_lds_per_elem(int p1, int q, int mode) {
  return (mode == kGLMass ? 1 : 2) * p1 * q * p1 +
         (mode == kGLMass ? 1 : 3) * q * q * gl_row_stride(p1);
}
constexpr int gl_epb(int p1, int q, int mode) {
  const int by_threads = q * q >= 256 ? 1 : 256 / (q * q);
  const int by_lds = (80 * 1024 - 1024) / (8 * gl_lds_per_elem(p1, q, mode));
  const int e = by_threads < by_lds ? by_threads : by_lds;
  return e < 1 ? 1 : e;
}

template <int P1, int Q, int MODE>
struct GLPlane {
  static constexpr int NA = MODE == kGLMass ? 1 : 2;  // tiles [j][c][i] per element
  static constexpr int NB = MODE == kGLMass ? 1 : 3;  // tiles [b][c][i] per element
  static constexpr int RS = gl_row_stride(P1);        // odd row stride of the B tiles
  static constexpr int EPB = gl_epb(P1, Q, MODE);
  static constexpr int USED = EPB * Q * Q;
  static constexpr int THREADS = ((USED + 63) / 64) * 64;
};

template <int P1, int Q, typename T, int MODE, bool LOCAL, bool WL, bool MULTI>
__device__ __forceinline__ void gl_body(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Gm,
    const T *__restrict__ Bb, const T *__restrict__ basis, const T *__restrict__ u,
    T *__restrict__ w, int64_t cs, int64_t ws, int ncomp, int c0, int masked,
    double *__restrict__ part, const int *__restrict__ done, int own) {
  using PL = GLPlane<P1, Q, MODE>;
  using EO = EvenOdd<Q, P1>;
  constexpr bool STIFF = MODE != kGLMass, HELM = MODE == kGLHelm;
  constexpr int N3 = P1 * P1 * P1, NQ = Q * Q * Q, QQ = Q * Q;
  constexpr int NG = STIFF ? 6 : 1;
  constexpr int LA = Q * P1;                // A tiles: [j][c][i]
  constexpr int RS = PL::RS, LB = Q * RS;   // B tiles: [b][c][i], rows of RS
  static_assert(Q == P1 + 1, "Gauss-Legendre kernel expects q = p1 + 1");
  // several stiffness components: v at the points goes through the pencil's
  // own LDS rows (RS >= q entries) instead of three register accumulators
  // beside G, which stays in registers for all components
  constexpr bool VST = MULTI && MODE == kGLStiff && RS >= Q;
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / QQ : 0;
  const int l = act ? t % QQ : QQ;  // lane in the element's plane (QQ: no role)
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  const bool live = act && e < nelem;
  const int64_t ec = live ? e : nelem - 1;  // element whose data the lane reads
  // roles: column (i, j) along t; pencil (i, c) along s; pencil (b, c) along r
  const bool col = l < P1 * P1;
  const int ci = col ? l % P1 : 0, cj = col ? l / P1 : 0;
  const bool spn = l < Q * P1;
  const int rl = l < QQ ? l : 0;
  const int rrow = (rl / Q) * LB + (rl % Q) * RS;  // the r-pencil's row in the B tiles

  __shared__ T sA[PL::EPB][PL::NA][P1 * LA];
  __shared__ T sB[PL::EPB][PL::NB][Q * LB];
  T *const A0 = sA[slot][0];
  T *const A1 = sA[slot][PL::NA - 1];
  T *const B0 = sB[slot][0];
  T *const B1 = sB[slot][STIFF ? 1 : 0];
  T *const B2 = sB[slot][PL::NB - 1];
  // even-odd tables of J^ and D^, compile-time constants (immediates)
  static constexpr GLTables<P1, Q, T> kTab{};
  static_assert(GLTables<P1, Q, T>::SIZE == EO::SIZE, "even-odd table size");
  const T *tJ = kTab.J;
  const T *tD = kTab.D;

  // one round trip: node column of the gather map, the r-pencil's G / B~
  int gk[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k)
    gk[k] = LOCAL ? (int)(ec * N3) + ci + P1 * (cj + P1 * k)
                  : idx[ec * N3 + ci + P1 * (cj + P1 * k)];
  T g[NG][Q];
  {
    const T *Ge = Gm + ec * NG * NQ + rl;
#pragma unroll
    for (int a = 0; a < Q; ++a)
#pragma unroll
      for (int n = 0; n < NG; ++n) g[n][a] = __builtin_nontemporal_load(Ge + n * NQ + a * QQ);
  }
  unsigned mb = 0;  // bit k: node k of the column is gathered and scattered
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = gk[k];
    if (live && col && (LOCAL || v >= 0 || !masked)) mb |= 1u << k;
    if (!LOCAL) gk[k] = v >= 0 ? v : -1 - v;
  }

  // components one after the other through the same tiles (MULTI), with G,
  // the map and the masks kept in registers
  const int nrun = MULTI ? ncomp : 1;
  // Several stiffness components (arithmetic and latency bound, not HBM
  // bound): the next component's column of u is requested during stage 4 of
  // the current one, so its gather latency overlaps the last two stages.
  // Lanes without a column read column (0, 0), a valid address.
  constexpr bool PREF = MULTI && STIFF;
  T un[PREF ? P1 : 1];
  if constexpr (PREF)
#pragma unroll
    for (int k = 0; k < P1; ++k) un[k] = u[gk[k]];
#pragma unroll 1
  for (int cc = 0; cc < nrun; ++cc) {
    if (cc > 0) __syncthreads();  // the previous component's A tiles have been read
    const T *const uc = u + (MULTI ? cc * cs : 0);
    T *const wc = w + (MULTI ? cc * ws : 0);
    // 1: gather, then along t
    if (col) {
      T uk[P1];
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        const T v = PREF ? un[PREF ? k : 0] : uc[gk[k]];
        uk[k] = (mb >> k & 1u) ? v : T(0);
      }
      const Folded<P1, T> f = fold(uk);
      T *a0 = A0 + cj * LA + ci;
      T *a1 = A1 + cj * LA + ci;
#pragma unroll
      for (int c = 0; c < EO::ROWS; ++c) {
        T ya, yb;
        eo_row<Q, P1, 1>(tJ, c, f, ya, yb);
        a0[c * P1] = ya;
        if (c < EO::HO) a0[(Q - 1 - c) * P1] = yb;
        if constexpr (STIFF) {
          eo_row<Q, P1, -1>(tD, c, f, ya, yb);
          a1[c * P1] = ya;
          if (c < EO::HO) a1[(Q - 1 - c) * P1] = yb;
        }
      }
    }
    __syncthreads();
    // 2: along s (pencil (i, c) = lane l: its column of the A tiles is l + j LA)
    if (spn) {
      const int ob = (l / P1) * RS + l % P1;  // (c, i) in the B tiles
      T x[P1];
#pragma unroll
      for (int j = 0; j < P1; ++j) x[j] = A0[j * LA + l];
      const Folded<P1, T> f = fold(x);
#pragma unroll
      for (int b = 0; b < EO::ROWS; ++b) {
        T ya, yb;
        eo_row<Q, P1, 1>(tJ, b, f, ya, yb);
        B0[b * LB + ob] = ya;
        if (b < EO::HO) B0[(Q - 1 - b) * LB + ob] = yb;
        if constexpr (STIFF) {
          eo_row<Q, P1, -1>(tD, b, f, ya, yb);
          B1[b * LB + ob] = ya;
          if (b < EO::HO) B1[(Q - 1 - b) * LB + ob] = yb;
        }
      }
      if constexpr (STIFF) {
#pragma unroll
        for (int j = 0; j < P1; ++j) x[j] = A1[j * LA + l];
        const Folded<P1, T> f1 = fold(x);
#pragma unroll
        for (int b = 0; b < EO::ROWS; ++b) {
          T ya, yb;
          eo_row<Q, P1, 1>(tJ, b, f1, ya, yb);
          B2[b * LB + ob] = ya;
          if (b < EO::HO) B2[(Q - 1 - b) * LB + ob] = yb;
        }
      }
    }
    __syncthreads();
    // 3: along r, the quadrature points, and back along r
    double en = 0.0;
    if (l < QQ) {
      T y[P1];
#pragma unroll
      for (int i = 0; i < P1; ++i) y[i] = B0[rrow + i];
      const Folded<P1, T> f0 = fold(y);
      if constexpr (!STIFF) {
        Unfold<P1, T> z;
        z.zero();
#pragma unroll
        for (int a = 0; a < EO::ROWS; ++a) {
          const bool pair = a < EO::HO;
          T xa, xb;
          eo_row<Q, P1, 1>(tJ, a, f0, xa, xb);
          const T va = g[0][a] * xa;
          const T vb = pair ? g[0][Q - 1 - a] * xb : T(0);
          if (live) en += (double)xa * (double)va + (pair ? (double)xb * (double)vb : 0.0);
          z.template add<Q, 1>(tJ, a, va, vb);
        }
        z.get(y);
#pragma unroll
        for (int i = 0; i < P1; ++i) B0[rrow + i] = y[i];
      } else {
#pragma unroll
        for (int i = 0; i < P1; ++i) y[i] = B1[rrow + i];
        const Folded<P1, T> f1 = fold(y);
#pragma unroll
        for (int i = 0; i < P1; ++i) y[i] = B2[rrow + i];
        const Folded<P1, T> f2 = fold(y);
        T bq[HELM ? Q : 1];
        if constexpr (HELM) {
          const T *Be = Bb + ec * NQ + rl;
#pragma unroll
          for (int a = 0; a < Q; ++a) bq[a] = Be[a * QQ];
        }
        Unfold<P1, T> zp, zr, zt;
        if constexpr (!VST) {
          zp.zero();
          zr.zero();
          zt.zero();
        }
#pragma unroll
        for (int a = 0; a < EO::ROWS; ++a) {
          const bool pair = a < EO::HO;
          const int b = Q - 1 - a;
          T ra, rb, sa, sb, ta, tb;
          eo_row<Q, P1, -1>(tD, a, f0, ra, rb);
          eo_row<Q, P1, 1>(tJ, a, f1, sa, sb);
          eo_row<Q, P1, 1>(tJ, a, f2, ta, tb);
          const T vra = g[0][a] * ra + g[1][a] * sa + g[2][a] * ta;
          const T vsa = g[1][a] * ra + g[3][a] * sa + g[4][a] * ta;
          const T vta = g[2][a] * ra + g[4][a] * sa + g[5][a] * ta;
          T vrb = 0, vsb = 0, vtb = 0;
          if (pair) {
            vrb = g[0][b] * rb + g[1][b] * sb + g[2][b] * tb;
            vsb = g[1][b] * rb + g[3][b] * sb + g[4][b] * tb;
            vtb = g[2][b] * rb + g[4][b] * sb + g[5][b] * tb;
          }
          if (live) {
            en += (double)ra * (double)vra + (double)sa * (double)vsa + (double)ta * (double)vta;
            if (pair)
              en += (double)rb * (double)vrb + (double)sb * (double)vsb + (double)tb * (double)vtb;
          }
          if constexpr (VST) {  // v at the points into the pencil's own rows
            B0[rrow + a] = vra;
            B1[rrow + a] = vsa;
            B2[rrow + a] = vta;
            if (pair) {
              B0[rrow + b] = vrb;
              B1[rrow + b] = vsb;
              B2[rrow + b] = vtb;
            }
          } else {
            zp.template add<Q, -1>(tD, a, vra, vrb);
            zr.template add<Q, 1>(tJ, a, vsa, vsb);
            zt.template add<Q, 1>(tJ, a, vta, vtb);
          }
          if constexpr (HELM) {
            T xa, xb;
            eo_row<Q, P1, 1>(tJ, a, f0, xa, xb);
            const T wa = bq[a] * xa;
            const T wb = pair ? bq[b] * xb : T(0);
            if (live) en += (double)xa * (double)wa + (pair ? (double)xb * (double)wb : 0.0);
            zp.template add<Q, 1>(tJ, a, wa, wb);
          }
        }
        if constexpr (VST) {
          zp.zero();
          zr.zero();
          zt.zero();
#pragma unroll
          for (int a = 0; a < EO::ROWS; ++a) {
            const bool pair = a < EO::HO;
            const int b = Q - 1 - a;
            zp.template add<Q, -1>(tD, a, B0[rrow + a], pair ? B0[rrow + b] : T(0));
            zr.template add<Q, 1>(tJ, a, B1[rrow + a], pair ? B1[rrow + b] : T(0));
            zt.template add<Q, 1>(tJ, a, B2[rrow + a], pair ? B2[rrow + b] : T(0));
          }
        }
        zp.get(y);
#pragma unroll
        for (int i = 0; i < P1; ++i) B0[rrow + i] = y[i];
        zr.get(y);
#pragma unroll
        for (int i = 0; i < P1; ++i) B1[rrow + i] = y[i];
        zt.get(y);
#pragma unroll
        for (int i = 0; i < P1; ++i) B2[rrow + i] = y[i];
      }
    }
    __syncthreads();
    if constexpr (PREF) {  // unconditional (the last component re-reads its own)
      const T *un_src = u + (cc + 1 < nrun ? cc + 1 : cc) * cs;
#pragma unroll
      for (int k = 0; k < P1; ++k) un[k] = un_src[gk[k]];
    }
    // 4: back along s (pencil (i, c) = lane l), into the A tiles in place
    if (spn) {
      const int ob = (l / P1) * RS + l % P1;
      Unfold<P1, T> s1, s2;
      s1.zero();
      if constexpr (STIFF) s2.zero();
#pragma unroll
      for (int b = 0; b < EO::ROWS; ++b) {
        const bool pair = b < EO::HO;
        const int bm = (Q - 1 - b) * LB + ob;
        s1.template add<Q, 1>(tJ, b, B0[b * LB + ob], pair ? B0[bm] : T(0));
        if constexpr (STIFF) {
          s1.template add<Q, -1>(tD, b, B1[b * LB + ob], pair ? B1[bm] : T(0));
          s2.template add<Q, 1>(tJ, b, B2[b * LB + ob], pair ? B2[bm] : T(0));
        }
      }
      T z[P1];
      s1.get(z);
#pragma unroll
      for (int j = 0; j < P1; ++j) A0[j * LA + l] = z[j];
      if constexpr (STIFF) {
        s2.get(z);
#pragma unroll
        for (int j = 0; j < P1; ++j) A1[j * LA + l] = z[j];
      }
    }
    __syncthreads();
    // 5: back along t and scatter
    if (col) {
      const T *a0 = A0 + cj * LA + ci;
      const T *a1 = A1 + cj * LA + ci;
      Unfold<P1, T> wz;
      wz.zero();
#pragma unroll
      for (int c = 0; c < EO::ROWS; ++c) {
        const bool pair = c < EO::HO;
        wz.template add<Q, 1>(tJ, c, a0[c * P1], pair ? a0[(Q - 1 - c) * P1] : T(0));
        if constexpr (STIFF)
          wz.template add<Q, -1>(tD, c, a1[c * P1], pair ? a1[(Q - 1 - c) * P1] : T(0));
      }
      T wk[P1];
      wz.get(wk);
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        if constexpr (LOCAL) {  // element-local output, one lane per entry: no assembly
          if (mb >> k & 1u) wc[gk[k]] = wk[k];
        } else if constexpr (WL) {
          // w_L of the element (0 at skipped nodes); the caller applies Q^T
          if (live) wc[ec * N3 + ci + P1 * (cj + P1 * k)] = (mb >> k & 1u) ? wk[k] : T(0);
        } else if (mb >> k & 1u) {
          if (own && interior_node<P1>(ci, cj, k))
            __builtin_nontemporal_store(wk[k], wc + gk[k]);  // a node of this element alone
          else
            atomic_add(wc + gk[k], wk[k]);
        }
      }
    }
    double enb[1] = {en};
    if (part)
      block_sum_store<1, PL::THREADS>(enb, part + (int64_t)blockIdx.x * ncomp + (MULTI ? cc : c0),
                                      1);
  }
}

template <int P1, int Q, typename T, int MODE, bool LOCAL = false, bool WL = false>
__global__ __launch_bounds__((GLPlane<P1, Q, MODE>::THREADS), 2) void k_op_gl(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Gm,
    const T *__restrict__ Bb, const T *__restrict__ basis, const T *__restrict__ u,
    T *__restrict__ w, int ncomp, int c0, int masked, double *__restrict__ part,
    const int *__restrict__ done, int own) {
  gl_body<P1, Q, T, MODE, LOCAL, WL, false>(nelem, idx, Gm, Bb, basis, u, w, 0, 0, ncomp, c0,
                                            masked, part, done, own);
}

template <int P1, int Q, typename T, int MODE, bool LOCAL = false, bool WL = false>
__global__ __launch_bounds__((GLPlane<P1, Q, MODE>::THREADS), 2) void k_op_gl_nc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Gm,
    const T *__restrict__ Bb, const T *__restrict__ basis, const T *__restrict__ u,
    T *__restrict__ w, int64_t cs, int64_t ws, int ncomp, int masked, double *__restrict__ part,
    const int *__restrict__ done, int own) {
  gl_body<P1, Q, T, MODE, LOCAL, WL, true>(nelem, idx, Gm, Bb, basis, u, w, cs, ws, ncomp, 0,
                                           masked, part, done, own);
}

// ---------------------------------------------------------------------------
// Geometric factors of eq. (gij) and B~ of eq. (mass) at set-up, one
// work-group per element (grid-stride over elements). The element's node
// coordinates are interpolated to the quadrature points with J^ along i, j
// and k (nothing to do with collocated GLL points), the derivatives
// dx_l/dr_m are taken there with D~ (exact: x is a polynomial of degree p < q
// in each variable), and the inverse Jacobian comes from the cofactor matrix:
// G_mm' = sum_l cof_lm cof_lm' w / det and B~ = det w, w the product of the
// 1D weights. Gauss-Legendre operators store the point index reversed
// ([a][b][c], c fastest; the layout their kernel reads coalesced). `bad`
// receives the smallest element index with det <= 0 (or non-finite) at some
// point. Dynamic LDS (interpolating rules only): two regions, A (coordinates,
// then the j-pass) and B (the i-pass, then the coordinates at the points);
// with collocated GLL points the derivatives are taken straight from the
// coordinate array. basis: J^ (q x p1) | D^ (q x p1) | D~ (q x q) | 1D weights (q).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_geometry(int64_t nelem, int p1, int q, int colloc,
                                                  const double *__restrict__ X,
                                                  const double *__restrict__ basis,
                                                  double *__restrict__ G,
                                                  double *__restrict__ Bt, int *__restrict__ bad) {
  extern __shared__ double gsm[];
  const int n3 = p1 * p1 * p1, nq = q * q * q;
  const int ra = 3 * (n3 > p1 * q * q ? n3 : p1 * q * q);
  double *A = gsm, *B = gsm + ra;
  const double *J = basis, *Dq = basis + 2 * q * p1, *rho = basis + 2 * q * p1 + q * q;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int64_t e = blockIdx.x; e < nelem; e += gridDim.x) {
    const double *Xq = X + e * 3 * n3;  // collocated: the nodes are the points
    if (!colloc) {
      for (int x = t; x < 3 * n3; x += nt) A[x] = Xq[x];
      __syncthreads();
      // along i: B[k][j][a][l] = sum_i J^[a][i] X[k][j][i][l]
      for (int x = t; x < 3 * p1 * p1 * q; x += nt) {
        const int l = x % 3, a = (x / 3) % q, kj = x / (3 * q);
        double sum = 0.0;
        for (int i = 0; i < p1; ++i) sum += J[a * p1 + i] * A[(kj * p1 + i) * 3 + l];
        B[x] = sum;
      }
      __syncthreads();
      // along j: A[k][b][a][l] = sum_j J^[b][j] B[k][j][a][l]
      for (int x = t; x < 3 * p1 * q * q; x += nt) {
        const int l = x % 3, a = (x / 3) % q, bq = (x / (3 * q)) % q, k = x / (3 * q * q);
        double sum = 0.0;
        for (int j = 0; j < p1; ++j) sum += J[bq * p1 + j] * B[((k * p1 + j) * q + a) * 3 + l];
        A[x] = sum;
      }
      __syncthreads();
      // along k: B[c][b][a][l] = sum_k J^[c][k] A[k][b][a][l]
      for (int x = t; x < 3 * nq; x += nt) {
        const int l = x % 3, ba = (x / 3) % (q * q), c = x / (3 * q * q);
        double sum = 0.0;
        for (int k = 0; k < p1; ++k) sum += J[c * p1 + k] * A[(k * q * q + ba) * 3 + l];
        B[x] = sum;
      }
      __syncthreads();
      Xq = B;
    }
    for (int n = t; n < nq; n += nt) {
      const int a = n % q, bq = (n / q) % q, c = n / (q * q);
      double M[3][3];  // M[l][m] = dx_l / dr_m
      for (int l = 0; l < 3; ++l) {
        double dr = 0.0, ds = 0.0, dt = 0.0;
        for (int m = 0; m < q; ++m) {
          dr += Dq[a * q + m] * Xq[((c * q + bq) * q + m) * 3 + l];
          ds += Dq[bq * q + m] * Xq[((c * q + m) * q + a) * 3 + l];
          dt += Dq[c * q + m] * Xq[((m * q + bq) * q + a) * 3 + l];
        }
        M[l][0] = dr;
        M[l][1] = ds;
        M[l][2] = dt;
      }
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
      if (!(det > 0.0) || !isfinite(det)) atomicMin(bad, (int)e);
      const double wq = rho[a] * rho[bq] * rho[c];
      const double sc = wq / det;
      const int ns = colloc ? n : (a * q + bq) * q + c;  // stored point index
      int comp = 0;
      for (int m = 0; m < 3; ++m)
        for (int mp = m; mp < 3; ++mp) {
          double g = 0.0;
          for (int l = 0; l < 3; ++l) g += cof[l][m] * cof[l][mp];
          G[(e * 6 + comp) * nq + ns] = g * sc;
          ++comp;
        }
      Bt[e * nq + ns] = det * wq;
    }
    __syncthreads();  // the regions are rewritten for the next element
  }
}

// ---------------------------------------------------------------------------
// Diagonal of the assembled operator (Jacobi preconditioner, section 3).
// diag(A^e)_{ijk} = sum_{mm'} sum_{abc} G_mm'(a,b,c) phi_m phi_m' with
// phi_1 = D[a][i] J[b][j] J[c][k], phi_2 = J[a][i] D[b][j] J[c][k],
// phi_3 = J[a][i] J[b][j] D[c][k]; mass: sum B~ J[a][i]^2 J[b][j]^2 J[c][k]^2.
// Sum-factorised per element (contract a, then b, then c), scatter-added.
// Runtime sizes; dynamic LDS of q^3 + q^2 p1 + q p1^2 + p1^3 + 2 q p1 values.
// rev: the quadrature data are stored with the point index reversed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag(int64_t nelem, int p1, int q, int stiff,
                                              const int32_t *__restrict__ idx,
                                              const double *__restrict__ Gm,
                                              const double *__restrict__ basis,
                                              double *__restrict__ d, int masked, int rev) {
  extern __shared__ double dsm[];
  const int q3 = q * q * q, n3 = p1 * p1 * p1;
  double *sg = dsm;                // [c][b][a]      q^3
  double *t1 = sg + q3;            // [c][b][i]      q^2 p1
  double *t2 = t1 + q * q * p1;    // [c][j][i]      q p1^2
  double *sd = t2 + q * p1 * p1;   // [k][j][i]      p1^3
  double *sJ = sd + n3;            // q x p1
  double *sD = sJ + q * p1;        // q x p1
  const int t = threadIdx.x, nt = blockDim.x;
  for (int x = t; x < q * p1; x += nt) {
    sJ[x] = basis[x];
    sD[x] = basis[q * p1 + x];
  }
  const int nterms = stiff ? 6 : 1;
  const int pm[6] = {0, 0, 0, 1, 1, 2}, pn[6] = {0, 1, 2, 1, 2, 2};
  // elements in a grid-stride loop (the grid is capped on the host)
  for (int64_t e = blockIdx.x; e < nelem; e += gridDim.x) {
    for (int x = t; x < n3; x += nt) sd[x] = 0.0;
    __syncthreads();
    for (int term = 0; term < nterms; ++term) {
      const double *src = stiff ? Gm + (e * 6 + term) * q3 : Gm + e * q3;
      for (int x = t; x < q3; x += nt)
        sg[x] = src[rev ? (x % q * q + x / q % q) * q + x / (q * q) : x];
      const int m0 = stiff ? pm[term] : -1, m1 = stiff ? pn[term] : -1;
      const double fac = (stiff && m0 != m1) ? 2.0 : 1.0;
      __syncthreads();
      // direction dir uses F(m0,dir) * F(m1,dir), F = D if m == dir else J
      for (int x = t; x < q * q * p1; x += nt) {
        const int i = x % p1, bb = (x / p1) % q, c = x / (p1 * q);
        double s = 0.0;
        for (int a = 0; a < q; ++a) {
          const double f0 = (m0 == 0 ? sD : sJ)[a * p1 + i];
          const double f1 = (m1 == 0 ? sD : sJ)[a * p1 + i];
          s += f0 * f1 * sg[(c * q + bb) * q + a];
        }
        t1[x] = s;
      }
      __syncthreads();
      for (int x = t; x < q * p1 * p1; x += nt) {
        const int i = x % p1, j = (x / p1) % p1, c = x / (p1 * p1);
        double s = 0.0;
        for (int bb = 0; bb < q; ++bb) {
          const double f0 = (m0 == 1 ? sD : sJ)[bb * p1 + j];
          const double f1 = (m1 == 1 ? sD : sJ)[bb * p1 + j];
          s += f0 * f1 * t1[(c * q + bb) * p1 + i];
        }
        t2[x] = s;
      }
      __syncthreads();
      for (int x = t; x < n3; x += nt) {
        const int i = x % p1, j = (x / p1) % p1, k = x / (p1 * p1);
        double s = 0.0;
        for (int c = 0; c < q; ++c) {
          const double f0 = (m0 == 2 ? sD : sJ)[c * p1 + k];
          const double f1 = (m1 == 2 ? sD : sJ)[c * p1 + k];
          s += f0 * f1 * t2[(c * p1 + j) * p1 + i];
        }
        sd[x] += fac * s;
      }
      __syncthreads();
    }
    for (int x = t; x < n3; x += nt) {
      const int v = idx[e * n3 + x];
      const int g = decode_index(v, true, masked);
      if (g >= 0) atomic_add(d + g, sd[x]);
    }
    __syncthreads();  // sd is cleared for the next element
  }
}

// ---------------------------------------------------------------------------
// Gradient with respect to the coefficient at the quadrature points
// (collocated GLL): g_q = - sum_c (D lam_c)_q^T G_q (D u_c)_q. The thread
// layout is that of the stiffness kernel: each lane owns an (i, j) column of
// an element and requests its G column and map once. Per component it takes
// the gradient of u (t in registers, r and s through one LDS tile) and forms
// v = G (D u) at its points, then the gradient of lam through the same tile
// and accumulates (D lam) . v, so only v, not both gradients, stays live.
// lam and u are masked on Dirichlet nodes (those read as 0).
// ---------------------------------------------------------------------------
template <int P1>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_grad_kappa_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const double *__restrict__ G,
    const double *__restrict__ lam, const double *__restrict__ u, double *__restrict__ gout,
    int64_t cstride, int ncomp) {
  using PL = Plane<P1, P1>;
  constexpr int N3 = P1 * P1 * P1, PP = P1 * P1, PAD = P1 + 1;
  static constexpr GLLDeriv<P1, double> kD{};  // D^[a][m] at a * p1 + m, compile-time
  const double *const Dg = kD.D;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ij = t % PL::N;
  const int i = ij % P1, j = ij / P1;
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  const bool live = act && e < nelem;
  const int64_t ec = live ? e : nelem - 1;  // element whose data the lane reads
  __shared__ double sD[P1][PAD];
  __shared__ double sx[PL::EPB][P1][P1][PAD];
  for (int x = t; x < PP; x += PL::THREADS) sD[x / P1][x % P1] = Dg[x];
  int gk[P1];
  double g[6][P1];
  unsigned mb = 0;  // bit k: node k is read (live and not a Dirichlet node)
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = idx[ec * N3 + ij + k * PP];
    if (live && v >= 0) mb |= 1u << k;
    gk[k] = v >= 0 ? v : -1 - v;
  }
#pragma unroll
  for (int k = 0; k < P1; ++k)
#pragma unroll
    for (int n = 0; n < 6; ++n) g[n][k] = G[ec * 6 * N3 + n * N3 + k * PP + ij];
  double acc[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k) acc[k] = 0.0;
#pragma unroll 1
  for (int c = 0; c < ncomp; ++c) {
    double vr[P1], vs[P1], vt[P1];
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const double *x = (pass == 0 ? u : lam) + c * cstride;
      double r[P1], rt[P1];
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        const double val = x[gk[k]];
        r[k] = (mb >> k & 1u) ? val : 0.0;
      }
      __syncthreads();  // the tile's previous contents have been read
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        if (act) sx[slot][k][j][i] = r[k];
        double a = 0.0;
#pragma unroll
        for (int m = 0; m < P1; ++m) a += Dg[k * P1 + m] * r[m];
        rt[k] = a;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        double dr = 0.0, ds = 0.0;
#pragma unroll
        for (int m = 0; m < P1; ++m) {
          dr += sD[i][m] * sx[slot][k][j][m];
          ds += sD[j][m] * sx[slot][k][m][i];
        }
        if (pass == 0) {
          vr[k] = g[0][k] * dr + g[1][k] * ds + g[2][k] * rt[k];
          vs[k] = g[1][k] * dr + g[3][k] * ds + g[4][k] * rt[k];
          vt[k] = g[2][k] * dr + g[4][k] * ds + g[5][k] * rt[k];
        } else {
          acc[k] += dr * vr[k] + ds * vs[k] + rt[k] * vt[k];
        }
      }
    }
  }
  if (live)
#pragma unroll
    for (int k = 0; k < P1; ++k) gout[e * N3 + k * PP + ij] = -acc[k];
}

}  // namespace bp
