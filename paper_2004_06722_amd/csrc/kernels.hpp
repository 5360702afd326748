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

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bp {

// Thread plane of an element: M x M threads, M = max(p1, q); EPB elements per
// work-group so that small orders still fill a wave; THREADS rounded up to
// whole waves (idle lanes take part in barriers and reductions only).
template <int P1, int Q>
struct Plane {
  static constexpr int M = P1 > Q ? P1 : Q;
  static constexpr int N = M * M;
  static constexpr int EPB = N >= 64 ? 1 : 64 / N;
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

// Work-group barrier that also stops the instruction scheduler from moving
// work across it. With one-wave work-groups the compiler drops s_barrier
// (LDS accesses of a wave are ordered), and without the scheduling fence it
// would hoist the LDS reads of every plane at once and run out of registers.
// The memory clobber also makes the compiler re-read the lane-dependent
// rows of D^ from LDS in every plane instead of keeping them all live.
__device__ __forceinline__ void plane_sync() {
  __syncthreads();
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Decoded gather index: global id, or -1 when the node is skipped
// (element slot not live, or a Dirichlet node under the mask).
__device__ __forceinline__ int decode_index(int v, bool live, int masked) {
  if (!live) return -1;
  if (v >= 0) return v;
  return masked ? -1 : -1 - v;
}

// ---------------------------------------------------------------------------
// BK5/BK6: stiffness with collocated GLL quadrature (J^ = I, q = p1).
// One component per launch: u and w point at component c0 (vectors are
// component-major, [ncomp][nglobal]); ncomp and c0 place the energy partial. Keeping
// the G column in registers across several components doubles the register
// footprint and halves occupancy, which costs more than re-reading G.
//
// The kernel is bound by HBM latency more than by arithmetic, so it is laid
// out to need few dependent round trips: each lane requests its whole column
// of G (6 x p1 values, GPRE planes of them at entry when GPRE = p1) and of
// the gather map at once, then gathers u, then computes from registers and
// LDS. The k direction stays in registers; the r and s contractions go
// through LDS tiles. Loads are branch-free: an element slot past the end
// reads the last element and a Dirichlet node reads its (valid) global
// entry, both masked. Entries of D^ with compile-time indices
// are scalar loads from Dg (global memory, D^[a][m] at a * p1 + m); the
// lane-dependent rows come from LDS. The local energy u_L^T A_L u_L is
// accumulated at the quadrature points as (D u)^T G (D u) = u_L^T w_L.
// HELM adds the Helmholtz term of eq. (hm2): with collocated GLL points the
// mass matrix is diagonal, so w_L += (beta B~) u_L node by node, with the
// beta-scaled B~ read beside G (one more word per point).
// ---------------------------------------------------------------------------
template <int P1, typename T, bool LOCAL = false, bool HELM = false>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_stiff_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ G, const T *Dg,
    const T *__restrict__ Bb, const T *__restrict__ u, T *__restrict__ w, int ncomp, int c0,
    int masked, double *__restrict__ part, const int *__restrict__ done) {
  constexpr int NC = 1;  // one component per launch; G is re-read per component
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

  // gather u (requested before D^ is staged, so both wait together)
  T ru[NC][P1];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      const T v = u[gk[k]];
      ru[c][k] = (mb >> k & 1u) ? v : T(0);
    }
  for (int x = t; x < PP; x += PL::THREADS) {
    sD[x / P1][x % P1] = Dg[x];
    sDt[x % P1][x / P1] = Dg[x];
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
        if constexpr (LOCAL)
          w[gk[k]] = acc;  // element-local output: no assembly
        else
          atomic_add(w + gk[k], acc);
      }
    }
  }
  if (part) block_sum_store<NC, PL::THREADS>(en, part + (int64_t)blockIdx.x * ncomp + c0, 1);
}

// ---------------------------------------------------------------------------
// Mass with collocated GLL quadrature: B_L is diagonal (section 5, remark
// after eq. (mass)); w = Q^T (B~ .* Q u).
// ---------------------------------------------------------------------------
template <int P1, typename T, bool LOCAL = false>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_mass_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Bt,
    const T *__restrict__ u, T *__restrict__ w, int64_t cstride, int ncomp, int masked,
    double *__restrict__ part, const int *__restrict__ done) {
  using PL = Plane<P1, P1>;
  constexpr int N3 = P1 * P1 * P1;
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ij = t % PL::N;
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
      if constexpr (LOCAL)
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
// Thread (a, b) of a q x q plane owns the quadrature column (a, b, .) and
// keeps it in registers, so every contraction along t is register-only; the
// r and s contractions go through padded LDS tiles. Lanes with a, b < p1
// also own node column (a, b, .) for the gather and the scatter.
// Stiffness (section 5, eq. (gradr2)-(gradt2) with shared partial sums):
//   u_t = J^_t u, then J^_s and D^_s of it, then J^_r and D^_r of those give
//   the interpolated values x, u_r and u_s; u_t = D~_t x along the column,
// where D^ = D~ J^ is the derivative of the nodal basis at the Gauss points.
// Then v = G (u_r, u_s, u_t) and the transposed chain back to the nodes.
// Mass: J^ along t, s, r, then B~, then J^T along r, s, t.
// Several elements share a work-group of up to 256 threads so that few lanes
// idle; the G (or B~) column and the gather map are requested at entry. The
// local energy is accumulated at the quadrature points. One component per
// launch (u and w point at component c0): keeping G live across a loop over
// components would cost the registers that the later stages reuse. With
// LOCAL the result is stored per element (added to w when accum is set).
// ---------------------------------------------------------------------------
// Scheduling fence between the quadrature levels of a stage: without it the
// scheduler issues the LDS reads of every level at once and the lane runs out
// of registers (the values already loaded, such as basis rows, stay live).
__device__ __forceinline__ void level_fence() { __builtin_amdgcn_sched_barrier(0); }

// Materialise a value where it is computed: the compiler may not sink its
// arithmetic to a later use and keep all the loaded inputs live instead.
__device__ __forceinline__ double pin(double v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ float pin(float v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

// VS: at q = 8 and q = 10 the stiffness kernel parks v_s in a fourth LDS
// tile instead of registers (the register file would otherwise spill); the
// larger LDS footprint then takes fewer elements per work-group.
template <int Q, bool STIFF>
struct QPlane {
  static constexpr bool VS = STIFF && (Q == 8 || Q == 10);
  static constexpr int NT = STIFF ? (VS ? 4 : 3) : 2;  // LDS tiles per element
  static constexpr int N = Q * Q;
  static constexpr int EPB = VS ? (Q == 8 ? 3 : 1) : (N >= 256 ? 1 : 256 / N);
  static constexpr int USED = EPB * N;
  static constexpr int THREADS = ((USED + 63) / 64) * 64;
};

template <int P1, int Q, typename T, bool STIFF, bool LOCAL = false>
__global__ __launch_bounds__((QPlane<Q, STIFF>::THREADS), 2) void k_op_interp(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Gm,
    const T *__restrict__ basis, const T *__restrict__ u, T *__restrict__ w, int ncomp, int c0,
    int masked, int accum, double *__restrict__ part, const int *__restrict__ done) {
  using PL = QPlane<Q, STIFF>;
  constexpr int N3 = P1 * P1 * P1, NQ = Q * Q * Q, QQ = Q * Q;
  constexpr int RP = Q + 1;       // tile row: q entries and one pad entry
  constexpr int TS = QQ * RP;     // tile [c][b][0..RP)
  constexpr int NG = STIFF ? 6 : 1;
  constexpr int NT = PL::NT;
  static_assert(Q == P1 + 1, "interpolating kernel expects q = p1 + 1");
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  // Lanes past the last plane act as column a = q of plane 0: their tile
  // stores land in the pad entries, which are never read, so no store needs
  // a guard. Columns a, b >= p1 of the node-indexed stages are written but
  // not read either.
  const int slot = act ? t / QQ : 0;
  const int a = act ? t % Q : Q;
  const int b = act ? (t % QQ) / Q : 0;
  const int ab = act ? t % QQ : 0;
  const int at = a < Q ? a : Q - 1;         // row of the basis tables
  const int ic = a < P1 ? a : P1 - 1;       // node index along r (clamped)
  const int jc = b < P1 ? b : P1 - 1;       // node index along s (clamped)
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  const bool live = act && e < nelem;
  const int64_t ec = live ? e : nelem - 1;  // element whose data the lane reads

  __shared__ T sJ[Q][P1];  // J^[a][i]
  __shared__ T sD[Q][P1];  // D^[a][i]
  __shared__ T tile[PL::EPB][NT][TS];
  T *const A = tile[slot][0];
  T *const B = tile[slot][1];
  T *const C = tile[slot][STIFF ? 2 : 1];  // third tile (stiffness only)
  T *const V = tile[slot][NT - 1];         // v_s: fourth tile with PL::VS, else B
  const int row = b * RP;           // offset of the lane's row in a level

  // one round trip: node column of the gather map, quadrature column of G / B~
  int gk[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k)
    gk[k] = LOCAL ? (int)(ec * N3) + ic + P1 * (jc + P1 * k) : idx[ec * N3 + ic + P1 * (jc + P1 * k)];
  T g[NG][Q];
  const T *Ge = Gm + ec * NG * NQ + ab;
#pragma unroll
  for (int c = 0; c < Q; ++c)
#pragma unroll
    for (int n = 0; n < NG; ++n) g[n][c] = __builtin_nontemporal_load(Ge + n * NQ + c * QQ);
  // bit k of mb: node k of the column is gathered and scattered
  unsigned mb = 0;
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = gk[k];
    if (live && a < P1 && b < P1 && (LOCAL || v >= 0 || !masked)) mb |= 1u << k;
    if (!LOCAL) gk[k] = v >= 0 ? v : -1 - v;
  }
  for (int x = t; x < Q * P1; x += PL::THREADS) {
    sJ[x / P1][x % P1] = basis[x];
    sD[x / P1][x % P1] = basis[Q * P1 + x];
  }
  const T *Jg = basis;               // J^[c][k] at c * P1 + k (uniform reads)
  const T *Dq = basis + 2 * Q * P1;  // D~[c][m] at c * Q + m

  {
    // gather; interpolate along t in registers: A[c][j][i] = sum_k J^[c][k] u(i, j, k)
    T uk[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      const T v = u[gk[k]];
      uk[k] = (mb >> k & 1u) ? v : T(0);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < P1; ++k) s += Jg[c * P1 + k] * uk[k];
      A[(c * Q) * RP + row + a] = s;
    }
    __syncthreads();
    // along s (lane (i, b)): B[c][b][i] = sum_j J^[b][j] A[c][j][i]; C with D^
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int j = 0; j < P1; ++j) {
        const T v = A[(c * Q + j) * RP + a];
        s0 += sJ[b][j] * v;
        if constexpr (STIFF) s1 += sD[b][j] * v;
      }
      B[(c * Q) * RP + row + a] = s0;
      if constexpr (STIFF) C[(c * Q) * RP + row + a] = s1;
      level_fence();
    }
    __syncthreads();
    // along r: the column's interpolated values x
    T x[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s0 = 0;
#pragma unroll
      for (int i = 0; i < P1; ++i) s0 += sJ[at][i] * B[(c * Q) * RP + row + i];
      x[c] = pin(s0);
      level_fence();
    }
    double en = 0.0;
    T S[Q];  // column after the transposed r and s contractions
    if constexpr (STIFF) {
      // per level: u_r, u_s along r, u_t along the column, G, energy;
      // v_r into A (free since the s stage), v_s and v_t kept for later
      T vsk[Q], vtk[Q];
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T r0 = 0, s0 = 0, ut = 0;
#pragma unroll
        for (int i = 0; i < P1; ++i) {
          r0 += sD[at][i] * B[(c * Q) * RP + row + i];
          s0 += sJ[at][i] * C[(c * Q) * RP + row + i];
        }
#pragma unroll
        for (int m = 0; m < Q; ++m) ut += Dq[c * Q + m] * x[m];
        const T vr = g[0][c] * r0 + g[1][c] * s0 + g[2][c] * ut;
        const T vs = g[1][c] * r0 + g[3][c] * s0 + g[4][c] * ut;
        const T vt = g[2][c] * r0 + g[4][c] * s0 + g[5][c] * ut;
        if (live) en += (double)r0 * (double)vr + (double)s0 * (double)vs + (double)ut * (double)vt;
        A[(c * Q) * RP + row + a] = vr;
        if constexpr (PL::VS)
          V[(c * Q) * RP + row + a] = vs;
        else
          vsk[c] = pin(vs);
        vtk[c] = pin(vt);
        level_fence();
      }
      // z = D~^T v_t along the column (values-space part of the t term)
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) s0 += Dq[m * Q + c] * vtk[m];
        x[c] = s0;
      }
      __syncthreads();  // B and C have been read
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        if constexpr (!PL::VS) B[(c * Q) * RP + row + a] = vsk[c];
        C[(c * Q) * RP + row + a] = x[c];
      }
      __syncthreads();
      // back along r (lane (i, b)): P = D^T v_r + J^T z, R = J^T v_s
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) {
          const int o = (c * Q) * RP + row + m;
          s0 += sD[m][ic] * A[o] + sJ[m][ic] * C[o];
          s1 += sJ[m][ic] * (PL::VS ? V[o] : B[o]);
        }
        vsk[c] = pin(s0);
        vtk[c] = pin(s1);
        level_fence();
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        A[(c * Q) * RP + row + a] = vsk[c];
        B[(c * Q) * RP + row + a] = vtk[c];
      }
      __syncthreads();
      // back along s (lane (i, j)): S = J^T P + D^T R
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) {
          const int o = (c * Q + m) * RP + ic;
          s0 += sJ[m][jc] * A[o] + sD[m][jc] * B[o];
        }
        S[c] = pin(s0);
        level_fence();
      }
    } else {
      // B~ at the points, energy; values into A (free since the s stage)
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const T v = g[0][c] * x[c];
        if (live) en += (double)x[c] * (double)v;
        A[(c * Q) * RP + row + a] = v;
      }
      __syncthreads();
      // back along r (lane (i, b)) into B (read before the last barrier)
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) s0 += sJ[m][ic] * A[(c * Q) * RP + row + m];
        B[(c * Q) * RP + row + a] = s0;
        level_fence();
      }
      __syncthreads();
      // back along s (lane (i, j))
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) s0 += sJ[m][jc] * B[(c * Q + m) * RP + ic];
        S[c] = pin(s0);
        level_fence();
      }
    }
    // back along t in registers and scatter: w(i, j, k) += sum_c J^[c][k] S[c]
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < Q; ++c) s += Jg[c * P1 + k] * S[c];
      if (mb >> k & 1u) {
        if constexpr (LOCAL)  // element-local output, one lane per entry: no assembly
          w[gk[k]] = accum ? w[gk[k]] + s : s;
        else
          atomic_add(w + gk[k], s);
      }
    }
    double enb[1] = {en};
    if (part) block_sum_store<1, PL::THREADS>(enb, part + (int64_t)blockIdx.x * ncomp + c0, 1);
  }
}

// ---------------------------------------------------------------------------
// Geometric factors of eq. (gij) and B~ of eq. (mass) at set-up, one
// work-group per element (grid-stride over elements). The element's node
// coordinates are interpolated to the quadrature points with J^ along i, j
// and k (nothing to do with collocated GLL points), the derivatives
// dx_l/dr_m are taken there with D~ (exact: x is a polynomial of degree p < q
// in each variable), and the inverse Jacobian comes from the cofactor matrix:
// G_mm' = sum_l cof_lm cof_lm' w / det and B~ = det w, w the product of the
// 1D weights. `bad` receives the smallest element index with det <= 0 (or
// non-finite) at some point. Dynamic LDS: two regions, A (coordinates, then
// the j-pass) and B (the i-pass, then the coordinates at the points).
// basis: J^ (q x p1) | D^ (q x p1) | D~ (q x q) | 1D weights (q).
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
    for (int x = t; x < 3 * n3; x += nt) A[x] = X[e * 3 * n3 + x];
    __syncthreads();
    const double *Xq = A;
    if (!colloc) {
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
      int comp = 0;
      for (int m = 0; m < 3; ++m)
        for (int mp = m; mp < 3; ++mp) {
          double g = 0.0;
          for (int l = 0; l < 3; ++l) g += cof[l][m] * cof[l][mp];
          G[(e * 6 + comp) * nq + n] = g * sc;
          ++comp;
        }
      Bt[e * nq + n] = det * wq;
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
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag(int64_t nelem, int p1, int q, int stiff,
                                              const int32_t *__restrict__ idx,
                                              const double *__restrict__ Gm,
                                              const double *__restrict__ basis,
                                              double *__restrict__ d, int masked) {
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
      for (int x = t; x < q3; x += nt) sg[x] = src[x];
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
// (collocated GLL): g_q = - sum_c (D lam_c)_q^T G_q (D u_c)_q.
// ---------------------------------------------------------------------------
template <int P1>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_grad_kappa_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const double *__restrict__ G,
    const double *__restrict__ basis, const double *__restrict__ lam,
    const double *__restrict__ u, double *__restrict__ gout, int64_t cstride, int ncomp) {
  using PL = Plane<P1, P1>;
  constexpr int N3 = P1 * P1 * P1, PAD = P1 + 1;
  __shared__ double sD[P1][P1];
  __shared__ double sl[PL::EPB][P1][P1][PAD];
  __shared__ double su[PL::EPB][P1][P1][PAD];
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ij = t % PL::N;
  const int i = ij % P1, j = ij / P1;
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  const bool live = act && e < nelem;
  for (int x = t; x < P1 * P1; x += PL::THREADS) sD[x / P1][x % P1] = basis[P1 * P1 + x];
  int gk[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = live ? idx[e * N3 + i + P1 * (j + P1 * k)] : -1;
    gk[k] = decode_index(v, live, 1);
  }
  double acc[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k) acc[k] = 0.0;
  for (int c = 0; c < ncomp; ++c) {
    double rl[P1], rv[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      rl[k] = gk[k] >= 0 ? lam[gk[k] + c * cstride] : 0.0;
      rv[k] = gk[k] >= 0 ? u[gk[k] + c * cstride] : 0.0;
      if (act) {
        sl[slot][k][j][i] = rl[k];
        su[slot][k][j][i] = rv[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      double lr = 0, ls = 0, lt = 0, ur = 0, us = 0, ut = 0;
#pragma unroll
      for (int m = 0; m < P1; ++m) {
        lr += sD[i][m] * sl[slot][k][j][m];
        ls += sD[j][m] * sl[slot][k][m][i];
        lt += sD[k][m] * rl[m];
        ur += sD[i][m] * su[slot][k][j][m];
        us += sD[j][m] * su[slot][k][m][i];
        ut += sD[k][m] * rv[m];
      }
      const double *Gq = G + (live ? e : 0) * 6 * N3 + k * P1 * P1 + ij;
      double g[6];
#pragma unroll
      for (int n = 0; n < 6; ++n) g[n] = live ? Gq[n * N3] : 0.0;
      acc[k] += lr * (g[0] * ur + g[1] * us + g[2] * ut) + ls * (g[1] * ur + g[3] * us + g[4] * ut) +
                lt * (g[2] * ur + g[4] * us + g[5] * ut);
    }
    __syncthreads();
  }
  if (live)
#pragma unroll
    for (int k = 0; k < P1; ++k) gout[e * N3 + k * P1 * P1 + ij] = -acc[k];
}

}  // namespace bp
