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
// entry, both scaled by a 0/1 mask. Entries of D^ with compile-time indices
// are scalar loads from Dg (global memory, D^[a][m] at a * p1 + m); the
// lane-dependent rows come from LDS. The local energy u_L^T A_L u_L is
// accumulated at the quadrature points as (D u)^T G (D u) = u_L^T w_L.
// ---------------------------------------------------------------------------
template <int P1, typename T>
__global__ __launch_bounds__((Plane<P1, P1>::THREADS)) void k_stiff_colloc(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ G, const T *Dg,
    const T *__restrict__ u, T *__restrict__ w, int ncomp, int c0, int masked,
    double *__restrict__ part, const int *__restrict__ done) {
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
  for (int k = 0; k < P1; ++k) gk[k] = __builtin_nontemporal_load(ie + k * PP);
#pragma unroll
  for (int k = 0; k < P1; ++k)
#pragma unroll
    for (int n = 0; n < 6; ++n) g[n][k] = __builtin_nontemporal_load(Ge + n * N3 + k * PP);

  // decode: global id and 0/1 mask (0 for dead slots and masked Dirichlet)
  T mk[P1];
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = gk[k];
    mk[k] = (live && (v >= 0 || !masked)) ? T(1) : T(0);
    gk[k] = v >= 0 ? v : -1 - v;
  }

  // gather u (requested before D^ is staged, so both wait together)
  T ru[NC][P1];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int k = 0; k < P1; ++k) ru[c][k] = u[gk[k]] * mk[k];
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
#pragma unroll
      for (int m = 0; m < P1; ++m) {
        acc += Dg[m * P1 + k] * rt[c][m];
        acc += sDt[i][m] * sr[slot][c][k][j][m];
        acc += sDt[j][m] * ss[slot][c][k][m][i];
      }
      if (mk[k] != T(0)) atomic_add(w + gk[k], acc);
    }
  }
  if (part) block_sum_store<NC, PL::THREADS>(en, part + (int64_t)blockIdx.x * ncomp + c0, 1);
}

// ---------------------------------------------------------------------------
// Mass with collocated GLL quadrature: B_L is diagonal (section 5, remark
// after eq. (mass)); w = Q^T (B~ .* Q u).
// ---------------------------------------------------------------------------
template <int P1, typename T>
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
    const int v = live ? idx[e * N3 + k * P1 * P1 + ij] : -1;
    gk[k] = decode_index(v, live, masked);
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
      atomic_add(w + o, wv);
    }
    if (part) block_sum_store<1, PL::THREADS>(en, part + (int64_t)blockIdx.x * ncomp + cc, 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BK1-BK4: Gauss-Legendre quadrature (q > p1). Interpolate to the quadrature
// points first (u~ = J u), differentiate there with the q x q matrix D~
// (section 5, eq. (gradr2)-(gradt2)), apply G (stiffness) or B~ (mass), and
// return with the transposed operations. Every stage is one 1D contraction
// between padded q x q x q LDS tiles, so a lane holds only one line of values
// at a time and registers stay free for the G column, which (with the gather
// map) is requested at entry. Thread (a, b) of the q x q plane owns the
// quadrature column (a, b, .); lanes with a, b < p1 also own node column
// (a, b, .). The local energy is accumulated at the quadrature points.
// ---------------------------------------------------------------------------
template <int P1, int Q, typename T, bool STIFF>
__global__ __launch_bounds__((Plane<P1, Q>::THREADS)) void k_op_interp(
    int64_t nelem, const int32_t *__restrict__ idx, const T *__restrict__ Gm,
    const T *__restrict__ basis, const T *__restrict__ u, T *__restrict__ w, int64_t cstride,
    int ncomp, int masked, double *__restrict__ part, const int *__restrict__ done) {
  using PL = Plane<P1, Q>;
  constexpr int N3 = P1 * P1 * P1, NQ = Q * Q * Q, QQ = Q * Q, QP = Q + 1;
  constexpr int NG = STIFF ? 6 : 1;
  constexpr int NT = STIFF ? 4 : 3;  // LDS tiles
  static_assert(Q > P1, "interpolating kernel expects q > p1");
  if (done && *done) return;
  const int t = threadIdx.x;
  const bool act = t < PL::USED;
  const int slot = act ? t / PL::N : 0;
  const int ab = t % PL::N;
  const int a = ab % Q, b = ab / Q;
  const int64_t e = (int64_t)blockIdx.x * PL::EPB + slot;
  if (PL::EPB == 1 && e >= nelem) return;  // uniform over the work-group
  const bool live = act && e < nelem;
  const int64_t ec = live ? e : nelem - 1;
  const bool own = live && a < P1 && b < P1;  // owns node column (i=a, j=b)

  __shared__ T sJ[Q][P1 + 1];   // sJ[a][i]  = J^[a][i]
  __shared__ T sJt[P1][QP];     // sJt[i][a] = J^[a][i]
  __shared__ T sDq[Q][QP];      // sDq[a][m] = D~[a][m]
  __shared__ T sDqt[Q][QP];     // sDqt[m][a] = D~[a][m]
  __shared__ T tile[NT][PL::EPB][Q][Q][QP];

  // one round trip: gather map (node columns) and G / B~ (quadrature columns)
  int gk[P1];
  T mk[P1];
  const int ia = a < P1 ? a : 0, jb = b < P1 ? b : 0;
#pragma unroll
  for (int k = 0; k < P1; ++k) gk[k] = idx[ec * N3 + ia + P1 * (jb + P1 * k)];
  T g[NG][Q];
  const T *Ge = Gm + ec * NG * NQ + ab;
#pragma unroll
  for (int c = 0; c < Q; ++c)
#pragma unroll
    for (int n = 0; n < NG; ++n) g[n][c] = __builtin_nontemporal_load(Ge + n * NQ + c * QQ);
#pragma unroll
  for (int k = 0; k < P1; ++k) {
    const int v = gk[k];
    mk[k] = (own && (v >= 0 || !masked)) ? T(1) : T(0);
    gk[k] = v >= 0 ? v : -1 - v;
  }
  for (int x = t; x < Q * P1; x += PL::THREADS) {
    const T v = basis[x];
    sJ[x / P1][x % P1] = v;
    sJt[x % P1][x / P1] = v;
  }
  for (int x = t; x < QQ; x += PL::THREADS) {
    const T v = basis[2 * Q * P1 + x];
    sDq[x / Q][x % Q] = v;
    sDqt[x % Q][x / Q] = v;
  }
  T(&A)[Q][Q][QP] = tile[0][slot];
  T(&B)[Q][Q][QP] = tile[1][slot];
  T(&C)[Q][Q][QP] = tile[2][slot];

  for (int comp = 0; comp < ncomp; ++comp) {
    // gather: A[k][j][i] = u
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      const T val = u[gk[k] + comp * cstride] * mk[k];
      if (act && a < P1 && b < P1) A[k][b][a] = val;
    }
    __syncthreads();
    // interpolate along r: B[k][j][a] = sum_i J[a][i] A[k][j][i]   (b plays j)
    if (act && b < P1)
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < P1; ++m) s += sJ[a][m] * A[k][b][m];
        B[k][b][a] = s;
      }
    __syncthreads();
    // along s: A[k][b][a] = sum_j J[b][j] B[k][j][a]
    if (act)
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < P1; ++m) s += sJ[b][m] * B[k][m][a];
        A[k][b][a] = s;
      }
    __syncthreads();
    // along t: B[c][b][a] = sum_k J[c][k] A[k][b][a]
    double en = 0.0;
    if (act) {
      T col[P1];
#pragma unroll
      for (int k = 0; k < P1; ++k) col[k] = A[k][b][a];
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < P1; ++k) s += sJ[c][k] * col[k];
        if constexpr (STIFF) {
          B[c][b][a] = s;
        } else {
          const T v = g[0][c] * s;  // B~ at the point
          en += (double)s * (double)v;
          B[c][b][a] = v;
        }
      }
    }
    __syncthreads();
    if constexpr (STIFF) {
      T(&Dt)[Q][Q][QP] = tile[3][slot];
      // derivatives at the quadrature points, G, into A (r), C (s), Dt (t)
      if (act)
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          T ur = 0, us = 0, ut = 0;
#pragma unroll
          for (int m = 0; m < Q; ++m) {
            ur += sDq[a][m] * B[c][b][m];
            us += sDq[b][m] * B[c][m][a];
            ut += sDq[c][m] * B[m][b][a];
          }
          const T vr = g[0][c] * ur + g[1][c] * us + g[2][c] * ut;
          const T vs = g[1][c] * ur + g[3][c] * us + g[4][c] * ut;
          const T vt = g[2][c] * ur + g[4][c] * us + g[5][c] * ut;
          en += (double)ur * (double)vr + (double)us * (double)vs + (double)ut * (double)vt;
          A[c][b][a] = vr;
          C[c][b][a] = vs;
          Dt[c][b][a] = vt;
        }
      __syncthreads();
      // transposed derivatives into B
      if (act)
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          T s = 0;
#pragma unroll
          for (int m = 0; m < Q; ++m) {
            s += sDqt[a][m] * A[c][b][m];
            s += sDqt[b][m] * C[c][m][a];
            s += sDqt[c][m] * Dt[m][b][a];
          }
          B[c][b][a] = s;
        }
      __syncthreads();
    }
    // transposed interpolation along t: A[k][b][a] = sum_c J[c][k] B[c][b][a]
    if (act) {
      T col[Q];
#pragma unroll
      for (int c = 0; c < Q; ++c) col[c] = B[c][b][a];
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < Q; ++c) s += sJt[k][c] * col[c];
        A[k][b][a] = s;
      }
    }
    __syncthreads();
    // along s: C[k][j][a] = sum_b J[b][j] A[k][b][a]
    if (act && b < P1)
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) s += sJt[b][m] * A[k][m][a];
        C[k][b][a] = s;
      }
    __syncthreads();
    // along r and scatter: w(i,j,k) = sum_a J[a][i] C[k][j][a]
    if (act && a < P1 && b < P1)
#pragma unroll
      for (int k = 0; k < P1; ++k) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) s += sJt[a][m] * C[k][b][m];
        if (mk[k] != T(0)) atomic_add(w + gk[k] + comp * cstride, s);
      }
    double enb[1] = {en};
    if (part) block_sum_store<1, PL::THREADS>(enb, part + (int64_t)blockIdx.x * ncomp + comp, 1);
    __syncthreads();
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
