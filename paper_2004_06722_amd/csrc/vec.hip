// Streaming vector kernels of the Jacobi-PCG iteration (section 3; section 8
// counts these updates as a few flops and memory words per DOF each) with
// deterministic reductions: every work-group writes its partial sums, a
// first stage folds them to at most 256 rows when there are many, and a
// single work-group adds the rows in a fixed order and updates alpha, beta
// and the convergence flag on the device, so the host never waits inside
// the iteration.
#include <cmath>

#include "bp_internal.h"
#include "launch.h"

namespace bp {

namespace {

constexpr int kFinThreads = 1024;

// Streaming access for the CG vectors when NT: each is touched once per
// kernel, and vectors larger than the last-level cache gain from the
// nontemporal hint (measured: 6.37 against 5.79 TB/s for the 3-read, 2-write
// direction update at 9e7 nodes); smaller ones lose by it (they are still
// cached when the next kernel reads them), so the launchers pick NT by size.
template <bool NT, typename T>
__device__ __forceinline__ T ld_v(const T *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_v(T *p, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
// vectors of at least this many bytes per component stream with NT
constexpr int64_t kStreamBytes = int64_t(64) << 20;

// Fixed-order sum of W columns over nb rows into res[col] (shared): thread t
// adds rows t, t + 1024, ... of every column in order (D loads in flight per
// column), each wave folds its 64 lanes with a fixed shuffle tree, and the
// first W threads add the 16 wave sums in order.
template <int W>
__device__ void reduce_columns(const double *__restrict__ part, int64_t nb, double *res) {
  constexpr int NW = kFinThreads / 64;
  constexpr int D = W <= 2 ? 8 : (W <= 6 ? 4 : 2);
  __shared__ double wsum[NW][W];
  double s[W];
#pragma unroll
  for (int c = 0; c < W; ++c) s[c] = 0.0;
  int64_t r = threadIdx.x;
  for (; r + (D - 1) * kFinThreads < nb; r += D * kFinThreads) {
    double v[D][W];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) v[q][c] = part[(r + q * kFinThreads) * W + c];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) s[c] += v[q][c];
  }
  for (; r < nb; r += kFinThreads)
#pragma unroll
    for (int c = 0; c < W; ++c) s[c] += part[r * W + c];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    double x = s[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) wsum[wid][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) x += wsum[k][threadIdx.x];
    res[threadIdx.x] = x;
  }
  __syncthreads();
}

// Stage 1 of the fixed-order reduction: work-group b adds rows
// [b * chunk, (b + 1) * chunk) of part[nb][width] into out[b][width].
__global__ __launch_bounds__(kVecThreads) void k_reduce_rows(const double *__restrict__ part,
                                                             int64_t nb, int width, int64_t chunk,
                                                             double *__restrict__ out) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < nb ? r0 + chunk : nb;
  __shared__ double sh[kVecThreads];
  for (int col = 0; col < width; ++col) {
    double s = 0.0;
    int64_t r = r0 + threadIdx.x;
    for (; r + 3 * kVecThreads < r1; r += 4 * kVecThreads) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = part[(r + q * kVecThreads) * width + col];
#pragma unroll
      for (int q = 0; q < 4; ++q) s += v[q];
    }
    for (; r < r1; r += kVecThreads) s += part[r * width + col];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = kVecThreads / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * width + col] = sh[0];
    __syncthreads();
  }
}

__device__ __forceinline__ bool converged(const DevScalars *sc, int nc) {
  bool ok = true;
  for (int c = 0; c < nc; ++c) {
    const double bb = sc->bb[c] > 0.0 ? sc->bb[c] : 1.0;
    ok = ok && (sc->rr[c] <= sc->tol2 * bb);
  }
  return ok;
}

// CG breakdown test: a step length alpha = num / den that is not positive
// (or not defined) while num = (r, z) is non-zero
__device__ __forceinline__ bool indefinite(double num, double den) {
  return num != 0.0 && (den == 0.0 || (num > 0.0) != (den > 0.0));
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_fill(T *x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kVecThreads)
    x[i] = v;
}

// The CG kernels run over a 2D grid: blockIdx.y is the component (vectors
// are component-major, [nc][n]) and work-group x covers nodes
// [256 x, 256 x + 256). A work-group writes its partial sum into row
// blockIdx.x, column (quantity * nc + component), of a [gridDim.x][q * nc]
// table; every entry is written by exactly one group.
//
// The iteration kernels give an FP32 thread two nodes of its group's 256
// (v and v + 128, 128 threads): a wave then has as many bytes in flight as
// an FP64 wave with one node per thread, and the partial tables keep one row
// per 256 nodes whatever the precision. The residual and direction updates
// of one component take two FP64 or four FP32 nodes per thread (their
// template parameter K; each 2% faster than one and two), those of several
// components two (the residual update up to four components);
// kNodesPerThread is the choice of the other kernels.
template <typename T>
constexpr int kNodesPerThread = sizeof(T) == 4 ? 2 : 1;
template <typename T>
constexpr int kGroupThreads = kVecThreads / kNodesPerThread<T>;
// Component c of a component-major vector starts (c n) mod 64 entries past a
// 64-entry boundary, so for n not a multiple of 64 a wave's 64 consecutive
// nodes of c > 0 straddle one more cache line than those of component 0
// (five 128-byte lines instead of four in FP64; measured on the
// three-component direction update at n = 337^3: 785 us against 718 us
// when realigned). The multi-component updates therefore shift the nodes of
// component c back by head = (c n) mod 64: slot s of the grid's span
// (gridDim.x * 256 >= n slots) takes node s - head, and the first head slots
// wrap round to the end of the span, so every node is still taken exactly
// once and the partial tables keep their rows.
__device__ __forceinline__ int64_t comp_head(int c, int64_t n) {
  return c ? ((int64_t)c * n) & 63 : 0;
}
__device__ __forceinline__ int64_t comp_node(int64_t slot, int64_t head) {
  const int64_t v = slot - head;
  return v < 0 ? v + (int64_t)gridDim.x * kVecThreads : v;
}

template <int TH = kVecThreads>
__device__ __forceinline__ void block_partial1(double v, double *part, int width, int col) {
  constexpr int NW = TH / 64;
  __shared__ double red[NW];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k];
    part[(int64_t)blockIdx.x * width + col] = s;
  }
  __syncthreads();
}

// r = b - w (w holds A x0), w = 0, p = z = dinv r; partials r.z, r.r, b.b.
// Entries of b on Dirichlet nodes are treated as zero. The iteration keeps
// the preconditioned residual z = dinv r (stored in `r`) rather than r: the
// residual update then advances z and the direction update reads z alone,
// ten vector words per DOF and iteration instead of eleven.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cg_init(int64_t n, const T *__restrict__ b,
                                                         T *__restrict__ r, T *__restrict__ w,
                                                         T *__restrict__ p,
                                                         const T *__restrict__ dinv,
                                                         double *__restrict__ part) {
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (v < n) {
    const int64_t f = comp * n + v;
    const T di = dinv[v];
    // dinv = 0 exactly on Dirichlet nodes: b is read as 0 there
    const bool free = di != T(0);
    const T bv = free ? b[f] : T(0);
    const T rv = free ? bv - w[f] : T(0);
    const T z = di * rv;
    r[f] = z;
    p[f] = z;
    w[f] = T(0);
    rz = (double)rv * (double)z;
    rr = (double)rv * (double)rv;
    bb = (double)bv * (double)bv;
  }
  block_partial1(rz, part, 3 * nc, comp);
  block_partial1(rr, part, 3 * nc, nc + comp);
  block_partial1(bb, part, 3 * nc, 2 * nc + comp);
}

template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_init(const double *__restrict__ part,
                                                          int64_t nb, DevScalars *sc) {
  constexpr int nc = NC;
  __shared__ double res[3 * NC];
  reduce_columns<3 * NC>(part, nb, res);
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int c = 0; c < nc; ++c) {
      sc->rz[c] = sc->rzs[0][c] = res[c];
      sc->rr[c] = res[nc + c];
      sc->bb[c] = res[2 * nc + c];
      sc->alpha[c] = sc->beta[c] = 0.0;
      bad |= !isfinite(res[c]) || !isfinite(res[nc + c]) || !isfinite(res[2 * nc + c]);
    }
    sc->iters = 0;
    sc->breakdown = 0;
    sc->nonfinite = bad;
    sc->done = bad || (!sc->fixed && converged(sc, nc));
    sc->halted = sc->done;  // x0 is already the answer
  }
}

template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_alpha(const double *__restrict__ part,
                                                           int64_t nb, DevScalars *sc, int check) {
  constexpr int nc = NC;
  if (check && sc->done) {
    if (threadIdx.x == 0) sc->halted = 1;
    return;
  }
  __shared__ double res[NC];
  reduce_columns<NC>(part, nb, res);
  if (threadIdx.x == 0) {
    int stop = 0;
    for (int c = 0; c < nc; ++c) {
      const double pap = res[c];
      sc->pap[c] = pap;
      sc->alpha[c] = pap != 0.0 ? sc->rz[c] / pap : 0.0;
      // alpha = (r.z) / (p.Ap) must be positive when r.z != 0: zero curvature
      // or curvature of the other sign than r.z means the preconditioned
      // operator is not definite on this Krylov space
      if (indefinite(sc->rz[c], pap)) {
        sc->breakdown = 1;
        stop = 1;
      }
      if (!isfinite(pap)) {
        sc->nonfinite = 1;
        stop = 1;
      }
    }
    // with a stopping test, end the solve here: the residual and solution
    // updates of this iteration are skipped, x keeps the last iterate
    if (check && stop) sc->done = sc->halted = 1;
  }
}

// z -= alpha dinv w (r -= alpha w on the stored z = dinv r); w = 0;
// partials r.z and r.r with r = z / dinv (0 on Dirichlet nodes, where
// dinv = 0). The matching x += alpha p is deferred to k_cg_update_xp, which
// reads p anyway: five vector words here and five there.
// check = 0 (a fixed number of iterations): no early exit on the done flag,
// so the loads do not wait for it (likewise in the other iteration kernels).
// Nodes below n_own are element-interior nodes in the internal order (see
// interior_first_order): the operator overwrites their w with plain stores,
// so w is cleared only from n_own on (likewise in k_sr_update).
template <typename T, bool NT, int K>
__global__ __launch_bounds__(kVecThreads / K) void k_cg_update_r(
    int64_t n, T *__restrict__ z, T *__restrict__ w, const T *__restrict__ dinv,
    double *__restrict__ part, const DevScalars *__restrict__ sc, int check, int64_t n_own) {
  constexpr int TH = kVecThreads / K;
  if (check && sc->done) return;
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const T al = (T)sc->alpha[comp];
  // all loads of the thread first, then the updates and stores
  T di[K], zo[K], wo[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    di[j] = zo[j] = wo[j] = T(0);
    if (v < n) {
      di[j] = ld_v<NT>(dinv + v);
      zo[j] = ld_v<NT>(z + comp * n + v);
      wo[j] = ld_v<NT>(w + comp * n + v);
    }
  }
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    if (v < n) {
      const int64_t f = comp * n + v;
      const T zv = zo[j] - (al * di[j]) * wo[j];
      st_v<NT>(z + f, zv);
      if (v >= n_own) st_v<NT>(w + f, T(0));
      const T rv = di[j] != T(0) ? zv / di[j] : T(0);
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  block_partial1<TH>(rz, part, 2 * nc, comp);
  block_partial1<TH>(rr, part, 2 * nc, nc + comp);
}

// Q^T w_L at one node: the sum of wc[pos[k]] over k in [k0, k1) in
// ascending order. The first four contributions are requested together and
// branch-free (two round trips: pos, then w_L; an index past the node's range
// is clamped to the last slot nl - 1 and its value dropped); a conforming
// hexahedral mesh gives every node 1, 2, 4 or 8, so only nodes shared by more
// than four elements go round the loop. Dropped values add an exact zero, so
// the order of the additions is that of the plain loop.
template <typename T>
__device__ __forceinline__ T gather_node(const T *__restrict__ wc,
                                         const int32_t *__restrict__ pos, int32_t k0,
                                         int32_t k1, int32_t last) {
  int32_t ps[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) ps[m] = pos[min(k0 + m, last)];
  T c[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) c[m] = wc[ps[m]];
  T acc = T(0);
#pragma unroll
  for (int m = 0; m < 4; ++m) acc += k0 + m < k1 ? c[m] : T(0);
  for (int32_t k = k0 + 4; k < k1; ++k) acc += wc[pos[k]];
  return acc;
}

// The same update with w = Q^T w_L formed per node from the element-local
// output of the mass kernel: w_v is the sum of wl[pos[k]] over
// k in [off[v], off[v+1]) in ascending order, a fixed order, so the result
// does not depend on scheduling as an atomic scatter does. No w vector is
// read, written or cleared; the pass reads z, dinv, the two offsets, and
// pos and w_L once per element-local slot.
template <typename T, bool NT>
__global__ __launch_bounds__(kGroupThreads<T>) void k_cg_update_r_gather(
    int64_t n, int64_t nl, T *__restrict__ z, const T *__restrict__ wl,
    const int32_t *__restrict__ off, const int32_t *__restrict__ pos,
    const T *__restrict__ dinv, double *__restrict__ part, const DevScalars *__restrict__ sc,
    int check) {
  constexpr int K = kNodesPerThread<T>, TH = kGroupThreads<T>;
  if (check && sc->done) return;
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const T al = (T)sc->alpha[comp];
  const T *wc = wl + comp * nl;
  T di[K], zo[K], wv[K];
  int32_t o0[K], o1[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    di[j] = zo[j] = wv[j] = T(0);
    o0[j] = o1[j] = 0;
    if (v < n) {  // the offsets first: the gather waits only for them
      o0[j] = off[v];
      o1[j] = off[v + 1];
      di[j] = ld_v<NT>(dinv + v);
      zo[j] = ld_v<NT>(z + comp * n + v);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) wv[j] = gather_node(wc, pos, o0[j], o1[j], (int32_t)(nl - 1));
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    if (v < n) {
      const T zv = zo[j] - (al * di[j]) * wv[j];
      st_v<NT>(z + comp * n + v, zv);
      const T rv = di[j] != T(0) ? zv / di[j] : T(0);
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  block_partial1<TH>(rz, part, 2 * nc, comp);
  block_partial1<TH>(rr, part, 2 * nc, nc + comp);
}

// Partial sums of W values over the work-group in a fixed order: row
// blockIdx.x of part[.][W] (one shuffle tree per wave, then the wave sums in
// order; one barrier for all W).
template <int W, int TH = kVecThreads>
__device__ __forceinline__ void block_partials(double (&v)[W], double *part) {
  constexpr int NW = TH / 64;
  __shared__ double red[NW][W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) x += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * W + threadIdx.x] = x;
  }
}

// The residual update for NC > 1 components: one thread per node for all
// of them, so dinv is read once per node (the component-per-row grid of
// k_cg_update_r reads it once per component). Partial columns as there:
// r.z of component c in column c, r.r in column NC + c.
template <typename T, bool NT, int NC, int K>
__global__ __launch_bounds__(kVecThreads / K) void k_cg_update_r_nc(
    int64_t n, T *__restrict__ z, T *__restrict__ w, const T *__restrict__ dinv,
    double *__restrict__ part, const DevScalars *__restrict__ sc, int check, int64_t n_own) {
  constexpr int TH = kVecThreads / K;
  if (check && sc->done) return;
  const int64_t s0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
  // component c takes node vc (shifted by comp_head); the nodes of one group
  // differ by less than 64 between components, so the extra dinv loads fall
  // on the cache lines component 0 brings in
  int64_t vc[K][NC];
  T di[K][NC], zo[K][NC], wo[K][NC];
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t v = vc[j][c] = comp_node(s0 + j * TH, comp_head(c, n));
      di[j][c] = zo[j][c] = wo[j][c] = T(0);
      if (v < n) {
        di[j][c] = ld_v<NT>(dinv + v);
        zo[j][c] = ld_v<NT>(z + c * n + v);
        wo[j][c] = ld_v<NT>(w + c * n + v);
      }
    }
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t v = vc[j][c];
      if (v < n) {
        const int64_t f = c * n + v;
        const T d = di[j][c];
        const T zv = zo[j][c] - ((T)sc->alpha[c] * d) * wo[j][c];
        st_v<NT>(z + f, zv);
        if (v >= n_own) st_v<NT>(w + f, T(0));
        const T rv = d != T(0) ? zv / d : T(0);
        acc[c] += (double)rv * (double)zv;
        acc[NC + c] += (double)rv * (double)rv;
      }
    }
  block_partials<2 * NC, TH>(acc, part);
}

// k_cg_update_r_gather for NC > 1 components: the node's offsets and slot
// positions are read once and each component gathers its w_L through them
// (the same fixed order per component).
template <typename T, bool NT, int NC>
__global__ __launch_bounds__(kVecThreads) void k_cg_update_r_gather_nc(
    int64_t n, int64_t nl, T *__restrict__ z, const T *__restrict__ wl,
    const int32_t *__restrict__ off, const int32_t *__restrict__ pos,
    const T *__restrict__ dinv, double *__restrict__ part, const DevScalars *__restrict__ sc,
    int check) {
  if (check && sc->done) return;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
  if (v < n) {
    const int32_t k0 = off[v], k1 = off[v + 1], last = (int32_t)(nl - 1);
    const T di = ld_v<NT>(dinv + v);
    T zo[NC], wv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) zo[c] = ld_v<NT>(z + c * n + v);
    int32_t ps[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) ps[m] = pos[min(k0 + m, last)];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T *wc = wl + c * nl;
      T cm[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) cm[m] = wc[ps[m]];
      T a = T(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) a += k0 + m < k1 ? cm[m] : T(0);
      wv[c] = a;
    }
    for (int32_t k = k0 + 4; k < k1; ++k) {
      const int32_t q = pos[k];
#pragma unroll
      for (int c = 0; c < NC; ++c) wv[c] += wl[c * nl + q];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T zv = zo[c] - ((T)sc->alpha[c] * di) * wv[c];
      st_v<NT>(z + c * n + v, zv);
      const T rv = di != T(0) ? zv / di : T(0);
      acc[c] = (double)rv * (double)zv;
      acc[NC + c] = (double)rv * (double)rv;
    }
  }
  block_partials<2 * NC>(acc, part);
}

// ---- the fused iteration of small meshes ----------------------------------
// With few partial rows every work-group of the residual update reduces the
// operator's partials itself, and every work-group of the direction update
// those of the residual update: each in the same fixed order (thread t adds
// rows t, t + 256, ...; a fixed shuffle tree per wave; the wave sums in
// order), so all work-groups hold bit-identical alpha and beta and the two
// single-work-group finishers of the standard iteration are not launched.
// Only work-group 0 writes the device scalars; nothing in a kernel reads a
// scalar that the same kernel writes (r.z by iteration parity: rzs).
template <int W>
__device__ __forceinline__ void block_reduce_rows(const double *__restrict__ part, int64_t nb,
                                                  double *res) {
  constexpr int NW = kVecThreads / 64;
  __shared__ double red[NW][W];
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  // rows t, t + 256, ... added in turn; the loads of four of them issued together
  constexpr int U = W <= 4 ? 4 : 2;
  int64_t r = threadIdx.x;
  for (; r + (U - 1) * kVecThreads < nb; r += U * kVecThreads) {
    double v[U][W];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) v[q][c] = part[(r + q * kVecThreads) * W + c];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] += v[q][c];
  }
  for (; r < nb; r += kVecThreads)
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] += part[r * W + c];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    double x = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) x += red[k][threadIdx.x];
    res[threadIdx.x] = x;
  }
  __syncthreads();
}

// z -= alpha dinv w for every component (one thread per node), alpha from
// the operator's partials pa[nba][NC] and r.z of this iteration (rz_old);
// partials of the new r.z and r.r into pr. A breakdown (see k_fin_alpha) or
// a non-finite p.Ap leaves z as it is in every work-group and, with a
// stopping test, ends the solve.
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_cg_update_r_fused(
    int64_t n, double *__restrict__ z, double *__restrict__ w, const double *__restrict__ dinv,
    const double *__restrict__ pa, int64_t nba, double *__restrict__ pr, DevScalars *sc,
    int parity, int check, int64_t n_own) {
  if (check && sc->done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->halted = 1;
    return;
  }
  // the node's vectors are requested first, so that they arrive while the
  // partial rows are reduced
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const bool in = v < n;
  double di = 0.0, zo[NC], wo[NC];
  if (in) {
    di = dinv[v];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      zo[c] = z[c * n + v];
      wo[c] = w[c * n + v];
    }
  }
  __shared__ double pap[NC];
  block_reduce_rows<NC>(pa, nba, pap);
  double al[NC];
  int bad = 0, brk = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double rz = sc->rzs[parity][c];
    al[c] = pap[c] != 0.0 ? rz / pap[c] : 0.0;
    brk |= indefinite(rz, pap[c]);
    bad |= !isfinite(pap[c]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < NC; ++c) {
      sc->pap[c] = pap[c];
      sc->alpha[c] = al[c];
    }
    if (brk) sc->breakdown = 1;
    if (bad) sc->nonfinite = 1;
    if (check && (brk || bad)) sc->done = sc->halted = 1;
  }
  if (check && (brk || bad)) return;
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
  if (in) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double zv = zo[c] - (al[c] * di) * wo[c];
      z[c * n + v] = zv;
      if (v >= n_own) w[c * n + v] = 0.0;
      const double rv = di != 0.0 ? zv / di : 0.0;
      acc[c] = rv * zv;
      acc[NC + c] = rv * rv;
    }
  }
  block_partials<2 * NC>(acc, pr);
}

// x += alpha p, then p = z + beta p unless the iteration converged; beta and
// the convergence test from the residual update's partials pr[nbv][2 NC] and
// r.z of this iteration; work-group 0 stores the new r.z into the other
// parity slot and updates the scalars the host polls.
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_cg_update_xp_fused(
    int64_t n, double *__restrict__ x, double *__restrict__ p, const double *__restrict__ z,
    const double *__restrict__ pr, int64_t nbv, DevScalars *sc, int parity, int check) {
  if (check && sc->halted) return;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const bool in = v < n;
  double pv[NC], xv[NC], zv[NC];
  if (in) {  // requested before the reduction, as in the residual update
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      pv[c] = p[c * n + v];
      xv[c] = x[c * n + v];
      zv[c] = z[c * n + v];
    }
  }
  __shared__ double res[2 * NC];
  block_reduce_rows<2 * NC>(pr, nbv, res);
  double al[NC], be[NC];
  bool conv = !sc->fixed;
  int bad = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double rzo = sc->rzs[parity][c], rzn = res[c], rr = res[NC + c];
    al[c] = sc->alpha[c];
    be[c] = rzo != 0.0 ? rzn / rzo : 0.0;
    const double bb = sc->bb[c] > 0.0 ? sc->bb[c] : 1.0;
    conv = conv && rr <= sc->tol2 * bb;
    bad |= !isfinite(rzn) || !isfinite(rr);
  }
  const bool dir = !(conv || bad);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < NC; ++c) {
      sc->rzs[parity ^ 1][c] = res[c];
      sc->rzp[c] = sc->rzs[parity][c];
      sc->rz[c] = res[c];
      sc->rr[c] = res[NC + c];
      sc->beta[c] = be[c];
    }
    sc->iters += 1;
    if (bad) sc->nonfinite = 1;
    if (!dir) sc->done = 1;
  }
  if (!in) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    x[c * n + v] = xv[c] + al[c] * pv[c];
    if (dir) p[c * n + v] = zv[c] + be[c] * pv[c];
  }
}

// The vector kernel of the two-launch iteration (PZIter): the operator has
// applied A to p_k = z_k + beta p_{k-1} and stored r_k.z_k into rzs[parity]
// and beta into sc->beta (iteration 0: p_0 = z_0, stored by the
// initialisation). alpha from the operator's partials pa[nba][NC]; per node
// p_k (stored), x += alpha p_k, z_{k+1} = z_k - alpha dinv w_k, w zeroed at
// the nodes the operator adds into (v >= n_own); partials of r_{k+1}.z_{k+1}
// and r_{k+1}.r_{k+1} into pr for the next operator launch, one row per
// K * 256 nodes (thread t takes nodes t, t + 256, ... of its group, added
// in that order): K = 1 on small meshes (more work-groups), kRxpNodes above
// 1024 rows, so that the table that every work-group of the operator reduces
// stays short. A breakdown or a non-finite p.Ap ends the
// solve as in k_cg_update_r_fused.
template <int NC, int K>
__global__ __launch_bounds__(kVecThreads) void k_cg_update_rxp_fused(
    int64_t n, double *__restrict__ x, double *__restrict__ p, double *__restrict__ z,
    double *__restrict__ w, const double *__restrict__ dinv, const double *__restrict__ pa,
    int64_t nba, double *__restrict__ pr, DevScalars *sc, int parity, int check, int first,
    int64_t n_own) {
  if (check && sc->done) return;  // x_k met the stopping test in the operator launch
  const int64_t v0 = (int64_t)blockIdx.x * (K * kVecThreads) + threadIdx.x;
  double di[K], zo[K][NC], wo[K][NC], po[K][NC], xo[K][NC];
#pragma unroll
  for (int j = 0; j < K; ++j) {  // requested before the reduction
    const int64_t v = v0 + j * kVecThreads;
    di[j] = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) zo[j][c] = wo[j][c] = po[j][c] = xo[j][c] = 0.0;
    if (v < n) {
      di[j] = dinv[v];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        zo[j][c] = z[c * n + v];
        wo[j][c] = w[c * n + v];
        po[j][c] = p[c * n + v];
        xo[j][c] = x[c * n + v];
      }
    }
  }
  __shared__ double pap[NC];
  block_reduce_rows<NC>(pa, nba, pap);
  double al[NC], be[NC];
  int bad = 0, brk = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double rz = sc->rzs[parity][c];
    al[c] = pap[c] != 0.0 ? rz / pap[c] : 0.0;
    be[c] = first ? 0.0 : sc->beta[c];
    brk |= indefinite(rz, pap[c]);
    bad |= !isfinite(pap[c]);
  }
  const bool stop = check && (brk || bad);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < NC; ++c) {
      sc->pap[c] = pap[c];
      sc->alpha[c] = al[c];
    }
    if (brk) sc->breakdown = 1;
    if (bad) sc->nonfinite = 1;
    if (stop)
      sc->done = sc->halted = 1;
    else
      sc->iters += 1;
  }
  if (stop) return;
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * kVecThreads;
    if (v >= n) continue;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double pk = first ? po[j][c] : __builtin_fma(be[c], po[j][c], zo[j][c]);
      if (!first) p[c * n + v] = pk;
      x[c * n + v] = xo[j][c] + al[c] * pk;
      const double zv = zo[j][c] - (al[c] * di[j]) * wo[j][c];
      z[c * n + v] = zv;
      if (v >= n_own) w[c * n + v] = 0.0;
      const double rv = di[j] != 0.0 ? zv / di[j] : 0.0;
      acc[c] += rv * zv;
      acc[NC + c] += rv * rv;
    }
  }
  block_partials<2 * NC>(acc, pr);
}

// The vector kernel of the four-launch form (one component, meshes above the
// two-launch bounds): the operator has applied A to p_k = z_k + beta p_{k-1}
// with beta from k_fin_beta, and k_fin_alpha has formed alpha; per node p_k
// (stored, the same fma as the operator's), x += alpha p_k, z_{k+1} =
// z_k - alpha dinv w_k, w cleared on the nodes the operator adds into;
// partials of r.z and r.r as k_cg_update_r writes them (for k_fin_beta).
// Five words read and three written per node, against the six and four of
// the residual and direction updates.
template <bool NT>
__global__ __launch_bounds__(kVecThreads) void k_cg_update_rxp(
    int64_t n, double *__restrict__ x, double *__restrict__ p, double *__restrict__ z,
    double *__restrict__ w, const double *__restrict__ dinv, double *__restrict__ part,
    const DevScalars *__restrict__ sc, int check, int first, int64_t n_own) {
  if (check && sc->done) return;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const double al = sc->alpha[0], be = first ? 0.0 : sc->beta[0];
  double rz = 0.0, rr = 0.0;
  if (v < n) {
    const double di = ld_v<NT>(dinv + v), zo = ld_v<NT>(z + v), wo = ld_v<NT>(w + v);
    const double po = ld_v<NT>(p + v), xo = ld_v<NT>(x + v);
    const double pk = first ? po : __builtin_fma(be, po, zo);
    if (!first) st_v<NT>(p + v, pk);
    st_v<NT>(x + v, xo + al * pk);
    const double zv = zo - (al * di) * wo;
    st_v<NT>(z + v, zv);
    if (v >= n_own) st_v<NT>(w + v, 0.0);
    const double rv = di != 0.0 ? zv / di : 0.0;
    rz = rv * zv;
    rr = rv * rv;
  }
  block_partial1(rz, part, 2, 0);
  block_partial1(rr, part, 2, 1);
}

// After the last iteration of the two-launch form: r.z and r.r of the last
// iterate from the partials pr, and its stopping test. Nothing to do once
// the solve halted (a stopping test met in an operator launch, which stored
// these scalars itself, or a breakdown, after which pr holds no new rows).
template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_rxp_fused(const double *__restrict__ pr,
                                                               int64_t nb, DevScalars *sc) {
  constexpr int nc = NC;
  if (sc->halted) return;
  __shared__ double res[2 * NC];
  reduce_columns<2 * NC>(pr, nb, res);
  if (threadIdx.x == 0) {
    for (int c = 0; c < nc; ++c) {
      sc->rz[c] = res[c];
      sc->rr[c] = res[nc + c];
      if (!isfinite(res[c]) || !isfinite(res[nc + c])) sc->nonfinite = 1;
    }
    if (!sc->done && !sc->fixed && converged(sc, nc)) sc->done = 1;
  }
}

// w[c][v] += Q^T w_L at node v (fixed order as above), one node per thread
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_gather_local(
    int64_t n, int64_t nl, const int32_t *__restrict__ off, const int32_t *__restrict__ pos,
    const T *__restrict__ wl, T *__restrict__ w, const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (v >= n) return;
  const T *wc = wl + blockIdx.y * nl;
  w[blockIdx.y * n + v] += gather_node(wc, pos, off[v], off[v + 1], (int32_t)(nl - 1));
}

template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_beta(const double *__restrict__ part,
                                                          int64_t nb, DevScalars *sc, int check) {
  constexpr int nc = NC;
  if (check && sc->done) return;
  __shared__ double res[2 * NC];
  reduce_columns<2 * NC>(part, nb, res);
  if (threadIdx.x == 0) {
    for (int c = 0; c < nc; ++c) {
      const double rz = res[c];
      sc->beta[c] = sc->rz[c] != 0.0 ? rz / sc->rz[c] : 0.0;
      sc->rzp[c] = sc->rz[c];
      sc->rz[c] = rz;
      sc->rr[c] = res[nc + c];
      if (!isfinite(rz) || !isfinite(res[nc + c])) sc->nonfinite = 1;
    }
    sc->iters += 1;
    if (sc->nonfinite || (!sc->fixed && converged(sc, nc))) sc->done = 1;
  }
}

// x += alpha p with the p of this iteration, then p = z + beta p unless
// the iteration just converged. `halted` (set by the next k_fin_alpha once
// done is seen) stops the x update in the launches queued after the last
// iteration.
template <typename T, bool NT, int K>
__global__ __launch_bounds__(kVecThreads / K) void k_cg_update_xp(int64_t n, T *__restrict__ x,
                                                                 T *__restrict__ p,
                                                                 const T *__restrict__ z,
                                                                 const DevScalars *__restrict__ sc,
                                                                 int check) {
  constexpr int TH = kVecThreads / K;
  if (check && sc->halted) return;
  const int comp = blockIdx.y;
  const int64_t s0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x, head = comp_head(comp, n);
  const T al = (T)sc->alpha[comp], be = (T)sc->beta[comp];
  // z is loaded whether or not the direction is updated, so that its load
  // does not wait for the done flag; only the store of p depends on it
  T pv[K], xv[K], zv[K];
  int64_t vj[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = vj[j] = comp_node(s0 + j * TH, head);
    pv[j] = xv[j] = zv[j] = T(0);
    if (v < n) {
      pv[j] = ld_v<NT>(p + comp * n + v);
      xv[j] = ld_v<NT>(x + comp * n + v);
      zv[j] = ld_v<NT>(z + comp * n + v);
    }
  }
  const bool dir = !sc->done;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = vj[j];
    if (v < n) {
      const int64_t f = comp * n + v;
      st_v<NT>(x + f, xv[j] + al * pv[j]);
      if (dir) st_v<NT>(p + f, zv[j] + be * pv[j]);
    }
  }
}

// r = b - w, w = 0; partials r.r and b.b. As in k_cg_init, entries of b on
// Dirichlet nodes (dinv = 0 there) are read as 0.
__global__ __launch_bounds__(kVecThreads) void k_dc_residual(int64_t n, const double *__restrict__ b,
                                                             double *__restrict__ r,
                                                             double *__restrict__ w,
                                                             const double *__restrict__ dinv,
                                                             double *__restrict__ part) {
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double rr = 0.0, bb = 0.0;
  if (v < n) {
    const int64_t f = comp * n + v;
    const double bv = dinv[v] != 0.0 ? b[f] : 0.0;
    const double rv = dinv[v] != 0.0 ? bv - w[f] : 0.0;
    r[f] = rv;
    w[f] = 0.0;
    rr = rv * rv;
    bb = bv * bv;
  }
  block_partial1(rr, part, 2 * nc, comp);
  block_partial1(bb, part, 2 * nc, nc + comp);
}

template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_norms(const double *__restrict__ part,
                                                           int64_t nb, DevScalars *sc) {
  constexpr int nc = NC;
  __shared__ double res[2 * NC];
  reduce_columns<2 * NC>(part, nb, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < nc; ++c) {
      sc->rr[c] = res[c];
      sc->bb[c] = res[nc + c];
    }
}

// sc->pap[c] = the sum of column c of part[nb][NC] in the fixed order of
// reduce_columns (the energies u^T M u per component of a mass apply)
template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_energy(const double *__restrict__ part,
                                                            int64_t nb, DevScalars *sc) {
  __shared__ double res[NC];
  reduce_columns<NC>(part, nb, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < NC; ++c) sc->pap[c] = res[c];
}

// d = a - b entry by entry (d may be a)
__global__ __launch_bounds__(kVecThreads) void k_difference(const double *a,
                                                            const double *__restrict__ b,
                                                            double *d, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kVecThreads)
    d[i] = a[i] - b[i];
}

__global__ __launch_bounds__(kVecThreads) void k_to_f32(const double *__restrict__ s,
                                                        float *__restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kVecThreads)
    d[i] = (float)s[i];
}

__global__ __launch_bounds__(kVecThreads) void k_accumulate(double *__restrict__ x,
                                                            const float *__restrict__ d,
                                                            int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kVecThreads)
    x[i] += (double)d[i];
}

__global__ __launch_bounds__(kVecThreads) void k_invert(const double *__restrict__ d,
                                                        double *__restrict__ di,
                                                        float *__restrict__ di32, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kVecThreads) {
    const double v = d[i] != 0.0 ? 1.0 / d[i] : 0.0;
    di[i] = v;
    if (di32) di32[i] = (float)v;
  }
}

// Gk[e][m][q] = kappa[e][q] * G[e][m][q]
// Index in the caller's [c][b][a] point order of stored point qp (qrev = q:
// stored reversed, [a][b][c]; 0: same order).
__device__ __forceinline__ int64_t natural_point(int64_t qp, int qrev) {
  if (!qrev) return qp;
  const int64_t a = qp / ((int64_t)qrev * qrev), b = qp / qrev % qrev, c = qp % qrev;
  return (c * qrev + b) * qrev + a;
}

__global__ __launch_bounds__(kVecThreads) void k_scale_geometry(const double *__restrict__ G,
                                                                const double *__restrict__ kap,
                                                                double *__restrict__ Gk,
                                                                float *__restrict__ Gk32,
                                                                int64_t nelem, int nq, int qrev) {
  const int64_t total = nelem * 6 * nq;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kVecThreads) {
    const int64_t e = i / (6 * (int64_t)nq);
    const int64_t qp = i % nq;
    const double v = kap[e * nq + natural_point(qp, qrev)] * G[i];
    Gk[i] = v;
    if (Gk32) Gk32[i] = (float)v;
  }
}

// ---- single-reduction PCG (Chronopoulos-Gear recurrences) -----------------
// With u = dinv r, w = A u and s = A p carried by recurrence, (r, u) comes
// from the vector pass and (u, w) from the operator's fused energy, so one
// finisher per iteration computes alpha and beta.

// r = b - w (w = A x0), u = dinv r, p = s = 0, w = 0; partials r.u, r.r, b.b
// (entries of b on Dirichlet nodes read as 0)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_sr_init(int64_t n, const T *__restrict__ b,
                                                         T *__restrict__ r, T *__restrict__ w,
                                                         T *__restrict__ u, T *__restrict__ p,
                                                         T *__restrict__ sv,
                                                         const T *__restrict__ dinv,
                                                         double *__restrict__ part) {
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double ru = 0.0, rr = 0.0, bb = 0.0;
  if (v < n) {
    const int64_t f = comp * n + v;
    const T di = dinv[v];
    const bool free = di != T(0);
    const T bv = free ? b[f] : T(0);
    const T rv = free ? bv - w[f] : T(0);
    const T uv = di * rv;
    r[f] = rv;
    u[f] = uv;
    p[f] = T(0);
    sv[f] = T(0);
    w[f] = T(0);
    ru = (double)rv * (double)uv;
    rr = (double)rv * (double)rv;
    bb = (double)bv * (double)bv;
  }
  block_partial1(ru, part, 3 * nc, comp);
  block_partial1(rr, part, 3 * nc, nc + comp);
  block_partial1(bb, part, 3 * nc, 2 * nc + comp);
}

// p = u + beta p; s = w + beta s; x += alpha p; r -= alpha s; u = dinv r;
// w = 0; partials r.u and r.r. Only u is kept: r = u / dinv (0 on Dirichlet
// nodes, where dinv = 0), so the pass moves 11 vector words per DOF; NT
// streams vectors larger than the last-level cache (see ld_v).
template <typename T, bool NT>
__global__ __launch_bounds__(kGroupThreads<T>) void k_sr_update(
    int64_t n, T *__restrict__ x, T *__restrict__ u, T *__restrict__ w, T *__restrict__ p,
    T *__restrict__ sv, const T *__restrict__ dinv, double *__restrict__ part,
    const DevScalars *__restrict__ sc, int check, int64_t n_own) {
  constexpr int K = kNodesPerThread<T>, TH = kGroupThreads<T>;
  if (check && sc->done) return;
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  const T al = (T)sc->alpha[comp], be = (T)sc->beta[comp];
  T di[K], uo[K], po[K], wo[K], so[K], xo[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    di[j] = uo[j] = po[j] = wo[j] = so[j] = xo[j] = T(0);
    if (v < n) {
      const int64_t f = comp * n + v;
      di[j] = ld_v<NT>(dinv + v);
      uo[j] = ld_v<NT>(u + f);
      po[j] = ld_v<NT>(p + f);
      wo[j] = ld_v<NT>(w + f);
      so[j] = ld_v<NT>(sv + f);
      xo[j] = ld_v<NT>(x + f);
    }
  }
  double ru = 0.0, rr = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t v = v0 + j * TH;
    if (v < n) {
      const int64_t f = comp * n + v;
      const T pn = uo[j] + be * po[j];
      const T s = wo[j] + be * so[j];
      st_v<NT>(p + f, pn);
      st_v<NT>(sv + f, s);
      st_v<NT>(x + f, xo[j] + al * pn);
      const T rv = (di[j] != T(0) ? uo[j] / di[j] : T(0)) - al * s;
      const T uv = di[j] * rv;
      st_v<NT>(u + f, uv);
      if (v >= n_own) st_v<NT>(w + f, T(0));
      ru += (double)rv * (double)uv;
      rr += (double)rv * (double)rv;
    }
  }
  block_partial1<TH>(ru, part, 2 * nc, comp);
  block_partial1<TH>(rr, part, 2 * nc, nc + comp);
}

// first: gamma, r.r, b.b from the vector pass, delta = (u, A u) from the
// operator; alpha = gamma / delta, beta = 0. Later: beta = gamma' / gamma,
// alpha = gamma' / (delta - beta gamma' / alpha); convergence on r.r.
template <int NC, bool FIRST>
__global__ __launch_bounds__(kFinThreads) void k_fin_sr(const double *__restrict__ pv,
                                                        int64_t nbv,
                                                        const double *__restrict__ pa,
                                                        int64_t nba, DevScalars *sc) {
  if (!FIRST && sc->done) return;
  constexpr int WV = FIRST ? 3 * NC : 2 * NC;
  __shared__ double rv[WV];
  __shared__ double ra[NC];
  reduce_columns<WV>(pv, nbv, rv);
  reduce_columns<NC>(pa, nba, ra);
  if (threadIdx.x == 0) {
    int bad = 0, brk = 0;
    for (int c = 0; c < NC; ++c) {
      const double g = rv[c], delta = ra[c];
      double alpha, beta = 0.0;
      // (r, u) != 0 with a curvature that does not give alpha > 0 is a breakdown
      if (FIRST) {
        alpha = delta != 0.0 ? g / delta : 0.0;
        sc->bb[c] = rv[2 * NC + c];
        if (indefinite(g, delta)) brk = 1;
      } else {
        beta = sc->rz[c] != 0.0 ? g / sc->rz[c] : 0.0;
        const double den = delta - (sc->alpha[c] != 0.0 ? beta * g / sc->alpha[c] : 0.0);
        alpha = den != 0.0 ? g / den : 0.0;
        if (indefinite(g, den)) brk = 1;
      }
      sc->rz[c] = g;
      sc->pap[c] = delta;
      sc->rr[c] = rv[NC + c];
      sc->alpha[c] = alpha;
      sc->beta[c] = beta;
      bad |= !isfinite(g) || !isfinite(delta) || !isfinite(rv[NC + c]);
    }
    if (FIRST) {
      sc->iters = 0;
      sc->breakdown = brk && !bad;
      sc->halted = 0;
    } else {
      sc->iters += 1;
      sc->breakdown = sc->breakdown || brk;
    }
    sc->nonfinite = bad;
    // a breakdown ends a solve that has a stopping test before the step
    // that would use its alpha (fixed iteration counts keep going)
    sc->done = bad || (!sc->fixed && (brk || converged(sc, NC)));
  }
}

// p = dinv r + beta p: the direction update left pending by a residual
// replacement (k_cg_update_xp skips it in the iteration that converged)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cg_direction(int64_t n, T *__restrict__ p,
                                                              const T *__restrict__ z,
                                                              const DevScalars *__restrict__ sc) {
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (v < n) {
    const int64_t f = blockIdx.y * n + v;
    p[f] = z[f] + (T)sc->beta[blockIdx.y] * p[f];
  }
}

// A replaced residual r (the search direction is kept; see cg_restart):
// z = dinv r in place, as the iteration stores it, and partials of r.z, r.r.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cg_dots(int64_t n, T *__restrict__ r,
                                                         const T *__restrict__ dinv,
                                                         double *__restrict__ part) {
  const int comp = blockIdx.y, nc = gridDim.y;
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (v < n) {
    const T rv = r[comp * n + v];
    const T zv = dinv[v] * rv;
    r[comp * n + v] = zv;
    rz = (double)rv * (double)zv;
    rr = (double)rv * (double)rv;
  }
  block_partial1(rz, part, 2 * nc, comp);
  block_partial1(rr, part, 2 * nc, nc + comp);
}

// Bb[i] = beta_i * Bt[i] with beta_i = beta_q[i], or beta if beta_q is NULL
__global__ __launch_bounds__(kVecThreads) void k_scale_mass(const double *__restrict__ Bt,
                                                            const double *__restrict__ beta_q,
                                                            double beta, double *__restrict__ Bb,
                                                            float *__restrict__ Bb32,
                                                            int64_t count, int nq, int qrev) {
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kVecThreads) {
    const double bq = beta_q ? beta_q[i / nq * nq + natural_point(i % nq, qrev)] : beta;
    const double v = bq * Bt[i];
    Bb[i] = v;
    if (Bb32) Bb32[i] = (float)v;
  }
}

// Between the caller's node order and the internal one, per component, as a
// gather (contiguous stores): dst[c][v] = src[c][map[v]].
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_permute(int64_t n, const int32_t *__restrict__ map,
                                                         const T *__restrict__ src,
                                                         T *__restrict__ dst) {
  const int64_t v = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (v >= n) return;
  const int64_t c = (int64_t)blockIdx.y * n;
  dst[c + v] = src[c + map[v]];
}

}  // namespace

template <typename T>
void permute_in(int nc, int64_t n, const int32_t *perm, const T *src, T *dst, hipStream_t s) {
  hipLaunchKernelGGL((k_permute<T>), dim3(vec_blocks(n), nc), dim3(kVecThreads), 0, s, n, perm,
                     src, dst);
}
template <typename T>
void permute_out(int nc, int64_t n, const int32_t *iperm, const T *src, T *dst, hipStream_t s) {
  hipLaunchKernelGGL((k_permute<T>), dim3(vec_blocks(n), nc), dim3(kVecThreads), 0, s, n, iperm,
                     src, dst);
}
template void permute_in<double>(int, int64_t, const int32_t *, const double *, double *,
                                 hipStream_t);
template void permute_in<float>(int, int64_t, const int32_t *, const float *, float *,
                                hipStream_t);
template void permute_out<double>(int, int64_t, const int32_t *, const double *, double *,
                                  hipStream_t);
template void permute_out<float>(int, int64_t, const int32_t *, const float *, float *,
                                 hipStream_t);

int64_t vec_blocks(int64_t n) {
  const int64_t b = (n + kVecThreads - 1) / kVecThreads;
  return b < 1 ? 1 : b;
}

int64_t grid_blocks(int64_t n) {
  int64_t b = (n + kVecThreads - 1) / kVecThreads;
  if (b > kVecMaxBlocks) b = kVecMaxBlocks;
  return b < 1 ? 1 : b;
}

// Reduce part[nb][width] to at most kStage2Rows rows in `stage` (nothing to
// do up to kDirectRows rows), then return the pointer and row count the
// single-work-group finisher reads.
static const double *reduce_stage1(const double *part, int64_t nb, int width, double *stage,
                                   int64_t *rows, hipStream_t s) {
  if (nb <= kDirectRows) {
    *rows = nb;
    return part;
  }
  const int64_t chunk = (nb + kStage2Rows - 1) / kStage2Rows;
  const int64_t blocks = (nb + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_reduce_rows, dim3(blocks), dim3(kVecThreads), 0, s, part, nb, width, chunk,
                     stage);
  *rows = blocks;
  return stage;
}

void fill_f64(double *x, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_blocks(n)), dim3(kVecThreads), 0, s, x, n, v);
}
void fill_f32(float *x, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_blocks(n)), dim3(kVecThreads), 0, s, x, n, v);
}
void to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_blocks(n)), dim3(kVecThreads), 0, s, src, dst, n);
}
void invert_diag(const double *d, double *dinv, float *dinv32, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(grid_blocks(n)), dim3(kVecThreads), 0, s, d, dinv, dinv32, n);
}
void scale_geometry(const double *G, const double *kappa, double *Gk, float *Gk32, int qrev,
                    int64_t nelem, int nq, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_geometry, dim3(grid_blocks(nelem * 6 * nq)), dim3(kVecThreads), 0, s,
                     G, kappa, Gk, Gk32, nelem, nq, qrev);
}

// after a residual replacement that ended an iteration before its direction
// update: r.z and r.r of the new residual, beta = (r.z)_new / (r.z) of the
// iteration (for the pending p = z + beta p); r.r also becomes the reference
// for the next relative reduction; the loop flags are cleared
template <int NC>
__global__ __launch_bounds__(kFinThreads) void k_fin_restart(const double *__restrict__ part,
                                                             int64_t nb, DevScalars *sc) {
  __shared__ double res[2 * NC];
  reduce_columns<2 * NC>(part, nb, res);
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int c = 0; c < NC; ++c) {
      sc->beta[c] = sc->rzp[c] != 0.0 ? res[c] / sc->rzp[c] : 0.0;
      sc->rz[c] = res[c];
      sc->rr[c] = sc->bb[c] = res[NC + c];
      bad |= !isfinite(res[c]) || !isfinite(res[NC + c]);
    }
    sc->nonfinite = bad;
    sc->done = bad;
    sc->halted = bad;
  }
}

enum class FinKind { Init, Alpha, Beta, Norms, Restart, Energy };

// the single-work-group finisher for nc components (compile-time widths)
template <int NC>
static void launch_fin_nc(FinKind k, const double *src, int64_t rows, DevScalars *sc,
                          hipStream_t s, int check) {
  switch (k) {
    case FinKind::Init:
      hipLaunchKernelGGL(k_fin_init<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc);
      break;
    case FinKind::Alpha:
      hipLaunchKernelGGL(k_fin_alpha<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc,
                         check);
      break;
    case FinKind::Beta:
      hipLaunchKernelGGL(k_fin_beta<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc,
                         check);
      break;
    case FinKind::Norms:
      hipLaunchKernelGGL(k_fin_norms<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc);
      break;
    case FinKind::Restart:
      hipLaunchKernelGGL(k_fin_restart<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc);
      break;
    case FinKind::Energy:
      hipLaunchKernelGGL(k_fin_energy<NC>, dim3(1), dim3(kFinThreads), 0, s, src, rows, sc);
      break;
  }
}

static void launch_fin(FinKind k, int nc, const double *src, int64_t rows, DevScalars *sc,
                       hipStream_t s, int check = 1) {
  switch (nc) {
    case 1: launch_fin_nc<1>(k, src, rows, sc, s, check); break;
    case 2: launch_fin_nc<2>(k, src, rows, sc, s, check); break;
    case 3: launch_fin_nc<3>(k, src, rows, sc, s, check); break;
    case 4: launch_fin_nc<4>(k, src, rows, sc, s, check); break;
    case 5: launch_fin_nc<5>(k, src, rows, sc, s, check); break;
    case 6: launch_fin_nc<6>(k, src, rows, sc, s, check); break;
    case 7: launch_fin_nc<7>(k, src, rows, sc, s, check); break;
    default: launch_fin_nc<kMaxComp>(k, src, rows, sc, s, check); break;
  }
}

void scale_mass(const double *Bt, const double *beta_q, double beta, double *Bb, float *Bb32,
                int nq, int qrev, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_mass, dim3(grid_blocks(count)), dim3(kVecThreads), 0, s, Bt, beta_q,
                     beta, Bb, Bb32, count, nq, qrev);
}

template <typename T>
void cg_init(int nc, int64_t n, const T *b, T *r, T *w, T *p, const T *dinv, double *part,
             DevScalars *sc, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_init<T>), dim3(nb, nc), dim3(kVecThreads), 0, s, n, b, r, w, p, dinv,
                     part);
  int64_t rows = 0;
  const double *src = reduce_stage1(part, nb, 3 * nc, part + nb * 3 * nc, &rows, s);
  launch_fin(FinKind::Init, nc, src, rows, sc, s);
}

void cg_fin_alpha(int nc, const double *part, int64_t nb, DevScalars *sc, hipStream_t s,
                  bool check) {
  int64_t rows = 0;
  const double *src = reduce_stage1(part, nb, nc, const_cast<double *>(part) + nb * nc, &rows, s);
  launch_fin(FinKind::Alpha, nc, src, rows, sc, s, check ? 1 : 0);
}

template <typename T, bool NT, int NC>
static void launch_update_r_nc(int64_t n, T *r, T *w, const T *dinv, double *part,
                               DevScalars *sc, hipStream_t s, int check, int64_t n_own) {
  // two nodes per thread up to four components (measured on three at
  // n = 337^3: 567 us against 573 us with one)
  constexpr int K = NC <= 4 ? 2 : 1;
  hipLaunchKernelGGL((k_cg_update_r_nc<T, NT, NC, K>), dim3(vec_blocks(n)), dim3(kVecThreads / K),
                     0, s, n, r, w, dinv, part, sc, check, n_own);
}

template <typename T, bool NT>
static void update_r_nc(int nc, int64_t n, T *r, T *w, const T *dinv, double *part,
                        DevScalars *sc, hipStream_t s, int check, int64_t n_own) {
  switch (nc) {
    case 2: launch_update_r_nc<T, NT, 2>(n, r, w, dinv, part, sc, s, check, n_own); break;
    case 3: launch_update_r_nc<T, NT, 3>(n, r, w, dinv, part, sc, s, check, n_own); break;
    case 4: launch_update_r_nc<T, NT, 4>(n, r, w, dinv, part, sc, s, check, n_own); break;
    case 5: launch_update_r_nc<T, NT, 5>(n, r, w, dinv, part, sc, s, check, n_own); break;
    case 6: launch_update_r_nc<T, NT, 6>(n, r, w, dinv, part, sc, s, check, n_own); break;
    case 7: launch_update_r_nc<T, NT, 7>(n, r, w, dinv, part, sc, s, check, n_own); break;
    default: launch_update_r_nc<T, NT, kMaxComp>(n, r, w, dinv, part, sc, s, check, n_own);
  }
}

template <typename T>
void cg_update_r(int nc, int64_t n, T *r, T *w, const T *dinv, double *part, DevScalars *sc,
                 hipStream_t s, bool check, int64_t n_own) {
  if (nc > 1) {  // one thread per node for every component: dinv read once
    if (n * (int64_t)sizeof(T) >= kStreamBytes)
      update_r_nc<T, true>(nc, n, r, w, dinv, part, sc, s, check ? 1 : 0, n_own);
    else
      update_r_nc<T, false>(nc, n, r, w, dinv, part, sc, s, check ? 1 : 0, n_own);
    return;
  }
  // one component: two FP64 or four FP32 nodes per thread
  constexpr int K = sizeof(T) == 4 ? 4 : 2;
  if (n * (int64_t)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_cg_update_r<T, true, K>), dim3(vec_blocks(n), nc),
                       dim3(kVecThreads / K), 0, s, n, r, w, dinv, part, sc, check ? 1 : 0, n_own);
  else
    hipLaunchKernelGGL((k_cg_update_r<T, false, K>), dim3(vec_blocks(n), nc),
                       dim3(kVecThreads / K), 0, s, n, r, w, dinv, part, sc, check ? 1 : 0, n_own);
}

void cg_fin_beta(int nc, int64_t nb, const double *part, DevScalars *sc, hipStream_t s,
                 bool check) {
  int64_t rows = 0;
  const double *src =
      reduce_stage1(part, nb, 2 * nc, const_cast<double *>(part) + nb * 2 * nc, &rows, s);
  launch_fin(FinKind::Beta, nc, src, rows, sc, s, check ? 1 : 0);
}

template <int NC>
static void launch_fused_nc(bool residual, int64_t n, double *x, double *p, double *z,
                            double *w, const double *dinv, const double *pa, int64_t nba,
                            double *pr, DevScalars *sc, int parity, int check, int64_t n_own,
                            hipStream_t s) {
  if (residual)
    hipLaunchKernelGGL((k_cg_update_r_fused<NC>), dim3(vec_blocks(n)), dim3(kVecThreads), 0, s,
                       n, z, w, dinv, pa, nba, pr, sc, parity, check, n_own);
  else
    hipLaunchKernelGGL((k_cg_update_xp_fused<NC>), dim3(vec_blocks(n)), dim3(kVecThreads), 0,
                       s, n, x, p, z, pr, vec_blocks(n), sc, parity, check);
}

static void launch_fused(bool residual, int nc, int64_t n, double *x, double *p, double *z,
                         double *w, const double *dinv, const double *pa, int64_t nba,
                         double *pr, DevScalars *sc, int parity, int check, int64_t n_own,
                         hipStream_t s) {
#define BP_FUSED(NC) \
  launch_fused_nc<NC>(residual, n, x, p, z, w, dinv, pa, nba, pr, sc, parity, check, n_own, s)
  switch (nc) {
    case 1: BP_FUSED(1); break;
    case 2: BP_FUSED(2); break;
    case 3: BP_FUSED(3); break;
    case 4: BP_FUSED(4); break;
    case 5: BP_FUSED(5); break;
    case 6: BP_FUSED(6); break;
    case 7: BP_FUSED(7); break;
    default: BP_FUSED(kMaxComp); break;
  }
#undef BP_FUSED
}

void cg_update_rxp_fused(int nc, int64_t n, double *x, double *p, double *z, double *w,
                         const double *dinv, const double *pa, int64_t nba, double *pr,
                         DevScalars *sc, int parity, hipStream_t s, bool check, bool first,
                         int64_t n_own) {
  (void)nc;  // one component (apply_pz_supported)
  if (vec_blocks(n) <= kFusedRows)
    hipLaunchKernelGGL((k_cg_update_rxp_fused<1, 1>), dim3(rxp_rows(n)), dim3(kVecThreads), 0,
                       s, n, x, p, z, w, dinv, pa, nba, pr, sc, parity, check ? 1 : 0,
                       first ? 1 : 0, n_own);
  else
    hipLaunchKernelGGL((k_cg_update_rxp_fused<1, kRxpNodes>), dim3(rxp_rows(n)),
                       dim3(kVecThreads), 0, s, n, x, p, z, w, dinv, pa, nba, pr, sc, parity,
                       check ? 1 : 0, first ? 1 : 0, n_own);
}

void cg_fin_rxp_fused(int nc, int64_t n, const double *pr, DevScalars *sc, hipStream_t s) {
  (void)nc;
  hipLaunchKernelGGL((k_fin_rxp_fused<1>), dim3(1), dim3(kFinThreads), 0, s, pr, rxp_rows(n),
                     sc);
}

void cg_update_rxp(int64_t n, double *x, double *p, double *z, double *w, const double *dinv,
                   double *part, DevScalars *sc, hipStream_t s, bool check, bool first,
                   int64_t n_own) {
  if (n * (int64_t)sizeof(double) >= kStreamBytes)
    hipLaunchKernelGGL((k_cg_update_rxp<true>), dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, n,
                       x, p, z, w, dinv, part, sc, check ? 1 : 0, first ? 1 : 0, n_own);
  else
    hipLaunchKernelGGL((k_cg_update_rxp<false>), dim3(vec_blocks(n)), dim3(kVecThreads), 0, s,
                       n, x, p, z, w, dinv, part, sc, check ? 1 : 0, first ? 1 : 0, n_own);
}

bool cg_streams(int64_t n) { return n * (int64_t)sizeof(double) >= kStreamBytes; }

int64_t rxp_rows(int64_t n) {
  if (vec_blocks(n) <= kFusedRows) return vec_blocks(n);
  const int64_t g = kRxpNodes * kVecThreads;
  return (n + g - 1) / g;
}

// Every work-group of each launch reads the other launch's whole partial
// table: the bound keeps those redundant reads (rows x work-groups) small
// against what the two dropped launches cost.
bool cg_fused2_fits(int64_t n, int64_t nb_apply) {
  const int64_t nv = rxp_rows(n);
  return nv <= kFused2VecRows && nb_apply <= kFused2ApplyRows &&
         nv * nb_apply <= kFused2Product;
}

bool cg_fused_fits(int64_t n, int64_t nb_apply) {
  return vec_blocks(n) <= kFusedRows && nb_apply <= kFusedRows;
}

void cg_update_r_fused(int nc, int64_t n, double *z, double *w, const double *dinv,
                       const double *pa, int64_t nba, double *pr, DevScalars *sc, int parity,
                       hipStream_t s, bool check, int64_t n_own) {
  launch_fused(true, nc, n, nullptr, nullptr, z, w, dinv, pa, nba, pr, sc, parity,
               check ? 1 : 0, n_own, s);
}

void cg_update_xp_fused(int nc, int64_t n, double *x, double *p, const double *z,
                        const double *pr, DevScalars *sc, int parity, hipStream_t s,
                        bool check) {
  launch_fused(false, nc, n, x, p, const_cast<double *>(z), nullptr, nullptr, nullptr, 0,
               const_cast<double *>(pr), sc, parity, check ? 1 : 0, 0, s);
}

template <typename T>
void cg_update_xp(int nc, int64_t n, T *x, T *p, const T *z, DevScalars *sc, hipStream_t s,
                  bool check) {
  // two nodes per thread, four for one FP32 component (measured: the
  // one-component FP64 update 2% faster with two than with one; the
  // three-component one, with its components realigned by comp_head, 692 us
  // against 767 us with one at n = 337^3)
  const bool nt = n * (int64_t)sizeof(T) >= kStreamBytes;
  const dim3 g(vec_blocks(n), nc);
  const int c = check ? 1 : 0;
  if (sizeof(T) == 4 && nc == 1) {  // one FP32 component: four nodes per thread
    if (nt)
      hipLaunchKernelGGL((k_cg_update_xp<T, true, 4>), g, dim3(kVecThreads / 4), 0, s, n, x, p,
                         z, sc, c);
    else
      hipLaunchKernelGGL((k_cg_update_xp<T, false, 4>), g, dim3(kVecThreads / 4), 0, s, n, x, p,
                         z, sc, c);
  } else if (nt) {
    hipLaunchKernelGGL((k_cg_update_xp<T, true, 2>), g, dim3(kVecThreads / 2), 0, s, n, x, p, z,
                       sc, c);
  } else {
    hipLaunchKernelGGL((k_cg_update_xp<T, false, 2>), g, dim3(kVecThreads / 2), 0, s, n, x, p, z,
                       sc, c);
  }
}

template <typename T>
void gather_local(int nc, int64_t n, int64_t nl, const int32_t *off, const int32_t *pos,
                  const T *wl, T *w, const int *done, hipStream_t s) {
  hipLaunchKernelGGL((k_gather_local<T>), dim3(vec_blocks(n), nc), dim3(kVecThreads), 0, s, n, nl,
                     off, pos, wl, w, done);
}

template <typename T, bool NT, int NC>
static void launch_gather_nc(int64_t n, int64_t nl, T *r, const T *wl, const int32_t *off,
                             const int32_t *pos, const T *dinv, double *part, DevScalars *sc,
                             hipStream_t s, int check) {
  hipLaunchKernelGGL((k_cg_update_r_gather_nc<T, NT, NC>), dim3(vec_blocks(n)),
                     dim3(kVecThreads), 0, s, n, nl, r, wl, off, pos, dinv, part, sc, check);
}

template <typename T, bool NT>
static void update_r_gather_nc(int nc, int64_t n, int64_t nl, T *r, const T *wl,
                               const int32_t *off, const int32_t *pos, const T *dinv,
                               double *part, DevScalars *sc, hipStream_t s, int check) {
  switch (nc) {
    case 2: launch_gather_nc<T, NT, 2>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    case 3: launch_gather_nc<T, NT, 3>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    case 4: launch_gather_nc<T, NT, 4>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    case 5: launch_gather_nc<T, NT, 5>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    case 6: launch_gather_nc<T, NT, 6>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    case 7: launch_gather_nc<T, NT, 7>(n, nl, r, wl, off, pos, dinv, part, sc, s, check); break;
    default:
      launch_gather_nc<T, NT, kMaxComp>(n, nl, r, wl, off, pos, dinv, part, sc, s, check);
  }
}

template <typename T>
void cg_update_r_gather(int nc, int64_t n, int64_t nl, T *r, const T *wl, const int32_t *off,
                        const int32_t *pos, const T *dinv, double *part, DevScalars *sc,
                        hipStream_t s, bool check) {
  if (nc > 1) {  // one thread per node for every component: map and dinv read once
    if (n * (int64_t)sizeof(T) >= kStreamBytes)
      update_r_gather_nc<T, true>(nc, n, nl, r, wl, off, pos, dinv, part, sc, s, check ? 1 : 0);
    else
      update_r_gather_nc<T, false>(nc, n, nl, r, wl, off, pos, dinv, part, sc, s, check ? 1 : 0);
    return;
  }
  if (n * (int64_t)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_cg_update_r_gather<T, true>), dim3(vec_blocks(n), nc),
                       dim3(kGroupThreads<T>), 0, s, n, nl, r, wl, off, pos, dinv, part, sc,
                       check ? 1 : 0);
  else
    hipLaunchKernelGGL((k_cg_update_r_gather<T, false>), dim3(vec_blocks(n), nc),
                       dim3(kGroupThreads<T>), 0, s, n, nl, r, wl, off, pos, dinv, part, sc,
                       check ? 1 : 0);
}

void operator_energies(int nc, double *part, int64_t rows, DevScalars *sc, hipStream_t s) {
  int64_t r = 0;
  const double *src = reduce_stage1(part, rows, nc, part + rows * nc, &r, s);
  launch_fin(FinKind::Energy, nc, src, r, sc, s);
}

void difference(const double *a, const double *b, double *d, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_difference, dim3(grid_blocks(count)), dim3(kVecThreads), 0, s, a, b, d,
                     count);
}

void dc_residual(int nc, int64_t n, const double *b, double *r, double *w, const double *dinv,
                 double *part, DevScalars *sc, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL(k_dc_residual, dim3(nb, nc), dim3(kVecThreads), 0, s, n, b, r, w, dinv,
                     part);
  int64_t rows = 0;
  const double *src = reduce_stage1(part, nb, 2 * nc, part + nb * 2 * nc, &rows, s);
  launch_fin(FinKind::Norms, nc, src, rows, sc, s);
}

template <typename T>
void sr_init(int nc, int64_t n, const T *b, T *r, T *w, T *u, T *p, T *sv, const T *dinv,
             double *part, hipStream_t s) {
  hipLaunchKernelGGL((k_sr_init<T>), dim3(vec_blocks(n), nc), dim3(kVecThreads), 0, s, n, b, r,
                     w, u, p, sv, dinv, part);
}

template <typename T>
void sr_update(int nc, int64_t n, T *x, T *u, T *w, T *p, T *sv, const T *dinv, double *part,
               DevScalars *sc, hipStream_t s, bool check, int64_t n_own) {
  if (n * (int64_t)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_sr_update<T, true>), dim3(vec_blocks(n), nc),
                       dim3(kGroupThreads<T>), 0, s, n, x, u, w, p, sv, dinv, part, sc,
                       check ? 1 : 0, n_own);
  else
    hipLaunchKernelGGL((k_sr_update<T, false>), dim3(vec_blocks(n), nc),
                       dim3(kGroupThreads<T>), 0, s, n, x, u, w, p, sv, dinv, part, sc,
                       check ? 1 : 0, n_own);
}

template <int NC>
static void launch_fin_sr_nc(bool first, const double *pv, int64_t nbv, const double *pa,
                             int64_t nba, DevScalars *sc, hipStream_t s) {
  if (first)
    hipLaunchKernelGGL((k_fin_sr<NC, true>), dim3(1), dim3(kFinThreads), 0, s, pv, nbv, pa, nba,
                       sc);
  else
    hipLaunchKernelGGL((k_fin_sr<NC, false>), dim3(1), dim3(kFinThreads), 0, s, pv, nbv, pa, nba,
                       sc);
}

void sr_fin(bool first, int nc, double *pv, int64_t nbv, double *pa, int64_t nba,
            DevScalars *sc, hipStream_t s) {
  const int wv = (first ? 3 : 2) * nc;
  int64_t rv = 0, ra = 0;
  const double *sv = reduce_stage1(pv, nbv, wv, pv + nbv * wv, &rv, s);
  const double *sa = reduce_stage1(pa, nba, nc, pa + nba * nc, &ra, s);
  switch (nc) {
    case 1: launch_fin_sr_nc<1>(first, sv, rv, sa, ra, sc, s); break;
    case 2: launch_fin_sr_nc<2>(first, sv, rv, sa, ra, sc, s); break;
    case 3: launch_fin_sr_nc<3>(first, sv, rv, sa, ra, sc, s); break;
    case 4: launch_fin_sr_nc<4>(first, sv, rv, sa, ra, sc, s); break;
    case 5: launch_fin_sr_nc<5>(first, sv, rv, sa, ra, sc, s); break;
    case 6: launch_fin_sr_nc<6>(first, sv, rv, sa, ra, sc, s); break;
    case 7: launch_fin_sr_nc<7>(first, sv, rv, sa, ra, sc, s); break;
    default: launch_fin_sr_nc<kMaxComp>(first, sv, rv, sa, ra, sc, s); break;
  }
}

template void sr_init<double>(int, int64_t, const double *, double *, double *, double *,
                              double *, double *, const double *, double *, hipStream_t);
template void sr_update<double>(int, int64_t, double *, double *, double *, double *, double *,
                                const double *, double *, DevScalars *, hipStream_t, bool,
                                int64_t);

template <typename T>
void cg_restart(int nc, int64_t n, T *r, T *p, const T *dinv, double *part,
                DevScalars *sc, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_dots<T>), dim3(nb, nc), dim3(kVecThreads), 0, s, n, r, dinv, part);
  int64_t rows = 0;
  const double *src = reduce_stage1(part, nb, 2 * nc, part + nb * 2 * nc, &rows, s);
  launch_fin(FinKind::Restart, nc, src, rows, sc, s);
  hipLaunchKernelGGL((k_cg_direction<T>), dim3(nb, nc), dim3(kVecThreads), 0, s, n, p, r, sc);
}

template void cg_restart<float>(int, int64_t, float *, float *, const float *, double *,
                                DevScalars *, hipStream_t);
template void cg_restart<double>(int, int64_t, double *, double *, const double *,
                                 double *, DevScalars *, hipStream_t);

void dc_accumulate(int64_t n, double *x, const float *d, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(grid_blocks(n)), dim3(kVecThreads), 0, s, x, d, n);
}

template void cg_init<double>(int, int64_t, const double *, double *, double *, double *,
                              const double *, double *, DevScalars *, hipStream_t);
template void cg_init<float>(int, int64_t, const float *, float *, float *, float *,
                             const float *, double *, DevScalars *, hipStream_t);
template void cg_update_r<double>(int, int64_t, double *, double *, const double *, double *,
                                  DevScalars *, hipStream_t, bool, int64_t);
template void cg_update_r<float>(int, int64_t, float *, float *, const float *, double *,
                                 DevScalars *, hipStream_t, bool, int64_t);
template void cg_update_xp<double>(int, int64_t, double *, double *, const double *,
                                   DevScalars *, hipStream_t, bool);
template void cg_update_xp<float>(int, int64_t, float *, float *, const float *, DevScalars *,
                                  hipStream_t, bool);
template void gather_local<double>(int, int64_t, int64_t, const int32_t *, const int32_t *,
                                   const double *, double *, const int *, hipStream_t);
template void gather_local<float>(int, int64_t, int64_t, const int32_t *, const int32_t *,
                                  const float *, float *, const int *, hipStream_t);
template void cg_update_r_gather<double>(int, int64_t, int64_t, double *, const double *,
                                         const int32_t *, const int32_t *, const double *,
                                         double *, DevScalars *, hipStream_t, bool);
template void cg_update_r_gather<float>(int, int64_t, int64_t, float *, const float *,
                                        const int32_t *, const int32_t *, const float *, double *,
                                        DevScalars *, hipStream_t, bool);

}  // namespace bp
