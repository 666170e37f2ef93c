// Batched matrix logarithm for many small matrices (n <= 128): persistent launches,
// one workgroup per matrix at a time (taken from a device work queue),
// every step of Algorithm 1 (Section 6) on the device, decisions included: scaled
// Denman-Beavers roots (eq. ScalDB), the finish test and degree selection (algo.hpp,
// shared with the single-matrix driver), the 1-norm estimator, and the
// computation-graph polynomial (eq. five_mult_degopt) with the 2^s rescale.
//
// Two size classes, one kernel each: n <= 64 (4 waves), where thread (wave w, lane l)
// holds row l and columns 16w..16w+15 of a register matrix, and 64 < n <= 128 (8
// waves), where it holds rows l and l + 64 and columns 16w..16w+15; the pad beyond n
// is the identity.
// Inversion is Gauss-Jordan elimination in those registers with one barrier per
// step: every wave finds the pivot itself (wave maximum of packed keys over the
// pivot column in LDS), the pivot row travels inside each wave through LDS, and the
// pivot row is left unscaled (its scale is applied when the inverse is stored), so
// the step is a pure FMA update.  Products keep the accumulator tile in the same
// layout and stream the right factor through LDS.  Per-workgroup buffers live in the
// caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "algo.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "logm.h"

namespace logm {
namespace {

typedef double d16 __attribute__((ext_vector_type(16)));

constexpr int BN_MAX = 128;   // largest n
constexpr int KC = 32;        // rows of a right factor staged per chunk
constexpr int NBUF = 2 * kKMax + 2;   // n x n buffers per workgroup

__device__ __forceinline__ int tid() { return threadIdx.x; }

// Register matrix of a size class: RA rows per lane (N = 64 RA rows), CW = 16 columns
// per wave (N / 16 waves, 256 RA threads); element (a, b) is row l + 64 a, column
// 16 w + b.  A row slice is one 16-wide vector, so a wave-uniform column index
// compiles to an indexed register move instead of scratch.
template <int RA, int CW>
struct RM {
  static_assert(CW == 16, "one 16-wide vector per row slice");
  d16 v[RA];
};
#define EL(m, a, b) ((m).v[a][b])

// Element (a, b) for a wave-uniform column b (indexed register move).
// Element (a, b) for a wave-uniform column b (indexed register move).
template <int RA, int CW>
__device__ __forceinline__ double dyn_get(const RM<RA, CW>& m, int a, int b) {
  return m.v[a][__builtin_amdgcn_readfirstlane(b)];
}

template <int RA, int CW>
__device__ __forceinline__ void dyn_set(RM<RA, CW>& m, int a, int b, double val) {
  m.v[a][__builtin_amdgcn_readfirstlane(b)] = val;
}

template <int RA, int CW>
struct Shm {
  static constexpr int N = 64 * RA;
  double chunk[KC][N + 2];   // product staging
  static constexpr int NW = N / CW;   // waves
  static constexpr int NT = 64 * NW;  // threads
  double colk[2][N];         // pivot column of the step, by step parity
  double rscale[N];          // 1 / pivot of each row, applied when the inverse is stored
  double pivabs[N];          // |pivot| of step k, for log|det| after the elimination
  double vec[5][N];          // estimator vectors
  double red[NT];            // reductions
  int perm[N];               // pivot row of step k
  int pinv[N];               // step at which row r was the pivot
};

// ---- workgroup reductions (fixed order, deterministic) ---------------------------
__device__ __forceinline__ int nthreads() { return blockDim.x; }

__device__ __forceinline__ double wg_sum(double* red, double v) {
  v = wave_sum(v);
  if ((tid() & 63) == 0) red[tid() >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nthreads() / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wg_max(double* red, double v) {
  v = wave_max(v);
  if ((tid() & 63) == 0) red[tid() >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < nthreads() / 64; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

// Largest column sum from per-thread partial sums of column tid % N over the row
// subset tid / N (threads / N = 4 subsets).
template <int N>
__device__ __forceinline__ double wg_colmax(double* red, double part) {
  red[tid()] = part;
  __syncthreads();
  double cs = 0.0;
  if (tid() < N)
    for (int g = 0; g < nthreads() / N; ++g) cs += red[tid() + g * N];
  __syncthreads();
  return wg_max(red, cs);
}

// ||M||_1 (n x n, ld n)
template <int N>
__device__ __forceinline__ double wg_norm1(double* red, const double* M, int n) {
  const int c = tid() % N, g = tid() / N;
  double s = 0.0;
  if (c < n)
    for (int i = g; i < n; i += nthreads() / N) s += fabs(M[i * n + c]);
  return wg_colmax<N>(red, s);
}

// ---- register matrices -----------------------------------------------------------
// Wave index as a uniform value (keeps wave-dependent addresses in scalar registers).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(tid() >> 6); }

// R = M (n x n, ld n) with the identity on the pad.  M must be a per-workgroup buffer
// of (64 RA)^2 elements: the N x N view with row stride n stays inside it, so every
// load is unconditional (one row pointer per row, constant column offsets).
template <int RA, int CW>
__device__ __forceinline__ void load_rm(RM<RA, CW>& R, const double* M, int n) {
  const int l = tid() & 63, w = wave_id();
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = l + 64 * a;
    const double* row = M + i * n + CW * w;
#pragma unroll
    for (int b = 0; b < CW; ++b) {
      const int j = CW * w + b;
      const double v = row[b];
      EL(R, a, b) = (i < n && j < n) ? v : (i == j ? 1.0 : 0.0);
    }
  }
}

template <int RA, int CW>
__device__ __forceinline__ void store_rm(const RM<RA, CW>& R, double* M, int n) {
  const int l = tid() & 63, w = wave_id();
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = l + 64 * a;
    double* row = M + i * n + CW * w;
    if (i < n) {
#pragma unroll
      for (int b = 0; b < CW; ++b)
        if (CW * w + b < n) row[b] = EL(R, a, b);
    }
  }
}

// C (registers) = A * B, A and B n x n in global memory.
template <int RA, int CW>
__device__ __forceinline__ void wg_gemm(Shm<RA, CW>& sh, RM<RA, CW>& C, const double* A,
                                        const double* B, int n) {
  constexpr int N = 64 * RA;
  const int l = tid() & 63, w = wave_id();
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < CW; ++b) EL(C, a, b) = 0.0;
  for (int k0 = 0; k0 < n; k0 += KC) {
    const int kc = min(KC, n - k0);
    for (int e = tid(); e < KC * N; e += nthreads()) {
      const int r = e / N, c = e % N;
      sh.chunk[r][c] = (r < kc && c < n) ? B[(k0 + r) * n + c] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double av[RA];
#pragma unroll
      for (int a = 0; a < RA; ++a) {   // in bounds for every lane (see load_rm)
        const int i = l + 64 * a;
        const double v = A[i * n + k0 + kk];
        av[a] = (i < n) ? v : 0.0;
      }
#pragma unroll
      for (int b = 0; b < CW; ++b) {
        const double bv = sh.chunk[kk][CW * w + b];
#pragma unroll
        for (int a = 0; a < RA; ++a) EL(C, a, b) = fma(av[a], bv, EL(C, a, b));
      }
    }
    __syncthreads();
  }
}

// Pivot key of row i: 1 + the high word of |v| without its low 7 bits (magnitudes
// within a factor 1 + 2^-13 tie), then the reversed row index, so that the wave
// maximum picks the largest magnitude and, among ties, the smallest row.  Every
// candidate's key is nonzero.
__device__ __forceinline__ unsigned pivot_key7(double v, int i) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffffu;
  return (((hi >> 7) + 1u) << 7) | (unsigned)(127 - i);
}

// Mi = M^{-1} (n x n, ld n) by Gauss-Jordan elimination with partial pivoting (the
// left division of eq. ScalDB) in registers; *logdet = log|det M|.  Returns false on
// an exact zero pivot.  Rows are never exchanged: the pivot of step k is the unused
// row p_k of largest magnitude in column k; it keeps its values (1 in column k), the
// other rows take row - (c_i / pivot) * pivot row, and on output
// Mi[k][p_c] = (row p_k)[c] / pivot_k.
template <int RA, int CW>
__device__ __forceinline__ bool wg_inverse(Shm<RA, CW>& sh, const double* M, double* Mi, int n,
                                           double* logdet) {
  const int l = tid() & 63, w = wave_id();
  RM<RA, CW> x;
  load_rm(x, M, n);
  bool used[RA];
#pragma unroll
  for (int a = 0; a < RA; ++a) used[a] = false;
  if (w == 0) {
#pragma unroll
    for (int a = 0; a < RA; ++a) sh.colk[0][l + 64 * a] = EL(x, a, 0);
  }
  __syncthreads();
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    const int q = k & 1;
    double c[RA];
    unsigned key = 0u;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = l + 64 * a;
      c[a] = sh.colk[q][i];
      const unsigned kk = (!used[a] && i < n) ? pivot_key7(c[a], i) : 0u;
      key = max(key, kk);
    }
    key = wave_max_u32(key);   // every wave finds the same pivot
    const int p = 127 - (int)(key & 127u);
    const int lp = p & 63;
    const double piv = readlane_d((RA == 2 && p >= 64) ? c[RA - 1] : c[0], lp);
    ok = ok && (piv != 0.0);
    const double rp = pivot_recip(piv);   // 0 for a zero pivot
    const int wk = k / CW, bk = k - wk * CW;
    // this wave's slice of the pivot row, with 1 in column k
    const int hp = p >> 6;   // row half of the pivot (the read below picks it)
    if (tid() == 0) {
      sh.perm[k] = p;
      sh.pinv[p] = k;
      sh.rscale[p] = rp;
      sh.pivabs[k] = fabs(piv);
    }
    double g[RA];
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const bool isp = (l + 64 * a == p);
      used[a] = used[a] || isp;
      g[a] = isp ? 0.0 : c[a] * rp;
      if (w == wk) dyn_set(x, a, bk, isp ? 1.0 : 0.0);
    }
    // this wave's slice of the pivot row straight from lane lp's registers (column k
    // already holds its 1); hp is wave-uniform, so the branch keeps indices static
    double rrow[CW];
    if (RA == 1 || hp == 0) {
#pragma unroll
      for (int b = 0; b < CW; ++b) rrow[b] = readlane_d(EL(x, 0, b), lp);
    } else {
#pragma unroll
      for (int b = 0; b < CW; ++b) rrow[b] = readlane_d(EL(x, RA - 1, b), lp);
    }
#pragma unroll
    for (int b = 0; b < CW; ++b) {
#pragma unroll
      for (int a = 0; a < RA; ++a) EL(x, a, b) = fma(-g[a], rrow[b], EL(x, a, b));
    }
    if (k + 1 < n) {   // the owner of column k + 1 publishes it
      const int w1 = (k + 1) / CW, b1 = (k + 1) - w1 * CW;
      if (w == w1) {
#pragma unroll
        for (int a = 0; a < RA; ++a) sh.colk[q ^ 1][l + 64 * a] = dyn_get(x, a, b1);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int r = l + 64 * a;
    if (r < n) {
      double* row = Mi + sh.pinv[r] * n;
      const double sc = sh.rscale[r];
#pragma unroll
      for (int b = 0; b < CW; ++b)
        if (CW * w + b < n) row[sh.perm[CW * w + b]] = sc * EL(x, a, b);
    }
  }
  __syncthreads();
  // log|det M| = sum of log|pivot_k|, off the elimination's critical path, in a fixed
  // order (strided per thread, then the workgroup sum); -inf for a zero pivot
  double lsum = 0.0;
  for (int k = tid(); k < n; k += nthreads()) lsum += log(sh.pivabs[k]);
  *logdet = wg_sum(sh.red, lsum);
  return ok;
}

// y = op(B2^q B^r) x on LDS vectors (op = transpose when adj): the source slot is
// preserved, the products ping-pong between slots s1 and s2; returns the result slot.
template <int RA, int CW>
__device__ int wg_apply(Shm<RA, CW>& sh, const double* B2, const double* B, int n, int q, int r,
                        bool adj, int src, int s1, int s2) {
  constexpr int N = 64 * RA;
  constexpr int NP = Shm<RA, CW>::NT / N;   // threads per output element (4)
  int cur = src, nxt = s1;
  // output i = tid % N, its sum over k split in NP contiguous parts (part tid / N),
  // the parts added in a fixed order; within a part the matrix loads are issued eight
  // (then four) at a time ahead of their FMAs (the sum stays in increasing k)
  auto step = [&](const double* M, bool t) {
    const int i = tid() % N, part = tid() / N;
    const int k0 = part * n / NP, k1 = (part + 1) * n / NP;
    const int64_t di = t ? 1 : n, dk = t ? n : 1;   // element (i, k) of op(M)
    double acc = 0.0;
    if (i < n) {
      const double* Mi = M + i * di;
      int k = k0;
      for (; k + 8 <= k1; k += 8) {
        double m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = Mi[(k + u) * dk];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(m[u], sh.vec[cur][k + u], acc);
      }
      if (k + 4 <= k1) {
        double m[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) m[u] = Mi[(k + u) * dk];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = fma(m[u], sh.vec[cur][k + u], acc);
        k += 4;
      }
      for (; k < k1; ++k) acc = fma(Mi[k * dk], sh.vec[cur][k], acc);
    }
    sh.red[tid()] = acc;
    __syncthreads();
    if (tid() < n) {
      double y = sh.red[tid()];
#pragma unroll
      for (int pp = 1; pp < NP; ++pp) y += sh.red[pp * N + tid()];
      sh.vec[nxt][tid()] = y;
    }
    __syncthreads();
    cur = nxt;
    nxt = (nxt == s1) ? s2 : s1;
  };
  if (!adj) {
    for (int i = 0; i < r; ++i) step(B, false);
    for (int i = 0; i < q; ++i) step(B2, false);
  } else {
    for (int i = 0; i < q; ++i) step(B2, true);
    for (int i = 0; i < r; ++i) step(B, true);
  }
  return cur;
}

// Deterministic Hager-Higham estimate of ||B2^q B^r||_1, the same steps as the
// single-matrix driver's estimator: start e/n, at most 5 sweeps, stop when the
// estimate does not grow, the sign vector repeats or the subgradient test holds,
// then the alternating-sign vector.  Slots: 0 x, 1-2 products, 3 sign, 4 previous sign.
template <int RA, int CW>
struct DevEstimator {
  Shm<RA, CW>& sh;
  const double* B2;
  const double* B;
  int n;
  int nmv;
  __device__ bool operator()(int q, int r, double* out) {
    constexpr int N = 64 * RA;
    const int t = tid();
    if (t < n) sh.vec[0][t] = (n == 1) ? 1.0 : 1.0 / n;
    __syncthreads();
    if (n == 1) {
      const int y = wg_apply(sh, B2, B, n, q, r, false, 0, 1, 2);
      nmv += q + r;
      *out = fabs(sh.vec[y][0]);
      __syncthreads();
      return true;
    }
    double est = -1.0;
    bool have_prev = false;
    for (int it = 1; it <= 5; ++it) {
      const int y = wg_apply(sh, B2, B, n, q, r, false, 0, 1, 2);
      nmv += q + r;
      const double ey = wg_sum(sh.red, t < n ? fabs(sh.vec[y][t]) : 0.0);
      if (it > 1 && ey <= est) break;
      est = ey;
      const double xi = (t < n) ? ((sh.vec[y][t] >= 0.0) ? 1.0 : -1.0) : 0.0;
      const double same = wg_sum(sh.red, (have_prev && t < n && xi == sh.vec[4][t]) ? 1.0 : 0.0);
      if (have_prev && same == (double)n) break;
      if (t < n) sh.vec[3][t] = xi;
      __syncthreads();
      const int z = wg_apply(sh, B2, B, n, q, r, true, 3, 1, 2);
      nmv += q + r;
      const double zv = (t < n) ? fabs(sh.vec[z][t]) : -1.0;
      const double ztx = wg_sum(sh.red, t < n ? sh.vec[z][t] * sh.vec[0][t] : 0.0);
      const double zmax = wg_max(sh.red, zv);
      // smallest index attaining the maximum
      const int j = N - (int)wg_max(sh.red, (t < n && zv == zmax) ? (double)(N - t) : -1.0);
      if (it > 1 && zmax <= ztx) break;
      if (t < n) {
        sh.vec[0][t] = (t == j) ? 1.0 : 0.0;
        sh.vec[4][t] = xi;
      }
      __syncthreads();
      have_prev = true;
    }
    if (t < n) sh.vec[0][t] = ((t % 2) ? -1.0 : 1.0) * (1.0 + (double)t / (n - 1));
    __syncthreads();
    const int y = wg_apply(sh, B2, B, n, q, r, false, 0, 1, 2);
    nmv += q + r;
    const double ea = 2.0 * wg_sum(sh.red, t < n ? fabs(sh.vec[y][t]) : 0.0) / (3.0 * n);
    *out = fmax(est, ea);
    return true;
  }
};

// Decision steps of Algorithm 1 (the finish test of the scaling loop and the degree
// selection), out of line: they run once per root, and keeping the tables and the
// estimator's state out of the kernel body keeps its register pressure down.
struct Decision {
  bool have_top = false, have_top1 = false;
  double e_top = 0.0, e_top1 = 0.0;
};

template <int RA, int CW>
__device__ __attribute__((noinline)) bool dev_finish_test(Shm<RA, CW>& sh, const double* B2,
                                                          const double* B, int n, double n1,
                                                          double n2, int k_max, int theta_source,
                                                          Decision* d) {
  const ThetaTable T = theta_table(theta_source);
  const SchemeSet K = scheme_set(k_max);
  const int ktop = K.k[K.n - 1];
  DevEstimator<RA, CW> est{sh, B2, B, n, 0};
  int nest = 0;
  bool ok = true;
  return finish_test(est, n1, n2, T.m[ktop], T.th[ktop], d->have_top, d->e_top, d->have_top1,
                     d->e_top1, &nest, &ok);
}

template <int RA, int CW>
__device__ __attribute__((noinline)) int dev_select_degree(Shm<RA, CW>& sh, const double* B2,
                                                           const double* B, int n, double n1,
                                                           double n2, int k_max, int theta_source,
                                                           const Decision* d) {
  const ThetaTable T = theta_table(theta_source);
  const SchemeSet K = scheme_set(k_max);
  DevEstimator<RA, CW> est{sh, B2, B, n, 0};
  int nest = 0;
  bool ok = true;
  return select_degree(est, T, K, n1, n2, d->have_top, d->e_top, d->have_top1, d->e_top1, &nest,
                       &ok);
}

__device__ __forceinline__ void wg_shift(double* B, const double* X, int n) {   // B = X - I
  for (int e = tid(); e < n * n; e += nthreads()) B[e] = X[e] - ((e / n == e % n) ? 1.0 : 0.0);
  __syncthreads();
}

// Scaled Denman-Beavers square root of X0 into Xr (eq. ScalDB).  Y, Xi, Yi are
// scratch.  Returns a status code; *iters receives the iterations used.
template <int RA, int CW>
__device__ __forceinline__ int wg_db_sqrt(Shm<RA, CW>& sh, const double* X0, double* Xr, double* Y,
                                          double* Xi, double* Yi, int n, int max_iter, int* iters) {
  constexpr int N = 64 * RA;
  const double tol = sqrt((double)n) * 1.1102230246251565e-16;
  bool scaled = true;
  double rel_prev = INFINITY, rel = INFINITY;
  for (int e = tid(); e < n * n; e += nthreads()) {
    Y[e] = (e / n == e % n) ? 1.0 : 0.0;
    Xr[e] = X0[e];
  }
  __syncthreads();
  for (int it = 1; it <= max_iter; ++it) {
    double ld[2] = {0.0, 0.0};
    for (int z = 0; z < (it > 1 ? 2 : 1); ++z)
      if (!wg_inverse(sh, z ? Y : Xr, z ? Yi : Xi, n, &ld[z])) return LOGM_ESINGULAR;
    const double mu = scaled ? exp(-(ld[0] + ld[1]) / (2.0 * n)) : 1.0;
    // X' = (mu X + Y^{-1}/mu)/2, Y' = (mu Y + X^{-1}/mu)/2; column sums of |X'-X|, |X'|
    const int j = tid() % N, g = tid() / N;
    double d = 0.0, a = 0.0;
    if (j < n) {
      constexpr int G = Shm<RA, CW>::NT / N;   // rows apart of one thread's elements
      int i = g;
      for (; i + 3 * G < n; i += 4 * G) {        // four rows' loads ahead of their stores
        double xr[4], yv[4], xv[4], yiv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = i + u * G, e = r * n + j;
          xr[u] = Xr[e];
          yv[u] = Y[e];
          xv[u] = Xi[e];
          yiv[u] = (it > 1) ? Yi[e] : ((r == j) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = (i + u * G) * n + j;
          const double xn = 0.5 * (mu * xr[u] + yiv[u] / mu);
          const double yn = 0.5 * (mu * yv[u] + xv[u] / mu);
          d += fabs(xn - xr[u]);
          a += fabs(xn);
          Xr[e] = xn;
          Y[e] = yn;
        }
      }
      for (; i < n; i += G) {
        const int e = i * n + j;
        const double yi = (it > 1) ? Yi[e] : ((i == j) ? 1.0 : 0.0);
        const double xn = 0.5 * (mu * Xr[e] + yi / mu);
        const double yn = 0.5 * (mu * Y[e] + Xi[e] / mu);
        d += fabs(xn - Xr[e]);
        a += fabs(xn);
        Xr[e] = xn;
        Y[e] = yn;
      }
    }
    const double dmax = wg_colmax<N>(sh.red, d);
    const double amax = wg_colmax<N>(sh.red, a);
    rel = dmax / amax;
    if (!isfinite(rel)) return LOGM_ENONFINITE;
    if (db_stop(rel, rel_prev, scaled, tol)) {
      *iters = it;
      return LOGM_OK;
    }
    rel_prev = rel;
  }
  *iters = max_iter;
  return (rel > 1e-6) ? LOGM_ENOCONV : LOGM_OK;
}

struct BatchArgs {
  int batch;
  const int* order;         // processing order: largest matrices first
  const int* dims;
  const int64_t* offsets;   // element offset of matrix i in A and L
  const double* A;
  double* L;
  double* ws;               // NBUF (64 RA)^2 doubles per workgroup
  int* status;              // 4 per matrix: code, s, k, packed Denman-Beavers iterations
  int* counter;             // work queue of this launch
  int64_t total_elems;      // elements of A and L
  int report_invalid;       // this launch reports blocks outside the arrays
  int split;                // class boundary: the n <= 64 class takes n <= split
  int n_max;                // largest size the workspace was sized for (<= BN_MAX)
  int k_max, max_sqrt, db_max_iter, theta_source;
  double coef[kSchemeCoefTotal];   // schemes k = 1 .. kKMax of eq. five_mult_degopt, packed
};

template <int RA, int CW>
__global__ __launch_bounds__(256 * RA, 4) void batched_logm_kernel(BatchArgs a) {
  constexpr int N = 64 * RA;
  __shared__ Shm<RA, CW> sh;
  __shared__ int s_item;
  const int64_t nn_cap = (int64_t)N * N;
  double* const base = a.ws + (int64_t)blockIdx.x * NBUF * nn_cap;
  auto buf = [&](int t) { return base + t * nn_cap; };
  for (;;) {
    if (tid() == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    // uniform in fact; readfirstlane keeps n, offsets and the loop bounds derived
    // from them in scalar registers
    const int q = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (q >= a.batch) return;   // uniform: every wave leaves together
    const int item = __builtin_amdgcn_readfirstlane(a.order[q]);
    const int n = a.dims[item];
    const int64_t off = a.offsets[item];
    // a block that lies outside the packed arrays is refused, never touched
    if (n < 1 || n > a.n_max || off < 0 || off > a.total_elems - (int64_t)n * n) {
      if (a.report_invalid && tid() == 0) {
        a.status[4 * item + 0] = LOGM_EINVAL;
        a.status[4 * item + 1] = a.status[4 * item + 2] = a.status[4 * item + 3] = 0;
      }
      continue;
    }
    if ((N == 64) ? (n > a.split) : (n <= a.split)) continue;   // the other size class
    double* X = buf(0);
    double* A2 = buf(1);
    double* B = buf(2);
    double* B2 = buf(3);
    const double* Ain = a.A + off;
    double* Lout = a.L + off;
    int code = LOGM_OK, s = 0, k = 0, dbits = 0;
    double bad = 0.0;
    for (int e = tid(); e < n * n; e += nthreads()) {
      const double v = Ain[e];
      X[e] = v;
      bad += isfinite(v) ? 0.0 : 1.0;
    }
    if (wg_sum(sh.red, bad) != 0.0) code = LOGM_ENONFINITE;
    double thtop;
    {
      const ThetaTable T = theta_table(a.theta_source);
      const SchemeSet K = scheme_set(a.k_max);
      thtop = T.th[K.k[K.n - 1]];
    }
    double n1 = 0.0, n2 = 0.0;
    Decision dec;
    if (code == LOGM_OK) {
      wg_shift(B, X, n);
      n1 = wg_norm1<N>(sh.red, B, n);
      {
        RM<RA, CW> R;
        wg_gemm(sh, R, B, B, n);   // B^2 at s = 0
        store_rm(R, B2, n);
        __syncthreads();
      }
      bool finished = n1 <= thtop;
      // at most max_sqrt roots, the finish test evaluated after each of them
      while (code == LOGM_OK && !finished) {
        n2 = wg_norm1<N>(sh.red, B2, n);
        finished = dev_finish_test(sh, B2, B, n, n1, n2, a.k_max, a.theta_source, &dec);
        if (!finished && s == a.max_sqrt) break;
        if (!finished) {
          double* t = X;   // A2 keeps the matrix whose root is taken
          X = A2;
          A2 = t;
          int its = 0;
          code = wg_db_sqrt(sh, A2, X, buf(4), buf(5), buf(6), n, a.db_max_iter, &its);
          if (s < 6) dbits |= (its < 31 ? its : 31) << (5 * s);
          ++s;
          wg_shift(B, X, n);
          n1 = wg_norm1<N>(sh.red, B, n);
          for (int e = tid(); e < n * n; e += nthreads())   // B2 = A2 - 2 X + I (eq. AI2)
            B2[e] = A2[e] - 2.0 * X[e] + ((e / n == e % n) ? 1.0 : 0.0);
          __syncthreads();
        }
      }
      if (code == LOGM_OK && !finished) code = LOGM_ENOCONV;
    }
    if (code == LOGM_OK) {
      n2 = wg_norm1<N>(sh.red, B2, n);
      k = dev_select_degree(sh, B2, B, n, n1, n2, a.k_max, a.theta_source, &dec);
      const PackedScheme S{a.coef + scheme_coef_base(k), k};
      const double scale = -ldexp(1.0, s);
      // accumulators: L_j, R_j (j = 2..k) and Z in buffers 4-6, 8..NBUF-1, A2's and
      // X's (X is free once B and B2 are formed)
      double* const spare[2] = {A2, X};
      constexpr int nhigh = NBUF - 8;
      static_assert(3 + nhigh + 2 >= 2 * kKMax - 1, "graph accumulators");
      auto acc = [&](int t) -> double* {
        return (t < 3) ? buf(4 + t) : ((t < 3 + nhigh) ? buf(5 + t) : spare[t - 3 - nhigh]);
      };
      auto Lacc = [&](int j) { return acc(2 * (j - 2)); };
      auto Racc = [&](int j) { return acc(2 * (j - 2) + 1); };
      double* Z = acc(2 * (k - 1));
      double* P = buf(7);
      // P_1 = I, P_2 = x = -B, P_3 = B2
      for (int e = tid(); e < n * n; e += nthreads()) {
        const double I = (e / n == e % n) ? 1.0 : 0.0;
        const double x = -B[e], x2 = B2[e];
        for (int j = 2; j <= k; ++j) {
          Lacc(j)[e] = S.h(j, 2) * x + S.h(j, 3) * x2;
          Racc(j)[e] = S.g(j, 2) * x + S.g(j, 3) * x2;
        }
        Z[e] = S.y(1) * I + S.y(2) * x + S.y(3) * x2;
      }
      __syncthreads();
      for (int j = 2; j <= k; ++j) {   // P_{j+2} = L_j R_j, folded into the later sums
        RM<RA, CW> R;
        wg_gemm(sh, R, Lacc(j), Racc(j), n);
        store_rm(R, P, n);
        __syncthreads();
        for (int e = tid(); e < n * n; e += nthreads()) {
          const double pv = P[e];
          for (int jp = j + 1; jp <= k; ++jp) {
            Lacc(jp)[e] = fma(S.h(jp, j + 2), pv, Lacc(jp)[e]);
            Racc(jp)[e] = fma(S.g(jp, j + 2), pv, Racc(jp)[e]);
          }
          Z[e] = fma(S.y(j + 2), pv, Z[e]);
        }
        __syncthreads();
      }
      double bad2 = 0.0;
      for (int e = tid(); e < n * n; e += nthreads()) {
        const double v = scale * Z[e];
        Lout[e] = v;
        bad2 += isfinite(v) ? 0.0 : 1.0;
      }
      if (wg_sum(sh.red, bad2) != 0.0) code = LOGM_ENONFINITE;
    }
    if (tid() == 0) {
      a.status[4 * item + 0] = code;
      a.status[4 * item + 1] = s;
      a.status[4 * item + 2] = k;
      a.status[4 * item + 3] = dbits;
    }
    __syncthreads();
  }
}

// Work-queue counters to zero and the processing order: a counting sort of the
// matrices by decreasing n (one workgroup; invalid sizes first, they are refused at
// once), so that the persistent workgroups take the longest matrices first and the
// batch does not end waiting for one large matrix started late.  Within a size the
// order is unspecified; every matrix's result is independent of it.
constexpr int ORDER_THREADS = 1024;
__global__ __launch_bounds__(ORDER_THREADS) void batched_reset_kernel(int* counters, int batch,
                                                                      const int* dims, int* order) {
  __shared__ int s_hist[BN_MAX + 2];
  __shared__ int s_pos[BN_MAX + 2];
  const int tid = threadIdx.x;
  if (tid < 2) counters[tid] = 0;
  for (int b = tid; b < BN_MAX + 2; b += ORDER_THREADS) s_hist[b] = 0;
  __syncthreads();
  // bucket 0: invalid size; bucket 1 + (BN_MAX - n): size n, largest first
  auto bucket = [&](int n) { return (n < 1 || n > BN_MAX) ? 0 : 1 + (BN_MAX - n); };
  for (int i = tid; i < batch; i += ORDER_THREADS) atomicAdd(&s_hist[bucket(dims[i])], 1);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b < BN_MAX + 1; ++b) {
      s_pos[b] = acc;
      acc += s_hist[b];
    }
  }
  __syncthreads();
  for (int i = tid; i < batch; i += ORDER_THREADS) {
    const int slot = atomicAdd(&s_pos[bucket(dims[i])], 1);
    order[min(max(slot, 0), batch - 1)] = i;
  }
}

// Resident workgroups of a size class over the whole device (the persistent grid).
template <int RA, int CW>
int class_blocks() {
  int dev = 0, ncu = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      ncu = v;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batched_logm_kernel<RA, CW>, 256 * RA, 0) ==
          hipSuccess &&
      occ > 0)
    per_cu = occ;
  return per_cu * ncu;
}

}  // namespace

// The two classes run concurrently (the small one on a second stream, forked and
// joined with events, so the call stays capturable), each in its own region.
size_t class_region_bytes(int batch, int nmax_class, int blocks) {
  return ((size_t)std::min(batch, blocks) * NBUF * nmax_class * nmax_class * sizeof(double) + 255) /
         256 * 256;
}

size_t batched_workspace_bytes(int batch, int n_max) {
  const size_t small = class_region_bytes(batch, 64, class_blocks<1, 16>());
  const size_t large = (n_max > 64) ? class_region_bytes(batch, 128, class_blocks<2, 16>()) : 0;
  return small + large + 256 + ((size_t)batch * sizeof(int) + 255) / 256 * 256;
}

namespace {
// Second stream and fork/join events per device, created on first use.
struct ForkRes {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_fork_mu;
std::map<int, ForkRes> g_fork;

// Creates nothing while `s` is being captured (the first call on a device then
// runs the classes one after the other).
bool fork_res(ForkRes& r, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_fork_mu);
  ForkRes& f = g_fork[dev];
  if (f.side == nullptr) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return false;
    if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) {
      f.side = nullptr;
      return false;
    }
    if (hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&f.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(f.side);
      f = ForkRes{};
      return false;
    }
  }
  r = f;
  return true;
}
}  // namespace

hipError_t launch_batched_logm(int batch, int n_max, const int* dims, const int64_t* offsets,
                               const double* A, double* L, int* status, void* ws, size_t ws_bytes,
                               int64_t total_elems, int k_max, int max_sqrt, int db_max_iter,
                               int theta_source, const double* coef, int split, hipStream_t s) {
  const int nb_small = std::min(batch, class_blocks<1, 16>());
  const int nb_large = std::min(batch, class_blocks<2, 16>());
  const size_t small_bytes = class_region_bytes(batch, 64, class_blocks<1, 16>());
  const size_t large_bytes = (n_max > 64) ? class_region_bytes(batch, 128, class_blocks<2, 16>()) : 0;
  const size_t order_bytes = ((size_t)batch * sizeof(int) + 255) / 256 * 256;
  if (ws_bytes < small_bytes + large_bytes + 256 + order_bytes) return hipErrorInvalidValue;
  BatchArgs a{};
  a.batch = batch;
  a.dims = dims;
  a.offsets = offsets;
  a.A = A;
  a.L = L;
  int* counters = reinterpret_cast<int*>(static_cast<char*>(ws) + small_bytes + large_bytes);
  int* order = reinterpret_cast<int*>(static_cast<char*>(ws) + small_bytes + large_bytes + 256);
  a.order = order;
  a.status = status;
  a.total_elems = total_elems;
  a.k_max = k_max;
  a.max_sqrt = max_sqrt;
  a.db_max_iter = db_max_iter;
  a.theta_source = theta_source;
  a.split = (n_max <= 64) ? 64 : std::min(std::max(split, 1), 64);
  a.n_max = n_max;
  for (int i = 0; i < kSchemeCoefTotal; ++i) a.coef[i] = coef[i];
  hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(ORDER_THREADS), 0, s, counters, batch, dims,
                     order);
  BatchArgs as = a, al = a;
  as.ws = static_cast<double*>(ws);
  as.counter = counters;
  as.report_invalid = 1;
  if (n_max <= 64) {
    hipLaunchKernelGGL((batched_logm_kernel<1, 16>), dim3(nb_small), dim3(256), 0, s, as);
    return hipGetLastError();
  }
  al.ws = reinterpret_cast<double*>(static_cast<char*>(ws) + small_bytes);
  al.counter = counters + 1;
  al.report_invalid = 0;
  ForkRes f;
  if (!fork_res(f, s)) {   // one stream: the classes one after the other
    hipLaunchKernelGGL((batched_logm_kernel<2, 16>), dim3(nb_large), dim3(512), 0, s, al);
    hipLaunchKernelGGL((batched_logm_kernel<1, 16>), dim3(nb_small), dim3(256), 0, s, as);
    return hipGetLastError();
  }
  hipError_t e;
  if ((e = hipEventRecord(f.fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(f.side, f.fork, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL((batched_logm_kernel<2, 16>), dim3(nb_large), dim3(512), 0, s, al);
  hipLaunchKernelGGL((batched_logm_kernel<1, 16>), dim3(nb_small), dim3(256), 0, f.side, as);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(f.join, f.side)) != hipSuccess) return e;
  return hipStreamWaitEvent(s, f.join, 0);
}

}  // namespace logm
