// Batched matrix logarithm for many small matrices (n <= 128): one persistent
// launch, one 256-thread workgroup per matrix at a time (taken from a device work
// queue), every step of Algorithm 1 (Section 6) on the device, decisions included:
// scaled Denman-Beavers roots (eq. ScalDB), the finish test and degree selection
// (algo.hpp, shared with the single-matrix driver), the 1-norm estimator, and the
// computation-graph polynomial (eq. five_mult_degopt) with the 2^s rescale.
//
// Register layout of an n x n matrix (n <= 128): thread (wave w, lane l) holds
// rows l and l + 64, columns 32 w .. 32 w + 31, entry (a, b) = M[l + 64 a][32 w + b];
// the pad beyond n is the identity.  Inversion is Gauss-Jordan with partial
// pivoting in these registers; products stream the right factor through LDS in
// 32-row chunks.  Per-matrix buffers live in the caller's workspace (L2-resident
// at these sizes).
#include <algorithm>

#include "algo.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "logm.h"

namespace logm {
namespace {

constexpr int BN_MAX = 128;   // largest n
constexpr int CW = 32;        // columns per wave
constexpr int KC = 32;        // rows of the right factor staged per chunk

struct Shared {
  double chunk[KC][BN_MAX + 2];     // product staging
  double rowk[2][BN_MAX];           // Gauss-Jordan: row p (the new pivot row) per parity
  double rowo[2][BN_MAX];           // Gauss-Jordan: old row k per parity
  double colk[2][BN_MAX];           // Gauss-Jordan: column k before the step, per parity
  int p[2];
  double piv[2];
  double vec[5][BN_MAX];            // estimator vectors
  double red[256];                  // reductions
  int flag;
};

__device__ __forceinline__ int tid() { return threadIdx.x; }

// ---- block reductions (fixed order, deterministic) ----------------------------
__device__ double wg_sum(Shared& sh, double v) {
  sh.red[tid()] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid() < s) sh.red[tid()] += sh.red[tid() + s];
    __syncthreads();
  }
  const double r = sh.red[0];
  __syncthreads();
  return r;
}

__device__ double wg_max(Shared& sh, double v) {
  sh.red[tid()] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid() < s) sh.red[tid()] = fmax(sh.red[tid()], sh.red[tid() + s]);
    __syncthreads();
  }
  const double r = sh.red[0];
  __syncthreads();
  return r;
}

// ||M||_1: column sums in fixed order, then the maximum.
__device__ double wg_norm1(Shared& sh, const double* M, int n) {
  double cs = 0.0;
  if (tid() < n)
    for (int i = 0; i < n; ++i) cs += fabs(M[(size_t)i * n + tid()]);
  return wg_max(sh, cs);
}

// ---- register layout -----------------------------------------------------------
struct RegMat {
  double x[2][CW];
};

__device__ void load_reg(RegMat& R, const double* M, int n) {
  const int l = tid() & 63, w = tid() >> 6;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = l + 64 * a;
#pragma unroll
    for (int b = 0; b < CW; ++b) {
      const int j = CW * w + b;
      R.x[a][b] = (i < n && j < n) ? M[(size_t)i * n + j] : (i == j ? 1.0 : 0.0);
    }
  }
}

__device__ void store_reg(const RegMat& R, double* M, int n) {
  const int l = tid() & 63, w = tid() >> 6;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = l + 64 * a;
#pragma unroll
    for (int b = 0; b < CW; ++b) {
      const int j = CW * w + b;
      if (i < n && j < n) M[(size_t)i * n + j] = R.x[a][b];
    }
  }
}

// C (registers) = A * B, A and B n x n in global memory.
__device__ void wg_gemm(Shared& sh, RegMat& C, const double* A, const double* B, int n) {
  const int l = tid() & 63, w = tid() >> 6;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < CW; ++b) C.x[a][b] = 0.0;
  for (int k0 = 0; k0 < n; k0 += KC) {
    const int kc = min(KC, n - k0);
    for (int e = tid(); e < KC * BN_MAX; e += 256) {
      const int r = e / BN_MAX, c = e % BN_MAX;
      sh.chunk[r][c] = (r < kc && c < n) ? B[(size_t)(k0 + r) * n + c] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double av[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = l + 64 * a;
        av[a] = (i < n) ? A[(size_t)i * n + k0 + kk] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < CW; ++b) {
        const double bv = sh.chunk[kk][CW * w + b];
#pragma unroll
        for (int a = 0; a < 2; ++a) C.x[a][b] = fma(av[a], bv, C.x[a][b]);
      }
    }
    __syncthreads();
  }
}

// Mi = M^{-1} by Gauss-Jordan elimination with partial pivoting (largest |entry|,
// smallest row on ties) in registers; *logdet = sum log|pivot|.  Returns false on an
// exact zero pivot.  One barrier per step: the LDS exchanges are double-buffered.
__device__ bool wg_inverse(Shared& sh, const double* M, double* Mi, int n, double* logdet) {
  const int l = tid() & 63, w = tid() >> 6;
  RegMat R;
  load_reg(R, M, n);
  __shared__ int s_perm[BN_MAX];
  double ld = 0.0;
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    const int q = k & 1;
    const int wk = k / CW, bk = k % CW;
    if (w == wk) {   // pivot search in the wave that owns column k
      double best = -1.0;
      int bi = BN_MAX;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = l + 64 * a;
        double v = -1.0;
#pragma unroll
        for (int b = 0; b < CW; ++b)
          if (b == bk) v = fabs(R.x[a][b]);
        if (i >= k && i < n && (v > best || (v == best && i < bi))) {
          best = v;
          bi = i;
        }
      }
      wave_argmax(best, bi);
      if (l == 0) {
        const int p = (bi < n) ? bi : k;
        sh.p[q] = p;
      }
      // column k before the step, every row (the pivot value included)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < CW; ++b)
          if (b == bk) v = R.x[a][b];
        sh.colk[q][l + 64 * a] = v;
      }
    }
    // old row k: its owning lane publishes its slice (it moves to row p's place)
    const int ak = k / 64, lk = k % 64;
    if (l == lk) {
#pragma unroll
      for (int b = 0; b < CW; ++b) sh.rowo[q][CW * w + b] = (ak == 0) ? R.x[0][b] : R.x[1][b];
    }
    __syncthreads();
    const int p = sh.p[q];
    const int ap = p / 64, lp = p % 64;
    // old row p (the new pivot row): its owning lane publishes its slice
    if (l == lp) {
#pragma unroll
      for (int b = 0; b < CW; ++b) sh.rowk[q][CW * w + b] = (ap == 0) ? R.x[0][b] : R.x[1][b];
    }
    // the swap: row p's place takes the old row k
    if (p != k && l == lp) {
#pragma unroll
      for (int b = 0; b < CW; ++b) {
        const double v = sh.rowo[q][CW * w + b];
        if (ap == 0) R.x[0][b] = v; else R.x[1][b] = v;
      }
    }
    const double piv = sh.colk[q][p];
    if (piv == 0.0) ok = false;
    const double rp = (piv != 0.0) ? 1.0 / piv : 0.0;
    ld += log(fabs(piv));
    if (tid() == 0) s_perm[k] = p;
    __syncthreads();
    // column k of the post-swap rows (row p now holds the old row k)
    double f[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = l + 64 * a;
      f[a] = (i == k) ? 0.0 : ((i == p) ? sh.colk[q][k] : sh.colk[q][i]);
    }
#pragma unroll
    for (int b = 0; b < CW; ++b) {
      const int j = CW * w + b;
      // the new row k scaled: its column k entry becomes 1 / piv
      const double rkb = ((j == k) ? 1.0 : sh.rowk[q][j]) * rp;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = l + 64 * a;
        const double xv = (j == k) ? 0.0 : R.x[a][b];
        R.x[a][b] = (i == k) ? rkb : fma(-f[a], rkb, xv);
      }
    }
  }
  __syncthreads();
  // undo the column permutation: the rows swapped at step k swap columns k and p
  // of the result, in reverse order
  store_reg(R, Mi, n);
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    const int p = s_perm[k];
    if (p != k && tid() < n) {
      const size_t r = (size_t)tid() * n;
      const double t = Mi[r + k];
      Mi[r + k] = Mi[r + p];
      Mi[r + p] = t;
    }
    __syncthreads();
  }
  *logdet = ld;
  return ok;
}

// y = op(B2^q B^r) x on LDS vectors (op = transpose when adj): the source slot is
// preserved, the products ping-pong between slots s1 and s2; returns the result slot.
__device__ int wg_apply(Shared& sh, const double* B2, const double* B, int n, int q, int r,
                        bool adj, int src, int s1, int s2) {
  int cur = src, nxt = s1;
  auto step = [&](const double* M, bool t) {
    double acc = 0.0;
    if (tid() < n) {
      if (!t)
        for (int k = 0; k < n; ++k) acc = fma(M[(size_t)tid() * n + k], sh.vec[cur][k], acc);
      else
        for (int k = 0; k < n; ++k) acc = fma(M[(size_t)k * n + tid()], sh.vec[cur][k], acc);
    }
    __syncthreads();
    if (tid() < n) sh.vec[nxt][tid()] = acc;
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
struct DevEstimator {
  Shared& sh;
  const double* B2;
  const double* B;
  int n;
  int nmv;
  __device__ bool operator()(int q, int r, double* out) {
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
      const double ey = wg_sum(sh, t < n ? fabs(sh.vec[y][t]) : 0.0);
      if (it > 1 && ey <= est) break;
      est = ey;
      const double xi = (t < n) ? ((sh.vec[y][t] >= 0.0) ? 1.0 : -1.0) : 0.0;
      const double same = wg_sum(sh, (t < n && xi == sh.vec[4][t]) ? 1.0 : 0.0);
      if (have_prev && same == (double)n) break;
      if (t < n) sh.vec[3][t] = xi;
      __syncthreads();
      const int z = wg_apply(sh, B2, B, n, q, r, true, 3, 1, 2);
      nmv += q + r;
      const double zv = (t < n) ? fabs(sh.vec[z][t]) : -1.0;
      const double ztx = wg_sum(sh, t < n ? sh.vec[z][t] * sh.vec[0][t] : 0.0);
      const double zmax = wg_max(sh, zv);
      // smallest index attaining the maximum
      const int j = BN_MAX - (int)wg_max(sh, (t < n && zv == zmax) ? (double)(BN_MAX - t) : -1.0);
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
    const double ea = 2.0 * wg_sum(sh, t < n ? fabs(sh.vec[y][t]) : 0.0) / (3.0 * n);
    *out = fmax(est, ea);
    return true;
  }
};

// ---- graph schemes (eq. five_mult_degopt; Table 1 for k = 5) --------------------
struct DevScheme {
  int k;
  double h[4][5], g[4][5];   // row j - 2: coefficients on P_2 .. P_{j+1}
  double y[7];               // weights of P_1 .. P_{k+2}
};

// Scheme coefficients for schemes 1, 2, 3, 5, copied from the host tables before
// every launch.
__constant__ DevScheme c_sch[4];

// Per-matrix buffers (n x n each) in the workspace: 0-1 X / A2 (they trade places
// at every root), 2 B, 3 B2, 4-6 Y and the inverses, 7 the graph product, 8-12
// with 4-6 and the free one of 0-1 the polynomial accumulators.
constexpr int NBUF = 13;

struct BatchArgs {
  int batch;
  const int* dims;
  const int64_t* offsets;   // element offset of matrix i in A and L
  const double* A;
  double* L;
  double* ws;               // NBUF * total elements
  int* status;              // 4 per matrix: code, s, k, packed Denman-Beavers iterations
  int* counter;             // work queue
  int64_t total_elems;      // elements of A, L (and of each workspace buffer)
  int k_max, max_sqrt, db_max_iter, theta_source;
};

// Elementwise helpers over n x n buffers.
__device__ void wg_shift(double* B, const double* X, int n) {   // B = X - I
  for (int e = tid(); e < n * n; e += 256) B[e] = X[e] - ((e / n == e % n) ? 1.0 : 0.0);
  __syncthreads();
}

// Scaled Denman-Beavers square root of X0 into Xr (eq. ScalDB).  Y, Xi, Yi are
// scratch.  Returns a status code; *iters receives the iterations used.
__device__ int wg_db_sqrt(Shared& sh, const double* X0, double* Xr, double* Y, double* Xi,
                          double* Yi, int n, int max_iter, int* iters) {
  const double tol = sqrt((double)n) * 1.1102230246251565e-16;
  bool scaled = true;
  double rel_prev = INFINITY, rel = INFINITY;
  for (int e = tid(); e < n * n; e += 256) {
    Y[e] = (e / n == e % n) ? 1.0 : 0.0;
    Xr[e] = X0[e];
  }
  __syncthreads();
  for (int it = 1; it <= max_iter; ++it) {
    double ldx = 0.0, ldy = 0.0;
    if (!wg_inverse(sh, Xr, Xi, n, &ldx)) return LOGM_ESINGULAR;
    if (it > 1) {
      if (!wg_inverse(sh, Y, Yi, n, &ldy)) return LOGM_ESINGULAR;
    }
    const double mu = scaled ? exp(-(ldx + ldy) / (2.0 * n)) : 1.0;
    // X' = (mu X + Y^{-1}/mu)/2, Y' = (mu Y + X^{-1}/mu)/2; column sums of |X'-X|, |X'|
    double d = 0.0, a = 0.0;
    if (tid() < n) {
      const int j = tid();
      for (int i = 0; i < n; ++i) {
        const size_t e = (size_t)i * n + j;
        const double yi = (it > 1) ? Yi[e] : ((i == j) ? 1.0 : 0.0);
        const double xn = 0.5 * (mu * Xr[e] + yi / mu);
        const double yn = 0.5 * (mu * Y[e] + Xi[e] / mu);
        d += fabs(xn - Xr[e]);
        a += fabs(xn);
        Xr[e] = xn;
        Y[e] = yn;
      }
    }
    const double dmax = wg_max(sh, d);
    const double amax = wg_max(sh, a);
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

__global__ __launch_bounds__(256) void batched_logm_kernel(BatchArgs a) {
  __shared__ Shared sh;
  __shared__ int s_item;
  for (;;) {
    if (tid() == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= a.batch) return;   // uniform: every wave leaves together
    const int n = a.dims[item];
    const int64_t off = a.offsets[item];
    // a block that lies outside the packed arrays is refused, never touched
    if (n < 1 || n > BN_MAX || off < 0 || off > a.total_elems - (int64_t)n * n) {
      if (tid() == 0) {
        a.status[4 * item + 0] = LOGM_EINVAL;
        a.status[4 * item + 1] = a.status[4 * item + 2] = a.status[4 * item + 3] = 0;
      }
      continue;
    }
    double* const base = a.ws + (int64_t)NBUF * off;
    const int64_t nn = (int64_t)n * n;
    double* X = base;
    double* A2 = base + nn;
    double* B = base + 2 * nn;
    double* B2 = base + 3 * nn;
    double* Y = base + 4 * nn;
    double* Xi = base + 5 * nn;
    double* Yi = base + 6 * nn;
    double* P = base + 7 * nn;
    const double* Ain = a.A + off;
    double* Lout = a.L + off;
    int code = LOGM_OK, s = 0, k = 0, dbits = 0;
    // input, non-finite check
    double bad = 0.0;
    for (int e = tid(); e < n * n; e += 256) {
      const double v = Ain[e];
      X[e] = v;
      bad += isfinite(v) ? 0.0 : 1.0;
    }
    if (wg_sum(sh, bad) != 0.0) code = LOGM_ENONFINITE;
    const ThetaTable T = theta_table(a.theta_source);
    const SchemeSet K = scheme_set(a.k_max);
    const int ktop = K.k[K.n - 1];
    const int mtop = T.m[ktop];
    const double thtop = T.th[ktop];
    DevEstimator est{sh, B2, B, n, 0};
    double n1 = 0.0, n2 = 0.0;
    bool have_top = false, have_top1 = false;
    double e_top = 0.0, e_top1 = 0.0;
    if (code == LOGM_OK) {
      wg_shift(B, X, n);
      n1 = wg_norm1(sh, B, n);
      {
        RegMat R;
        wg_gemm(sh, R, B, B, n);   // B^2 at s = 0
        store_reg(R, B2, n);
        __syncthreads();
      }
      bool finished = n1 <= thtop;
      while (code == LOGM_OK && !finished && s < a.max_sqrt) {
        n2 = wg_norm1(sh, B2, n);
        int nest = 0;
        bool ok = true;
        finished = finish_test(est, n1, n2, mtop, thtop, have_top, e_top, have_top1, e_top1,
                               &nest, &ok);
        if (!finished) {
          double* t = X;   // A2 keeps the matrix whose root is taken
          X = A2;
          A2 = t;
          int its = 0;
          code = wg_db_sqrt(sh, A2, X, Y, Xi, Yi, n, a.db_max_iter, &its);
          if (s < 6) dbits |= (its < 31 ? its : 31) << (5 * s);
          ++s;
          wg_shift(B, X, n);
          n1 = wg_norm1(sh, B, n);
          for (int e = tid(); e < n * n; e += 256)   // B2 = A2 - 2 X + I (eq. AI2)
            B2[e] = A2[e] - 2.0 * X[e] + ((e / n == e % n) ? 1.0 : 0.0);
          __syncthreads();
        }
      }
      if (code == LOGM_OK && !finished) code = LOGM_ENOCONV;
    }
    if (code == LOGM_OK) {
      n2 = wg_norm1(sh, B2, n);
      int nest = 0;
      bool ok = true;
      k = select_degree(est, T, K, n1, n2, have_top, e_top, have_top1, e_top1, &nest, &ok);
      const DevScheme& S = c_sch[k == 5 ? 3 : k - 1];
      const double scale = -ldexp(1.0, s);
      // accumulators: L_j, R_j (j = 2..k) and Z in buffers 4-6, 8-12 and A2's
      auto acc = [&](int t) -> double* {
        return (t < 3) ? base + (4 + t) * nn : ((t < 8) ? base + (5 + t) * nn : A2);
      };
      auto Lacc = [&](int j) { return acc(2 * (j - 2)); };
      auto Racc = [&](int j) { return acc(2 * (j - 2) + 1); };
      double* Z = acc(2 * (k - 1));
      // P_1 = I, P_2 = x = -B, P_3 = B2
      for (int e = tid(); e < n * n; e += 256) {
        const double I = (e / n == e % n) ? 1.0 : 0.0;
        const double x = -B[e], x2 = B2[e];
        for (int j = 2; j <= k; ++j) {
          Lacc(j)[e] = S.h[j - 2][0] * x + S.h[j - 2][1] * x2;
          Racc(j)[e] = S.g[j - 2][0] * x + S.g[j - 2][1] * x2;
        }
        Z[e] = S.y[0] * I + S.y[1] * x + S.y[2] * x2;
      }
      __syncthreads();
      for (int j = 2; j <= k; ++j) {   // P_{j+2} = L_j R_j, folded into the later sums
        RegMat R;
        wg_gemm(sh, R, Lacc(j), Racc(j), n);
        store_reg(R, P, n);
        __syncthreads();
        for (int e = tid(); e < n * n; e += 256) {
          const double pv = P[e];
          for (int jp = j + 1; jp <= k; ++jp) {
            Lacc(jp)[e] = fma(S.h[jp - 2][j], pv, Lacc(jp)[e]);
            Racc(jp)[e] = fma(S.g[jp - 2][j], pv, Racc(jp)[e]);
          }
          Z[e] = fma(S.y[j + 1], pv, Z[e]);
        }
        __syncthreads();
      }
      double bad2 = 0.0;
      for (int e = tid(); e < n * n; e += 256) {
        const double v = scale * Z[e];
        Lout[e] = v;
        bad2 += isfinite(v) ? 0.0 : 1.0;
      }
      if (wg_sum(sh, bad2) != 0.0) code = LOGM_ENONFINITE;
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

__global__ void batched_reset_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

}  // namespace

size_t batched_workspace_bytes(int64_t total_elems) {
  return (size_t)NBUF * (size_t)total_elems * sizeof(double) + 256;
}

hipError_t launch_batched_logm(int batch, const int* dims, const int64_t* offsets,
                               const double* A, double* L, int* status, void* ws,
                               int64_t total_elems, int k_max, int max_sqrt, int db_max_iter,
                               int theta_source, const double (*h)[4][5],
                               const double (*g)[4][5], const double (*y)[7], int nblocks,
                               hipStream_t s) {
  BatchArgs a{};
  a.batch = batch;
  a.dims = dims;
  a.offsets = offsets;
  a.A = A;
  a.L = L;
  a.ws = static_cast<double*>(ws);
  a.counter = reinterpret_cast<int*>(static_cast<char*>(ws) +
                                     (size_t)NBUF * (size_t)total_elems * sizeof(double));
  a.status = status;
  a.total_elems = total_elems;
  a.k_max = k_max;
  a.max_sqrt = max_sqrt;
  a.db_max_iter = db_max_iter;
  a.theta_source = theta_source;
  DevScheme sch[4];
  const int ks[4] = {1, 2, 3, 5};
  for (int i = 0; i < 4; ++i) {
    sch[i].k = ks[i];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 5; ++c) {
        sch[i].h[r][c] = h[i][r][c];
        sch[i].g[r][c] = g[i][r][c];
      }
    for (int c = 0; c < 7; ++c) sch[i].y[c] = y[i][c];
  }
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_sch), sch, sizeof(sch), 0,
                                        hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, s, a.counter);
  hipLaunchKernelGGL(batched_logm_kernel, dim3(std::min(nblocks, batch)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace logm
