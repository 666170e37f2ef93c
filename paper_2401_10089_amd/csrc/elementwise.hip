// Bandwidth-bound kernels of the logm path (gfx950): the Denman-Beavers update
// (eq. ScalDB) with the inverse's column order folded into its reads, the shifted
// matrices B = X - I and B^2 = A_2 - 2X + I (eq. AI2), exact 1-norms through
// deterministic column-sum partials, matrix-vector products for the 1-norm
// estimator, and the linear combinations that seed the graph accumulators.
//
// Row-block kernels: workgroup b owns rows [b*rpb, (b+1)*rpb) and walks the columns
// in chunks of 256 (one column per thread, coalesced), keeping per-column partial
// sums in registers; partial sums are reduced in a fixed order, so every norm is
// bitwise reproducible.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace logm {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ void row_range(int n, int nblk, int& i0, int& i1) {
  const int rpb = (n + nblk - 1) / nblk;
  i0 = blockIdx.x * rpb;
  i1 = min(n, i0 + rpb);
}

// Padded workspace matrices are n_pad x n_pad with the valid n x n block in the
// corner; X-like matrices carry the identity on the pad and B-like ones zero, so
// every matrix is block diagonal and the pad never mixes into the valid block.
// Row-block kernels below write the whole padded range and sum norms over the
// valid block only.

// Four times the usual workgroup: one row block per workgroup is all the partial-sum
// layout allows, and the column gathers through the inverses' row maps need more
// waves in flight than one per SIMD.  Each column still has one thread, which sums
// its rows in order.
constexpr int DB_TPB = 4 * TPB;
__global__ __launch_bounds__(DB_TPB) void db_update_kernel(DbArgs a, int nblk) {
  __shared__ double s_mu;
  const int n = a.n;
  const int np = (int)a.ld;
  if (threadIdx.x == 0) {
    double sx = 0.0, sy = 0.0;
    for (int t = 0; t < a.nslots; ++t) sx += a.ldx[t];
    if (a.ldy != nullptr)
      for (int t = 0; t < a.nslots; ++t) sy += a.ldy[t];
    const double mu = a.scaled ? exp(-(sx + sy) / (2.0 * n)) : 1.0;
    s_mu = mu;
    if (blockIdx.x == 0) *a.mu_out = mu;
  }
  __syncthreads();
  const double mu = s_mu;
  int i0, i1;
  row_range(np, nblk, i0, i1);
  double* p0 = a.part + (int64_t)blockIdx.x * n;
  double* p1 = a.part + (int64_t)(nblk + blockIdx.x) * n;
  for (int c = threadIdx.x; c < np; c += DB_TPB) {
    const int qx = a.px[c];
    const int qy = (a.py != nullptr) ? a.py[c] : -1;
    double sdiff = 0.0, snew = 0.0;
    if (c >= n) {   // pad column: identity
      for (int i = i0; i < i1; ++i) {
        const int64_t o = (int64_t)i * a.ld;
        a.Xout[o + c] = (i == c) ? 1.0 : 0.0;
        a.Yout[o + c] = (i == c) ? 1.0 : 0.0;
      }
      continue;
    }
    // groups of RG rows: every load of the group is issued before its stores (the
    // update is in place, so loads may not pass stores otherwise); sums in row order
    constexpr int RG = 4;
    for (int ib = i0; ib < i1; ib += RG) {
      double x[RG], y[RG], xi[RG], yi[RG];
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const int i = min(ib + r, i1 - 1);
        const int64_t o = (int64_t)i * a.ld;
        const bool valid = i < n;
        x[r] = valid ? a.Xin[o + c] : 0.0;
        y[r] = (valid && a.Yin != nullptr) ? a.Yin[o + c] : (i == c ? 1.0 : 0.0);
        xi[r] = valid ? a.Xinv[o + qx] : 0.0;
        yi[r] = (valid && qy >= 0) ? a.Yinv[o + qy] : (i == c ? 1.0 : 0.0);
      }
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const int i = ib + r;
        if (i >= i1) break;
        const int64_t o = (int64_t)i * a.ld;
        if (i >= n) {   // pad row: identity
          a.Xout[o + c] = (i == c) ? 1.0 : 0.0;
          a.Yout[o + c] = (i == c) ? 1.0 : 0.0;
          continue;
        }
        const double xn = 0.5 * (mu * x[r] + yi[r] / mu);
        const double yn = 0.5 * (mu * y[r] + xi[r] / mu);
        a.Xout[o + c] = xn;
        a.Yout[o + c] = yn;
        sdiff += fabs(xn - x[r]);
        snew += fabs(xn);
      }
    }
    if (c < n) {
      p0[c] = sdiff;
      p1[c] = snew;
    }
  }
}

// Sum over the nblk row-block partials part[b][c] for the 64 columns of this
// workgroup: wave w adds blocks w, w + 4, ... for column c = 64 blockIdx.x + lane
// (coalesced rows), then the four wave sums are added in a fixed order.  The result
// is valid in wave 0.
constexpr int CS_COLS = 64;
__device__ __forceinline__ double colsum64(const double* part, int nblk, int n, double* s_red) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * CS_COLS + lane;
  double s = 0.0;
  if (c < n)
    for (int b = w; b < nblk; b += TPB / 64) s += part[(int64_t)b * n + c];
  s_red[w * 64 + lane] = s;
  __syncthreads();
  return (s_red[lane] + s_red[64 + lane]) + (s_red[128 + lane] + s_red[192 + lane]);
}

__global__ __launch_bounds__(TPB) void colsum_blockmax_kernel(const double* part, int nblk, int n,
                                                              double* bm) {
  __shared__ double s_red[TPB];
  const int q = blockIdx.y;
  const double t = colsum64(part + (int64_t)q * nblk * n, nblk, n, s_red);
  if (threadIdx.x < 64) {
    const int c = blockIdx.x * CS_COLS + threadIdx.x;
    const double m = wave_max(c < n ? t : 0.0);
    if (threadIdx.x == 0) bm[q * gridDim.x + blockIdx.x] = m;
  }
}

__global__ void max_reduce_kernel(const double* bm, int nb, double* out) {
  const int q = blockIdx.x;
  double m = 0.0;
  for (int t = threadIdx.x; t < nb; t += 64) m = fmax(m, bm[q * nb + t]);
  m = wave_max(m);
  if (threadIdx.x == 0) out[q] = m;
}

__global__ __launch_bounds__(TPB) void shift_kernel(const double* X, double* B, int n, int64_t ld,
                                                    double* part, int nblk) {
  const int np = (int)ld;
  int i0, i1;
  row_range(np, nblk, i0, i1);
  double* p = part + (int64_t)blockIdx.x * n;
  for (int c = threadIdx.x; c < np; c += TPB) {
    double s = 0.0;
    for (int i = i0; i < i1; ++i) {
      const int64_t o = (int64_t)i * ld + c;
      const double b = X[o] - (i == c ? 1.0 : 0.0);
      B[o] = b;
      if (i < n) s += fabs(b);
    }
    if (c < n) p[c] = s;
  }
}

__global__ __launch_bounds__(TPB) void b2_kernel(const double* A2, const double* X, double* B2,
                                                 int n, int64_t ld, double* part, int nblk) {
  const int np = (int)ld;
  int i0, i1;
  row_range(np, nblk, i0, i1);
  double* p = part + (int64_t)blockIdx.x * n;
  for (int c = threadIdx.x; c < np; c += TPB) {
    double s = 0.0;
    for (int i = i0; i < i1; ++i) {
      const int64_t o = (int64_t)i * ld + c;
      const double v = A2[o] - 2.0 * X[o] + (i == c ? 1.0 : 0.0);
      B2[o] = v;
      if (i < n) s += fabs(v);
    }
    if (c < n) p[c] = s;
  }
}

__global__ __launch_bounds__(TPB) void abs_colsum_kernel(const double* M, int n, int64_t ld,
                                                         double* part, int nblk) {
  int i0, i1;
  row_range(n, nblk, i0, i1);
  double* p = part + (int64_t)blockIdx.x * n;
  for (int c = threadIdx.x; c < n; c += TPB) {
    double s = 0.0;
    for (int i = i0; i < i1; ++i) s += fabs(M[(int64_t)i * ld + c]);
    p[c] = s;
  }
}

__global__ void load_padded_kernel(const double* src, int64_t lds, double* dst, int n, int n_pad,
                                   double padval, int* nonfinite) {
  const int i = blockIdx.y;
  bool bad = false;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_pad; j += gridDim.x * blockDim.x) {
    double v;
    if (i < n && j < n) {
      v = src[(int64_t)i * lds + j];
      bad |= !isfinite(v);
    } else {
      v = (i == j) ? padval : 0.0;
    }
    dst[(int64_t)i * n_pad + j] = v;
  }
  if (bad && nonfinite != nullptr) atomicOr(nonfinite, 1);
}

__global__ void copy_kernel(const double* src, double* dst, size_t count) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// y[i] = sum_c M[i][c] x[c]: one wave per row.
__global__ __launch_bounds__(TPB) void gemv_n_kernel(const double* M, int64_t ld, int n,
                                                     const double* x, double* y) {
  const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  const double* r = M + (int64_t)row * ld;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s = fma(r[c], x[c], s);
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// partial z over a row block: part[b][c] = sum_{i in block b} M[i][c] x[i]
__global__ __launch_bounds__(TPB) void gemv_t_part_kernel(const double* M, int64_t ld, int n,
                                                          const double* x, double* part, int nblk) {
  int i0, i1;
  row_range(n, nblk, i0, i1);
  const int c = blockIdx.y * TPB + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s = fma(M[(int64_t)i * ld + c], x[i], s);
  part[(int64_t)blockIdx.x * n + c] = s;
}

__global__ __launch_bounds__(TPB) void gemv_t_reduce_kernel(const double* part, int nblk, int n,
                                                            double* z) {
  __shared__ double s_red[TPB];
  const double t = colsum64(part, nblk, n, s_red);
  const int c = blockIdx.x * CS_COLS + threadIdx.x;
  if (threadIdx.x < 64 && c < n) z[c] = t;
}

__global__ void lincomb_init_kernel(LincombArgs a) {
  const int i = blockIdx.y;
  const int np = (int)a.ld;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < np; j += gridDim.x * blockDim.x) {
    const int64_t o = (int64_t)i * a.ld + j;
    const bool valid = i < a.n && j < a.n;
    const double p2 = valid ? a.P2[o] : 0.0;
    const double p3 = valid ? a.P3[o] : 0.0;
    const double d = (valid && i == j) ? 1.0 : 0.0;
    for (int t = 0; t < a.nout; ++t) a.out[t][o] = a.c2[t] * p2 + a.c3[t] * p3 + a.c1[t] * d;
  }
}

__global__ void scale_out_kernel(const double* src, int64_t ld, double* dst, int64_t ldd, int n,
                                 double scale, int* nonfinite) {
  const int i = blockIdx.y;
  bool bad = false;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double v = scale * src[(int64_t)i * ld + j];
    bad |= !isfinite(v);
    dst[(int64_t)i * ldd + j] = v;
  }
  if (bad && nonfinite != nullptr) atomicOr(nonfinite, 1);
}

__global__ void check_finite_kernel(const double* M, int64_t ld, int n, int* flag) {
  const int i = blockIdx.y;
  bool bad = false;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    bad |= !isfinite(M[(int64_t)i * ld + j]);
  if (bad) atomicOr(flag, 1);
}

// out[e] = beta out[e] + sum_t c[t] in[t][e] over the valid n x n block (row stride ld);
// out may be one of the inputs (each element is read before it is written).
__global__ void lincomb_gen_kernel(LincombGen a) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += gridDim.x * blockDim.x) {
    const int64_t o = (int64_t)i * a.ld + j;
    double v = (a.beta != 0.0) ? a.beta * a.out[o] : 0.0;
    for (int t = 0; t < a.m; ++t) v = fma(a.c[t], a.in[t][o], v);
    a.out[o] = v;
  }
}

// dst[j][i] = scale * src[i][j] for i, j < n, through 32 x 32 LDS tiles (one padding
// column avoids bank conflicts); reads and writes are both coalesced.
__global__ __launch_bounds__(256) void transpose_kernel(const double* src, int64_t lds, double* dst,
                                                        int64_t ldd, int n, double scale) {
  __shared__ double t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int i = r0 + r, j = c0 + tx;
    t[r][tx] = (i < n && j < n) ? src[(int64_t)i * lds + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = c0 + r, j = r0 + tx;   // dst row = src column
    if (i < n && j < n) dst[(int64_t)i * ldd + j] = scale * t[tx][r];
  }
}

// Balancing (steps 1 and 14 of Algorithm 1), in place on the n x n block (row stride
// ld), in one workgroup.  With perm != null, first the permutation step: while some
// index of the active range [lo, hi] has a row with no nonzero off the diagonal among
// the active columns, the largest such index is exchanged with hi (rows and columns)
// and hi drops by one; then, while some index has such a column among the active
// rows, the smallest is exchanged with lo and lo rises by one.  Counts of the active
// off-diagonal nonzeros of every row and column (cnt, 2n ints) are formed once and
// updated per isolated index, so the step costs O(n^2) in all.  perm[i] receives the
// original index at position i.  Then B = T^{-1} B T with T = diag(d), d_i powers of
// two, by Gauss-Seidel sweeps over the active indices: index i takes the power of two
// f that brings the 2-norms of its column (c) and row (r) over the active range within
// a factor 2 of each other, and keeps it only if c + r drops below 0.95 of its old
// value; an index with a zero or overflowing norm is skipped; sweeps stop when no
// index changes (at most max_sweeps).  Every update is an exchange or an exact
// power-of-two scaling.
constexpr int BAL_T = 1024;
__device__ void bal_exchange(double* M, int64_t ld, int n, int a, int b, int* perm, int* rc,
                             int* cc) {
  const int t = threadIdx.x;
  if (a != b) {
    for (int k = t; k < n; k += BAL_T) {
      const double x = M[(int64_t)a * ld + k];
      M[(int64_t)a * ld + k] = M[(int64_t)b * ld + k];
      M[(int64_t)b * ld + k] = x;
    }
    __syncthreads();
    for (int k = t; k < n; k += BAL_T) {
      const double x = M[(int64_t)k * ld + a];
      M[(int64_t)k * ld + a] = M[(int64_t)k * ld + b];
      M[(int64_t)k * ld + b] = x;
    }
    if (t == 0) {
      int v = perm[a]; perm[a] = perm[b]; perm[b] = v;
      v = rc[a]; rc[a] = rc[b]; rc[b] = v;
      v = cc[a]; cc[a] = cc[b]; cc[b] = v;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(BAL_T) void balance_kernel(double* M, int64_t ld, int n, double* d,
                                                        int max_sweeps, int* sweeps_out, int* perm,
                                                        int* cnt) {
  __shared__ double red[2][BAL_T / 64];
  __shared__ int s_pick;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += BAL_T) d[i] = 1.0;
  int lo = 0, hi = n - 1;
  if (perm != nullptr) {
    int* rc = cnt;       // active off-diagonal nonzeros of row i
    int* cc = cnt + n;   // ... and of column i
    for (int i = t; i < n; i += BAL_T) {
      perm[i] = i;
      int r = 0, c = 0;
      for (int k = 0; k < n; ++k)
        if (k != i) {
          r += (M[(int64_t)i * ld + k] != 0.0);
          c += (M[(int64_t)k * ld + i] != 0.0);
        }
      rc[i] = r;
      cc[i] = c;
    }
    __syncthreads();
    while (hi > lo) {    // isolated rows to the bottom, the largest index first
      if (t == 0) s_pick = -1;
      __syncthreads();
      int best = -1;
      for (int j = lo + t; j <= hi; j += BAL_T)
        if (rc[j] == 0) best = j;
      if (best >= 0) atomicMax(&s_pick, best);
      __syncthreads();
      const int j = s_pick;
      if (j < 0) break;  // uniform
      // column j leaves the active range: rows with a nonzero there lose one
      for (int r = lo + t; r <= hi; r += BAL_T)
        if (r != j && M[(int64_t)r * ld + j] != 0.0) rc[r] -= 1;
      __syncthreads();
      bal_exchange(M, ld, n, j, hi, perm, rc, cc);
      --hi;
    }
    while (hi > lo) {    // isolated columns to the top, the smallest index first
      if (t == 0) s_pick = n;
      __syncthreads();
      int best = n;
      for (int j = hi - t; j >= lo; j -= BAL_T)
        if (cc[j] == 0) best = j;
      if (best < n) atomicMin(&s_pick, best);
      __syncthreads();
      const int j = s_pick;
      if (j >= n) break;  // uniform
      // row j leaves the active range: columns with a nonzero there lose one
      for (int c = lo + t; c <= hi; c += BAL_T)
        if (c != j && M[(int64_t)j * ld + c] != 0.0) cc[c] -= 1;
      __syncthreads();
      bal_exchange(M, ld, n, j, lo, perm, rc, cc);
      ++lo;
    }
  }
  int sweeps = 0;
  for (int sw = 1; sw <= max_sweeps; ++sw) {
    sweeps = sw;
    bool changed = false;
    for (int i = lo; i <= hi; ++i) {
      double cs = 0.0, rs = 0.0;
      for (int k = lo + t; k <= hi; k += BAL_T) {
        const double a = M[(int64_t)k * ld + i];
        const double b = M[(int64_t)i * ld + k];
        cs = fma(a, a, cs);
        rs = fma(b, b, rs);
      }
      cs = wave_sum(cs);
      rs = wave_sum(rs);
      if ((t & 63) == 0) {
        red[0][t >> 6] = cs;
        red[1][t >> 6] = rs;
      }
      __syncthreads();
      double c2 = 0.0, r2 = 0.0;
      for (int w = 0; w < BAL_T / 64; ++w) {
        c2 += red[0][w];
        r2 += red[1][w];
      }
      __syncthreads();
      double c = sqrt(c2), r = sqrt(r2);
      if (c == 0.0 || r == 0.0 || !isfinite(c) || !isfinite(r)) continue;   // uniform
      const double before = c + r;
      double f = 1.0;
      while (c < r / 2.0) {
        c *= 2.0;
        r /= 2.0;
        f *= 2.0;
      }
      while (c >= 2.0 * r) {
        c /= 2.0;
        r *= 2.0;
        f /= 2.0;
      }
      if (c + r < 0.95 * before) {   // uniform
        changed = true;
        const double g = 1.0 / f;    // exact: f is a power of two
        if (t == 0) d[i] *= f;
        // the same thread scales row i then column i at k = i, so a_ii comes back
        for (int k = t; k < n; k += BAL_T) M[(int64_t)i * ld + k] *= g;
        for (int k = t; k < n; k += BAL_T) M[(int64_t)k * ld + i] *= f;
        __syncthreads();
      }
    }
    if (!changed) break;
  }
  if (t == 0 && sweeps_out != nullptr) *sweeps_out = sweeps;
}

// L[perm[i]][perm[j]] = LB[i][j] d[i] / d[j]: L = P T LB T^{-1} P^T (exact, powers
// of two and an exchange of entries).
__global__ void unbalance_perm_kernel(const double* LB, int64_t ldb, double* L, int64_t ldl, int n,
                                      const double* d, const int* perm) {
  const int i = blockIdx.y;
  const double di = d[i];
  const int64_t pi = perm[i];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    L[pi * ldl + perm[j]] = LB[(int64_t)i * ldb + j] * (di / d[j]);
}

// Complex input through its real representation: P (2n x 2n, row stride ldp) =
// [[Re A, -Im A], [Im A, Re A]] from A (n x n complex, interleaved (re, im), row
// stride lda in complex elements).  The map is an injective algebra homomorphism,
// so P^{1/2}, P^{-1} and log P are the images of A^{1/2}, A^{-1} and log A.
__global__ void embed_complex_kernel(const double* A, int64_t lda, int n, double* P, int64_t ldp) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double re = A[2 * ((int64_t)i * lda + j)];
    const double im = A[2 * ((int64_t)i * lda + j) + 1];
    P[(int64_t)i * ldp + j] = re;
    P[(int64_t)i * ldp + n + j] = -im;
    P[(int64_t)(n + i) * ldp + j] = im;
    P[(int64_t)(n + i) * ldp + n + j] = re;
  }
}

// L (n x n complex, interleaved, row stride ldl) from the left block column of its
// real representation R (2n x 2n, row stride ldr): Re L = R[0:n, 0:n], Im L = R[n:2n, 0:n].
__global__ void extract_complex_kernel(const double* R, int64_t ldr, int n, double* L, int64_t ldl) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    L[2 * ((int64_t)i * ldl + j)] = R[(int64_t)i * ldr + j];
    L[2 * ((int64_t)i * ldl + j) + 1] = R[(int64_t)(n + i) * ldr + j];
  }
}

// Batched real representations (complex batch, n_i <= 64): matrix i of the complex
// packing (n_i x n_i interleaved at element offset off[i]) becomes the 2n_i x 2n_i
// real block at offset 4 off[i] (non-overlapping when the complex blocks are).  A
// matrix whose size or block is out of range gets real size 0, which the batched
// kernel reports as invalid and leaves alone.
__global__ void batch_complex_prep_kernel(int batch, int n_lim, int64_t total, const int* dims,
                                          const int64_t* off, int* dims2, int64_t* off2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += gridDim.x * blockDim.x) {
    const int n = dims[i];
    const int64_t o = off[i];
    const bool ok = n >= 1 && n <= n_lim && o >= 0 && o + (int64_t)n * n <= total;
    dims2[i] = ok ? 2 * n : 0;
    off2[i] = ok ? 4 * o : 0;
  }
}

// One workgroup per matrix: P_i = [[Re A_i, -Im A_i], [Im A_i, Re A_i]].
__global__ void batch_embed_complex_kernel(const double* A, const int* dims2, const int64_t* off2,
                                           double* P) {
  const int i = blockIdx.x;
  const int m = dims2[i];
  if (m == 0) return;
  const int n = m / 2;
  const int64_t oc = off2[i] / 4;
  double* Pi = P + off2[i];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    const double re = A[2 * (oc + e)];
    const double im = A[2 * (oc + e) + 1];
    Pi[(int64_t)r * m + c] = re;
    Pi[(int64_t)r * m + n + c] = -im;
    Pi[(int64_t)(n + r) * m + c] = im;
    Pi[(int64_t)(n + r) * m + n + c] = re;
  }
}

// One workgroup per matrix: L_i from the left block column of log P_i.
__global__ void batch_extract_complex_kernel(const double* R, const int* dims2, const int64_t* off2,
                                             double* L) {
  const int i = blockIdx.x;
  const int m = dims2[i];
  if (m == 0) return;
  const int n = m / 2;
  const int64_t oc = off2[i] / 4;
  const double* Ri = R + off2[i];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e % n;
    L[2 * (oc + e)] = Ri[(int64_t)r * m + c];
    L[2 * (oc + e) + 1] = Ri[(int64_t)(n + r) * m + c];
  }
}

// Well-conditioned test matrix for timing runs: I + 0.5 u_ij / sqrt(n) with u_ij in
// [-1, 1) from an integer hash of (seed, i, j); identity on the pad.
__global__ void fill_test_matrix_kernel(double* M, int n, int n_pad, unsigned seed) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_pad; j += gridDim.x * blockDim.x) {
    double v = (i == j) ? 1.0 : 0.0;
    if (i < n && j < n) {
      unsigned h = seed ^ (0x9e3779b9u * (unsigned)(i + 1)) ^ (0x85ebca6bu * (unsigned)(j + 7));
      h ^= h >> 16;
      h *= 0x7feb352du;
      h ^= h >> 15;
      h *= 0x846ca68bu;
      h ^= h >> 16;
      v += 0.5 * ((double)h * (2.0 / 4294967296.0) - 1.0) / sqrt((double)n);
    }
    M[(int64_t)i * n_pad + j] = v;
  }
}

inline dim3 row_grid(int n, int rows) { return dim3((unsigned)std::min(8, (n + 255) / 256), (unsigned)rows); }

}  // namespace

hipError_t launch_db_update(const DbArgs& a, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(db_update_kernel, dim3(nblk), dim3(DB_TPB), 0, s, a, nblk);
  return hipGetLastError();
}

hipError_t launch_colsum_max(const double* part, int nq, int nblk, int n, double* out,
                             double* bm, hipStream_t s) {
  const int gx = (n + CS_COLS - 1) / CS_COLS;
  hipLaunchKernelGGL(colsum_blockmax_kernel, dim3(gx, nq), dim3(TPB), 0, s, part, nblk, n, bm);
  hipLaunchKernelGGL(max_reduce_kernel, dim3(nq), dim3(64), 0, s, bm, gx, out);
  return hipGetLastError();
}

hipError_t launch_shift(const double* X, double* B, int n, int64_t ld, double* part, int nblk,
                        hipStream_t s) {
  hipLaunchKernelGGL(shift_kernel, dim3(nblk), dim3(TPB), 0, s, X, B, n, ld, part, nblk);
  return hipGetLastError();
}

hipError_t launch_b2_from_root(const double* A2, const double* X, double* B2, int n, int64_t ld,
                               double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(b2_kernel, dim3(nblk), dim3(TPB), 0, s, A2, X, B2, n, ld, part, nblk);
  return hipGetLastError();
}

hipError_t launch_abs_colsum(const double* M, int n, int64_t ld, double* part, int nblk,
                             hipStream_t s) {
  hipLaunchKernelGGL(abs_colsum_kernel, dim3(nblk), dim3(TPB), 0, s, M, n, ld, part, nblk);
  return hipGetLastError();
}

hipError_t launch_load_padded(const double* src, int64_t lds, double* dst, int n, int n_pad,
                              double padval, int* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(load_padded_kernel, row_grid(n_pad, n_pad), dim3(256), 0, s, src, lds, dst, n,
                     n_pad, padval, nonfinite);
  return hipGetLastError();
}

hipError_t launch_lincomb_gen(const LincombGen& a, hipStream_t s) {
  if (a.m < 0 || a.m > LincombGen::kMax || a.n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lincomb_gen_kernel, row_grid(a.n, a.n), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd, int n,
                            double scale, hipStream_t s) {
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, dim3(t, t), dim3(256), 0, s, src, lds, dst, ldd, n, scale);
  return hipGetLastError();
}

hipError_t launch_balance(double* M, int64_t ld, int n, double* d, int max_sweeps, int* sweeps,
                          int* perm, int* cnt, hipStream_t s) {
  if (perm != nullptr && cnt == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(balance_kernel, dim3(1), dim3(BAL_T), 0, s, M, ld, n, d, max_sweeps, sweeps,
                     perm, cnt);
  return hipGetLastError();
}

hipError_t launch_unbalance_perm(const double* LB, int64_t ldb, double* L, int64_t ldl, int n,
                                 const double* d, const int* perm, hipStream_t s) {
  hipLaunchKernelGGL(unbalance_perm_kernel, row_grid(n, n), dim3(256), 0, s, LB, ldb, L, ldl, n, d,
                     perm);
  return hipGetLastError();
}

hipError_t launch_embed_complex(const double* A, int64_t lda, int n, double* P, int64_t ldp,
                                hipStream_t s) {
  hipLaunchKernelGGL(embed_complex_kernel, row_grid(n, n), dim3(256), 0, s, A, lda, n, P, ldp);
  return hipGetLastError();
}

hipError_t launch_extract_complex(const double* R, int64_t ldr, int n, double* L, int64_t ldl,
                                  hipStream_t s) {
  hipLaunchKernelGGL(extract_complex_kernel, row_grid(n, n), dim3(256), 0, s, R, ldr, n, L, ldl);
  return hipGetLastError();
}

hipError_t launch_batch_complex_prep(int batch, int n_lim, int64_t total, const int* dims,
                                     const int64_t* off, int* dims2, int64_t* off2, hipStream_t s) {
  const int blocks = std::min((batch + 255) / 256, 1024);
  hipLaunchKernelGGL(batch_complex_prep_kernel, dim3(blocks), dim3(256), 0, s, batch, n_lim, total,
                     dims, off, dims2, off2);
  return hipGetLastError();
}

hipError_t launch_batch_embed_complex(int batch, const double* A, const int* dims2,
                                      const int64_t* off2, double* P, hipStream_t s) {
  hipLaunchKernelGGL(batch_embed_complex_kernel, dim3(batch), dim3(256), 0, s, A, dims2, off2, P);
  return hipGetLastError();
}

hipError_t launch_batch_extract_complex(int batch, const double* R, const int* dims2,
                                        const int64_t* off2, double* L, hipStream_t s) {
  hipLaunchKernelGGL(batch_extract_complex_kernel, dim3(batch), dim3(256), 0, s, R, dims2, off2, L);
  return hipGetLastError();
}

hipError_t launch_fill_test_matrix(double* M, int n, int n_pad, unsigned seed, hipStream_t s) {
  hipLaunchKernelGGL(fill_test_matrix_kernel, row_grid(n_pad, n_pad), dim3(256), 0, s, M, n, n_pad, seed);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t count, hipStream_t s) {
  const size_t blocks = std::min<size_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_gemv(const double* M, int64_t ld, int n, const double* x, double* y,
                       bool transposed, double* part, int nblk, hipStream_t s) {
  if (!transposed) {
    hipLaunchKernelGGL(gemv_n_kernel, dim3((n + 3) / 4), dim3(TPB), 0, s, M, ld, n, x, y);
  } else {
    hipLaunchKernelGGL(gemv_t_part_kernel, dim3(nblk, (n + TPB - 1) / TPB), dim3(TPB), 0, s, M, ld,
                       n, x, part, nblk);
    hipLaunchKernelGGL(gemv_t_reduce_kernel, dim3((n + CS_COLS - 1) / CS_COLS), dim3(TPB), 0, s, part,
                       nblk, n, y);
  }
  return hipGetLastError();
}

hipError_t launch_lincomb_init(const LincombArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lincomb_init_kernel, row_grid((int)a.ld, (int)a.ld), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* M, int64_t ld, int n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(check_finite_kernel, row_grid(n, n), dim3(256), 0, s, M, ld, n, flag);
  return hipGetLastError();
}

hipError_t launch_scale_out(const double* src, int64_t ld, double* dst, int64_t ldd, int n,
                            double scale, int* nonfinite, hipStream_t s) {
  hipLaunchKernelGGL(scale_out_kernel, row_grid(n, n), dim3(256), 0, s, src, ld, dst, ldd, n,
                     scale, nonfinite);
  return hipGetLastError();
}

}  // namespace logm
