// Blocked Gauss-Jordan inversion with tournament pivoting (gfx950).
//
// The square-root iteration (eq. ScalDB) needs X^{-1}, Y^{-1} and |det X det Y|.
// Gauss-Jordan elimination computes the inverse in place with 2 n^3 flops in n/nb
// uniform rank-nb updates, which suits the matrix cores better than LU + triangular
// inversion.  Two blocking levels:
//
//  outer step (width nbo <= 256, columns K = [k0, k0+nbo)):
//    with Mp the matrix in the pivot order chosen for this step and S = Mp[K,K],
//      out[i][c] = U[i][c-k0]                                         c in K
//      out[i][c] = [i not in K] Mp[i][c] + sum_t U[i][t] Mp[k0+t][c]  c not in K
//    where U = Gauss-Jordan processed panel: U[i,:] = -Mp[i,K] S^{-1} (i not in K),
//    U[K,:] = S^{-1}.  This is one MFMA GEMM with K-dimension nbo (gemm_f64.hip).
//
//  inner steps (width 64, inside the n_pad x nbo panel Pw): the panel alone is taken
//    through the same step, 64 columns at a time.  With the 64 pivot rows factored
//    as S64 = L U (partial pivoting order):
//      C[p,:] solves C U = Pw[p, block]          (p not in the block)
//      C[p,:] = -U^{-1}[p - r0, :]                (p in the block)
//      G = C L^{-1}
//      out[p][c] = -G[p][c - c0]                              c in the inner block
//      out[p][c] = [p not in block] Pw[p][c] - G[p,:] R[:, c]   otherwise
//    R being the pivot rows.  C is computed by block substitution with explicit
//    inverses of the 16 x 16 diagonal blocks of U only: multiplying by an explicit
//    S^{-1} (or U^{-1}) instead loses up to two digits on the ill-conditioned
//    iterates of the square-root iteration, while 16 x 16 blocks keep the accuracy
//    of LAPACK's LU-based inverse.
//
// Pivot rows of each inner block are chosen by tournament pivoting: leaves run
// partial-pivoting LU on 128-row chunks of the candidate rows and forward their 64
// pivot rows; the last workgroup to arrive at a tree node merges its children the
// same way.  The root keeps the LU factors of the selected block, forms the
// triangular inverses and records log|det| = sum log|u_jj|.  Row exchanges are
// never applied in place: every update reads its input rows through the gather map,
// and the accumulated order ptot gives A^{-1}[:, ptot(c)] = M_final[:, c].
#include "common.hpp"
#include "kernels.hpp"

namespace logm {
namespace {

constexpr int NB = 64;
constexpr int LEAF = 128;
constexpr int LDA = NB + 1;
constexpr int IU_ROWS = 32;

__device__ __forceinline__ int load_coherent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Partial-pivoting LU on an nrows x 64 block in LDS (row ids in rid).  Rows are
// swapped physically; afterwards rid[0 .. min(64, nrows)) are the pivot rows in
// pivot order.  A column whose remaining entries are all zero is skipped.
__device__ void lds_gepp(double (*a)[LDA], int* rid, int nrows, int* s_piv) {
  const int tid = threadIdx.x;
  const int npiv = min(NB, nrows);
  for (int j = 0; j < npiv; ++j) {
    if (tid < 64) {
      // lanes without rows offer (-1, j); a NaN entry counts as 0, so the winner is
      // always a row in [j, nrows)
      double v = -1.0;
      int idx = j;
      for (int r = j + tid; r < nrows; r += 64) {
        double x = fabs(a[r][j]);
        if (!(x == x)) x = 0.0;
        if (x > v) {
          v = x;
          idx = r;
        }
      }
      wave_argmax(v, idx);
      if (tid == 0) *s_piv = (idx >= j && idx < nrows) ? idx : j;
    }
    __syncthreads();
    const int p = *s_piv;
    if (p != j) {
      if (tid < NB) {
        const double t = a[j][tid];
        a[j][tid] = a[p][tid];
        a[p][tid] = t;
      }
      if (tid == 0) {
        const int t = rid[j];
        rid[j] = rid[p];
        rid[p] = t;
      }
    }
    __syncthreads();
    const double d = a[j][j];
    if (d != 0.0) {
      for (int r = j + 1 + tid; r < nrows; r += 256) a[r][j] = a[r][j] / d;
      __syncthreads();
      const int cols = NB - 1 - j;
      const int rows = nrows - 1 - j;
      for (int e = tid; e < rows * cols; e += 256) {
        const int r = j + 1 + e / cols;
        const int c = j + 1 + e % cols;
        a[r][c] = fma(-a[r][j], a[j][c], a[r][c]);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void tournament_kernel(GjeArgs A, int nleaves) {
  __shared__ double a[LEAF][LDA];
  __shared__ int rid[LEAF];
  __shared__ int s_piv, s_last, s_nv;
  __shared__ int s_in[NB];
  __shared__ int s_V[NB];
  __shared__ int s_D[NB];
  __shared__ int s_old_pi[2 * NB];
  __shared__ int s_old_pt[2 * NB];

  const GjeMat& m = A.m[blockIdx.y];
  const double* P = m.P[A.pcur];
  const int nbo = A.nbo;
  const int c0 = A.c0;
  const int r0 = A.r0;
  const int tid = threadIdx.x;

  int node = blockIdx.x;
  int nodes = nleaves;
  int level_off = 0;

  // leaf: rows [first, first + nrows)
  const int first = r0 + node * LEAF;
  int nrows = min(LEAF, A.n_pad - first);
  for (int e = tid; e < nrows * NB; e += 256) {
    const int r = e / NB;
    const int c = e % NB;
    a[r][c] = P[(int64_t)(first + r) * nbo + c0 + c];
  }
  for (int r = tid; r < nrows; r += 256) rid[r] = first + r;
  __syncthreads();
  lds_gepp(a, rid, nrows, &s_piv);
  int ncand = min(NB, nrows);

  while (nodes > 1) {
    int* slot = m.cand + (level_off + node) * 65;
    if (tid == 0) slot[0] = ncand;
    if (tid < ncand) slot[1 + tid] = rid[tid];
    __threadfence();
    __syncthreads();
    const int parent = node >> 1;
    const int nchild = min(2, nodes - 2 * parent);
    const int next_off = level_off + nodes;
    if (tid == 0) {
      const int old = atomicAdd(&m.cnt[next_off + parent], 1);
      s_last = (old == nchild - 1);
      if (s_last) atomicExch(&m.cnt[next_off + parent], 0);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (nchild == 2) {
      const int* c0s = m.cand + (level_off + 2 * parent) * 65;
      const int* c1s = c0s + 65;
      const int n0 = load_coherent(c0s);
      const int n1 = load_coherent(c1s);
      for (int r = tid; r < n0 + n1; r += 256)
        rid[r] = (r < n0) ? load_coherent(c0s + 1 + r) : load_coherent(c1s + 1 + (r - n0));
      nrows = n0 + n1;
      __syncthreads();
      for (int e = tid; e < nrows * NB; e += 256) {
        const int r = e / NB;
        const int c = e % NB;
        a[r][c] = P[(int64_t)rid[r] * nbo + c0 + c];
      }
      __syncthreads();
      lds_gepp(a, rid, nrows, &s_piv);
      ncand = min(NB, nrows);
    }
    // nchild == 1: the single child's selection (still in rid) passes through
    node = parent;
    level_off = next_off;
    nodes = (nodes + 1) >> 1;
  }

  // ---- root: a[0..63][0..63] holds L (strictly lower, unit diagonal) and U of the
  // selected rows in pivot order.  Wave 0 forms U^{-1}, wave 1 L^{-1}, one column
  // per lane (back / forward substitution); wave 2 records log|det|.
  __syncthreads();
  {
    double (*xs)[LDA] = reinterpret_cast<double (*)[LDA]>(&a[NB][0]);   // rows 64..127
    const int w = tid >> 6;
    const int c = tid & 63;
    double* Uinv = m.tri + NB * NB;
    double* Linv = m.tri + 2 * NB * NB;
    if (w == 0) {
      // X = U^{-1}: X[r][c] = (delta_rc - sum_{t=r+1..c} U[r][t] X[t][c]) / U[r][r]
      for (int r = NB - 1; r >= 0; --r) {
        double v = 0.0;
        if (r <= c) {
          double acc = (r == c) ? 1.0 : 0.0;
          for (int t = r + 1; t <= c; ++t) acc = fma(-a[r][t], xs[t][c], acc);
          v = acc / a[r][r];
        }
        xs[r][c] = v;
      }
      for (int r = 0; r < NB; ++r) Uinv[r * NB + c] = xs[r][c];
    } else if (w == 1) {
      // Y = L^{-1} (unit lower): Y[r][c] = delta_rc - sum_{t=c..r-1} L[r][t] Y[t][c]
      double ycol[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < r; ++t) acc = fma(-a[r][t], ycol[t], acc);
        ycol[r] = (r < c) ? 0.0 : acc;
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) Linv[r * NB + c] = ycol[r];
    } else if (w == 2 && c == 0) {
      double logsum = 0.0;
      for (int j = 0; j < NB; ++j) {
        const double piv = a[j][j];
        if (piv == 0.0) atomicOr(&m.err[0], 1);
        logsum += log(fabs(piv));
      }
      m.logdet[r0 / NB] = logsum;
    }
    __syncthreads();
    // U with its 16 x 16 diagonal blocks replaced by those of U^{-1}
    for (int e = tid; e < NB * NB; e += 256) {
      const int r = e / NB;
      const int cc = e % NB;
      const bool diag_blk = (r >> 4) == (cc >> 4);
      m.tri[e] = diag_blk ? xs[r][cc] : (cc > r ? a[r][cc] : 0.0);
    }
  }

  // gather map of this inner step: position r0+j <- rid[j]; the block rows that were
  // not chosen (D, ascending) move to the vacated positions of chosen rows outside
  // the block (V, ascending).
  if (tid < NB) s_in[tid] = 0;
  __syncthreads();
  if (tid < NB && rid[tid] < r0 + NB) s_in[rid[tid] - r0] = 1;
  __syncthreads();
  if (tid < NB) {
    const int q = rid[tid];
    if (q >= r0 + NB) {
      int rank = 0;
      for (int j = 0; j < NB; ++j) rank += (rid[j] >= r0 + NB && rid[j] < q);
      s_V[rank] = q;
    }
    if (!s_in[tid]) {
      int rank = 0;
      for (int t = 0; t < tid; ++t) rank += !s_in[t];
      s_D[rank] = r0 + tid;
    }
    if (tid == 0) {
      int nv = 0;
      for (int t = 0; t < NB; ++t) nv += !s_in[t];
      s_nv = nv;
    }
  }
  __syncthreads();
  const int nv = s_nv;
  if (tid < NB) {
    m.qsel[tid] = rid[tid];
    s_old_pi[tid] = m.pi[rid[tid]];
    s_old_pt[tid] = m.ptot[rid[tid]];
    if (tid < nv) {
      m.vac[1 + tid] = s_V[tid];
      m.vac[65 + tid] = s_D[tid];
      s_old_pi[NB + tid] = m.pi[s_D[tid]];
      s_old_pt[NB + tid] = m.ptot[s_D[tid]];
    }
    if (tid == 0) m.vac[0] = nv;
  }
  __syncthreads();
  if (tid < NB) {
    m.pi[r0 + tid] = s_old_pi[tid];
    m.ptot[r0 + tid] = s_old_pt[tid];
    if (tid < nv) {
      m.pi[s_V[tid]] = s_old_pi[NB + tid];
      m.ptot[s_V[tid]] = s_old_pt[NB + tid];
    }
  }
}

// C-block (IU_ROWS x 64) = As (IU_ROWS x 64) * Bs (64 x 64), MFMA; wave w owns row
// block w/2 and column blocks 2(w%2), 2(w%2)+1.  Result in acc[2] (lane layout of
// the 16x16x4 instruction: element r of lane l is row 4r + l/16, column l%16).
__device__ __forceinline__ void mm32x64(const double (*As)[LDA], const double (*Bs)[LDA],
                                        f64x4 acc[2]) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int rb = w >> 1;
  const int cb = (w & 1) * 2;
  const int lr = lane & 15;
  const int lk = lane >> 4;
  acc[0] = f64x4{0.0, 0.0, 0.0, 0.0};
  acc[1] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < NB / 4; ++ks) {
    const double av = As[rb * 16 + lr][ks * 4 + lk];
    const double b0 = Bs[ks * 4 + lk][cb * 16 + lr];
    const double b1 = Bs[ks * 4 + lk][(cb + 1) * 16 + lr];
    acc[0] = mfma_f64_16x16x4(av, b0, acc[0]);
    acc[1] = mfma_f64_16x16x4(av, b1, acc[1]);
  }
}

__global__ __launch_bounds__(256) void inner_update_kernel(GjeArgs A) {
  __shared__ double B1[NB][LDA];     // U (block form), then L^{-1}
  __shared__ double B2[NB][LDA];     // pivot rows R of one column chunk
  __shared__ double Cs[IU_ROWS][LDA];
  __shared__ double Ts[IU_ROWS][17];
  __shared__ int s_src[IU_ROWS];
  __shared__ int s_q[NB];

  const GjeMat& m = A.m[blockIdx.y];
  const double* P = m.P[A.pcur];
  double* Q = m.P[A.pcur ^ 1];
  const int nbo = A.nbo;
  const int r0 = A.r0;
  const int c0 = A.c0;
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * IU_ROWS;
  const bool inblock = row0 >= r0 && row0 < r0 + NB;

  if (tid < IU_ROWS) {
    const int p = row0 + tid;
    int src = p;
    if (p >= r0 && p < r0 + NB) {
      src = m.qsel[p - r0];
    } else {
      const int nv = m.vac[0];
      for (int i = 0; i < nv; ++i)
        if (m.vac[1 + i] == p) src = m.vac[65 + i];
    }
    s_src[tid] = src;
  }
  if (tid < NB) s_q[tid] = m.qsel[tid];
  __syncthreads();

  // ---- C rows
  if (inblock) {
    const double* Uinv = m.tri + NB * NB;
    for (int e = tid; e < IU_ROWS * NB; e += 256) {
      const int r = e / NB;
      const int c = e % NB;
      Cs[r][c] = -Uinv[(row0 - r0 + r) * NB + c];
    }
  } else {
    for (int e = tid; e < NB * NB; e += 256) B1[e / NB][e % NB] = m.tri[e];
    for (int e = tid; e < IU_ROWS * NB; e += 256) {
      const int r = e / NB;
      const int c = e % NB;
      Cs[r][c] = P[(int64_t)s_src[r] * nbo + c0 + c];
    }
    __syncthreads();
    // C U = Acol by 16-column blocks: rhs = Acol_b - C_{<b} U_{<b,b}; C_b = rhs inv(U_bb)
    for (int b = 0; b < 4; ++b) {
      for (int e = tid; e < IU_ROWS * 16; e += 256) {
        const int r = e >> 4;
        const int c = b * 16 + (e & 15);
        double acc = Cs[r][c];
        for (int t = 0; t < b * 16; ++t) acc = fma(-Cs[r][t], B1[t][c], acc);
        Ts[r][e & 15] = acc;
      }
      __syncthreads();
      for (int e = tid; e < IU_ROWS * 16; e += 256) {
        const int r = e >> 4;
        const int cl = e & 15;
        double acc = 0.0;
        for (int t = 0; t <= cl; ++t) acc = fma(Ts[r][t], B1[b * 16 + t][b * 16 + cl], acc);
        Cs[r][b * 16 + cl] = acc;
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // ---- G = C L^{-1} (kept in Cs)
  const double* Linv = m.tri + 2 * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) B1[e / NB][e % NB] = Linv[e];
  __syncthreads();
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int rb = w >> 1;
  const int cb = (w & 1) * 2;
  const int lr = lane & 15;
  const int lk = lane >> 4;
  {
    f64x4 acc[2];
    mm32x64(Cs, B1, acc);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) Cs[rb * 16 + 4 * r + lk][(cb + b) * 16 + lr] = acc[b][r];
  }
  __syncthreads();

  // ---- output chunks
  for (int cc = 0; cc < nbo; cc += NB) {
    if (cc == c0) {
      for (int e = tid; e < IU_ROWS * NB; e += 256) {
        const int r = e / NB;
        const int c = e % NB;
        Q[(int64_t)(row0 + r) * nbo + cc + c] = -Cs[r][c];
      }
      continue;
    }
    for (int e = tid; e < NB * NB; e += 256) {
      const int t = e / NB;
      const int c = e % NB;
      B2[t][c] = P[(int64_t)s_q[t] * nbo + cc + c];
    }
    __syncthreads();
    f64x4 acc[2];
    mm32x64(Cs, B2, acc);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lk;
        const int c = cc + (cb + b) * 16 + lr;
        const double base = inblock ? 0.0 : P[(int64_t)s_src[rr] * nbo + c];
        Q[(int64_t)(row0 + rr) * nbo + c] = base - acc[b][r];
      }
    __syncthreads();
  }
}

__global__ void begin_kernel(GjeArgs A, int nslots, int ncnt) {
  const GjeMat& m = A.m[blockIdx.y];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pad; p += gridDim.x * blockDim.x)
    m.ptot[p] = p;
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < nslots; t += blockDim.x) m.logdet[t] = 0.0;
    for (int t = threadIdx.x; t < ncnt; t += blockDim.x) m.cnt[t] = 0;
    if (threadIdx.x < 4) m.err[threadIdx.x] = 0;
  }
}

__global__ void panel_copy_kernel(GjeArgs A) {
  const GjeMat& m = A.m[blockIdx.y];
  const int nbo = A.nbo;
  const int64_t total = (int64_t)A.n_pad * nbo;
  double* P = m.P[A.pcur];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nbo;
    const int c = (int)(e % nbo);
    P[e] = m.Min[i * A.n_pad + A.k0 + c];
    if (c == 0) m.pi[i] = (int)i;
  }
}

__global__ void finish_kernel(GjeArgs A) {
  const GjeMat& m = A.m[blockIdx.y];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pad; p += gridDim.x * blockDim.x)
    m.pinv[m.ptot[p]] = p;
}

__global__ void unpermute_kernel(const double* M, const int* pinv, int64_t ld, double* dst,
                                 int64_t ldd, int n) {
  const int i = blockIdx.y;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
    dst[(int64_t)i * ldd + q] = M[(int64_t)i * ld + pinv[q]];
}

}  // namespace

hipError_t launch_gje_begin(const GjeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(begin_kernel, dim3((a.n_pad + 255) / 256, a.nmat), dim3(256), 0, s, a,
                     a.n_pad / NB, gje_cnt_ints(a.n_pad));
  return hipGetLastError();
}

hipError_t launch_gje_panel_copy(const GjeArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)a.n_pad * a.nbo;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(panel_copy_kernel, dim3(blocks, a.nmat), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gje_tournament(const GjeArgs& a, hipStream_t s) {
  const int ncand = a.n_pad - a.r0;
  const int nleaves = (ncand + LEAF - 1) / LEAF;
  hipLaunchKernelGGL(tournament_kernel, dim3(nleaves, a.nmat), dim3(256), 0, s, a, nleaves);
  return hipGetLastError();
}

hipError_t launch_gje_inner_update(const GjeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(inner_update_kernel, dim3(a.n_pad / IU_ROWS, a.nmat), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gje_finish(const GjeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3((a.n_pad + 255) / 256, a.nmat), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gje_unpermute(const double* Mfinal, const int* pinv, int64_t ld, double* dst,
                                int64_t ldd, int n, hipStream_t s) {
  hipLaunchKernelGGL(unpermute_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, Mfinal, pinv,
                     ld, dst, ldd, n);
  return hipGetLastError();
}

}  // namespace logm
