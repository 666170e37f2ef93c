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
constexpr int LDA = NB + 1;
constexpr int IU_ROWS = 32;
#ifndef LOGM_TOURN_WAVES
#define LOGM_TOURN_WAVES 8
#endif
#ifndef LOGM_TOURN_RPL
#define LOGM_TOURN_RPL 8
#endif
constexpr int NW = LOGM_TOURN_WAVES;   // waves; wave w owns columns [CPW w, CPW (w + 1))
constexpr int TT = 64 * NW;            // threads of a tournament node
constexpr int CPW = NB / NW;           // columns per wave
constexpr int RPL = LOGM_TOURN_RPL;    // candidate rows per lane: lane l owns rows l + 64 i
constexpr int TR = 64 * RPL;           // candidate rows per node
constexpr int FAN = TR / NB;           // children merged by one node

__device__ __forceinline__ int load_coherent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// u[c] = x[iL][c] of lane L, for wave-uniform iL and L.  The uniform switch keeps
// every register index static (a dynamic index would spill the row block to
// scratch) and executes only one case.
__device__ __forceinline__ void read_owner_row(const double (&x)[RPL][CPW], int iL, int L,
                                               double (&u)[CPW]) {
#define LOGM_ROW_CASE(I)                                                                 \
  if (I < RPL && iL == I) {                                                              \
    _Pragma("unroll") for (int c = 0; c < CPW; ++c) u[c] = readlane_d(x[(I < RPL) ? I : 0][c], L); \
    return;                                                                              \
  }
  LOGM_ROW_CASE(0)
  LOGM_ROW_CASE(1)
  LOGM_ROW_CASE(2)
  LOGM_ROW_CASE(3)
  LOGM_ROW_CASE(4)
  LOGM_ROW_CASE(5)
  LOGM_ROW_CASE(6)
  LOGM_ROW_CASE(7)
#undef LOGM_ROW_CASE
  _Pragma("unroll") for (int c = 0; c < CPW; ++c) u[c] = readlane_d(x[0][c], L);
}

// Lane holding the wave's largest v among lanes with ok (lowest lane on ties), or
// -1.  The DPP maximum is checked with a ballot; the shuffle reduction decides if
// no lane matches it.
__device__ __forceinline__ int wave_argmax_lane(double v, bool ok) {
  const double m = wave_max_dpp(ok ? v : -1.0);
  unsigned long long bal = __ballot(ok && v == m);
  if (bal == 0ull) {
    if (__ballot(ok) == 0ull) return -1;
    int idx = ok ? (int)(threadIdx.x & 63) : 64;
    double vv = ok ? v : -1.0;
    wave_argmax(vv, idx);
    return idx;
  }
  return __ffsll((long long)bal) - 1;
}

// Tournament pivot selection for the inner block [c0, c0+64) of the panel over the
// candidate positions [r0, n_pad).  A node runs partial-pivoting LU on up to TR
// candidate rows held in registers: wave w keeps columns CPW w .. CPW w + CPW - 1 of
// every row, lane l rows l, l+64, ...  The pivot of column j is found inside the wave owning
// column j; only its multipliers cross waves (through LDS, one barrier per
// column), and every wave reads its slice of the pivot row from the owning lane.
// Leaves take TR consecutive candidates, inner nodes the <= 64 winners of each of
// their <= FAN children (the last child to finish does the merge).  The root
// writes the LU factors of the 64 selected rows (pivot order) to m.tri and builds
// the row maps of the step.
__global__ __launch_bounds__(TT) __attribute__((amdgpu_waves_per_eu(1, 2))) void tournament_kernel(GjeArgs A, int nleaves) {
  __shared__ __attribute__((aligned(16))) double s_lu[NB][NB + 2];
  __shared__ double s_l[2][TR];
  __shared__ int s_p[2];
  __shared__ int s_rid[TR];
  __shared__ int s_sel[NB];
  __shared__ int s_off[FAN + 1];
  __shared__ int s_last;
  __shared__ int s_in[NB];
  __shared__ int s_V[NB];
  __shared__ int s_D[NB];
  __shared__ int s_nv;
  __shared__ int s_old_pi[2 * NB];
  __shared__ int s_old_pt[2 * NB];

  const GjeMat& m = A.m[blockIdx.y];
  const double* P = m.P[A.pcur];
  const int nbo = A.nbo;
  const int c0 = A.c0;
  const int r0 = A.r0;
  const int np = A.n_pad;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;

  int node = blockIdx.x;
  int nodes = nleaves;
  int level_off = 0;
  int nrows;
  {
    const int first = r0 + node * TR;
    nrows = min(TR, np - first);
    for (int r = tid; r < TR; r += TT) s_rid[r] = first + min(r, nrows - 1);
    if (tid < NB) s_sel[tid] = min(tid, nrows - 1);
  }
  __syncthreads();
  bool need_lu = true;
  int npiv = 0;
  while (true) {
    if (need_lu) {
      double x[RPL][CPW];
      unsigned act = 0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = lane + 64 * i;
        const int pos = s_rid[min(r, nrows - 1)];
        const f64x2* src = reinterpret_cast<const f64x2*>(P + (int64_t)pos * nbo + c0 + CPW * wave);
#pragma unroll
        for (int c = 0; c < CPW / 2; ++c) {
          const f64x2 v = src[c];
          x[i][2 * c] = (r < nrows) ? v.x : 0.0;
          x[i][2 * c + 1] = (r < nrows) ? v.y : 0.0;
        }
        act |= (r < nrows) ? (1u << i) : 0u;
      }
      npiv = min(NB, nrows);
#pragma unroll 1
      for (int g = 0; g < NW; ++g) {
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc) {
          const int j = CPW * g + cc;
          if (j < npiv) {
          if (wave == g) {
            // ---- pivot search in the owning wave
            double best = -1.0, bestv = 0.0;
            int bi = 0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
              double a = fabs(x[i][cc]);
              if (!(a == a)) a = 0.0;
              if (((act >> i) & 1u) && a > best) {
                best = a;
                bestv = x[i][cc];
                bi = i;
              }
            }
            const int L = wave_argmax_lane(best, best >= 0.0);
            const int iL = __builtin_amdgcn_readlane(bi, L);
            const double piv = readlane_d(bestv, L);
            const int p = L + 64 * iL;
            if (lane == L) act &= ~(1u << iL);
            const double rp = (piv != 0.0) ? 1.0 / piv : 0.0;
            double l[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
              l[i] = ((act >> i) & 1u) ? x[i][cc] * rp : 0.0;
              s_l[j & 1][lane + 64 * i] = l[i];
            }
            if (lane == 0) s_p[j & 1] = p;
            // this wave's slice of row p (before the update)
            double u[CPW];
            read_owner_row(x, iL, L, u);
            if (lane == 0) {
#pragma unroll
              for (int c = 0; c < CPW; c += 2)
                *reinterpret_cast<f64x2*>(&s_lu[j][CPW * wave + c]) = f64x2{u[c], u[c + 1]};
              s_sel[j] = p;
            }
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
              if ((act >> i) & 1u) x[i][cc] = l[i];
#pragma unroll
              for (int c = cc + 1; c < CPW; ++c) x[i][c] = fma(-l[i], u[c], x[i][c]);
            }
          }
          __syncthreads();
          if (wave != g) {
            const int p = s_p[j & 1];
            const int L = p & 63;
            const int iL = p >> 6;
            if (lane == L) act &= ~(1u << iL);
            double u[CPW];
            read_owner_row(x, iL, L, u);
            if (lane == 0) {
#pragma unroll
              for (int c = 0; c < CPW; c += 2)
                *reinterpret_cast<f64x2*>(&s_lu[j][CPW * wave + c]) = f64x2{u[c], u[c + 1]};
            }
            if (wave > g) {
#pragma unroll
              for (int i = 0; i < RPL; ++i) {
                const double li = s_l[j & 1][lane + 64 * i];
#pragma unroll
                for (int c = 0; c < CPW; ++c) x[i][c] = fma(-li, u[c], x[i][c]);
              }
            }
          }
          }
        }
      }
      __syncthreads();
    }
    if (nodes == 1) break;

    // ---- publish this node's winners and find out whether this workgroup merges
    int* slot = m.cand + (level_off + node) * 65;
    if (tid == 0) slot[0] = npiv;
    if (tid < npiv) slot[1 + tid] = s_rid[s_sel[tid]];
    __threadfence();
    __syncthreads();
    const int parent = node / FAN;
    const int nchild = min(FAN, nodes - parent * FAN);
    const int next_off = level_off + nodes;
    if (tid == 0) {
      const int old = atomicAdd(&m.cnt[next_off + parent], 1);
      s_last = (old == nchild - 1);
      if (s_last) atomicExch(&m.cnt[next_off + parent], 0);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    need_lu = nchild > 1;
    if (need_lu) {
      if (tid == 0) {
        int off = 0;
        for (int ch = 0; ch < nchild; ++ch) {
          s_off[ch] = off;
          off += min(NB, max(0, load_coherent(m.cand + (level_off + parent * FAN + ch) * 65)));
        }
        s_off[nchild] = off;
      }
      __syncthreads();
      nrows = s_off[nchild];
      for (int ch = 0; ch < nchild; ++ch) {
        const int cnt = s_off[ch + 1] - s_off[ch];
        const int* cs = m.cand + (level_off + parent * FAN + ch) * 65 + 1;
        if (tid < cnt) s_rid[s_off[ch] + tid] = min(max(load_coherent(cs + tid), 0), np - 1);
      }
      __syncthreads();
      for (int r = nrows + tid; r < TR; r += TT) s_rid[r] = s_rid[0];
      if (tid < NB) s_sel[tid] = min(tid, nrows - 1);
      __syncthreads();
    }
    node = parent;
    level_off = next_off;
    nodes = (nodes + FAN - 1) / FAN;
  }

  // ---- root: LU factors of the selected rows, log|det|, row maps of the step
  for (int e = tid; e < NB * NB; e += TT) m.tri[e] = s_lu[e / NB][e % NB];
  if (tid < NB) s_sel[tid] = s_rid[min(max(s_sel[tid], 0), TR - 1)];   // local row -> position
  if (wave == 1) {   // log|det| of the pivot block: one pivot per lane, fixed-order sum
    const double piv = s_lu[lane][lane];
    if (__ballot(piv == 0.0) != 0ull && lane == 0) atomicOr(&m.err[0], 1);
    const double ls = wave_sum(log(fabs(piv)));
    if (lane == 0) m.logdet[r0 / NB] = ls;
  }
  if (tid < NB) {
    s_in[tid] = 0;
    s_V[tid] = r0 + tid;
    s_D[tid] = r0 + tid;
  }
  __syncthreads();
  // gather map of this inner step: position r0+j <- s_sel[j]; the block rows that
  // were not chosen (D, ascending) move to the vacated positions of chosen rows
  // outside the block (V, ascending).  The selection is a set of distinct rows, so
  // |V| = |D|; the lists are pre-filled and indices clamped all the same.
  if (tid < NB && s_sel[tid] >= r0 && s_sel[tid] < r0 + NB) s_in[s_sel[tid] - r0] = 1;
  __syncthreads();
  if (tid < NB) {
    const int q = s_sel[tid];
    if (q >= r0 + NB) {
      int rank = 0;
      for (int j = 0; j < NB; ++j) rank += (s_sel[j] >= r0 + NB && s_sel[j] < q);
      s_V[min(rank, NB - 1)] = q;
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
    const int q = min(max(s_sel[tid], 0), np - 1);
    const int vq = min(max(s_V[tid], 0), np - 1);
    const int dq = min(max(s_D[tid], 0), np - 1);
    m.qsel[tid] = q;
    s_old_pi[tid] = m.pi[q];
    s_old_pt[tid] = m.ptot[q];
    if (tid < nv) {
      m.vac[1 + tid] = vq;
      m.vac[65 + tid] = dq;
      s_old_pi[NB + tid] = m.pi[dq];
      s_old_pt[NB + tid] = m.ptot[dq];
    }
    if (tid == 0) m.vac[0] = nv;
  }
  __syncthreads();
  if (tid < NB) {
    m.pi[r0 + tid] = s_old_pi[tid];
    m.ptot[r0 + tid] = s_old_pt[tid];
    if (tid < nv) {
      const int vq = min(max(s_V[tid], 0), np - 1);
      m.pi[vq] = s_old_pi[NB + tid];
      m.ptot[vq] = s_old_pt[NB + tid];
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

// Inner Gauss-Jordan step on the panel, IU_ROWS rows per workgroup (see the file
// comment): C U = Acol and G L = C are solved by 16-column block substitution with
// explicit inverses of the 16 x 16 diagonal blocks only, then out = base - G R.
__global__ __launch_bounds__(256) void inner_update_kernel(GjeArgs A) {
  __shared__ double LU[NB][LDA];          // L (strict lower) and U of the pivot block
  __shared__ double Di[8][16][17];        // inverses of the diagonal blocks: 0-3 of U, 4-7 of L
  __shared__ double Rs[NB][LDA];          // pivot rows of one column chunk
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
  {
    double t[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] = m.tri[tid + 256 * k];
#pragma unroll
    for (int k = 0; k < 16; ++k) LU[(tid + 256 * k) / NB][(tid + 256 * k) % NB] = t[k];
  }
  __syncthreads();

  // diagonal block inverses: thread (blk, col) runs one column of a 16 x 16 substitution
  if (tid < 128) {
    const int blk = tid >> 4;
    const int c = tid & 15;
    const int b0 = (blk & 3) * 16;
    double x[16];
    if (blk < 4) {  // upper: X U_bb = I  (column c of U_bb^{-1} by back substitution)
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int t = r + 1; t < 16; ++t) acc = fma(-LU[b0 + r][b0 + t], x[t], acc);
        x[r] = (r <= c) ? acc / LU[b0 + r][b0 + r] : 0.0;
      }
    } else {        // unit lower: column c of L_bb^{-1} by forward substitution
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < r; ++t) acc = fma(-LU[b0 + r][b0 + t], x[t], acc);
        x[r] = (r >= c) ? acc : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) Di[blk][r][c] = x[r];
  }
  // right-hand side of C U = Acol: panel rows, or -E (identity rows) inside the block
  {
    double t[IU_ROWS * NB / 256];
#pragma unroll
    for (int k = 0; k < IU_ROWS * NB / 256; ++k) {
      const int e = tid + 256 * k;
      const int r = e / NB;
      const int c = e % NB;
      t[k] = inblock ? ((row0 - r0 + r == c) ? -1.0 : 0.0) : P[(int64_t)s_src[r] * nbo + c0 + c];
    }
#pragma unroll
    for (int k = 0; k < IU_ROWS * NB / 256; ++k) {
      const int e = tid + 256 * k;
      Cs[e / NB][e % NB] = t[k];
    }
  }
  __syncthreads();

  // C U = Acol, blocks left to right: C_b = (Acol_b - C_{<b} U_{<b,b}) inv(U_bb)
  for (int b = 0; b < 4; ++b) {
    for (int e = tid; e < IU_ROWS * 16; e += 256) {
      const int r = e >> 4;
      const int c = b * 16 + (e & 15);
      double acc = Cs[r][c];
      for (int t = 0; t < b * 16; ++t) acc = fma(-Cs[r][t], LU[t][c], acc);
      Ts[r][e & 15] = acc;
    }
    __syncthreads();
    for (int e = tid; e < IU_ROWS * 16; e += 256) {
      const int r = e >> 4;
      const int cl = e & 15;
      double acc = 0.0;
      for (int t = 0; t <= cl; ++t) acc = fma(Ts[r][t], Di[b][t][cl], acc);
      Cs[r][b * 16 + cl] = acc;
    }
    __syncthreads();
  }
  // G L = C, blocks right to left: G_b = (C_b - G_{>b} L_{>b,b}) inv(L_bb)
  for (int b = 3; b >= 0; --b) {
    for (int e = tid; e < IU_ROWS * 16; e += 256) {
      const int r = e >> 4;
      const int c = b * 16 + (e & 15);
      double acc = Cs[r][c];
      for (int t = (b + 1) * 16; t < NB; ++t) acc = fma(-Cs[r][t], LU[t][c], acc);
      Ts[r][e & 15] = acc;
    }
    __syncthreads();
    for (int e = tid; e < IU_ROWS * 16; e += 256) {
      const int r = e >> 4;
      const int cl = e & 15;
      double acc = 0.0;
      for (int t = cl; t < 16; ++t) acc = fma(Ts[r][t], Di[4 + b][t][cl], acc);
      Cs[r][b * 16 + cl] = acc;
    }
    __syncthreads();
  }

  // ---- output chunks: -G in the inner block, base - G R elsewhere
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int rb = w >> 1;
  const int cb = (w & 1) * 2;
  const int lr = lane & 15;
  const int lk = lane >> 4;
  for (int cc = 0; cc < nbo; cc += NB) {
    if (cc == c0) {
      for (int e = tid; e < IU_ROWS * NB; e += 256) {
        const int r = e / NB;
        const int c = e % NB;
        Q[(int64_t)(row0 + r) * nbo + cc + c] = -Cs[r][c];
      }
      continue;
    }
    {
      double t[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k;
        t[k] = P[(int64_t)s_q[e / NB] * nbo + cc + e % NB];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = tid + 256 * k;
        Rs[e / NB][e % NB] = t[k];
      }
    }
    double base[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lk;
        base[b][r] = inblock ? 0.0 : P[(int64_t)s_src[rr] * nbo + cc + (cb + b) * 16 + lr];
      }
    __syncthreads();
    f64x4 acc[2];
    mm32x64(Cs, Rs, acc);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lk;
        const int c = cc + (cb + b) * 16 + lr;
        Q[(int64_t)(row0 + rr) * nbo + c] = base[b][r] - acc[b][r];
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
  const int nleaves = (ncand + TR - 1) / TR;
  hipLaunchKernelGGL(tournament_kernel, dim3(nleaves, a.nmat), dim3(TT), 0, s, a, nleaves);
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
