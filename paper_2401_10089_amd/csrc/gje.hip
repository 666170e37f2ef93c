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
// partial-pivoting LU on 512-row chunks of the candidate rows and forward their 64
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
#ifndef LOGM_TOURN_RPL
#define LOGM_TOURN_RPL 8
#endif
constexpr int NW = 8;                  // waves of a tournament node
constexpr int TT = 64 * NW;            // threads of a tournament node
constexpr int SL = NB / NW;            // column slots per wave: wave w owns columns w + NW t
constexpr int RPL = LOGM_TOURN_RPL;    // candidate rows per lane: lane l owns rows l + 64 i
constexpr int TR = 64 * RPL;           // candidate rows per node
constexpr int FAN = TR / NB;           // children merged by one node

__device__ __forceinline__ int load_coherent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// u[c] = x[iL][c] of lane L for slots c >= c_first (a compile-time value after
// unrolling), for wave-uniform iL and L.  The uniform if-chain keeps every register
// index static (a dynamic index would spill the row block to scratch) and runs
// one case.
__device__ __forceinline__ void read_owner_row(const double (&x)[RPL][SL], int c_first, int iL,
                                               int L, double (&u)[SL]) {
#define LOGM_ROW_CASE(I)                                                                 \
  if (I < RPL && iL == I) {                                                              \
    _Pragma("unroll") for (int c = c_first; c < SL; ++c) u[c] = readlane_d(x[(I < RPL) ? I : 0][c], L); \
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
  _Pragma("unroll") for (int c = c_first; c < SL; ++c) u[c] = readlane_d(x[0][c], L);
}

// Packed pivot key of candidate slot i: bits 31..3 hold 1 + the high word of |a|
// shifted right by 3 (exponent and 17 leading mantissa bits), bits 2..0 the slot;
// rows that are no longer candidates get 0.  The chosen pivot is therefore within a
// factor 1 + 2^-17 of the largest magnitude in the column (a threshold variant of
// partial pivoting); an exact zero wins only when every candidate is below 2^-1019.
__device__ __forceinline__ unsigned pivot_key(double a, int i, unsigned act) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(a) >> 32) & 0x7fffffffu;
  const unsigned k = ((((hi >> 3) + 1u) << 3) | (unsigned)i);
  return ((act >> i) & 1u) ? k : 0u;
}

// Branch-free select on the bit pattern: v if bit else +0.
__device__ __forceinline__ double masked(double v, unsigned bit) {
  const unsigned m = 0u - (bit & 1u);
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)b & m, hi = (unsigned)(b >> 32) & m;
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Step ring of the pipelined node factorization: LDS flags instead of barriers.
// A step's record: stamp (step + 1 once published), pivot row, reciprocal pivot.
struct __attribute__((aligned(16))) StepRec {
  int stamp;
  int p;
  double rp;
};
constexpr int RING = 16;                      // steps in flight
constexpr int SPIN_LIMIT = 1 << 22;           // bounded waits (about 0.3 s)

// Wait until the LDS word *f reaches target; false if the bound is hit (the caller
// records an error and carries on with whatever is there, all indices stay clamped).
// The polled value is made wave-uniform, so the loop is a scalar loop.
__device__ __forceinline__ bool lds_wait_ge(const int* f, int target) {
  for (int it = 0; it < SPIN_LIMIT; ++it) {
    const int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (v >= target) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// Wait for a step record and return its pivot row and reciprocal pivot (uniform).
// Publishers issue s_wakeup, which ends the sleep of the waiting waves early.
__device__ __forceinline__ bool lds_wait_rec(const StepRec* r, int target, int& p, double& rp) {
  const bool ok = lds_wait_ge(&r->stamp, target);
  p = __builtin_amdgcn_readfirstlane(r->p);
  const long long b = __double_as_longlong(r->rp);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  rp = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  return ok;
}

// Tournament pivot selection for the inner block [c0, c0+64) of the panel over the
// candidate positions [r0, n_pad).  A node runs partial-pivoting LU on up to TR
// candidate rows held in registers: lane l of wave w keeps rows l, l+64, ... and
// the columns w, w+NW, w+2NW, ... of each (slot t holds column w + NW t).  Column j
// is owned by wave j % NW, so consecutive pivot searches run in different waves.
// Step j: the owner of column j applies step j-1 to that column, publishes the
// updated column and then, at raised wave priority, searches it and publishes pivot
// row p_j and its value; every wave (the owner included) forms the multipliers of
// step j-1 from the published column and applies step j-1 to its other columns.
// Steps are handed over through a ring of RING LDS slots with flags rather than
// barriers: the serial path is the chain of column updates and searches, and the
// bulk updates of a wave may trail it by up to RING steps.
// Rows arrive through LDS in 128-row chunks so that every global load is a
// contiguous 512-byte row segment.
// Leaves take TR consecutive candidates, inner nodes the <= 64 winners of each of
// their <= FAN children (the last child to finish does the merge).  The root
// writes the LU factors of the 64 selected rows (pivot order) to m.tri and builds
// the row maps of the step.
constexpr int STG_ROWS = 128;                 // staged rows per chunk
constexpr int STG_LD = NB + 1;                // odd stride: conflict-free column reads
constexpr int BUF_DOUBLES = (STG_ROWS * STG_LD > NB * (NB + 2)) ? STG_ROWS * STG_LD : NB * (NB + 2);

__global__ __launch_bounds__(TT) __attribute__((amdgpu_waves_per_eu(1, 2))) void tournament_kernel(GjeArgs A, int nleaves) {
  __shared__ __attribute__((aligned(16))) double s_buf[BUF_DOUBLES];   // row staging, then LU rows
  __shared__ double s_raw[RING][TR];
  __shared__ StepRec s_rec[RING];  // step j in slot j % RING, stamp j + 1 once published
  __shared__ int s_bcons[NW];      // waves done with all steps of a block
  __shared__ int s_rid[TR];
  __shared__ int s_stepof[TR];
  __shared__ int s_sel[NB];
  __shared__ int s_off[FAN + 1];
  __shared__ int s_last;
  __shared__ int s_in[NB];
  __shared__ int s_V[NB];
  __shared__ int s_D[NB];
  __shared__ int s_nv;
  __shared__ int s_old_pi[2 * NB];
  __shared__ int s_old_pt[2 * NB];
  double (*s_lu)[NB + 2] = reinterpret_cast<double (*)[NB + 2]>(s_buf);

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
      double x[RPL][SL];
      unsigned act = 0;
      // ---- rows into registers through LDS, 128 rows per chunk: a wave load
      // instruction covers two contiguous 512-byte row segments
      {
        f64x2 st[STG_ROWS * NB / 2 / TT];
        auto gload = [&](int ch) {
#pragma unroll
          for (int e = 0; e < STG_ROWS * NB / 2 / TT; ++e) {
            const int lr = ch * STG_ROWS + (wave * (STG_ROWS * NB / 2 / TT) + e) * 2 + (lane >> 5);
            const int pos = s_rid[min(lr, TR - 1)];
            st[e] = *reinterpret_cast<const f64x2*>(P + (int64_t)pos * nbo + c0 + 2 * (lane & 31));
          }
        };
        gload(0);
#pragma unroll
        for (int ch = 0; ch < RPL / 2; ++ch) {
#pragma unroll
          for (int e = 0; e < STG_ROWS * NB / 2 / TT; ++e) {
            const int rr = (wave * (STG_ROWS * NB / 2 / TT) + e) * 2 + (lane >> 5);
            s_buf[rr * STG_LD + 2 * (lane & 31)] = st[e].x;
            s_buf[rr * STG_LD + 2 * (lane & 31) + 1] = st[e].y;
          }
          __syncthreads();
          if (ch + 1 < RPL / 2) gload(ch + 1);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int i = 2 * ch + h;
            const bool ok = lane + 64 * i < nrows;
#pragma unroll
            for (int t = 0; t < SL; ++t) x[i][t] = masked(s_buf[(lane + 64 * h) * STG_LD + SL * wave + t], ok);
            act |= ok ? (1u << i) : 0u;
          }
          __syncthreads();
        }
      }
      npiv = min(NB, nrows);
      if (tid < RING) s_rec[tid].stamp = 0;
      if (tid < NW) s_bcons[tid] = 0;
      __syncthreads();
      bool stuck = false;
      const int jb = SL * wave;              // first column (step) of this wave's block
      // ---- steps of the earlier blocks, as their owners publish them
#pragma unroll 1
      for (int j = 0; j < min(jb, npiv); ++j) {
        const int q = j & (RING - 1);
        int pp = 0;
        double rp = 0.0;
        if (!stuck) stuck = !lds_wait_rec(&s_rec[q], j + 1, pp, rp);
        // all loads first, then branch-free masking: a conditional load would be
        // sunk into its own branch and serialize the LDS latency
        double rv[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) rv[i] = s_raw[q][lane + 64 * i];
        const int Lp = pp & 63;
        const int iLp = (pp >> 6) & (RPL - 1);
        if (lane == Lp) act &= ~(1u << iLp);
        // rows chosen earlier hold garbage from here on (their slices were saved when
        // they were chosen), so the multipliers need no masking
        double lp[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) lp[i] = rv[i] * rp;
        double u[SL];
        read_owner_row(x, 0, iLp, Lp, u);
        if (lane == 0) {   // this wave's slice of pivot row j, final from now on
#pragma unroll
          for (int c = 0; c < SL; ++c) s_lu[j][SL * wave + c] = u[c];
        }
#pragma unroll
        for (int t = 0; t < SL; ++t) {
#pragma unroll
          for (int i = 0; i < RPL; ++i) x[i][t] = fma(-lp[i], u[t], x[i][t]);
        }
        if ((j & (SL - 1)) == SL - 1 && lane == 0)   // done with block j / SL
          __hip_atomic_fetch_add(&s_bcons[j / SL], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      // the ring slots of this block last held block wave - 2: wait until all of its
      // consumers (the waves after it) are done with it
      if (wave >= RING / SL && jb < npiv && !stuck)
        stuck = !lds_wait_ge(&s_bcons[wave - RING / SL], NW - 1 - (wave - RING / SL));
      // ---- this wave's block: eight pivot steps back to back, all in registers
      __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int t = 0; t < SL; ++t) {
        const int j = jb + t;
        if (j < npiv) {
          const int r = j & (RING - 1);
#pragma unroll
          for (int i = 0; i < RPL; ++i) s_raw[r][lane + 64 * i] = x[i][t];
          unsigned k[RPL];
#pragma unroll
          for (int i = 0; i < RPL; ++i) k[i] = pivot_key(x[i][t], i, act);
#pragma unroll
          for (int w = 1; w < RPL; w *= 2)
#pragma unroll
            for (int i = 0; i + w < RPL; i += 2 * w) k[i] = max(k[i], k[i + w]);
          const unsigned best = k[0];
          // each lane's best value of the column by a select tree (runs beside the
          // wave maximum)
          const int bi = (int)(best & 7u);
          double v[RPL];
#pragma unroll
          for (int i = 0; i < RPL; ++i) v[i] = x[i][t];
#pragma unroll
          for (int w = 1; w < RPL; w *= 2)
#pragma unroll
            for (int i = 0; i + w < RPL; i += 2 * w) v[i] = ((bi & w) != 0) ? v[i + w] : v[i];
          const unsigned kmax = wave_max_u32(best);
          const unsigned long long bal = __ballot(best == kmax);
          const int L = bal ? (__ffsll((long long)bal) - 1) : 0;
          const int iL = (int)(kmax & 7u) & (RPL - 1);
          // the winning lane saves this wave's slice of the pivot row (multipliers left
          // of column t, U entries from t on: final, the row is never updated again)
          // for the LU factors and for the broadcast below
          if (lane == L) {
#pragma unroll
            for (int i = 0; i < RPL; ++i)
              if (i == iL) {
#pragma unroll
                for (int c = 0; c < SL; ++c) s_lu[j][SL * wave + c] = x[i][c];
              }
          }
          const double rpj = pivot_recip(readlane_d(v[0], L));
          if (lane == L) act &= ~(1u << iL);
          // every lane stores the same uniform values: no divergent branch
          s_rec[r].p = L + 64 * iL;
          s_rec[r].rp = rpj;
          s_sel[j] = L + 64 * iL;
          __hip_atomic_store(&s_rec[r].stamp, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          asm volatile("s_wakeup" ::: "memory");   // end the sleep of waiting waves
          // this column's multipliers (L factor); the rows chosen so far, this pivot
          // row included, take garbage, their slices being saved already
          double l[RPL];
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            l[i] = x[i][t] * rpj;
            x[i][t] = l[i];
          }
          if (t + 1 < SL) {   // step j on the rest of the block, the next column first
            double u[SL];
            // lane L's stores above precede these loads in the wave's LDS order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = t + 1; c < SL; ++c) u[c] = s_lu[j][SL * wave + c];   // broadcast loads
#pragma unroll
            for (int c = t + 1; c < SL; ++c) {
#pragma unroll
              for (int i = 0; i < RPL; ++i) x[i][c] = fma(-l[i], u[c], x[i][c]);
            }
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
      if (stuck && lane == 0) atomicOr(&m.err[0], 2);
      __syncthreads();
      // A pivot row is left alone by every later step: the slices of rows chosen up
      // to a wave's last step were saved when chosen, the rows chosen after it hold
      // their final values in that wave's columns now.
      for (int r = tid; r < TR; r += TT) s_stepof[r] = -1;
      __syncthreads();
      if (tid < npiv) s_stepof[min(max(s_sel[tid], 0), TR - 1)] = tid;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int st = s_stepof[lane + 64 * i];
        if (st >= jb + SL) {
#pragma unroll
          for (int t = 0; t < SL; ++t) s_lu[st][SL * wave + t] = x[i][t];
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

// Given row order: factors the 64 x 64 block at rows r0s.., columns c0s.. of src
// (leading dimension ld) without a search and publishes it: tri_out (row-major,
// unit L strictly below the diagonal, U on and above), *logdet_out = sum log|u_jj|
// (fixed order), err[1] |= 1 when a multiplier exceeds tau in magnitude or a pivot
// is zero; s_piv holds 128 doubles (pivots, their logs).  Right-looking in four
// 16-column panels on the block in LDS (A, 64 x LDA):
// wave 0 factors a panel with its rows in registers (lane = row, the pivot row
// broadcast by cross-lane reads, no barrier per step), the 16 x 16 unit-lower
// solve gives the U rows right of the panel, and the matrix cores take the Schur
// update.  All 256 threads of the workgroup.
__device__ __noinline__ void lu64_publish(const double* src, int ld, int r0s, int c0s, double tau,
                             double* tri_out, double* logdet_out, int* err, double (*A)[LDA],
                             double* s_piv) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
#pragma unroll
  for (int k = 0; k < NB * NB / 256; ++k) {
    const int e = tid + 256 * k;
    A[e / NB][e % NB] = src[(int64_t)(r0s + e / NB) * ld + c0s + e % NB];
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int kb = 0; kb < NB / 16; ++kb) {
    const int cb = 16 * kb;
    if (wave == 0) {   // panel: rows cb..63, columns cb..cb+15; lane = row
      // the serial chain of the factorization: ahead of co-resident waves
      __builtin_amdgcn_s_setprio(3);
      double p[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) p[t] = (lane >= cb) ? A[lane][cb + t] : 0.0;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = cb + jj;
        const double piv = readlane_d(p[jj], j);
        double u[16];
#pragma unroll
        for (int t = jj + 1; t < 16; ++t) u[t] = readlane_d(p[t], j);
        const double rp = pivot_recip(piv);
        bad |= (piv == 0.0);
        if (lane > j) {
          const double l = p[jj] * rp;
          bad |= !(fabs(l) <= tau);
          p[jj] = l;
#pragma unroll
          for (int t = jj + 1; t < 16; ++t) p[t] = fma(-l, u[t], p[t]);
        }
        if (lane == 0) s_piv[j] = piv;
      }
      if (lane >= cb) {
#pragma unroll
        for (int t = 0; t < 16; ++t) A[lane][cb + t] = p[t];
      }
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    // log|u_jj| of this panel's pivots on a wave the next phase leaves idle
    if (wave == 1 && lane < 16) s_piv[NB + cb + lane] = log(fabs(s_piv[cb + lane]));
    if (kb + 1 < NB / 16) {
      const int nr = NB - cb - 16;   // rows and columns right of / below the panel
      // U rows of the panel right of it: solve L11 X = A12 (unit lower, 16 x 16),
      // one column per thread
      if (tid < nr) {
        const int c = cb + 16 + tid;
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double acc = A[cb + r][c];
#pragma unroll
          for (int t = 0; t < r; ++t) acc = fma(-A[cb + r][cb + t], x[t], acc);
          x[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) A[cb + r][c] = x[r];
      }
      __syncthreads();
      // Schur update A22 -= L21 U12 on 16 x 16 tiles, k = 16 (four matrix-core steps)
      const int nt = nr / 16;
      const int lr = lane & 15;
      const int lk = lane >> 4;
      for (int tile = wave; tile < nt * nt; tile += 4) {
        const int r0t = cb + 16 + 16 * (tile / nt);
        const int c0t = cb + 16 + 16 * (tile % nt);
        f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          acc = mfma_f64_16x16x4(A[r0t + lr][cb + 4 * kk + lk], A[cb + 4 * kk + lk][c0t + lr], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) A[r0t + 4 * r + lk][c0t + lr] -= acc[r];
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < NB * NB / 256; ++k) {
    const int e = tid + 256 * k;
    tri_out[e] = A[e / NB][e % NB];
  }
  __syncthreads();
  if (tid < 64) {
    const double ls = wave_sum(s_piv[NB + tid]);
    if (tid == 0) *logdet_out = ls;
  }
  if (__syncthreads_or(bad ? 1 : 0) && tid == 0) atomicOr(&err[1], 1);
}

// ---- pieces of an inner step on IU_ROWS rows (see the file comment) ----
// LDS of one workgroup: the LU factors of the pivot block (later the pivot rows of
// one column chunk), the inverses of the 16 x 16 diagonal blocks with a scratch
// block, and the IU_ROWS x 64 right-hand side C.
struct StepLds {
  double a[NB * LDA];                        // LU (L strictly lower, U) / Rs
  double b[8 * 16 * 17 + IU_ROWS * 17];      // Di: inverses, 0-3 of U, 4-7 of L; Ts
  double c[IU_ROWS][LDA];                    // C
};

// Factors of the pivot block (row-major 64 x 64, device) into LDS; with inverses,
// also the inverses of its 16 x 16 diagonal blocks (thread (blk, col) runs one
// column of a 16 x 16 substitution).  Ends with a barrier.
__device__ void step_factors(StepLds& L, const double* tri, bool inverses = true) {
  const int tid = threadIdx.x;
  double (*LU)[LDA] = reinterpret_cast<double (*)[LDA]>(L.a);
  double (*Di)[16][17] = reinterpret_cast<double (*)[16][17]>(L.b);
  {
    double t[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] = tri[tid + 256 * k];
#pragma unroll
    for (int k = 0; k < 16; ++k) LU[(tid + 256 * k) / NB][(tid + 256 * k) % NB] = t[k];
  }
  __syncthreads();
  if (inverses && tid < 128) {
    const int blk = tid >> 4;
    const int c = tid & 15;
    const int b0 = (blk & 3) * 16;
    double x[16];
    if (blk < 4) {  // upper: X U_bb = I  (column c of U_bb^{-1} by back substitution)
      double rd[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) rd[r] = 1.0 / LU[b0 + r][b0 + r];
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
        for (int t = r + 1; t < 16; ++t) acc = fma(-LU[b0 + r][b0 + t], x[t], acc);
        x[r] = (r <= c) ? acc * rd[r] : 0.0;
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
  __syncthreads();
}

// C U = C and G L = C in place on the IU_ROWS x 64 block C (LDS), blocks of 16 with
// the diagonal-block inverses: C_b = (C_b - C_{<b} U_{<b,b}) inv(U_bb) left to right,
// then G_b = (C_b - G_{>b} L_{>b,b}) inv(L_bb) right to left.  Every loop has a
// compile-time trip count (each thread owns IU_ROWS * 16 / 256 elements per block),
// so the LDS loads are issued ahead of the FMA chains (the long sums unrolled by 8:
// fully unrolled they spill); the products with the diagonal-block inverses run
// over all 16 terms, the inverses holding exact zeros outside their triangle.
// check: returns true when |C| after the first solve (the multipliers of candidate
// rows) exceeds tau anywhere.
__device__ bool step_solve(StepLds& L, bool check, double tau) {
  const int tid = threadIdx.x;
  double (*LU)[LDA] = reinterpret_cast<double (*)[LDA]>(L.a);
  double (*Di)[16][17] = reinterpret_cast<double (*)[16][17]>(L.b);
  double (*Ts)[17] = reinterpret_cast<double (*)[17]>(L.b + 8 * 16 * 17);
  double (*Cs)[LDA] = L.c;
  static_assert(IU_ROWS * 16 % 256 == 0, "whole elements per thread");
  constexpr int EPT = IU_ROWS * 16 / 256;
  bool bad = false;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e >> 4;
      const int c = b * 16 + (e & 15);
      double acc = Cs[r][c];
#pragma unroll 8
      for (int t = 0; t < b * 16; ++t) acc = fma(-Cs[r][t], LU[t][c], acc);
      Ts[r][e & 15] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e >> 4;
      const int cl = e & 15;
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) acc = fma(Ts[r][t], Di[b][t][cl], acc);
      Cs[r][b * 16 + cl] = acc;
      if (check) bad |= !(fabs(acc) <= tau);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 3; b >= 0; --b) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e >> 4;
      const int c = b * 16 + (e & 15);
      double acc = Cs[r][c];
#pragma unroll 8
      for (int t = (b + 1) * 16; t < NB; ++t) acc = fma(-Cs[r][t], LU[t][c], acc);
      Ts[r][e & 15] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = tid + 256 * k;
      const int r = e >> 4;
      const int cl = e & 15;
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) acc = fma(Ts[r][t], Di[4 + b][t][cl], acc);
      Cs[r][b * 16 + cl] = acc;
    }
    __syncthreads();
  }
  return bad;
}

// Output of the step for IU_ROWS rows, column chunk by column chunk: -G in the
// inner block c0, base - G R elsewhere.  rrow(j) is pivot row j (nbo doubles),
// base_row(r) row r of this block's input (nullptr inside the pivot block: base 0),
// out_row(r) where output row r goes.  The next chunk of pivot rows is loaded into
// registers while the current one is multiplied.
template <class RRow, class Base, class Out>
__device__ void step_output(StepLds& L, int nbo, int c0, RRow rrow, Base base_row, Out out_row) {
  const int tid = threadIdx.x;
  double (*Rs)[LDA] = reinterpret_cast<double (*)[LDA]>(L.a);
  double (*Cs)[LDA] = L.c;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int rb = w >> 1;
  const int cb = (w & 1) * 2;
  const int lr = lane & 15;
  const int lk = lane >> 4;
  auto load_r = [&](int cc, double (&t)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      t[k] = rrow(e / NB)[cc + e % NB];
    }
  };
  int cc = (c0 == 0) ? NB : 0;   // first chunk outside the inner block
  double t[16];
  if (cc < nbo) load_r(cc, t);
  for (int e = tid; e < IU_ROWS * NB; e += 256) out_row(e / NB)[c0 + e % NB] = -Cs[e / NB][e % NB];
  while (cc < nbo) {
    int nx = cc + NB;
    if (nx == c0) nx += NB;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int e = tid + 256 * k;
      Rs[e / NB][e % NB] = t[k];
    }
    double base[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lk;
        const double* br = base_row(rr);
        base[b][r] = (br != nullptr) ? br[cc + (cb + b) * 16 + lr] : 0.0;
      }
    __syncthreads();
    if (nx < nbo) load_r(nx, t);
    f64x4 acc[2];
    mm32x64(Cs, Rs, acc);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lk;
        out_row(rr)[cc + (cb + b) * 16 + lr] = base[b][r] - acc[b][r];
      }
    __syncthreads();
    cc = nx;
  }
}

// Right-hand side of C U = Acol for IU_ROWS rows, in two halves so that its loads
// can be issued before the factors are set up: rhs_load reads src_row(r)'s inner
// block, or forms -E (identity rows, as C = -U^{-1} gives the rows of S^{-1}) inside
// the pivot block (inblock: local row r is pivot row row_in_block + r); rhs_store
// puts it into LDS and ends with a barrier.
constexpr int RHS_PT = IU_ROWS * NB / 256;
template <class Src>
__device__ void rhs_load(bool inblock, int row_in_block, int c0, Src src_row, double (&t)[RHS_PT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < RHS_PT; ++k) {
    const int e = tid + 256 * k;
    const int r = e / NB;
    const int c = e % NB;
    t[k] = inblock ? ((row_in_block + r == c) ? -1.0 : 0.0) : src_row(r)[c0 + c];
  }
}
__device__ void rhs_store(StepLds& L, const double (&t)[RHS_PT]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < RHS_PT; ++k) {
    const int e = tid + 256 * k;
    L.c[e / NB][e % NB] = t[k];
  }
  __syncthreads();
}

// Given row order: true once a multiplier check of either matrix has failed (the
// attempt will be redone with the search, so its remaining steps are skipped).  Read
// by one thread and shared, so that the whole workgroup takes the same branch.
__device__ __forceinline__ bool given_aborted(const GjeArgs& A, int* s_flag) {
  if (threadIdx.x == 0) {
    int f = 0;
    for (int z = 0; z < A.nmat; ++z)
      f |= __hip_atomic_load(&A.m[z].err[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = f;
  }
  __syncthreads();
  return *s_flag != 0;
}

// Inner Gauss-Jordan step on the panel, IU_ROWS rows per workgroup (see the file
// comment): C U = Acol and G L = C are solved by 16-column block substitution with
// explicit inverses of the 16 x 16 diagonal blocks only, then out = base - G R.
// Search (KNOWN = false): rows are read through the step's row maps, the factors
// are the tournament root's.  Given order (KNOWN = true): the pivot rows are the
// positions r0..r0+63, whose factors were published before the launch (tri slot
// c0 / 64 % 2); the multipliers of the rows below the block are checked against
// tau, and the last of the two workgroups that produce the next block's pivot rows
// factors that block (lu64_publish, the other slot) for the next launch.  Those two
// workgroups take the first two indices, so that the factorization runs beside the
// other workgroups' updates.
template <bool KNOWN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void inner_update_kernel(GjeArgs A) {
  __shared__ __attribute__((aligned(16))) StepLds L;
  __shared__ int s_src[IU_ROWS];
  __shared__ int s_q[NB];
  __shared__ int s_last;

  const GjeMat& m = A.m[blockIdx.y];
  const double* P = m.P[A.pcur];
  double* Q = m.P[A.pcur ^ 1];
  const int nbo = A.nbo;
  const int r0 = A.r0;
  const int c0 = A.c0;
  const int tid = threadIdx.x;
  const bool next = KNOWN && c0 + NB < nbo;   // a next pivot block to factor
  const int nrb = A.n_pad / IU_ROWS;
  const int row0 = (next ? (blockIdx.x + (r0 + NB) / IU_ROWS) % nrb : blockIdx.x) * IU_ROWS;
  const bool inblock = row0 >= r0 && row0 < r0 + NB;
  const bool below = row0 >= r0 + NB;
  const double* tri = KNOWN ? m.tri + (int64_t)((c0 / NB) & 1) * NB * NB : m.tri;
  if (KNOWN && given_aborted(A, &s_last)) return;
  // the panel chain is the critical path beside the trailing update's waves
  __builtin_amdgcn_s_setprio(2);

  if (KNOWN) {
    if (tid < IU_ROWS) s_src[tid] = row0 + tid;
    if (tid < NB) s_q[tid] = r0 + tid;
  } else {
    // source row of each output row: the selected row inside the block, the displaced
    // block row at a vacated position, the row itself elsewhere
    if (tid < IU_ROWS) s_src[tid] = inblock ? m.qsel[row0 - r0 + tid] : row0 + tid;
    if (tid < NB) s_q[tid] = m.qsel[tid];
    __syncthreads();
    if (!inblock && tid < NB) {
      const int nv = m.vac[0];
      const int v = m.vac[1 + tid];
      const int src = m.vac[65 + tid];
      if (tid < nv && v >= row0 && v < row0 + IU_ROWS) s_src[v - row0] = src;
    }
  }
  __syncthreads();   // the row maps above are complete
  double rhs[RHS_PT];
  rhs_load(inblock, row0 - r0, c0, [&](int r) { return P + (int64_t)s_src[r] * nbo; }, rhs);
  step_factors(L, tri);
  rhs_store(L, rhs);
  const bool bad = step_solve(L, KNOWN && below, A.tau);
  if (KNOWN && __syncthreads_or(bad ? 1 : 0) && tid == 0) atomicOr(&m.err[1], 1);
  step_output(
      L, nbo, c0, [&](int j) { return P + (int64_t)s_q[j] * nbo; },
      [&](int r) -> const double* { return inblock ? nullptr : P + (int64_t)s_src[r] * nbo; },
      [&](int r) { return Q + (int64_t)(row0 + r) * nbo; });
  if (next && row0 >= r0 + NB && row0 < r0 + 2 * NB) {
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const int old = atomicAdd(&m.cnt[0], 1);
      s_last = (old == NB / IU_ROWS - 1);
      if (s_last) atomicExch(&m.cnt[0], 0);
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      lu64_publish(Q, nbo, r0 + NB, c0 + NB, A.tau, m.tri + (int64_t)(((c0 / NB) + 1) & 1) * NB * NB,
                   m.logdet + (r0 + NB) / NB, m.err, reinterpret_cast<double (*)[LDA]>(L.a), L.b);
    }
  }
}

// The first pivot block of a panel in a given row order (one workgroup per matrix):
// its factors to tri slot 0.
__global__ __launch_bounds__(256) void lu64_kernel(GjeArgs A) {
  __shared__ double s_blk[NB][LDA];
  __shared__ double s_piv[2 * NB];
  __shared__ int s_abort;
  if (given_aborted(A, &s_abort)) return;
  const GjeMat& m = A.m[blockIdx.y];
  lu64_publish(m.P[A.pcur], A.nbo, A.k0, 0, A.tau, m.tri, m.logdet + A.k0 / NB, m.err, s_blk, s_piv);
}

__global__ void begin_kernel(GjeArgs A, int nslots, int ncnt) {
  const GjeMat& m = A.m[blockIdx.y];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pad; p += gridDim.x * blockDim.x)
    m.ptot[p] = A.known ? min(max(m.order[p], 0), A.n_pad - 1) : p;
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < nslots; t += blockDim.x) m.logdet[t] = 0.0;
    for (int t = threadIdx.x; t < ncnt; t += blockDim.x) m.cnt[t] = 0;
    if (threadIdx.x < 4) m.err[threadIdx.x] = 0;
  }
}

// Four panel rows per workgroup, one wave per row, 16-byte loads of the contiguous
// row segment (n_pad and k0 are multiples of 64).
__global__ __launch_bounds__(256) void panel_copy_kernel(GjeArgs A) {
  const GjeMat& m = A.m[blockIdx.y];
  const int nbo = A.nbo;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= A.n_pad) return;
  // the first outer step of a given-order inversion reads the rows in that order
  const bool gather = A.known && A.k0 == 0;
  const int src = gather ? min(max(m.order[i], 0), A.n_pad - 1) : i;
  const f64x2* from = reinterpret_cast<const f64x2*>(m.Min + (int64_t)src * A.n_pad + A.k0);
  f64x2* to = reinterpret_cast<f64x2*>(m.P[A.pcur] + (int64_t)i * nbo);
  for (int q = lane; q < nbo / 2; q += 64) to[q] = from[q];
  if (lane == 0 && m.pi != nullptr) m.pi[i] = src;
}

__global__ void finish_kernel(GjeArgs A) {
  const GjeMat& m = A.m[blockIdx.y];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pad; p += gridDim.x * blockDim.x) {
    const int q = m.ptot[p];
    m.pinv[q] = p;
    if (m.order != nullptr) m.order[p] = q;
  }
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
  hipLaunchKernelGGL(panel_copy_kernel, dim3((a.n_pad + 3) / 4, a.nmat), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gje_tournament(const GjeArgs& a, hipStream_t s) {
  const int ncand = a.n_pad - a.r0;
  const int nleaves = (ncand + TR - 1) / TR;
  hipLaunchKernelGGL(tournament_kernel, dim3(nleaves, a.nmat), dim3(TT), 0, s, a, nleaves);
  return hipGetLastError();
}

hipError_t launch_gje_inner_update(const GjeArgs& a, hipStream_t s) {
  if (a.known)
    hipLaunchKernelGGL(inner_update_kernel<true>, dim3(a.n_pad / IU_ROWS, a.nmat), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(inner_update_kernel<false>, dim3(a.n_pad / IU_ROWS, a.nmat), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gje_lu64(const GjeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lu64_kernel, dim3(1, a.nmat), dim3(256), 0, s, a);
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
