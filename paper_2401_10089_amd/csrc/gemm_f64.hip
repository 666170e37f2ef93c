// FP64 matrix-core GEMM for gfx950 with pluggable operand loaders and fused
// epilogues.  Used for
//  * plain products (the saved square B^2 at s = 0),
//  * the computation-graph nodes P_{j+2} = L_j R_j of the degree-optimal
//    polynomial form, whose epilogue folds the linear combinations into the
//    accumulators so that no P_j is stored,
//  * the rank-NB trailing update of the blocked Gauss-Jordan inversion.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup (2 x 2 waves of 64 x 64),
// k-slabs of 16 staged through LDS with a double buffer; each wave issues
// 16 independent v_mfma_f64_16x16x4 per k-step of 4.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace logm {
namespace {

constexpr int BM = 128;   // default tile
constexpr int BN = 128;
constexpr int BK = 16;
constexpr int PAD = 4;

// Map the linear workgroup id to a tile so that the workgroups that land on one
// XCD (ids congruent mod 8) cover a compact block of tiles and share L2 traffic.
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int total = tiles_m * tiles_n;
  int t = bid;
  if (total >= 64 && (total % 8) == 0) {
    const int per = total / 8;
    t = (bid % 8) * per + bid / 8;  // consecutive tiles for each XCD
  }
  // group rows of 8 tiles so that successive tiles reuse B panels
  const int group = 8;
  const int width = group * tiles_n;
  const int g = t / width;
  const int first_m = g * group;
  const int gm = min(tiles_m - first_m, group);
  const int in = t % width;
  tm = first_m + in % gm;
  tn = in / gm;
}

// Column tiles a launch covers: [a0, a0 + na) followed by [b0, b0 + nb).
struct TileCols {
  int a0, na, b0, nb;
};

// Tile TM x TN per 256-thread workgroup: 2 x 2 waves of (TM/2) x (TN/2), each made
// of MI x NI blocks of 16 x 16 (MI = TM/32, NI = TN/32).  At least two waves per
// SIMD: left alone the compiler keeps the 128 accumulator registers of a 128 x 128
// tile in AGPRs beside about 200 VGPRs, one wave per SIMD, and every barrier and LDS
// wait then idles the matrix core (46.7 TFLOP/s at n = 4096 against 62.2 with two).
template <class Op, int TM = BM, int TN = BN, bool F32 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_kernel(Op op, int M, int N, int K, TileCols tc) {
  constexpr int MI = TM / 32;
  constexpr int NI = TN / 32;
  constexpr int APT = TM * BK / 256;   // A elements per thread per k-slab
  constexpr int BPT = TN * BK / 256;   // B elements per thread per k-slab
  // F32: operands rounded to fp32 when staged, fp32 matrix cores with fp32
  // accumulation; the epilogue still receives the tile widened to fp64
  using T = typename std::conditional<F32, float, double>::type;
  using Acc = typename std::conditional<F32, f32x4, f64x4>::type;
  __shared__ T As[2][BK][TM + PAD];
  __shared__ T Bs[2][BK][TN + PAD];

  op.select(blockIdx.z);
  const int tid = threadIdx.x;
  if constexpr (Op::kCanSkip) {   // a work item given up upstream: nothing to do
    __shared__ int s_skip;
    if (tid == 0) s_skip = op.skip() ? 1 : 0;
    __syncthreads();
    if (s_skip) return;
  }
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wm = wave >> 1;
  const int wn = wave & 1;
  const int tiles_m = (M + TM - 1) / TM;
  const int ntiles = tiles_m * (tc.na + tc.nb);
  // persistent: a workgroup walks tiles blockIdx.x, + gridDim.x, ...; with a grid that
  // is a multiple of 8 every tile of one workgroup stays on the same XCD group
  for (int bid = blockIdx.x; bid < ntiles; bid += gridDim.x) {
  int tm, vn;
  tile_of(bid, tiles_m, tc.na + tc.nb, tm, vn);
  const int tn = (vn < tc.na) ? tc.a0 + vn : tc.b0 + (vn - tc.na);
  const int row0 = tm * TM;
  const int col0 = tn * TN;

  if (op.copy_tile(row0, col0, TN)) {
    for (int e = tid; e < TM * TN; e += 256) {
      const int i = row0 + e / TN;
      const int j = col0 + e % TN;
      if (i < M && j < N) op.copy(i, j);
    }
    continue;
  }

  // global -> register staging assignment
  const int ra = tid / (BK / APT);          // A: row within tile
  const int ka = (tid % (BK / APT)) * APT;  // A: first k of APT
  const int kb = tid / (TN / BPT);          // B: k row
  const int cb = (tid % (TN / BPT)) * BPT;  // B: first column of BPT
  const bool a_row_ok = (row0 + ra) < M;
  const double* arow = a_row_ok ? op.a_row(row0 + ra) : nullptr;
  const bool full_n = (col0 + TN) <= N;

  double va[APT], vb[BPT];
  auto gload = [&](int k0) {
    const int kA = k0 + ka;
    if (a_row_ok && kA + APT <= K && ((reinterpret_cast<uintptr_t>(arow + kA) & 15) == 0)) {
      const f64x2* p = reinterpret_cast<const f64x2*>(arow + kA);
#pragma unroll
      for (int e = 0; e < APT / 2; ++e) {
        f64x2 v = p[e];
        va[2 * e] = v.x;
        va[2 * e + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < APT; ++e) va[e] = (a_row_ok && kA + e < K) ? arow[kA + e] : 0.0;
    }
    const int kB = k0 + kb;
    if (kB < K) {
      const double* brow = op.b_row(kB) + col0 + cb;
      if (full_n && ((reinterpret_cast<uintptr_t>(brow) & 15) == 0)) {
        const f64x2* p = reinterpret_cast<const f64x2*>(brow);
#pragma unroll
        for (int e = 0; e < BPT / 2; ++e) {
          f64x2 v = p[e];
          vb[2 * e] = v.x;
          vb[2 * e + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < BPT; ++e) vb[e] = (col0 + cb + e < N) ? brow[e] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < BPT; ++e) vb[e] = 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < APT; ++e) As[buf][ka + e][ra] = (T)va[e];
#pragma unroll
    for (int e = 0; e < BPT; ++e) Bs[buf][kb][cb + e] = (T)vb[e];
  };

  Acc acc[MI][NI];
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = Acc{0, 0, 0, 0};

  const int nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  const int lr = lane & 15;
  const int lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const bool more = (kt + 1) < nk;
    if (more) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      T af[MI], bf[NI];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi) af[mi] = As[buf][kk * 4 + lk][wm * (TM / 2) + mi * 16 + lr];
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) bf[ni] = Bs[buf][kk * 4 + lk][wn * (TN / 2) + ni * 16 + lr];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = mfma_16x16x4(af[mi], bf[ni], acc[mi][ni]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: per 16-row group each lane owns four rows -- 4r + lk for the fp64
  // instruction, 4 lk + r for the fp32 one (element r of lane l) -- and columns
  // 16 ni + lr (ni < NI) of the wave's block
#pragma unroll
  for (int mi = 0; mi < MI; ++mi) {
    int rows[4], cols[NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      rows[r] = row0 + wm * (TM / 2) + mi * 16 + (F32 ? 4 * lk + r : 4 * r + lk);
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) cols[ni] = col0 + wn * (TN / 2) + ni * 16 + lr;
    double v[4][NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) v[r][ni] = (double)acc[mi][ni][r];
    op.template store_group<NI>(rows, cols, v, M, N);
  }
  }
}

// ------------------------------------------------------------------ ops ---
struct PlainOp {
  static constexpr bool kCanSkip = false;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha, beta;
  __device__ void select(int) {}
  __device__ bool copy_tile(int, int, int) const { return false; }
  __device__ void copy(int, int) const {}
  __device__ const double* a_row(int i) const { return A + (int64_t)i * lda; }
  __device__ const double* b_row(int k) const { return B + (int64_t)k * ldb; }
  // all loads of the group are issued before any store
  template <int NI>
  __device__ void store_group(const int* rows, const int* cols, double (*v)[NI], int M, int N) const {
    double old[4][NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const int i = min(rows[r], M - 1);
        const int j = min(cols[ni], N - 1);
        old[r][ni] = (beta == 0.0) ? 0.0 : C[(int64_t)i * ldc + j];
      }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni)
        if (rows[r] < M && cols[ni] < N)
          C[(int64_t)rows[r] * ldc + cols[ni]] = alpha * v[r][ni] + beta * old[r][ni];
  }
};

struct PolyOp {
  static constexpr bool kCanSkip = false;
  PolyGemmArgs a;
  __device__ void select(int) {}
  __device__ bool copy_tile(int, int, int) const { return false; }
  __device__ void copy(int, int) const {}
  __device__ const double* a_row(int i) const { return a.Lf + (int64_t)i * a.ld; }
  __device__ const double* b_row(int k) const { return a.Rf + (int64_t)k * a.ld; }
  // tiles can overhang the n x n matrices (n_pad is a multiple of 64, tiles are
  // 128 wide): loads are clamped into the matrix and stores predicated
  template <int NI>
  __device__ void store_group(const int* rows, const int* cols, double (*v)[NI], int M, int N) const {
    int64_t o[4][NI];
    bool in[4][NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        in[r][ni] = rows[r] < M && cols[ni] < N;
        o[r][ni] = (int64_t)min(rows[r], M - 1) * a.ld + min(cols[ni], N - 1);
      }
    for (int t = 0; t < a.nacc; ++t) {
      double* p = a.acc[t];
      const double cf = a.coef[t];
      double old[4][NI];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) old[r][ni] = p[o[r][ni]];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
          if (in[r][ni]) p[o[r][ni]] = fma(cf, v[r][ni], old[r][ni]);
    }
    if (a.dst != nullptr) {
      double b[4][NI];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) b[r][ni] = a.base[o[r][ni]];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
          if (in[r][ni] && rows[r] < a.nvalid && cols[ni] < a.nvalid)
            a.dst[(int64_t)rows[r] * a.ldd + cols[ni]] = a.scale * (b[r][ni] + a.ycoef * v[r][ni]);
    }
  }
};

// Rank-nbo Gauss-Jordan trailing update (see gje.hip for the derivation):
//   out[i][c] = U[i][c-k0]                                    c in K
//   out[i][c] = [i not in K] * Min[pi(i)][c] + sum_t U[i][t] Min[pi(k0+t)][c]   otherwise
// where U (n_pad x nbo) is the fully processed panel; pi == nullptr is the identity.
// With Pn set, the columns [pn_k0, pn_k0 + pn_ld) go to the next step's panel Pn
// (leading dimension pn_ld) instead of Mout: the look-ahead update of an inversion
// in a given row order writes that panel directly.
struct GjeOuterOp {
  static constexpr bool kCanSkip = true;
  const int* abort[2];   // given row order: the multiplier-check flags (err[1]) of both matrices
  const double* U[2];
  const double* Min[2];
  const int* pi[2];
  double* Mout[2];
  double* Pn[2];
  int64_t ld;
  int k0, nbo;
  int pn_k0, pn_ld;
  const double* u;
  const double* mi;
  const int* p;
  double* mo;
  double* pn;
  __device__ void select(int z) {
    const bool one = (z != 0);
    u = one ? U[1] : U[0];
    mi = one ? Min[1] : Min[0];
    p = one ? pi[1] : pi[0];
    mo = one ? Mout[1] : Mout[0];
    pn = one ? Pn[1] : Pn[0];
  }
  __device__ int row_of(int i) const { return p != nullptr ? p[i] : i; }
  // a rejected given-order attempt is redone with the search: its remaining updates
  // are skipped
  __device__ bool skip() const {
    bool r = false;
#pragma unroll
    for (int z = 0; z < 2; ++z)
      if (abort[z] != nullptr) r |= __hip_atomic_load(abort[z], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    return r;
  }
  __device__ bool copy_tile(int, int col0, int tn) const { return col0 >= k0 && col0 + tn <= k0 + nbo; }
  __device__ void copy(int i, int j) const { mo[(int64_t)i * ld + j] = u[(int64_t)i * nbo + (j - k0)]; }
  __device__ const double* a_row(int i) const { return u + (int64_t)i * nbo; }
  __device__ const double* b_row(int t) const { return mi + (int64_t)row_of(k0 + t) * ld; }
  // branch-free: every load of the group is issued before the first store
  template <int NI>
  __device__ void store_group(const int* rows, const int* cols, double (*v)[NI], int M, int N) const {
    const double* src[4];
    bool rowk[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = min(rows[r], M - 1);
      src[r] = mi + (int64_t)row_of(i) * ld;
      rowk[r] = rows[r] >= k0 && rows[r] < k0 + nbo;
    }
    bool colk[NI];
    bool anyk = false;
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      colk[ni] = cols[ni] >= k0 && cols[ni] < k0 + nbo;
      anyk |= colk[ni];
    }
    double base[4][NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) base[r][ni] = src[r][min(cols[ni], N - 1)];
    double uv[4][NI];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) uv[r][ni] = 0.0;
    if (anyk) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
          if (colk[ni]) uv[r][ni] = u[(int64_t)min(rows[r], M - 1) * nbo + (cols[ni] - k0)];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const double out = colk[ni] ? uv[r][ni] : ((rowk[r] ? 0.0 : base[r][ni]) + v[r][ni]);
        if (rows[r] < M && cols[ni] < N) {
          const int cn = cols[ni] - pn_k0;
          if (pn != nullptr && cn >= 0 && cn < pn_ld)
            pn[(int64_t)rows[r] * pn_ld + cn] = out;
          else
            mo[(int64_t)rows[r] * ld + cols[ni]] = out;
        }
      }
  }
};

// max_wgs > 0 caps the workgroups per matrix (the kernel then loops over tiles).
template <class Op, int TM = BM, int TN = BN, bool F32 = false>
hipError_t launch(const Op& op, int M, int N, int K, int nz, TileCols tc, hipStream_t s,
                  int max_wgs = 0) {
  const int tiles = ((M + TM - 1) / TM) * (tc.na + tc.nb);
  if (tiles == 0) return hipSuccess;
  const int grid = (max_wgs > 0 && tiles > max_wgs) ? max_wgs : tiles;
  hipLaunchKernelGGL((gemm_kernel<Op, TM, TN, F32>), dim3(grid, 1, nz), dim3(256), 0, s, op, M,
                     N, K, tc);
  return hipGetLastError();
}

TileCols all_cols(int N) { return TileCols{0, (N + BN - 1) / BN, 0, 0}; }

}  // namespace

hipError_t launch_gemm_plain(int M, int N, int K, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             hipStream_t s) {
  PlainOp op{A, lda, B, ldb, C, ldc, alpha, beta};
  return launch(op, M, N, K, 1, all_cols(N), s);
}

hipError_t launch_gemm_poly(int n, const PolyGemmArgs& a, bool fp32, hipStream_t s) {
  PolyOp op{a};
  if (fp32) return launch<PolyOp, BM, BN, true>(op, n, n, n, 1, all_cols(n), s);
  return launch(op, n, n, n, 1, all_cols(n), s);
}

hipError_t launch_gje_outer_update(const GjeArgs& a, int c_lo, int c_hi, bool inside,
                                   int max_wgs, hipStream_t s, double* const* next_panel,
                                   int next_nbo) {
  GjeOuterOp op{};
  for (int z = 0; z < a.nmat; ++z) {
    op.U[z] = a.m[z].P[a.pcur];
    op.Min[z] = a.m[z].Min;
    op.pi[z] = a.m[z].pi;
    op.Mout[z] = a.m[z].Mout;
    op.Pn[z] = (next_panel != nullptr) ? next_panel[z] : nullptr;
    op.abort[z] = a.known ? a.m[z].err + 1 : nullptr;
  }
  op.ld = a.n_pad;
  op.k0 = a.k0;
  op.nbo = a.nbo;
  op.pn_k0 = c_lo;
  op.pn_ld = next_nbo;
  if (inside) {
    // the look-ahead columns are on the critical path: small tiles spread them over
    // every CU (c_lo is a multiple of 128, so also of 64)
    constexpr int ST = 64;
    const int tn = (a.n_pad + ST - 1) / ST;
    const int t_lo = std::min(std::max(c_lo / ST, 0), tn);
    const int t_hi = std::min(std::max((c_hi + ST - 1) / ST, t_lo), tn);
    return launch<GjeOuterOp, ST, ST>(op, a.n_pad, a.n_pad, a.nbo, a.nmat,
                                      TileCols{t_lo, t_hi - t_lo, 0, 0}, s, max_wgs);
  }
  const int tn = (a.n_pad + BN - 1) / BN;
  const int t_lo = std::min(std::max(c_lo / BN, 0), tn);
  const int t_hi = std::min(std::max((c_hi + BN - 1) / BN, t_lo), tn);
  return launch(op, a.n_pad, a.n_pad, a.nbo, a.nmat, TileCols{0, t_lo, t_hi, tn - t_hi}, s,
                max_wgs);
}

}  // namespace logm
