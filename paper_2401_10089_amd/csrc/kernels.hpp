// Internal launch interface between the host driver and the HIP kernels.
// Not part of the public C ABI (include/logm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "algo.hpp"

namespace logm {

// ----------------------------------------------------------------- GEMM ----
// C = alpha * A * B + beta * C, row-major, fp64 MFMA.  M, N, K arbitrary >= 1.
hipError_t launch_gemm_plain(int M, int N, int K, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                             hipStream_t s);

// Graph-node product P = Lf * Rf (n x n, leading dimension ld) whose result is
// never stored: the epilogue adds coef[t] * P into accumulator acc[t] for every
// t < nacc, and, when dst != nullptr, writes dst = scale * (base + ycoef * P)
// restricted to the leading nvalid x nvalid block (leading dimension ldd).  The
// first product of the largest scheme feeds the most accumulators: the two factors
// of each later product and the output sum.
struct PolyGemmArgs {
  static constexpr int kMaxAcc = 2 * (kKMax - 2) + 1;
  const double* Lf;
  const double* Rf;
  int64_t ld;
  int nacc;
  double* acc[kMaxAcc];
  double coef[kMaxAcc];
  double* dst;
  int64_t ldd;
  const double* base;
  double ycoef;
  double scale;
  int nvalid;
};
// fp32: the product runs on the fp32 matrix cores (operands rounded to fp32, fp32
// accumulation); the accumulators and the output stay fp64.
hipError_t launch_gemm_poly(int n, const PolyGemmArgs& a, bool fp32, hipStream_t s);

// ------------------------------------------------------ Gauss-Jordan ------
// Per-matrix state of the blocked Gauss-Jordan inversion (see gje.hip).
struct GjeMat {
  const double* Min;     // matrix at the start of the outer step (n_pad x n_pad, ld n_pad)
  double* Mout;          // matrix after the outer step
  double* P[2];          // ping-pong panels n_pad x nbo (ld = nbo)
  double* tri;           // 64 x 64: LU factors of the current pivot block (pivot order);
                         // a given order alternates two such slots by inner step
  int* pi;               // n_pad: gather map of the current outer step
  int* ptot;             // n_pad: accumulated row order (position -> original row)
  int* pinv;             // n_pad: inverse of ptot (filled by launch_gje_finish)
  int* qsel;             // 64 selected positions of the current inner step
  int* vac;              // [0] = count, [1..64] vacated positions, [65..128] their sources
  int* cand;             // tournament scratch
  int* cnt;              // tournament arrival counters (self-resetting)
  double* logdet;        // n_pad / 64 slots: log|det| of each pivot block
  int* err;              // error flags: [0] bit 0 zero pivot met, bit 1 a bounded wait gave up;
                         // [1] a multiplier of a given-order inversion exceeded tau
  int* order;            // n_pad: row order of the previous inversion of this matrix
                         // (position -> original row), kept by launch_gje_finish
};

struct GjeArgs {
  GjeMat m[2];
  int nmat;
  int n_pad;
  int nbo;               // outer block width for this step (multiple of 64)
  int k0;                // first column of the outer block
  int pcur;              // which P[] holds the current panel
  int c0;                // inner block offset inside the panel (multiple of 64)
  int r0;                // first candidate position (k0 + c0)
  int known;             // 1: pivot rows in the given order (m.order), no search
  double tau;            // known order: largest multiplier magnitude accepted
};

// Tournament scratch sizes (ints) per matrix.
inline int gje_cand_ints(int n_pad) { return 2 * (n_pad / 128 + 2) * 65; }
inline int gje_cnt_ints(int n_pad) { return 2 * (n_pad / 128 + 2); }

// Reset ptot to the identity (a.known: to m.order), zero the error flags, logdet
// slots and counters.
hipError_t launch_gje_begin(const GjeArgs& a, hipStream_t s);
// P[pcur] = Min[:, k0:k0+nbo]; pi = identity.  With a.known the first outer step
// (k0 = 0) gathers the rows in the given order instead: P[i] = Min[order[i]],
// pi = order.
hipError_t launch_gje_panel_copy(const GjeArgs& a, hipStream_t s);
hipError_t launch_gje_tournament(const GjeArgs& a, hipStream_t s);
// Inner step on the panel (P[pcur] -> P[pcur ^ 1]) with the tournament's pivot rows,
// or (a.known) with the pivot rows r0..r0+63 in order, whose factors are in tri slot
// c0 / 64 % 2; the launch then also factors the next block into the other slot.
// err[1] is raised when a multiplier exceeds a.tau or a pivot is zero.
hipError_t launch_gje_inner_update(const GjeArgs& a, hipStream_t s);
// Given order: the factors of the panel's first pivot block (rows k0..k0+63 of
// P[pcur]) into tri slot 0, with log|det| and the multiplier check.
hipError_t launch_gje_lu64(const GjeArgs& a, hipStream_t s);
// Outer update of the columns [c_lo, c_hi) (inside) or of all others (!inside);
// c_lo is a multiple of 128, the ranges are rounded out to whole 128-column tiles.
// max_wgs > 0 caps the workgroups per matrix (persistent tiles), leaving CUs to
// work that runs beside it.  A null m[z].pi reads Min without a gather.
// next_panel[z] (inside only): the columns [c_lo, c_lo + next_nbo) are written to
// that n_pad x next_nbo panel instead of Mout.
hipError_t launch_gje_outer_update(const GjeArgs& a, int c_lo, int c_hi, bool inside,
                                   int max_wgs, hipStream_t s, double* const* next_panel = nullptr,
                                   int next_nbo = 0);
// pinv = ptot^{-1}; order = ptot (the next inversion of the matrix may reuse it).
hipError_t launch_gje_finish(const GjeArgs& a, hipStream_t s);
// dst (n x n, ldd) = A^{-1}: dst[i][ptot[c]] = Mfinal[i][c].
hipError_t launch_gje_unpermute(const double* Mfinal, const int* pinv, int64_t ld, double* dst,
                                int64_t ldd, int n, hipStream_t s);

// ---------------------------------------------------- elementwise etc. ----
// Denman-Beavers update with the column permutation of the inverses folded in.
struct DbArgs {
  const double* Xin;      // X_k (may equal Xout: the update is row-local)
  double* Xout;           // X_{k+1}
  const double* Yin;      // Y_k (nullptr: Y_0 = I)
  double* Yout;           // Y_{k+1}
  const double* Xinv;     // permuted inverses (Gauss-Jordan output)
  const double* Yinv;
  const int* px;          // pinv of X's inversion
  const int* py;          // pinv of Y's inversion (nullptr: Y = I, inverse I)
  const double* ldx;      // logdet slots of X (nslots)
  const double* ldy;      // logdet slots of Y (nullptr: 0)
  int nslots;
  int n;                  // valid size
  int64_t ld;             // n_pad
  int scaled;
  double* part;           // partial column sums, 2 x nblk x n
  double* mu_out;         // device scalar: mu used
};
hipError_t launch_db_update(const DbArgs& a, int nblk, hipStream_t s);

// Reduce partial column sums part[q][b][c] (q < nq, b < nblk, c < n) to
// out[q] = max_c sum_b part[q][b][c]; bm is scratch of nq * ceil(n / 64) doubles.
hipError_t launch_colsum_max(const double* part, int nq, int nblk, int n, double* out,
                             double* bm, hipStream_t s);

// Padded workspace matrices: n_pad = ld, valid block n x n, the rest of an X-like
// matrix is the identity and of a B-like matrix zero.  The kernels below write the
// whole padded matrix and sum norms over the valid block.
// B = X - I; column-sum partials of |B| into part[0].
hipError_t launch_shift(const double* X, double* B, int n, int64_t ld, double* part, int nblk,
                        hipStream_t s);
// B2 = A2 - 2 X + I (valid block), column-sum partials of |B2| into part[0].
hipError_t launch_b2_from_root(const double* A2, const double* X, double* B2, int n, int64_t ld,
                               double* part, int nblk, hipStream_t s);
// Column-sum partials of |M| (valid n x n) into part[0].
hipError_t launch_abs_colsum(const double* M, int n, int64_t ld, double* part, int nblk,
                             hipStream_t s);

// Load an n x n user matrix into a padded n_pad x n_pad buffer; pad gets diag(padval).
hipError_t launch_load_padded(const double* src, int64_t lds, double* dst, int n, int n_pad,
                              double padval, int* nonfinite, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t count, hipStream_t s);

// y = M x (transposed = false) or y = M^T x (true); M is n x n row-major (ld).
hipError_t launch_gemv(const double* M, int64_t ld, int n, const double* x, double* y,
                       bool transposed, double* part, int nblk, hipStream_t s);

// Polynomial accumulator initialisation: out[t] = c2[t] * P2 + c3[t] * P3 + c1[t] * I
// on the valid n x n block, zero on the rest of the padded ld x ld matrix (at most
// 2 kKMax - 1 outputs: L_j, R_j for j = 2..kKMax and the output sum).
struct LincombArgs {
  static constexpr int kMax = 2 * kKMax - 1;
  const double* P2;
  const double* P3;
  int nout;
  double* out[kMax];
  double c1[kMax];
  double c2[kMax];
  double c3[kMax];
  int n;
  int64_t ld;
};
hipError_t launch_lincomb_init(const LincombArgs& a, hipStream_t s);

// out = beta out + sum_{t < m} c[t] in[t] over the valid n x n block (row stride ld);
// out may alias an input.
struct LincombGen {
  // the reverse mode's largest sum: the output adjoint and both factor adjoints of
  // every product of the largest scheme
  static constexpr int kMax = 2 * kKMax - 1;
  const double* in[kMax];
  double c[kMax];
  int m;
  double beta;
  double* out;
  int n;
  int64_t ld;
  // appends coef * p; false (nothing appended) when the operand list is full
  bool add(const double* p, double coef) {
    if (m >= kMax) return false;
    in[m] = p;
    c[m++] = coef;
    return true;
  }
};
hipError_t launch_lincomb_gen(const LincombGen& a, hipStream_t s);

// Balancing in place on the n x n block (row stride ld): M <- T^{-1} P^T M P T,
// d = diag(T) (n doubles, powers of two), perm (n ints, may be null: no permutation
// step) the original index at each position, cnt 2n ints of scratch (needed with
// perm), *sweeps = sweeps used (device int, may be null).
hipError_t launch_balance(double* M, int64_t ld, int n, double* d, int max_sweeps, int* sweeps,
                          int* perm, int* cnt, hipStream_t s);
// L = P T LB T^{-1} P^T (LB and L distinct).
hipError_t launch_unbalance_perm(const double* LB, int64_t ldb, double* L, int64_t ldl, int n,
                                 const double* d, const int* perm, hipStream_t s);

// P (2n x 2n) = [[Re A, -Im A], [Im A, Re A]] for complex A (interleaved, lda in
// complex elements); L (complex) = the left block column of R (2n x 2n).
hipError_t launch_embed_complex(const double* A, int64_t lda, int n, double* P, int64_t ldp,
                                hipStream_t s);
hipError_t launch_extract_complex(const double* R, int64_t ldr, int n, double* L, int64_t ldl,
                                  hipStream_t s);
// Complex batch through real representations (n_i <= n_lim): real sizes and offsets
// (2 n_i, 4 off_i; 0 for an invalid block), the embedding, and the extraction of the
// left block column; one workgroup per matrix for the latter two.
hipError_t launch_batch_complex_prep(int batch, int n_lim, int64_t total, const int* dims,
                                     const int64_t* off, int* dims2, int64_t* off2, hipStream_t s);
hipError_t launch_batch_embed_complex(int batch, const double* A, const int* dims2,
                                      const int64_t* off2, double* P, hipStream_t s);
hipError_t launch_batch_extract_complex(int batch, const double* R, const int* dims2,
                                        const int64_t* off2, double* L, hipStream_t s);

// Padded n_pad x n_pad test matrix I + 0.5 u / sqrt(n) (u hashed from seed), identity
// on the pad; for timing runs only.
hipError_t launch_fill_test_matrix(double* M, int n, int n_pad, unsigned seed, hipStream_t s);

// dst = scale * src^T for the n x n blocks (dst must not overlap src).
hipError_t launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd, int n,
                            double scale, hipStream_t s);

// flag |= 1 if the valid n x n block of M holds a NaN or Inf.
hipError_t launch_check_finite(const double* M, int64_t ld, int n, int* flag, hipStream_t s);

// dst (n x n, ldd) = scale * src (valid block of ld-matrix).
hipError_t launch_scale_out(const double* src, int64_t ld, double* dst, int64_t ldd, int n,
                            double scale, int* nonfinite, hipStream_t s);

// -------------------------------------------------------- fixed scratch --
// Largest n and the scratch bytes of logm_forward_noalloc (a logm of n <= 256 needs
// about 10 MB of workspace; the driver checks that its plan fits).
constexpr int kNoallocMaxN = 256;
constexpr size_t kNoallocBytes = (size_t)16 << 20;
// Device address of the current device's scratch array (looked up on the first call
// on each device, with that device current).
hipError_t noalloc_scratch(void** ptr);

// ---------------------------------------------------------------- batched --
// Workspace bytes of the batched path: 13 buffers of the size class's largest
// matrix per resident workgroup of the device, one region per class (n <= 64
// always, 64 < n <= 128 when n_max > 64; the classes run concurrently), plus two
// work-queue counters and the processing order (one int per matrix).
size_t batched_workspace_bytes(int batch, int n_max);
// Persistent launches over the batch (n_i <= 128): L_i = log(A_i) by Algorithm 1
// on the device, one workgroup per matrix from a work queue; a kernel that zeroes the
// queue counters and orders the matrices by decreasing n (largest first), then the
// large class (8 waves, n > split) on `s` beside the small class (4 waves,
// n <= split) on a second stream (forked and joined with events); split (1..64)
// applies when n_max > 64, otherwise every matrix is in the small class.  No host
// synchronisation and no memset, so the sequence can be captured in a graph.  h, g:
// [scheme k - 1 for k = 1..5][row j - 2][P_2..P_{j+1}], y: [scheme][P_1..P_{k+2}].
hipError_t launch_batched_logm(int batch, int n_max, const int* dims, const int64_t* offsets,
                               const double* A, double* L, int* status, void* ws, size_t ws_bytes,
                               int64_t total_elems, int k_max, int max_sqrt, int db_max_iter,
                               int theta_source, const double* coef, int split, hipStream_t s);

}  // namespace logm
