/*
 * logm.h - C ABI of the MI355X (gfx950) matrix-logarithm library.
 *
 * The library computes the principal logarithm log(A) of an n x n matrix with no
 * eigenvalues on the closed negative real axis by the inverse scaling and squaring
 * algorithm of Jarlebring, Sastre and Ibanez, "Polynomial approximations for the
 * matrix logarithm with computation graphs" (arXiv 2401.10089), Algorithm 1 of
 * Section 6:
 *   - square roots by the scaled Denman-Beavers iteration (eq. ScalDB),
 *   - the number of roots s and the scheme k chosen from the backward-error bound
 *     of Section 5 (eqs. Eb, theta_Eb, Table 2) with 1-norm estimates
 *     (eqs. alphaapprox, AI2, normAm9, alpha2term1, normAm9plus1 and the
 *     degree-selection procedure after Algorithm 1),
 *   - log(I+B) ~ -S(-B) (eqs. Taylor_log, logipASTM) evaluated as the
 *     degree-optimal computation graph of eq. five_mult_degopt (schemes with
 *     k = 1 to 9 matrix products; k = 5 uses Table 1, k = 4, 6, 7, 8, 9 fits of
 *     the same form with b_i = 1/i for i <= 14, 20, 24, 27, 28, since Table 2 gives
 *     their orders and Theta but no coefficients),
 *   - the squaring phase L = 2^s L.
 * Balancing (the pre- and post-processing steps of Algorithm 1) is optional
 * (logm_opts.balance, forward entry points only) and off by default.
 *
 * Conventions (all entry points):
 *   - Matrices are row-major with a leading dimension ld >= n (elements between
 *     rows are neither read nor written).  Every norm is the 1-norm of the matrix
 *     as stored (largest column sum).
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *     device work is enqueued on it.  Calls that take data-dependent decisions
 *     synchronise the stream and return when their outputs are complete.
 *   - Workspace: `ws` is caller-owned device memory of at least the size reported
 *     by the matching *_workspace_size call, aligned to 256 bytes.  If ws is NULL
 *     the library allocates the workspace on `stream` and frees it before
 *     returning.  The library keeps no pointer to caller memory after a call.
 *   - Return value: a LOGM_* status code; outputs are unspecified on error.
 *     Argument checks happen before any device work.  Concurrent calls on
 *     different streams must use different workspaces.
 */
#ifndef LOGM_H
#define LOGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LOGM_OK = 0,
  LOGM_EINVAL = 1,      /* bad argument: n < 1, NULL pointer, ld < n, bad option */
  LOGM_ENOTSUP = 2,     /* reserved: not returned (entry points with a dtype take both types) */
  LOGM_EWORKSPACE = 3,  /* ws_bytes smaller than required */
  LOGM_ENONFINITE = 4,  /* NaN or Inf in the input or the result */
  LOGM_ESINGULAR = 5,   /* exact zero pivot: singular matrix, log undefined */
  LOGM_ENOCONV = 6,     /* square roots did not converge (eigenvalue on or near R^-) */
  LOGM_EHIP = 7         /* HIP runtime error; the hipError_t is in info->status_detail */
};

typedef enum { LOGM_R64 = 0, LOGM_C128 = 1 } logm_dtype;

/* Options of Algorithm 1 (Section 6). */
typedef struct logm_opts {
  int32_t k_max;        /* largest scheme (matrix products) allowed: 1 to 9 (default 9) */
  int32_t max_sqrt;     /* maximum number of square roots, "maxiter" (default 50, at most 64) */
  int32_t db_max_iter;  /* maximum Denman-Beavers iterations per root (default 30) */
  int32_t theta_source; /* 0: Theta values of Table 2 as printed (default), except
                           k = 7, 8, 9, whose fits' own Theta (0.5284, 0.5739,
                           0.6371) are below the printed ones and replace them;
                           1: also Theta_5 = 0.2448 recomputed from Table 1 and
                           Theta_6 = 0.4258 recomputed for the six-product fit
                           (above the printed 0.372) */
  int32_t graph_fp32;   /* 0: graph products in fp64 (default); 1: the k - 1 products of
                           eq. five_mult_degopt on the fp32 matrix cores (operands rounded
                           to fp32, fp32 accumulation); the linear combinations, the
                           output sum and 2^s stay fp64, as do the square roots, the
                           inverses and the norm estimates.  Result error about u_32 ||B||
                           relative instead of u_64. */
  int32_t balance;      /* 0: no preprocessing (default); 1: steps 1 and 14 of
                           Algorithm 1, run on B = T^{-1} P^T A P T and return
                           P T log(B) T^{-1} P^T, P the permutation isolating
                           eigenvalues of a reducible A and T the power-of-two
                           diagonal of Parlett-Reinsch balancing (the paper calls
                           MATLAB's balance; see logm_balance_f64).  logm_forward
                           only: logm_backward differentiates the unbalanced map (the
                           same function) and logm_batched_f64 rejects it. */
  int32_t pivot_search; /* 0 (default): for n above 256, an inversion of the
                           square-root iteration may take the row order of the previous
                           inversion of the same iterate (X or Y) instead of searching
                           for pivots; the result is kept only if every elimination
                           multiplier is at most 4 in magnitude, otherwise the inversion
                           is redone with the search.  The reverse mode (taped forward and
                           its replays) reuses orders only within one square root, and
                           a backward call must use the taped forward's setting;
                           1: pivot search (tournament) for every inversion */
  int32_t reserved;     /* must be zero */
} logm_opts;

/* Decisions and counters of one call (host memory). */
typedef struct logm_info {
  int32_t s;             /* number of square roots taken */
  int32_t k;             /* scheme used (matrix products of the polynomial) */
  int32_t m;             /* its Taylor order m_k (Table 2) */
  int32_t n_inv;         /* matrix inverses computed (sum over roots of 2*iters - 1) */
  int32_t n_gemm;        /* matrix products (B^2 at s = 0 plus k - 1 graph products) */
  int32_t n_matvec;      /* matrix-vector products of the 1-norm estimator */
  int32_t n_est;         /* 1-norm estimates */
  int32_t db_iters[64];  /* Denman-Beavers iterations of each root */
  double flops;          /* algorithmic flops: 2n^3 (n_inv + n_gemm) + 2n^2 n_matvec */
  double norm1_b;        /* ||A^{1/2^s} - I||_1 */
  double norm1_b2;       /* ||(A^{1/2^s} - I)^2||_1 (saved-product form, eq. AI2) */
  int32_t status_detail; /* hipError_t when LOGM_EHIP */
  int32_t n_inv_reordered; /* inverses computed in a previous inversion's row order */
  int32_t n_order_rejected; /* such attempts rejected by the multiplier check (and redone
                               with the pivot search; not counted in n_inv twice) */
} logm_info;

/* Fill *o with the defaults listed above. */
void logm_default_opts(logm_opts* o);

/* Human-readable name of a status code (static string). */
const char* logm_strerror(int code);

/* Workspace bytes for logm_forward on an n x n matrix of the given dtype (for
 * LOGM_R64 also sufficient for every component entry point below with the same n).
 * Returns LOGM_EINVAL for n < 1. */
int logm_workspace_size(int32_t dtype, int64_t n, const logm_opts* o, size_t* bytes);

/* L = log(A) (Algorithm 1).  A (device, n x n, lda) is not modified; L (device,
 * n x n, ldl) must not overlap A.  o may be NULL (defaults); info (host) may be
 * NULL.  LOGM_C128: A and L interleaved (re, im) like torch.complex128, lda and ldl
 * in complex elements; the method runs on the real representation
 * P = [[Re A, -Im A], [Im A, Re A]] (2n x 2n), whose logarithm is the representation
 * of log A, so info describes that 2n x 2n run (decisions, counts, real flops). */
int logm_forward(int32_t dtype, int64_t n, const void* A, int64_t lda, void* L, int64_t ldl,
                 const logm_opts* o, logm_info* info, void* ws, size_t ws_bytes, void* stream);

/* L = log(A) like logm_forward for a real n x n matrix with 1 <= n <= 256, with no
 * workspace argument and no device memory allocation: for callers that cannot
 * allocate (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc).  The workspace is a fixed 16 MiB device array inside the library, one
 * per device, held until the process ends; every call on a device shares it, so
 * calls that overlap on one device race (issue them on one stream, or serialise
 * them).  A, L, o, info and stream as for logm_forward (dtype LOGM_R64); n > 256
 * gives LOGM_EINVAL.  Synchronises `stream` like logm_forward. */
int logm_forward_noalloc(int64_t n, const double* A, int64_t lda, double* L, int64_t ldl,
                         const logm_opts* o, logm_info* info, void* stream);

/* ---- reverse mode ---- */

/* Minimum workspace bytes for logm_backward: the forward workspace plus
 * (o->max_sqrt + 2 * o->db_max_iter + 46) padded n x n matrices (checkpointed root
 * inputs, the graph factors and adjoints, and a ring of taped inverses that holds
 * one root).  Any workspace beyond the minimum lengthens the ring by one inverse per
 * n_pad * n_pad * 8 bytes (n_pad = n rounded up to a multiple of 64, rounded up to
 * 256 bytes): a root whose inverses from the forward pass are still in the ring is
 * not replayed, so with room for all of them (info->n_inv) the call costs one
 * forward pass plus the adjoint products. */
int logm_backward_workspace_size(int32_t dtype, int64_t n, const logm_opts* o, size_t* bytes);

/* gradA = d<G, log A>_F / dA, for real A the adjoint Frechet derivative
 * L_log(A^T, G), by reverse-mode differentiation of Algorithm 1 (Section 6)
 * through the graph polynomial of eq. five_mult_degopt (a composition of sums and
 * products, Section 3) and through the scaled Denman-Beavers iterates of eq.
 * ScalDB.  The decisions (s, k, iterations per root) are those of the forward pass
 * run inside this call, and each scaling factor mu is a constant of the map (the
 * iteration reaches the same root for any positive mu sequence).  A, G (n x n,
 * row-major, lda, ldg >= n) are read; gradA (ldga >= n) must not overlap A or G.
 * The computation is FP64 whatever o->graph_fp32 says; info (host, may be NULL)
 * receives the forward decisions and the flops of the whole call.  Synchronises
 * `stream` at the decisions like logm_forward.  LOGM_C128 (interleaved, ld in complex
 * elements): gradA = L_log(A^H, G), the adjoint for the inner product Re tr(X^H Y)
 * (the gradient convention of holomorphic functions), computed by the real reverse
 * mode on the 2n x 2n representation, whose transpose is the representation of A^H;
 * logm_backward_workspace_size takes the dtype into account. */
int logm_backward(int32_t dtype, int64_t n, const void* A, int64_t lda, const void* G, int64_t ldg,
                  void* gradA, int64_t ldga, const logm_opts* o, logm_info* info, void* ws,
                  size_t ws_bytes, void* stream);

/* The same reverse mode split in two calls, for callers that run the forward first
 * (autograd): logm_forward_taped computes L = log A like logm_forward and leaves in
 * ws (logm_backward_workspace_size bytes or more, required) the root checkpoints, the
 * taped inverses and a record of the decisions; logm_backward_taped then computes
 * gradA = d<G, log A>/dA from that tape without running the forward again.  Between
 * the two calls ws must not be touched, and n, the options and ws_bytes must be the
 * same; otherwise logm_backward_taped returns LOGM_EINVAL.  The tape stays valid, so
 * several G may follow one forward.  info of logm_backward_taped: the forward's
 * decisions, and the counters and flops of this call only.  o->balance must be 0.
 * LOGM_C128 runs both halves on the real representation with logm_backward's layout
 * (same workspace size query) and returns gradA = L_log(A^H, G). */
int logm_forward_taped(int32_t dtype, int64_t n, const void* A, int64_t lda, void* L, int64_t ldl,
                       const logm_opts* o, logm_info* info, void* ws, size_t ws_bytes,
                       void* stream);
int logm_backward_taped(int32_t dtype, int64_t n, const void* G, int64_t ldg, void* gradA,
                        int64_t ldga, const logm_opts* o, logm_info* info, void* ws,
                        size_t ws_bytes, void* stream);

/* ---- batched path: many small matrices in one launch ---- */

/* Workspace bytes for logm_batched_f64 over `batch` matrices of size n_i <= n_max
 * <= 128: 13 buffers of 64 x 64 doubles per resident workgroup of the n <= 64 class,
 * plus (n_max > 64) 13 buffers of 128 x 128 doubles per resident workgroup of the
 * 64 < n <= 128 class (the classes run concurrently), plus 256 bytes of queue
 * counters and one int per matrix for the processing order (largest matrices
 * first); the buffers do not grow with the batch beyond the device's resident
 * workgroups.  total_elems is validated only. */
int logm_batched_workspace_size(int32_t batch, int64_t total_elems, int32_t n_max, size_t* bytes);

/* L_i = log(A_i), i < batch, by Algorithm 1 with every decision (roots, estimates,
 * eq. alpha2term1 / normAm9plus1 finish test, degree selection) taken on the device:
 * one persistent launch, one workgroup per matrix from a device work queue.
 * dims (device int32[batch]): n_i, 1 <= n_i <= n_max <= 128.  offsets (device
 * int64[batch]): element offset of matrix i in A and L, both packed row-major with
 * ld = n_i; the blocks must not overlap and sum to total_elems.  status (device
 * int32[4 * batch]): per matrix {LOGM_* code, s, k, iterations}, where iterations
 * packs the Denman-Beavers iteration count of root r < 6 into bits 5r..5r+4
 * (saturating at 31).  A matrix that fails gets its code and leaves L_i undefined;
 * the other matrices are unaffected; a block with n_i outside [1, n_max] or reaching
 * outside [0, total_elems) gets LOGM_EINVAL and is not read or written.
 * ws (device, required, logm_batched_workspace_size bytes, queried on the device
 * the call runs on).  Only o->graph_fp32 = 0.
 * Enqueues work on `stream` and returns without synchronising (capturable into a
 * HIP graph); argument errors are returned before any device work. */
int logm_batched_f64(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                     const int64_t* offsets, const double* A, double* L, const logm_opts* o,
                     int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Launch-shape autotuner of the batched path.  When a batch holds matrices above 64,
 * both kernels run: the 4-wave kernel takes n_i <= split and the 8-wave kernel the
 * rest (split = 64 by default).  logm_batched_autotune runs logm_batched_f64 on the
 * caller's batch (same arguments; L and status are overwritten) with split in
 * {64, 56, 48, 40, 32}, one warm-up and one timed run each (HIP events on `stream`),
 * keeps the fastest for later batched calls on the current device (process-wide,
 * complex batches included) and returns it in *best_split (host) with its time in
 * *best_ms (host, may be NULL).  With n_max <= 64 only 64 is timed.  Synchronises
 * `stream`; not capturable.  logm_batched_set_split sets the boundary directly
 * (1..64) and returns the previous one, or -1 for an out-of-range value. */
int logm_batched_autotune(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                          const int64_t* offsets, const double* A, double* L, const logm_opts* o,
                          int32_t* status, void* ws, size_t ws_bytes, void* stream,
                          int32_t* best_split, double* best_ms);
int32_t logm_batched_set_split(int32_t split);

/* Workspace bytes for logm_batched_c128 over `batch` complex matrices of size
 * n_i <= n_max <= 64 whose packed blocks span total_elems complex elements: the real
 * batched path's workspace at size 2 n_max, two real buffers of 4 total_elems
 * doubles (the real representations of A and L) and the real sizes and offsets. */
int logm_batched_c128_workspace_size(int32_t batch, int64_t total_elems, int32_t n_max,
                                     size_t* bytes);

/* Complex batch (LOGM_C128 matrices, interleaved (re, im) like torch.complex128):
 * L_i = log(A_i) through the real representation P_i = [[Re A_i, -Im A_i],
 * [Im A_i, Re A_i]] (2 n_i x 2 n_i), as logm_forward does for one complex matrix:
 * the embedding, logm_batched_f64's persistent launch on the P_i and the extraction
 * of the left block column of log P_i, all on `stream`, no host synchronisation
 * (capturable).  dims, offsets, total_elems as for logm_batched_f64 with complex
 * elements, 1 <= n_i <= n_max <= 64 (P_i must fit the batched path's 128).  status
 * as for logm_batched_f64, with the decisions (s, k, iterations) of P_i; a block
 * with n_i outside [1, n_max] or reaching outside [0, total_elems) gets
 * LOGM_EINVAL and is not read or written.  ws (device, required,
 * logm_batched_c128_workspace_size bytes).  Only o->graph_fp32 = 0, o->balance = 0. */
int logm_batched_c128(int32_t batch, int32_t n_max, int64_t total_elems, const int32_t* dims,
                      const int64_t* offsets, const void* A, void* L, const logm_opts* o,
                      int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* ---- components of the path (fp64, device pointers), used for step-level checks ---- */

/* C = alpha * A * B + beta * C (m x k times k x n) on the fp64 matrix cores. */
int logm_gemm_f64(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* stream);

/* Ainv = A^{-1} by blocked Gauss-Jordan elimination with tournament pivoting (the
 * left division of eq. ScalDB); *logabsdet (host) = log|det A|.  A may equal Ainv
 * only if lda == ldi. */
int logm_inverse_f64(int64_t n, const double* A, int64_t lda, double* Ainv, int64_t ldi,
                     double* logabsdet, void* ws, size_t ws_bytes, void* stream);

/* X = A^{1/2} by the scaled Denman-Beavers iteration (eq. ScalDB) with the stopping
 * rule of the library (rel <= sqrt(n) u, or stagnation below 1e-6 once scaling is
 * off; scaling stops once rel < 1e-2).  *iters (host) = iterations used. */
int logm_sqrt_f64(int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                  int32_t db_max_iter, int32_t* iters, void* ws, size_t ws_bytes, void* stream);

/* L = -2^s S_k(-B) with P_3 = B2 = B*B supplied (eq. five_mult_degopt with the
 * saved product of eq. AI2); 1 <= k <= 9, 0 <= s <= 64. */
int logm_poly_f64(int64_t n, int32_t k, int32_t s, const double* B, int64_t ldb, const double* B2,
                  int64_t ldb2, double* L, int64_t ldl, void* ws, size_t ws_bytes, void* stream);

/* *est (host) = estimate of ||B2^q B^r||_1 (r in {0, 1}, q >= 1) by the
 * deterministic Hager-Higham 1-norm estimator; *nmatvec (host) = products used. */
int logm_normest_f64(int64_t n, const double* B2, int64_t ldb2, const double* B, int64_t ldb,
                     int32_t q, int32_t r, double* est, int32_t* nmatvec, void* ws,
                     size_t ws_bytes, void* stream);

/* B = T^{-1} P^T A P T (n x n, row-major, lda, ldb >= n; B may equal A when
 * lda == ldb): the balancing of steps 1 and 14 of Algorithm 1.  With perm (device, n
 * ints) not NULL, first the permutation step isolating eigenvalues of reducible
 * matrices (indices whose row, then column, has no nonzero off the diagonal in the
 * active range go to the bottom, then the top); perm[i] receives the index of A at
 * position i, (P^T A P)[i][j] = A[perm[i]][perm[j]].  NULL skips that step (P = I).
 * Then T = diag(d) of powers of two over the active range (Gauss-Seidel sweeps of the
 * Parlett-Reinsch rule with 2-norms, at most 100).  d (device, n doubles) receives
 * T's diagonal, *sweeps (host, may be NULL) the sweeps used.  Every update is an
 * exchange or an exact scaling, so B is exactly the similarity. */
int logm_balance_f64(int64_t n, const double* A, int64_t lda, double* B, int64_t ldb, double* d,
                     int32_t* perm, int32_t* sweeps, void* ws, size_t ws_bytes, void* stream);

/* Launch-shape autotuner: for matrices padded like n, times the inversion of two
 * synthetic n x n matrices (the shape of a Denman-Beavers iteration) with each
 * candidate cap on the workgroups of the trailing-update GEMM that runs beside the
 * panel factorization, once with the pivot search (caps 96 .. 256) and once in the
 * row order the search left (caps 224 .. 512: that panel chain is shorter, so the
 * GEMM may take more of the device), and keeps the fastest of each for all later
 * calls of this process with that padded size (the compile-time defaults,
 * overridable by LOGM_LOOKAHEAD_WGS and LOGM_LOOKAHEAD_WGS_REORDERED at build time,
 * apply until then).  best_wgs (host, 2 entries) receives the caps [search, given
 * order], best_ms (host, 2 entries, may be NULL) the time of one inversion pair in
 * each mode.  ws as for logm_forward with the same n (NULL: allocated and freed).
 * Synchronises `stream`. */
int logm_autotune(int64_t n, void* ws, size_t ws_bytes, void* stream, int32_t* best_wgs,
                  double* best_ms);

/* Host-side tables: the coefficients of scheme k (h and g rows j = 2..k on
 * P_2..P_{j+1}, concatenated; y on P_1..P_{k+2}), its order m_k and Theta_{m_k}.
 * Any output pointer may be NULL.  *nh receives the number of h (= g) values
 * (k (k + 1) / 2 - 1, at most 44); y receives k + 2 values. */
int logm_scheme(int32_t k, int32_t theta_source, double* h, double* g, double* y, int32_t* nh,
                int32_t* m, double* theta);

/* Kernel timing for performance reports.  When enabled, the library brackets every
 * launch of the Gauss-Jordan trailing-update kernel (the dominant kernel) with HIP
 * events on the stream it runs on and accumulates, at its own synchronisation
 * points, the launch count, total device milliseconds and the algorithmic flops and
 * HBM bytes of those launches.  Process-wide; not thread-safe. */
void logm_profile_enable(int32_t on);
void logm_profile_reset(void);
int logm_profile_get(int64_t* launches, double* ms_total, double* flops_total, double* bytes_total);

/* Library version string. */
const char* logm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LOGM_H */
