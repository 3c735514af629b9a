/*
 * rnnls.h -- C ABI of librnnls.so: RandomizedNNLS on AMD Instinct MI355X (gfx950).
 *
 * Method: C. Boutsidis and P. Drineas, "Random Projections for the Nonnegative
 * Least-Squares Problem".  Given A (n x d, n >> d) and b (n), Algorithm 1
 * (RandomizedNNLS) flips the sign of every row of [A | b] with a random +-1
 * diagonal D (step 4), applies the n x n Hadamard-Walsh matrix H_n of Section 2
 * (Sylvester recursion, normalised by 1/sqrt(n), rows zero-padded to the next
 * power of two n'), keeps each row with probability r/n' rescaled by
 * sqrt(n'/r) (steps 2-3), and solves the small nonnegative least-squares
 * problem of Definition 1 on the kept rows exactly (step 5).  The exact solver
 * here is Lawson-Hanson's active-set method (the paper's lsqnonneg), run in
 * the Gram form Q = A^T A, q = A^T b that Section 3.4 describes.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are column-major (LAPACK convention): column k of A starts at
 *    A + k*lda and holds n contiguous floats; lda >= n.
 *  - Every data pointer is DEVICE memory owned by the caller; the library never
 *    allocates, frees or keeps any of it.  Scratch memory comes from the
 *    caller's workspace `ws` of `ws_bytes` bytes (size it with
 *    rnnls_workspace_bytes; 256-byte alignment).  Results are undefined if
 *    inputs, outputs and the workspace overlap.
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = the default
 *    stream) and is asynchronous: the call returns once the kernels are
 *    launched.  Calls sharing a workspace must be ordered on one stream.
 *  - Row indices are 0-based (the paper's row i is row i-1 here).  H_n' is in
 *    natural (Sylvester) order: H[i][j] = (-1)^popcount(i & j).
 *  - Return value: RNNLS_OK, or -(1-based position of the first invalid
 *    argument) (LAPACK "info" style), or one of the RNNLS_E_* codes.  Argument
 *    checks happen on the host before anything is launched.  Outcomes that are
 *    only known on the device (solver status) are written to device memory.
 *
 * Random streams (the paper fixes only the probabilities; this definition is
 * the library's):
 *  mix64(z)      SplitMix64 output function (Steele, Lea & Flood 2014; shifts
 *                30, 27, 31; multipliers 0xBF58476D1CE4E5B9, 0x94D049BB133111EB)
 *  key(seed, s)  mix64(seed ^ (s * 0x9E3779B97F4A7C15))        (mod 2^64)
 *  h(seed, s, i) mix64(key(seed, s) + i)
 *  D_jj = -1 iff bit 63 of h(seed, 1, j) is set                (0 <= j < n')
 *  EXACT rows:     {pi(k) : 0 <= k < r} ascending; pi is the bijection of
 *                  [0, 2^m), m = log2 n', given by 4 rounds t = 0..3 of
 *                  x ^= ka_t; x = x * (kb_t | 1) mod 2^m; x ^= x >> ceil(m/2)
 *                  with ka_t = h(seed,3,2t) mod 2^m, kb_t = h(seed,3,2t+1) mod 2^m.
 *  BERNOULLI rows: {i : h(seed, 2, i) < r * 2^(64-m)} ascending (each row kept
 *                  with probability exactly r/n', Algorithm 1 step 2 as written).
 *  Both modes scale kept rows by sqrt(n'/r) * (1/sqrt(n')) = 1/sqrt(r).
 */
#ifndef RNNLS_H
#define RNNLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define RNNLS_OK 0
#define RNNLS_E_HIP (-100)          /* a HIP runtime call failed             */
#define RNNLS_E_WORKSPACE (-101)    /* ws NULL, misaligned or too small       */
#define RNNLS_E_UNSUPPORTED (-102)  /* valid but unsupported (see limits)     */

/* ---- per-problem solver status (device int32) --------------------------- */
#define RNNLS_SOLVE_OK 0            /* converged, KKT certificate holds       */
#define RNNLS_SOLVE_MAX_ITER 1      /* outer-iteration cap hit; x feasible    */
#define RNNLS_SOLVE_KKT_FAIL 2      /* finished but the KKT check failed      */
#define RNNLS_SOLVE_NO_ROWS 3       /* Bernoulli sample kept no row           */
#define RNNLS_SOLVE_OVERFLOW 4      /* Bernoulli sample exceeded r_cap rows   */
#define RNNLS_SOLVE_BAD_BOUNDS 5    /* box bounds: some lo not finite or hi < lo */

/* ---- options ----------------------------------------------------------- */
#define RNNLS_SAMPLE_EXACT 0        /* exactly r distinct rows (default)      */
#define RNNLS_SAMPLE_BERNOULLI 1    /* r~ ~ Bin(n', r/n') rows                */

#define RNNLS_PREC_FP32 0           /* FP32 transform                         */
#define RNNLS_PREC_SPLIT_BF16 1     /* split-BF16 matrix-core transform (below) */

/* Limits of this version: 1 <= d <= RNNLS_MAX_D (RNNLS_MAX_D_SOLVE for the
 * single-problem calls, below); 1 <= r < n'; r (or r_cap)
 * <= RNNLS_MAX_R; n' <= 2^30.
 *
 * RNNLS_PREC_SPLIT_BF16: the in-tile Hadamard transform runs two of its three
 * factors on BF16 matrix cores with every input split x = hi + lo
 * (hi = bf16(x), lo = bf16(x - hi)) and FP32 accumulation; the third factor,
 * the combine across tiles, moments and Lawson-Hanson are unchanged (FP32 /
 * FP64).  Each split loses about 2^-16 relatively, so sketch columns agree
 * with the exact transform to about 1e-4 norm-wise (FP32: about 1e-6).
 * Needs r_cap <= 16384 when n' >= 2^14 (else RNNLS_E_UNSUPPORTED, nothing
 * launched); problems with n' < 2^14 run the FP32 transform. */
#define RNNLS_MAX_D 128
#define RNNLS_MAX_R 32768
/* rnnls_srht_sketch, rnnls_nnls_solve, rnnls_rand_nnls (and its
 * allocation-free variant) take 1 <= d <= RNNLS_MAX_D_SOLVE: problems with
 * d > RNNLS_MAX_D are solved by a Lawson-Hanson kernel whose sweep tableau
 * (d x d FP64, upper triangle) lives in the workspace; batches, many
 * right-hand sides, repetition, box bounds and the learned proposal keep
 * d <= RNNLS_MAX_D. */
#define RNNLS_MAX_D_SOLVE 512

typedef struct rnnls_opts {
  int32_t sample_mode; /* RNNLS_SAMPLE_*                                      */
  int32_t precision;   /* RNNLS_PREC_*                                        */
  int32_t max_iter;    /* Lawson-Hanson outer-iteration cap; <= 0: 3*d        */
  int32_t r_cap;       /* Bernoulli: rows the sketch buffers hold; <= 0: the
                          default r + 8*ceil(sqrt(r)) + 64; either is clamped
                          to n' (a sample keeps at most n' rows) (EXACT:
                          ignored)                                            */
  double tol;          /* dual tolerance tau; <= 0: 10*eps*||M||_1*max(m,d),
                          ||M||_1 the largest column 1-norm (lsqnonneg's rule) */
} rnnls_opts;          /* NULL opts = all defaults                            */

/* Which entry point rnnls_workspace_bytes sizes. */
#define RNNLS_OP_SKETCH 0
#define RNNLS_OP_SOLVE 1
#define RNNLS_OP_RAND_NNLS 2

/* Library version (major*10000 + minor*100 + patch). */
int rnnls_version(void);

/* Number of gfx950 compute units the library schedules for on the current
 * device (cached per device), or a negative RNNLS_E_* code. */
int rnnls_device_cus(void);

/* Device workspace, in bytes, that entry point `op` needs for these sizes
 * (for RNNLS_OP_SOLVE, n is the row count m of the problem).  Returns 0 for
 * invalid sizes. */
size_t rnnls_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t r,
                             const rnnls_opts* opts);

/* rnnls_srht_sketch -- steps 1-4 of Algorithm 1.
 *
 *   [SA | Sb] = (1/sqrt r) * (H_n' D [A | b])[rows, :]
 *
 *  n, d        A is n x d (n >= 2, 1 <= d <= RNNLS_MAX_D_SOLVE)
 *  r           target row count, 1 <= r < n' (n' = 2^ceil(log2 n))
 *  seed        seed of the random streams (see above)
 *  A, lda      input, column-major, lda >= n
 *  b           input right-hand side of length n, or NULL (then Sb is unused)
 *  SA, ldsa    output, column-major R x d with ldsa >= R_cap where R_cap = r
 *              (EXACT) or the clamped opts->r_cap (BERNOULLI); rows beyond the kept
 *              count are left untouched
 *  Sb          output of length R_cap (ignored when b is NULL)
 *  rows        output int32[R_cap]: kept rows of H_n', ascending; may be NULL
 *  r_out       output int32[1]: number of kept rows; may be NULL
 *  sign_bits   output uint32[n'/32] (n' >= 32): bit (j % 32) of word j / 32 is
 *              set iff D_jj = -1; may be NULL
 *  status      output int32[1]: RNNLS_SOLVE_OK, or RNNLS_SOLVE_NO_ROWS /
 *              RNNLS_SOLVE_OVERFLOW in Bernoulli mode; may be NULL
 */
int rnnls_srht_sketch(int64_t n, int32_t d, int32_t r, uint64_t seed,
                      const float* A, int64_t lda, const float* b,
                      float* SA, int64_t ldsa, float* Sb,
                      int32_t* rows, int32_t* r_out, uint32_t* sign_bits,
                      int32_t* status, const rnnls_opts* opts,
                      void* ws, size_t ws_bytes, void* stream);

/* rnnls_nnls_solve -- Definition 1 solved exactly (Lawson-Hanson, LH74 ch. 23)
 * for a problem already on the device:  x = argmin_{x >= 0} ||M x - f||_2.
 *
 *  m, d        M is m x d (m >= 1, 1 <= d <= RNNLS_MAX_D_SOLVE)
 *  M, ldm      input, column-major, ldm >= m
 *  f           input right-hand side of length m
 *  m_dev       optional device int32[1] holding the row count actually used
 *              (<= m), e.g. r_out of a Bernoulli sketch; NULL = m
 *  x           output double[d] (x >= 0)
 *  w           output double[d]: dual vector M^T (f - M x); may be NULL
 *  rnorm       output double[1]: ||M x - f||_2; may be NULL
 *  iters       output int32[1]: outer iterations; may be NULL
 *  status      output int32[1]: RNNLS_SOLVE_*; may be NULL
 * The solve runs in FP64: the Gram matrix M^T M and M^T f are accumulated in
 * FP64 from the FP32 inputs (products are exact); the passive-set systems go
 * through a symmetric sweep tableau of [Q q] (one sweep when a column enters,
 * one reverse sweep when it leaves), and the returned w and the KKT status
 * are computed from Q itself.
 */
int rnnls_nnls_solve(int64_t m, int32_t d, const float* M, int64_t ldm,
                     const float* f, const int32_t* m_dev,
                     double* x, double* w, double* rnorm, int32_t* iters,
                     int32_t* status, const rnnls_opts* opts,
                     void* ws, size_t ws_bytes, void* stream);

/* rnnls_rand_nnls -- Algorithm 1 end to end: sketch (as rnnls_srht_sketch)
 * then the exact solve of the sketched problem (as rnnls_nnls_solve).
 *
 *  n, d, r, seed, A, lda, b   as rnnls_srht_sketch (b required)
 *  x           output double[d]: x~ of Algorithm 1 (x~ >= 0)
 *  rnorm       output double[1]: ||SA x~ - Sb||_2 (sketched residual); may be NULL
 *  iters, status  as rnnls_nnls_solve; may be NULL
 *  SA, ldsa, Sb, rows, r_out  optional copies of the sketch (as
 *              rnnls_srht_sketch); pass NULL to keep them in the workspace
 */
int rnnls_rand_nnls(int64_t n, int32_t d, int32_t r, uint64_t seed,
                    const float* A, int64_t lda, const float* b,
                    double* x, double* rnorm, int32_t* iters, int32_t* status,
                    float* SA, int64_t ldsa, float* Sb, int32_t* rows,
                    int32_t* r_out, const rnnls_opts* opts,
                    void* ws, size_t ws_bytes, void* stream);

/* ---- without a workspace ------------------------------------------------
 * rnnls_rand_nnls_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): rnnls_rand_nnls with the same arguments and results, minus
 * ws and ws_bytes.  Its scratch is a fixed array of
 * RNNLS_NOALLOC_SCRATCH_BYTES in the library's device memory, one per device,
 * held until the process ends; the call allocates nothing (no hipMalloc, no
 * library allocation) and frees nothing.
 *  - Sizes whose workspace (rnnls_workspace_bytes(RNNLS_OP_RAND_NNLS, ...))
 *    exceeds RNNLS_NOALLOC_SCRATCH_BYTES return RNNLS_E_WORKSPACE before
 *    anything is launched (2^20 x 64 at r = 4096 needs about 15 MB, 2^22 x 128
 *    at r = 8192 about 14 MB).  Invalid arguments return as rnnls_rand_nnls.
 *  - Every call on a device shares that device's array, which keeps the last
 *    call's contents; nothing in it has to start at zero.  Calls that
 *    overlap on one device (other streams, other host threads) race on it:
 *    order them on one stream.
 *  - The array's device address is read with hipGetSymbolAddress on the
 *    first call made with each device current (RNNLS_E_HIP if that fails).
 */
#define RNNLS_NOALLOC_SCRATCH_BYTES (64 << 20)

int rnnls_rand_nnls_noalloc(int64_t n, int32_t d, int32_t r, uint64_t seed,
                            const float* A, int64_t lda, const float* b,
                            double* x, double* rnorm, int32_t* iters, int32_t* status,
                            float* SA, int64_t ldsa, float* Sb, int32_t* rows,
                            int32_t* r_out, const rnnls_opts* opts, void* stream);

/* ---- box constraints on the same sketch ---------------------------------
 * rnnls_rand_box -- the conclusions remark that the sketch of Algorithm 1 does
 * not depend on the constraint set.  Steps 1-4 as rnnls_rand_nnls, then step 5
 * with box bounds: x~ = argmin_{lo <= x <= hi} ||H~ D A x - H~ D b||_2^2
 * (lo = 0, hi = +inf is Algorithm 1 itself).  The small problem is solved by a
 * bounded-variable active-set method (Stark and Parker's BVLS: Lawson-Hanson's
 * outer and inner loops with two bounds) in FP64 Gram form, one wavefront,
 * the free systems through a symmetric sweep tableau of G (one sweep when a
 * variable leaves its bound, one reverse sweep when it returns to one); the
 * closing certificate is computed from G itself.  Every variable starts
 * at its lower bound; the entering variable is the bound one whose dual most
 * violates its condition (lowest index on ties); tau, the dependence test and
 * the default cap of 3d outer steps are those of rnnls_nnls_solve.
 *
 *  n, d, r, seed, A, lda, b   as rnnls_rand_nnls, but 1 <= d <= RNNLS_MAX_BOX_D
 *  lo, hi      input device double[d]: bounds; every lo finite, hi >= lo, hi may
 *              be +inf (else status RNNLS_SOLVE_BAD_BOUNDS and x = 0)
 *  x           output double[d] in the box
 *  rnorm       output double[1]: ||H~ D (A x - b)||_2; may be NULL
 *  iters       output int32[1]: outer steps; may be NULL
 *  status      output int32[1]: RNNLS_SOLVE_OK, _MAX_ITER, _KKT_FAIL (optimality
 *              conditions w_j <= tau at a lower bound, -w_j <= tau at an upper
 *              one, |w_j| <= 1e3 tau when free, with the dual w = q - G x of
 *              G = (H~DA)^T H~DA, q = (H~DA)^T H~Db), _NO_ROWS, _OVERFLOW or
 *              _BAD_BOUNDS; may be NULL
 * All pointers are device memory owned by the caller; lo and hi are only read.
 * Workspace: rnnls_workspace_bytes(RNNLS_OP_RAND_NNLS, n, d, r, opts).  Returns
 * as rnnls_rand_nnls; -8 lo NULL, -9 hi NULL, -10 x NULL (argument positions).
 * The solve is timed as RNNLS_TIMER_SOLVE.
 */
#define RNNLS_MAX_BOX_D 64

int rnnls_rand_box(int64_t n, int32_t d, int32_t r, uint64_t seed, const float* A,
                   int64_t lda, const float* b, const double* lo, const double* hi,
                   double* x, double* rnorm, int32_t* iters, int32_t* status,
                   const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* ---- repetition ---------------------------------------------------------
 * rnnls_rand_nnls_boost -- Theorem 1's guarantee holds with probability at
 * least 1/2; its footnote notes that a few repetitions raise that.  Runs
 * Algorithm 1 k times (as rnnls_rand_nnls) with the random streams of seeds
 * seed, seed+1, ..., seed+k-1, then keeps the x~ whose full residual
 * ||A x~ - b||_2 is least (one FP64 pass over A for all k candidates), so the
 * (1+eps) bound holds with probability at least 1 - 2^-k.  Candidates whose
 * solve did not end with RNNLS_SOLVE_OK are passed over unless none did;
 * ties go to the lowest index.
 *
 *  n, d, r, seed, A, lda, b   as rnnls_rand_nnls
 *  k           repetitions, 1 <= k <= RNNLS_MAX_BOOST
 *  x           output double[d]: the kept x~
 *  resid       output double[k]: ||A x_i - b||_2 of every candidate; may be NULL
 *  best        output int32[1]: index i of the kept candidate (seed + i); may be NULL
 *  status      output int32[1]: the kept candidate's solve status; may be NULL
 * Workspace: rnnls_boost_workspace_bytes(n, d, r, k, opts).  Returns as
 * rnnls_rand_nnls (argument positions in this signature).
 */
#define RNNLS_MAX_BOOST 8

size_t rnnls_boost_workspace_bytes(int64_t n, int32_t d, int32_t r, int32_t k,
                                   const rnnls_opts* opts);
int rnnls_rand_nnls_boost(int64_t n, int32_t d, int32_t r, int32_t k, uint64_t seed,
                          const float* A, int64_t lda, const float* b, double* x,
                          double* resid, int32_t* best, int32_t* status,
                          const rnnls_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* ---- many right-hand sides sharing one A -------------------------------
 * rnnls_rand_nnls_multi -- Algorithm 1 for the k problems min ||A x_j - b_j||,
 * x_j >= 0, j < k, that share A (the extension Section 5 names, e.g. the
 * alternating updates of a nonnegative matrix factorisation).  One sketch
 * [SA | SB] = (1/sqrt r) (H_n' D [A | B])[rows, :] with the same D and rows
 * for all columns, one Gram matrix G = SA^T SA, then k Lawson-Hanson solves
 * sharing G.
 *
 *  n, d, r, seed, A, lda   as rnnls_rand_nnls
 *  k           right-hand sides, 1 <= k <= RNNLS_MAX_K
 *  B, ldb      input, column-major n x k, ldb >= n
 *  X, ldx      output, column-major d x k (FP64), ldx >= d
 *  rnorm       output double[k] (sketched residuals); may be NULL
 *  iters, status  output int32[k]; may be NULL
 * Workspace: rnnls_multi_workspace_bytes(n, d, k, r, opts).
 */
#define RNNLS_MAX_K 4096

size_t rnnls_multi_workspace_bytes(int64_t n, int32_t d, int32_t k, int32_t r,
                                   const rnnls_opts* opts);
int rnnls_rand_nnls_multi(int64_t n, int32_t d, int32_t k, int32_t r, uint64_t seed,
                          const float* A, int64_t lda, const float* B, int64_t ldb,
                          double* X, int64_t ldx, double* rnorm, int32_t* iters,
                          int32_t* status, const rnnls_opts* opts,
                          void* ws, size_t ws_bytes, void* stream);

/* ---- batches of independent problems ----------------------------------
 * A batch plan runs Algorithm 1 on `count` independent problems of different
 * sizes with a fixed number of fused launches (random streams, sketch per
 * tile-size group, reduce, moments, Lawson-Hanson), whatever the count.
 *
 * rnnls_problem: one problem; sizes and limits as rnnls_rand_nnls (A, b and x
 * required, rnorm, iters, status may be NULL).  All pointers are device
 * memory and must stay valid, with the same addresses, for the plan's life.
 *
 * rnnls_batch_workspace_bytes  workspace for rnnls_batch_create (covers every
 *              tile shape rnnls_batch_autotune tries); 0 for invalid input.
 * rnnls_batch_create  validates the problems (returns -3 if one is invalid;
 *              *bad_index, if not NULL, receives its index), plans the
 *              launches and binds `ws` (device, 256-byte aligned, caller
 *              owned, kept until destroy).  Allocates the plan's device-side
 *              descriptor tables (hipMalloc) and uploads them synchronously,
 *              and creates one stream and two events of its own.
 * rnnls_batch_run     enqueues one pass over all problems on `stream`; the
 *              solves of problems with d <= 64 run on the plan's own stream,
 *              forked from `stream` and joined back into it, beside those
 *              with d > 64 (so later work on `stream` sees every result).
 * rnnls_batch_autotune  times every candidate tile shape of the sketch on
 *              the plan's own problems (synchronising `stream`), keeps the
 *              fastest for this plan and reports it in *chosen (may be NULL).
 * rnnls_batch_capture records one pass into a HIP graph held by the plan
 *              (replaced by a later capture, dropped by autotune).
 * rnnls_batch_launch  replays the captured graph on `stream`
 *              (RNNLS_E_UNSUPPORTED if nothing was captured).
 * rnnls_batch_destroy waits for the device, frees the plan and its graph.
 * Calls on one plan must not overlap (they share the workspace).
 */
typedef struct rnnls_tuning {
  int32_t srht_log_tile;
  int32_t srht_wgs_per_cu;
} rnnls_tuning;

typedef struct rnnls_problem {
  int64_t n;
  int32_t d;
  int32_t r;
  uint64_t seed;
  const float* A;
  int64_t lda;
  const float* b;
  double* x;
  double* rnorm;
  int32_t* iters;
  int32_t* status;
} rnnls_problem;

typedef struct rnnls_batch rnnls_batch;

size_t rnnls_batch_workspace_bytes(int32_t count, const rnnls_problem* probs,
                                   const rnnls_opts* opts);
int rnnls_batch_create(rnnls_batch** plan, int32_t count, const rnnls_problem* probs,
                       const rnnls_opts* opts, void* ws, size_t ws_bytes,
                       int32_t* bad_index);
int rnnls_batch_run(rnnls_batch* plan, void* stream);
int rnnls_batch_autotune(rnnls_batch* plan, void* stream, rnnls_tuning* chosen);
int rnnls_batch_capture(rnnls_batch* plan);
int rnnls_batch_launch(rnnls_batch* plan, void* stream);
int rnnls_batch_destroy(rnnls_batch* plan);

/* ---- learned passive-set proposals --------------------------------------
 * A 3-layer perceptron maps per-column features of a sketched problem to the
 * probability that the column is passive (x_j > 0) at the optimum; the
 * proposal warm-starts Lawson-Hanson (the paper always starts from x = 0,
 * Section 4.1), whose KKT certificate judges the result: a rejected warm
 * start is replaced by a cold start from x = 0.
 *
 * Features of column j from the Gram form (G, q, c) of the sketched problem,
 * C_jk = G_jk / sqrt(G_jj G_kk) (0 for a zero column):
 *   f0 = q_j / sqrt(G_jj c); f1 = q_j / max|q|; f2 = (q_j - mean q) / std q;
 *   f3 = mean_{k!=j} C_jk; f4 = max_{k!=j} C_jk; f5 = mean_{k!=j} C_jk f0_k;
 *   f6 = log(G_jj / mean_k G_kk) clamped to [-30, 30]; f7 = d / 128.
 * Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), p = sigmoid(w3.h2 + b3)
 * with BF16 weights W1 (128x8), W2 (128x128), w3 (128), FP32 biases and FP32
 * accumulation.  FP32 master parameters theta[RNNLS_MLP_PARAMS] in the order
 * W1 (row-major), b1, W2 (row-major), b2, w3, b3; the BF16 copy
 * wb[RNNLS_MLP_BF16_WEIGHTS] holds W1, W2, w3 rounded to nearest even.
 * Training loss: mean binary cross-entropy with logits over the rows.
 */
#define RNNLS_MLP_FEATURES 8
#define RNNLS_MLP_WIDTH 128
#define RNNLS_MLP_PARAMS 17793
#define RNNLS_MLP_BF16_WEIGHTS 17536
#define RNNLS_MLP_MAX_ROWS (1 << 24)

/* Features of one problem from its device Gram form: G (d x d, row-major
 * FP64), q (d), c (1) -> X (d x 8 FP32, row-major). */
int rnnls_features(int32_t d, const double* G, const double* q, const double* c, float* X,
                   void* stream);
/* wb <- bf16(theta's weights). */
int rnnls_mlp_sync_bf16(const float* theta, uint16_t* wb, void* stream);
/* prob[i] = p(X[i]) (nullable), flags[i] = prob > threshold (nullable). */
int rnnls_mlp_forward(int64_t rows, const float* X, const float* theta, const uint16_t* wb,
                      float* prob, uint8_t* flags, float threshold, void* stream);
/* Workspace of rnnls_mlp_gradient / rnnls_mlp_train_step for `rows` rows. */
size_t rnnls_mlp_workspace_bytes(int64_t rows);
/* grad[RNNLS_MLP_PARAMS] = d loss / d theta (the BF16 weights are used in the
 * forward pass; their gradient is applied to the FP32 master copy); loss[1]
 * (nullable) = mean loss.  Deterministic (fixed-order reductions). */
int rnnls_mlp_gradient(int64_t rows, const float* X, const uint8_t* y, const float* theta,
                       const uint16_t* wb, float* grad, float* loss, void* ws,
                       size_t ws_bytes, void* stream);
/* One Adam step (bias-corrected, step >= 1) on theta, refreshing wb. */
int rnnls_mlp_adam(float* theta, uint16_t* wb, const float* grad, float* m, float* v,
                   int32_t step, float lr, float beta1, float beta2, float eps, void* stream);
/* Gradient + Adam (beta 0.9 / 0.999, eps 1e-8) on one mini-batch. */
int rnnls_mlp_train_step(int64_t rows, const float* X, const uint8_t* y, float* theta,
                         uint16_t* wb, float* m, float* v, int32_t step, float lr, float* loss,
                         void* ws, size_t ws_bytes, void* stream);

/* Batch plans and the learned proposal:
 * rnnls_batch_columns    total columns (sum of d) of the plan's problems
 * rnnls_batch_features   X (columns x 8, problems in order) of the last pass
 *                        and, if passive != NULL, its solutions' flags x_j > 0
 * rnnls_batch_set_model  theta/wb (device, kept by the caller; wb 4-byte
 *                        aligned, else -3) warm-start every later pass from
 *                        the proposal prob > threshold; NULL theta turns the
 *                        warm start off.  Each Lawson-Hanson workgroup computes
 *                        its problem's features and runs the perceptron
 *                        itself (no separate launches) before solving.
 * rnnls_batch_warm_used  int32[count]: 1 where the last pass kept the warm start
 * rnnls_batch_proposal   uint8[columns]: the last warm-started pass's proposal
 *                        (1 = proposed passive), problems in order
 */
int rnnls_batch_columns(const rnnls_batch* plan, int64_t* columns);
int rnnls_batch_features(rnnls_batch* plan, float* X, uint8_t* passive, void* stream);
int rnnls_batch_set_model(rnnls_batch* plan, const float* theta, const uint16_t* wb,
                          float threshold);
int rnnls_batch_warm_used(rnnls_batch* plan, int32_t* out, void* stream);
int rnnls_batch_proposal(rnnls_batch* plan, uint8_t* out, void* stream);

/* ---- launch tuning ------------------------------------------------------
 * Process-wide launch shape of the sketch kernel (all fields 0 = automatic:
 * 2^13-row tiles with three workgroups per CU when r_cap <= 4096 and fewer than
 * 16 tiles fall on each workgroup, 2^14-row tiles with two when more, else
 * 2^15-row tiles with one; tiles are widened when r_cap needs more than 32 kept rows
 * per thread).
 *  srht_log_tile   log2 of the rows one workgroup transforms at a time:
 *                  12..15 (capped at log2 n'); workgroups have 2^(tile-5) threads
 *  srht_wgs_per_cu persistent workgroups per compute unit, 1..16
 * Returns RNNLS_OK or -(1-based field number) for an invalid field; NULL
 * restores the automatic choice.  Not synchronised with calls in flight on
 * other host threads. */

int rnnls_set_tuning(const rnnls_tuning* tuning);
int rnnls_get_tuning(rnnls_tuning* tuning);

/* ---- the autotuner's cache -----------------------------------------------
 * rnnls_batch_autotune keeps each plan's choice in a process-wide table keyed
 * by the plan's shapes (the device's CU count, the sampling mode and every
 * problem's n', d and row capacity); a later plan with the same key takes the
 * stored choice without timing anything.
 * rnnls_tuning_cache_entries  number of entries
 * rnnls_tuning_cache_clear    empties the table
 * rnnls_tuning_cache_save     writes the table to a text file, one entry per
 *                             line: key (16 hex digits), log2 tile rows,
 *                             workgroups per CU
 * rnnls_tuning_cache_load     merges such a file into the table; a malformed
 *                             file merges nothing
 * save/load return RNNLS_OK, -1 for a NULL path, RNNLS_E_UNSUPPORTED when the
 * file cannot be opened, written or parsed.  Thread-safe (one mutex). */
int rnnls_tuning_cache_entries(void);
int rnnls_tuning_cache_clear(void);
int rnnls_tuning_cache_save(const char* path);
int rnnls_tuning_cache_load(const char* path);

/* ---- kernel timing ------------------------------------------------------
 * Off by default.  When on, the library brackets every launch of the timed
 * kernels with two HIP events recorded on the launch stream (no extra
 * synchronisation).  rnnls_timing_read waits for the recorded events, returns
 * the summed elapsed milliseconds and the launch count since the previous read
 * of that timer, and forgets them.  Host-side bookkeeping is mutex-protected;
 * a timer's begin/end pairs must not interleave across host threads. */
#define RNNLS_TIMER_SKETCH 0   /* the sketch transform kernel (steps 1-4)      */
#define RNNLS_TIMER_MOMENTS 1  /* Gram-form moments of the small problem       */
#define RNNLS_TIMER_SOLVE 2    /* Lawson-Hanson kernel (or the box solver)     */
#define RNNLS_TIMER_STREAM_READ 3  /* the streaming-read reference kernel      */
#define RNNLS_TIMER_RESIDUAL 4 /* full residuals of the repetition candidates  */
#define RNNLS_TIMER_STREAMS 5  /* random streams: sign words and kept rows     */
#define RNNLS_TIMER_REDUCE 6   /* fixed-order sum of the sketch partials and the
                                  1/sqrt(r) scale (steps 1-4 are STREAMS +
                                  SKETCH + REDUCE)                             */
#define RNNLS_TIMER_COUNT 7

int rnnls_timing_enable(int on);
int rnnls_timing_read(int32_t which, double* total_ms, int64_t* launches);

/* ---- streaming-read reference -------------------------------------------
 * Not a step of the method: the sketch reads A once, so the fastest plain
 * read of a buffer on the same device is its practical bandwidth ceiling, and
 * its fraction of HBM peak is also stated against this measured rate.
 * rnnls_stream_read reads x[0..n) (device, FP32, 16-byte aligned, n >= 0)
 * once with 16-byte loads on a persistent grid of rnnls_stream_read_blocks()
 * workgroups and writes partials[w] = the sum of the elements workgroup w
 * read (device, caller-owned, that many floats; their total is sum(x) up to
 * FP32 rounding).  Asynchronous on `stream`; timed as RNNLS_TIMER_STREAM_READ.
 * Returns RNNLS_OK, -1 for an invalid argument (NULL, negative n, misaligned
 * x) or RNNLS_E_HIP. */
int rnnls_stream_read_blocks(void);
int rnnls_stream_read(const float* x, int64_t n, float* partials, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RNNLS_H */
