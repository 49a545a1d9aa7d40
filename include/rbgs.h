/*
 * rbgs.h -- C ABI of the MI355X (gfx950) randomized block Gram-Schmidt library.
 *
 * The library computes the RBGS QR factorization W = Q R of a tall matrix W
 * (n x m, m <= k << n) with respect to the sketched inner product
 * <Theta x, Theta y>, where Theta (k x n) is a random sketching operator
 * regenerated on the fly from a counter-based generator and never stored.
 * Reference: O. Balabanov and L. Grigori, "Randomized block Gram-Schmidt
 * process for the solution of linear systems and eigenvalue problems",
 * arXiv 2111.14641: Section 2 (Algorithm "RBGS"), Section 2.1 (least-squares
 * step), Section 2.2 (inter-block QR: RCholeskyQR and RCholeskyQR with
 * postponed sketching), Section 3 (certificates Delta and Delta~).
 *
 * Conventions for every call below:
 *  - Matrices are column-major.  "Device" pointers are HIP device memory
 *    (e.g. allocated by PyTorch); "host" pointers are ordinary host memory.
 *  - The caller owns every array it passes.  A handle owns only its internal
 *    workspace, which grows on demand, is reused between calls and is freed by
 *    rbgs_destroy.
 *  - Work is enqueued on the stream given in the options (NULL = the null
 *    stream) and the call returns without waiting, unless stated otherwise.
 *  - Argument errors are detected on the host before anything is enqueued and
 *    are reported as RBGS_EINVAL / RBGS_EUNSUPPORTED; nothing is written then.
 *  - No call throws.  A handle must not be used by two threads at once.
 *  - Results are bitwise reproducible for identical inputs, options and device:
 *    every reduction runs in a fixed order and no floating-point atomics are
 *    used.
 */
#ifndef RBGS_H
#define RBGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported entry points (the library is built with hidden default visibility). */
#ifndef RBGS_API
#define RBGS_API __attribute__((visibility("default")))
#endif

typedef struct rbgs_handle_s* rbgs_handle;

typedef enum {
  RBGS_OK = 0,
  RBGS_EINVAL = -1,        /* invalid argument (checked on the host)              */
  RBGS_ENOMEM = -2,        /* device workspace allocation failed                 */
  RBGS_EDEVICE = -3,       /* a HIP runtime call failed (see rbgs_last_error)    */
  RBGS_EBREAKDOWN = -4,    /* a diagonal entry of R is zero or not finite        */
  RBGS_ENOTCONV = -5,      /* reserved for iterative solvers                     */
  RBGS_EUNSUPPORTED = -6   /* valid request outside what the kernels implement   */
} rbgs_status;

/* Element type of W and Q. */
typedef enum { RBGS_STORE_F64 = 0, RBGS_STORE_F32 = 1 } rbgs_store;

/* Arithmetic of the high-dimensional update Q'_(i) = W_(i) - Q_(1:i-1) R_(1:i-1,i)
 * (step 3 of Algorithm RBGS, the "coarse" unit roundoff u_crs of Section 2).
 *  F64  FP64 matrix-core products and accumulation; with FP32 storage the FP32
 *       data are converted exactly and only the result Q'_(i) is rounded to
 *       FP32.  Valid with either storage.
 *  F32  FP32 matrix-core products with FP32 accumulation and R rounded to FP32;
 *       FP32 storage only.  Its rounding errors, of size u32 ||W||, exceed Q'_(i)
 *       itself once W is numerically rank deficient at FP32 level, and then the
 *       sketched orthogonality is lost (the certificate Delta exposes it).
 *  BF16X3 split products on the bf16 matrix cores with FP32 accumulation; FP32
 *       storage only.  Each FP32 element a of Q is split as a_hi = bf16(a),
 *       a_lo = bf16(a - a_hi) and each element b of R_(1:i-1,i) as
 *       b_hi = bf16(fl32(b)), b_lo = bf16(fl32(b - b_hi)) (round to nearest
 *       even), and a b is taken as a_hi b_hi + a_hi b_lo + a_lo b_hi.  Each
 *       product carries a relative error of about 3 2^-16 (the dropped
 *       a_lo b_lo and the parts beyond two pieces), so the update is less
 *       accurate than with F32 and loses the sketched orthogonality sooner.
 * The sketches, the least-squares problem, the QR of the sketch and the
 * substitution always run in FP64 (the "fine" unit roundoff of Section 2). */
typedef enum { RBGS_MATH_F64 = 0, RBGS_MATH_F32 = 1, RBGS_MATH_BF16X3 = 2 } rbgs_math;

/* Sketching operator Theta (Section 1.3).  Entries are defined from
 * Philox-4x32-10 (key = seed; column r of Theta = row r of W):
 *  GAUSSIAN    Theta = Z / sqrt(k), Z[4j+e][r] from counter (r_lo, r_hi, j,
 *              0x47415553) through a single-precision Box-Muller transform;
 *              k % 4 == 0.
 *  SPARSE_SIGN Theta = B / sqrt(zeta): column r has zeta entries +-1, one in
 *              each of the zeta segments of k/zeta rows, from counters
 *              (r_lo, r_hi, c, 0x53504152), c = 0, 1; 1 <= zeta <= 8,
 *              k % zeta == 0, k <= 2048.
 *  IDENTITY    Theta = I, k == n (testing: RBGS then reduces to block
 *              Gram-Schmidt with exact projections).
 *  RADEMACHER  Theta = B / sqrt(k), B[t][r] = +-1 (the other dense
 *              oblivious embedding of Section 1.3): bit t % 32 of word
 *              (t % 128) / 32 of the output of counter (r_lo, r_hi, t / 128,
 *              0x52414445), a set bit meaning -1; k % 4 == 0.
 *  SRHT        Theta = P H D / sqrt(k) (subsampled randomized Hadamard
 *              transform, Section 1.3, zero padding to N = 2^L rows): D =
 *              diag(d_r), d_r = -1 if bit r % 128 of the output of counter
 *              (r / 128 lo, hi, 0, 0x53524854) is set; H[s][r] =
 *              (-1)^popcount(s & r) (Sylvester order); row j of P selects
 *              s_j = the top L bits of word j % 4 of counter (j / 4, 0, 1,
 *              0x53524854) (uniform, with replacement).  L = zeta if zeta > 0,
 *              else the smallest L with 2^L >= the rows of the call (row0 + n
 *              for the sketch calls; give zeta explicitly when sketching row
 *              ranges separately); k <= 2048. */
typedef enum {
  RBGS_SKETCH_GAUSSIAN = 0,
  RBGS_SKETCH_SPARSE_SIGN = 1,
  RBGS_SKETCH_IDENTITY = 2,
  RBGS_SKETCH_RADEMACHER = 3,
  RBGS_SKETCH_SRHT = 4
} rbgs_sketch_kind;

/* Inter-block QR in steps 4-5 (Section 2.2):
 *  PLAIN    RCholeskyQR: S'_(i) = Theta Q'_(i) computed from Q'_(i).
 *  LOWSYNC  RCholeskyQR with postponed sketching:
 *           S'_(i) = P_(i) - S_(1:i-1) R_(1:i-1,i); the update and the
 *           substitution are then one pass over the rows and each block needs
 *           a single device-wide reduction (the sketch of Q_(i)).
 *  TWICE    RCholeskyQR run twice (Section 2.2.4): after PLAIN gives
 *           Q'_(i) = Q*_(i) R1, RCholeskyQR of Q*_(i) gives Q*_(i) = Q_(i) R2
 *           and R_(i,i) = R2 R1 (one more sketch, QR and substitution).
 *  L2QR     l2-QR + RCholeskyQR (Section 2.2.4, the form the paper's
 *           experiments use): R' of the l2 QR of Q'_(i) by a Householder
 *           TSQR tree, Q*_(i) = Q'_(i) R'^-1 by substitution, RCholeskyQR of
 *           Q*_(i) = Q_(i) R'' and R_(i,i) = R'' R'. */
typedef enum {
  RBGS_VARIANT_PLAIN = 0,
  RBGS_VARIANT_LOWSYNC = 1,
  RBGS_VARIANT_TWICE = 2,
  RBGS_VARIANT_L2QR = 3
} rbgs_variant;

typedef struct {
  int32_t kind;      /* rbgs_sketch_kind                                  */
  int32_t zeta;      /* sparse sign: nonzeros per column (1..8); SRHT:
                        log2 of the transform size (0: derived)           */
  int64_t k;         /* sketch dimension (rows of Theta), m <= k <= n     */
  uint64_t seed;     /* Philox key                                        */
} rbgs_sketch;

typedef struct {
  int32_t store;     /* rbgs_store                                        */
  int32_t math;      /* rbgs_math                                         */
  int32_t variant;   /* rbgs_variant                                      */
  int32_t ls_iters;  /* Least-squares step (step 2).  l >= 1: Richardson
                        sweeps (supplement, Section SM.1); error <=
                        Delta^l |y|.  0: the direct Householder solver of
                        Section 2.1: a Householder QR of the sketch
                        S_(1:i-1), extended by each block's S_(i), applied
                        to P_(i) and solved with its R (one workgroup, FP64;
                        slower, for checking the sweeps); it needs k <= 1024,
                        at most 1024 columns before the last block and
                        p <= 16 when k > 512 (else RBGS_EUNSUPPORTED), and
                        batched calls run such problems one by one.  Outside
                        [0, 16]: RBGS_EINVAL.                              */
  void* stream;      /* hipStream_t or NULL                               */
} rbgs_opts;

/* A-posteriori certificate (step 6 of Algorithm RBGS). */
typedef struct {
  double delta;          /* ||I - S^T S||_F                                */
  double delta_tilde;    /* ||P - S R||_F / ||P||_F                         */
  int64_t breakdown_col; /* first column j with R_jj == 0 or not finite, -1 */
  int32_t nonfinite;     /* 1 if any entry of R or S is not finite          */
  int32_t reserved;
} rbgs_cert;

/* Create a handle bound to HIP device `device`.  No device memory is touched
 * until the first computing call.  Returns RBGS_EINVAL if h is NULL or device
 * is negative. */
RBGS_API rbgs_status rbgs_create(rbgs_handle* h, int device);

/* Free the handle's workspace (after waiting for its streams) and the handle.
 * A NULL handle is accepted. */
RBGS_API rbgs_status rbgs_destroy(rbgs_handle h);

/* RBGS QR factorization (Algorithm RBGS of Section 2).
 *   W    device, n x m (ld ldw >= n), element type opts->store; read only
 *        unless Q == W.
 *   p    block width (the paper's m_p); the blocks are columns [c0, c0+p);
 *        the last block is narrower when p does not divide m.  1 <= p <= 32.
 *   sk   host, the sketching operator; m <= sk->k <= n.
 *   opts host.
 *   Q    device, n x m (ld ldq >= n), element type opts->store.  Q == W (with
 *        ldq == ldw) factorizes in place; any other overlap is invalid.
 *   R    device, m x m FP64 (ld ldr >= m); upper triangular with positive
 *        diagonal on return; the strictly lower part is set to zero.
 *   S_out device or NULL, k x m FP64 (ld k): the sketch S = Theta Q.  (Without
 *        S_out and cert the sketch of the last block, which only they use, is
 *        not taken.)
 *   cert host or NULL.  When given, the call also computes Delta and Delta~,
 *        waits for the stream, and returns RBGS_EBREAKDOWN if a diagonal entry
 *        of R is zero or not finite (cert->breakdown_col names it; Q and R are
 *        valid up to the preceding block).  Without cert the call does not
 *        wait and a breakdown shows up as non-finite entries of Q.
 */
RBGS_API rbgs_status rbgs_qr(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m, int64_t p,
                    const rbgs_sketch* sk, const rbgs_opts* opts, void* Q, int64_t ldq,
                    double* R, int64_t ldr, double* S_out, rbgs_cert* cert);

/* Bytes of the device scratch array that rbgs_qr_noalloc works in (64 MiB). */
#define RBGS_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* rbgs_qr without any allocation, for callers that cannot allocate device or
 * host memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments and results as
 * rbgs_qr without the certificate (which needs a host wait); Q, R and S_out
 * are bitwise identical to rbgs_qr's for the same inputs and options.
 *  - Workspace: a fixed device array of RBGS_NOALLOC_SCRATCH_BYTES per device
 *    (part of the library's code object, held until the process ends)
 *    instead of the handle's workspace.  Its address is looked up on the first
 *    call on each device; that first call must not be under graph capture.
 *    The call itself makes no hipMalloc, hipFree, host-pinned allocation or
 *    event creation (profiling is not recorded for it).
 *  - A factorization whose workspace exceeds the array returns RBGS_ENOMEM
 *    before anything is enqueued (rbgs_last_error gives the bytes needed; the
 *    n = 10^6, m = 256, p = 16, k = 1024 sparse-sign FP32 factorization needs
 *    about 62 MB and fits).
 *  - Every call on one device shares that device's array, and the array keeps
 *    the contents of the last call.  Calls that may overlap on one device
 *    (other streams, other threads, other handles) race and must be ordered
 *    by the caller.  Everything the factorization needs cleared is cleared by
 *    its own kernels at the start of each call.
 *  - Errors: as rbgs_qr (RBGS_EINVAL, RBGS_EUNSUPPORTED on the host;
 *    RBGS_EDEVICE if a launch or the symbol lookup fails). */
RBGS_API rbgs_status rbgs_qr_noalloc(rbgs_handle h, const void* W, int64_t ldw, int64_t n, int64_t m,
                            int64_t p, const rbgs_sketch* sk, const rbgs_opts* opts, void* Q,
                            int64_t ldq, double* R, int64_t ldr, double* S_out);

/* One problem of a batch.  W, Q, R as for rbgs_qr (device); the struct itself
 * is host memory. */
typedef struct {
  const void* W;
  int64_t ldw;
  int64_t n, m;
  void* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  int64_t p;        /* block width; 0 = chosen by rbgs_autotune (set on return) */
  int64_t k;        /* sketch rows; 0 = chosen by rbgs_autotune (set on return) */
  int32_t status;   /* out: rbgs_status of this problem                        */
  int32_t reserved;
} rbgs_problem;

/* Flags of rbgs_qr_batched. */
#define RBGS_BATCH_GRAPH 1
#define RBGS_BATCH_PERSISTENT 2

/* Independent RBGS QR factorizations (Algorithm RBGS of Section 2) of a batch
 * of problems with their own n, m, p and k.
 *   probs host, `count` problems.  Problem i uses the sketch (sk->kind,
 *         sk->zeta, seed sk->seed + i, its own k); sk->k is ignored.
 *   opts  host; store, math, variant and ls_iters apply to every problem; the
 *         batch is enqueued on opts->stream.
 *   graph RBGS_BATCH_GRAPH: the first call with a given batch (same pointers,
 *         sizes, options, flags) runs it and records the whole enqueue
 *         sequence as a HIP graph; a later call with the identical batch
 *         launches that graph, one launch for the batch.  The graph reads W at
 *         run time, so W may change between calls.
 *         RBGS_BATCH_PERSISTENT (may be combined with RBGS_BATCH_GRAPH): every
 *         problem the persistent queue takes (FP32 storage, FP64 arithmetic,
 *         low-sync form, sparse sign with zeta <= 8, p <= 32, k <= 1024, and
 *         (K_last + 3) / 4 * 4 * w + w * w + w <= 18432 with K_last the columns
 *         before the last block and w = 16 for p <= 16, 32 otherwise) runs in
 *         ONE launch of one workgroup per compute unit that works through a
 *         device queue of the problems' stages (plan of Theta, sketch of W and
 *         its reduction, then per block the small factors, the update, the
 *         sketch of Q_(i) and its reduction), after an initialisation launch;
 *         stages of different problems run at the same time.  The call then
 *         waits for opts->stream and returns RBGS_EDEVICE if the queue did not
 *         drain (a workgroup waited more than 4 s for a stage; no such wait is
 *         expected).  Calls that overlap on one handle race.
 *         0: no graph, lock-step groups.
 * Without RBGS_BATCH_PERSISTENT, problems that share m, p and k (low-sync
 * form, sparse sign, p <= 32, k <= 2048; two or more of them) run in lock step
 * on opts->stream: block by block, one launch per kernel and block step for
 * the whole group, from a device array of per-problem descriptors and
 * workspaces in the handle's batch arena (laid out, uploaded and -- if an
 * earlier batch may still use it -- waited for on the host before anything is
 * enqueued).  The other problems are spread over four internal streams
 * (largest first, each to the least loaded stream), joined back to
 * opts->stream.  A call that lays the arena out again drops the recorded
 * graph.  Problems with p or k equal to 0 are tuned first (rbgs_autotune,
 * which waits for the device).
 * Every problem is validated before anything is enqueued: on an invalid
 * problem the call returns RBGS_EINVAL (or RBGS_EUNSUPPORTED) with that
 * problem's status set and enqueues nothing.  No certificate is computed. */
RBGS_API rbgs_status rbgs_qr_batched(rbgs_handle h, int64_t count, rbgs_problem* probs,
                                     const rbgs_sketch* sk, const rbgs_opts* opts, int32_t graph);

/* Autotuner for batched problems: measures RBGS QR on the device for an n x m
 * problem of synthetic data with every candidate (p, k), p in {16, 32} (not
 * above m) and k in {2m, 3m, 4m} (rounded up to a multiple of 8, at most n),
 * and returns the fastest.  Every candidate keeps k >= 2m, so the expected
 * cond2(Q) = cond2(Theta U) stays below about 6 (Section 3).  Results are
 * cached in the handle per (m, ceil(log2 n), store, math, kind, variant).
 * Waits for the device; uses the handle's workspace and a temporary
 * allocation of 2 n m elements freed before returning. */
RBGS_API rbgs_status rbgs_autotune(rbgs_handle h, int64_t n, int64_t m, const rbgs_sketch* sk,
                                   const rbgs_opts* opts, int64_t* p, int64_t* k);

/* Sparse matrix in compressed sparse row form (device arrays). */
typedef struct {
  int64_t n;                /* rows = columns                                */
  int64_t nnz;
  const int64_t* row_ptr;   /* n + 1 offsets                                 */
  const int32_t* col_idx;   /* nnz column indices, each in [0, n)            */
  const double* val;        /* nnz FP64 values                               */
} rbgs_csr;

/* Y = alpha A X + beta Y0 for a block of bs <= 32 vectors (the product of
 * step 2 of Algorithm RBGS-Arnoldi, Section 4.1).  X: n x bs (ld ldx),
 * element type xstore; Y: n x bs (ld ldy), element type ystore; Y0: n x bs
 * FP64 (ld ldy0) or NULL (then beta is ignored); Y must not overlap X.
 * FP64 arithmetic.  Enqueued on `stream`. */
RBGS_API rbgs_status rbgs_spmm(rbgs_handle h, const rbgs_csr* A, int32_t xstore, const void* X,
                               int64_t ldx, int64_t bs, double alpha, double beta, const double* Y0,
                               int64_t ldy0, int32_t ystore, void* Y, int64_t ldy, void* stream);

/* RBGS block Arnoldi (Algorithm RBGS-Arnoldi, Section 4.1): W_(1) = B and
 * W_(i) = A Q_(i-1) for i = 2..nblocks, each followed by iteration i of
 * RBGS.  On return Q (n x m, m = nblocks bs, element type opts->store) is
 * orthonormal with respect to the sketched product and R (m x m FP64, ld
 * ldr) holds the RBGS R factor: the Arnoldi identity reads
 * A Q_(1:p-1) = Q R_(1:p,2:p), so H = R[:, bs:m] and R_(1:p,1) = B's
 * coordinates.  B: n x bs (ld ldb), element type opts->store.  sk: as for
 * rbgs_qr with m <= sk->k <= n.  cert: as for rbgs_qr. */
RBGS_API rbgs_status rbgs_block_arnoldi(rbgs_handle h, const rbgs_csr* A, const void* B,
                                        int64_t ldb, int64_t bs, int64_t nblocks,
                                        const rbgs_sketch* sk, const rbgs_opts* opts, void* Q,
                                        int64_t ldq, double* R, int64_t ldr, rbgs_cert* cert);

/* Restarted randomized block GMRES (Section 4.2) for A X = B: each cycle
 * forms the residual R0 = B - A X (FP64), runs RBGS-Arnoldi on it with
 * blocks_per_cycle + 1 blocks (basis stored as opts->store), solves the
 * block Hessenberg least-squares problem min_Z ||H Z - R_(1:p,1)||_F in FP64
 * on the device, and updates X <- X + Q_(1:p-1) Z.  Stops when
 * ||B - A X||_F / ||B||_F <= tol (checked at the start of each cycle and at
 * the end) or after max_cycles.
 *   B, X   device, n x bs FP64 (ld n); X is the initial guess on entry.
 *   iters  host out: block iterations done (cycles x blocks_per_cycle).
 *   relres host out: final ||B - A X||_F / ||B||_F.
 *   history host or NULL, max_cycles + 1 doubles: relative residual at the
 *          start of every cycle and at the end (unused entries are -1).
 * Waits for the device once per cycle.  Returns RBGS_ENOTCONV (with X, iters
 * and relres valid) if tol is not reached. */
RBGS_API rbgs_status rbgs_block_gmres(rbgs_handle h, const rbgs_csr* A, const double* B, double* X,
                                      int64_t bs, int64_t blocks_per_cycle, int64_t max_cycles,
                                      double tol, const rbgs_sketch* sk, const rbgs_opts* opts,
                                      int64_t* iters, double* relres, double* history);

/* Cholesky-QR post-processing of a factorization W = Q R (the remark on
 * post-processing in Section 2.2): R' = upper Cholesky factor of Q^T Q (FP64,
 * Gram matrix on FP64 matrix cores), then Q <- Q R'^{-1} (block substitution,
 * FP64 arithmetic) and R <- R' R.  For the well-conditioned Q that RBGS
 * returns, the new Q is orthonormal in the l2 sense to about u cond(Q)^2 (plus
 * the rounding of the storage type) and W = Q R still holds.
 *   store  rbgs_store of Q.
 *   Q      device, n x m (ld ldq >= n), overwritten.
 *   R      device, m x m FP64 upper triangular (ld ldr >= m), overwritten.
 *   breakdown_col  host or NULL: if given, the call waits for the stream and
 *          stores the first pivot j at which Q^T Q was not positive definite
 *          (-1 if none; then RBGS_EBREAKDOWN is returned).
 * 1 <= m <= min(n, 8192).  Enqueued on `stream`. */
RBGS_API rbgs_status rbgs_cholqr_post(rbgs_handle h, int32_t store, void* Q, int64_t ldq, int64_t n,
                                      int64_t m, double* R, int64_t ldr, int64_t* breakdown_col,
                                      void* stream);

/* Sketch of a block of rows: out = Theta[:, row0:row0+n] X (Section 1.3), the
 * operation of steps 1 and 5 of Algorithm RBGS.
 *   X   device, n x c (ld ldx >= n), element type `store` (rbgs_store).
 *   out device, k x c FP64 (ld ldo >= k), overwritten.
 *   row0 global row index of the first row of X (Theta's columns are indexed
 *        by global rows, so sketches of row ranges add up to the full sketch).
 * Enqueued on `stream`. */
RBGS_API rbgs_status rbgs_sketch_apply(rbgs_handle h, const rbgs_sketch* sk, int32_t store, const void* X,
                              int64_t ldx, int64_t n, int64_t c, int64_t row0, double* out,
                              int64_t ldo, void* stream);

/* Explicit unscaled sketching matrix, for brute-force checks of the
 * definition above: out[t + k*(r - row0)] = Z[t][r] (Gaussian), B[t][r]
 * (sparse sign, +-1 or 0), B[t][r] (Rademacher), (H D)[s_t][r] (SRHT) or
 * I[t][r] (identity) for t < k, row0 <= r < row0+n.
 *   out device, k x n float (ld k), overwritten.  Theta = scale * out with
 *   scale = 1/sqrt(k) (Gaussian, Rademacher, SRHT), 1/sqrt(zeta) (sparse
 *   sign), 1 (identity). */
RBGS_API rbgs_status rbgs_theta_dense(rbgs_handle h, const rbgs_sketch* sk, int64_t n, int64_t row0,
                             float* out, void* stream);

/* Kernel timing for measurements.  rbgs_profile_enable takes a bit mask of
 * kernel classes (bit c enables class c; 0 disables; -1 enables all) and
 * clears the totals.  For every enabled class the handle records HIP events
 * around each launch on the stream it enqueues it on.  rbgs_profile_get waits for the recorded events and
 * returns, for kernel class `which`, the summed duration in milliseconds, the
 * number of launches and the summed algorithmic bytes (the minimal HBM
 * traffic of those launches: each input element read once, each output
 * element written once).
 *   which: 0 = update (steps 3 [+5 fused]), 1 = sketch partial products,
 *          2 = sketch reduction, 3 = small FP64 factors, 4 = substitutions
 *          and l2 QR passes over the block (all variants but LOWSYNC). */
RBGS_API rbgs_status rbgs_profile_enable(rbgs_handle h, int32_t enable);
RBGS_API rbgs_status rbgs_profile_get(rbgs_handle h, int32_t which, double* ms, int64_t* launches,
                             double* bytes);

RBGS_API const char* rbgs_status_string(rbgs_status s);
/* Text of the last error detected on this handle ("" if none). */
RBGS_API const char* rbgs_last_error(rbgs_handle h);

#ifdef __cplusplus
}
#endif

#endif /* RBGS_H */
