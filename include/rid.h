/*
 * rid.h -- randomized interpolative decomposition by LU with partial pivoting
 * on a Gaussian sketch, for AMD Instinct MI355X (gfx950).
 *
 * Method: Pearce, Chen, Dong, Martinsson, "Adaptive parallelizable algorithms
 * for interpolative decompositions via partially pivoted LU" (arXiv
 * 2310.09417).  Column form: for A (m x n) the library selects k columns J
 * and an interpolation matrix T (k x (n-k)) with
 *     A(:, J^c) ~= A(:, J) * T ,
 * i.e. A ~= A(:, J) X with X(:, J) = I_k and X(:, J^c) = T (Sec. 2.2.1,
 * column ID).  The row ID of the paper is the column ID of A^T.
 *
 * Conventions shared by every entry point
 *  - Pointers marked (device) are device pointers; everything else is host.
 *  - A is row-major with leading dimension lda >= n (element (i,j) at
 *    A[i*lda + j]).  The library never writes A.
 *  - J receives the skeleton columns in pivot order, 0-based.
 *  - T is row-major with leading dimension ldt >= n; column q of T belongs to
 *    the q-th non-skeleton column of A in ascending index order.
 *  - The caller owns every buffer, including the device workspace `work` of
 *    at least rid_workspace_bytes(...) bytes, exclusively for the duration of
 *    the call.  The library allocates nothing.
 *  - Besides device memory, the library keeps a small per-process pool of HIP
 *    streams and events (default priority, created on first use on a device,
 *    kept until the process ends).  The adaptive calls fork independent work
 *    (the growth of L1^{-1}) from `stream` to one of those streams and join it
 *    back by events before returning, so all of a call's work is ordered
 *    before any later work on `stream`; this also holds under stream capture.
 *    After hipDeviceReset the pooled streams are gone and the adaptive calls
 *    return RID_ERR_HIP.
 *  - Calls are asynchronous on `stream` and never synchronize with the host.
 *    The return value reports only argument / workspace / launch errors that
 *    the host can see.  The numerical outcome (rank, estimate, status) is
 *    written to the device scalars k_out, err_est, status and is valid once
 *    the stream has completed.
 *  - Not reentrant on one workspace; distinct workspaces may be used
 *    concurrently.
 */
#ifndef RID_H
#define RID_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RID_OK = 0,              /* tolerance met (or fixed rank done)                      */
  RID_NOT_CONVERGED = 1,   /* maximum rank reached with the estimate above tolerance  */
  RID_RANK_DEFICIENT = 2,  /* an exactly zero pivot: the sketch has rank k_out        */
  RID_ERR_ARG = -1,        /* invalid argument (host-detected)                        */
  RID_ERR_NONFINITE = -2,  /* A holds a NaN or an infinity (device-detected)          */
  RID_ERR_HIP = -3,        /* a HIP launch failed, or a device wait ran out           */
  RID_ERR_WORKSPACE = -4   /* workspace too small (host-detected)                     */
} rid_status;

typedef enum {
  RID_F64 = 0,       /* double                                             */
  RID_F32 = 1,       /* float                                              */
  RID_BF16 = 2,      /* bfloat16 bit patterns (uint16); storage of A only   */
  RID_FP8_E4M3 = 3   /* OCP FP8 e4m3 codes (uint8) with a power-of-two scale
                        per 128-column tile; storage of A only              */
} rid_dtype;

typedef struct {
  rid_dtype dtype;      /* factor type: storage of T; LUPP, Schur updates and
                           the interpolation solve run in this precision; every
                           norm and the stopping test accumulate in FP64.
                           RID_F64 or RID_F32.                                  */
  int tol_relative;     /* 1: stop when E <= tol * ||A||_F; 0: when E <= tol   */
  uint64_t seed;        /* key of the Gaussian embedding: entry (c, i) of sketch
                           vector c is a pure function of (seed, c, i)          */
  rid_dtype a_type;     /* storage type of A.  Equal to dtype, or, with dtype
                           RID_F32, RID_BF16 or RID_FP8_E4M3: the sketch then
                           multiplies in that format on the matrix cores (the
                           Gaussian entries rounded to nearest even into it)
                           with FP32 accumulation, summed across row ranges in
                           FP64.  The precision forms of the sketch step.      */
  const float* a_col_scale; /* (device) RID_FP8_E4M3 only: ceil(n/128) powers of
                           two; A(i, j) = code(i, j) * a_col_scale[j / 128].
                           NULL otherwise.                                      */
  int refine;           /* 0, or (dtype RID_F32 only) one iterative-refinement
                           step on T whose residual Y(:,J) T - Y(:,J^c) is
                           formed in FP64 from the FP32 sketch.  1: the device
                           then keeps whichever of the unrefined and refined T
                           has the smaller FP64 residual on the last drawn
                           estimate block (the method's independent sample,
                           an unbiased estimate of each ID's squared error;
                           the refined T when there is none: p = 0, k =
                           min(m, n), a rank-deficient stop).  2: keeps the
                           refined T unconditionally.                        */
  int estimator;        /* stopping estimate, one of rid_estimator.  0 (the
                           default) is the Schur estimate of eq. (errSch) on the
                           next block; 1-3 are the residual-triangle estimates
                           of Sec. 3.2, Remark 1 (see below)                    */
  int resid_p;          /* adaptive calls with estimator > 0: number p of
                           vectors set aside for the estimate, 1..16            */
  double* est_out;      /* (device, nullable) with estimator > 0: the three
                           Remark-1 estimates (sample, normUest, maxUest) last
                           taken: those of the returned rank when the call
                           stopped on the estimate or at kmax, of an earlier
                           rank when the ID then became exact (k = min(m, n))
                           or the sketch rank-deficient; -1 each when none was
                           taken.  Pass the same cfg to rid_workspace_bytes.  */
  int embedding;        /* rid_embedding of the sketch: RID_EMB_GAUSSIAN (the
                           default) or RID_EMB_SPARSE_SIGN (a_type == dtype
                           only; not on the batched path)                      */
  int side;             /* rid_side: RID_COLUMNS (0, the default) or RID_ROWS */
} rid_config;

/*
 * Which ID (Sec. 2.2): RID_COLUMNS selects columns J of A with
 * A(:, J^c) ~= A(:, J) T (the column ID, the form used throughout this
 * header).  RID_ROWS selects rows I of A with A(I^c, :) ~= T^T A(I, :) (the
 * row ID, A ~= W A(I, :) with W(I, :) = I and W(I^c, :) = T^T), i.e. the
 * column ID of A^T: the sketch is Y = A Omega with Omega n x l Gaussian,
 * formed from A in place (its rows are contracted, no transposed copy), and
 * LU with partial pivoting on Y picks the rows.  Then J receives row indices
 * (in [0, m)), T is k x (m - k) with leading dimension ldt >= m (column q for
 * the q-th non-skeleton row in ascending order), and relative tolerances
 * refer to ||A||_F as before.  RID_ROWS is supported by rid_lupp_fixed_rank,
 * rid_lupp_fixed_rank_noalloc, rid_lupp_adaptive, rid_workspace_bytes and
 * rid_debug_sketch with a_type == dtype (RID_F64 or RID_F32 storage); the
 * other entry points return RID_ERR_ARG (or 0 bytes) for it.
 */
typedef enum { RID_COLUMNS = 0, RID_ROWS = 1 } rid_side;

/*
 * Random embeddings of the sketch (Sec. 5, random matrix distributions).
 *   RID_EMB_GAUSSIAN     unit-variance Gaussian entries, a pure function of
 *                        (seed, vector, row) (Philox4x32-10 + Box-Muller).
 *   RID_EMB_SPARSE_SIGN  sparse sign, zeta = 8: in each draw of w vectors
 *                        (a block of the method), column i of Omega (row i of
 *                        A) holds min(8, w) entries +-sqrt(w / min(8, w)) at a
 *                        uniformly random subset of the draw's w rows (Floyd
 *                        sampling on Philox words at counter (i, first vector
 *                        of the draw, 0x53534e31, 0..2)), so that
 *                        E[Omega^T Omega] = w I and the estimate keeps its
 *                        scale.  The certificate always draws Gaussian vectors.
 */
typedef enum { RID_EMB_GAUSSIAN = 0, RID_EMB_SPARSE_SIGN = 1 } rid_embedding;

/*
 * Stopping estimates (Sec. 3.2, Remark 1).  With P the row permutation of the
 * factorisation and Yr = Omega_r A an independent Gaussian sample of p
 * vectors, the LU factors of P [Y Yr]^T end in a p x p upper triangle U_r
 * ("residual triangle"): U_r is the U factor of LU with partial pivoting on
 * the Schur complement S_r = (P Yr^T)(rest) - L2 L1^{-1} (P Yr^T)(pivots).
 * With nr = n - k candidates left and gamma(k) = 1 / max(1, k / (4 ln k))
 * (gamma(1) = 1; the reciprocal of the asymptotic LU growth bound k/(4 log k)):
 *   RID_EST_SAMPLE  ||S_r||_F / sqrt(p)
 *   RID_EST_UR_FRO  gamma(k) sqrt(nr) ||U_r||_F          (eq. normUest)
 *   RID_EST_UR_MAX  gamma(k) sqrt(nr) max |U_r(i, j)|    (eq. maxUest; may
 *                   under-estimate, as the remark notes)
 * Adaptive calls draw the p sample vectors once (stream indices 2^31 + j of
 * the seed's stream, in the call's embedding) and take the estimate of the current rank after
 * every factored block, so no block is drawn only to be measured; the rank
 * returned is the first block edge whose estimate meets the tolerance.
 * Fixed-rank calls use their p oversampling vectors as the sample.  The LU of
 * S_r stops at an exactly zero pivot column; the rows of U_r not reached are
 * zero.
 */
typedef enum {
  RID_EST_SCHUR = 0,
  RID_EST_SAMPLE = 1,
  RID_EST_UR_FRO = 2,
  RID_EST_UR_MAX = 3
} rid_estimator;

/*
 * Workspace size in bytes for a call with these sizes.  kmax is the rank
 * cap (fixed rank: k + p; adaptive: kmax), b the block width (fixed rank:
 * pass p).  Returns 0 for invalid arguments.
 */
size_t rid_workspace_bytes(int64_t m, int64_t n, int64_t kmax, int64_t b, const rid_config* cfg);

/* Human-readable name of a status code (static storage). */
const char* rid_status_string(int status);

/*
 * Fixed-rank randomized LUPP ID (randLUPP; Sec. 3.1 and Sec. 3.2).
 *   Y = Omega A with Omega (k+p) x m Gaussian, generated on the device from
 *   (seed, vector, row) for each sketch launch.  LU with partial pivoting on the first k columns of Y^T selects J
 *   (|J| = k, ties to the lowest column index); T = L1^{-T} L2^T
 *   (eq. (inty)).  The p remaining sketch vectors form an independent sample:
 *   err_est = ||S||_F / sqrt(p) for the Schur block S of eq. (errSch), the
 *   unbiased estimate of ||A - A(:,J) X||_F (0 <= p; p = 0 gives -1).  With
 *   cfg->estimator > 0 err_est is that Remark-1 estimate instead (p >= 1).
 * Arguments: 1 <= k <= min(m, n); J (device, int64[k]); T (device, dtype,
 *   k rows of ldt); k_out, status (device int32), err_est (device double).
 * Errors: RID_ERR_ARG for bad sizes or null pointers, RID_ERR_WORKSPACE when
 *   work_bytes is too small, RID_ERR_HIP when a launch fails.
 */
int rid_lupp_fixed_rank(const void* A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                        const rid_config* cfg, int64_t* J, void* T, int64_t ldt, int32_t* k_out,
                        double* err_est, int32_t* status, void* work, size_t work_bytes,
                        hipStream_t stream);

/*
 * rid_lupp_fixed_rank without a caller workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, arithmetic and results
 * as rid_lupp_fixed_rank, minus work / work_bytes: the workspace is a
 * file-scope device array of rid_noalloc_max_bytes() bytes (64 MiB) that
 * every device using the library holds until the process ends.  Its device
 * address is looked up on the first call on each device.  The call
 * allocates nothing and clears what must start at zero.
 * All calls on one device share that array: calls that overlap on one device
 * (two streams, two host threads) race and give undefined results; order
 * them on one stream or serialize them.
 * Errors: RID_ERR_WORKSPACE when the sizes need more than
 *   rid_noalloc_max_bytes() (rid_workspace_bytes(m, n, k + p, p, cfg) tells);
 *   RID_ERR_HIP when the array's address cannot be found; otherwise as
 *   rid_lupp_fixed_rank.
 */
size_t rid_noalloc_max_bytes(void);
int rid_lupp_fixed_rank_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                                int64_t p, const rid_config* cfg, int64_t* J, void* T,
                                int64_t ldt, int32_t* k_out, double* err_est, int32_t* status,
                                hipStream_t stream);

/*
 * Adaptive blocked randomized LUPP ID (randLUPPadap; Alg. 1, Sec. 4.2).
 *   The first block of b sketch vectors is factored.  Each further block
 *   Y^(t) is reduced by the current factors, U2 = L1^{-1} (P Y^(t))(top) and
 *   S = (P Y^(t))(bottom) - L2 U2; E = ||S||_F / sqrt(b) (FP64 accumulation).
 *   If E <= tol (times ||A||_F when relative) the call stops with rank k and
 *   status RID_OK; otherwise S is factored with partial pivoting and appended.
 *   At k = kmax (capped by min(m, n)) with E above tolerance the status is
 *   RID_NOT_CONVERGED; at k = min(m, n) the ID is exact (E = 0, RID_OK).
 *   With cfg->estimator > 0 the stopping estimate is a Remark-1 estimate of
 *   the rank just factored (see rid_estimator) and err_est holds it.
 * Arguments: 1 <= b <= 128; kmax >= 1; J (device, int64, capacity
 *   min(kmax, m, n)); T (device, capacity min(kmax,m,n) rows of ldt).
 * Errors: as rid_lupp_fixed_rank.
 */
int rid_lupp_adaptive(const void* A, int64_t m, int64_t n, int64_t lda, int64_t b, double tol,
                      int64_t kmax, const rid_config* cfg, int64_t* J, void* T, int64_t ldt,
                      int32_t* k_out, double* err_est, int32_t* status, void* work,
                      size_t work_bytes, hipStream_t stream);

/*
 * Row skeletons of C = A(:, J) for the two-sided ID and CUR (Sec. 2.4: with
 * the column skeletons J found, a second, direct LUPP on the small m x k
 * matrix C selects k rows I; Sec. 2.2: two-sided ID A ~= W A(I, J) X, with X
 * the column interpolation matrix of J and W = C A(I, J)^{-1} the row
 * interpolation matrix, W(I, :) = I_k).  LU with partial pivoting over the
 * m rows (ties to the lowest row index, as for columns); with P C = [L1; L2] U,
 * W(I^c, :) = L2 L1^{-1}.  CUR takes C = A(:, J) and R = A(I, :) from the
 * same skeletons.
 * Arguments: A as for rid_lupp_adaptive, stored in cfg->dtype (RID_F64 or
 *   RID_F32; no refinement, no estimator); J (device, int64[k]), the column
 *   skeletons, 1 <= k <= min(m, n); I (device, int64[k]) receives the row
 *   skeletons in pivot order; Tr (device, cfg->dtype, k rows of ldtr >= m)
 *   receives W(I^c, :)^T in the layout of T (the row ID is the column ID of
 *   A^T): Tr(s, q) = W(q-th non-skeleton row in ascending index, s), for
 *   s < k_out and q < m - k_out; k_out, status (device int32).
 *   Workspace: rid_rows_workspace_bytes(m, k, cfg).
 * Outcome (device): status RID_OK with k_out = k; RID_RANK_DEFICIENT with
 *   k_out = the steps taken when a pivot is exactly zero (C has rank k_out);
 *   RID_ERR_ARG when a J entry is outside [0, n) (k_out = 0, A not read
 *   there); RID_ERR_NONFINITE when C holds a NaN or infinity.
 * Errors (return value): RID_ERR_ARG / RID_ERR_WORKSPACE / RID_ERR_HIP.
 */
size_t rid_rows_workspace_bytes(int64_t m, int64_t k, const rid_config* cfg);
int rid_lupp_rows(const void* A, int64_t m, int64_t n, int64_t lda, const int64_t* J, int64_t k,
                  const rid_config* cfg, int64_t* I, void* Tr, int64_t ldtr, int32_t* k_out,
                  int32_t* status, void* work, size_t work_bytes, hipStream_t stream);

/*
 * A-posteriori certificate of an ID (the check Remark 1 ends with, after
 * Martinsson and Tropp, 2020): with Yc = Omega_c A for the p Gaussian vectors
 * c0 .. c0+p-1 of cfg->seed's stream,
 *     *cert = ||Yc(:, J^c) - Yc(:, J) T||_F / sqrt(p),
 * whose square is an unbiased estimate of ||A(:, J^c) - A(:, J) T||_F^2.
 * Use vectors the decomposition did not draw (e.g. c0 = 2^30).
 * Arguments: A as for rid_lupp_adaptive, stored in cfg->a_type; J (device,
 *   int64[k], any order, 0 <= k <= n), T (device, cfg->dtype, k rows of ldt;
 *   unused and may be NULL when k = 0 or k = n;
 *   rows in the order of J, column q for the q-th non-skeleton column in
 *   ascending index), 1 <= p <= 32, cert (device double).  Sums in FP64.
 * Errors: RID_ERR_ARG / RID_ERR_WORKSPACE / RID_ERR_HIP as above (workspace:
 *   rid_certificate_workspace_bytes).  A J entry out of range or repeated is
 *   found on the device and gives *cert = -1.
 */
size_t rid_certificate_workspace_bytes(int64_t m, int64_t n, int64_t p, const rid_config* cfg);
int rid_certificate(const void* A, int64_t m, int64_t n, int64_t lda, const int64_t* J, int64_t k,
                    const void* T, int64_t ldt, int64_t p, int64_t c0, const rid_config* cfg,
                    double* cert, void* work, size_t work_bytes, hipStream_t stream);

/*
 * Batched adaptive LUPP IDs of many independent blocks in one persistent
 * launch (the batch extension named as future work in the paper's
 * conclusions, applied to Alg. 1 per block).  Every array argument is a
 * DEVICE array of length nblk:
 *   A[i]  (device pointer, a_type) block i, m[i] x n[i], row-major, ld lda[i]
 *   kmax[i]  rank cap;  k_hint[i] (nullable array; entries <= 0 mean none):
 *            width of the first factored block, e.g. a predicted rank, so
 *            that the first pass can certify it; otherwise the first block
 *            has b vectors (Alg. 1);
 *   J[i]  (device pointer, int32, capacity min(kmax[i], m[i], n[i]))
 *   T[i]  (device pointer, dtype (the factor type), capacity min(kmax, m, n)
 *         rows of ldt[i])
 *   k_out, err_est, status, passes (nullable): per-block results, with
 *   passes[i] = number of sketch passes over block i.
 *   order (nullable): processing order (a permutation of 0..nblk-1), e.g.
 *   largest blocks first.
 * Storage and factor types: cfg->a_type == cfg->dtype (RID_F64 or RID_F32),
 * or FP32 blocks factored in FP64 (cfg->dtype RID_F64, cfg->a_type RID_F32:
 * the blocks are read at 4 bytes per entry and every step after the load runs
 * in FP64; T[i] is FP64).  No refinement, estimator or sparse embedding.
 * Block i uses the Gaussian stream of seed cfg->seed + i.  b <= 32; every n[i]
 * must be <= max_n <= 1024 (blocks outside the plan get status RID_ERR_ARG);
 * ranks are capped at min(max_kmax, max_n).  Workspace:
 * rid_batched_workspace_bytes(max_n, max_kmax, b, cfg).  A call factored in
 * FP32 takes at most as many blocks as the device has compute units (one
 * block per resident workgroup; more returns RID_ERR_ARG): such batches in
 * which a workgroup went on to a second block ended with a GPU memory fault
 * whose cause has not been found.  Calls factored in FP64 (FP64 or FP32
 * storage) take any number of blocks.
 */
size_t rid_batched_workspace_bytes(int32_t max_n, int32_t max_kmax, int32_t b,
                                   const rid_config* cfg);
int rid_lupp_batched(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                     const int32_t* n, int32_t b, double tol, const int32_t* kmax,
                     const int32_t* k_hint, const rid_config* cfg, int32_t* const* J,
                     void* const* T, const int64_t* ldt, int32_t* k_out, double* err_est,
                     int32_t* status, int32_t* passes, const int32_t* order, int32_t max_n,
                     int32_t max_kmax, void* work, size_t work_bytes, hipStream_t stream);

/*
 * Persistent grid of the batched kernel (the number of workgroups that take
 * blocks from the queue; factorisations in FP64): by default one per compute
 * unit.  A grid chosen for a key (device, storage and factor types, b, max_n
 * rounded up to a power of two) is used by every later rid_lupp_batched call
 * with that key.  The grid changes which workgroup takes which block, not
 * any block's arithmetic: results are identical for every grid.
 * rid_batched_set_grid: grid >= 1 workgroups (capped at the compute units),
 *   0 = the default.
 * rid_batched_autotune: with the arguments of rid_lupp_batched (its outputs
 *   are overwritten), times the candidate grids (all, three quarters and
 *   half of the compute units; one untimed call, then the median of three,
 *   HIP events on `stream`, which it synchronizes: a tuning call, not for
 *   capture), records the fastest, returns it in *grid_out (host, nullable)
 *   and the three medians in ms_out[3] (host, nullable; -1 for candidates
 *   not timed).  FP32 factorisations keep one block per workgroup, so only
 *   the default is timed for them.
 * Both return RID_ERR_ARG for invalid arguments (set_grid: also for an FP32
 * factorisation).
 */
int rid_batched_set_grid(const rid_config* cfg, int32_t b, int32_t max_n, int32_t grid);
int rid_batched_autotune(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                         const int32_t* n, int32_t b, double tol, const int32_t* kmax,
                         const int32_t* k_hint, const rid_config* cfg, int32_t* const* J,
                         void* const* T, const int64_t* ldt, int32_t* k_out, double* err_est,
                         int32_t* status, int32_t* passes, const int32_t* order, int32_t max_n,
                         int32_t max_kmax, void* work, size_t work_bytes, hipStream_t stream,
                         int32_t* grid_out, float* ms_out);

/*
 * Test export: materialises the Gaussian embedding block
 *   out[c * m + i] = omega(c0 + c, i), 0 <= c < w, 0 <= i < m
 * in the given dtype (device buffer).  The decomposition keeps Omega only
 * as the workspace tiles of one sketch launch; this exists so the generator
 * can be checked on its own.
 */
int rid_debug_gaussian(uint64_t seed, int64_t c0, int64_t w, int64_t m, int dtype, void* out,
                       hipStream_t stream);

/*
 * Test export: the sketch alone, Yt = (Omega(c0:c0+w, :) A)^T stored as an
 * n x w row-major matrix with leading dimension ldy (device, dtype), using
 * the same kernels as the decomposition (with c0 == 0 the launch also sums
 * ||A||_F^2, as the first sketch of a decomposition does).  Requires a
 * workspace of rid_workspace_bytes(m, n, w, w, cfg) bytes.  w <= 128.
 */
int rid_debug_sketch(const void* A, int64_t m, int64_t n, int64_t lda, int64_t c0, int64_t w,
                     const rid_config* cfg, void* Yt, int64_t ldy, void* work, size_t work_bytes,
                     hipStream_t stream);

/*
 * Learned rank (callers that size the batched sketch up front through
 * rid_lupp_batched's k_hint).  The paper notes that the adaptive method
 * re-sketches until its estimate meets the tolerance (Sec. 4.2, Alg. 1); a
 * predicted rank lets the first pass draw about that many vectors at once,
 * and the adaptive loop continues from there when the prediction is short.
 *
 * rid_rank_features: 19 features per block (features: nblk x 19 FP32,
 * device): log2 m, log2 n, log10 of the relative tolerance, and
 * log10(E_s / ||A||_F) for s = 0..15, E_s = ||S_s||_F / sqrt(16 - s) the
 * Schur-complement estimate (Sec. 4.2, eq. errSch) after s LUPP steps on the
 * block's first 16 sketch vectors (the stream of seed + block index, as in
 * rid_lupp_batched).  Blocks as in rid_lupp_batched (device arrays of
 * pointers, lda, m, n; cfg->dtype = storage type F64 or F32, cfg->seed,
 * cfg->tol_relative).  A block with n > 1024 gets NaN features.
 */
int rid_rank_features(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                      const int32_t* n, double tol, const rid_config* cfg, float* features,
                      hipStream_t stream);

/*
 * The rank MLP: 19 -> 128 -> 128 -> 1, GELU (erf form), predicting log2 of the
 * rank.  params: rid_mlp_param_count() FP32 values (device), in the order
 * W1 (128 x 19, row-major), b1 (128), W2 (128 x 128), b2 (128), w3 (128), b3;
 * weight matrices are used rounded to BF16 (nearest even), everything else
 * is FP32.  xnorm (device, nullable): 19 means then 19 inverse standard
 * deviations applied to the features first.
 *
 * rid_mlp_forward: y[B] (device); z1, z2 (B x 128, nullable) keep the
 *   pre-activations for rid_mlp_backward.
 * rid_mlp_backward: gradient (device, param_count FP32) of the mean pinball
 *   loss rho_q(target - y) over the B samples, and that loss (device double,
 *   nullable).  Deterministic (fixed-order reduction).  work: device buffer of
 *   rid_mlp_workspace_bytes(B) bytes.  q in (0, 1).
 * rid_mlp_adamw: one AdamW step (moments m1, m2 device, zero-initialised by
 *   the caller; step >= 1; decoupled weight decay on weight matrices only).
 * rid_rank_hint: k_hint[i] = min(kcap[i], ceil(2^y[i] (1 + margin))), at least
 *   1; 0 (no hint) for a non-finite prediction.
 * All return RID_ERR_ARG on null or invalid arguments.
 */
int32_t rid_mlp_param_count(void);
size_t rid_mlp_workspace_bytes(int32_t B);
int rid_mlp_forward(int32_t B, const float* X, const float* xnorm, const float* params, float* y,
                    float* z1, float* z2, hipStream_t stream);
int rid_mlp_backward(int32_t B, const float* X, const float* xnorm, const float* z1,
                     const float* z2, const float* y, const float* target, float q,
                     const float* params, float* grad, double* loss, void* work,
                     size_t work_bytes, hipStream_t stream);
int rid_mlp_adamw(float* params, const float* grad, float* m1, float* m2, int32_t step, float lr,
                  float beta1, float beta2, float eps, float weight_decay, hipStream_t stream);
int rid_rank_hint(int32_t B, const float* y, float margin, const int32_t* kcap, int32_t* k_hint,
                  hipStream_t stream);

/*
 * Test export: one wave checks the matrix-instruction layouts and number
 * conversions of the low-precision sketch.  D is 16 x 16 FP32 (device).
 *   kind 0: D = A B with A 16 x 32 and B 32 x 16 BF16 bit patterns (uint16,
 *           row-major, device)
 *   kind 1: the same with OCP FP8-e4m3 codes (uint8)
 *   kind 2: A holds 64 floats; D[i] = BF16 pattern and D[64 + i] = e4m3 code
 *           of A[i], both rounded to nearest even
 *   kind 3: B holds the 256 e4m3 codes; D[c] = value of code c
 * Returns RID_ERR_ARG for another kind or a null pointer.
 */
int rid_debug_mfma_probe(int kind, const void* A, const void* B, float* D, hipStream_t stream);

/*
 * Optional timing.  After rid_profile_start(), every kernel launch of the
 * library is bracketed by two HIP events on the call's stream (host-side
 * event objects are created on first use and reused).  rid_profile_stop()
 * waits for the recorded events and returns, per kernel class, the summed
 * elapsed milliseconds and the number of launches; it also ends recording.
 * Classes: 0 sketch, 1 sketch reduction, 2 U2 = L1^{-1} (P Y)(top),
 * 3 Schur update, 4 panel LUPP, 5 interpolation matrix, 6 update of L1^{-1},
 * 7 batched persistent kernel, 8 generation of the sketch vectors' Gaussian
 * entries, 9 Remark-1 estimate, 10 two-block low-precision sketch (128
 * vectors per pass).  Process-wide state:
 * not for concurrent use from several host threads.
 */
int rid_profile_start(void);
int rid_profile_stop(double* ms, int64_t* launches, int nclass);

/*
 * Releases the library's host-side resources: the pooled HIP streams and
 * events of the adaptive calls (after waiting for their work) and the
 * profiling events, on every device that created them; the current device
 * is restored.  Later calls create them again as needed.  Call it after all
 * of the library's work has been issued and before the process tears the
 * HIP runtime down (e.g. under a profiler that reports at exit).  Returns
 * RID_ERR_ARG (and leaves that set alone) if a call on another host thread
 * still holds a stream set, RID_ERR_HIP if a HIP call fails.
 */
int rid_release(void);

#ifdef __cplusplus
}
#endif
#endif /* RID_H */
