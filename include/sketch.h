/*
 * sketch.h -- C ABI of the MI355X sketch library (libsketch.so).
 *
 * The operation (paper Sec. I-A, eq. (1)): given a tall sparse A (m x n,
 * m >> n) and a sketch size d (n < d <= 4n typical), sample S (d x m) with
 * i.i.d. entries from a prescribed distribution and return A_hat = S A.
 * S is never stored: it is regenerated on the fly from a counter-based
 * generator (Sec. IV-B-1), Philox4x32-10 keyed by the 64-bit seed with
 * counter (S-row group, S column), so every entry is a pure function of
 * (seed, row, column) and the result does not depend on tiling or launch
 * shape (Sec. IV-C).
 *
 * Conventions common to every call:
 *  - All matrix/vector pointers are DEVICE pointers owned by the caller; the
 *    library never allocates device memory (the caller passes a workspace;
 *    the one exception is the fixed per-device array of sk_sketch_noalloc),
 *    so device-memory accounting by the caller is exact.
 *  - Indices are 0-based (the paper's pseudocode is 1-based).
 *  - A is CSC: colptr int64[n+1] (colptr[0] = 0, colptr[n] = nnz, non-
 *    decreasing), rowidx int32[nnz] strictly increasing within a column and
 *    in [0, m), vals[nnz] of type vtype.  Explicit zeros are structural.
 *    FP64 values are rounded to FP32 (round to nearest even) on load.
 *  - Outputs are column-major FP32 with leading dimension ld >= rows, and
 *    are overwritten (not accumulated into).
 *  - Calls are asynchronous on the caller's HIP stream (hip_stream may be
 *    NULL for the default stream).  Argument errors (null pointers, bad
 *    sizes, too-small workspace) are returned synchronously.  Errors in the
 *    CSC *contents* are detected on the device; they make the call write
 *    NaN into the output and record a status in the workspace, which
 *    sk_sketch_status() returns (it synchronises the stream).
 *  - HIP launch failures map to SK_EHIP.
 *  - The library holds no mutable global state besides the fixed device
 *    array of sk_sketch_noalloc (below); concurrent calls on different
 *    streams with different workspaces are independent.
 */
#ifndef SKETCH_H
#define SKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SK_OK = 0,
  SK_EINVAL = -1,       /* bad argument (null pointer, size < 1, ld < rows, ...) */
  SK_EUNSORTED = -2,    /* row indices not strictly increasing within a column   */
  SK_ERANGE = -3,       /* a row index outside [0, m)                            */
  SK_EWORKSPACE = -4,   /* workspace pointer null or smaller than required       */
  SK_EHIP = -5,         /* a HIP runtime call or kernel launch failed            */
  SK_EUNSUPPORTED = -6, /* valid request this build does not support             */
  SK_ECOLPTR = -7       /* colptr not non-decreasing from 0 to nnz               */
} sk_status;

/* Distribution of the i.i.d. entries of S (Sec. I-A): uniform on {+1,-1},
 * uniform on (-1,1), standard Gaussian. */
typedef enum { SK_RADEMACHER = 0, SK_UNIFORM = 1, SK_GAUSSIAN = 2 } sk_dist;

/* Element type of the CSC values. */
typedef enum { SK_F64 = 0, SK_F32 = 1, SK_BF16 = 2 } sk_vtype;

/* Operand precision of row blocks that are dense enough to run as a dense
 * contraction on the matrix cores.  SK_PREC_F32 keeps FP32 operands; BF16 and
 * FP8 (E4M3) hold +-1 entries of S exactly and are accepted for the +-1
 * distribution only.  Accumulation is always FP32. */
typedef enum { SK_PREC_F32 = 0, SK_PREC_BF16 = 1, SK_PREC_FP8 = 2 } sk_prec;

/* A sparse CSC matrix in device memory (see the conventions above). */
typedef struct {
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int32_t* rowidx;
  const void* vals;
  int32_t vtype; /* sk_vtype */
} sk_csc;

/* Optional tuning override (NULL = the library's own choice from the shape).
 * Any valid setting gives the same S and A_hat up to FP32 summation order. */
typedef struct {
  int32_t rows_per_block; /* nonempty A rows per S tile (0 = auto)            */
  int32_t splits;         /* row-range splits combined by a fixed-order sum   */
  int32_t variant;        /* kernel shape id (0 = auto); see sk_variant_count */
  int32_t dense_min_pct;  /* densify a row block at >= this % density (0 = auto,
                             101 = never)                                      */
  int32_t phases;         /* 0 = all; else a mask of 1 = validate + inspector,
                             2 = S tiles + sparse accumulation, 4 = split
                             reduction, 8 = dense blocks on the matrix cores.
                             Running a subset reuses the workspace contents of
                             an earlier full call with the same A (unchanged),
                             d, distribution, precision and tuning: phases
                             2|4|8 sketch another seed or row0 from that call's
                             layout without validating and inspecting A again
                             (repeated sketches of one A; also used to time
                             one phase in isolation).                         */
  int32_t tile_rows;      /* S rows per workgroup tile (0 = autotuner's choice;
                             else a power-of-two multiple of the kernel shape's
                             rows per column group)                           */
  int32_t col_split;      /* heavy-column splitting: 0 = auto (on for n >= 512),
                             1 = off, 2 = on                                  */
  int32_t row_pad;        /* S-tile row padding in floats: 0 = none (rows of
                             d_b floats), else this many extra floats per row
                             (a multiple of 4)                                */
  int32_t count_rng;      /* nonzero: run the sparse kernel's call-counting
                             instantiation, which also adds up its generator
                             calls (read with sk_sketch_rng_calls; same
                             A_hat; for checks, not for speed)                */
  int32_t rng_mode;       /* generator of the distribution-cost ablation
                             (Sec. III-A's cost h of a random number; Sec. V's
                             "junk" generator): 0 = Philox4x32-10 (the
                             product); 1 = a junk counter hash (NOT random:
                             times the sketch without the generator's cost;
                             A_hat is not S A); 3 = (-1,1) only: S kept as
                             the integers 2^24 s, A_hat scaled by 2^-24 at the
                             end (the integer-scaling trick; same A_hat as 0).
                             Modes 1 and 3 run on the kernel shapes 3, 6 and 9
                             without dense blocks; else SK_EUNSUPPORTED.    */
  int32_t kernel;         /* 0 = auto, 1 = the S-tile kernel (Algorithm 4's
                             reuse of an S tile across a row block; every
                             field above applies to it), 2 = the Algorithm 3
                             loop-order kernel of sk_sketch_colwise (FP32,
                             Philox only; the fields above are ignored except
                             count_rng and rng_mode, which it refuses with
                             SK_EUNSUPPORTED).  Auto takes the Algorithm 3
                             kernel only for FP32 requests that set no other
                             field, when its predicted time (from the shape
                             alone) is under half the S-tile kernel's.     */
  int32_t balance;        /* row blocks of the S-tile kernel (single sketches):
                             0 = auto, 1 = nonempty rows in order, 2 =
                             balanced: inside super-blocks of up to 16 blocks
                             the rows are dealt to blocks so that each
                             column's entry count per block is about even
                             (the lockstep of the column walk then wastes
                             less; A_hat is the same up to rounding, S being
                             a function of the row index).  Needs n <= 2048
                             (else rows in order).  Auto: on for 512 <= n <=
                             2048 when nonempty rows hold four or more
                             nonzeros on average, a block about 1 to 16
                             entries per column, and the matrix at least four
                             super-blocks of nonempty rows.  It adds to the
                             inspector's time (on 2e6 rows of ten nonzeros
                             about 1 ms) and saves more in the kernel (2.4
                             ms there).  Batched calls keep rows in order.   */
} sk_tuning;

/* Human-readable name of a status code (static storage). */
const char* sk_status_string(int status);

/* Number of kernel shape variants accepted in sk_tuning.variant (1..count). */
int sk_variant_count(void);

/* Workspace bytes sk_sketch needs for this A, d and tuning (tune may be
 * NULL).  Host-only; touches no device memory.  Returns SK_EINVAL on bad
 * sizes. */
sk_status sk_sketch_workspace(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                              const sk_tuning* tune, size_t* bytes);

/* A_hat[0:d, 0:n] = S[row0 : row0+d, 0:m] * A   (eq. (1); the row offset is
 * the paper's r in compute_kernel(A_hat[i:, j:], A[:, j:], i), Algorithm 1).
 * A_hat: device FP32, column-major, leading dimension ld >= d, written in
 * full.  ws: device workspace of ws_bytes >= sk_sketch_workspace().  The
 * call validates A on the device (see sk_sketch_status), builds the blocked
 * row layout of A (the inspector), regenerates S tile by tile and
 * accumulates in FP32.  Asynchronous on hip_stream. */
sk_status sk_sketch(const sk_csc* A, int64_t row0, int64_t d, int32_t dist, uint64_t seed,
                    int32_t prec, const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                    size_t ws_bytes, void* hip_stream);

/* Allocation-free form of sk_sketch, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation and result as sk_sketch with the
 * same arguments, but the workspace is a fixed device array inside the
 * library, SK_NOALLOC_SCRATCH_BYTES per device, which every GPU the library
 * runs on holds until the process ends.  The caller still owns A and A_hat.
 * The call allocates nothing and frees nothing; it resolves the array's
 * device address on its first call on each device (the current device).
 * Returns SK_EWORKSPACE when sk_sketch_workspace() for these arguments
 * exceeds SK_NOALLOC_SCRATCH_BYTES.  All calls on one device share its one
 * array: calls that overlap on a device (different streams, or other host
 * threads) race and must be serialised by the caller.  Every call clears
 * what must start at zero itself.  Errors in the CSC contents give NaN in
 * A_hat (the status record sits in the shared array, with no reader call). */
#define SK_NOALLOC_SCRATCH_BYTES (64ull << 20)
sk_status sk_sketch_noalloc(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                            uint64_t seed, int32_t prec, const sk_tuning* tune, float* Ahat,
                            int64_t ld, void* hip_stream);

/* The sketch with S given explicitly instead of generated (the stored-S
 * sparse product of the distribution-cost ablation: what regenerating S
 * saves against reading it from memory): A_hat[0:d, 0:n] = S A with S
 * device FP32, column-major d x m, leading dimension lds >= d rounded up to a
 * multiple of 128 (rows past d are read but never used), 16-byte aligned.
 * Same workspace as sk_sketch(A, d, SK_UNIFORM, SK_PREC_F32, tune) on the
 * S-tile kernel (tune->kernel = 1), which it always runs; same kernel shapes
 * as sk_tuning.rng_mode.  Asynchronous on hip_stream. */
sk_status sk_sketch_stored(const sk_csc* A, int64_t d, const float* S, int64_t lds,
                           const sk_tuning* tune, float* Ahat, int64_t ld, void* ws,
                           size_t ws_bytes, void* hip_stream);

/* The sketch in the loop order of Algorithm 3 (variant kji, Sec. II-B):
 * A_hat[0:d, 0:n] = S[row0 : row0+d, :] A where every nonzero a_jk
 * regenerates its S column segment S[row0 : row0+d, j] and adds a_jk times
 * it into column k; no S tile is reused across columns and A is used as the
 * given CSC (validated on the device, no inspector).  Same S, so the same
 * A_hat as sk_sketch up to FP32 summation order (each entry here sums the
 * column's nonzeros in row order).  Generator calls: nnz x (groups of 4, or
 * of 128 for +-1, that the rows touch per 256 / 2048 rows).  A column with
 * more than C nonzeros (C a power of two >= 512 chosen from nnz and d so that
 * the partials stay within 256 MiB) is split into chunks of C nonzeros
 * walked in parallel, whose partial sums are then added in chunk order (each
 * entry of such a column is a sum of per-chunk sums).  Workspace:
 * sk_sketch_colwise_workspace bytes for this A and d (the validation status,
 * read with sk_sketch_status; the chunk bookkeeping and the partials).
 * Asynchronous on hip_stream. */
sk_status sk_sketch_colwise_workspace(const sk_csc* A, int64_t d, size_t* bytes);
sk_status sk_sketch_colwise(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                            uint64_t seed, float* Ahat, int64_t ld, void* ws, size_t ws_bytes,
                            void* hip_stream);

/* The same in FP64: A's values in FP64 (FP32 and BF16 widen exactly), the same
 * S entries (exact in FP64), FP64 sums; A_hat device FP64, column-major, ld >=
 * d.  For uses that need the sketch beyond FP32 accuracy (the SVD form of
 * sketch-and-precondition drops singular values only below sigma_max / 1e12).
 * Workspace and status as sk_sketch_colwise. */
sk_status sk_sketch_colwise_f64(const sk_csc* A, int64_t row0, int64_t d, int32_t dist,
                                uint64_t seed, double* Ahat, int64_t ld, void* ws,
                                size_t ws_bytes, void* hip_stream);

/* Generator throughput, for measuring the cost of one call (the h of Sec.
 * III-A): blocks x 256 threads each make `calls` calls of the generator
 * (gen 0 = Philox4x32-10, 1 = the junk hash of sk_tuning.rng_mode) with the
 * transform of `dist` (+-1: the raw words), for counters (call index, thread
 * index), fold all outputs of a thread into one word and write it to
 * sink[thread] (device, blocks * 256 words).  Asynchronous on hip_stream; the
 * caller times it. */
sk_status sk_rng_throughput(int32_t dist, int32_t gen, int64_t calls, int32_t blocks,
                            uint64_t seed, uint32_t* sink, void* hip_stream);

/* Status of the last sk_sketch that used this workspace (synchronises
 * hip_stream).  Also reports the inspector's counts when the pointers are
 * non-NULL: nonempty rows of A and row blocks.  Returns SK_OK, SK_EUNSORTED,
 * SK_ERANGE, SK_ECOLPTR or SK_EHIP. */
sk_status sk_sketch_status(const void* ws, void* hip_stream, int64_t* nonempty_rows,
                           int64_t* row_blocks);

/* Generator calls the last sk_sketch on this workspace made in its sparse
 * kernel, counted only when it ran with sk_tuning.count_rng set (else 0).
 * Each S tile is generated once per row block, so the count is
 * sum over (tile, block) of |rows of the block| x (generator groups the
 * tile's S rows touch): 4 rows per group for (-1,1) and the Gaussian, 128
 * for +-1 (Sec. III-B counts the random numbers a blocked sketch draws).
 * Synchronises hip_stream. */
sk_status sk_sketch_rng_calls(const void* ws, void* hip_stream, uint64_t* calls);

/* Autotuner, model form: the tuning sk_sketch(prec SK_PREC_F32) would choose
 * for this shape with tune NULL (the cached plan of the shape class if
 * sk_autotune_measure filled one; else the cost model: the kernel, then for
 * the S-tile kernel the S-row tile height and rows per block by cost, the
 * kernel shape by column count, the splits by occupancy).  Host-only. */
sk_status sk_autotune(const sk_csc* A, int64_t d, int32_t dist, sk_tuning* out);

/* The cost model's view of a request, for inspection (host-only): info[0] =
 * predicted S-tile kernel time (us), info[1] = predicted Algorithm 3 kernel
 * time (us), info[2] = the kernel auto picks (1 or 2), info[3] = the S-tile
 * plan's cost (CU-cycles), info[4] = its kernel shape (1-based), info[5] =
 * its blocks per balanced super-block (0: rows in order, see
 * sk_tuning.balance); the first ninfo of these are written.  tune as for sk_sketch (NULL: the cached
 * plan, else the model). */
sk_status sk_plan_info(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                       const sk_tuning* tune, double* info, int32_t ninfo);

/* Autotuner, measured form: runs the candidates on the device and keeps the
 * fastest.  Stage one times the Algorithm 3 kernel (FP32 only) and every
 * S-tile kernel shape at the model's splits (the matrix-core path: its one
 * shape); stage two times splits 1..64 for the three fastest S-tile shapes
 * (balanced row blocks as the model's rule decides); stage three times the
 * winner with the balanced row blocks switched the other way (balance 1 or
 * 2), where the S-tile kernel runs it and the plan allows the switch.
 * Each candidate: one untimed call, then the best of up to three calls timed
 * with events on hip_stream (one when already 1.5x slower than the best).
 * The winner (fields kernel, variant, splits, balance; the rest 0) is
 * written to *out,
 * its time in ms to *best_ms (may be NULL), and stored in the process-wide
 * plan cache under the request's shape class: distribution, precision and
 * the sizes m, n, nnz, d each rounded to half an octave.  From then on
 * sk_sketch, sk_sketch_workspace, sk_sketch_noalloc and sk_autotune called
 * with tune NULL on a request of that class use it (query the workspace
 * after tuning).  The class does not see where the nonzeros sit: matrices of
 * one size class but different structure (Table VI) should pass their own
 * tuning.  Synchronises hip_stream; on return A_hat (device FP32, ld >= d)
 * holds the sketch with the winning tuning (S from seed, rows 0..d-1).  ws:
 * device workspace of sk_autotune_workspace bytes (the largest any candidate
 * takes).  An A that fails validation returns its status code and caches
 * nothing. */
sk_status sk_autotune_workspace(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                                size_t* bytes);
sk_status sk_autotune_measure(const sk_csc* A, int64_t d, int32_t dist, uint64_t seed,
                              int32_t prec, float* Ahat, int64_t ld, void* ws, size_t ws_bytes,
                              void* hip_stream, sk_tuning* out, double* best_ms);

/* The plan cache (host-only; guarded by one mutex): lookup returns 1 and
 * writes the cached tuning of the request's shape class, or 0 when there is
 * none (SK_EINVAL on NULL arguments); clear empties it. */
int sk_plan_cache_lookup(const sk_csc* A, int64_t d, int32_t dist, int32_t prec,
                         sk_tuning* out);
void sk_plan_cache_clear(void);

/* Many independent sketches in one pass (the batched form of sk_sketch):
 * item i computes Ahat[i] = S_i[0:d[i], :] A[i] with S_i from seed[i] and
 * dist[i].  A, d, dist, seed, Ahat and ld are HOST arrays of `count`
 * entries; the matrices and outputs they describe are device memory.  tune
 * is NULL or a host array of per-item overrides (kernel shape must agree
 * across the batch).  One batched inspector pass covers all items, then one
 * persistent launch per distribution runs every item's work units from a
 * longest-first list (the only shared state is one atomic work counter);
 * each item's result is bitwise the one sk_sketch gives with the tuning
 * sk_sketch_batched_plan reports for it.  prec SK_PREC_BF16 / SK_PREC_FP8
 * (all items +-1, else SK_EUNSUPPORTED): items of density >= 1% (or the
 * item's dense_min_pct) run as a dense contraction on the matrix cores with
 * +-1 S exact in that format, in their own persistent launch; the others run
 * the FP32 sparse kernel.  Asynchronous on hip_stream; per-item device
 * validation status via sk_sketch_batched_status. */
sk_status sk_sketch_batched_workspace(int32_t count, const sk_csc* A, const int64_t* d,
                                      const int32_t* dist, int32_t prec, const sk_tuning* tune,
                                      size_t* bytes);
sk_status sk_sketch_batched(int32_t count, const sk_csc* A, const int64_t* d, const int32_t* dist,
                            const uint64_t* seed, int32_t prec, const sk_tuning* tune,
                            float* const* Ahat, const int64_t* ld, void* ws, size_t ws_bytes,
                            void* hip_stream);

/* The per-item tunings the batched call uses (host only; chosen has `count`
 * entries). */
sk_status sk_sketch_batched_plan(int32_t count, const sk_csc* A, const int64_t* d,
                                 const int32_t* dist, int32_t prec, const sk_tuning* tune,
                                 sk_tuning* chosen);

/* Per-item device validation status of the last batched call on this
 * workspace (synchronises hip_stream); returns the last failing status or
 * SK_OK. */
sk_status sk_sketch_batched_status(const void* ws, int32_t count, void* hip_stream,
                                   int32_t* statuses);

/* Test hook: S[row0 : row0+d, col0 : col0+ncols] into S (device FP32,
 * column-major, leading dimension ld >= d), from the same device generator
 * the sketch uses.  Asynchronous on hip_stream. */
sk_status sk_materialize_s(int64_t row0, int64_t d, int64_t col0, int64_t ncols, int32_t dist,
                           uint64_t seed, float* S, int64_t ld, void* hip_stream);

/* Test hook (host only, no device): the FP32 coefficient tables the device
 * generator uses, for comparison with an independent derivation:
 * log_c[5], sin_c[7], cos_c[8], misc[3] = {ln2_hi, ln2_lo, sqrt2}. */
void sk_rng_tables(float* log_c, float* sin_c, float* cos_c, float* misc);

/* ------------------------------------------------------------------------
 * Sketch-and-precondition least squares (paper Sec. V-E): x = argmin ||Ax - b||
 * for tall A.  The sketch A_hat = S A (d >= n rows, FP32) is widened to FP64
 * and factored by Householder QR, A_hat = Q R; LSQR then solves
 * min ||(A R^{-1}) y - b|| and x = R^{-1} y.  The QR, R^{-1} and every LSQR
 * recurrence run in FP64 on the device.
 * ------------------------------------------------------------------------ */

/* Householder QR of a d x n FP64 matrix (d >= n >= 1, column-major, lda >= d),
 * in place: on return the upper triangle of A holds R and the reflectors sit
 * below the diagonal; R (n x n, upper, zeros below, ldr >= n) is also copied
 * out.  Blocked (compact WY) right-looking factorisation.  ws: device
 * workspace of sk_qr_f64_workspace bytes.  Asynchronous on hip_stream. */
sk_status sk_qr_f64_workspace(int64_t d, int64_t n, size_t* bytes);
sk_status sk_qr_f64(int64_t d, int64_t n, double* A, int64_t lda, double* R, int64_t ldr,
                    void* ws, size_t ws_bytes, void* hip_stream);

/* Rinv = R^{-1} for an n x n upper triangular FP64 R with nonzero diagonal
 * (1 <= n <= 8192; ldr, ldi >= n; device memory).  Asynchronous. */
sk_status sk_trinv_f64(int64_t n, const double* R, int64_t ldr, double* Rinv, int64_t ldi,
                       void* hip_stream);

/* One-sided Jacobi SVD in FP64 (the decomposition of the SVD form of
 * sketch-and-precondition, Sec. V-E-1): G (rows x n, column-major, ld = rows,
 * rows >= n, 1 <= n <= 8192; device) is orthogonalised in place by plane
 * rotations of column pairs in the round-robin parallel order until every
 * pair satisfies |g_p . g_q| <= sqrt(rows) 2^-52 |g_p| |g_q| or holds a
 * column at the rounding floor, |g| <= 2^-52 |G|_F (such a column is noise
 * and its singular value far below any drop threshold); the same rotations
 * accumulate V (n x n, ld = n; device, overwritten).  On return
 * G = U diag(sigma) (columns orthogonal), V orthogonal, the input equals
 * G V^T, and sigma[j] = |g_j| (device, n entries, in column order, not
 * sorted).  *sweeps (host, may be NULL) receives the sweeps run, negated when
 * the iteration stopped at 40 sweeps without converging.  ws: device
 * workspace of sk_svd_f64_workspace bytes.  Synchronises hip_stream
 * (between batches of sweeps). */
sk_status sk_svd_f64_workspace(int64_t rows, int64_t n, size_t* bytes);
sk_status sk_svd_f64(int64_t rows, int64_t n, double* G, double* V, double* sigma,
                     int32_t* sweeps, void* ws, size_t ws_bytes, void* hip_stream);

typedef struct {
  int64_t d;        /* sketch rows, n <= d (the paper uses d = 2n)            */
  int32_t dist;     /* sk_dist of S                                           */
  int32_t prec;     /* sk_prec of the sketch                                  */
  uint64_t seed;
  double atol;      /* LSQR stopping tolerances (Paige-Saunders' atol, btol,  */
  double btol;      /* conlim); conlim <= 0 disables the condition test       */
  double conlim;
  int32_t iter_lim; /* LSQR iteration limit                                   */
  int32_t method;   /* SK_SAP_QR or SK_SAP_SVD                                */
} sk_sap_params;

/* sk_sap_params.method.  SK_SAP_QR: preconditioner R^{-1} from the QR of the
 * sketch (A must have full column rank).  SK_SAP_SVD (Sec. V-E-1, for A with
 * singular values near zero): the sketch's singular values sigma_j and right
 * singular vectors v_j (the QR's R orthogonalised by one-sided Jacobi
 * rotations in FP64), the singular values below sigma_max / 1e12 dropped;
 * preconditioner N = sum over the kept j of v_j e_j^T / sigma_j, and x = N y,
 * so x has no component along the dropped directions (for an exactly
 * rank-deficient A: the minimum-norm least-squares solution).  The SVD form
 * sketches in FP64 (sk_sketch_colwise_f64; prec must be SK_PREC_F32, else
 * SK_EUNSUPPORTED), since an FP32 sketch's rounding leaves singular values
 * near 1e-7 sigma_max where A has none.  It synchronises hip_stream inside
 * sk_sap_begin (between Jacobi sweeps, to stop once a sweep rotates nothing;
 * at most 40 sweeps). */
enum { SK_SAP_QR = 0, SK_SAP_SVD = 1 };

/* Solver info; the first sizeof(sk_sap_info) bytes of an SAP workspace hold it
 * (device memory) from sk_sap_begin on.  istop follows LSQR's codes: 0 running,
 * 1 residual small, 2 normal-equation residual small, 3 condition limit,
 * 4-6 the same at machine precision, 7 iteration limit; and 8: the sketch's
 * device validation rejected A (done is set at once, no iteration runs and x
 * is not meaningful; sk_sap_read_info returns the input error). */
typedef struct {
  int32_t iterations, istop, done, iter_lim;
  double rnorm;   /* ||b - A x|| estimate               */
  double arnorm;  /* ||(A R^{-1})^T r|| estimate        */
  double anorm;   /* ||A R^{-1}||_F estimate            */
  double acond;   /* cond(A R^{-1}) estimate            */
  double xnorm;   /* ||y|| estimate                     */
  double bnorm;
  double test1, test2, test3;
  int32_t rank;   /* columns of the preconditioner kept (n for SK_SAP_QR) */
  int32_t sweeps; /* Jacobi sweeps (SK_SAP_SVD; 0 for SK_SAP_QR)         */
} sk_sap_info;

/* Workspace for one solve (device bytes; includes the sketch's workspace, the
 * FP64 QR, R^{-1} (or, for the SVD form, the Jacobi matrices and N), a
 * row-major copy of A and the LSQR vectors).  The sketch runs with tune NULL,
 * so a plan the measured tuner caches for its shape class afterwards can
 * change the size: query the workspace after tuning. */
sk_status sk_sap_workspace(const sk_csc* A, const sk_sap_params* p, size_t* bytes);

/* Enqueue on hip_stream: sketch, widen, QR, R^{-1} (or the Jacobi SVD and N),
 * the row-major copy of A, and LSQR's start from b (device FP64, m
 * entries). */
sk_status sk_sap_begin(const sk_csc* A, const double* b, const sk_sap_params* p, void* ws,
                       size_t ws_bytes, void* hip_stream);

/* Enqueue `iters` LSQR iterations (each returns at once after the solve has
 * stopped, so extra iterations cost only their launches). */
sk_status sk_sap_iterate(const sk_csc* A, const sk_sap_params* p, int32_t iters, void* ws,
                         size_t ws_bytes, void* hip_stream);

/* Enqueue x = R^{-1} y, or x = N y (x: device FP64, n entries). */
sk_status sk_sap_finish(const sk_csc* A, const sk_sap_params* p, double* x, void* ws,
                        size_t ws_bytes, void* hip_stream);

/* Copy the solver info to the host (synchronises hip_stream); also returns the
 * sketch's validation status (SK_OK or the input error). */
sk_status sk_sap_read_info(const sk_csc* A, const sk_sap_params* p, const void* ws,
                           size_t ws_bytes, void* hip_stream, sk_sap_info* info);

#ifdef __cplusplus
}
#endif
#endif /* SKETCH_H */
