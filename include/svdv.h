/*
 * svdv -- singular values of dense matrices on one AMD Instinct MI355X (gfx950).
 *
 * The method is the two-stage QR-based singular-value algorithm whose stage-1
 * kernels the paper auto-tunes (evaluation section, "Algorithm", Algorithm 1
 * and Algorithm 2):
 *   stage 1  dense -> upper band of bandwidth TS (the tile size): for each
 *            diagonal tile k, a QR sweep on the tile column and an LQ sweep on
 *            the tile row, each a panel factorisation followed by a trailing
 *            update that applies the panel's orthogonal factor;
 *   stage 2  band -> upper bidiagonal (bulge chasing);
 *   stage 3  bidiagonal -> singular values.
 * Every transform is orthogonal, so the singular values are those of A.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major with a leading dimension (lda >= max(1, rows)).
 *   A row-major (m, n) array is the column-major (n, m) matrix A^T, which has
 *   the same singular values: pass it as (n, m, lda = n).
 * - Every matrix / vector pointer is a DEVICE pointer unless stated otherwise.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls only
 *   enqueue work and never synchronise the host; a return of SVDV_OK means
 *   "enqueued", results are valid once the caller synchronises the stream.
 *   Faults inside kernels surface as HIP errors at that synchronisation.
 * - The caller owns A and S.  A is never written.  The library owns a
 *   workspace per (device, stream), grown on demand with hipMalloc (the first
 *   call at a new size allocates) and released by svdv_release().  Calls that
 *   overlap on the same stream are ordered by the stream; calls on different
 *   streams use different workspaces.
 * - Errors are negative svdv_status values; the library never aborts and
 *   never throws across this interface.  svdv_last_error() gives detail.
 */
#ifndef SVDV_H
#define SVDV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SVDV_F32 = 0, SVDV_F64 = 1 } svdv_dtype;

typedef enum {
  SVDV_OK = 0,
  SVDV_ERR_INVALID_ARG = -1, /* negative size, lda too small, NULL pointer with nonzero size, bad dtype */
  SVDV_ERR_UNSUPPORTED = -2, /* configuration outside the compiled set or beyond LDS / thread limits */
  SVDV_ERR_NO_MEMORY = -3,   /* workspace allocation failed */
  SVDV_ERR_HIP = -4          /* a HIP runtime call failed (launch, event, graph) */
} svdv_status;

/*
 * Tunable configuration (the auto-tuner's search space; Eq. 1 of the paper
 * picks the argmin over these).
 *   tile         TS = bandwidth of stage 1, in {16, 32, 64, 128}.  It fixes the
 *                number of panel steps (2 * ceil(n / TS)): the paper's only
 *                pipeline parameter.
 *   threads      workgroup size of the stage-1 trailing-update kernel,
 *                {64, 128, 256, 512, 1024}; its waves split the rows of one
 *                panel chunk (the split-K of Algorithm 2).
 *   inner_block  16-column MFMA tiles per workgroup of the trailing update,
 *                {1, 2, 4, 8} (columns per block, register blocking).
 *   sweep_width  bulge-chasing sweeps advanced together by one workgroup in
 *                stage 2, {1, ..., 8}.
 *   update_precision  0 = trailing updates in the input precision;
 *                2 = BF16 MFMA operands, 3 = FP16 MFMA operands (float32 input
 *                only, and configurations whose trailing-update strip fits in
 *                registers; accumulation stays float32, panels with their
 *                float64 norms, stage 2 and stage 3 are unaffected).
 */
typedef struct {
  int32_t tile;
  int32_t threads;
  int32_t inner_block;
  int32_t sweep_width;
  int32_t update_precision;
} svdv_config;

/*
 * Singular values of the m x n matrix A (dtype SVDV_F32 or SVDV_F64), written
 * to S[0 .. min(m,n)-1] in A's dtype, descending and non-negative.
 * m == 0 or n == 0: returns SVDV_OK and writes nothing.
 * An A holding a NaN or an infinity has no singular values: every entry of S
 * is NaN after the stream completes (the staging pass that finds max|a| marks
 * the input, and the stage that writes S reads the mark).
 * The tuned default configuration for (m, n, dtype) is used: the auto-tuner's
 * measured best (Eq. 1's argmin) of the cell of the same dtype nearest to
 * min(m, n) on a log scale, compiled into the library from its tuned table
 * (svdv_default_config returns it).
 */
int svd_values(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream);

/* As svd_values with an explicit configuration (cfg == NULL: tuned default).
 * SVDV_ERR_UNSUPPORTED marks a configuration the auto-tuner must skip. */
int svd_values_ex(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream,
                  const svdv_config* cfg);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): svd_values_ex on a
 * fixed device array of SVDV_NOALLOC_SCRATCH_BYTES bytes that the library holds
 * on every GPU it runs on, from its load until the process ends, instead of the
 * allocated workspace.  Same arguments, kernels and results as svd_values_ex
 * (bitwise, for the same cfg).  This call allocates nothing: no hipMalloc or
 * hipFree, and no per-stage timing events (svdv_timing is ignored for it).
 * A call whose workspace exceeds the array (for example n above about 2048 in
 * float64 or about 2900 in float32 at tile 16) returns SVDV_ERR_UNSUPPORTED
 * before any GPU work.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (each call clears what must start at zero):
 * calls that overlap in time on one GPU (different streams, or host threads)
 * race and must be serialised by the caller.
 */
#define SVDV_NOALLOC_SCRATCH_BYTES (64 << 20)
int svd_values_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream,
                       const svdv_config* cfg);
/* Size in bytes of the fixed array svd_values_noalloc works in. */
int64_t svdv_noalloc_capacity(void);

/*
 * Batched singular values of `batch` independent matrices of uneven sizes.
 *   A_array   HOST array [batch] of device pointers to column-major matrices.
 *   m, n, lda HOST arrays [batch].
 *   S         device buffer; matrix i writes min(m[i], n[i]) values at
 *             S + S_offset[i] elements (S_offset: HOST array [batch]).
 *   cfg       NULL: per-size tuned defaults; otherwise one config for all.
 * A matrix holding a NaN or an infinity gets NaN values; the other matrices
 * of the batch are not affected.
 * The whole batch is one stream-ordered sequence of persistent launches over
 * all matrices at once, captured in a hipGraph and replayed on later calls
 * with the same shapes.
 */
int svd_values_batched(const void* const* A_array, const int64_t* m, const int64_t* n, const int64_t* lda,
                       int64_t batch, int32_t dtype, void* S, const int64_t* S_offset, void* stream,
                       const svdv_config* cfg);

/* The configuration svd_values would use for (m, n, dtype) (HOST out-pointer). */
int svdv_default_config(int64_t m, int64_t n, int32_t dtype, svdv_config* out);

/* SVDV_OK if cfg is runnable for (m, n, dtype), else SVDV_ERR_UNSUPPORTED / SVDV_ERR_INVALID_ARG.
 * Needs no GPU (pure host validation). */
int svdv_check_config(int64_t m, int64_t n, int32_t dtype, const svdv_config* cfg);

/*
 * Per-stage entry points.  They run the same kernels as svd_values (not a
 * second code path) and exist so each stage can be checked on its own.
 *
 * svdv_stage_band: stage 1 (Algorithm 1).  Writes the n' x n' band
 *   (n' = min(m, n)) as float64 into `band`, row i at band + i * ldband,
 *   band[i * ldband + d] = B(i, i + d) for d = 0 .. TS (entries past column
 *   n'-1 are zero).  ldband >= TS + 1.  Values are unscaled (the internal
 *   power-of-two scaling is undone exactly).  An A holding a NaN or an
 *   infinity gives a band of NaN.
 */
int svdv_stage_band(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, double* band, int64_t ldband,
                    void* stream, const svdv_config* cfg);

/*
 * svdv_stage_bidiag: stage 2.  Input: an n x n upper band of bandwidth b in the
 * layout written by svdv_stage_band (float64).  Output: the upper bidiagonal,
 * d[0..n-1] (diagonal) and e[0..n-2] (superdiagonal), float64.  Signs of d, e
 * are not normalised.  cfg->sweep_width selects the schedule; the result is
 * bitwise identical for every sweep_width.  b must be one of the tile sizes.
 * Any finite magnitude is accepted (the band is scaled by a power of two
 * internally, exactly, and d and e scaled back).
 * If the band holds a NaN or an infinity, or a bounded wait between the
 * chase's workgroups gives up (it never does in a correct launch), every entry
 * of d and e is NaN after the stream completes.
 */
int svdv_stage_bidiag(const double* band, int64_t n, int64_t b, int64_t ldband, double* d, double* e, void* stream,
                      const svdv_config* cfg);

/*
 * svdv_stage_values: stage 3.  Singular values of the upper bidiagonal (d, e)
 * (float64, n and n-1 entries), written descending to S in out_dtype.  Each
 * value is located by Sturm-count multisection in float64 to an absolute
 * width of 4u (max|d| + max|e|) for SVDV_F64 output and 2^-32 (max|d| + max|e|)
 * for SVDV_F32 output, then rounded to out_dtype.  Any finite magnitude is
 * accepted (d and e are scaled by a power of two internally, exactly).  If d or
 * e holds a NaN or an infinity, every value is NaN.
 */
int svdv_stage_values(const double* d, const double* e, int64_t n, int32_t out_dtype, void* S, void* stream);

/*
 * svdv_apply_qt: the stage-1 trailing-update kernel on its own (Algorithm 2's
 * operation, in compact-WY form): C <- (I - V T V^T)^T C for side = 0, or
 * C <- C (I - V T V^T) for side = 1.
 *   V  h x k (side 0) or w x k (side 1), column-major, leading dimension ldv,
 *      unit lower trapezoidal as stored (entries above the diagonal must be 0,
 *      the diagonal must be 1: they are read as given).
 *   T  k x k upper triangular, column-major, leading dimension ldt.
 *   C  h x w, column-major, leading dimension ldc, updated in place.
 *   k  <= cfg->tile.  All three in `dtype`.
 *   A reflector length (h for side 0, w for side 1) above 32768 / cfg->tile (the
 *   rows one workgroup can hold in registers) runs the split form when the
 *   configuration has a register strip: partial V^T C over row ranges into the
 *   library's workspace, their sum in a fixed order with T^T applied, then
 *   C - V Z' per block of 32768 / cfg->tile rows (bitwise reproducible from call
 *   to call); else the streaming form of the kernel; a configuration with
 *   neither returns SVDV_ERR_UNSUPPORTED.  Tall panels take float32/float64
 *   updates only.
 */
int svdv_apply_qt(const void* V, int64_t ldv, const void* T, int64_t ldt, void* C, int64_t ldc, int64_t h, int64_t w,
                  int64_t k, int32_t dtype, int32_t side, void* stream, const svdv_config* cfg);

/*
 * Stage timing (instrumentation).  svdv_timing(1) makes every later call on the
 * calling thread record HIP events on its stream around: [0] input staging,
 * [1] stage 1 (all panel and update launches), [2] band packing, [3] the
 * bulge-chase kernel, [4] the bisection kernels.  svdv_last_timing waits for
 * the last call's events and writes up to n elapsed times in milliseconds
 * (HOST array) followed by [5] the whole call and [6] the bulge-chase launch
 * alone; returns the count written.
 * svdv_timing(2) in addition brackets every stage-1 kernel launch with an event
 * pair (for svdv_last_kernel_stats; the extra events lengthen stage 1);
 * svdv_timing(0) switches timing off.
 */
int svdv_timing(int enable);
int svdv_last_timing(double* ms, int n);
/*
 * svdv_last_kernel_stats: per kernel class of the last timed call (kind 0: the
 * stage-1 trailing update, Algorithm 2's operation; kind 1: the stage-1 panel
 * factorisation), writes to the HOST array out[0..3]: number of launches, sum
 * of their event-timed durations in milliseconds, algorithmic flops and
 * algorithmic bytes (trailing update of an r x w block with k reflectors:
 * 4 r w k flops, (2 r w + r k) elements; panel of r x b: 2 r b^2 flops, 2 r b
 * elements).  Requires svdv_timing(2) before the call.  Returns 4, or an error
 * status (n < 4, bad kind, no timed call).
 */
int svdv_last_kernel_stats(int kind, double* out, int n);

/*
 * Learned cost model of the auto-tuner (GPU kernels; the paper's tuning loop,
 * Eq. 1, chooses x* = argmin f(K_x) over measured times -- this model predicts
 * f from a configuration's features so that only the most promising
 * configurations need measuring).
 * A 3-layer perceptron SVDV_MLP_IN -> SVDV_MLP_HIDDEN -> SVDV_MLP_HIDDEN -> 1
 * with ReLU, float32.  params: device vector of SVDV_MLP_NPARAM floats laid out
 * as W1[IN][H] (row-major), b1[H], W2[H][H], b2[H], w3[H], b3.  X: device,
 * n x IN row-major features; t, y: device, n floats.
 *   svdv_mlp_forward   y = model(X).
 *   svdv_mlp_gradient  grad (device, NPARAM floats) = d loss / d params with
 *                      loss = (1/n) sum (model(X) - t)^2, written to *loss
 *                      (device float) when loss is not NULL; work: device
 *                      scratch of svdv_mlp_work_size(n) floats owned by the caller.
 *   svdv_mlp_adam_step one Adam update (step >= 1) of params with moment
 *                      vectors m, v (device, NPARAM floats each, zero at step 1).
 * All run on `stream`, return SVDV_OK or an error status.
 */
#define SVDV_MLP_IN 6
#define SVDV_MLP_HIDDEN 64
#define SVDV_MLP_NPARAM (SVDV_MLP_IN * SVDV_MLP_HIDDEN + SVDV_MLP_HIDDEN + SVDV_MLP_HIDDEN * SVDV_MLP_HIDDEN + \
                         SVDV_MLP_HIDDEN + SVDV_MLP_HIDDEN + 1)
int64_t svdv_mlp_work_size(int64_t n);
int svdv_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream);
int svdv_mlp_gradient(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                      float* work, void* stream);
int svdv_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                       float beta2, float eps, void* stream);

/* Text for a status code (static string). */
const char* svdv_status_string(int status);
/* Detail of the last error on the calling thread (thread-local, static lifetime). */
const char* svdv_last_error(void);
/* Free every cached workspace and graph (synchronises the devices that own them). */
int svdv_release(void);

#ifdef __cplusplus
}
#endif

#endif /* SVDV_H */
