/*
 * opdhg — restarted PDHG with online diagonal preconditioning for linear
 * programs, on AMD Instinct MI355X (gfx950).
 *
 * Method: Lu & Zhang, "Enhanced PDHG for Linear Programming with Online
 * Preconditioning". Each iteration is the PDHG step with adaptive step size
 * and primal weight (Section 3.2, eq. (6)); every phi-th iteration the
 * diagonal preconditioners T and Sigma take one projected online-gradient
 * step with the gradients of eq. (7), optionally normalized (Section 3.2,
 * Algorithm 1), under an AdaGrad schedule (Section 4.1). Restarts keep the
 * preconditioners (Section 3.2).
 *
 * Problem (the paper's standard form, Section 2 eq. (1), widened to mixed
 * row senses and two-sided bounds):
 *
 *     minimize    c^T x + obj_offset
 *     subject to  A_i x  = b_i      for rows with row_sense[i] == 0
 *                 A_i x >= b_i      for rows with row_sense[i] == 1
 *                 l <= x <= u       (l_j may be -INFINITY, u_j +INFINITY)
 *
 * Dual sign convention: the Lagrangian is c^T x - y^T (A x - b) (eq. (2)),
 * so y_i >= 0 on >= rows.
 *
 * Conventions shared by every entry point
 *   - Every function returning int returns 0 on success or a negative
 *     OPDHG_ERR_* code; opdhg_last_error() then describes the failure
 *     (thread-local string, valid until the next call on that thread).
 *   - The solver's outcome (optimal, limits, numerical failure) is a status
 *     in opdhg_result, not an error.
 *   - LP arrays are host pointers borrowed for the duration of the call;
 *     the library copies, rescales and uploads them.
 *   - Device memory is never allocated by the library. The caller passes a
 *     workspace (device pointer + size) that must hold at least the bytes
 *     opdhg_workspace_bytes() reports; it must stay valid and untouched
 *     until the call (or session / server) that uses it is finished.
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream. All device work of a call is ordered on the given stream.
 *   - Output vectors are host arrays owned by the caller, always FP64 and
 *     in the unscaled space, even when the solver computes in FP32.
 *   - Calls with distinct workspaces may run concurrently from different
 *     threads. A session or server handle is used by one thread at a time
 *     (a server is internally synchronized).
 */
#ifndef OPDHG_H
#define OPDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (negative return values) ---- */
#define OPDHG_OK 0
#define OPDHG_ERR_INVALID_ARGUMENT (-1)
#define OPDHG_ERR_WORKSPACE_TOO_SMALL (-2)
#define OPDHG_ERR_OVER_BUDGET (-3)
#define OPDHG_ERR_DEVICE (-4)
#define OPDHG_ERR_NOT_READY (-5)
#define OPDHG_ERR_CANCELLED (-6)
#define OPDHG_ERR_UNKNOWN_TICKET (-7)

/* ---- solver status (opdhg_result.status) ---- */
#define OPDHG_STATUS_OPTIMAL 0          /* relative KKT error <= tol */
#define OPDHG_STATUS_ITERATION_LIMIT 1  /* max_iter accepted iterations */
#define OPDHG_STATUS_TIME_LIMIT 2       /* time_limit_s of wall time */
#define OPDHG_STATUS_NUMERICAL_ERROR 3  /* non-finite reductions or too many step rejections;
                                           the current iterate is returned with its KKT error */
#define OPDHG_STATUS_RUNNING 4          /* sessions only: paused before finishing */

/* ---- precision ---- */
#define OPDHG_FP64 0 /* everything in FP64 */
#define OPDHG_FP32 1 /* A, vectors and SpMV in FP32; reductions, step sizes, KKT in FP64 */

/* ---- online learning-rate schedule (Section 4.1 names AdaGrad) ---- */
#define OPDHG_SCHEDULE_ADAGRAD_DIAG 0 /* per coordinate: H += G^2, P -= lr G / sqrt(H) */
#define OPDHG_SCHEDULE_ADAGRAD_NORM 1 /* scalar: H += |G|^2, P -= lr G / sqrt(H) */
#define OPDHG_SCHEDULE_CONSTANT 2     /* plain OGD: P -= lr G */

/* ---- step-size rule ---- */
#define OPDHG_STEP_ADAPTIVE 0 /* PDLP's adaptive rule (the paper runs on top of cuPDLP.jl, Section 4.3) */
#define OPDHG_STEP_CONSTANT 1 /* vanilla PDHG (Sections 2 and 4.2): eta = step_scale / |A~|_2 estimate,
                                 every attempt accepted */

/* ---- norms of the adaptive step rule's movement term ---- */
#define OPDHG_STEP_NORM_PLAIN 0   /* 0.5 omega |dx|^2 + 0.5 |dy|^2 / omega */
#define OPDHG_STEP_NORM_PRECOND 1 /* |dx|^2_{T^-1} and |dy|^2_{Sigma^-1}: the norms of the
                                     preconditioned step (eq. (6)); equal to PLAIN at T = Sigma = I */

/* ---- windowed sparse products (FP32) ---- */
#define OPDHG_WINDOWS_AUTO 0   /* a side whose rows give at least 128 windowed chunks uses them */
#define OPDHG_WINDOWS_OFF 1    /* every row in tiles that gather from global memory */
#define OPDHG_WINDOWS_ALWAYS 2 /* every windowable chunk, however few (small LPs, checks) */

/* ---- where the rescaling and the scaled data are computed ---- */
#define OPDHG_PREP_AUTO 0   /* on the device for LPs of 2^20 nonzeros or more, else on the host;
                               a packed set whose nonzeros reach 2^20 in total is prepared on
                               the device when that matches the host bit for bit (pc_beta 1 or
                               < 0) */
#define OPDHG_PREP_HOST 1   /* host threads (FP64) */
#define OPDHG_PREP_DEVICE 2 /* device kernels (FP64), same results (with OPDHG_STEP_CONSTANT the
                               power iteration runs on the device too) */

/* ---- restart scheme ---- */
#define OPDHG_RESTART_ADAPTIVE 0 /* PDLP's KKT-based restarts, preconditioners kept (Section 3.2) */
#define OPDHG_RESTART_NONE 1     /* vanilla PDHG (Section 4.2): evaluations test termination only;
                                    the primal weight keeps its initial value */

/* LP in CSR form; all pointers are host pointers. */
typedef struct opdhg_lp {
  int64_t m;                /* rows (>= 0) */
  int64_t n;                /* columns (>= 1) */
  int64_t nnz;              /* stored entries, < 2^31 */
  const int64_t* row_ptr;   /* m + 1 offsets, row_ptr[0] = 0, nondecreasing, row_ptr[m] = nnz */
  const int32_t* col_idx;   /* nnz column indices in [0, n); no (row, col) twice */
  const double* val;        /* nnz finite values */
  const double* b;          /* m finite right-hand sides */
  const int8_t* row_sense;  /* m senses: 0 '=', 1 '>=' */
  const double* c;          /* n finite costs */
  const double* l;          /* n lower bounds, < +inf (may be -INFINITY) */
  const double* u;          /* n upper bounds, > -inf, >= l (may be +INFINITY) */
  double obj_offset;        /* constant added to both objectives */
} opdhg_lp;

/* Solver parameters. Fill with opdhg_default_params() and override. */
typedef struct opdhg_params {
  double tol;            /* relative KKT tolerance (Section 4.1: 1e-4) */
  int64_t max_iter;      /* accepted-iteration limit */
  double time_limit_s;   /* wall-clock limit of the iteration loop */
  int32_t precision;     /* OPDHG_FP64 or OPDHG_FP32 */
  int32_t schedule;      /* OPDHG_SCHEDULE_* */
  double lr;             /* online learning rate alpha; 0 gives plain PDLP */
  int32_t phi;           /* preconditioner update period (Section 3.2; 20 or 1) */
  int32_t normalize;     /* 1: normalized online loss (Section 3.2) */
  double precond_floor;  /* projection of T, Sigma onto diagonals >= floor */
  int32_t ruiz_iters;    /* Ruiz infinity-norm passes (Section 2) */
  double pc_beta;        /* Pock-Chambolle exponent (Section 2); < 0 skips the pass */
  int32_t eval_every;    /* accepted iterations between KKT evaluations */
  int32_t max_step_retries; /* rejections allowed per iteration */
  double beta_suff;      /* restart on sufficient KKT decay */
  double beta_nec;       /* restart on necessary decay without progress */
  double beta_art;       /* artificial restart when t >= beta_art * k */
  double pw_smoothing;   /* primal-weight smoothing at restarts */
  double step_growth;    /* exponent of the step growth factor */
  double step_reduction; /* exponent of the step reduction factor */
  int32_t tile_nnz;      /* SpMV tile target in nonzeros; 0 picks automatically */
  int32_t lanes;         /* lanes per row in SpMV tiles; 0 picks per tile */
  int32_t workgroups;    /* workgroups per sparse-product launch; 0 picks automatically */
  int32_t step_rule;     /* OPDHG_STEP_* */
  int32_t restart_scheme; /* OPDHG_RESTART_* */
  int32_t l2_rescale;    /* 1: one L2-norm pass after the Ruiz passes (Section 4.2) */
  int32_t power_iters;   /* constant step: power-iteration rounds at most (>= 1) */
  double step_scale;     /* constant step: eta = step_scale / estimate of |A~|_2 (> 0) */
  double power_tol;      /* power iteration stops when |A~|_2^2 moves less than this, relatively */
  int32_t step_norm;     /* OPDHG_STEP_NORM_*: norms of the adaptive rule's movement term */
  int32_t windows;       /* OPDHG_WINDOWS_*: FP32 only; FP64 and the server never use windows */
  int32_t window_buckets; /* LDS window per pass in buckets of 1024 entries, 1..28, for chunks
                             of one pass and of several alike; 0: 28 per pass, and up to 38 for a
                             chunk of one pass (its row sums then reuse the window's LDS) */
  int32_t window_rows;   /* rows per windowed chunk, 1..10240; 0: picked from the side's size */
  int32_t prep;          /* OPDHG_PREP_*: rescaling passes and scaled data on the host or device */
  int32_t eval_slots;    /* attempt slots between the guarded evaluation steps inside a launch
                            sequence (an LP that becomes due mid-sequence waits at most this
                            many slots); 0: automatic; < 0: none (only the evaluation that opens
                            each sequence). Results do not depend on it. */
} opdhg_params;

typedef struct opdhg_result {
  int32_t status;        /* OPDHG_STATUS_* */
  int32_t which;         /* 0: current iterate returned, 1: step-weighted average */
  int64_t iterations;    /* accepted iterations */
  int64_t attempts;      /* step attempts including rejected ones */
  int64_t restarts;
  double primal_obj;     /* c^T x + obj_offset */
  double dual_obj;
  double rel_primal;     /* |b - Ax|_violated / (1 + |b|) */
  double rel_dual;       /* |reduced-cost residual| / (1 + |c|) */
  double rel_gap;        /* |p - d| / (1 + |p| + |d|) */
  double rel_kkt;        /* max of the three */
  double solve_seconds;  /* wall time of the iteration loop */
  double eta;            /* final step size */
  double omega;          /* final primal weight */
} opdhg_result;

/* Scaled-space state of a session, for tracing and checkpoints. */
typedef struct opdhg_state {
  int64_t k;          /* accepted iterations */
  int64_t t;          /* accepted iterations since the last restart */
  int64_t attempts;
  int64_t restarts;
  int32_t status;
  int32_t need_eval;  /* an evaluation is due before the next step */
  double eta;
  double omega;
  double w;           /* sum of accepted step sizes in this restart period */
} opdhg_state;

typedef struct opdhg_session opdhg_session;
typedef struct opdhg_server opdhg_server;

/* Defaults: tol 1e-4, max_iter 100000, time limit 600 s, FP64, AdaGrad
 * (diagonal), lr 0, phi 20, normalize 1, floor 0, 10 Ruiz passes, no L2
 * pass, Pock-Chambolle beta 1, eval every 64, 60 step retries, adaptive
 * steps and restarts, restart constants 0.2 / 0.8 / 0.36, smoothing 0.5,
 * step exponents 0.6 / 0.3, plain step norms, automatic tiling and
 * windows; for the constant step:
 * step_scale 0.9, at most 200 power-iteration rounds, power_tol 1e-7.
 *
 * The vanilla PDHG runs of Section 4.2 take OPDHG_STEP_CONSTANT,
 * OPDHG_RESTART_NONE, l2_rescale 1, pc_beta -1, normalize 1, phi 1 and
 * max_iter 50000. */
void opdhg_default_params(opdhg_params* p);

/* Check an LP without touching the device. Returns OPDHG_ERR_INVALID_ARGUMENT
 * (with a message) unless: n >= 1, m >= 0, nnz < 2^31; row_ptr starts at 0,
 * never decreases and ends at nnz; columns in [0, n) without duplicates in a
 * row; A, b, c finite; l < +inf, u > -inf, l <= u (no NaN); senses 0 or 1. */
int opdhg_validate(const opdhg_lp* lp);

/* Exact device bytes one LP needs under these parameters (a pure function of
 * the LP's sparsity pattern and the parameters: the tiling, the windowed
 * chunks planned from the pattern in FP32, and, with device-side
 * preparation, the unscaled values' staging). Host only. */
int opdhg_workspace_bytes(const opdhg_lp* lp, const opdhg_params* p, size_t* bytes);

/* Host-only rescaling, exposed for checking: the Ruiz passes, the optional
 * L2 pass and the Pock-Chambolle pass of Section 2 as applied before the
 * iteration (the device-side preparation gives the same bits for
 * pc_beta 1 or < 0; for other exponents it agrees to rounding).
 * Outputs (caller-allocated host arrays): scaled_val[nnz] in the order of
 * lp->val, d_row[m], d_col[n] with A~ = diag(d_row) A diag(d_col). */
int opdhg_rescale(const opdhg_lp* lp, const opdhg_params* p, double* scaled_val,
                  double* d_row, double* d_col);

/* Host-only estimate of |A~|_2 for the rescaled matrix A~ (rescaling as in
 * opdhg_rescale, with the parameters' passes), exposed for checking: power
 * iteration on A~^T A~ from the normalized all-ones vector, lam = |A~^T A~ v|
 * and v = A~^T A~ v / lam per round, stopping after p->power_iters rounds or
 * when lam changes by at most p->power_tol * lam; *norm_out = sqrt(lam), 0
 * when A~ v vanishes. The constant step (Section 2: tau sigma |A|_2^2 < 1)
 * is eta = p->step_scale / *norm_out. Sums are double-double, so the result
 * does not depend on the thread count. */
int opdhg_spectral_norm(const opdhg_lp* lp, const opdhg_params* p, double* norm_out);

/* Solve one LP (blocking). x_out[n], y_out[m] receive the returned iterate
 * (unscaled); res receives status and statistics. In FP64 the result does
 * not depend on the tiling, the windows or the preparation side (exact
 * sums); in FP32 the row sums of windowed chunks and of tiles are formed in
 * different orders and the partial sums of each tile are plain FP64, so the
 * FP32 result moves with the tile sizes and the windows by rounding only. In
 * both precisions it does not depend on the workgroup count and is the
 * same on every run. */
int opdhg_solve(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                size_t workspace_bytes, void* hip_stream, double* x_out, double* y_out,
                opdhg_result* res);

/* Bytes for a batch: sum of per-LP needs plus the batch tables. */
int opdhg_batch_workspace_bytes(int count, const opdhg_lp* lps, const opdhg_params* p,
                                size_t* bytes);

/* Solve count independent LPs packed into one set of launches: each kernel
 * covers the tiles of every still-running LP, each LP keeps its own step
 * size, restarts and termination, and finished LPs drop out without a new
 * launch configuration. Each LP's arithmetic does not depend on the others,
 * so its result equals its solo solve bit for bit. x_out[i] / y_out[i] are
 * host arrays of lps[i].n / lps[i].m doubles. */
int opdhg_solve_batch(int count, const opdhg_lp* lps, const opdhg_params* p,
                      void* d_workspace, size_t workspace_bytes, void* hip_stream,
                      double* const* x_out, double* const* y_out, opdhg_result* res);

/* The same packed solve in two calls, so that the set is prepared once:
 * opdhg_batch_prepare validates and prepares the LPs (structure, tiling,
 * windows, and their scaled data when the host prepares them) and sizes
 * the workspace exactly (opdhg_batch_bytes), where
 * opdhg_batch_workspace_bytes followed by opdhg_solve_batch prepares each
 * LP twice. The LPs' arrays are borrowed: they must stay valid and
 * unchanged until opdhg_batch_solve returns. opdhg_batch_solve runs once
 * per handle (OPDHG_ERR_INVALID_ARGUMENT after that); its results equal
 * opdhg_solve_batch's bit for bit. opdhg_batch_destroy frees the handle
 * (NULL is ignored). */
typedef struct opdhg_batch opdhg_batch;
int opdhg_batch_prepare(int count, const opdhg_lp* lps, const opdhg_params* p,
                        opdhg_batch** out);
int opdhg_batch_bytes(const opdhg_batch* b, size_t* bytes);
int opdhg_batch_solve(opdhg_batch* b, void* d_workspace, size_t workspace_bytes,
                      void* hip_stream, double* const* x_out, double* const* y_out,
                      opdhg_result* res);
void opdhg_batch_destroy(opdhg_batch* b);

/* ---- allocation-free solve ----
 * For callers that cannot allocate device memory or let a library create
 * HIP objects: tight serving loops that must not call hipMalloc, harnesses
 * that forbid allocation. opdhg_solve_noalloc is opdhg_solve with the
 * library's own static device scratch of OPDHG_NOALLOC_SCRATCH_BYTES as its
 * workspace. It allocates no device or pinned host memory and creates no
 * stream, event or graph: its kernels are launched directly on hip_stream
 * (which must belong to the current device), and it synchronizes that
 * stream, so it cannot itself be captured into a graph. Results equal
 * opdhg_solve's with the same parameters bit for bit.
 *   - The scratch is a file-scope device array: every device the library is
 *     loaded on holds its own copy until the process ends. Its address is
 *     looked up on the first call on each device.
 *   - Every call uploads its LP image and launch tables over the part of
 *     the scratch it uses before any kernel reads it, so nothing of an
 *     earlier call (which the scratch keeps) is read.
 *   - Calls on one device share its scratch: calls from several threads of
 *     one process run one at a time (a per-device lock); calls that overlap
 *     on one device any other way would race.
 *   - An LP needing more than the scratch holds (opdhg_workspace_bytes)
 *     returns OPDHG_ERR_WORKSPACE_TOO_SMALL with a message; nothing runs. */
#define OPDHG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int opdhg_solve_noalloc(const opdhg_lp* lp, const opdhg_params* p, void* hip_stream,
                        double* x_out, double* y_out, opdhg_result* res);

/* ---- autotuning of the sparse-product tiling ----
 * Not part of the method: a performance helper. The LPs are prepared once;
 * each candidate tiling (tile size in nonzeros x workgroups per launch,
 * lanes per row picked per tile) is uploaded, captured and timed over
 * `replays` launch sequences (64 step attempts each) with the LPs kept
 * running. In FP32 with automatic windows, the best tiling is timed once
 * more with windowed chunks of up to 10240 rows (7168 on the A^T side)
 * wherever they stage at most half of their matrix bytes
 * (OPDHG_WINDOWS_ALWAYS): LDS-staged
 * gathers instead of one gather per nonzero from global memory. The
 * fastest candidate by step attempts per second, summed over the set, is
 * returned; pass its fields as tile_nnz, lanes, workgroups, windows and
 * window_rows of opdhg_params (each LP then equals its solo solve with the
 * same parameters bit for bit). In FP64 every tiling gives identical
 * results; in FP32 results move only by rounding. The workspace is
 * overwritten. */
typedef struct opdhg_tuning {
  int32_t tile_nnz;       /* chosen tile size (nonzeros) */
  int32_t lanes;          /* chosen lanes per row (0: per tile) */
  int32_t workgroups;     /* chosen workgroups per launch */
  int32_t candidates;     /* candidates timed */
  double attempts_per_s;  /* measured for the chosen tiling */
  double default_attempts_per_s; /* measured for the automatic tiling */
  double executed_fraction; /* chosen tiling: attempts run / step-attempt slots launched (the
                               slots an LP leaves idle while an evaluation is due) */
  int32_t windows;        /* chosen OPDHG_WINDOWS_* (the parameters' own unless windows won) */
  int32_t window_rows;    /* chosen window_rows */
} opdhg_tuning;

/* Workspace bytes opdhg_autotune needs for these LPs (the largest
 * candidate's). Host only. */
int opdhg_autotune_workspace_bytes(int count, const opdhg_lp* lps, const opdhg_params* p,
                                   size_t* bytes);
int opdhg_autotune(int count, const opdhg_lp* lps, const opdhg_params* p, void* d_workspace,
                   size_t workspace_bytes, void* hip_stream, int replays, opdhg_tuning* out);

/* ---- sessions: step an LP under host control (tracing, checkpoints) ---- */

int opdhg_session_create(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                         size_t workspace_bytes, void* hip_stream, opdhg_session** out);

/* A session in two calls, so that the LP is prepared once: opdhg_prepare
 * validates and prepares it (structure, tiling, windows, and its scaled
 * data when the host prepares it) and sizes the workspace exactly
 * (opdhg_prepared_bytes), where opdhg_workspace_bytes followed by
 * opdhg_session_create prepares the LP twice. opdhg_session_create_prepared
 * then creates the session as opdhg_session_create does (same results bit
 * for bit); it takes the prepared data, so it runs once per handle
 * (OPDHG_ERR_INVALID_ARGUMENT after that). The LP's arrays are borrowed:
 * they must stay valid and unchanged until the session is created.
 * opdhg_prepared_destroy frees the handle (NULL is ignored). */
typedef struct opdhg_prepared opdhg_prepared;
int opdhg_prepare(const opdhg_lp* lp, const opdhg_params* p, opdhg_prepared** out);
int opdhg_prepared_bytes(const opdhg_prepared* pr, size_t* bytes);
int opdhg_session_create_prepared(opdhg_prepared* pr, void* d_workspace, size_t workspace_bytes,
                                  void* hip_stream, opdhg_session** out);
void opdhg_prepared_destroy(opdhg_prepared* pr);

/* Run until k >= k_target accepted iterations or the solve finishes
 * (k_target < 0: until it finishes). An evaluation due at k_target is left
 * for the next call, so a paused state is the state after k_target
 * iterations and before the evaluation at the top of the next one. */
int opdhg_session_run(opdhg_session* s, int64_t k_target);
/* Enqueue exactly `replays` launch sequences (one evaluation step plus
 * min(eval_every, 64) attempts each) on the session's stream and wait for them,
 * without reading the state in between; limits and termination still
 * apply on the device (finished LPs make the remaining launches no-ops).
 * For timing the iteration at a fixed amount of work. */
int opdhg_session_replay(opdhg_session* s, int replays);
/* Scaled-space iterate and preconditioners (FP64 host arrays; any pointer
 * may be NULL to skip that vector): x[n], y[m], T[n], Sigma[m]. */
int opdhg_session_state(opdhg_session* s, double* x, double* y, double* T, double* Sigma,
                        opdhg_state* st);
/* Unscaled returned iterate and result of a finished (or paused) session. */
int opdhg_session_result(opdhg_session* s, double* x_out, double* y_out, opdhg_result* res);
/* Average device time of one launch of the primal kernel (CSR(A^T) SpMV
 * fused with the primal step) over reps launches, timed with HIP events on
 * the session's stream. The kernel only rewrites the candidate buffers, so
 * the session state is unchanged. */
int opdhg_session_time_primal_kernel(opdhg_session* s, int reps, double* avg_ms);
/* Average device times of one launch of the primal kernel and of the dual
 * kernel (CSR(A) SpMV of the candidate x fused with the dual step), each
 * over reps back-to-back launches timed with HIP events on the session's
 * stream. Timing launches write only the candidate buffers (no
 * preconditioner update, no online gradient), so the state is unchanged. */
int opdhg_session_time_kernels(opdhg_session* s, int reps, double* primal_ms, double* dual_ms);
void opdhg_session_destroy(opdhg_session* s);

/* ---- serving: continuous batching under a device-memory budget ---- */

typedef struct opdhg_server_cfg {
  size_t budget_bytes;   /* admission budget for resident LPs; capped at what the arena
                            holds after the launch tables */
  int32_t max_active;    /* at most this many LPs on the device at once (1..65535) */
  int32_t attempts_per_replay; /* step attempts per launch sequence (1..64); each sequence
                                  starts with the due KKT evaluations, admissions and
                                  retirements happen between sequences */
  int32_t precision;     /* OPDHG_FP64 or OPDHG_FP32; every request must use it */
  int32_t workgroups;    /* workgroups of the sparse-product launches; 0: automatic */
  int32_t prep_threads;  /* host threads preparing submitted LPs; 0: automatic */
  int32_t fallback;      /* OPDHG_FALLBACK_*: what happens to an FP32 request that ends
                            without reaching its tolerance */
  double poll_interval_s; /* idle wait of the scheduler thread */
} opdhg_server_cfg;

/* Server fallback. FP32 stores A, the iterates and the gathered vectors in
 * single precision; on an LP that needs a tiny primal weight, the rounding
 * of the gathered y, multiplied by the primal step eta / omega, can stop
 * progress (the iterate moves by noise and the restarts keep lowering
 * omega). With OPDHG_FALLBACK_FP64 a request whose FP32 solve ends with
 * OPDHG_STATUS_ITERATION_LIMIT or OPDHG_STATUS_NUMERICAL_ERROR is solved
 * again from the start in FP64, with the same parameters, by a host thread
 * of the server on a stream of its own (default priority), in arena memory
 * taken like an admission; its result replaces the FP32 one, and
 * opdhg_server_precision reports it. The server keeps each request's copy of
 * the LP until the request is done. No fallback for a request that hit its
 * time limit, was cancelled, or whose FP64 workspace exceeds the budget
 * (the FP32 result is delivered). Ignored when the server runs FP64. */
#define OPDHG_FALLBACK_NONE 0
#define OPDHG_FALLBACK_FP64 1

/* Defaults: budget = whole arena, 256 active LPs, 64 attempts per sequence,
 * FP32, automatic workgroups and preparation threads, no fallback, 1 ms
 * idle wait. */
void opdhg_server_default_cfg(opdhg_server_cfg* cfg);

typedef struct opdhg_server_stats {
  int64_t submitted;
  int64_t completed;
  int64_t cancelled;
  int64_t failed;
  int64_t active;        /* LPs resident on the device */
  int64_t queued;        /* waiting for memory or a slot */
  int64_t replays;       /* launch sequences issued */
  size_t bytes_in_use;   /* arena bytes held by resident LPs */
  size_t peak_bytes;
  int64_t fallbacks;     /* requests solved again in FP64 (OPDHG_FALLBACK_FP64) */
} opdhg_server_stats;

/* Create a server over a caller-owned device arena (the launch tables take
 * the first arena_bytes / 64 bytes, clamped to [4 MiB, 1 GiB]; the LPs share
 * the rest up to budget_bytes). Three streams: compute, host-to-device
 * uploads and device-to-host downloads; a NULL upload or download stream
 * uses the compute stream. The server runs host threads of its own:
 * workers prepare submitted LPs (validation, rescaling, tiling), taking
 * them in submission order, and a scheduler admits prepared LPs in
 * submission order as memory and slots free up,
 * uploads them while the resident LPs iterate, launches the shared launch
 * sequence, and retires finished LPs. An LP's arithmetic does not depend
 * on what else is resident, so each result equals its solo solve with the
 * same parameters bit for bit. Returns NULL on failure (see
 * opdhg_last_error). */
opdhg_server* opdhg_server_create(const opdhg_server_cfg* cfg, void* d_arena,
                                  size_t arena_bytes, void* compute_stream,
                                  void* h2d_stream, void* d2h_stream);
/* Queue an LP (copied at submit). Admitted FIFO as memory and slots free
 * up; OPDHG_ERR_OVER_BUDGET if it can never fit the budget. */
int opdhg_server_submit(opdhg_server* s, const opdhg_lp* lp, const opdhg_params* p,
                        uint64_t* ticket);
/* OPDHG_ERR_NOT_READY until the ticket's solve is done; then fills the
 * outputs (unscaled x[n], y[m], result) and releases the ticket. */
int opdhg_server_poll(opdhg_server* s, uint64_t ticket, double* x, double* y,
                      opdhg_result* res);
/* Block until the ticket is done (or timeout_s passes: OPDHG_ERR_NOT_READY). */
int opdhg_server_wait(opdhg_server* s, uint64_t ticket, double timeout_s, double* x,
                      double* y, opdhg_result* res);
int opdhg_server_cancel(opdhg_server* s, uint64_t ticket);
int opdhg_server_get_stats(opdhg_server* s, opdhg_server_stats* out);
/* Latency of the ticket: submit time to result-on-host, in seconds (valid
 * after poll returned the result). */
int opdhg_server_latency(opdhg_server* s, uint64_t ticket, double* seconds);
/* Precision of the solve that produced the ticket's result: the server's,
 * or OPDHG_FP64 after a fallback (valid after poll returned the result). */
int opdhg_server_precision(opdhg_server* s, uint64_t ticket, int32_t* precision);
void opdhg_server_destroy(opdhg_server* s);

const char* opdhg_last_error(void);
const char* opdhg_status_name(int status);
/* Library version and the GPU architecture it was built for. */
const char* opdhg_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* OPDHG_H */
