/*
 * lpdec.h -- C ABI of the MI355X (gfx950) adaptive LP decoder.
 *
 * The library decodes binary linear codes by LP decoding (Taghavi, Shokrollahi, Siegel,
 * "Efficient Implementation of Linear Programming Decoding"): minimise gamma^T u over the
 * fundamental polytope of the parity-check matrix H (Sec. II-B, eq. LP decoding), with gamma
 * the channel log-likelihood ratios (eq. def gamma). It runs the modified adaptive LP
 * decoder MALP-A (Algorithm 3) or MALP-B (Sec. III-A), which keeps at most one cut per check
 * (Theorem 3). Each LP is solved by the infeasible primal-dual path-following method of
 * Sec. IV-B; its Newton system (A D^2 A^T) dy = w is solved by preconditioned conjugate
 * gradient (Algorithm 4) with the triangular preconditioner of Sec. V found by the
 * column-wise greedy search (Algorithm 7).
 *
 * Conventions for every call:
 *   - Return value: LPDEC_OK (0) or a negative status; lpdec_last_error() explains the last
 *     failure of a context. A numerical failure of one frame is NOT an API error: it is
 *     reported in that frame's flag (< 0).
 *   - H is given in CSR form: rows = checks (m), columns = variables (n), 0-based, column
 *     indices strictly increasing within a row, no empty row, row degree <= 15, column
 *     degree <= 16, m + n <= 16383. The library copies H; the caller keeps ownership of its arrays.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are GPU memory of the
 *     context's device (for example torch CUDA tensors), owned by the caller.
 *   - Batched layouts are frame-major: element i of frame f of an n-vector is at f*n + i.
 *   - Bit convention: xhat_i = 0 when the decision favours bit 0 (gamma_i >= 0 for the hard
 *     decision, Sec. II-C eq. initial constraints).
 *   - Output flag per frame: 1 = the LP optimum is integral and satisfies every check, so it
 *     is the ML codeword (ML certificate, Sec. II-B); 0 = fractional optimum (pseudocodeword,
 *     decoding failure declared); < 0: LPDEC_FLAG_* numerical failure.
 *   - One context per host thread. Calls on one context are not thread safe; the serving
 *     object has its own lock.
 */
#ifndef LPDEC_H
#define LPDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lpdec_status;
#define LPDEC_OK 0
#define LPDEC_EINVAL (-1)    /* bad argument (sizes, null pointer, malformed H) */
#define LPDEC_ENOMEM (-2)    /* device or host allocation failed */
#define LPDEC_EDEVICE (-3)   /* HIP runtime error */
#define LPDEC_ENOCONV (-4)   /* reserved */
#define LPDEC_EBUSY (-5)     /* serving: result not ready yet */
#define LPDEC_ENOTFOUND (-6) /* serving: unknown ticket */

/* per-frame flags < 0 */
#define LPDEC_FLAG_IPM_CAP (-1)     /* an LP did not meet the IPM termination test in time */
#define LPDEC_FLAG_NONFINITE (-2)   /* non-finite iterate (e.g. NaN/Inf in gamma) */
#define LPDEC_FLAG_MALP_CAP (-3)    /* MALP iteration cap reached with cuts still violated */
#define LPDEC_FLAG_INCONSISTENT (-4)/* integral output that violates a check */
#define LPDEC_FLAG_COST_DECREASE (-5)/* an LP's cost fell below the previous LP's beyond TAU_COST
                                        (impossible in exact arithmetic, Theorem 2b) */
#define LPDEC_FLAG_ALP_CAPACITY (-6) /* ALP only: the LP outgrew the list encoding (a variable in
                                        more than 16 cuts, or more than 16383 - n cuts) */
#define LPDEC_FLAG_CUT_CYCLE (-7)    /* MALP: the cut set of an LP recurred two LPs later (an
                                        optimum that is not unique at the IPM's accuracy, against
                                        the uniqueness Theorem 2 assumes); u, the decisions and
                                        the objective are those of the costlier LP of the two */

typedef struct lpdec_ctx lpdec_ctx;
typedef struct lpdec_code lpdec_code;
typedef struct lpdec_server lpdec_server;

/* Per-frame statistics (all counts summed over the decode). */
typedef struct {
    int32_t malp_iters;   /* LPs solved (MALP iterations with a cut added) */
    int32_t ipm_iters;    /* interior-point iterations, all LPs */
    int32_t pcg_iters;    /* PCG iterations, all Newton solves and refinement rounds */
    int32_t p_max;        /* most cuts in one LP (<= m, Corollary 3) */
    int32_t ref_rounds;   /* iterative-refinement rounds of dy beyond the first solve */
    int32_t mts_rounds;   /* parallel rounds of Algorithm 7, all IPM iterations */
    int32_t max_levels;   /* deepest level schedule of a preconditioner solve */
    int32_t status;       /* 0 or the failing LPDEC_FLAG_* */
    int32_t escalations;  /* Newton solves switched from FP32 to FP64 PCG */
    int32_t direct_solves;/* Newton solves finished by the dense fallback (DIRECT_FALLBACK) */
    int64_t pcg_rows;     /* sum over PCG iterations of the LP's row count p */
    int64_t ipm_cols;     /* sum over IPM iterations of the LP's column count q = n + p */
    int64_t ticks_mts;    /* device clock ticks (100 MHz) in the triangular-set search */
    int64_t ticks_solve;  /* ticks in the Newton solves (PCG, refinement) */
    int64_t ticks_total;  /* ticks of the whole decode of the frame */
    int64_t ticks_pcg;    /* ticks inside PCG iterations (part of ticks_solve) */
    int64_t ticks_dense;  /* ticks in dense-fallback solves (part of ticks_solve) */
    int64_t dense_cube;   /* sum over dense-fallback solves of P^3, P = LP rows padded to 32 */
} lpdec_stats;

/* ---- context ---------------------------------------------------------------------- */
/* Creates a context on HIP device `device`. */
lpdec_status lpdec_ctx_create(int device, lpdec_ctx **out);
lpdec_status lpdec_ctx_destroy(lpdec_ctx *ctx);
/* Text of the last error on this context (never NULL; "" when none). */
const char *lpdec_last_error(const lpdec_ctx *ctx);

/* Options (key, value). Values are converted to the key's type.
 *   MALP_MODE      0 = MALP-A (Algorithm 3), 1 = MALP-B (all inactive cuts removed first)
 *   PRECISION      1 = FP64 PCG vectors (default): the hot path is latency-bound, so FP32
 *                  vectors cost the same per PCG iteration and need several times more
 *                  iterations on the ill-conditioned late Newton systems;
 *                  0 = FP32 PCG vectors with FP64 refinement of dy (a solve whose FP32
 *                  rounds stall continues with FP64 vectors in global memory);
 *                  -1 = the default
 *   TAU_VIOL       a cut is violated when its left-hand side is below 1 - TAU_VIOL (1e-4)
 *   TAU_ACT        a cut is inactive when its slack exceeds max(TAU_ACT, dual slack) (1e-4)
 *   TAU_INT        integrality threshold of the output (1e-4)
 *   IPM_EPS        termination tolerance of the IPM: relative gap, primal and dual residuals (1e-8)
 *   SIGMA          centering factor: mu = SIGMA * x^T z / q (0.1)
 *   ETA            fraction-to-boundary factor of the step lengths (0.9995)
 *   PCG_TOL        PCG stops at ||r|| <= PCG_TOL ||rhs|| (1e-6)
 *   PCG_MAXIT      PCG iteration cap per round; 0 (default) = automatic: with the dense
 *                  fallback, min(2000, max(300, p^2 / 3500)) for an LP of p rows (p^2 / 3500
 *                  is about the PCG iterations that cost as much as two dense solves), else
 *                  500. With the
 *                  fallback on, a round inside the IPM that reaches the cap ends the PCG
 *                  attempt (no refinement rounds after it)
 *   REF_TOL        refinement of dy stops at ||w - Q dy|| <= REF_TOL ||w|| (1e-10)
 *   REF_MAX        refinement rounds after the first solve (3)
 *   IPM_MAX        IPM iteration cap per LP (100)
 *   MALP_MAX       MALP iteration cap (200)
 *   BLOCK          threads per frame (64..256, multiple of 64; 0 = automatic)
 *   PRECOND        1 = triangular preconditioner from Algorithm 7 (column-wise greedy,
 *                  default), 2 = from Algorithm 8 (row-wise greedy, diagonal expansion),
 *                  3 = Algorithm 8 with triangular expansion (the unmatched rows by the
 *                  column-wise greedy over the columns of unmatched rows only), 0 = the slack
 *                  columns as preconditioning set (a diagonal preconditioner), 4 = no
 *                  preconditioner (plain CG on A D^2 A^T in FP64, the baseline of Sec. VI-B),
 *                  5 = from Algorithm 6 (incremental greedy search with the Triangulation Step
 *                  of Algorithm 5; O(q^2) work per search, blocks of columns tested at once)
 *   XI_TOL         inside the IPM a Newton solve is accurate enough once its residual
 *                  perturbs the complementarity equation by at most XI_TOL * mu (0.9)
 *   DIRECT_FALLBACK 1 (default) = a Newton solve whose PCG rounds end without meeting the
 *                  XI_TOL goal is solved again by a dense Cholesky factorisation of
 *                  A D^2 A^T on the GPU (FP64 matrix cores, in the frame's global workspace,
 *                  8 mp^2 bytes per frame, mp = m rounded up to 32), and so are the LP's
 *                  later Newton systems; 0 = keep the PCG result
 *   IPM_STALL      once the largest of the three IPM error measures is below IPM_STALL but
 *                  has not at least halved over the last two iterations, the LP counts as
 *                  solved (the double-precision floor of a degenerate LP) (1e-7)
 *   MTS_REUSE      R >= 1: the preconditioning set is searched on IPM iterations 0, R, 2R, ...
 *                  of each LP and kept in between (1 = every iteration, Sec. V-B; default)
 *   WARM_START     1 = from the second IPM iteration of an LP on, a Newton solve starts from
 *                  the previous direction dy when that leaves a smaller residual than 0
 *                  (Algorithm 4's initial guess); 0 (default) = starts from 0
 *   IPM_WARM       theta >= 0: with theta > 0, every LP after a decode's first starts the
 *                  IPM from the previous LP's x + theta, z + theta (and its y) on the columns
 *                  and cuts the two LPs share, new cuts from x = z = 1, y = 0; 0 (default) =
 *                  every LP starts from x = e, y = 0, z = e
 *   SERVER_STREAMS HIP streams (waves in flight) of a server created afterwards (1..32, 8).
 *                  Streams beyond the process's hardware queues (HIP's GPU_MAX_HW_QUEUES,
 *                  4 unless set before HIP starts) share queues and their waves serialize
 *   SERVER_MODE    scheduling of a server created afterwards. 0 = waves: a stream (of
 *                  SERVER_STREAMS) takes every queued request of the head's code and launches
 *                  one workgroup per frame; a new wave starts when a stream's previous wave
 *                  has ended. 1 (default) = persistent: each code gets an engine, a kernel of up to
 *                  min(max_slots, CUs) workgroups (fewer if the budget is short) that stays
 *                  resident and takes the next request as soon as a workgroup is free; the
 *                  compute units are shared evenly among the engines that have requests, and
 *                  a kernel leaves after about 5 ms in which no request was decoded or waiting
 *                  and is launched again on the next one. An engine holds its
 *                  workspace until the server is destroyed or its budget is needed by another
 *                  code's engine while it has no work. Results are bit-identical to mode 0
 *   TAU_COST       the costs gamma^T u of successive LP solutions increase strictly
 *                  (Theorem 2b); a decrease by more than TAU_COST (1 + c^T x) ends the decode
 *                  with LPDEC_FLAG_COST_DECREASE (1e-8). Every LP solution is put back on
 *                  the box [0, 1]^n (Theorem 2a) before the cut search
 *   DISPATCH_ORDER 1 (default) = a decode batch larger than the device holds at once takes
 *                  its frames hardest-first (see lpdec_decode_batch); 0 = in index order.
 *                  Results do not depend on it
 */
enum {
    LPDEC_OPT_MALP_MODE = 0, LPDEC_OPT_PRECISION, LPDEC_OPT_TAU_VIOL, LPDEC_OPT_TAU_ACT,
    LPDEC_OPT_TAU_INT, LPDEC_OPT_IPM_EPS, LPDEC_OPT_SIGMA, LPDEC_OPT_ETA, LPDEC_OPT_PCG_TOL,
    LPDEC_OPT_PCG_MAXIT, LPDEC_OPT_REF_TOL, LPDEC_OPT_REF_MAX, LPDEC_OPT_IPM_MAX,
    LPDEC_OPT_MALP_MAX, LPDEC_OPT_BLOCK, LPDEC_OPT_PRECOND, LPDEC_OPT_XI_TOL,
    LPDEC_OPT_IPM_STALL, LPDEC_OPT_DIRECT_FALLBACK, LPDEC_OPT_MTS_REUSE, LPDEC_OPT_WARM_START,
    LPDEC_OPT_SERVER_STREAMS, LPDEC_OPT_IPM_WARM, LPDEC_OPT_SERVER_MODE,
    LPDEC_OPT_DISPATCH_ORDER, LPDEC_OPT_TAU_COST, LPDEC_OPT__COUNT
};
lpdec_status lpdec_set_option(lpdec_ctx *ctx, int32_t key, double value);
lpdec_status lpdec_get_option(const lpdec_ctx *ctx, int32_t key, double *value);

/* ---- code --------------------------------------------------------------------------- */
/* Copies and validates H (m checks, n variables; CSR as described above) to the device. */
lpdec_status lpdec_code_create(lpdec_ctx *ctx, int32_t m, int32_t n, const int32_t *h_rowptr,
                               const int32_t *h_col, lpdec_code **out);
lpdec_status lpdec_code_destroy(lpdec_code *code);

/* ---- decoding --------------------------------------------------------------------- */
/* One frame, host pointers, synchronous (the "plain" form: one frame per launch).
 * gamma: host double[n] LLRs. Outputs: xhat host uint8[n]; flag (see above);
 * objective gamma^T u of the LP optimum (nullable); stats (nullable); u host double[n]
 * LP optimum (nullable). */
lpdec_status lpdec_decode(lpdec_ctx *ctx, const lpdec_code *code, const double *gamma,
                          uint8_t *xhat, int32_t *flag, double *objective, lpdec_stats *stats,
                          double *u);

/* A batch of frames, device pointers, asynchronous on `stream` (hipStream_t; NULL = the
 * null stream). gamma_dev: nframes*n values of type gamma_dtype (0 = float32, 1 = float64).
 * Outputs (device): xhat_dev uint8[nframes*n]; flag_dev int32[nframes];
 * obj_dev double[nframes] (nullable); stats_dev lpdec_stats[nframes] (nullable);
 * u_dev double[nframes*n] (nullable). Workspace is owned by the context and reused; a
 * second call on the same context may start only after the first has finished on the
 * device, unless both use the same stream. A batch with more frames than the device holds at
 * once (workgroups per compute unit x compute units) is launched as one resident set of
 * workgroups that take the frames in turn from a counter in the workspace. With
 * DISPATCH_ORDER 1 (default) they take them hardest-first: four small kernels on `stream`
 * first order the frames by descending syndrome weight of their hard decisions. Outputs stay
 * indexed by frame and do not depend on either. */
lpdec_status lpdec_decode_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                const void *gamma_dev, int32_t gamma_dtype, uint8_t *xhat_dev,
                                int32_t *flag_dev, double *obj_dev, lpdec_stats *stats_dev,
                                double *u_dev, void *stream);

/* Same as lpdec_decode_batch, and records the cut set after every MALP iteration:
 * trace_dev uint32[nframes * trace_cap * m], the V bit mask of each check's cut (bit k = k-th
 * variable of the check in ascending order; 0 = no cut), iterations beyond trace_cap are not
 * recorded. Synchronous. */
lpdec_status lpdec_decode_batch_trace(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                      const void *gamma_dev, int32_t gamma_dtype,
                                      uint8_t *xhat_dev, int32_t *flag_dev, double *obj_dev,
                                      lpdec_stats *stats_dev, double *u_dev,
                                      uint32_t *trace_dev, int32_t trace_cap);

/* Same as lpdec_decode_batch, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that forbid allocation): the call allocates nothing. Its
 * workspace is a fixed device region of LPDEC_NOALLOC_SCRATCH_BYTES inside the library, one
 * per device, set up by lpdec_ctx_create and held until the process ends. A batch runs as a
 * resident set of workgroups that take the frames in turn, as many as the region holds
 * arenas for (at most as many as the device holds at once), so any nframes fits; results are
 * bit-identical to lpdec_decode_batch with the same options. Returns LPDEC_EINVAL when one
 * frame's workspace (plus the batch's ordering arrays, 8 bytes per frame) exceeds the region,
 * e.g. the irregular n=8192 code with DIRECT_FALLBACK 1 (its dense system alone is 134 MB).
 * Every call on a device shares that device's region and leaves its contents behind: calls
 * that overlap on one device (on different streams or contexts, or from different host
 * threads) race. */
#define LPDEC_NOALLOC_SCRATCH_BYTES (128u << 20)
lpdec_status lpdec_decode_batch_noalloc(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                        const void *gamma_dev, int32_t gamma_dtype, uint8_t *xhat_dev,
                                        int32_t *flag_dev, double *obj_dev, lpdec_stats *stats_dev,
                                        double *u_dev, void *stream);

/* ALP decoding (Algorithm 1, Sec. II-C) of a batch, for comparison with MALP (Sec. III-D):
 * every violated parity inequality found by Algorithm 2 at the last solution is added and no
 * cut is ever removed, so a check can hold several cuts and an LP has one row per cut. Host
 * pointers, synchronous: gamma double[nframes*n]; outputs xhat uint8[nframes*n], flag
 * int32[nframes] (as lpdec_decode; LPDEC_FLAG_ALP_CAPACITY when the LP outgrows the list
 * encoding), objective double[nframes] (nullable), stats lpdec_stats[nframes] (nullable;
 * malp_iters = LPs solved, p_max = cuts in the largest LP), u double[nframes*n] (nullable).
 * The iterations run in lockstep over the frames still decoding: each runs Algorithm 2 on
 * every check of every such frame in one launch, appends the new cuts on the host, and solves
 * every frame's LP in one interior-point launch in which each frame has its own matrix (a copy
 * of its cut's check row per cut). Uses the context's options (TAU_VIOL, IPM settings,
 * PRECOND, PRECISION, ...). */
lpdec_status lpdec_alp_decode_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                    const double *gamma, uint8_t *xhat, int32_t *flag, double *objective,
                                    lpdec_stats *stats, double *u);

/* ---- steps of the hot path, one frame per workgroup, device pointers, synchronous ----- */
/* Algorithm 2 on every check at the points u_dev (double[nframes*n]):
 * vmask_dev uint32[nframes*m] = V of the check's minimising odd set, viol_dev uint8[nframes*m]
 * = 1 when its left-hand side is below 1 - TAU_VIOL, lhs_dev double[nframes*m] (nullable). */
lpdec_status lpdec_cut_search_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                    const double *u_dev, uint32_t *vmask_dev, uint8_t *viol_dev,
                                    double *lhs_dev);

/* The triangular-set search of the context's PRECOND on the LP whose rows are the checks
 * with hascut_dev[f*m+j] != 0: Algorithm 7 (PRECOND 0, 1 or 4; columns ordered by weight
 * descending, then index ascending), Algorithm 8 with diagonal (PRECOND 2) or triangular
 * (PRECOND 3) expansion (the lowest-indexed row of degree 1 first, columns removed by weight
 * ascending, then index ascending; the triangular expansion then uses Algorithm 7's order), or
 * Algorithm 6 (PRECOND 5; columns tried by weight descending, then index ascending; the
 * Triangulation Step peels in rounds, a column proposed by several rows of degree 1 going to the
 * lowest-indexed one). Column weights w_dev float[nframes*(n+m)] (standard column i at i, slack of
 * check j at n+j). Outputs: pair_dev int32[nframes*m]
 * = column matched to row j (-1 for checks without a cut); lev_b_dev / lev_f_dev
 * int32[nframes*m] = dependency level of row j in the back- and forward-substitution of the
 * preconditioner solve (-1 without a cut); rounds_dev int32[nframes] (nullable) = greedy
 * steps taken (one per LP row, p), or Triangulation Steps run (PRECOND 5). */
lpdec_status lpdec_mts_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                             const uint8_t *hascut_dev, const float *w_dev, int32_t *pair_dev,
                             int32_t *lev_b_dev, int32_t *lev_f_dev, int32_t *rounds_dev);

/* l = (A D^2 A^T) h for the LP of cut set vmask_dev (uint32[nframes*m]) and channel signs of
 * gamma_dev (double[nframes*n]); d2_dev double[nframes*(n+m)]; h_dev, l_dev double[nframes*m]
 * (check space; entries of checks without a cut are ignored / returned as 0). precision:
 * 0 = FP32 arithmetic (inputs rounded to float), 1 = FP64. */
lpdec_status lpdec_normal_matvec_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                       const uint32_t *vmask_dev, const double *gamma_dev,
                                       const double *d2_dev, const double *h_dev, double *l_dev,
                                       int32_t precision);

/* Solves (A D^2 A^T) y = w (check space) by PCG with the Algorithm-7 preconditioner built
 * from float(d2), with the context's PCG_TOL, PCG_MAXIT, REF_TOL, REF_MAX, PRECOND and the
 * given precision (0 = FP32 PCG + FP64 refinement, 1 = FP64). iters_dev int32[nframes]
 * (nullable) = PCG iterations; resid_dev double[nframes] (nullable) = ||w - Q y|| / ||w||
 * in FP64. */
lpdec_status lpdec_newton_solve_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                                      const uint32_t *vmask_dev, const double *gamma_dev,
                                      const double *d2_dev, const double *w_dev, double *y_dev,
                                      int32_t *iters_dev, double *resid_dev, int32_t precision);

/* Solves the LP of cut set vmask_dev by the IPM (Sec. IV-B): x_dev, z_dev
 * double[nframes*(n+m)] (slack of check j at n+j; 0 for checks without a cut), y_dev
 * double[nframes*m], iters_dev int32[nframes], status_dev int32[nframes] (0 converged, else a
 * negative LPDEC_FLAG_*). */
lpdec_status lpdec_ipm_batch(lpdec_ctx *ctx, const lpdec_code *code, int32_t nframes,
                             const uint32_t *vmask_dev, const double *gamma_dev, double *x_dev,
                             double *y_dev, double *z_dev, int32_t *iters_dev,
                             int32_t *status_dev, int32_t precision);

/* ---- serving: continuous batching over mixed codes ------------------------------------ */
/* A server admits frames of any registered code as device memory (hbm_budget_bytes) and
 * slots (max_slots frames in flight) free up, runs them in waves on several streams so that
 * waves overlap on the device, and hands results back by ticket. */
lpdec_status lpdec_server_create(lpdec_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots,
                                 lpdec_server **out);
/* Queues one frame (gamma host double[n], copied). Returns a ticket. */
lpdec_status lpdec_server_submit(lpdec_server *srv, const lpdec_code *code, const double *gamma,
                                 uint64_t *ticket);
/* Collects a result (host outputs, xhat uint8[n]); LPDEC_EBUSY while the frame is queued or
 * running. latency_s = completion time - submission time (host clock). Each ticket can be
 * collected once. */
lpdec_status lpdec_server_poll(lpdec_server *srv, uint64_t ticket, uint8_t *xhat, int32_t *flag,
                               double *objective, double *latency_s);
/* Waits until every submitted frame has finished. */
lpdec_status lpdec_server_drain(lpdec_server *srv);
lpdec_status lpdec_server_destroy(lpdec_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* LPDEC_H */
