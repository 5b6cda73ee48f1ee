/*
 * mam.h -- C ABI of the MI355X (gfx950) Method of Averaged Marginals library.
 *
 * MAM (Mimouni, Malisani, Zhu, de Oliveira, arXiv 2309.05315) computes a
 * fixed-support Wasserstein barycenter, balanced or unbalanced, by running
 * the Douglas-Rachford iteration of Alg. 1 on the M transport plans
 * theta^(m) in R^{R x S^m}.  One iteration (Alg. 1, Steps 1-3) is
 *
 *   p      = sum_m a_m p^(m),  a_m = (1/S^m) / sum_j (1/S^j)      (Prop. 2, eq. (pr))
 *   t      = 1 if rho*d <= gamma, else gamma/(rho*d),
 *            d = sqrt(sum_m ||p - p^(m)||^2 / S^m)                (Alg. 1, t^k rule)
 *   b^(m)  = t (p - p^(m)) / S^m                                  (Prop. 2, eq. (row_sol))
 *   per column s of measure m:
 *     w      = theta_{:,s} + 2 b^(m) - c_{:,s} / rho
 *     pi_hat = Proj_{Delta_R(q_s)}(w)                             (Prop. 3, eq. (proj-s))
 *     theta_{:,s} <- pi_hat - b^(m)
 *   p^(m)  = row sums of the new theta^(m)                        (Alg. 1, Step 3)
 *
 * and the barycenter is p-bar = sum_m a_m p^(m) of the current plans.
 *
 * Conventions shared by every call:
 *
 *  * Status: every call returns mam_status; 0 (MAM_OK) is success, negative
 *    values are errors.  mam_last_error() returns a message for the last
 *    failure on the calling thread.  No C++ exception crosses this ABI.  A
 *    failed mam_create leaves nothing allocated.
 *  * Memory: every device buffer is owned by the caller and must stay valid
 *    while a handle uses it.  The library allocates no device memory: its
 *    scratch state lives in a caller-provided workspace whose size
 *    mam_workspace_bytes() reports.  The library owns only the host handle.
 *  * Layout: plans are stored column-major.  Global column j = off_m + s
 *    (off_m = S^1 + ... + S^(m-1)) starts at element j*ld of theta, and its R
 *    entries are contiguous; rows R..ld-1 are padding that is never written.
 *    theta holds T*ld elements, T = sum_m S^m.  Cost columns follow the same
 *    rule with cost_ld.  q (length T) holds every q^(m) concatenated.
 *    Element type of theta, cost and q: float (MAM_F32) or double (MAM_F64).
 *    Marginals, barycenter and thresholds are always double.
 *  * Streams: 'stream' is a hipStream_t passed as void* (NULL = default
 *    stream).  Work is enqueued on it in order and returns at once, except
 *    where a call says it synchronizes.
 *  * Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef MAM_H
#define MAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mam_status;

#define MAM_OK             0
#define MAM_EINVAL        -1  /* invalid argument or size */
#define MAM_ENOMEM        -2  /* workspace missing or too small */
#define MAM_EHIP          -3  /* a HIP runtime call failed */
#define MAM_ENOTBALANCED  -4  /* balanced mode (gamma = inf) with unequal masses */
#define MAM_ENONFINITE    -5  /* a NaN/Inf or negative weight in the inputs or state */
#define MAM_EUNSUPPORTED  -6  /* a size or feature outside what the path taken
                                  provides: R > 2^28 or M > 65535 (mam_create),
                                  R > 8192 inside a batch, a schedule no kernel
                                  instance covers, reverse mode or bundles on
                                  long columns (R > 8192), the theta stopping
                                  test with MAM_FLAG_SPARSE_STORE */
#define MAM_ESTATE        -7  /* call out of order (e.g. iterate before init) */

#define MAM_F32 0
#define MAM_F64 1

/* Cost layout (mam_desc.cost_mode). */
#define MAM_COST_PER_COLUMN 0  /* cost column j for plan column j (R x T) */
#define MAM_COST_SHARED     1  /* one R x S cost for every measure: column s of
                                  measure m uses cost column s (all S^m <= cost_ncols) */
#define MAM_COST_INDEXED    2  /* plan column j uses cost column cost_col_index[j] */
#define MAM_COST_GRID       3  /* the cost of (HugeLP) formed in the kernels from
                                  points: the barycenter support is a regular grid
                                  (mam_set_grid), column s of every measure is the
                                  point cost[s*dim ..] (cost_ncols points of dim
                                  doubles), c_rs = sum_k (x_rk - z_sk)^2 rounded to
                                  the dtype.  Single problems, long-column path. */

/* mam_desc.flags */
#define MAM_FLAG_DIAG 1u       /* compute diagnostics on the last iteration of
                                  every mam_iterate call */
#define MAM_FLAG_COLD 2u       /* start every threshold search from w_max - q_s
                                  instead of the column's previous threshold
                                  (same results; for testing and timing) */
#define MAM_FLAG_RELAXED 4u    /* the full unbalanced extension (the section
                                  relaxing the marginals of q^(m) as well):
                                  Step 2 projects every column onto
                                  {u >= 0, sum_r u_r <= q_s} instead of
                                  Delta_R(q_s), i.e. max(w - max(lambda, 0), 0)
                                  with lambda the simplex threshold.  The
                                  mismatch penalty alpha_m*eta of that problem
                                  enters through the cost: pass c - eta.  The
                                  balanced mass check is skipped; no reverse
                                  mode; mam_diag.meas_resid reports the excess
                                  max(sum_r pi_hat_rs - q_s, 0). */
#define MAM_FLAG_SPARSE_STORE 8u /* long columns only (ignored otherwise): between
                                  the iterations of one call the plans are not
                                  kept dense.  Every inactive entry of theta'
                                  equals -b^(m)_r (Step 2 subtracts b from a
                                  projection that is 0 there), so each
                                  (column, wave sub-tile) keeps only its
                                  entries above lambda (at most the candidate
                                  slots; a sub-tile with more is written dense)
                                  and each (measure, row) its value -b^(m)_r.
                                  The write pass then stores a few entries per
                                  column instead of the whole column, and the
                                  bound theta is written back once, when
                                  mam_iterate, mam_iterate_until or
                                  mam_support_update returns.  Results are
                                  identical bit for bit; the workspace grows by
                                  the patch slots (about 8 bytes x candidate
                                  slots per column and 1024 rows in FP32).
                                  The write-back costs about one dense write
                                  pass, so the flag pays off for calls of
                                  more than one iteration. */

typedef struct mam_problem mam_problem;

/* Problem description.  The measures' support points enter only through the
 * cost (squared Euclidean in the paper, (HugeLP)); mam_cost_sq_euclid builds
 * it from points. */
typedef struct mam_desc {
  int32_t dtype;        /* MAM_F32 or MAM_F64: element type of theta, cost, q   */
  int32_t cost_mode;    /* MAM_COST_*                                           */
  int64_t R;            /* barycenter support size = rows of every plan, >= 1  */
  int64_t M;            /* number of measures, >= 1                             */
  const int64_t* S;     /* host array of M column counts S^m >= 1               */
  int64_t ld;           /* column stride of theta in elements (0 -> R)          */
  int64_t cost_ld;      /* column stride of the cost in elements (0 -> R)       */
  int64_t cost_ncols;   /* number of cost columns held by the cost buffer       */
  double rho;           /* DR prox parameter rho > 0 (step tau = 1/rho)         */
  double gamma;         /* unbalanced penalty in [0, inf]; INFINITY = balanced  */
  uint32_t flags;       /* MAM_FLAG_*                                           */
} mam_desc;

/* Figures of the last iteration run with diagnostics (Sec. 5, stopping
 * criteria; Sec. 6.3 objective and feasibility figures). */
typedef struct mam_diag {
  int64_t iterations;   /* iterations run since mam_init                        */
  double t;             /* damping t^k of that iteration (1 when balanced)      */
  double W_hat;         /* sum_m <c^(m), pi_hat^(m)>                             */
  double dist_L;        /* dist_L(pi_hat): distance of the plans to balance     */
  double meas_resid;    /* max_{m,s} |sum_r pi_hat_rs - q_s|                    */
  double dtheta_inf;    /* ||theta^{k+1} - theta^k||_inf                        */
  double dp_norm;       /* ||p^{k+1} - p^k||_2                                  */
  double p_mass;        /* sum_r p_r of the current barycenter                  */
  double rounds_per_column;  /* threshold rounds per column with q_s > 0        */
  double active_per_column;  /* entries with pi_hat > 0 per such column         */
} mam_diag;

/* Launch schedule of the column kernel (normally chosen by the library).
 * In mam_set_schedule a 0 field means automatic; values_per_thread and
 * vector_width are outputs of mam_get_schedule only. */
typedef struct mam_schedule {
  int32_t threads_per_column; /* 64, 128, 256, 512 or 1024 threads per column;
                                 16 or 32 for short columns (R <= 16*nt rows):
                                 sub-wave groups, 64/nt columns per wave side
                                 by side, one column in flight, no
                                 diagnostics (MAM_FLAG_DIAG, the theta
                                 stopping test) or reverse mode with them
                                 (MAM_EUNSUPPORTED).  0 automatic (64 or more) */
  int32_t values_per_thread;  /* rows held per thread (out)                     */
  int32_t columns_in_flight;  /* columns a group advances together: 1, 2 or 4   */
  int32_t workgroups;         /* workgroups per iteration (see team_size for
                                 how they share the columns); 0 automatic: as
                                 many as the device holds at once for the
                                 kernel (known after mam_init; at most 1024)     */
  int32_t xcd_remap;          /* consecutive runs on one XCD (shared L2): 1 on,
                                 -1 off, 0 automatic (on when the columns are
                                 ordered cost-block-major)                        */
  int32_t vector_width;       /* elements per load: 4 (float), 2 (double) or 1 (out) */
  int32_t order;              /* column order: 1 measure-major, 2 cost-block-major
                                 (columns sharing cost columns close in time;
                                 shared costs, or indexed costs sorted within
                                 each measure), 0 automatic                       */
  int32_t streaming;          /* plans loaded and stored with the non-temporal
                                 (streaming) cache policy, so they do not evict
                                 the cost from the caches: 1 on, -1 off, 0
                                 automatic (on when the group's plans exceed
                                 256 MiB, i.e. do not stay in the 256 MB
                                 Infinity Cache between iterations).  Applies to
                                 the vector-load, one-column-in-flight kernels. */
  int32_t rows_per_tile;      /* long-column path (single problems): rows of a
                                 column tile, 1024, 2048 or 4096.  0 automatic:
                                 the path is taken when R > 8192, with 4096
                                 (float) or 2048 (double) rows.  A value > 0
                                 forces the path at any R.                      */
  int32_t candidate_slots;    /* long-column path: candidates kept per
                                 (column, wave sub-tile of 64*rows_per_tile/256
                                 rows), 1..64; 0 automatic (64).  A sub-tile
                                 with more candidates in an iteration is
                                 recomputed from theta and c (same result,
                                 slower).                                       */
  int32_t team_size;          /* short columns: workgroups per team sweep.  A
                                 team takes an equal contiguous share of the
                                 column order and deals it out in blocks, round
                                 robin over its workgroups, so the columns in
                                 flight lie close together in memory.  1: every
                                 workgroup its own contiguous run; 0 automatic
                                 (1: on the measured workloads each extra
                                 segment's pipeline restart cost more than the
                                 sweep saved). */
} mam_schedule;

/* ABI version of this header (1). */
int32_t mam_abi_version(void);

/* Message for the last failing call on this thread ("" if none). */
const char* mam_last_error(void);

/* Validate d and create a handle.  No HIP call is made.  Errors: MAM_EINVAL
 * (R, M, S^m < 1; ld < R; rho <= 0 or not finite; gamma < 0 or NaN; unknown
 * dtype or cost_mode; shared cost with some S^m > cost_ncols),
 * MAM_EUNSUPPORTED (R > 2^28, the long-column path's int32 row indices, or
 * M > 65535).  Columns of up to 8192 rows are held by one workgroup; longer
 * ones take the long-column path (several workgroups per column).  On
 * error *out is set to NULL. */
mam_status mam_create(mam_problem** out, const mam_desc* d);

/* Override the launch schedule; must precede mam_set_workspace. */
mam_status mam_set_schedule(mam_problem* p, const mam_schedule* s);

/* Read back the schedule in use. */
mam_status mam_get_schedule(const mam_problem* p, mam_schedule* s);

/* Bytes of device workspace the handle needs (0 for a NULL handle). */
size_t mam_workspace_bytes(const mam_problem* p);

/* Give the handle its workspace: 'dev' is a device pointer aligned to 256
 * bytes holding at least mam_workspace_bytes(p) bytes.  Errors: MAM_ENOMEM
 * if too small, MAM_EINVAL if misaligned. */
mam_status mam_set_workspace(mam_problem* p, void* dev, size_t bytes);

/* Bind the caller's device buffers: theta (T*ld elements, read and written),
 * cost (cost_ncols*cost_ld elements, read only), q (T elements, read only),
 * cost_col_index (T int32 values in [0, cost_ncols), MAM_COST_INDEXED only,
 * else NULL).  No HIP call is made.  Errors: MAM_EINVAL on NULL buffers or a
 * missing/unexpected index. */
mam_status mam_bind(mam_problem* p, void* theta, const void* cost,
                    const int32_t* cost_col_index, const void* q);

/* Alg. 1, Step 0: theta^0 = q_s/R in every entry of column s (theta0 NULL),
 * or a copy of the caller's theta0 (same layout); then p^(m) and p.
 * Validates the inputs on the device and SYNCHRONIZES the stream:
 * MAM_ENONFINITE for a negative or non-finite weight or cost,
 * MAM_ENOTBALANCED when gamma = inf and the masses sum q^(m) differ by more
 * than 1e-6 (MAM_F32) or 1e-12 (MAM_F64) relative. */
mam_status mam_init(mam_problem* p, const void* theta0, void* stream);

/* Run 'iters' >= 0 deterministic MAM iterations (M^k = all measures,
 * Alg. 1).  Asynchronous.  Errors: MAM_ESTATE before mam_init. */
mam_status mam_iterate(mam_problem* p, int64_t iters, void* stream);

/* Grid of a MAM_COST_GRID problem (Theorem c: with measures on one grid and
 * alpha_m = 1/M the support Xi of a barycenter is itself a regular grid).
 * Row r is the grid point of index (i_0, ..., i_{dim-1}), last axis fastest
 * (r = i_0 * n[1] + i_1 for dim 2), with coordinates
 * x_rk = origin[k] + i_k * spacing[k] (one product and one sum, each
 * rounded).  Host arrays of dim values, dim 1 or 2; the point count must be
 * R.  Must precede mam_init.  Errors: MAM_EINVAL (mode, sizes, non-finite
 * values). */
mam_status mam_set_grid(mam_problem* p, int32_t dim, const int64_t* n, const double* origin, const double* spacing);

/* ---- stopping tests ----------------------------------------------------------
 * Alg. 1 with "while not converged" made concrete by one of the stopping
 * tests of Sec. 5 (Stopping criteria), evaluated on the device.  After every
 * check_every-th iteration of the run (iterations j = check_every,
 * 2 check_every, ... counted from the call) the test's value is computed for
 * that iteration; when value <= tol the run stops there: the plans and
 * marginals stay at that iterate, and every launch the library had already
 * enqueued for the run returns at once (a flag in the workspace gates
 * them).  A NaN value never stops the run.
 *   MAM_STOP_DTHETA: ||theta^{k+1} - theta^k||_inf over all plan entries, in
 *                    the stored precision (the check iteration computes the
 *                    diagnostics of mam_diag);
 *   MAM_STOP_DP:     ||p^{k+1} - p^k||_2 of the averaged marginals;
 *   MAM_STOP_DIST:   dist_L(pi_hat^k), distance of the projected plans to
 *                    the balanced set (a heuristic test, Sec. 5). */
#define MAM_STOP_DTHETA 0
#define MAM_STOP_DP     1
#define MAM_STOP_DIST   2

typedef struct mam_stop_result {
  int64_t iterations;   /* iterations run by the call                           */
  int64_t checks;       /* tests evaluated                                      */
  int32_t converged;    /* 1 if the test held (the run stopped on it)           */
  double value;         /* value at the last check (NaN if no check ran)        */
} mam_stop_result;

/* Run at most max_iters >= 0 iterations with stopping test 'test' (MAM_STOP_*)
 * and tolerance tol (not NaN) evaluated every check_every >= 1 iterations;
 * iterations past the last multiple of check_every run without a test.
 * Single problems.  Periods of check_every iterations run from a captured
 * HIP graph when mam_graph has turned graphs on (and timing is off), else as
 * plain launches; at most max(2, ceil(32/check_every)) periods are in flight.
 * SYNCHRONIZES the stream (it returns when the run has ended) and fills
 * *out.  mam_diagnostics afterwards describes the last iteration when it was
 * a MAM_STOP_DTHETA check.  Errors: MAM_EINVAL (arguments), MAM_ESTATE
 * (before mam_init), MAM_EUNSUPPORTED (batch; MAM_STOP_DTHETA on long
 * columns with MAM_FLAG_SPARSE_STORE). */
mam_status mam_iterate_until(mam_problem* p, int64_t max_iters, int32_t test, double tol, int64_t check_every,
                             mam_stop_result* out, void* stream);

/* Barycenter p-bar = sum_m a_m p^(m) of the current plans: R doubles into
 * the device buffer p_dev (asynchronous) or the host buffer p_host
 * (synchronizes). */
mam_status mam_barycenter(mam_problem* p, double* p_dev, void* stream);
mam_status mam_barycenter_host(mam_problem* p, double* p_host, void* stream);

/* Marginals p^(m) of the current plans: M*R doubles, row m at m*R, into a
 * device buffer.  Asynchronous. */
mam_status mam_marginals(mam_problem* p, double* pm_dev, void* stream);

/* Diagnostics of the last iteration that ran with MAM_FLAG_DIAG.
 * SYNCHRONIZES the stream.  MAM_ESTATE if none ran yet, MAM_ENONFINITE if
 * the barycenter holds a NaN or Inf (the struct is still filled).  Short and
 * long columns; on long columns W_hat, meas_resid and the per-column counts
 * come from the threshold pass (pi_hat = max(w - lambda, 0) at the entries
 * the write pass patches, summed per column in a fixed order and over
 * columns in column order), dtheta_inf from the write pass, and with
 * MAM_FLAG_SPARSE_STORE dtheta_inf is NaN (no dense copy of the previous
 * plans exists to compare with). */
mam_status mam_diagnostics(mam_problem* p, mam_diag* out, void* stream);

/* Kernel timing: while enabled, HIP events bracket every launch of the
 * column kernel on the stream (graph replay is off meanwhile).  mam_timing_read synchronizes and returns the
 * summed milliseconds and the launch count since the last reset. */
mam_status mam_timing_enable(mam_problem* p, int32_t enable);
mam_status mam_timing_read(mam_problem* p, double* total_ms, int64_t* launches);

/* ---- support step ----------------------------------------------------------
 * The support problem of the fixed-support approach (Sec. 2: with the plans
 * fixed, the support points minimise sum_m alpha_m sum_rs ||xi_r - zeta_s||^2 pi_rs)
 * in the closed form of the free-support proposition (Prop. 4):
 *   mass_r = sum_m alpha_m sum_s pi^(m)_rs,
 *   xi_r   = sum_m alpha_m sum_s pi^(m)_rs zeta^(m)_s / mass_r.
 * mam_support_update first runs one more iteration of Alg. 1 (exactly as
 * mam_iterate(p, 1, stream) would) and takes as pi^(m) that iteration's
 * projected plans pi_hat^(m) (Step 2: non-negative, column sums q_s),
 * rebuilt from the stored theta' as theta' + b^(m); an entry stored as
 * exactly -b^(m)_r (an inactive one) counts as 0.  A row with mass_r <= 0
 * keeps its point.  Alternating this call with a cost rebuilt on the new
 * points (e.g. mam_cost_sq_euclid, scaled by alpha_m/2) is Alg. 2.
 *
 *   alpha: host, M doubles, finite and >= 0 (the barycenter weights alpha_m
 *          of (WB); they are not read from the cost).
 *   zeta:  device, T x dim doubles: the point of plan column j (measures in
 *          order, the columns of measure m at its column offset) at j*dim.
 *   xi:    device, R x dim doubles, row-major; read for rows without mass,
 *          written for the others.
 *   mass:  device, R doubles, or NULL.
 *   dim:   1, 2 or 3.
 *   ws:    device workspace of mam_support_workspace_bytes(p, dim) bytes
 *          (256-byte aligned, caller-owned; 0 is returned for invalid input).
 * Two passes in fixed orders (bitwise reproducible).  Stream-ordered on
 * 'stream'; the call synchronizes it once, after queueing the upload of
 * its column tables (host memory the call owns and frees on return), and
 * the support passes it launches then run asynchronously.  Single
 * problems, short and long columns, FP32 and FP64 plans.
 * Errors: MAM_EINVAL (NULL pointer, dim, alpha, misaligned workspace),
 * MAM_ENOMEM (workspace NULL or too small), MAM_ESTATE (before mam_init),
 * MAM_EUNSUPPORTED (batch handles have no such call). */
size_t mam_support_workspace_bytes(const mam_problem* p, int32_t dim);
mam_status mam_support_update(mam_problem* p, const double* alpha, const double* zeta, int32_t dim,
                              double* xi, double* mass, void* ws, size_t bytes, void* stream);

/* ---- reverse mode ----------------------------------------------------------
 * Gradients through the iteration of Alg. 1 (the paper does not treat
 * differentiation; this is the exact derivative of the computed map away
 * from the measure-zero set where an active set changes).  One balanced
 * iteration is piecewise affine in (theta, q, c): on a column's active set A
 * (w_r > lambda) the projection of Prop. 3 is w - lambda with
 * lambda = (sum_A w - q_s)/|A|, so its Jacobian is D_A - 1_A 1_A^T/|A| and
 * its derivative in q_s is 1_A/|A|.  The reverse sweep propagates
 * dL/dtheta^k as a part supported on the active sets plus one R-vector per
 * measure; it reads the active-set bit masks of the forward (R/8 bytes per
 * column and iteration), never theta or c.
 *
 * Scope: single problems, balanced or unbalanced, started with the default
 * theta^0 = q_s/R (mam_init with theta0 = NULL), any cost mode and dtype.
 * With a finite gamma, Step 1's damping t = gamma/(rho d) (eq.
 * (Unbalanced-prox)) depends on the plans through d; its derivative adds a
 * rank-one term to the transposed averaging, for which the forward also
 * keeps p, p^(m) and d of every recorded iteration (O(M R) per iteration).
 * Gradients are accumulated in double and written in the problem's dtype.
 *
 * Memory: the adjoint workspace (caller-owned device memory, 256-byte
 * aligned) holds the masks of one window of C = ckpt_every iterations
 * (C+1 slots), a checkpoint of theta at the start of every later window,
 * two R x T double arrays (the sparse adjoint and the cost adjoint per plan
 * column) and O(M R + T + cost columns) more.  ckpt_every <= 0 or >= iters
 * keeps every mask of the run (no recomputation).  The size depends on the
 * schedule: query it after mam_set_schedule.  Returns 0 for a batch handle,
 * a NULL handle or iters < 0. */
size_t mam_adjoint_workspace_bytes(const mam_problem* p, int64_t iters, int64_t ckpt_every);

/* Forward pass for the reverse mode: 'iters' iterations exactly as
 * mam_iterate (same results), recording what mam_backward needs into
 * 'adj_ws' ('bytes' long).  Must follow a mam_init with theta0 = NULL and
 * no iteration since.  SYNCHRONIZES the stream once at the start (table
 * upload); then asynchronous.  Errors: MAM_ESTATE (not freshly initialised
 * with the default start), MAM_EUNSUPPORTED (batch),
 * MAM_ENOMEM (workspace NULL or too small), MAM_EINVAL (misaligned, iters < 0). */
mam_status mam_record(mam_problem* p, int64_t iters, int64_t ckpt_every, void* adj_ws, size_t bytes,
                      void* stream);

/* Reverse sweep of the last mam_record: given grad_p = dL/dp_bar (R
 * doubles, device), writes grad_q = dL/dq (T elements of the dtype, device)
 * and grad_cost = dL/dc (cost_ncols columns of R elements at stride
 * cost_ld, device; columns no plan column reads get 0).  Reruns windows of
 * the forward from their checkpoints where the mask ring does not hold
 * them, so it may be called again (same results) while adj_ws, q and the
 * cost are unchanged.  Leaves theta and the marginals at an intermediate
 * iterate: mam_init is needed before further iterations.  Asynchronous.
 * Errors: MAM_ESTATE (no mam_record), MAM_EINVAL (NULL gradient buffer). */
mam_status mam_backward(mam_problem* p, const double* grad_p, void* grad_q, void* grad_cost, void* stream);

/* ---- randomized variant ----------------------------------------------------
 * Alg. 1 with M^k a subset of the measures (eq. (DR-random), and the remark
 * on bundles after the algorithm): the measures are partitioned into nb
 * bundles, and an iteration that draws bundle i updates the plans and
 * marginals of bundle i only (Steps 2 and 3), while Step 1 still averages
 * every marginal.  The draws are the caller's: seq[k] is the bundle of
 * iteration k, so a run can be replayed exactly.  Single problems only; no
 * diagnostics, no graph replay for these iterations.
 *
 * bundle_of: host array of M bundle indices in [0, nb), every bundle
 * non-empty.  The bundle workspace (caller-owned device memory, 256-byte
 * aligned) holds each bundle's column schedule; its size depends on the
 * device (query after mam_init).  mam_bundle_workspace_bytes returns 0 for
 * an invalid partition, a batch or a NULL handle. */
size_t mam_bundle_workspace_bytes(const mam_problem* p, const int32_t* bundle_of, int32_t nb);

/* Build and upload the bundles' schedules (SYNCHRONIZES the stream).  Must
 * follow mam_init.  Errors: MAM_EINVAL (partition, alignment), MAM_ENOMEM
 * (workspace NULL or too small), MAM_ESTATE (no mam_init), MAM_EUNSUPPORTED
 * (batch). */
mam_status mam_set_bundles(mam_problem* p, const int32_t* bundle_of, int32_t nb, void* bundle_ws, size_t bytes,
                           void* stream);

/* 'iters' randomized iterations; iteration k updates bundle seq[k] (host
 * array of iters entries, each in [0, nb)).  Asynchronous after the host
 * check of seq.  Errors: MAM_EINVAL (seq NULL or out of range), MAM_ESTATE
 * (no mam_init or no mam_set_bundles). */
mam_status mam_iterate_bundles(mam_problem* p, int64_t iters, const int32_t* seq, void* stream);

/* Destroy a handle (NULL is allowed).  Device buffers stay with the caller. */
void mam_destroy(mam_problem* p);

/* A measurement helper, not a step of the method: copy 'bytes' (a multiple
 * of 16) from src to dst, both device buffers with 16-byte alignment, with
 * non-temporal 16-byte loads and stores over 'workgroups' workgroups of 256
 * threads in grid-stride order.  It gives the read-plus-write streaming
 * ceiling of the device against which the column kernels' bandwidth is
 * compared, and calibrates the HBM counters.  Asynchronous on 'stream'.
 * Errors: MAM_EINVAL (NULL buffer, size or alignment, workgroups < 1). */
mam_status mam_stream_copy(void* dst, const void* src, size_t bytes, int32_t workgroups, void* stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): one whole solve with no workspace
 * argument and no device allocation.  It does what mam_create,
 * mam_set_workspace, mam_bind, mam_init, mam_iterate and mam_barycenter do
 * in turn, on a handle that lives for the call, with the workspace taken
 * from a static device array of the library: 128 MiB per GPU, allocated
 * when the library's code is loaded on that GPU and held until the process
 * ends.
 *   d, theta, cost, cost_col_index, q: as for mam_create and mam_bind
 *          (theta: the caller's R x T plans, written; on return it holds
 *          theta^iters);
 *   theta0: as for mam_init (NULL: theta^0 = q_s/R);
 *   iters:  >= 0 iterations of Alg. 1;
 *   p_out:  device, R doubles: the barycenter of theta^iters.
 * Results are those of the handle sequence above, bit for bit.  Every call
 * on one GPU uses the same array and leaves its contents behind (every
 * region a call reads is written by that call first): calls that overlap
 * on one GPU (other threads, or streams that run concurrently) race.
 * Synchronizes 'stream' as mam_init does; the iterations and the
 * barycenter are queued on it.  Errors: those of the calls above;
 * MAM_EINVAL (NULL argument, iters < 0), MAM_ENOMEM (the problem needs
 * more workspace than the array holds: mam_workspace_bytes of its handle
 * exceeds 128 MiB), MAM_EUNSUPPORTED (MAM_COST_GRID, which needs
 * mam_set_grid on a handle). */
mam_status mam_solve_static(const mam_desc* d, void* theta, const void* cost, const int32_t* cost_col_index,
                            const void* q, const void* theta0, int64_t iters, double* p_out, void* stream);

/* Graph replay: capture 'iters_per_launch' iterations once as a HIP graph
 * (on a stream of the library's own) and let mam_iterate replay it on the
 * caller's stream, running any remainder (and a diagnostics iteration)
 * directly.  0 turns graphs off.  Rebinding or re-initialising drops the
 * captured graph.  No memset nodes are captured. */
mam_status mam_graph(mam_problem* p, int64_t iters_per_launch);

/* ---- batches -------------------------------------------------------------
 * Many independent problems (same dtype; any R <= 8192, M, S^m, cost mode,
 * rho, gamma) advanced together: each iteration is one column-kernel launch
 * per shape group (problems whose columns need the same threads per column
 * and values per thread; inside a captured graph the groups run
 * concurrently on streams of the library's own, default priority, forked
 * from and joined back into the capturing stream), then one marginal and
 * one averaging launch for all
 * problems; mam_batch_graph captures whole iterations as one graph.
 * Diagnostics (MAM_FLAG_DIAG) are not computed for batches. */
typedef struct mam_batch mam_batch;

/* Validate n >= 1 descriptions (rules of mam_create) and create a batch. */
mam_status mam_batch_create(mam_batch** out, const mam_desc* descs, int32_t n);

/* Number of shape groups, and the group of problem i (-1 if none). */
int32_t mam_batch_groups(const mam_batch* b);
int32_t mam_batch_group_of(const mam_batch* b, int32_t i);

/* Schedule of one shape group (rules of mam_set_schedule). */
mam_status mam_batch_set_schedule(mam_batch* b, int32_t group, const mam_schedule* s);
mam_status mam_batch_get_schedule(const mam_batch* b, int32_t group, mam_schedule* s);

/* Workspace for the whole batch (rules of mam_workspace_bytes and
 * mam_set_workspace). */
size_t mam_batch_workspace_bytes(const mam_batch* b);
mam_status mam_batch_set_workspace(mam_batch* b, void* dev, size_t bytes);

/* Buffers of problem i (rules of mam_bind). */
mam_status mam_batch_bind(mam_batch* b, int32_t i, void* theta, const void* cost,
                          const int32_t* cost_col_index, const void* q);

/* Alg. 1 Step 0 for every problem (theta^0 = q_s/R) with the checks of
 * mam_init; SYNCHRONIZES the stream. */
mam_status mam_batch_init(mam_batch* b, void* stream);

/* 'iters' iterations of every problem; asynchronous. */
mam_status mam_batch_iterate(mam_batch* b, int64_t iters, void* stream);

/* Graph replay for batches (rules of mam_graph). */
mam_status mam_batch_graph(mam_batch* b, int64_t iters_per_launch);

/* Barycenter of problem i: R_i doubles into a device buffer; asynchronous. */
mam_status mam_batch_barycenter(mam_batch* b, int32_t i, double* p_dev, void* stream);

/* Column-kernel timing for batches (rules of mam_timing_enable/read; one
 * launch = all groups' column kernels of one iteration). */
mam_status mam_batch_timing_enable(mam_batch* b, int32_t enable);
mam_status mam_batch_timing_read(mam_batch* b, double* total_ms, int64_t* launches);

/* Destroy a batch (NULL is allowed). */
void mam_batch_destroy(mam_batch* b);

/* Cost helper (the cost of (HugeLP) from support points):
 * out[s*out_ld + r] = ||xi_r - zeta_s||^2, divided by its maximum over all
 * (r, s) when normalize_max != 0.  xi: R*dim doubles (point r at r*dim) and
 * zeta: S*dim doubles, device pointers; out: S*out_ld elements of 'dtype'
 * (device).  Distances are formed in double and rounded once to 'dtype'.
 * normalize_max needs 'scratch', one device double the call overwrites.
 * Asynchronous.  Errors: MAM_EINVAL on NULL buffers, sizes < 1,
 * out_ld < R, unknown dtype, or normalize_max without scratch. */
mam_status mam_cost_sq_euclid(const double* xi, int64_t R, const double* zeta,
                              int64_t S, int32_t dim, int32_t normalize_max,
                              void* out, int64_t out_ld, int32_t dtype,
                              double* scratch, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MAM_H */
