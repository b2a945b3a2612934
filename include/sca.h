/*
 * sca.h -- C ABI of libsca, the MI355X (gfx950) hot path of the fixed-stepsize
 * successive-convex-approximation block method (AsyFLEXA, Algorithm 1 of Cannelli,
 * Facchinei, Kungurtsev, Scutari, arXiv:1701.04900) for
 *
 *     min_x  1/2 ||A x - b||^2 - c ||x||^2 + lambda * sum_j h(x_j)
 *     s.t.   -beta <= x_j <= beta,
 *
 * with h = |.| (LASSO, Section 4.2) or one of the DC regularisers of Section 4.3.
 *
 * One ROUND k (steps S.1-S.5 of Algorithm 1 for every drawn block, all reading the
 * same x^k and r^k = A x^k - b):
 *   S.1  block i is drawn iff word 0 of Philox4x32-10(counter = (i, k mod 2^32,
 *        k div 2^32, instance), key = (seed mod 2^32, seed div 2^32)) is below
 *        floor(select_p * 2^32)  (select_p = 1 draws every block);
 *   S.2  for every coordinate j of a drawn block:
 *          g_j  = a_j^T r - 2 c x_j - lambda * (h^-)'(x_j)
 *          q_j  = ||a_j||^2 + tau
 *          xh_j = clip(soft(x_j - g_j/q_j, lambda*eta/q_j), -beta, beta)
 *        (the closed-form minimiser of the block surrogate, subproblem (2));
 *   S.4  x_j += gamma_k (xh_j - x_j)   (update (3));
 *        r += sum over moved j of a_j * dx_j  (keeps r = A x - b).
 * gamma_k = gamma for a fixed step; with gamma_mu > 0 it follows
 * gamma_{k+1} = gamma_k (1 - gamma_mu gamma_k) from gamma_0 = gamma (Section 4.1).
 *
 * Conventions for every entry point
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA tensors);
 *     *_host are host pointers.  Scalars are passed by value.
 *   - 'stream' is a hipStream_t (NULL = the null stream).  Work is enqueued on it in
 *     order; entry points that return host scalars synchronise that stream and say so.
 *   - Every argument is validated on the host before any launch; a failure returns
 *     SCA_EINVAL (nothing is enqueued) and sca_last_error() describes it.
 *   - dtype SCA_F32: A, b, x, r are float and every accumulation of the round is in
 *     float; objective, merit, M_F and fresh residuals accumulate in double.
 *     dtype SCA_F64: everything is double.
 *   - Status codes are returned; no exception crosses the ABI.
 */
#ifndef SCA_H
#define SCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCA_OK = 0,
  SCA_EINVAL = 1,     /* invalid argument; nothing was enqueued                          */
  SCA_ENOMEM = 2,     /* a device allocation failed                                      */
  SCA_EHIP = 3,       /* a HIP runtime call failed                                       */
  SCA_ENONFINITE = 4, /* the objective became NaN/Inf at a check (divergence)            */
  SCA_ENOTCONV = 5    /* max_rounds reached before the tolerance (stats are filled in)   */
} sca_status;

typedef enum { SCA_F32 = 0, SCA_F64 = 1 } sca_dtype;

/* Regulariser h (Section 4.3): L1 h=|x|; EXP h=1-exp(-theta|x|), eta=theta;
 * LOG h=log(1+theta|x|)/log(1+theta), eta=theta/log(1+theta).  The concave part
 * h^- = eta|x| - h is linearised in the best response. */
typedef enum { SCA_REG_L1 = 0, SCA_REG_EXP = 1, SCA_REG_LOG = 2 } sca_reg;

enum { SCA_FLAG_PROFILE = 1 }; /* time the kernels of sca_step with HIP events */

typedef struct sca_problem sca_problem; /* opaque, owned by the library */

typedef struct {
  size_t struct_size;    /* = sizeof(sca_opts)                                           */
  double gamma;          /* step (3), in (0, 1]; initial value of the diminishing rule     */
  double gamma_mu;       /* >= 0; 0 = fixed step                                          */
  double tau;            /* >= 0, proximal weight of the surrogate (q_j = ||a_j||^2 + tau) */
  double select_p;       /* (0, 1], probability that a block is drawn in a round          */
  uint64_t seed;         /* Philox key                                                    */
  uint32_t instance;     /* Philox counter word 3                                         */
  uint32_t flags;        /* SCA_FLAG_*                                                    */
  int64_t max_rounds;    /* sca_solve: round budget                                       */
  int64_t check_every;   /* sca_solve: rounds between objective checks (>= 1)             */
  int64_t refresh_every; /* sca_solve: recompute r = Ax-b every this many checks (0 = no) */
  double tol_rel_obj;    /* sca_solve: stop at (F - F_star)/|F_star| <= tol (0 = off)     */
  double F_star;         /* reference optimum for tol_rel_obj                              */
  double tol_merit;      /* sca_solve: stop at ||xh(x) - x||_inf <= tol (0 = off)          */
  int64_t delay_chunks;  /* > 1: bounded-delay rounds (dense problems only; see below)     */
  int64_t delay_stale;   /* staleness of the bounded-delay rounds, in groups (>= 0)        */
  int64_t async_workgroups; /* > 0: lock-free rounds on this many workgroups (see below)   */
} sca_opts;

/* Bounded-delay rounds (delayed iterates of Algorithm 1, delays bounded as in Assumption
 * D1): with delay_chunks = q > 1 the drawn coordinates of a round (ascending) are updated in
 * q consecutive groups of ceil(|S|/q); group t reads the residual left by groups
 * 0..t-1-delay_stale of the round, its own coordinates being current (D4).  Every update
 * then misses at most (delay_stale + 1) * ceil(|S|/q) - 1 others.  q <= 1, or
 * delay_stale >= q - 1, is the ordinary round (all drawn coordinates read the same
 * iterate); delay_stale = 0 is a Gauss-Seidel sweep over the groups.  Deterministic.  The
 * sparse, batched and multi-right-hand-side paths reject delay_chunks > 1 (SCA_EINVAL).
 *
 * Lock-free rounds (Algorithm 1 with the delays of Assumption D1 left to the hardware, as in
 * the paper's shared-memory implementation, Section 4): with async_workgroups = W in
 * [1, 65536] the drawn coordinates of a round are taken one at a time from a shared counter
 * by W workgroups; each reads the residual r as it stands in device memory (it may miss the
 * folds of the at most W - 1 coordinates in flight on other workgroups), updates its own
 * x_j and folds its move into r with atomic adds.  The result depends on the timing for
 * W > 1 (not reproducible run to run); W = 1 is a sequential sweep over the drawn
 * coordinates in ascending order.  Dense problems only, and not with delay_chunks > 1
 * (SCA_EINVAL); for a study of the delay's effect, not for speed (one atomic add per row of
 * every moved column). */

typedef struct {
  size_t struct_size;    /* = sizeof(sca_stats)                                          */
  int64_t rounds;        /* rounds run                                                    */
  int64_t coord_updates; /* sum over rounds of the drawn coordinates                      */
  int64_t moved_updates; /* sum over rounds of the coordinates that moved (columns folded) */
  double F;              /* final objective with a freshly computed residual (FP64 acc.)  */
  double merit;          /* final ||xh(x) - x||_inf                                       */
  double MF;             /* final ||M_F(x)||_2 (unit-step prox residual, Section 3)      */
  double rel_err;        /* (F - F_star)/|F_star| when F_star != 0, else 0               */
  double seconds;        /* host wall time of the call                                    */
  int64_t nnz;           /* nonzeros of xh(x)                                             */
  int32_t status;        /* sca_status of the solve                                       */
  int32_t checks;        /* objective checks performed                                    */
} sca_stats;

/* Kernel kinds reported by sca_profile_get (indices into its arrays). */
enum { SCA_K_SELECT = 0, SCA_K_GRAD = 1, SCA_K_COMPACT = 2, SCA_K_FOLD = 3, SCA_K_NKINDS = 4 };

/* Library version string (static storage). */
const char* sca_version(void);

/* Message of the last failing call on this host thread (static, thread-local storage). */
const char* sca_last_error(void);

/* Create a problem over a dense A.
 *  A_colmajor_dev: column j at A + j*lda, m valid rows; the buffer holds lda*n elements of
 *    the dtype, base 16-byte aligned, lda >= m and lda a multiple of 16/sizeof(element).
 *    Rows m..lda-1 are never read.  BORROWED: A must outlive the problem; it is not copied.
 *  b_dev: m elements, borrowed.  lambda >= 0, c >= 0, beta > 0 (INFINITY = no box).
 *  block_ptr_host: nblocks+1 ascending offsets, block_ptr[0] = 0, block_ptr[nblocks] = n,
 *    every block nonempty (Assumption D4: a block is updated by one worker).  Copied.
 * Computes ||a_j||^2 (FP64) and checks that b is finite; synchronises 'stream' once. */
sca_status sca_problem_create_dense(sca_problem** out, sca_dtype dtype, int64_t m, int64_t n,
                                    const void* A_colmajor_dev, int64_t lda, const void* b_dev,
                                    double lambda, double c, double beta,
                                    const int64_t* block_ptr_host, int64_t nblocks, void* stream);

/* Create a problem over a sparse A given in CSR (row-major) form (the sparse LASSO data of
 * the paper's Section 4.2 experiments; problem (1) with f = 1/2||Ax - b||^2): rowptr_dev (m+1 int64),
 * colidx_dev (nnz int32 in [0,n)), vals_dev (nnz of the dtype), b_dev (m).  The library
 * builds and owns a column-major (CSC) copy with rows ascending inside each column; the
 * caller may free the CSR once this call returns.  Limits: 0 <= nnz < 2^31, m <= 2^23
 * (SCA_EINVAL beyond); a repeated (row, column) entry or a column index outside [0, n) is
 * SCA_EINVAL.  Device memory: the CSC copy plus a fold workspace of nnz entries (8 bytes
 * each in FP32, 16 in FP64); where r fits in NP <= 16 row panels of 140 KiB (m <= 573440
 * FP32, 286720 FP64), also n x (NP+1) int32 panel offsets and NP x n partial sums of the
 * dtype for the panel-split gradient (when those do not fit, the slower panel-walk gradient
 * runs instead).  Other arguments as for the dense form.  Synchronises 'stream'.
 * The residual fold of a sparse problem sums the products a_ij * dx_j of a row exactly in
 * fixed point: each product and each row's sum must stay below 2^55 in magnitude; a row
 * that receives a larger or non-finite product becomes NaN, so the next objective check
 * of sca_solve returns SCA_ENONFINITE. */
sca_status sca_problem_create_csr(sca_problem** out, sca_dtype dtype, int64_t m, int64_t n,
                                  int64_t nnz, const int64_t* rowptr_dev,
                                  const int32_t* colidx_dev, const void* vals_dev,
                                  const void* b_dev, double lambda, double c, double beta,
                                  const int64_t* block_ptr_host, int64_t nblocks, void* stream);

/* Select the regulariser (default SCA_REG_L1).  theta > 0 for EXP and LOG. */
sca_status sca_problem_set_regularizer(sca_problem* p, sca_reg reg, double theta);

/* Replace the right-hand side (borrowed, m elements) and lambda of a problem, e.g. for a
 * lambda sweep or a finite-difference probe.  Checks that b is finite; synchronises. */
sca_status sca_problem_update_rhs(sca_problem* p, const void* b_dev, double lambda, void* stream);

/* Release the problem and its workspace (A and b stay with the caller).  NULL is a no-op. */
void sca_problem_destroy(sca_problem* p);

/* Run rounds round_begin .. round_begin+nrounds-1 in place on x_dev (n elements) and
 * r_dev (m elements, 16-byte aligned), which must satisfy r = A x - b on entry (see
 * sca_residual).  The step of round k is gamma_k from opts.  Stream-ordered; does not
 * synchronise (except with SCA_FLAG_PROFILE, which waits for its events at the end). */
sca_status sca_step(sca_problem* p, const sca_opts* opts, int64_t round_begin, int64_t nrounds,
                    void* x_dev, void* r_dev, void* stream);

/* r_dev <- A x_dev - b with FP64 accumulation, rounded to the dtype: the residual the
 * partial gradients of Algorithm 1 step S.2 read (a_j^T r is the partial gradient of
 * 1/2||Ax - b||^2, the smooth part of the Section 4.2 LASSO).  x_dev: n elements, r_dev: m
 * elements (16-byte aligned), both of the problem's dtype, caller-owned.  Stream-ordered. */
sca_status sca_residual(sca_problem* p, const void* x_dev, void* r_dev, void* stream);

/* Fill mask_dev[i] (uint8, nblocks) with 1 when block i is drawn in round k (step S.1).
 * Stream-ordered.  Exposes the selection the rounds use. */
sca_status sca_select_blocks(sca_problem* p, const sca_opts* opts, int64_t k, uint8_t* mask_dev,
                             void* stream);

/* Philox4x32-10 on the device: for i < count, in_dev[6i..6i+5] = (ctr0..3, key0..1),
 * out_dev[4i..4i+3] = output words.  Stream-ordered. */
sca_status sca_philox4x32_10(const uint32_t* in_dev, uint32_t* out_dev, int64_t count,
                             void* stream);

/* Stationarity report at x_dev (n elements) with a fresh residual (FP64 accumulation):
 * F = 1/2||Ax-b||^2 - c||x||^2 + lam sum h(x_j) (the objective whose relative error
 * Section 4.2 measures), the merit ||xh(x)-x||_inf of Section 4.3, ||M_F(x)||_2 (the
 * unit-step proximal residual of Section 3) and nnz(xh(x)); any output pointer may be NULL.
 * opts supplies tau.  Synchronises 'stream'. */
sca_status sca_objective(sca_problem* p, const sca_opts* opts, const void* x_dev, double* F,
                         double* merit, double* MF, int64_t* nnz, void* stream);

/* Solve from x_dev (in: x^0, out: final x) until tol_rel_obj / tol_merit / max_rounds
 * (Section 4.2 measures relative objective error, Section 4.3 the merit).  The stopping
 * test runs every check_every rounds and is confirmed with a fresh residual.  stats may
 * be NULL.  Synchronises 'stream'.  Returns SCA_ENOTCONV when the budget ran out. */
sca_status sca_solve(sca_problem* p, const sca_opts* opts, void* x_dev, sca_stats* stats,
                     void* stream);

/* Implicit-differentiation adjoint at a fixed point x* = xh(x*) (regulariser L1 only).
 * Support S = {j : xh_j(x*) != 0, |xh_j(x*)| < beta}, s = sign(xh_S); solves
 * (A_S^T A_S - 2c I) w = xbar_S by conjugate gradients (FP64 dot products) to relative
 * residual cg_tol (<= 0: 1e-12 in F64, 1e-6 in F32) within cg_maxit iterations, then
 * bbar_dev = A_S w (m elements), *lambar_host = -s^T w.  opts supplies tau.
 * Returns SCA_ENOTCONV when CG did not converge and SCA_EINVAL when H_S shows a
 * non-positive curvature.  Synchronises 'stream'. */
sca_status sca_adjoint(sca_problem* p, const sca_opts* opts, const void* xstar_dev,
                       const void* xbar_dev, void* bbar_dev, double* lambar_host,
                       double cg_tol, int64_t cg_maxit, void* stream);

/* sca_adjoint without any device allocation, for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid hipMalloc): sca_adjoint allocates its
 * workspace on its first call with a problem; this variant keeps it in a fixed 32 MiB
 * device array of the library (one per GPU, held until the process ends).  Same
 * arguments, results and errors as sca_adjoint; in addition SCA_EINVAL (nothing enqueued)
 * when the problem needs more than the array holds: about 54 n + 264 m bytes (n columns,
 * m rows; 10.6 MB at 20000 x 100000).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other host threads, other streams) race and must be serialised
 * by the caller.  Synchronises 'stream' (the conjugate-gradient loop reads its convergence
 * flags on the host), so it cannot be captured into a graph. */
sca_status sca_adjoint_noalloc(sca_problem* p, const sca_opts* opts, const void* xstar_dev,
                               const void* xbar_dev, void* bbar_dev, double* lambar_host,
                               double cg_tol, int64_t cg_maxit, void* stream);

/* Accumulated kernel times (ms) and launch counts of sca_step calls made with
 * SCA_FLAG_PROFILE, indexed by SCA_K_*; arrays of SCA_K_NKINDS entries.  reset != 0
 * clears them after reading. */
sca_status sca_profile_get(sca_problem* p, double* ms_host, int64_t* launches_host,
                           double* bytes_host, int reset);

/* Launch shape of the gradient kernel (the dominant kernel).
 *  grad_kind 0: one wave per drawn column, grad_unroll in {4, 8, 16} 16-byte loads in flight;
 *  grad_kind 1: one 256-thread workgroup walks grad_cols columns together with grad_unroll
 *    row steps in flight, (cols, unroll) in {(2,4), (4,1), (4,2), (4,4), (8,1), (8,2), (16,1),
 *    (16,2)}, non-temporal loads;
 *  grad_kind 2: as 1 with ordinary loads, (cols, unroll) in {(8,2), (16,1)};
 *  grad_kind 3: every wave walks its own group of grad_cols columns (short columns),
 *    (cols, unroll) in {(4,2), (4,4), (8,1)};
 *  grad_kind 4: fused round of a dense problem (steps S.2-S.5 of Algorithm 1 in one pass
 *    over the drawn columns): one 1024-thread workgroup per compute unit holds a whole
 *    column, r and its own fold partial in registers and walks its share of the drawn list
 *    grad_cols columns at a time; a second kernel adds the partials to r.  Needs
 *    m <= 20480 (FP32) or m <= 6144 (FP64); grad_cols in {1, 2, 4, 8} is reduced to the
 *    largest group the registers hold for this m; grad_unroll = grad_wg_per_cu = 1.
 *    With bounded delay (delay_chunks > 1) each group of a round runs the fused kernel on
 *    its own coordinates (gradients from the stale residual version).
 *  grad_wg_per_cu in [1, 16]: persistent workgroups per compute unit. */
typedef struct {
  size_t struct_size; /* = sizeof(sca_launch) */
  int32_t grad_kind;
  int32_t grad_cols;
  int32_t grad_unroll;
  int32_t grad_wg_per_cu;
} sca_launch;

/* One row of the tuning table.  target 0: single problems of this dtype with
 * m_lo <= m <= m_hi get 'launch' (the shapes above); target 1: batches of this dtype whose
 * largest instance has m_lo <= m <= m_hi get 'launch' (the shapes of sca_batch_set_launch). */
typedef struct {
  int32_t dtype; /* sca_dtype */
  int32_t target; /* 0: single problem, 1: batch */
  int64_t m_lo, m_hi;
  sca_launch launch;
} sca_tune_entry;

/* Replace the process-wide tuning table (count rows, copied; count 0 clears it).  Problems
 * created afterwards take the first matching row, else the built-in default. */
sca_status sca_tuning_set(const sca_tune_entry* entries_host, int64_t count);

/* Read / override the launch shape of one problem.  Rejects shapes outside the lists above
 * and the fused kind where the problem cannot take it (sparse, or m too large); the shape
 * read back is the one in effect. */
sca_status sca_problem_get_launch(sca_problem* p, sca_launch* out);
sca_status sca_problem_set_launch(sca_problem* p, const sca_launch* launch);

/* Measurement utilities (not part of the method): a streaming copy of 'bytes' from src to
 * dst and a streaming read of src, 16-byte accesses over 'grid' workgroups of 256 threads
 * (grid <= 0: four per compute unit).  sink_dev receives at most 'grid' floats and is
 * practically never written.  Buffers 16-byte aligned, bytes a multiple of 16.
 * Stream-ordered.  They give the achievable bandwidth and calibrate byte counters. */
sca_status sca_stream_copy(void* dst_dev, const void* src_dev, int64_t bytes, int32_t grid,
                           void* stream);
sca_status sca_stream_read(const void* src_dev, int64_t bytes, void* sink_dev, int32_t grid,
                           void* stream);

/* ------------------------------------------------------------------------------------
 * Batched form: many dense instances of uneven size advance together, one round of every
 * active instance per launch sequence (a block-diagonal problem).  Instance k follows the
 * trajectory of the plain path run with opts.instance = item.instance: the batch shares
 * gamma, gamma_mu, select_p and seed from sca_opts; tau, lambda, c, beta and F_star are
 * per instance.  x and r of the batch are concatenations laid out as sca_batch_layout
 * reports (r offsets padded to 16 bytes; padding entries are never read).
 * ------------------------------------------------------------------------------------ */
typedef struct sca_batch sca_batch; /* opaque, owned by the library */

typedef struct {
  size_t struct_size;            /* = sizeof(sca_batch_item)                            */
  int64_t m, n;                  /* rows and columns of this instance                   */
  const void* A_dev;             /* column-major, as for sca_problem_create_dense; borrowed */
  int64_t lda;
  const void* b_dev;             /* m elements; copied into the batch at create          */
  double lambda, c, beta;        /* as for sca_problem_create_dense                      */
  double tau;                    /* proximal weight of this instance                     */
  double F_star;                 /* reference optimum for tol_rel_obj (0 = unknown)      */
  const int64_t* block_ptr_host; /* nblocks+1 offsets, copied                            */
  int64_t nblocks;
  uint32_t instance;             /* Philox counter word 3 of this instance               */
  uint32_t reserved;
} sca_batch_item;

/* Create a batch over count instances (items_host: count entries).  Validation as for the
 * dense create, per item.  Synchronises 'stream'. */
sca_status sca_batch_create(sca_batch** out, sca_dtype dtype, int64_t count,
                            const sca_batch_item* items_host, void* stream);

/* Release the batch (the A matrices stay with the caller).  NULL is a no-op. */
void sca_batch_destroy(sca_batch* batch);

/* Offsets (count+1 entries each, host) of every instance in the concatenated x and r. */
sca_status sca_batch_layout(sca_batch* batch, int64_t* x_offsets_host, int64_t* r_offsets_host);

/* Launch shape of the batch's rounds (Algorithm 1, steps S.1-S.5 of every instance).
 *  grad_kind 1: fused round -- one pass over the drawn columns: a 512-thread workgroup holds
 *    a group of columns of one instance, that instance's r and its own fold partial in
 *    registers (Q = 1, 2 or 4 row groups of 16 bytes per thread as the instance's m needs,
 *    and 8, 4 or 1 columns per group for Q = 1, 2, 4; grad_cols = 4 names this shape and is
 *    the only value accepted); the workgroups (grad_wg_per_cu in [1, 4] per compute unit) take contiguous
 *    shares of the round's work cut by cost (rows + 16384 per drawn column), so the sums have a
 *    fixed order; a second kernel adds the partials of instances that were shared between
 *    workgroups.  Needs every instance's m <= 8192 (FP32) or <= 4096 (FP64).
 *  grad_kind 0: two-pass round (gradient pass, then an ordered fold of the moved columns).
 * A new batch takes the tuning table's first target-1 row matching its dtype and largest m,
 * else the fused kind (grad_wg_per_cu 2) where it fits and the two-pass kind otherwise.
 * set rejects a shape outside these (SCA_EINVAL); grad_unroll is ignored. */
sca_status sca_batch_get_launch(sca_batch* batch, sca_launch* out);
sca_status sca_batch_set_launch(sca_batch* batch, const sca_launch* launch);

/* Regulariser shared by every instance (as sca_problem_set_regularizer). */
sca_status sca_batch_set_regularizer(sca_batch* batch, sca_reg reg, double theta);

/* Replace the per-instance F_star (count entries, host). */
sca_status sca_batch_set_fstar(sca_batch* batch, const double* F_star_host);

/* r_all <- A_k x_k - b_k for every instance, FP64 accumulation.  Stream-ordered. */
sca_status sca_batch_residual(sca_batch* batch, const void* x_all_dev, void* r_all_dev,
                              void* stream);

/* Rounds round_begin .. round_begin+nrounds-1 of every instance, in place (parity path;
 * r_all must equal A x - b on entry).  Stream-ordered. */
sca_status sca_batch_step(sca_batch* batch, const sca_opts* opts, int64_t round_begin,
                          int64_t nrounds, void* x_all_dev, void* r_all_dev, void* stream);

/* Solve every instance from x_all (in: x^0, out: x).  Rounds run in graph launches of
 * check_every rounds followed by, per instance, the test (F - F_star)/|F_star| <=
 * tol_rel_obj (Section 4.2) on the running residual, confirmed for the instances that pass
 * with a fresh FP64 residual of their own columns (a failed confirmation restarts that
 * instance's running residual from the fresh one), as sca_solve does; when tol_merit > 0
 * instead a fresh FP64 residual of every instance, both tests on it and, at the cost of a
 * full pass over every A, ||xh(x) - x||_inf <= tol_merit (Section 4.3).  A converged
 * instance stops drawing blocks.  stats
 * (count entries, may be NULL) receive per-instance results (coord_updates per instance;
 * moved_updates is the batch-wide total of moved coordinates, the same in every entry).
 * Synchronises 'stream';
 * returns SCA_ENOTCONV when an instance ran out of max_rounds. */
sca_status sca_batch_solve(sca_batch* batch, const sca_opts* opts, void* x_all_dev,
                           sca_stats* stats_host, void* stream);

/* Replace every instance's right-hand side (b_all_dev in the r layout; valid rows are
 * copied) and lambda (lambda_host, count entries).  Synchronises 'stream'. */
sca_status sca_batch_update_rhs(sca_batch* batch, const void* b_all_dev, const double* lambda_host,
                                void* stream);

/* The adjoint of sca_adjoint for every instance at once (x*, xbar in the x layout, bbar in
 * the r layout, lambar_host: count entries).  Each instance runs its own conjugate
 * gradients with its own scalars and stopping test.  Synchronises 'stream'. */
sca_status sca_batch_adjoint(sca_batch* batch, const sca_opts* opts, const void* xstar_all_dev,
                             const void* xbar_all_dev, void* bbar_all_dev, double* lambar_host,
                             double cg_tol, int64_t cg_maxit, void* stream);

/* Per-instance F, merit, ||M_F|| and nnz(xh) with fresh residuals (arrays of count
 * entries, any may be NULL).  Synchronises 'stream'. */
sca_status sca_batch_objective(sca_batch* batch, const sca_opts* opts, const void* x_all_dev,
                               double* F_host, double* merit_host, double* MF_host,
                               int64_t* nnz_host, void* stream);

/* ---------------------------------------------------------------------------------------
 * Many right-hand sides over one dense A (a sweep over lambda as in the experiments of
 * Section 4.3, or the perturbed problems of a finite-difference check): K problems
 *   min 1/2||A x_k - b_k||^2 - c||x_k||^2 + lambda_k ||x_k||_1,  -beta <= x_k <= beta,
 * k = 0..K-1, solved together with Algorithm 1 under one block draw (the seed and instance
 * word of the options are shared), so that the partial gradients of a round, A_S^T R, and
 * its residual update, A_J dX_J, are matrix products run on the matrix cores.  Each
 * column of X follows, round for round, the iterates the single-problem path produces for
 * (b_k, lambda_k) with the same options, up to the order of floating-point additions.
 * The l1 regulariser only.
 *
 * Layouts: A as for sca_problem_create_dense (borrowed); B (m x K, column k = b_k, leading
 * dimension ldb >= m, borrowed); X (n x K, column k = x_k, leading dimension n); R
 * (m x K, column k = A x_k - b_k, leading dimension lda, 16-byte aligned).  1 <= K <= 64.
 * --------------------------------------------------------------------------------------- */
typedef struct sca_multi sca_multi;

/* Create the K-problem set.  lambda_host: K values >= 0.  Errors as for
 * sca_problem_create_dense, and SCA_EINVAL for K outside [1, 64] or ldb < m.  Synchronises
 * 'stream'. */
sca_status sca_multi_create(sca_multi** out, sca_dtype dtype, int64_t m, int64_t n,
                            const void* A_colmajor_dev, int64_t lda, int64_t K,
                            const void* B_dev, int64_t ldb, const double* lambda_host,
                            double c, double beta, const int64_t* block_ptr_host,
                            int64_t nblocks, void* stream);
void sca_multi_destroy(sca_multi* mp);

/* F*_k of every problem (K values, nonzero), used by the relative-error stop of
 * sca_multi_solve. */
sca_status sca_multi_set_fstar(sca_multi* mp, const double* F_star_host);

/* R = A X - B with FP64 accumulation (rounded once into the dtype).  Stream-ordered. */
sca_status sca_multi_residual(sca_multi* mp, const void* X_dev, void* R_dev, void* stream);

/* Rounds [round_begin, round_begin + nrounds) of Algorithm 1 on every problem, in place
 * on X and R (R must hold A X - B on entry).  Stream-ordered; nothing is read back. */
sca_status sca_multi_step(sca_multi* mp, const sca_opts* opts, int64_t round_begin,
                          int64_t nrounds, void* X_dev, void* R_dev, void* stream);

/* Per problem (arrays of K, any may be NULL): F_k with a fresh FP64-accumulated residual,
 * the merit ||xh(x_k) - x_k||_inf (Section 4.3) and nnz(xh(x_k)).  The merit's partial
 * gradients use FP64 products.  Synchronises 'stream'. */
sca_status sca_multi_objective(sca_multi* mp, const sca_opts* opts, const void* X_dev,
                               double* F_host, double* merit_host, int64_t* nnz_host,
                               void* stream);

/* Solve from X (in: start, out: result) until every problem meets the stop of
 * sca_solve (relative objective error against its F*, or merit), checked every
 * check_every rounds; a problem that meets it is frozen (its X column no longer moves)
 * while the others continue.  stats_host: K entries (struct_size set by the caller);
 * coord_updates counts the drawn coordinates of the rounds in which that problem was
 * active, moved_updates the coordinates moved in any problem (shared), MF is not computed
 * (NaN).  Returns SCA_ENOTCONV when a problem did not meet its stop within max_rounds.
 * Synchronises 'stream'. */
sca_status sca_multi_solve(sca_multi* mp, const sca_opts* opts, void* X_dev,
                           sca_stats* stats_host, void* stream);

/* Kernel times of the sca_multi_step / sca_multi_solve calls made with SCA_FLAG_PROFILE
 * (which then launch eagerly, with HIP events around each step), indexed by SCA_K_*
 * (SCA_K_GRAD: the gradient product; SCA_K_COMPACT: best response and listing of the moved
 * coordinates; SCA_K_FOLD: the residual-update product and its reduction); arrays of
 * SCA_K_NKINDS entries.  reset != 0 clears them. */
sca_status sca_multi_profile_get(sca_multi* mp, double* ms_host, int64_t* launches_host,
                                 int reset);

#ifdef __cplusplus
}
#endif

#endif /* SCA_H */
