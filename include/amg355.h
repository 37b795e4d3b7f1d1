/*
 * amg355.h -- C ABI of the MI355X (gfx950) AMG-preconditioned flexible CG.
 *
 * Method: Bernaschi, Celestini, D'Ambra, Vella, "Multi-GPU aggregation-based
 * AMG preconditioner for iterative linear solvers", arXiv 2303.02352.
 *   - Sec. 3, Alg. 1: flexible (Notay) preconditioned conjugate gradient for
 *     A x = b with A symmetric positive definite.
 *   - Sec. 3.1, Alg. 2: V-cycle with l1-Jacobi smoothing, piecewise-constant
 *     restriction / prolongation, direct solve at the coarsest level.
 *   - Sec. 3.1, Alg. 3 and Sec. 4.1: coarsening by 1/2-approximate maximum
 *     weight matching (Suitor), pairwise prolongators composed s times,
 *     Galerkin products P^T A P.
 *   - Sec. 5: stopping rule (relative l2 residual, iteration limit) and the
 *     operator complexity reported by amg_info.
 *
 * All compute runs on the GPU in this library's HIP kernels.  Indices are
 * int32, values IEEE binary64 (float copies for AMG_PREC_MIXED).
 *
 * Errors: every entry point returns an int status (AMG_OK = 0; AMG_NOT_CONVERGED
 * = 1 is a warning; negative values are errors).  No exception, abort or
 * longjmp crosses this boundary.  amg_last_error() returns a thread-local
 * message for the last failure on the calling thread.
 *
 * Threading: a hierarchy may be used by one host thread at a time; different
 * hierarchies may be used from different threads at once.  All work is
 * ordered on the hierarchy's stream (amg_params.stream, or, when it is NULL,
 * a library-owned stream of the hierarchy's own that is ordered with
 * null-stream work); calls that return host-visible results synchronise that
 * stream.
 */
#ifndef AMG355_H
#define AMG355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- statuses */
#define AMG_OK 0
#define AMG_NOT_CONVERGED 1       /* maxit reached with relres > rtol (warning) */
#define AMG_ERR_INVALID (-1)      /* bad argument or malformed / unsymmetric CSR */
#define AMG_ERR_NOT_SPD (-2)      /* a_ii <= 0, Cholesky pivot <= 0, or rho <= 0 in PCG */
#define AMG_ERR_NONFINITE (-3)    /* NaN or Inf in the input or produced by the iteration */
#define AMG_ERR_NOMEM (-4)        /* device allocation failed */
#define AMG_ERR_DEVICE (-5)       /* any other HIP runtime error */
#define AMG_ERR_UNSUPPORTED (-6)  /* a parameter combination the library does not provide */
#define AMG_ERR_MODEL (-7)        /* the learned smooth vector was unusable (non-finite or
                                     non-positive): reported in amg_info_t.smooth_status while
                                     amg_setup falls back to AMG_SMOOTH_RELAX and succeeds */

/* coarse_solver */
#define AMG_COARSE_CHOLESKY 0     /* dense FP64 Cholesky (coarsest n <= 1024, else Jacobi sweeps) */
#define AMG_COARSE_JACOBI 1       /* coarse_sweeps l1-Jacobi sweeps (Sec. 5 setting) */
/* smooth_vec */
#define AMG_SMOOTH_ONES 0         /* w = 1 */
#define AMG_SMOOTH_RELAX 1        /* smooth_sweeps l1-Jacobi sweeps on A w = 0 from w = 1, w /= max|w| */
#define AMG_SMOOTH_GIVEN 2        /* w supplied in amg_params.smooth_vector (e.g. a learned surrogate) */
#define AMG_SMOOTH_LEARNED 3      /* w predicted by the message-passing network (amg_mpnn below)
                                     with amg_params.model_params; relaxation (smooth_sweeps)
                                     when the prediction is unusable.  The network's buffers
                                     (about 224 bytes per fine row) are kept per device until
                                     the process ends and reused by later learned setups, which
                                     take turns on a device */
/* precision */
#define AMG_PREC_DOUBLE 0         /* everything in binary64 */
#define AMG_PREC_MIXED 1          /* V-cycle below the coarsest level in binary32; PCG,
                                     residuals, dots and the coarsest solve in binary64 */
/* value_coding: how the solve kernels read matrix values (results are the
 * same bits either way) */
#define AMG_VALUES_PLAIN 0        /* one binary64 (binary32) value per stored entry */
#define AMG_VALUES_AUTO 1         /* a level whose stored values take at most 256 distinct
                                     bit patterns keeps one byte per entry, an index into a
                                     per-level table of those values; other levels plain */
/* cycle_type (Appendix A option set) */
#define AMG_CYCLE_V 0             /* one coarse-grid correction per level (Alg. 2) */
#define AMG_CYCLE_H 1             /* two corrections on odd levels, one on even levels */
#define AMG_CYCLE_W 2             /* two coarse-grid corrections on every level */
/* relax_type / coarse_relax (Appendix A codes) */
#define AMG_RELAX_JACOBI 0        /* x <- x + (r - A x) / a_ii */
#define AMG_RELAX_GS 1            /* forward Gauss-Seidel before, backward after the correction */
#define AMG_RELAX_SYM_GS 3        /* each sweep a forward then a backward Gauss-Seidel pass */
#define AMG_RELAX_L1_JACOBI 4     /* x <- x + (r - A x) / sum_j |a_ij|  (Sec. 3.1) */
/* bootstrap_type: composition rule of the hierarchies of a bootstrap composite */
#define AMG_BOOTSTRAP_MULT 0      /* B_1, then B_2 on the remaining residual, ... */
#define AMG_BOOTSTRAP_SYMMULT 1   /* B_1 ... B_m, then B_{m-1} ... B_1 */
#define AMG_BOOTSTRAP_ADD 2       /* B_1 + ... + B_m */

/* Square sparse matrix in CSR form.
 *   row_ptr: n+1 entries, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx: nnz entries, strictly ascending within each row, in [0, n),
 *            the diagonal present in every row
 *   val:     nnz entries; A must be bitwise symmetric (a_ij == a_ji) with
 *            a_ii > 0 (s.p.d. is assumed, Sec. 1 and 3; violations found
 *            later surface as AMG_ERR_NOT_SPD)
 *   on_device: 1 if the three arrays are device pointers, 0 if host pointers.
 * The arrays are only read, during amg_setup; the caller keeps ownership. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
  int32_t on_device;
} amg_csr;

/* Method parameters.  amg_params_default() fills:
 *   aggr_steps 2 (aggregates of at most 4), max_levels 40, coarse_max 100,
 *   coarse_solver CHOLESKY, coarse_sweeps 20, pre/post sweeps 4/4,
 *   smooth_vec ONES, smooth_sweeps 20, precond 1, precision DOUBLE,
 *   value_coding AUTO, n_parts 1, cycle_type V, relax_type and coarse_relax
 *   L1_JACOBI, max_hrc 1, bootstrap_type MULT, bootstrap_its 15,
 *   bootstrap_seed 1, bootstrap_rate 0.8, smooth_vector NULL, model_params
 *   NULL, model_path NULL, stream NULL.
 * The paper's own runs (Sec. 5, Appendix A) use aggr_steps 3, coarse_max
 * 40*nd, coarse_solver JACOBI with 20 sweeps. */
typedef struct {
  int32_t aggr_steps;      /* s >= 1: pairwise matching steps composed per level (Sec. 3.1) */
  int32_t max_levels;      /* >= 1, fine level included */
  int32_t coarse_max;      /* >= 1: stop coarsening when n <= coarse_max (Alg. 3) */
  int32_t coarse_solver;   /* AMG_COARSE_* */
  int32_t coarse_sweeps;   /* >= 1 */
  int32_t pre_sweeps;      /* >= 0 */
  int32_t post_sweeps;     /* >= 0 */
  int32_t smooth_vec;      /* AMG_SMOOTH_* */
  int32_t smooth_sweeps;   /* >= 0 */
  int32_t precond;         /* 1: AMG V-cycle; 0: B = I, plain CG (Appendix A) */
  int32_t precision;       /* AMG_PREC_* */
  int32_t value_coding;    /* AMG_VALUES_* */
  int32_t n_parts;         /* 1 .. 2^24: decoupled aggregation (Sec. 4.1): the rows of every
                              level are split into n_parts blocks of consecutive rows (block p
                              = [floor(p n / n_parts), floor((p+1) n / n_parts)) on the fine
                              level; a coarse row belongs to the block of its aggregate) and
                              each block is matched on its own subgraph: edges between blocks
                              are never matched, so P is block diagonal.  1 = one block. */
  int32_t cycle_type;      /* AMG_CYCLE_* */
  int32_t relax_type;      /* AMG_RELAX_*: pre- and post-smoother */
  int32_t coarse_relax;    /* AMG_RELAX_*: the coarsest-level sweeps when they are used */
  int32_t max_hrc;         /* 1 .. 16: bootstrap composite of at most max_hrc hierarchies */
  int32_t bootstrap_type;  /* AMG_BOOTSTRAP_* */
  int32_t bootstrap_its;   /* >= 1: composite iterations on A x = 0 per rate estimate */
  int32_t bootstrap_seed;  /* seed of the bootstrap's random start vectors */
  double bootstrap_rate;   /* (0, 1]: desired convergence rate of the composite */
  const double *smooth_vector; /* n values, same memory space as the CSR, for AMG_SMOOTH_GIVEN */
  const float *model_params;   /* AMG_SMOOTH_LEARNED: AMG_MPNN_NPARAMS floats in host memory */
  const char *model_path;      /* AMG_SMOOTH_LEARNED without model_params: a file of the
                                  parameters, read by amg_mpnn_read_params; a file that
                                  cannot be read is an unusable model (relaxation is used and
                                  smooth_status reports AMG_ERR_MODEL) */
  void *stream;            /* hipStream_t on which the solve-phase work is ordered; NULL =
                              a blocking stream the library keeps for this hierarchy alone
                              (reused after amg_destroy).  A caller's stream must stay
                              valid until amg_destroy.  amg_setup waits for the work
                              already on it, runs on a library stream that lives for the
                              process (the hierarchy's device memory comes from the
                              device's memory pool and is only ever freed on such
                              streams), and returns with the setup finished.  Objects may
                              share a stream; their work on it is then serialised, and
                              every call that synchronises (amg_pcg_solve, ...) waits for
                              all of it. */
} amg_params;

typedef struct amg_hierarchy amg_hierarchy;   /* opaque, owned by the library */

#define AMG_MAX_LEVELS 64
#define AMG_MAX_HRC 16
typedef struct {
  int32_t levels;
  int32_t n[AMG_MAX_LEVELS];
  int64_t nnz[AMG_MAX_LEVELS];
  double opc;                   /* sum_k nnz(A_k) / nnz(A_0)  (Sec. 5) */
  int32_t coarse_dense;         /* 1 if the coarsest level is solved by Cholesky */
  int32_t matching_rounds;      /* total GPU matching rounds over all pairwise steps */
  double setup_ms;              /* wall time of amg_setup (stream-synchronised) */
  double setup_match_ms;        /* part spent in weights + matching + aggregation */
  double setup_rap_ms;          /* part spent in Galerkin products */
  int64_t device_bytes;         /* device memory held by the hierarchy */
  int32_t dict_size[AMG_MAX_LEVELS]; /* distinct values of a coded level's table, 0 = plain */
  double setup_smooth_ms;       /* part spent on the fine smooth vector (relaxation or copy) */
  int32_t nhrc;                 /* hierarchies in the bootstrap composite (1 without) */
  int32_t nrates;               /* rate estimates taken by the bootstrap */
  double rates[AMG_MAX_HRC];    /* rates[j-1]: estimated rate of the first j hierarchies */
  double setup_bootstrap_ms;    /* part spent on rate estimates and further hierarchies */
  int32_t smooth_status;        /* AMG_OK, or AMG_ERR_MODEL when LEARNED fell back to RELAX */
} amg_info_t;

/* Fill *p with the defaults above.  Returns AMG_OK or AMG_ERR_INVALID (p NULL). */
int amg_params_default(amg_params *p);

/* Build the hierarchy (Alg. 3 with s-step composition, Sec. 3.1/4.1) on the
 * GPU: validate A, copy it to library-owned device memory, compute the smooth
 * vector, then per level match / aggregate / form P / Galerkin product, and
 * factor the coarsest matrix.  The result is deterministic: aggregate maps,
 * coarse patterns and coarse values do not depend on thread scheduling.
 * On success *h_out owns all device memory; release it with amg_destroy.
 * Errors: INVALID (NULL args, bad parameters, malformed or unsymmetric CSR),
 * NOT_SPD (a_ii <= 0 or a non-positive Cholesky pivot), NONFINITE, NOMEM,
 * DEVICE, UNSUPPORTED (a level whose sliced storage -- 64 rows per slice, each
 * slice as wide as its longest row -- would need 2^31 or more slots; slot
 * offsets are int32).  On error *h_out is NULL. */
int amg_setup(const amg_csr *A, const amg_params *p, amg_hierarchy **h_out);

/* Solve A x = b with flexible PCG (Alg. 1) preconditioned by one V-cycle
 * (Alg. 2) per iteration.  b, x: device pointers to n doubles; x holds the
 * initial guess on entry and the solution on exit; b is not modified.
 * Stops when ||r_i||_2 <= rtol ||r_0||_2 (recurrence residual, tested after
 * every update of r) or after maxit iterations (Sec. 5).  *iters_out = number
 * of preconditioner applications (0 when r_0 = 0); *relres_out = ||r||/||r_0||.
 * Returns OK, NOT_CONVERGED, NOT_SPD (rho <= 0), NONFINITE, INVALID (rtol <= 0,
 * maxit < 1, NULL), DEVICE.  Synchronises the hierarchy's stream. */
int amg_pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                  int32_t *iters_out, double *relres_out);

/* The same solve as amg_pcg_solve, for callers that cannot allocate memory
 * during a solve (tight serving loops, harnesses that forbid allocation): it
 * calls no hipMalloc, hipFree, graph instantiation or event creation.  The
 * PCG scalars and the partial sums of the fine-level reductions live in a
 * static device array of 4 MiB, one per device, held until the process ends
 * (its address is looked up once per device by amg_setup); everything else
 * is the hierarchy's, allocated by amg_setup.  Each iteration's kernels are
 * launched one by one (no graph), and the host waits by polling the scalars
 * the GPU copies to the hierarchy's pinned memory.  Results are bit-identical
 * to amg_pcg_solve's.
 * Limit: n_0 <= amg_pcg_solve_noalloc_max_rows() (89,473,024 rows); a larger
 * hierarchy gives AMG_ERR_INVALID before any work is queued.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (from different host
 * threads, or on streams that run concurrently) race and give wrong results.
 * Arguments, statuses and synchronisation as amg_pcg_solve. */
int amg_pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol,
                          int32_t maxit, int32_t *iters_out, double *relres_out);
int64_t amg_pcg_solve_noalloc_max_rows(void);

/* Release everything held by h.  NULL-safe.  Synchronises the stream first. */
void amg_destroy(amg_hierarchy *h);

/* Static description of a status code. */
const char *amg_strerror(int code);

/* Message for the last failure on the calling thread ("" if none). */
const char *amg_last_error(void);

/* Sizes, operator complexity and setup timings. */
int amg_info(const amg_hierarchy *h, amg_info_t *out);

/* Hierarchy j (0-based) of a bootstrap composite, j = 0 being h itself:
 * a borrowed handle, owned by h and valid until amg_destroy(h), for
 * amg_info, amg_export_level, amg_vcycle (which then applies that
 * hierarchy's own V-cycle), amg_spmv and amg_sweep, all ordered on h's
 * stream; never pass it to amg_destroy.  NULL (and INVALID as the last
 * error) when j is out of range. */
amg_hierarchy *amg_component(amg_hierarchy *h, int32_t j);

/* Introspection for parity tests: copy level k to HOST buffers (any may be
 * NULL).  row_ptr n_k+1, col_idx/val nnz_k (canonical CSR, columns
 * ascending), dinv n_k (1 / l1 row sum), w n_k (smooth vector), and for
 * k < levels-1 agg n_k (row of level k+1 holding fine row i) and pval n_k
 * (the one nonzero of row i of the composite prolongator).  Synchronises. */
int amg_export_level(const amg_hierarchy *h, int32_t k, int32_t *row_ptr, int32_t *col_idx,
                     double *val, double *dinv, double *w, int32_t *agg, double *pval);

/* z = B r: one V-cycle of Alg. 2 (B = I when precond = 0); with a bootstrap
 * composite, its composition of the hierarchies' V-cycles.  r, z: device
 * pointers to n_0 doubles, may not alias.  Enqueued on the stream; returns
 * without synchronising. */
int amg_vcycle(amg_hierarchy *h, const double *r, double *z);

/* y = A_k x on level k with the solve-phase SpMV kernel.  Device pointers to
 * n_k doubles, may not alias.  Enqueued on the stream, not synchronised. */
int amg_spmv(amg_hierarchy *h, int32_t k, const double *x, double *y);

/* One l1-Jacobi sweep on level k with the solve-phase kernel:
 * xn = x + (r - A_k x) / M_k.  Device pointers, xn must not alias x or r. */
int amg_sweep(amg_hierarchy *h, int32_t k, const double *r, const double *x, double *xn);

/* Timing of one solve-phase kernel in its solve launch configuration:
 * kernel 0 = SpMV (+3 dots) on level k, 1 = l1-Jacobi sweep on level k,
 * 2 = residual + restriction from level k, 3 = prolongation into level k,
 * 4 = the fused PCG vector update (level 0 only), 5 = prolongation into
 * level k fused with the first post-smoothing sweep.  It is launched `reps`
 * times on the hierarchy's stream between two HIP events on that stream,
 * operating on the hierarchy's own work vectors; *avg_ms is the mean
 * duration and *bytes the algorithmic bytes one launch moves.  Synchronises. */
int amg_time_kernel(amg_hierarchy *h, int32_t kernel, int32_t k, int32_t reps, double *avg_ms,
                    double *bytes);


/* ------------------------------------------------------------------ batched
 * Many independent systems, each with nrhs right-hand sides, solved together
 * (every (system, right-hand side) pair is its own flexible CG, Alg. 1, with
 * its own stopping test).  The hierarchies are built per system with the
 * single-system setup and stacked level by level; vectors are RHS-
 * interleaved.  The iterations run as hipGraph launches of two iterations
 * each, the host checking between launches whether every pair has converged;
 * converged pairs stay frozen, so per-pair iteration counts are exact.  Every
 * system must end in a direct coarsest solve (coarse_solver CHOLESKY,
 * coarsest n <= 1024). */
typedef struct amg_batch amg_batch;   /* opaque, owned by the library */

typedef struct {
  int32_t nsys;
  int32_t levels;                     /* depth of the deepest system */
  int32_t n[AMG_MAX_LEVELS];          /* stacked rows per level */
  int32_t n_smoothed[AMG_MAX_LEVELS]; /* rows of systems that continue below the level */
  int64_t nnz[AMG_MAX_LEVELS];
  int32_t cols_per_lane[AMG_MAX_LEVELS];  /* tuned: lanes per row = nrhs / cols_per_lane */
  double setup_ms, tune_ms;
  int32_t cols_per_lane_corr[AMG_MAX_LEVELS];  /* tuned, for the sweep that adds the coarse correction */
  int32_t tile_rows;                  /* rows per reduction tile of the level-0 PCG kernels (fixed: the
                                         dot products fold per tile, so it sets their rounding) */
  int32_t spmm_cols;                  /* right-hand-side columns per thread of the level-0 SpMM + dots (fixed) */
} amg_batch_info_t;

/* Build the hierarchies of nsys systems A[0..nsys-1] (same parameters for
 * all; smooth_vec GIVEN is not accepted).  Errors as amg_setup, plus
 * UNSUPPORTED when a system does not end in a direct coarsest solve.  The
 * systems are set up by up to 8 host threads at once; the environment
 * variable AMG_BUILD_THREADS (1 .. 8) lowers that number.  The first solve
 * with a given nrhs also times the sweep variants (columns per lane, which do
 * not change any result bit; the picks are reported by amg_batch_info). */
int amg_batch_setup(int32_t nsys, const amg_csr *A, const amg_params *p, amg_batch **out);

/* Solve A_s X_s = B_s for every system s.  B, X: device pointers; systems are
 * stored one after another in the order given to amg_batch_setup, each as an
 * n_s x nrhs row-major block (entry (i, c) of system s at (off_s + i) * nrhs + c,
 * off_s = n_0 + ... + n_{s-1}).  X holds initial guesses on entry.  nrhs in
 * {1, 2, 4, 8, 16}.  Outputs (host arrays of nsys * nrhs, index s * nrhs + c):
 * iterations, recurrence relative residual, status of the pair.  Returns the
 * most severe pair status (OK, NOT_CONVERGED or an error).  The first call
 * with a given nrhs allocates vectors, times the smoothing-kernel variants
 * and captures the iteration graph.  Synchronises. */
int amg_batch_solve(amg_batch *bt, int32_t nrhs, const double *B, double *X, double rtol,
                    int32_t maxit, int32_t *iters, double *relres, int32_t *status);

/* amg_batch_solve with one pair of vectors per system: B[s], X[s] (host arrays
 * of nsys device pointers, s in the order given to amg_batch_setup), each an
 * n_s x nrhs row-major block (entry (i, c) at i * nrhs + c).  Same outputs,
 * errors and results as amg_batch_solve; INVALID when a pointer is NULL. */
int amg_batch_solve_systems(amg_batch *bt, int32_t nrhs, const double *const *B, double *const *X,
                            double rtol, int32_t maxit, int32_t *iters, double *relres,
                            int32_t *status);

/* Z = B_s R for every system and right-hand side (one batched V-cycle), same
 * layout as amg_batch_solve.  Synchronises. */
int amg_batch_vcycle(amg_batch *bt, int32_t nrhs, const double *R, double *Z);

int amg_batch_info(const amg_batch *bt, amg_batch_info_t *out);

/* NULL-safe. */
void amg_batch_destroy(amg_batch *bt);

/* ------------------------------------------------- learned smooth vector
 * A two-layer message-passing network over the graph of A that predicts
 * log w, w being the smooth vector that drives the matching weights (Sec. 3.1
 * leaves its source open; the targets are the method's own relaxation
 * vectors, AMG_SMOOTH_RELAX).  Node features (8): 1, log(a_ii)/4,
 * s_i/a_ii with s_i = sum_{j!=i}|a_ij|, two l1-Jacobi sweeps on A w = 0 from
 * ones, log(max/min off-diagonal |a_ij|)/4, (#off-diagonals)/6, 0.
 * Aggregation (Ahat X)_i = sum_{j!=i}|a_ij| X_j / s_i.
 *   h1 = ReLU([X | Ahat X] W1 + b1), h2 = ReLU([h1 | Ahat h1] W2 + b2),
 *   y = h2 wh + bh,  w = exp(y).
 * Parameters (binary32, flat): W1 16x32 row-major, b1[32], W2 64x32, b2[32],
 * wh[32], bh[1].  Dense products read bfloat16 activations and weights and
 * accumulate in binary32 (MFMA).  The CSR must be in device memory. */
#define AMG_MPNN_NPARAMS 2657
typedef struct amg_mpnn amg_mpnn;

/* params: host array of AMG_MPNN_NPARAMS floats (NULL = all zero).
 * stream: hipStream_t (NULL = a library-owned stream). */
int amg_mpnn_create(const float *params, void *stream, amg_mpnn **out);
/* Read AMG_MPNN_NPARAMS parameters from a text file into the host array
 * params: the numbers of the first [...] list after a "params" key (the JSON
 * model files the Python module writes), or, in a file without that key,
 * its first AMG_MPNN_NPARAMS numbers (separated by white space or commas).
 * Host only (no device needed).  Errors: INVALID (NULL argument), MODEL
 * (file unreadable, too few numbers, or text that is not a number). */
int amg_mpnn_read_params(const char *path, float *params);
/* Copy the current parameters to a host array of AMG_MPNN_NPARAMS floats. */
int amg_mpnn_get_params(const amg_mpnn *m, float *params);
/* Node features as the network stores them (bfloat16 values widened to
 * binary32), host array of 8 n floats, row-major.  Synchronises. */
int amg_mpnn_features(amg_mpnn *m, const amg_csr *A, float *X_host);
/* Predict: w_out (device, n doubles) = exp(y) and/or y_host (host, n floats). */
int amg_mpnn_predict(amg_mpnn *m, const amg_csr *A, double *w_out, float *y_host);
/* One training step on one graph: loss = mean (y - log w_target)^2 with
 * w_target a device array of n positive doubles; the gradient is copied to
 * grad_host (host, AMG_MPNN_NPARAMS floats) when given; then one Adam step
 * (beta 0.9 / 0.999) with learning rate lr (lr = 0: no update).  Synchronises. */
int amg_mpnn_train_step(amg_mpnn *m, const amg_csr *A, const double *w_target, float lr,
                        float *loss_out, float *grad_host);
/* NULL-safe. */
void amg_mpnn_destroy(amg_mpnn *m);

#ifdef __cplusplus
}
#endif
#endif /* AMG355_H */
