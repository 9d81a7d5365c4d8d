/*
 * iccg.h -- C ABI of the MI355X block-multicolored ICCG library (libiccg.so).
 *
 * The library solves A x = b for a symmetric positive definite sparse A with
 * the conjugate gradient method preconditioned by IC(0), applied by forward
 * and backward substitution over a block-multicolored ordering, as studied in
 * "Comparison of Algebraic Block Multi-Coloring and Leiden Methods for
 * Parallel Preconditioning in the ICCG Method":
 *   - Section 3: ABMC blocking, block coloring, Algorithm 1 (forward
 *     substitution: colors in sequence, the blocks of one color in parallel,
 *     the rows of a block in ascending order), backward substitution in
 *     reverse order;
 *   - Section 4: Leiden blocking with modularity (Eq. 1) or CPM (Eq. 2);
 *   - Section 5: stopping rule ||r||_2 / ||b||_2 <= tol;
 *   - Section 6.1 / 7.1: greedy block coloring; Leiden blocks numbered by
 *     descending size.
 *
 * Conventions for every function:
 *   - int32 indices; CSR with ascending column indices inside each row and the
 *     diagonal stored; nnz < 2^31.
 *   - Host pointers are read during the call only and stay owned by the
 *     caller.  "Device" pointers are HIP device memory owned by the caller
 *     (for example torch tensors); the library never frees them.
 *   - Every call returns an int status (ICCG_OK = 0 or a negative ICCG_E*);
 *     no exception crosses the ABI.  iccg_last_error() gives a message for
 *     the calling thread's last failure.
 *   - A context is not thread safe; distinct contexts are independent.
 *     Device work is enqueued on the context's stream (iccg_options.stream);
 *     functions that return host-visible results synchronize that stream.
 */
#ifndef ICCG_H
#define ICCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ICCG_OK          0
#define ICCG_EINVAL     -1  /* bad argument (null pointer, size, option)            */
#define ICCG_EPATTERN   -2  /* pattern not symmetric, diagonal missing, unsorted    */
#define ICCG_EBADORDER  -3  /* block_ptr/color_ptr malformed or same-color blocks adjacent */
#define ICCG_EBREAKDOWN -4  /* non-positive or non-finite IC(0) pivot               */
#define ICCG_ENOCONV    -5  /* maxit reached before the tolerance                    */
#define ICCG_ENAN       -6  /* (p, Ap) <= 0 or a non-finite CG scalar                */
#define ICCG_EHIP       -7  /* HIP runtime error                                     */
#define ICCG_ENOMEM     -8  /* device or host allocation failed                      */
#define ICCG_ESTATE     -9  /* call out of order (e.g. ic_apply before a factor)     */

#define ICCG_FP64 0
#define ICCG_FP32 1

#define ICCG_QUALITY_MODULARITY 0
#define ICCG_QUALITY_CPM        1

typedef struct iccg_ctx iccg_ctx;

typedef struct {
    int   precision;    /* ICCG_FP64: factor and sweeps in FP64.  ICCG_FP32: factor
                           stored and sweeps computed in FP32 (r is rounded to FP32
                           on load, z widened to FP64 on store); CG vectors, dots and
                           residuals stay FP64 either way.                        */
    void *stream;       /* hipStream_t for all device work; NULL = null stream    */
    int   check_every;  /* CG iterations enqueued between host reads of the
                           device-side convergence flag (>= 1, default 32)        */
    int   pack_rows;    /* max rows one wavefront task packs from consecutive small
                           blocks of one color (1..64, default 64)                */
    int   use_graph;    /* 1 = replay the iteration batch as a captured HIP graph  */
    int   sweep_launch; /* 0 = one kernel launch per color (default); 1 = one
                           persistent launch per sweep, each wavefront task waiting
                           only for the earlier-color tasks it reads; 2 = hybrid:
                           one launch per large color, and the small last colors
                           of the forward sweep (first of the backward sweep) in
                           one such dataflow launch.  Same arithmetic and
                           bit-identical results in all three.  Modes 1 and 2
                           need every workgroup of the dataflow launch resident
                           and the runtime's round-robin XCD placement; a failed
                           placement check or a dependency wait beyond its spin
                           limit makes the call return ICCG_EHIP, naming the
                           cause (iccg_last_error), and its output is invalid.
                           Every wave still exits.                               */
    int   sweep_grid;   /* single-launch sweep: its workgroups, all of which must
                           be resident at once (0 = 8 per compute unit; otherwise
                           this many, bounded by the resident capacity and rounded
                           down to a multiple of 8, at least 8)                  */
    int   flow_tail;    /* hybrid sweeps: at most this many tasks in the dataflow
                           part (0 = 700)                                       */
    int   wide_blocks;  /* per-color launches: a block of more than 256 rows is
                           run by one workgroup in pieces of 64 rows per
                           wavefront, each piece level-scheduled as a whole (1,
                           default): 16 wavefronts and 1,024-row pieces when no
                           row of the sweep has more than 8 entries, else 8
                           wavefronts and 512-row pieces; or (0) by one
                           wavefront in 64-row chunks.
                           The forward sweep is bit-identical either way; the
                           backward sweep's per-row sums group the entries by
                           piece instead of by chunk (equal up to rounding).   */
    int   host_factor;  /* ic0_factor on the device over the forward sweep's
                           schedule (0, default) or serially on the host (1);
                           both give the serial FP64 factorization bit for bit */
    int   fuse_turn;    /* per-color sweeps inside iccg_solve: the last color's
                           forward and backward substitutions in one launch, task
                           by task (1, default; bit-identical), or in two (0)  */
} iccg_options;

/* Fills *opt with the defaults above (FP64, null stream, 32, 64, 1, 0, 0, 0, 1, 0, 1). */
void iccg_default_options(iccg_options *opt);

/* ------------------------------------------------------------------------ */
/* Host setup: ordering (deterministic for given inputs and seed)            */
/* ------------------------------------------------------------------------ */

/*
 * ABMC blocking with block size block_size (Section 3; s = ceil(n/n_b),
 * Section 6.1), greedy block coloring (Section 6.1), color-major numbering.
 * Inputs: pattern of A (rowptr[n+1], col[nnz]); values are not needed.
 * Outputs (caller-allocated): perm[n] with perm[new] = old; *nblocks;
 * block_ptr[nblocks+1] (capacity n+1): first new row of every block;
 * *ncolors; color_ptr[ncolors+1] (capacity n+1): first block of every color.
 * Blocks are numbered colors-first; within a color in blocking order; rows of
 * a block keep ascending original index.
 */
int iccg_order_abmc(int n, const int *rowptr, const int *col, int block_size,
                    int *perm, int *nblocks, int *block_ptr, int *ncolors, int *color_ptr);

/*
 * Leiden blocking (Section 4; Section 7.1 settings: beta = 0.01, two
 * iterations) of the unweighted pattern graph with quality
 * ICCG_QUALITY_MODULARITY (Eq. 1, resolution gamma) or ICCG_QUALITY_CPM
 * (Eq. 2, resolution gamma); blocks renumbered by descending size (ties: the
 * block holding the smaller original index first), then greedy coloring and
 * color-major numbering as for ABMC.  Randomness: one SplitMix64 stream seeded
 * with seed.  Outputs as iccg_order_abmc.
 */
int iccg_order_leiden(int n, const int *rowptr, const int *col, int quality, double gamma,
                      double beta, int n_iter, uint64_t seed,
                      int *perm, int *nblocks, int *block_ptr, int *ncolors, int *color_ptr);

/*
 * Load-imbalance statistics of an ordering (Section 7.3, Table 6):
 * out[0] n_b, out[1] n_c, out[2] the Gini coefficient G of the block sizes
 * (sum over all ordered pairs of |s_i - s_j| divided by 2 n_b^2 times the mean
 * size), out[3] B_max, out[4] B_max / B_avg, out[5] C_max / C_avg (rows of the
 * largest color over the mean rows per color).  block_ptr[nblocks+1] and
 * color_ptr[ncolors+1] as returned by the ordering calls; out: host double[6].
 * ICCG_EBADORDER for an empty block or color or pointers that do not start at
 * 0; host only.
 */
int iccg_block_stats(int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                     double *out);

/*
 * A' = P A P^T (perm[new] = old) with sorted columns.  prow[n+1], pcol[nnz],
 * pval[nnz] are caller-allocated.
 */
int iccg_permute(int n, const int *rowptr, const int *col, const double *val, const int *perm,
                 int *prow, int *pcol, double *pval);

/* ------------------------------------------------------------------------ */
/* Device path                                                               */
/* ------------------------------------------------------------------------ */

/*
 * Create a context for the permuted SPD matrix A' (host CSR; deep-copied to
 * the device) and its ordering block_ptr[nblocks+1], color_ptr[ncolors+1].
 * Validates: symmetric pattern, sorted columns, diagonal present
 * (ICCG_EPATTERN); block_ptr monotone from 0 to n, color_ptr monotone from 0
 * to nblocks, and no stored a'_ij joining two different blocks of one color
 * (ICCG_EBADORDER).  Builds the per-wavefront substitution schedules for both
 * sweeps.  opt may be NULL (defaults).  *out is NULL on failure.  An empty
 * matrix (n < 1) is rejected with ICCG_EINVAL; non-finite values likewise.
 */
int iccg_setup(iccg_ctx **out, int n, const int *rowptr, const int *col, const double *val,
               int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
               const iccg_options *opt);

/*
 * IC(0) factor of A' (Section 3): L with pattern(L) = lower(A') and
 * (L L^T)_ij = a'_ij on that pattern, in FP64 (rounded to FP32 for the sweeps
 * of ICCG_FP32).  By default on the device: one launch per color over the
 * forward sweep's schedule (blocks of a color in parallel, the rows of a
 * chunk level by level), each row computed in the serial order of operations
 * without fused multiply-adds, so the result equals the serial
 * factorization bit for bit; iccg_options.host_factor = 1 computes it
 * serially on the host instead.  On a pivot that is not > 0 or not finite
 * returns ICCG_EBREAKDOWN with *breakdown_row set to the first such row
 * (else -1); the context then holds no factor.
 */
int ic0_factor(iccg_ctx *c, int *breakdown_row);

/*
 * Install factor values computed elsewhere (the learned form) on the same
 * pattern: lvals_dev is a DEVICE array of nnz FP64 values at the positions of
 * A''s CSR, lower triangle including the diagonal used, upper ignored.
 * Checks every diagonal entry is finite and > 0 and every off-diagonal value
 * finite; on failure returns ICCG_EBREAKDOWN with *bad_row set and keeps the
 * previous factor.
 */
int iccg_set_factor(iccg_ctx *c, const double *lvals_dev, int *bad_row);

/* Reinstall the IC(0) factor computed by ic0_factor (the learned form's
 * fallback).  ICCG_ESTATE if ic0_factor has not succeeded on this context. */
int iccg_restore_ic0(iccg_ctx *c);

/* Copy the current factor (A' CSR positions, upper part zero) to host lvals[nnz]. */
int iccg_get_factor(iccg_ctx *c, double *lvals);

/*
 * Preconditioner application z = (L L^T)^{-1} r (Algorithm 1 and the
 * backward sweep).  r, z: DEVICE FP64 arrays of n; r is not modified; r and
 * z must not alias.
 */
int ic_apply(iccg_ctx *c, const double *r, double *z);

/* Forward sweep only, y = L^{-1} r (Algorithm 1).  DEVICE FP64 r, y. */
int ic_forward(iccg_ctx *c, const double *r, double *y);

/* Backward sweep only, z = L^{-T} y.  DEVICE FP64 y, z. */
int ic_backward(iccg_ctx *c, const double *y, double *z);

/* q = A' p (the CG step's SpMV); *pq_host (may be NULL) receives (p, q). DEVICE p, q. */
int iccg_spmv(iccg_ctx *c, const double *p, double *q, double *pq_host);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): iccg_spmv
 * with the dot product left on the device.  q = A'p and *pq_dev = (p, q)
 * (DEVICE p, q of n; pq_dev: one DEVICE double), enqueued on the context's
 * stream with no host synchronization; results equal iccg_spmv's bit for bit.
 * The per-workgroup partial sums live in a library-wide static device array of
 * 2^18 doubles (2 MiB per GPU, held until the process ends), so the call
 * allocates nothing; every partial is rewritten before it is read, so nothing
 * needs clearing.  All calls on one GPU share that array: calls that overlap
 * on one GPU (other streams, other threads) race.  ICCG_EINVAL for n > 2^24
 * rows, for null or equal p and q, or a null pq_dev.
 */
int iccg_spmv_dot_noalloc(iccg_ctx *c, const double *p, double *q, double *pq_dev);

/* *out_host = (a, b), deterministic two-pass FP64 reduction.  DEVICE a, b of n. */
int iccg_dot(iccg_ctx *c, const double *a, const double *b, double *out_host);

/*
 * PCG on A' x = b (Section 5): x = x0 (DEVICE, in/out), r = b - A'x, z = M^{-1} r,
 * p = z; per iteration q = A'p, alpha = (r,z)/(p,q), x += alpha p, r -= alpha q,
 * stop when ||r||_2/||b||_2 <= tol, else z = M^{-1} r, beta = (r,z)_new/(r,z),
 * p = z + beta p.  Outputs: *iters, *relres (recursive), *relres_true
 * (||b - A'x||/||b|| recomputed at exit); any may be NULL.  Returns ICCG_OK,
 * ICCG_ENOCONV (x = last iterate), ICCG_ENAN, or ICCG_ESTATE without a factor.
 * b, x: DEVICE FP64 arrays of n.
 */
int iccg_solve(iccg_ctx *c, const double *b, double *x, double tol, int maxit,
               int *iters, double *relres, double *relres_true);

/*
 * Blocks of right-hand sides: repeated solves that reuse one ordering and one
 * factor (the paper amortizes the blocking cost over repeated solves,
 * Sections 7.6 and 10).  k independent PCG solves, 1 <= k <= 16, whose
 * kernels read A' and the factor once for all k columns (a workgroup of k
 * wavefronts per sweep task and per SpMV slice, one wavefront per column).
 * B, X: DEVICE FP64 [k][n], column-major (column j at offset j * n); X holds
 * x0 on entry and the solutions on exit.  iters, relres, relres_true: host
 * arrays of k (any may be NULL), per column as for iccg_solve.  Each column
 * computes exactly what iccg_solve computes for it (same iterations, same x
 * bit for bit) when the context has no wide tasks (wide_blocks = 0 or no
 * block of more than 256 rows); with wide tasks the backward sweep's per-row
 * sums group the terms by chunk instead of by piece (equal up to rounding).
 * Returns ICCG_OK when every column converged, ICCG_ENAN if any column broke
 * down, else ICCG_ENOCONV; ICCG_EINVAL for k outside [1, 16].  The context
 * keeps work buffers of 7 k n doubles after the first call.
 */
int iccg_solve_multi(iccg_ctx *c, int k, const double *B, double *X, double tol, int maxit,
                     int *iters, double *relres, double *relres_true);

/* Z = (L L^T)^{-1} R column by column for k <= 16 columns (DEVICE FP64
 * [k][n] column-major, no aliasing); each column equals ic_apply's output for
 * it (under the wide-task condition of iccg_solve_multi). */
int ic_apply_multi(iccg_ctx *c, int k, const double *R, double *Z);

/* Q = A' P column by column for k <= 16 columns (DEVICE FP64 [k][n]
 * column-major); each column equals iccg_spmv's output for it. */
int iccg_spmv_multi(iccg_ctx *c, int k, const double *P, double *Q);

/*
 * iccg_solve run eagerly with a HIP event pair around every SpMV and every
 * per-color sweep launch (the phase split of the paper's Table 8: forward
 * substitution, backward substitution, SpMV, other).  Same arguments and
 * return as iccg_solve; out[10] (host) receives: [0] device time of the solve
 * in ms, [1] SpMV ms, [2] forward-sweep ms, [3] backward-sweep ms (sums of
 * per-launch durations), [4] the rest (reductions, vector updates, launch
 * gaps), [5] forward launches, [6] backward launches, [7] SpMV launches,
 * [8] iterations, [9] true relative residual.
 */
int iccg_profile_solve(iccg_ctx *c, const double *b, double *x, double tol, int maxit,
                       double *out);

/* Residual history of the last iccg_solve: hist[k] = ||r_k||/||b||, k = 0..iters
 * (capacity cap); returns the number written or a negative status. */
int iccg_residual_history(iccg_ctx *c, double *hist, int cap);

typedef struct {
    int    n, nnz, nnz_lower;      /* nnz_lower: strictly lower entries          */
    int    nblocks, ncolors;
    int    ntasks_fwd, nchunks_fwd; /* wavefront tasks / 64-row chunks, forward   */
    int    max_block, max_depth;    /* largest block; deepest intra-chunk level   */
    int    precision;
    int    has_factor;
    double sweep_bytes;             /* algorithmic bytes of one sweep (precision) */
    double spmv_bytes;              /* algorithmic bytes of one SpMV              */
    double last_solve_ms;           /* device time of the last iccg_solve         */
    int    last_iters;
    int    sweep_resident;          /* single-launch sweep: workgroups of the last
                                       launch (0 before the first)                */
    long long remote_tasks;         /* single-launch sweep (forward schedule):
                                       tasks with a dependency in another region  */
    long long exported_rows;        /* rows written through for other regions     */
    double gini;                    /* Table 6 statistics of the context's ordering */
    double bmax_over_avg;           /* (as iccg_block_stats)                      */
    double cmax_over_avg;
} iccg_info;

int iccg_get_info(iccg_ctx *c, iccg_info *info);

/* ------------------------------------------------------------------------ */
/* Learned factor form                                                       */
/* ------------------------------------------------------------------------ */
/*
 * A message-passing network that predicts corrections to the IC(0) factor
 * values on the same pattern; the sweeps are unchanged.  (The paper has no
 * learned component; this is the added learned-factor form.)  In the scaled
 * space s_i = 1/sqrt(a'_ii), A~ = S A' S, L~0 = S L0:
 *   node features [L~0_ii, sum_{j!=i}|A~_ij|, deg_i/26];
 *   edge features [A~_ij, j<i, j==i, L~0 at the lower position of (i,j)];
 *   3 layers, width 32: h_i <- relu(W_s h_i + b + sum_{j!=i} relu(W_m [h_j; f_ij] + b_m));
 *   readout on lower entries (i,j), j<=i: d = w_o . relu(W_r [h_i; h_j; f_ij] + b_r) + b_o;
 *   factor L_ij = L0_ij + 0.1 d / s_i (so w_o = 0, b_o = 0 reproduces IC(0) exactly);
 *   training loss: mean over probes z of ||L~ L~^T z - A~ z||^2 / ||A~ z||^2.
 * Parameters (FP32, iccg_mpnn_param_count() of them): per layer W_s[32][d], b[32],
 * W_m[32][d+4], b_m[32] with d = 3, 32, 32; then W_r[32][68], b_r[32], w_o[32],
 * b_o; matrices row-major.  Contexts used with a network need ic0_factor first.
 */
typedef struct iccg_mpnn iccg_mpnn;

int  iccg_mpnn_param_count(void);
/* params: host FP32 array of iccg_mpnn_param_count(); stream: hipStream_t or NULL */
int  iccg_mpnn_create(iccg_mpnn **out, const float *params, void *stream);
int  iccg_mpnn_get_params(iccg_mpnn *m, float *params);
/* replaces the parameters and resets the Adam state */
int  iccg_mpnn_set_params(iccg_mpnn *m, const float *params);
/*
 * Probe loss and its gradient for the matrix of context c (FP32 forward and
 * backward kernels).  probes: DEVICE FP64 [nprobes][n] (row-major, one probe
 * per row, drawn by the caller).  *loss (host, may be NULL); grad: host FP32
 * array of param_count (may be NULL).
 */
int  iccg_mpnn_loss_grad(iccg_mpnn *m, iccg_ctx *c, const double *probes, int nprobes,
                         double *loss, float *grad);
/* One training step: loss, gradient and an Adam update (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias corrected) with learning rate lr.  *loss may be NULL (then the
 * call does not synchronize). */
int  iccg_mpnn_train_step(iccg_mpnn *m, iccg_ctx *c, const double *probes, int nprobes,
                          float lr, double *loss);
/* Inference: the predicted factor of A' into DEVICE lvals[nnz] (A' CSR positions,
 * upper part 0), ready for iccg_set_factor.  bf16 = 1 stores weights and
 * activations in BF16 (FP32 accumulation); 0 runs in FP32. */
int  iccg_mpnn_predict(iccg_mpnn *m, iccg_ctx *c, int bf16, double *lvals);
/* Smoothed training probes for the matrix of context c: for each of the
 * nprobes rows z_i of the DEVICE FP64 array z[nprobes][n] (row-major, drawn by
 * the caller), out_i = D^{1/2} M^{-1} D^{1/2} z_i rescaled to 2-norm sqrt(n),
 * with D = diag(A') and M = L L^T the context's current factor (the plain
 * IC(0) factor for training).  out: DEVICE FP64 [nprobes][n], not aliasing z.
 * ICCG_ESTATE without a factor. */
int  iccg_mpnn_smooth_probes(iccg_ctx *c, const double *z, int nprobes, double *out);
void iccg_mpnn_destroy(iccg_mpnn *m);

/* Host only: no device call, no context.  Checks the permuted system and its
 * ordering exactly as iccg_setup does, builds both substitution schedules
 * (the chunk packing of Algorithm 1's blocks, Section 3, with pack_rows as in
 * iccg_options), re-derives their invariants (chunks tile every color; each
 * row's entries before-chunk first and ascending; every dependency in an
 * earlier color and at an earlier launch position; every row read across
 * chunks is waited for; rows read from another region are exported; slot
 * layout jagged or padded as the chunk's width requires) and writes 18 counts
 * to out: for the forward, then the backward schedule, {tasks, chunks, slots,
 * max level depth, max row width, dependencies, tasks with a dependency in
 * another region, exported rows, padded chunks (widest row above 8 entries,
 * every row stored at the chunk's width)}.
 * Returns the iccg_setup error codes, or ICCG_EINVAL naming a violated
 * invariant.  The caller owns every array. */
int iccg_schedule_stats(int n, const int *rowptr, const int *col, const double *val,
                        int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                        int pack_rows, long long *out);

const char *iccg_strerror(int status);
const char *iccg_last_error(void);
void iccg_destroy(iccg_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* ICCG_H */
