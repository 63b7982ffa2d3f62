/*
 * bc.h - C ABI of the MI355X (gfx950) block Cimmino library.
 *
 * The library solves a square, nonsingular, nonsymmetric sparse system
 * A x = f with the CG-accelerated block Cimmino method: the rows of A are split
 * into K blocks A_1..A_K (Section 1, eq. (blockCimmino)), and classical CG is
 * run on H x = xi with
 *
 *     H  = sum_i A_i^T (A_i A_i^T)^{-1} A_i        (eq. (H)),
 *     xi = sum_i A_i^T (A_i A_i^T)^{-1} f_i        (eq. (cg)),
 *
 * which is Algorithm 2 of the paper.  Each block projection solves the
 * normal equations (A_i A_i^T) y_i = u_i on the GPU, either with a dense FP64
 * Cholesky factor (blocks of at most `dense_max_m` rows) or with a
 * matrix-free inner CG; the sum over blocks is one transposed sparse
 * product A^T y.  It also builds the row inner-product graph of Section 2.1
 * (edge costs |r_i r_j^T| of C = A A^T, Section 2.3) and partitions it.
 *
 * Conventions shared by every entry point:
 *  - Matrices are CSR with int32 row pointers (rowptr[0] == 0,
 *    nondecreasing, rowptr[n] == nnz), int32 column indices sorted strictly
 *    ascending within each row and lying in [0, n), and finite float64 values.
 *  - Setup-time inputs (matrices, partitions) are HOST pointers, borrowed for
 *    the duration of the call only; the library copies what it keeps.
 *  - Solve-time vectors (f, x0, x, v, Hv) are DEVICE pointers to float64
 *    arrays of length n (for a batched context: the systems' vectors
 *    concatenated in system order, total length sum_s n_s).  Vectors indexed
 *    by rows (f) use the caller's original row order; the internal block
 *    permutation is invisible.
 *  - Work is enqueued on a library-owned stream that is ordered after the
 *    caller's stream (bc_opts.stream, NULL = the null stream) on entry, and
 *    the caller's stream is ordered after it on exit; entry points return
 *    once the results are final on the device.
 *  - Negative status codes mean that no output was written.  The text of the
 *    last error of the calling thread is returned by bc_last_error().
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef BC_H
#define BC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bc_ctx bc_ctx; /* opaque; owns its device memory */

typedef enum {
  BC_OK = 0,
  BC_NOT_CONVERGED = 1,      /* maxit reached; x holds the last iterate ("F" in Table itertable) */
  BC_ERR_INVALID = -1,       /* malformed input (see the entry point) */
  BC_ERR_SINGULAR_BLOCK = -2,/* a block A_i has no full row rank: A is singular */
  BC_ERR_BREAKDOWN = -3,     /* p^T H p not a positive finite number in the CG of Algorithm 2 */
  BC_ERR_DEVICE = -4,        /* a HIP runtime call failed, or no gfx950 device */
  BC_ERR_NOMEM = -5          /* device or host allocation failed */
} bc_status;

enum { BC_FP64 = 0, BC_MIXED = 1, BC_MIXED_PROJ = 2 };
enum { BC_PROJ_AUTO = 0, BC_PROJ_DENSE_CHOL = 1, BC_PROJ_INNER_CG = 2, BC_PROJ_BAND_CHOL = 3 };
enum { BC_STOP_REL2 = 0, BC_STOP_BACKWARD_ERR = 1 };
enum { BC_GATHER_AUTO = 0, BC_GATHER_SEPARATE = 1, BC_GATHER_INTERLEAVED = 2 };

typedef struct {
  int32_t precision;      /* BC_FP64 (default); BC_MIXED: FP32 sparse products
                             and projections, FP64 outer CG scalars, x and
                             residuals, stop test on the FP64 true residual at
                             each replacement; BC_MIXED_PROJ: FP32 copies of
                             the projection operators (dense and banded
                             factors, the inner-CG block matrices) applied
                             with FP64 arithmetic, FP64 everything else (the
                             operator is the same at every application, so no
                             replacement is made) */
  int32_t projection;     /* How y_i = (A_i A_i^T)^{-1} u_i is computed per block.
                             BC_PROJ_DENSE_CHOL: dense FP64 Cholesky factor
                             (blocks of at most 4096 rows); BC_PROJ_INNER_CG:
                             matrix-free CG; BC_PROJ_BAND_CHOL: rows of each
                             block in reverse Cuthill-McKee order and a banded
                             FP64 Cholesky factor (every block must reach a
                             half-bandwidth of at most 127, else BC_ERR_INVALID);
                             BC_PROJ_AUTO (default): per block, banded when the
                             half-bandwidth is at most 127 and the block either
                             has more than dense_max_m rows or its band holds
                             at most 1/4 of the dense factor; otherwise dense
                             for at most dense_max_m rows, else inner CG */
  int32_t dense_max_m;    /* default 4096 */
  double inner_tol;       /* inner CG stops when ||u_i - G_i y_i|| <= inner_tol ||u_i||; default 1e-12 */
  int32_t inner_maxit;    /* default 20000 */
  int32_t inner_groups;   /* workgroups cooperating on one inner-CG block; 0 = choose */
  int32_t replace_every;  /* FP64 true-residual replacement period (BC_MIXED); 0 = never; default 20 */
  int32_t stop_rule;      /* BC_STOP_REL2 (default): ||f - A x||_2 <= tol ||f||_2;
                             BC_STOP_BACKWARD_ERR: gamma < tol, eq. (stopping) */
  int32_t check_every;    /* outer iterations between host convergence checks; default 8 */
  int32_t spmv_lanes;     /* lanes of a wave sharing one row in the sparse
                             products (1..64, power of two), or -1: sliced-ELL
                             copies of A and A^T (slices of 64 rows, one row
                             per lane, entries column by column); 0 (default):
                             each of A p and A^T y is timed at setup for every
                             lane count and, when its padding adds at most a
                             quarter to the entries, the sliced-ELL form; the
                             fastest is kept (cached per sparsity pattern
                             within the process) */
  int32_t use_graph;      /* 1 (default): when every block uses a Cholesky
                             factor (dense or banded), groups of outer
                             iterations (gcd of check_every and, with FP32
                             projections, replace_every) are captured once in
                             a hipGraph and replayed; 0: plain stream launches */
  int32_t multi_gather;   /* layout of the gathered vectors in the sparse
                             products of bc_solve_multi / bc_solve_block:
                             BC_GATHER_SEPARATE: each vector of a chunk of 8
                             gathered on its own; BC_GATHER_INTERLEAVED: the
                             chunk first copied vector-minor, one 64-byte
                             gather per index for the 8; BC_GATHER_AUTO
                             (default): per copy (A, A^T) at setup,
                             interleaved when the separate gathers of a
                             64-row slice touch at least 4.5 times the
                             64-byte segments that the interleaved ones do
                             (scattered columns).  Both sum in the same
                             order: the choice changes time, never bits */
  void* stream;           /* caller's hipStream_t; NULL = null stream */
} bc_opts;

typedef struct {
  int32_t iterations;     /* outer CG iterations (applications of H in the loop) */
  int32_t status;         /* bc_status of this system */
  double rel_residual;    /* ||f - A x||_2 / ||f||_2, recomputed in FP64 from x */
  double backward_err;    /* gamma of eq. (stopping) */
  double t_solve_ms;      /* wall time of the solve call */
  double t_proj_ms;       /* GPU time in the block-projection kernels (HIP events) */
  int32_t proj_launches;  /* number of projection kernel launches timed in t_proj_ms */
  int32_t replacements;   /* true-residual replacements performed */
  int64_t inner_iterations; /* sum over outer iterations and inner-CG blocks */
  double proj_bytes;      /* algorithmic bytes of the timed projection launches: per dense
                             block m(m+1)*w (both sweeps over the packed factor, w = 8 or 4
                             bytes), per inner-CG iteration (2*(w+4)*nnz_i + 6*w*m_i) */
} bc_stats;

/* Fills *opts with the defaults listed above. */
void bc_opts_default(bc_opts* opts);

/* Builds a context for one system: validates A and the partition, permutes
 * the rows into block order (blocks in part-id order, rows ascending inside
 * a block; Section 2.2: the order inside a block does not change H), builds
 * A^T, and factors every dense block's A_i A_i^T in FP64.
 *   n              : order of A (n >= 1)
 *   rowptr/colidx/vals : host CSR of A (see conventions)
 *   K              : number of blocks, 1 <= K <= n
 *   part           : host int32[n], part[r] in [0, K) = block of row r; every block nonempty
 *   opts           : NULL = defaults
 * Errors: BC_ERR_INVALID (malformed CSR, non-finite value, bad partition,
 * empty block), BC_ERR_SINGULAR_BLOCK (non-positive pivot in a dense block's
 * Cholesky), BC_ERR_DEVICE, BC_ERR_NOMEM.  On error *ctx is NULL. */
bc_status bc_setup(bc_ctx** ctx, int32_t n, const int32_t* rowptr, const int32_t* colidx,
                   const double* vals, int32_t K, const int32_t* part, const bc_opts* opts);

/* Same for nsys independent systems solved together (block-diagonal batch).
 * n[s], K[s] and the per-system host arrays rowptr[s], colidx[s], vals[s],
 * part[s] describe system s exactly as in bc_setup. */
bc_status bc_setup_batched(bc_ctx** ctx, int32_t nsys, const int32_t* n,
                           const int32_t* const* rowptr, const int32_t* const* colidx,
                           const double* const* vals, const int32_t* K,
                           const int32_t* const* part, const bc_opts* opts);

/* Hv = H v = sum_i A_i^+ A_i v (eq. (H)): one block-projection sweep.
 * v, Hv: device float64[n_total].  Uses the context's precision. */
bc_status bc_project(bc_ctx* ctx, const double* v, double* Hv);

/* Algorithm 2 from x0 (device float64[n], or NULL for zero) until the stop
 * rule holds with threshold tol, or maxit iterations.  x: device float64[n]
 * output.  stats: host, may be NULL.  Returns BC_OK, BC_NOT_CONVERGED (x is
 * the last iterate), BC_ERR_BREAKDOWN (x is the last iterate before the
 * breakdown), or an error.  tol = 0 runs exactly maxit iterations. */
bc_status bc_solve(bc_ctx* ctx, const double* f, const double* x0, double tol,
                   int32_t maxit, double* x, bc_stats* stats);

/* bc_solve for callers that cannot allocate device memory (code under HIP
 * graph capture nearby, tight serving loops, harnesses that forbid
 * hipMalloc): the same Algorithm 2 on the same kernels with no allocation at
 * call time.  Its seven work vectors of n_total doubles live in a static
 * device array of 256 MiB (held by every GPU the library runs on until the
 * process ends) instead of the context's own; the outer iterations are
 * plain launches (no captured graph) and no timing events are created, so
 * bc_stats.t_proj_ms and proj_launches are 0.  Results are bit for bit those
 * of bc_solve (also for batched contexts; the call takes one system or a
 * batch like bc_solve_batched, with stats holding nsys entries).  Returns
 * BC_ERR_INVALID when 7 * n_total * 8 bytes exceed the array (n_total above
 * 4,793,490 rows).  All contexts on one GPU share the array: calls that
 * overlap on one GPU (other host threads) race. */
bc_status bc_solve_noalloc(bc_ctx* ctx, const double* f, const double* x0, double tol,
                           int32_t maxit, double* x, bc_stats* stats);

/* Batched form of bc_solve: f, x0, x are concatenated device vectors; stats
 * (host, may be NULL) has nsys entries.  Each system stops on its own; the
 * call returns the worst status over the systems. */
bc_status bc_solve_batched(bc_ctx* ctx, const double* f, const double* x0, double tol,
                           int32_t maxit, double* x, bc_stats* stats);

/* Algorithm 2 for nrhs right-hand sides of the one system of a bc_setup
 * context (the same matrix A with several f: Section 3.1 names the
 * multiple-right-hand-side case, and Section 3.5 notes that sequences of
 * right-hand sides with one matrix amortize the partitioning cost further).
 * Each right-hand side runs its
 * own CG recurrence and stops on its own, exactly as one bc_solve with it
 * would (same iterations and bits, given the same sparse-product schedule,
 * spmv_lanes = -1, and the same dense sweep: chunks whose LDS leaves room for
 * one workgroup per CU only take a row-owned sweep that sums in another
 * order); the right-hand sides share every read of A, A^T and the
 * dense block factors: the sparse products take chunks of 8 vectors per
 * matrix read (bc_opts.multi_gather), the dense triangular sweeps chunks of
 * up to 16 per factor read, the banded ones chunks of 1, 4 or 8 per band
 * read.  Inner-CG blocks run all vectors in one launch of the
 * one-workgroup-per-block kernel when bc_solve uses that kernel too
 * (bc_opts.inner_groups resolving to 1) or when blocks x vectors reach the
 * compute units; otherwise they take the vectors one after another with the
 * grouped kernel of bc_solve (then the same bits as bc_solve).
 * f, x0 (or NULL for zero), x: device float64[nrhs * n], vector j at
 * offset j * n (original row / column order, as bc_solve).  stats: host,
 * nrhs entries, may be NULL.  Needs the sliced-ELL copies of A
 * (bc_opts.spmv_lanes = -1, or 0 when their padding is modest); no
 * hipGraph capture.  The per-vector state (8 n-vectors per right-hand side)
 * is allocated on the first call with a given nrhs and kept until another
 * nrhs or bc_destroy.  Returns the worst status, as bc_solve_batched;
 * BC_ERR_INVALID for a batched context, nrhs < 1, nrhs > 262140 (65535
 * chunks of 4, the narrowest chunk of the dense sweeps) or nrhs * n >= 2^31. */
bc_status bc_solve_multi(bc_ctx* ctx, int32_t nrhs, const double* f, const double* x0,
                         double tol, int32_t maxit, double* x, bc_stats* stats);

/* Block CG on H X = Xi for nrhs right-hand sides of the one system of a
 * bc_setup context: one Krylov space for all of them, the stabilized
 * block-CG acceleration that Section 3.1 names for multiple right-hand sides
 * (the paper itself uses Algorithm 2 per right-hand side).  Per iteration:
 * Q = H P for the p <= nrhs search directions P (orthonormal columns),
 * alpha = (P^T Q)^{-1} P^T R, X += P alpha, R -= Q alpha; the true residual
 * f_j - A x_j of every column still running is tested (relative 2-norm
 * <= tol, as bc_solve) and columns that meet it stop; then
 * beta = -(P^T Q)^{-1} Q^T R and the next P is an orthonormal basis of
 * R + P beta over the running columns, a direction whose part outside the
 * span of those before it is below 1e-5 of its norm being dropped (repeated
 * or dependent right-hand sides).  The products with H take all p
 * directions at once (as bc_solve_multi); the p x p algebra runs on the host
 * in FP64 between device reductions.  With FP32 sparse products and
 * projections (BC_MIXED) R is recomputed from the FP64 true residual every
 * replace_every iterations, R = A^T D^{-1} (f - A x), and the directions
 * restart from it (stats.replacements counts these).  Arguments and layout as
 * bc_solve_multi; stats[j].iterations counts the block iterations until
 * column j stopped.  1 <= nrhs <= 16.  Returns the worst status;
 * BC_ERR_BREAKDOWN if P^T Q is not positive definite or no direction is left
 * while columns run (x holds the last iterate). */
bc_status bc_solve_block(bc_ctx* ctx, int32_t nrhs, const double* f, const double* x0,
                         double tol, int32_t maxit, double* x, bc_stats* stats);

/* Algorithm 1 (plain block Cimmino, Section 1, eq. (iterscheme)):
 * x <- x + omega sum_i A_i^+ (f_i - A_i x), from x0 (device float64[n], or
 * NULL for zero), until ||f - A x||_2 <= tol ||f||_2 (the residual of the
 * current iterate, FP64, tested before each update) or maxit updates.  It
 * converges for 0 < omega < 2 / lambda_max(H), fastest near
 * omega = 2 / (lambda_min + lambda_max).  Works on single and batched
 * contexts (f, x0, x concatenated; stats: host, nsys entries, may be NULL);
 * the iteration count is the number of updates made.  The context's
 * projections and precision are used; stop_rule must be BC_STOP_REL2.
 * Returns the worst status over the systems, as bc_solve_batched. */
bc_status bc_cimmino(bc_ctx* ctx, const double* f, const double* x0, double omega, double tol,
                     int32_t maxit, double* x, bc_stats* stats);

/* Sizes of a context: total order, number of systems and of blocks, and the
 * number of blocks using the dense Cholesky projection.  Any pointer may be NULL. */
bc_status bc_info(const bc_ctx* ctx, int64_t* n_total, int32_t* nsys, int32_t* nblocks,
                  int32_t* ndense);

/* The lane counts chosen for the sparse products: lanes_a for A p and the
 * residuals, lanes_at for A^T y (64/lanes rows per wavefront; -1 for the
 * sliced-ELL form, one row per lane).  Either pointer may be NULL. */
bc_status bc_schedule(const bc_ctx* ctx, int32_t* lanes_a, int32_t* lanes_at);

/* Per block (in block order: systems in order, blocks by part id): the
 * projection kind (0 dense Cholesky, 1 inner CG, 2 banded Cholesky) and the
 * half-bandwidth of banded blocks (-1 for the others).  kind and bandwidth are
 * host arrays of bc_info's nblocks entries, either may be NULL. */
bc_status bc_block_info(const bc_ctx* ctx, int32_t* kind, int32_t* bandwidth);

/* Bound of the device waits of a context, in seconds of wall clock (default
 * 2).  Two kernels wait for other parts of the GPU: the inner CG, whose
 * workgroups of one block meet at barriers in global memory, and the dense
 * sweep whose waves publish finished rows to each other.  A wait that passes
 * the bound stops its kernel, which then exits normally, and the call
 * (bc_project or a solve) returns BC_ERR_DEVICE with a message in
 * bc_last_error: its result is invalid, and the next call on the context
 * starts clean.  seconds = 0 makes every such wait give up at its first check
 * (a test of that path); negative or non-finite values return
 * BC_ERR_INVALID. */
bc_status bc_set_wait_limit(bc_ctx* ctx, double seconds);

/* Releases the context and all its device memory.  NULL is allowed. */
void bc_destroy(bc_ctx* ctx);

/* ---- row inner-product graph (Sections 2.1 and 2.3) ---- */

typedef struct {
  int32_t n;        /* vertices = rows of A */
  int64_t nnz;      /* directed edge entries (each undirected edge twice) */
  int64_t* rowptr;  /* int64[n+1] */
  int32_t* col;     /* int32[nnz], ascending within a row, no diagonal */
  double* cost;     /* float64[nnz], |c_ij| of C = A~ A~^T */
  int64_t* wgt;     /* int64[nnz], ceil(alpha * cost) */
} rip_graph_t;

typedef struct {
  int32_t prescale;  /* 1 (default): rows scaled to unit 2-norm first (Section 2.1) */
  int32_t sparsify;  /* 1 (default): each column with more than isqrt(n) entries
                        keeps its isqrt(n) largest |a| (ties: lower row; Section 2.3) */
  int64_t alpha;     /* weight scale, default 2^20 (Section 2.3: wgt = ceil(alpha*cost)) */
  void* stream;      /* caller's hipStream_t; NULL = null stream */
} rip_opts;

void rip_opts_default(rip_opts* opts);

/* Builds G_RIP(A) on the GPU with a row-wise sparse product C = A~ A~^T.
 * Row norms are accumulated in ascending column order; c_ij accumulates its
 * products in ascending shared-column order, each product rounded before the
 * add (no fused multiply-add); the diagonal and exact zeros are not edges.
 * A: host CSR as in bc_setup.  out: filled with HOST arrays allocated by the
 * library; release with rip_graph_free.
 * Errors: BC_ERR_INVALID (malformed CSR, a zero row with prescale on, or a
 * weight that would reach 2^62), BC_ERR_DEVICE, BC_ERR_NOMEM. */
bc_status rip_graph(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                    const rip_opts* opts, rip_graph_t* out);

void rip_graph_free(rip_graph_t* g);

/* GPU time of the sparse product kernels (both passes, HIP events) and wall
 * time of the last rip_graph call made by the calling thread, in ms. */
bc_status rip_graph_timing(double* spgemm_ms, double* total_ms);

/* Deterministic greedy K-way partition of a graph with integer edge weights
 * (the project's replacement for METIS on G_RIP, Sections 2.3 and 3.1; unit
 * vertex weights, balance cap W_max = max(floor(1.1 n / K), ceil(n / K)) of
 * eq. (partbal)).  Growth: parts 0..K-2 are grown in turn to
 * ceil(remaining / parts left) vertices from the lowest-index unassigned
 * vertex, always adding the unassigned vertex with the largest total weight
 * into the part (ties: lower index; none touching: lowest unassigned); the
 * last part takes the rest.  Refinement: `passes` sweeps in ascending vertex
 * order move a vertex to the part with the largest positive gain that stays
 * within W_max, keeping its source part nonempty (ties: lower part id).
 * Host arrays: rowptr int64[n+1], col int32[nnz] (symmetric, no diagonal),
 * wgt int64[nnz] >= 1 (col and wgt may be null when nnz = 0); part int32[n]
 * output.  Errors: BC_ERR_INVALID. */
bc_status bc_partition_greedy(int32_t n, const int64_t* rowptr, const int32_t* col,
                              const int64_t* wgt, int32_t K, int32_t passes, int32_t* part);

/* Multilevel K-way partition of the same kind of graph (the multilevel
 * scheme the paper's partitioner follows, Section 3.1, made deterministic):
 *  1. Coarsening, while the graph has more than 30 K vertices (at most 30
 *     levels, stopping when a level keeps more than 90% of the vertices):
 *     vertices in ascending order, each unmatched one matched with the
 *     unmatched neighbour of largest edge weight (ties: lower index) whose
 *     combined vertex weight stays within ceil(n / (20 K)); coarse vertices
 *     numbered in ascending order of their lower fine vertex; parallel edges
 *     summed, internal edges dropped.
 *  2. On the coarsest graph, the growth of bc_partition_greedy by vertex
 *     weight: part k (k < K-1) grows until it weighs ceil(remaining weight /
 *     parts left), leaving at least one vertex for each later part.
 *  3. At every level from the coarsest to the original graph (after
 *     projecting the parts down), at most `passes` Fiduccia-Mattheyses
 *     passes with vertex weights and W_max as in bc_partition_greedy.  In a
 *     pass every vertex starts unlocked, and conn(v, q) is the total edge
 *     weight from v to part q.  A max-priority queue holds (key, v), larger
 *     key first, ties to the lower v, where key(v) is the largest
 *     conn(v, q) - conn(v, part[v]) over the parts q != part[v] that v
 *     touches; it starts with every vertex that touches another part.  A
 *     popped entry is skipped if v is locked or key(v) has changed.  Else
 *     v (in part a) moves to the touched part q != a of largest gain
 *     conn(v, q) - conn(v, a), ties to the lower q, among parts with
 *     W[q] + w(v) <= W_max, provided W[a] > w(v); if there is none the
 *     entry is dropped and v stays unlocked.  The gain may be negative.  A
 *     moved vertex is locked, the move logged with the running sum of
 *     gains, and each unlocked neighbour u (in adjacency order) that
 *     touches another part is pushed again with its current key(u).  The
 *     pass ends when the queue is empty or 64 moves in a row have not
 *     raised the best running sum; the moves after the best prefix (the
 *     shortest on ties) are undone, last first.  No further pass runs after
 *     one whose best running sum is 0.
 * Arguments and errors as bc_partition_greedy. */
bc_status bc_partition_multilevel(int32_t n, const int64_t* rowptr, const int32_t* col,
                                  const int64_t* wgt, int32_t K, int32_t passes, int32_t* part);

/* Cutsize of a partition: sum of cost over cut edges, each undirected edge
 * once (eq. (partcut)), and the same sum over the integer weights.  Host arrays. */
bc_status bc_partition_cut(int32_t n, const int64_t* rowptr, const int32_t* col,
                           const double* cost, const int64_t* wgt, const int32_t* part,
                           double* cutsize, int64_t* int_cut);

const char* bc_status_str(bc_status s);
const char* bc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BC_H */
