/*
 * fj.h -- C ABI of libfjgpu: Friedkin-Johnsen equilibrium and opinion indices
 * on one AMD Instinct MI355X (gfx950).
 *
 * What is computed (Xu, Bao, Zhang, "Fast Evaluation for Relevant Quantities
 * of Opinion Dynamics", WWW 2021):
 *   - the equilibrium expressed opinions z = (I + L)^{-1} s of the FJ model
 *     (Section 3.1, Eq. FJmodel02), where L = D - A is the Laplacian of a
 *     weighted undirected graph (Section 2.1) and s in [0,1]^n are the
 *     internal opinions;
 *   - the five indices of Section 3.2 (Definitions; Proposition 1;
 *     Lemma 4.1), each to a certified relative error eps, which is the
 *     eps-approximation guarantee of the Theorem in Section 4 (the output of
 *     Algorithm 1, Approxim(G, s, eps)).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer owned by the caller, unless it
 *     is documented as host. The library never allocates device memory: the
 *     caller provides the plan and the workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every call is ordered on that stream. Calls that return results to host
 *     memory (fj_indices, fj_solve's info) synchronise with the stream before
 *     returning.
 *   - Every function returns an int status (FJ_OK = 0 on success). No C++
 *     exception crosses the ABI and the library never aborts the process: a
 *     failed host allocation inside the library returns FJ_ERR_HOST_MEMORY,
 *     any other C++ exception FJ_ERR_INTERNAL (fj_last_error has the detail).
 *     After either from a fj_server_* call, destroy the server.
 *   - Calls are thread-safe when concurrent calls use distinct workspaces.
 *     A plan may be shared by concurrent calls once fj_prepare has completed.
 *   - Per calling thread and device the library keeps a small pinned host
 *     block (about 2 KiB) and a few HIP events, created on first use.
 */
#ifndef FJ_H
#define FJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FJ_OK                 0
#define FJ_ERR_INVALID_ARG    1  /* a null pointer, n < 0, eps outside (0, 1/2), ... */
#define FJ_ERR_INVALID_GRAPH  2  /* FJ_VALIDATE_GRAPH found a violation of the CSR contract */
#define FJ_ERR_OPINION_RANGE  3  /* some s_i is NaN or outside [0,1] (Section 3.1 assumes s in [0,1]) */
#define FJ_ERR_WORKSPACE      4  /* plan or workspace smaller than the queried size, or misaligned */
#define FJ_ERR_NOT_CONVERGED  5  /* max_iter reached; results and bounds are still written */
#define FJ_ERR_BREAKDOWN      6  /* CG breakdown (p^T (I+L) p <= 0 or not finite) */
#define FJ_ERR_UNCERTIFIABLE  7  /* an index is too close to 0 for a relative bound (bound[] = inf for it);
                                    the indices, residual_norm and the finite abs_bound[] are written */
#define FJ_ERR_HIP            8  /* a HIP runtime call failed */
#define FJ_ERR_CANCELLED      9  /* the request was withdrawn with fj_server_cancel */
#define FJ_ERR_HOST_MEMORY   10  /* a host allocation inside the library failed (std::bad_alloc) */
#define FJ_ERR_INTERNAL      11  /* any other C++ exception inside the library (a bug) */

/* ---- graph -------------------------------------------------------------- */
#define FJ_VAL_UNIT 0  /* every edge has weight 1; val must be NULL */
#define FJ_VAL_F32  1  /* val is float[nnz] */
#define FJ_VAL_F64  2  /* val is double[nnz] */

/*
 * Weighted undirected simple graph G = (V, E, w) of Section 2.1 in CSR form,
 * both directions of every edge stored: entry (i, j) with weight w_ij and
 * entry (j, i) with the same weight. Column indices strictly increasing inside
 * each row (no repeated edges), no self-loops, weights finite and > 0.
 * Isolated nodes are allowed (the paper assumes a connected graph; I + L is
 * positive definite regardless, so the equilibrium is still unique).
 * Limits: 0 <= n, nnz < 2^31 (int32 row pointers).
 */
typedef struct fj_csr {
    int32_t n;                /* number of nodes */
    int64_t nnz;              /* stored entries = 2 * number of edges = row_ptr[n] */
    const int32_t *row_ptr;   /* device, n + 1 entries, row_ptr[0] = 0 */
    const int32_t *col_idx;   /* device, nnz entries */
    const void *val;          /* device, nnz entries of float/double, or NULL (FJ_VAL_UNIT) */
    int32_t val_type;         /* FJ_VAL_UNIT, FJ_VAL_F32 or FJ_VAL_F64 */
} fj_csr;

/* ---- options ------------------------------------------------------------ */
#define FJ_FP64  0  /* FP64 operator, vectors and reductions throughout */
#define FJ_MIXED 1  /* FP32 inner CG wrapped in FP64 residual-and-correction refinement */

#define FJ_TWO_SOLVE       1u  /* Algorithm 1 literally: solve for s and for the centred s too */
#define FJ_NO_RANGE_CHECK  2u  /* accept opinions outside [0,1] (the algebra holds for any real s) */
#define FJ_VALIDATE_GRAPH  4u  /* fj_prepare checks the CSR contract (synchronises) */
#define FJ_PROFILE         8u  /* time every SpMV launch with HIP events (fills fj_info.ms_*) */
#define FJ_NO_TUNE        16u  /* batched solves: skip the SpMM autotuner, use 1 column per lane and the full grid */
#define FJ_WARM_START     32u  /* fj_solve, k = 1: Z holds the starting guess on entry (e.g. an earlier solution) */
#define FJ_ZERO_START     64u  /* plain Jacobi-PCG from z = 0. By default every CG solve (FP64, the FP32
                                  inner solves of FJ_MIXED, batched columns) starts from mean(rhs) 1 and is
                                  deflated by the constant vector: every step is centred, so mean(z) = mean(s)
                                  holds throughout, and fewer iterations are needed */
#define FJ_DIAG_PRECOND  128u  /* one-vector solves: Jacobi (diagonal) preconditioning only. By default, on
                                  graphs of >= 65536 nodes (FJ_MIXED: also mean degree >= 16), CG uses 2x2
                                  blocks of I + L on a heavy-edge matching made by fj_prepare
                                  (z_i = c1_i r_i + c2_i r_j for a pair i, j): fewer iterations, most on
                                  graphs whose edge weights spread widely */
#define FJ_BLOCK_CG      256u  /* k >= 2 opinion vectors, FJ_FP64: O'Leary's block CG, one Krylov space shared by
                                  the columns of each block of up to 64 (at least 16 wide: narrower blocks are
                                  padded), its search block kept A-orthonormal; the k x k products run on the
                                  matrix cores. By default (and in the server) every column runs its own CG, so
                                  a column's result does not depend on the others; with this flag it does.
                                  Not with FJ_TWO_SOLVE or FJ_WARM_START */
#define FJ_MULTILEVEL    512u  /* one opinion vector (k = 1), FJ_FP64: precondition CG with the aggregation
                                  V-cycle of opts->hierarchy (fj_hierarchy_create) instead of the 2x2 blocks or
                                  Jacobi; for graphs whose edge weights spread over many orders of magnitude.
                                  Not with FJ_DIAG_PRECOND, FJ_BLOCK_CG, FJ_TWO_SOLVE (a 2-column batched
                                  solve), in the server or fj_indices_noalloc */
#define FJ_WINDOW_SPMV  1024u  /* one-vector solves (any preconditioner): run the CG SpMV on the row windows
                                  (CSR order) even on graphs of >= 65536 nodes, where by default it runs on the
                                  time-phased layout of the plan (see fj_prepare). The index epilogue always
                                  runs on the row windows */
#define FJ_PHASED_SPMV  2048u  /* one-vector solves: run the CG SpMV on the time-phased layout on any graph (by
                                  default only from 65536 nodes on). Not with FJ_WINDOW_SPMV */

typedef struct fj_hierarchy fj_hierarchy;

typedef struct fj_opts {
    double eps;           /* certified relative error of every index, in (0, 1/2) (Algorithm 1 input) */
    double rtol;          /* relative residual ||s-(I+L)z||/||s|| of the first CG pass; 0 = eps * 1e-2 */
    int32_t max_iter;     /* CG iterations over all passes; 0 = 2000 */
    int32_t precision;    /* FJ_FP64 or FJ_MIXED */
    uint32_t flags;       /* FJ_* flags above */
    int32_t reserved;     /* must be 0 */
    const fj_hierarchy *hierarchy;  /* FJ_MULTILEVEL: the hierarchy of this graph; otherwise ignored */
} fj_opts;

/* Fill *opts with the defaults: eps = 1e-6, rtol = 0, max_iter = 0, FJ_FP64, no flags, no hierarchy. */
void fj_default_opts(fj_opts *opts);

/* ---- results ------------------------------------------------------------ */
/* Section 3.2 indices; dc_index is reported through its equal form s^T z. */
typedef struct fj_indices_t {
    double internal_conflict;  /* C_I  = sum_i (z_i - s_i)^2 = ||L z||^2        */
    double disagreement;       /* D    = sum_{(i,j) in E} w_ij (z_i - z_j)^2     */
    double polarization;       /* P    = sum_i (z_i - mean(z))^2                 */
    double controversy;        /* C    = sum_i z_i^2                             */
    double dc_index;           /* I_dc = D + C = s^T z                           */
} fj_indices_t;

typedef struct fj_info {
    int32_t status;        /* per-column status (same codes as the return value) */
    int32_t iters;         /* CG iterations over all passes */
    int32_t passes;        /* CG passes (each pass restarts from the true residual) */
    int32_t outer_iters;   /* FJ_MIXED refinement steps (0 for FJ_FP64) */
    double rel_residual;   /* ||s - (I+L) z||_2 / ||s||_2, true residual in FP64 */
    double bound[5];       /* certified relative error bound of each index, order of fj_indices_t */
    double ms_spmv;        /* FJ_PROFILE: total milliseconds inside the CG SpMV kernel */
    int32_t n_spmv;        /* FJ_PROFILE: number of CG SpMV launches timed */
    int32_t reserved;
    double residual_norm;  /* rho = ||s - (I+L) z||_2, the true FP64 residual the bounds are built from */
    double abs_bound[5];   /* |X - X~| <= abs_bound[i] for each index X (order of fj_indices_t), from the
                              same certificate as bound[] (Section 4: I <= I + L, so the error
                              e = (I+L)^{-1} r has ||e||, ||L e||, ||e - mean(e) 1|| <= rho and
                              ||W^{1/2} B e|| <= rho / 2): rho_X (2 sqrt(X~) + rho_X) for the four squared
                              norms, (||z~|| + rho) rho for s^T z. Always finite: the error information
                              for an index too close to 0 for a relative bound (FJ_ERR_UNCERTIFIABLE) */
} fj_info;

/* ---- entry points ------------------------------------------------------- */

/* Human-readable name of a status code (static string). */
const char *fj_status_string(int status);

/* Detail of the last FJ_ERR_HIP or FJ_ERR_INVALID_GRAPH on the calling thread
 * ("" if none). The string stays valid until the thread's next call. */
const char *fj_last_error(void);

/* Bytes of device memory fj_prepare needs for the per-graph plan of g. */
size_t fj_plan_bytes(const fj_csr *g);

/*
 * One-time set-up of the operator I + L for graph g (Section 2.1): the
 * Jacobi preconditioner diag(I + D)^{-1}, the heavy-edge matching and the
 * coefficients of the 2x2 block preconditioner (see FJ_DIAG_PRECOND), the
 * row-window partition that balances the sparse passes, and the time-phased
 * layout of the entries: the rows dealt to wave-sized chunks of about equal
 * entries (at most 1248 rows, or 1600 on graphs with many entries per chunk),
 * each chunk's entries ordered by column range of 131072 nodes
 * ("phase") and by row, so that the whole GPU gathers from one column range
 * at a time and each XCD's L2 holds it. The host deals the rows to the
 * chunks from row_ptr alone and turns the GPU's counts into offsets; the GPU
 * counts, sums the degrees and places the entries. fj_prepare therefore
 * synchronises `stream`. A graph whose layout would need 2^31 entry slots or
 * more, or more than 2048 phases, has none. Writes `plan`
 * (device, >= fj_plan_bytes, 256-byte aligned; the layout takes about
 * 4 + value bytes + 2 bytes per entry, plus 16 bytes per node).
 * FJ_VALIDATE_GRAPH also checks the CSR contract first. opts may be NULL.
 */
int fj_prepare(const fj_csr *g, const fj_opts *opts, void *plan, size_t plan_bytes, void *stream);

/* Bytes of device workspace a solve of k right-hand sides needs. */
size_t fj_workspace_bytes(const fj_csr *g, int32_t k, const fj_opts *opts);

/*
 * y = (I + L) x (Section 2.1, L = D - A), FP64. x, y: device double[n],
 * distinct. Asynchronous on `stream`.
 */
int fj_apply(const fj_csr *g, const void *plan, const double *x, double *y, void *stream);

/*
 * y = (I + L) x as fj_apply, on the time-phased layout of the plan (the pass
 * that one-vector CG steps run on large graphs): row sums
 * ((I + L) x)_i = x_i + d_i x_i - sum_j w_ij x_j with the weighted degree d_i,
 * added in a fixed order. x, y: device double[n], distinct. Asynchronous on
 * `stream`. FJ_ERR_INVALID_ARG when the graph has no such layout (see fj_prepare).
 */
int fj_apply_phased(const fj_csr *g, const void *plan, const double *x, double *y, void *stream);

/*
 * Z ~= (I + L)^{-1} S (Eq. FJmodel02) for k columns. S and Z are node-major:
 * column c of node i is S[i * lds + c] (lds >= k), likewise Z with ldz.
 * Each column is solved by Jacobi-preconditioned CG deflated by the constant
 * vector (see FJ_ZERO_START), independently of the other columns.
 * Stops when the true relative residual is <= opts->rtol (0 means eps*1e-2).
 * info: host array of k entries (may be NULL). Synchronises before returning.
 */
int fj_solve(const fj_csr *g, const void *plan, int32_t k, const double *S, int64_t lds,
             double *Z, int64_t ldz, const fj_opts *opts, void *ws, size_t ws_bytes,
             void *stream, fj_info *info);

/*
 * Algorithm 1's a-priori solver accuracy for an n-node graph with weights in
 * [w_min, w_max], centred opinions of norm sbar_norm and error parameter
 * eps: delta = eps w_min ||sbar|| / (3 w_max n^3 (n w_max + 1) sqrt(n)).
 * Reported beside the a-posteriori certificate that the library uses
 * instead (delta lies far below FP64 resolution at these sizes). Host only;
 * returns NaN for arguments outside the algorithm's domain.
 */
double fj_apriori_delta(int64_t n, double w_min, double w_max, double sbar_norm, double eps);

/*
 * The SpMM launch shape the autotuner chose for this graph (same pointers, n
 * and nnz), block width kb (2, 4, ..., 64) and precision (FJ_FP64: FP64
 * vectors; FJ_MIXED: the FP32 inner vectors) on the current device:
 * *cpl columns per lane (kb / *cpl lanes work together), *grid workgroups,
 * *split = 1 when each window's rows and entries are split evenly over
 * the lane groups (0: one lane group per row), and *passes column passes
 * over the CSR (1; or 2 or 4 for 32- and 64-column blocks, one lane group per
 * row: each pass gathers kb / *passes values per neighbour, so the gathered
 * part of a wide block stays in the 256 MB Infinity Cache). The first batched
 * solve of such a combination times every candidate shape once and keeps
 * the fastest for the life of the process. Returns FJ_ERR_INVALID_ARG when
 * nothing has been tuned for it yet.
 */
int fj_spmm_choice(const fj_csr *g, int32_t kb, int32_t precision, int32_t *cpl, int32_t *grid,
                   int32_t *split, int32_t *passes);

/*
 * Pin the SpMM launch shape for this graph, kb and precision on the current
 * device instead of tuning it (for instance to reproduce another process's
 * choice bit for bit): cpl in {1, 2, 4} dividing kb, grid in [1, 4096],
 * split 0 or 1, passes 1, or 2 or 4 with split 0, cpl <= 2 and at least 16
 * columns per pass. Later batched solves and servers created afterwards use it.
 */
int fj_spmm_set_choice(const fj_csr *g, int32_t kb, int32_t precision, int32_t cpl, int32_t grid,
                       int32_t split, int32_t passes);

/*
 * Optional operator set-up (the relabelling step of the operator's setup):
 * relabel the nodes by non-increasing degree (number of stored entries, ties
 * in the old order). Every CG step gathers a node's value once per
 * neighbour, so this puts the most gathered values side by side at the front
 * of every vector, where they share cache lines and stay in L2 (on the 4M-node
 * workload the bare gather takes 1.61 ms randomly labelled, 1.21 ms hub-first).
 * Writes the relabelled CSR (device, caller-allocated, g's sizes: row_ptr_out
 * int32[n + 1], col_out int32[nnz] with each row's columns sorted, val_out of
 * g's value type or NULL for unit weights) and perm (device int32[n]): new
 * node i is old node perm[i]. Runs on the host from a device-to-host copy of
 * the CSR (synchronous on `stream`). The five indices of Section 3.2 are sums
 * over nodes and edges and do not change under a relabelling: solve the new
 * graph with fj_permute(perm, s) and bring z back with the inverse
 * permutation. FJ_ERR_INVALID_ARG for a null output that the graph needs.
 */
int fj_reorder_by_degree(const fj_csr *g, int32_t *perm, int32_t *row_ptr_out, int32_t *col_out, void *val_out,
                         void *stream);

/*
 * Move a node-major block between labellings: y[i * ldy + c] =
 * x[perm[i] * ldx + c] (inverse = 0: old labels to new) or y[perm[i] * ldy + c]
 * = x[i * ldx + c] (inverse = 1: new to old), c < k. perm must be a
 * permutation of 0..n-1 (entries outside that range are skipped). x, y:
 * distinct device arrays. Asynchronous on `stream`.
 */
int fj_permute(int32_t n, int32_t k, const int32_t *perm, const double *x, int64_t ldx, double *y, int64_t ldy,
               int32_t inverse, void *stream);

/*
 * The multilevel preconditioner of FJ_MULTILEVEL, a stand-in for the Laplacian
 * solver the method calls (Lemma ST: a nearly-linear-time solver for
 * Laplacian systems, built there by approximate Gaussian elimination) in the
 * same class: an aggregation hierarchy of I + L with a V-cycle.
 *   Level 0 is I + L = diag(a_0) - W_0 (a_0 = 1 + weighted degree). Node by
 *   node in index order, each joins the group of its heaviest neighbour (ties
 *   broken by a hash of the edge) unless the union would exceed 64 nodes; the
 *   groups are the aggregates, the nodes of the next level.
 *   The next level keeps the form diag(a) - W (Galerkin: P^T A P with P the
 *   0/1 aggregate indicator): W sums the weights between aggregates, the
 *   identity part becomes the aggregate sizes. Coarsening stops at
 *   <= coarse_max nodes (0: 1024), after 16 levels, or when a level shrinks by
 *   less than 10 %; the last level is inverted exactly (dense, FP64) if it has
 *   at most 4096 nodes and is otherwise smoothed by one Jacobi step.
 *   One V-cycle: damped Jacobi (weight 0.9) before and after the coarse
 *   correction on every level; it is a fixed symmetric positive definite
 *   operator, so CG stays CG.
 * Built on the host from a device-to-host copy of the CSR (synchronous on
 * `stream`), then uploaded: the hierarchy holds its own copy of every level
 * (12 bytes per stored entry: int column, FP64 weight) and the V-cycle's work
 * vectors (up to seven doubles per node of each level),
 * allocated here. Rebuild it if the graph's weights change. A hierarchy
 * serves one solve at a time (its work vectors are shared): concurrent solves
 * need one each.
 * FJ_ERR_INVALID_ARG for a null out or coarse_max < 0; FJ_ERR_HOST_MEMORY or
 * FJ_ERR_HIP when an allocation fails (nothing is leaked).
 */
int fj_hierarchy_create(const fj_csr *g, int32_t coarse_max, fj_hierarchy **out, void *stream);

/* Shape of a hierarchy: *levels (counting level 0 and the last), and, for
 * level l < min(levels, 16), its nodes n[l] and stored off-diagonal entries
 * nnz[l] (host arrays of 16, may be NULL). *dense = 1 if the last level is
 * inverted exactly. */
int fj_hierarchy_shape(const fj_hierarchy *h, int32_t *levels, int32_t *n, int64_t *nnz, int32_t *dense);

/* Free a hierarchy (waits for the device first). NULL is accepted. */
int fj_hierarchy_destroy(fj_hierarchy *h);

/*
 * Measurement aid (not part of any solve): the bare gather of an SpMV over
 * this CSR in storage order, y[t] = sum_{e = 8t}^{8t+7} w_e x[col_e], with
 * eight gathers in flight per thread and no row bookkeeping. Its duration is
 * the floor for any pass that reads the CSR once and gathers x per entry in
 * this order (the gather rate, not HBM bandwidth, bounds such passes on
 * power-law graphs). x: device double[n]; y: device double[(nnz + 7) / 8].
 * Asynchronous on `stream`.
 */
int fj_gather_bound(const fj_csr *g, const double *x, double *y, void *stream);

/*
 * Measurement aid (not part of any solve): the gather of fj_gather_bound over
 * the same entries regrouped into `slices` streams, to see what confining each
 * XCD's gathers to a slice of x buys. slices = 1: one stream in CSR order (the
 * same grouping as fj_gather_bound, so y is bitwise equal to its y).
 * slices = 8: the columns [hub_cols, n) are cut into eight ranges of about
 * equal entry count and range s is read only by stream s; the entries of the
 * hub columns [0, hub_cols) are dealt to the eight streams in equal runs in
 * CSR order (each stream reads the whole hub range). Workgroup b of the launch
 * works on stream b % 8, which on MI355X keeps a stream on one XCD, so that
 * XCD's L2 holds the hub range plus one tail range of x.
 * x: device double[n] (x_bytes 8) or float[n] (x_bytes 4). y: device
 * double[(nnz + 7) / 8 + 8]; y[t] of stream s's group t sits at off_s / 8 + t.
 * check: optional device int32[2], added to: [0] the workgroups whose
 * hardware XCD id equals b % 8, [1] all workgroups. bounds: optional host
 * int64[9], the range edges (bounds[s] .. bounds[s + 1] is tail range s;
 * bounds[0] = min(hub_cols, n)).
 * The streams are built on the host from a device-to-host copy of the CSR on
 * the first call for a graph (synchronous, seconds for 10^8 entries) and held
 * in device memory until a call on another graph, stream count or hub width,
 * or process end; later calls only launch, asynchronously on `stream`.
 * FJ_ERR_INVALID_ARG for slices other than 1 or 8, x_bytes other than 4 or
 * 8, negative hub_cols or a null x or y with nnz > 0.
 */
int fj_gather_bound_sliced(const fj_csr *g, const void *x, int32_t x_bytes, double *y, int32_t slices,
                           int32_t hub_cols, int32_t *check, int64_t *bounds, void *stream);

/*
 * The FJ opinion dynamics itself (Section 3.1, Eq. FJmodel): up to `steps`
 * synchronous updates z_i <- (s_i + sum_j w_ij z_j) / (1 + sum_j w_ij) from
 * z0 (NULL: start from s). Stops after the first step whose largest change
 * max_i |z_i' - z_i| is <= tol (tol < 0: run all steps). s, z0, z: device
 * double[n]; z receives the last iterate (z0 == z is allowed). ws: a
 * workspace of at least fj_workspace_bytes(g, 1, FJ_FP64 opts) bytes.
 * info (host, may be NULL): iters = steps taken, rel_residual = the last
 * step's largest change, status. Returns FJ_OK when tol was met or tol < 0,
 * FJ_ERR_NOT_CONVERGED when steps ran out first (z still written), and
 * FJ_ERR_BREAKDOWN on a non-finite iterate. Synchronises before returning.
 * From 65536 nodes on the sweeps run on the time-phased layout of the plan
 * (see fj_prepare), with the weighted degrees the plan holds.
 */
int fj_dynamics(const fj_csr *g, const void *plan, const double *s, const double *z0, double *z,
                int32_t steps, double tol, void *ws, size_t ws_bytes, void *stream, fj_info *info);

/*
 * Algorithm 1 (Approxim): the five indices of Section 3.2 for each of k
 * opinion vectors, each certified to relative error <= opts->eps. S as in
 * fj_solve. out and info are host arrays of k entries (info may be NULL).
 * Returns FJ_OK only when every index of every column is certified.
 * Synchronises before returning.
 */
int fj_indices(const fj_csr *g, const void *plan, int32_t k, const double *S, int64_t lds,
               const fj_opts *opts, void *ws, size_t ws_bytes, void *stream,
               fj_indices_t *out, fj_info *info);

/*
 * fj_indices without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, results and statuses as
 * fj_indices; the workspace is a static device array of
 * FJ_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library, one per GPU, held
 * until the process ends. A solve whose fj_workspace_bytes exceeds it returns
 * FJ_ERR_WORKSPACE (FP64, one vector: up to about 1.39M nodes; FJ_MIXED up to
 * about 1.67M). The call allocates no device memory and calls no allocating
 * HIP or torch routine; its first call on each device sets up (the array's
 * device address and a 2 KiB pinned control block). Batched columns always
 * run with FJ_NO_TUNE; FJ_PROFILE is rejected (FJ_ERR_INVALID_ARG). All
 * calls on one GPU share the array: the library runs them one at a time (a
 * per-device lock), so calls from several threads on one GPU serialise, and
 * each call initialises every scratch byte it reads (it keeps no state
 * between calls). Synchronises before returning.
 */
#define FJ_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int fj_indices_noalloc(const fj_csr *g, const void *plan, int32_t k, const double *S, int64_t lds,
                       const fj_opts *opts, void *stream, fj_indices_t *out, fj_info *info);

/* ---- serving ------------------------------------------------------------ */
/*
 * A continuous-batching server for index requests on resident graphs
 * (Algorithm 1 for many opinion vectors arriving over time). Graphs and
 * plans stay caller-owned on the device. Each graph with work gets a block of
 * CG state for `block_columns` opinion vectors, carved from the caller's HBM
 * arena; a block stays allocated while its graph is idle, and a graph whose
 * block does not fit first releases idle blocks of other graphs (least
 * recently used first), else waits until one becomes idle. The columns of a request (k <= block_columns vectors) enter free
 * columns of its graph's block in arrival order as soon as columns free up,
 * a request possibly in several pieces, while the other columns keep
 * iterating (continuous batching). Blocks replay HIP graphs of captured CG
 * iterations on lanes (streams) by graph size, so different graphs overlap
 * on the device and small graphs' work does not queue behind large graphs'. Every column is certified to eps exactly as fj_indices would, and
 * its result does not depend on the other requests in its block.
 * The server is driven by one host thread calling fj_server_step.
 */
typedef struct fj_server fj_server;

typedef struct fj_server_opts {
    void *arena;                /* device memory for the blocks, 256-byte aligned (caller-owned) */
    size_t arena_bytes;
    int32_t block_columns;      /* 16 or 64 opinion vectors per graph block */
    int32_t iters_per_replay;   /* CG iterations per captured HIP graph (e.g. 8) */
    double eps;                 /* certified relative error of every index, in (0, 1/2) */
    int32_t max_iter;           /* CG iterations per column over all passes; 0 = 2000 */
    int32_t precision;          /* FJ_FP64, or FJ_MIXED (FP32 inner CG, FP64 refinement, as fj_indices) */
    int32_t large_lanes;        /* streams shared by the blocks of large graphs, 1..8; 0 = 2. One more stream
                                   carries every other graph, so short work never waits in a hardware queue
                                   behind a large graph's replay */
    int32_t large_iters_per_replay;  /* CG iterations per replay for large graphs (shorter replays let requests
                                        join sooner); 0 = max(1, iters_per_replay / 4) */
    int32_t large_blocks;            /* blocks per large graph, 1..4; 0 = 1. With more than one, a request goes
                                        whole to the block of that graph with the fewest columns waiting or
                                        running, and the blocks replay on different large lanes */
    int64_t large_entries;      /* a graph with n + nnz >= this is large; 0 = 2^22 */
} fj_server_opts;

typedef struct fj_server_done {
    uint64_t request_id;
    int32_t graph_id;
    int32_t status;             /* FJ_OK when every vector of the request is certified */
    double latency_ms;          /* from fj_server_submit to the step that retired the request */
} fj_server_done;

/* Device bytes of one block for a graph of n nodes (0 for invalid arguments). */
size_t fj_server_block_bytes(int32_t n, int32_t block_columns, int32_t precision);

int fj_server_create(const fj_server_opts *opts, fj_server **out);

/* Waits for all device work of the server, then frees its host state and streams. */
int fj_server_destroy(fj_server *srv);

/*
 * Register a prepared graph (fj_prepare) that stays resident; *graph_id
 * receives its id. `stream` is the stream on which the caller produced the
 * graph and its plan (NULL: the default stream): the server's work on this
 * graph is ordered after the work queued on it so far.
 */
int fj_server_add_graph(fj_server *srv, const fj_csr *g, const void *plan, int32_t *graph_id, void *stream);

/*
 * Queue a request: k opinion vectors S (device, node-major, leading dimension
 * lds >= k, caller-owned until the request completes). out and info are host
 * arrays of k entries filled when the request completes (info may be NULL).
 * `stream` is the stream on which S was produced (NULL: the default stream):
 * the server reads S only after the work queued on it so far.
 */
int fj_server_submit(fj_server *srv, int32_t graph_id, int32_t k, const double *S, int64_t lds,
                     fj_indices_t *out, fj_info *info, uint64_t *request_id, void *stream);

/* One non-blocking scheduling round; *busy_blocks = blocks with work in flight. */
int fj_server_step(fj_server *srv, int32_t *busy_blocks);

/* Completed requests since the last poll (up to max); *count receives how many. */
int fj_server_poll(fj_server *srv, fj_server_done *done, int32_t max, int32_t *count);

/*
 * Withdraw a request that has not completed: its waiting columns leave the
 * queue, its columns in the block stop iterating and free their slots, and
 * fj_server_poll then reports it with status FJ_ERR_CANCELLED (its outputs
 * are undefined). FJ_ERR_INVALID_ARG for an unknown or already completed
 * request.
 */
int fj_server_cancel(fj_server *srv, uint64_t request_id);

#ifdef __cplusplus
}
#endif

#endif /* FJ_H */
