/*
 * hylu.h - C ABI of an MI355X (gfx950) implementation of HYLU's numerical
 * factorisation and forward-backward substitution (arXiv 2509.07690).
 *
 * The paper solves A x = b in three phases (Sec. 2): preprocessing (static
 * pivoting and scaling by maximum weighted matching, a fill-reducing ordering,
 * symbolic factorisation with flop count and supernode detection, Sec. 2.1),
 * numerical factorisation (up-looking LU with row-row, sup-row and sup-sup
 * kernels, supernode diagonal pivoting and pivot perturbation, levelised
 * parallel scheduling, Sec. 2.2 and 2.2.1), and forward-backward substitution
 * with automatic iterative refinement after perturbation (Sec. 2.3).  The
 * repeated-solve option (Sec. 3.2) is hylu_refactor: same pattern, new values.
 *
 * Conventions
 *  - CSR input: 0-based, int64 row pointers (n+1), int32 column indices
 *    sorted and unique within each row, float64 values.  Right-hand sides and
 *    solutions are n x nrhs column-major with leading dimension ld >= n.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are MI355X
 *    memory (e.g. from torch tensors on cuda:0).  `stream` is a hipStream_t
 *    (NULL = the null stream); calls taking a stream are asynchronous with
 *    respect to the host unless stated otherwise.
 *  - Ownership: the caller owns every pointer it passes.  hylu_analyze copies
 *    what it needs from its host arrays before returning.  Device inputs must
 *    stay valid until the work queued on `stream` has completed.  The handle
 *    owns all internal device memory and frees it in hylu_destroy.
 *  - Errors: every call returns a hylu_status; no C++ exception crosses this
 *    ABI.  A device failure is sticky for the handle.  A handle is not
 *    thread-safe; distinct handles are independent.
 */
#ifndef HYLU_H
#define HYLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hylu_handle_s* hylu_handle;

typedef enum {
    HYLU_OK = 0,
    HYLU_ERR_ARG = -1,              /* NULL pointer, bad size or option */
    HYLU_ERR_CSR = -2,              /* unsorted / duplicate / out-of-range column */
    HYLU_ERR_STRUCT_SINGULAR = -3,  /* no perfect matching (empty row or column, ...) */
    HYLU_ERR_NOT_ANALYZED = -4,     /* factorize/solve before analyze */
    HYLU_ERR_NOT_FACTORIZED = -5,   /* refactor/solve before factorize */
    HYLU_ERR_OOM = -6,              /* host or device allocation failed; handle stays valid */
    HYLU_ERR_DEVICE = -7,           /* a HIP call failed, or a kernel reported a failure (a pipeline-mode wait that gave up) */
    HYLU_ERR_NONFINITE = -8,        /* NaN or Inf in the input values */
    HYLU_ERR_INTERNAL = -9,
    HYLU_ERR_SCRATCH = -10,         /* hylu_solve_noalloc: n x nrhs beyond its fixed scratch */
    HYLU_WARN_IR_NOT_CONVERGED = 1  /* solve finished, backward error above ir_tol */
} hylu_status;

/* Options of the preprocessing and numerical phases. */
typedef struct {
    int32_t ordering;      /* 0 AMD, 1 nested dissection (separators from breadth-first level structures),
                              2 natural, 3 user_perm, 4 nested dissection with multilevel separators (smaller
                              separators on 3D meshes) (Sec. 2.1) */
    const int32_t* user_perm; /* host, n entries, new -> old; read by hylu_analyze only */
    int32_t static_pivot;  /* 1: maximum-product matching + scaling (Sec. 2.1); 0: identity, unit scaling */
    int32_t precision;     /* 0: FP64 factors; 1: FP32 factors + FP64 iterative refinement */
    double pivot_tau;      /* perturbation threshold relative to max|B|; <= 0: sqrt(eps) of FP64 (1.49e-8), for
                              FP32 factors too */
    double ir_tol;         /* target normwise backward error of refinement (default 1e-12) */
    int32_t ir_maxit;      /* refinement iteration cap (default 10 for FP64, 30 for FP32) */
    int32_t sn_min;        /* shortest run of rows kept as a supernode (default 2) */
    int32_t sn_max;        /* longest supernode; longer runs are split (default 1<<30) */
    int32_t kernel_mode;   /* 0 automatic choice, 1 row-row only (no supernodes), 2 supernodal */
    int32_t repeated;      /* reserved: the relative-index maps are always precomputed */
    int32_t nd_leaf;       /* nested dissection: parts up to this size are ordered by AMD (default 256) */
    double amd_dense;      /* AMD: rows with more than max(16, amd_dense*sqrt(n)) entries are ordered last;
                              0 (default): more than max(16, min(10 sqrt(n), 6 x the mean degree)) */
    double dense_tail;     /* factor the trailing block of at least this density densely (0: never; default 0.5) */
    int32_t tail_min;      /* smallest dense tail in rows (default 64) */
    int32_t tail_max;      /* largest dense tail in rows (default 32768) */
    int32_t sn_dense;      /* supernodes outside the dense tail with at least this many rows are factored by
                              the blocked panel / TRSM / MFMA-GEMM kernels instead of one workgroup each
                              (0: never; default 64) */
    int32_t sn_tile;       /* supernodes outside the dense tail with at least this many rows take their
                              updates from earlier nodes by 16-row tiles (MFMA for supernode sources) instead
                              of one row per workgroup (0: never; default 0: on the 3D grids measured so far
                              the per-tile triangular solves make it slower than the row kernel) */
    int32_t sn_inverse;    /* 1: after its LU, each supernode outside the dense tail with at most 256 rows keeps
                              the inverse of its block in pivot order, and target rows form their multipliers
                              for it as one product with that inverse instead of a triangular solve (default 1) */
    int32_t tail_sparse;   /* 1: the dense tail's trailing updates and triangular solves skip the 64 x 64 blocks
                              that are zero by structure (same factors to the bit; default 1) */
    int32_t side_rows;     /* 1: deferred standalone rows and tail rows whose sources are complete early join the
                              launches of the factor levels with fewer than 256 rows (a long tail row in pieces
                              over several of them, its sources in order) instead of waiting for the final level;
                              0: all of them in the final level (same factors either way; default 1) */
    int32_t pipeline_rows; /* pipeline mode of Sec. 2.2.1: > 0 runs every run of at least three consecutive
                              factor levels (after level 0, before the deferred final level) of at most this many
                              rows (capped at 512), whose nodes are standalone rows or supernodes of at most 64 rows
                              that no blocked or tile kernel takes, as chain launches: one workgroup whose
                              wavefronts take the rows' updates and the supernodes' block LUs in level order and
                              wait per source node (flags in LDS) instead of per level.  The factors equal bulk
                              mode's bit for bit.  The analysis checks the schedule (HYLU_ERR_INTERNAL otherwise);
                              a wait that gives up makes the factorisation return HYLU_ERR_DEVICE.  Deferred rows
                              are not placed into chain levels.  0: bulk mode only (default) */
    int32_t group_min_rows;  /* blocked dense LU (large supernodes, dense tail): row panels go in groups of four
                                (one trailing update per group) while at least this many rows remain below them
                                (<= 0: default 2048) */
    int32_t group_tail_rows; /* a block-sparse dense tail takes panel groups from this many rows on, or when its
                                plan keeps over half of the dense work (<= 0: default 16384) */
    int32_t solve_chain;     /* 1: runs of at least 3 consecutive narrow forward / backward solve levels (at most 16
                                nodes of at most 64 rows and 8192 entries in their L (U) part each) are solved by one
                                workgroup in one launch, a barrier between levels, instead of one launch per level
                                (Sec. 2.3; default 1) */
    int32_t gpu_symbolic;    /* 1: hylu_analyze computes the symbolic structure of the factors and the four level sets
                                on the current GPU (Sec. 2.1, 2.2.1): the same structure, supernodes and levels as the
                                host analysis, to the bit.  Independent blocks (a batch's members) of at most 1 << 20
                                rows each; HYLU_ERR_ARG otherwise.  0: on the host (default) */
    int32_t pipeline_spin;   /* pipeline mode: polls of a wait before it gives up, which ends every other wait of
                                the launch and makes the factorisation return HYLU_ERR_DEVICE (the factors are
                                void); <= 0: default 2^21 (tens of milliseconds, far beyond any real wait) */
    int32_t solve_split;     /* 1: a supernode of 8..64 rows with at least 8192 entries in its L region (forward
                                solve) or in its U columns past the diagonal block (backward solve) has the sums over
                                them spread over workgroups of 8 rows each, then its diagonal block solved, with the
                                same values to the bit; in the transposed solves every node of 8 rows or more has
                                its sums over the entries outside its block spread over workgroups of 8 columns,
                                then its block solved 64 columns at a time (another summation order); and the
                                large supernodes of a forward / backward solve level share their launches (their
                                gathers, then each panel step; the same values to the bit).  Default 1.  0: one
                                workgroup per node, its rows (columns) one after the other, and one launch
                                sequence per large supernode */
} hylu_options;

/* Optional device allocator (e.g. the PyTorch caching allocator).  alloc
 * returns NULL on failure; both are called from the host with the stream the
 * memory is used on. */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, void* stream);
} hylu_allocator;

typedef struct {
    int64_t n, nnz_a, nnz_l, nnz_u;   /* exact structure; U includes the diagonal */
    uint64_t flops;                   /* F = sum_k l_k (1 + 2 u_k) on the exact structure */
    uint64_t flops_padded;            /* rows padded to whole source supernodes */
    int64_t factor_entries;           /* stored panel values (padding included) */
    int32_t n_nodes, n_supernodes, rows_in_supernodes, max_supernode;
    int32_t n_levels[4];              /* factor / L solve, U solve, U^T solve, L^T solve */
    int32_t n_perturbed;              /* perturbed pivots of the last (re)factorisation */
    int32_t ir_iters;                 /* refinement steps of the last solve */
    double berr;                      /* normwise backward error ||b-Ax||_inf / (||A||_inf ||x||_inf + ||b||_inf)
                                         of the last refined solve or hylu_residual call (largest over the
                                         right-hand sides and batch members); -1 when neither has run since the
                                         last unrefined solve */
    double pivot_tau;                 /* absolute perturbation threshold used */
    int32_t tail_rows;                /* rows of the dense tail (0: none) */
    int32_t tail_panels;              /* row panels of the dense tail */
    uint64_t flops_issued;            /* flops the kernels issue (padding, dense tail included) */
    double resid_1;                   /* the accuracy measure of Sec. 3.3, ||Ax-b||_1 / ||b||_1, of the same
                                         solution as berr (largest over right-hand sides and members); -1 likewise */
    int32_t n_dense_sn;               /* supernodes outside the tail factored by the blocked dense kernels */
    int32_t sn_groups, tail_groups;   /* panel groups of more than one panel in their plans / in the tail's */
    int32_t pipe_tasks;               /* tasks of the chain launches (row updates and supernode block LUs;
                                         0: bulk mode only) */
    int32_t chain_levels;             /* forward + backward solve levels solved inside chains (solve_chain) */
    double sym_ms;                    /* wall time of the symbolic factorisation, supernodes and level sets in
                                         hylu_analyze (host or GPU, transfers included) */
    double sym_kernel_ms;             /* of which GPU kernel time (gpu_symbolic; else 0) */
    uint64_t sym_hash;                /* hash of the compressed structure and the level sets (equal hashes: equal
                                         analyses) */
    int32_t split_sn;                 /* supernode solves (Sec. 2.3), summed over the forward, backward and two
                                         transposed solves, whose sums over the entries outside the node's block are
                                         spread across workgroups by rows (columns when transposed; solve_split) */
} hylu_info;

/* Analysis export for checking: every array is host memory the caller
 * allocates with the sizes from hylu_get_info (n, nnz_a, n_nodes). */
typedef struct {
    int32_t* perm_r;     /* n: row i' of B is row perm_r[i'] of A */
    int32_t* perm_c;     /* n: column j' of B is column perm_c[j'] of A */
    double* dr;          /* n: row scaling, by row of A */
    double* dc;          /* n: column scaling, by column of A */
    int32_t* node_ptr;   /* n_nodes+1: row boundaries of the nodes */
    uint8_t* is_sn;      /* n_nodes: 1 for a supernode */
    int32_t* levels;     /* 4*n_nodes: level of each node in the four task graphs */
} hylu_symbolic_view;

hylu_status hylu_default_options(hylu_options* opt);
const char* hylu_status_string(hylu_status s);

/* Create a handle.  alloc may be NULL (hipMalloc/hipFree are used). */
hylu_status hylu_create(hylu_handle* h, const hylu_allocator* alloc);
hylu_status hylu_destroy(hylu_handle h);

/* Preprocessing (Sec. 2.1), on the host: validates the CSR, computes the
 * matching/scaling, the ordering, the symbolic structure, flop count,
 * supernodes, the level sets (Sec. 2.2.1) and the device layout, and uploads
 * the index tables.  row_ptr, col, val: host.  val is read for the matching. */
hylu_status hylu_analyze(hylu_handle h, int32_t n, const int64_t* row_ptr, const int32_t* col,
                         const double* val, const hylu_options* opt);

/* Batched analysis of `count` matrices of uneven sizes on one handle.  The
 * handle's matrix is their block diagonal: member k owns rows and columns
 * [row_off[k], row_off[k+1]) and values [nnz_off[k], nnz_off[k+1]) in member
 * order (hylu_batch_offsets), so hylu_factorize / hylu_refactor take the
 * members' value arrays back to back and hylu_solve their right-hand sides
 * back to back.  Every member is matched, scaled and ordered on its own (on
 * host threads); the structural analysis then runs once on the union, so the
 * members' levels share every launch and one refactorisation of the whole
 * batch replays as one HIP graph.  opt->ordering 3 (user) is rejected and
 * dense_tail is not used.  Iterative refinement stops on the largest
 * backward error over the members and right-hand sides.  n, row_ptr, col,
 * val: host arrays of count entries, each pointing at a member's host CSR. */
hylu_status hylu_analyze_batch(hylu_handle h, int32_t count, const int32_t* n, const int64_t* const* row_ptr,
                               const int32_t* const* col, const double* const* val, const hylu_options* opt);

/* Member layout of a batched handle (one member after hylu_analyze):
 * *count, and row_off / nnz_off of count+1 entries each (host; may be null). */
hylu_status hylu_batch_offsets(hylu_handle h, int32_t* count, int64_t* row_off, int64_t* nnz_off);

/* Numerical factorisation with pivot search (Sec. 2.2).  d_val: device,
 * nnz float64 values in the CSR order given to hylu_analyze. */
hylu_status hylu_factorize(hylu_handle h, const double* d_val, void* stream);

/* Refactorisation with new values on the same pattern, reusing the pivot
 * order of the last hylu_factorize (the repeated-solve scenario, Sec. 3.2).
 * Perturbation stays active.  The level sequence is replayed as a HIP graph,
 * one per d_val address (at most 16 are kept; the cache is emptied, after a
 * device synchronisation, when a 17th address arrives). */
hylu_status hylu_refactor(hylu_handle h, const double* d_val, void* stream);

/* Forward-backward substitution (Sec. 2.3): solves A x = b (transpose = 0) or
 * A^T x = b (transpose = 1) for nrhs columns.  d_b, d_x: device, n x nrhs,
 * column-major, leading dimension ld; d_x may equal d_b.  Iterative
 * refinement in FP64 runs when a pivot was perturbed or precision = 1; its
 * residual uses the handle's copy of the values of the last (re)factorisation.
 * Refinement stops at ir_tol, on stagnation (a correction that does not halve
 * the backward error) or after ir_maxit corrections, and returns the iterate
 * with the smallest backward error (HYLU_WARN_IR_NOT_CONVERGED when that is
 * above ir_tol).  Synchronises the stream when refinement runs (the stopping
 * test reads the backward error on the host).  Graphs are cached per
 * (d_b, d_x, nrhs, ld, transpose) like those of hylu_refactor. */
hylu_status hylu_solve(hylu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                       int32_t transpose, void* stream);

/* hylu_solve without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same substitution and refinement as hylu_solve, with
 * its work vectors in a fixed device array of 64 MiB that the library holds
 * on each GPU it runs on (set up by the first hylu_factorize on that device;
 * no hipMalloc, hipFree or allocating library call here, and no graph: the
 * launches go straight onto `stream`).  Limits: at most 64 right-hand sides
 * and 2 n nrhs (factor-precision size) + 3 n nrhs 8 bytes of work vectors
 * plus the norms, within 64 MiB (FP64 factors: n nrhs up to about 1.6e6);
 * beyond that HYLU_ERR_SCRATCH and a message on stderr.  transpose = 1 needs
 * the transposed column lists, built by an earlier hylu_solve with
 * transpose = 1 on this handle; HYLU_ERR_ARG otherwise.  Every call on one
 * GPU shares that GPU's scratch (its contents are those the last call left):
 * calls that overlap in time on one GPU, from any handles or streams, race
 * and must be serialised by the caller.  Arguments, layout and results as for
 * hylu_solve. */
hylu_status hylu_solve_noalloc(hylu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                               int32_t transpose, void* stream);

/* Gradient of a scalar loss through X = A^{-1} B with respect to the values of
 * A (the adjoint of the solve): d_gval[p] = -sum_k Lambda[row p, k] X[col p, k]
 * for every stored entry p, where Lambda = A^{-T} dL/dX (from hylu_solve with
 * transpose = 1) and the sum runs over the nrhs columns.  Device arrays:
 * d_lambda and d_x are n x nrhs column-major with leading dimension ld >= n,
 * d_gval holds nnz entries in the CSR order given to hylu_analyze and is
 * overwritten.  HYLU_ERR_ARG for a null pointer, nrhs <= 0 or ld < n. */
hylu_status hylu_grad_values(hylu_handle h, const double* d_lambda, const double* d_x, int32_t nrhs, int64_t ld,
                             double* d_gval, void* stream);

/* Accuracy of a solution (Sec. 3.3): r = b - op(A) x in FP64 on the values of
 * the last (re)factorisation (op(A) = A, or A^T when transpose = 1), then the
 * normwise backward error ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) in
 * *berr and the paper's measure ||r||_1 / ||b||_1 in *resid1 (host, either may
 * be null), each the largest over the nrhs right-hand sides and the members of
 * a batch.  d_b, d_x: device, n x nrhs column-major, leading dimension ld.
 * Synchronises the stream; the values also appear in hylu_get_info. */
hylu_status hylu_residual(hylu_handle h, const double* d_b, const double* d_x, int32_t nrhs, int64_t ld,
                          int32_t transpose, void* stream, double* berr, double* resid1);

/* Statistics of the analysis and of the last numerical calls (synchronises). */
hylu_status hylu_get_info(hylu_handle h, hylu_info* out);

/* Copies of the analysis results (host arrays, sizes from hylu_get_info). */
hylu_status hylu_export_symbolic(hylu_handle h, const hylu_symbolic_view* v);

/* Copies of the factors after a (re)factorisation, as host arrays in the
 * oracle-independent panel form: values (factor_entries of float64), the
 * panel offsets and widths, and the pivot order.  For checking.  Sizes:
 * vals factor_entries; node_voff n_nodes+1 (int64); node_lw, node_W n_nodes;
 * cols: sum of W; piv n (global column of each row's pivot). */
hylu_status hylu_export_factors(hylu_handle h, double* vals, int64_t* node_voff, int32_t* node_lw,
                                int32_t* node_W, int64_t* node_coff, int32_t* cols, int32_t* piv);
hylu_status hylu_export_sizes(hylu_handle h, int64_t* ncols_total);

/* Autotuner of the factorisation's launch shapes: for every level, the threads
 * given to one target row (64, 128, 256 or 1024) and to one supernode's
 * internal LU (64 or 256).  Runs `reps` rounds of four complete refactorisations with
 * d_val (each trial gives every level one shape; every shape computes
 * bit-identical factors), times each level's launches with HIP events on
 * `stream`, keeps the fastest shape per level and drops the refactorisation
 * graphs captured before.  Leaves the factors of d_val.  ms_default /
 * ms_tuned (host, may be null): summed level times with the built-in shapes
 * and with the chosen ones.  Needs a prior hylu_factorize (pivot order). */
hylu_status hylu_autotune(hylu_handle h, const double* d_val, void* stream, int32_t reps, double* ms_default,
                          double* ms_tuned);

/* Per-kernel-class measurement of one refactorisation + solve, run eagerly
 * (not from the graph) with a pair of HIP events around every launch on
 * `stream`.  For every class: launches, summed device time, and the
 * algorithmic bytes and flops of those launches (computed on the host from the
 * layout: values and indices each launch must read or write once, flops of
 * the entries it updates).  d_b, d_x: one right-hand side (device).  Returns
 * the number of classes written (at most max_classes) in *count. */
typedef struct {
    char name[32];
    int32_t launches;
    double ms;
    double bytes;
    double flops;
} hylu_kernel_stats;
hylu_status hylu_profile(hylu_handle h, const double* d_val, const double* d_b, double* d_x, void* stream,
                         hylu_kernel_stats* stats, int32_t max_classes, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* HYLU_H */
