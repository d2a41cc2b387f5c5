// Launch interface of the gfx950 kernels (HYLU numerical factorisation and
// substitution).  All pointers are device pointers; every launcher enqueues on
// `stream` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hylu {

// Per-edge descriptor: target node t takes source node s.  Precomputed so a
// kernel reads one 48-byte record per source instead of chasing node arrays.
struct EdgeDesc {
    int64_t uoff;   // value offset of the source's diagonal block (voff[s] + lw[s])
    int64_t roff;   // offset of the relative map of the source's T into the target
    int32_t Ws;     // source panel width
    int32_t ms;     // source rows
    int32_t ws;     // source T width
    int32_t lp;     // slot of the source's first column in the target's L region
    int32_t r0s;    // first row of the source (pivot table offset)
    int32_t srcp;   // task of the target's chain launch that completes the source, else -1
    int64_t ioff;   // offset of the inverse of the source's block in pivot order, or -1
};

// Inverse of a supernode's block in pivot order: with U_pp(b, b') = U(b, pl_b')
// (upper triangular), Uinv = U_pp^{-1} is stored row-major (m x m) at
// uinv + inv_off[v]; a target row's multipliers for the supernode are then
// l = x_p Uinv (x_p: the row's entries at the source's pivot columns in pivot
// order) with no sequential dependency.
constexpr int32_t kInvMax = 256;   // largest supernode given an inverse

// Device view of the panel layout.
struct DevLayout {
    int32_t n, nnodes;
    int32_t tail_node0;     // nodes from here on belong to the dense tail
    const int32_t* r0;
    const int32_t* m;
    const int32_t* lw;
    const int32_t* W;
    const int64_t* voff;
    const int64_t* coff;
    const int32_t* cols;
    const int64_t* eptr;
    const EdgeDesc* edges;
    const int32_t* rel;
    const int32_t* row_node;
    const void* uinv;       // inverses of the supernode blocks (factor precision), see EdgeDesc::ioff
    int32_t* pl;            // per row: natural local block column of its pivot
    int32_t* qinv;          // per column: row whose pivot is this column
    // column lists for the transposed solves: entries of other nodes' panels
    const int64_t* ut_ptr;  // per column (n+1): T-region entries in that column
    const int64_t* ut_slot;
    const int32_t* ut_row;
    const uint8_t* dense_sn;  // per node: 1 when the forward / backward solves take it by the dense-view kernels
    const int64_t* lt_ptr;  // per column (n+1): L-region entries in that column
    const int64_t* lt_slot;
    const int32_t* lt_row;
    // compact rows (dense-tail nodes): per node the number of positions its
    // outside sources touch (0: none kept), and those positions (sorted, from
    // cpos_off[v]); crel: the relative maps with those of a compact node's
    // sources indexing that list instead of the row (rel: always the row)
    const int32_t* cw;
    const int64_t* cpos_off;
    const int32_t* cpos;
    const int32_t* crel;
    // small supernodes whose block LU the row launch of their level does
    // (snfuse[v] = 1): per node the rows finished so far (zero between
    // factorisations)
    const uint8_t* snfuse;
    int32_t* sncnt;
};

// Dense tail: rows and columns [t0, n) of the factors as one dense block whose
// rows live inside their nodes' panels (row a starts at vals + trow[a]).  The
// same view describes a large supernode factored by the same blocked kernels:
// its m rows, its block plus T columns, pivot windows its whole block.
struct TailView {
    int32_t mT, t0;
    int32_t nc;             // columns (>= mT): a supernode's block plus its T columns; mT for the tail
    const int64_t* trow;    // value offset of tail row a's dense part
    const int32_t* tlo;     // tail-local block range of row a's node: its pivot window
    const int32_t* thi;
    int32_t* tpiv;          // tail-local column of row a's pivot
    int32_t* tstep;         // per tail column: the tail row that pivots it (INT32_MAX before)
    void* lbuf;             // kNB x mT workspace: the current panel's multipliers, transposed
};

// Several dense views in one launch (the large supernodes of one level): a
// table of the views, and per workgroup its view, its block within that
// view's own launch and the operation's arguments.
struct ViewDesc {
    TailView TV;
    const int32_t* sp;      // solve panels (p0, p1 pairs)
    void* inv;              // inverses of their diagonal blocks
};
// one workgroup of a forward / backward solve step of one large supernode,
// several supernodes per launch: the view, the step's panels (p: the one
// whose contribution goes out, empty on the first step; q: the one solved
// with the inverse of its diagonal block, number `inv` of the view's
// inverses), the range of rows the contribution reaches and the
// workgroup's block (0: the solve of q; 1..: four rows each)
struct SolveJob {
    int32_t view, blk, p0, p1, q0, q1, inv, first, count;
};
struct ViewJob {
    int32_t v;              // view
    int32_t blk;            // TRSM block; GEMM tile (ty << 16 | tx); inverse block (2 panel + kind)
    int32_t a[6];           // panel: p0 p1 c0 c1 | TRSM: p0 p1 c1 nA kb0 kof | GEMM: kb0 K rb re cg0 mstep
};
// every job's panel by the wide-window kernel with the window in LDS
// (lds: the largest job's bytes); TRSM, trailing GEMM (every tile, one
// panel) and diagonal-block inverses of the jobs
hipError_t launch_tail_panel_views(bool fp32, const DevLayout& D, const ViewDesc* vd, void* vals, const ViewJob* jobs,
                                   int32_t njobs, size_t lds, double tau, int32_t* pert, int32_t search, hipStream_t st);
hipError_t launch_tail_trsm_views(bool fp32, const ViewDesc* vd, void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st);
hipError_t launch_tail_gemm_views(bool fp32, const ViewDesc* vd, void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st);
hipError_t launch_tail_dinv_views(bool fp32, const ViewDesc* vd, const void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st);
// LDS bytes of the wide-window panel kernel with the window staged (0 when it
// does not fit that kernel)
size_t tail_panel_wide_lds(bool fp32, int32_t np, int32_t wc);

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_tail_init(const TailView& T, hipStream_t st);
hipError_t launch_tail_panel(bool fp32, const DevLayout& D, const TailView& T, void* vals, int32_t p0, int32_t p1,
                             int32_t c0, int32_t c1, double tau, int32_t* pert, int32_t search, hipStream_t st);
// panels are processed in groups of up to kGroup: the rows of a group take the
// group's earlier panels left-looking, the rows below the group take the whole
// group in one trailing update (K up to kGroup * 64), so the trailing matrix is
// read and written once per group instead of once per panel.  lbuf holds
// kGroup * 64 rows (k-major), panel j of a group at rows kof..kof+np.
constexpr int kNB = 64;      // rows of a dense-view panel (solves) and of its diagonal block
constexpr int kGroup = 4;
// panel [p0, p1): U right of the window, and the multipliers of the rows
// below (their pivot columns already carry the group's earlier panels),
// written to lbuf rows kof.. (kb0: first panel row of the group, unused here)
// blocks (optional, device): the blocks to run, indices into [0, nA + nB) with
// nA = column blocks of U right of the window, nB = row blocks below the panel;
// a row block flagged kTrsmZero only writes zero multipliers to lbuf
constexpr int32_t kTrsmZero = 1 << 30;
hipError_t launch_tail_trsm(bool fp32, const TailView& T, void* vals, int32_t p0, int32_t p1, int32_t c1, int32_t kb0,
                            int32_t kof, const int32_t* blocks, int32_t nblocks, hipStream_t st);
// rows [rb, re): X[r][c] -= sum_{k < K} lbuf[k][r] X[kb0 + k][c] over the
// columns from cg0 still unpivoted before step mstep, or (gnp > 0) over the
// pivot columns of panel rows gp0 .. gp0+gnp.  tiles (optional, device):
// ntiles entries (ty << 16) | (tx << 4) | panel mask, or kTileNone; kbnd
// (host, optional): the K offsets 0 <= kbnd[1] <= kbnd[2] <= kbnd[3] <= K of
// the group's panels the mask bits stand for.
constexpr uint32_t kTileNone = 0xFFFFFFFFu;
hipError_t launch_tail_gemm(bool fp32, const TailView& T, void* vals, int32_t kb0, int32_t K, int32_t rb, int32_t re,
                            int32_t cg0, int32_t mstep, int32_t gp0, int32_t gnp, const uint32_t* tiles,
                            int32_t ntiles, const int32_t* kbnd, hipStream_t st);
// dense tail solves; y/x/h/w are the solve work vectors (n x nrhs, factor precision)
hipError_t launch_tail_lext(bool fp32, const DevLayout& D, const void* vals, int32_t tail_node0, int32_t t0,
                            void* y, int32_t nrhs, hipStream_t st);
hipError_t launch_tail_utext(bool fp32, const DevLayout& D, const TailView& T, const void* vals, void* h,
                             const void* w, int32_t nrhs, hipStream_t st);
// inverses of the diagonal blocks of the nsp solve panels (spanels: device
// pairs p0, p1): (I + L)^-1 and U^-1 in pivot order, 64 x 64 column-major each,
// panel s's at out + (2 s + {0, 1}) * 64 * 64 values
hipError_t launch_tail_dinv(bool fp32, const TailView& T, const void* vals, const int32_t* spanels, int32_t nsp,
                            void* out, hipStream_t st);
// one step of a dense view's forward (mode 0, L) or backward (mode 1, U) solve,
// or of the transposed ones (mode 2, U^T ascending; mode 3, L^T descending;
// the tail only): the contribution of panel [p0, p1) to every target still to
// come, and the diagonal solve of the next panel [q0, q1) (adjacent to it)
// with its inverse inv (L's for modes 0 and 3, U's for 1 and 2)
hipError_t launch_tail_step(bool fp32, const TailView& T, const void* vals, int32_t p0, int32_t p1, int32_t q0, int32_t q1,
                            const void* inv, int32_t n, void* y, void* x, int32_t nrhs, int32_t mode, hipStream_t st);
// one large supernode's rows (dense view TV, node v): forward, the L-region
// gather y_i -= sum_{t < lw} L(i, t) y[source of t]; backward, the T-region
// gather y_i -= sum_{t in T} U(i, t) x[column t] (before its block panels)
hipError_t launch_sn_lext(bool fp32, const DevLayout& D, const TailView& TV, const void* vals, int32_t v, void* y,
                          int32_t nrhs, hipStream_t st);
hipError_t launch_sn_utext(bool fp32, const DevLayout& D, const TailView& TV, const void* vals, int32_t v, void* y,
                           const void* x, int32_t nrhs, hipStream_t st);
// the same gathers for several large supernodes in one launch (jobs: node,
// block of four rows pairs; upper: the backward solve's T-region gathers)
hipError_t launch_sn_ext_views(bool fp32, const DevLayout& D, const void* vals, const int32_t* jobs, int32_t njobs,
                               void* y, const void* x, int32_t nrhs, int32_t upper, hipStream_t st);
// one forward (mode 0) or backward (mode 1) solve step of several large
// supernodes (views vd) in one launch, a SolveJob per workgroup; each
// workgroup computes what the same block of launch_tail_step computes
hipError_t launch_view_steps(bool fp32, const ViewDesc* vd, const SolveJob* jobs, int32_t njobs, const void* vals,
                             int32_t n, void* y, void* x, int32_t nrhs, int32_t mode, hipStream_t st);
hipError_t launch_scatter(bool fp32, const double* aval, const int64_t* amap, const double* asr,
                          const double* asc, int64_t nnz, void* vals, double* acopy, hipStream_t st);
hipError_t launch_init_pivots(const DevLayout& D, hipStream_t st);
// nt: threads per row (64, 128 or 256; 0 picks by the widest row of the launch)
// stage: source entries staged per batch in LDS (a multiple of 64, from
// kStageSmall to kStageMax); lds_cap: the row accumulator sits in LDS for rows
// up to this width (0: the default 4096).  Levels of few rows run one row per
// CU and may take a large stage and cap; factor_rows_lds gives the dynamic
// LDS bytes of a choice, at most kLdsMax: the 160 KiB a workgroup may hold
// less 1 KiB for the kernel's static LDS and its alignment (a dispatch that
// asks for more than the device allows is refused by the queue).
constexpr int32_t kStageSmall = 1024, kStageMax = 8192;
constexpr size_t kLdsMax = 160 * 1024 - 1024;
size_t factor_rows_lds(bool fp32, int32_t stage, int32_t cap);
// pivot check (perturbation) of standalone rows that take no updates
hipError_t launch_perturb_rows(bool fp32, const DevLayout& D, void* vals, const int32_t* rows, int32_t count,
                               double tau, int32_t* pert, hipStream_t st);
// ranges (optional, device): per row, the first and one-past-last index of
// the sources it takes in this launch (a long row's sources may be split over
// several launches, in order); null: every source.  A row of a supernode with
// D.snfuse set also counts itself done, and the last row of that supernode
// factors its block (pivot search when `search`) and, when inv_off[v] >= 0,
// its inverse
hipError_t launch_factor_rows(bool fp32, const DevLayout& D, void* vals, const int32_t* rows, const int64_t* ranges,
                              int32_t nrows, int32_t maxW, double tau, int32_t* pert, int32_t nt, int32_t stage,
                              int32_t lds_cap, int32_t search, const int64_t* inv_off, hipStream_t st);
// row tiles (16 rows) of supernode targets: tiles = pairs (node, first local row)
hipError_t launch_factor_tile(bool fp32, const DevLayout& D, void* vals, const int32_t* tiles, int32_t ntiles,
                              hipStream_t st);
// pipeline mode (Sec. 2.2.1): one workgroup of kChainThreads threads whose nw
// wavefronts take the ntask tasks in order, task t by wavefront t mod nw:
// tasks[t] >= 0 the outside updates of that row, -(v + 1) the block LU (and
// inverse) of supernode v after its row tasks (the m tasks before it when it
// has sources).  A row waits per source on the tasks of the launch
// (EdgeDesc::srcp: the task completing the source node); a row of at most cap
// columns sits in LDS; sw (>= kInvMax) staging values per wavefront; sthr[t]
// the staging size the bulk row kernel would use for the task's level (it
// decides the arithmetic path, so the factors equal bulk mode's).  A wait
// gives up after `spin` polls and sets pert[1] (a device error for the host).
constexpr int kChainThreads = 512;   // eight wavefronts (256 VGPRs each)
hipError_t launch_factor_chain(bool fp32, const DevLayout& D, void* vals, const int32_t* tasks, const int32_t* sthr,
                               int32_t ntask, int32_t nw, int32_t cap, int32_t sw, double tau, int32_t* pert,
                               int32_t search, const int64_t* inv_off, int32_t spin, hipStream_t st);
// dynamic LDS bytes of the chain workgroup
size_t chain_lds(bool fp32, int32_t ntask, int32_t nw, int32_t cap, int32_t sw);
// nt: threads per supernode (64 or 256; 0 = 256)
// inverses of the blocks of the listed supernodes (each 2 <= m <= kInvMax)
hipError_t launch_sn_inverse(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                             int32_t maxm, const int64_t* inv_off, void* uinv, hipStream_t st);
// inv_off (optional, device): per node the offset of its block inverse in
// D.uinv or -1; listed nodes with one compute it right after their LU
hipError_t launch_factor_snlu(bool fp32, const DevLayout& D, void* vals, const int32_t* nodes, int32_t count,
                              int32_t maxm, double tau, int32_t* pert, int32_t search, int32_t nt,
                              const int64_t* inv_off, hipStream_t st);
// forward L solve of a level.  The one-wavefront kernel takes the `count`
// nodes of `nodes` except supernodes of sn_min..64 rows (sn_min > 0; count 0:
// no launch); those are listed in sn_nodes (solved by one four-wavefront
// workgroup each) or, with a long L region, in split_nodes: their outside sums
// first by `ntasks` workgroups of kSplitRows rows (tasks: node, first row
// pairs), then their diagonal blocks
constexpr int kSplitRows = 8;
hipError_t launch_lsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                         const int32_t* sn_nodes, int32_t sn_count, const int32_t* split_nodes, int32_t split_count,
                         const int32_t* tasks, int32_t ntasks, void* y, int32_t nrhs, int32_t sn_min, hipStream_t st);
// backward U solve of a level, the same way (split_nodes: the gathers over
// the columns past the block spread by rows, subtracted from y in place)
hipError_t launch_usolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                         const int32_t* sn_nodes, int32_t sn_count, const int32_t* split_nodes, int32_t split_count,
                         const int32_t* tasks, int32_t ntasks, void* y, void* x, int32_t nrhs, int32_t sn_min,
                         hipStream_t st);
// a chain of narrow solve levels [l0, l1) in one launch of one workgroup
// (kChainWaves wavefronts, a node per wavefront, a barrier between levels);
// lev_ptr: the level pointers of the solve graph's node list `nodes`; every
// node of those levels has at most kChainRows rows and no dense view
constexpr int kChainWaves = 16;
constexpr int kChainRows = 64;
hipError_t launch_lsolve_chain(bool fp32, const DevLayout& D, const void* vals, const int32_t* lev_ptr,
                               const int32_t* nodes, int32_t l0, int32_t l1, void* y, int32_t nrhs, hipStream_t st);
hipError_t launch_usolve_chain(bool fp32, const DevLayout& D, const void* vals, const int32_t* lev_ptr,
                               const int32_t* nodes, int32_t l0, int32_t l1, const void* y, void* x, int32_t nrhs,
                               hipStream_t st);
// transposed solves of a level: the `count` nodes of `nodes` column by column
// (one workgroup each), the blk_count nodes of blk_nodes by their outside
// sums (ntasks workgroups of kSplitRows columns; tasks: node, first column)
// and then their blocks 64 columns at a time.  U^T: h is the permuted
// right-hand side, updated in place; L^T: in place in w
hipError_t launch_utsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                          const int32_t* blk_nodes, int32_t blk_count, const int32_t* tasks, int32_t ntasks,
                          void* h, void* w, int32_t nrhs, hipStream_t st);
hipError_t launch_ltsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                          const int32_t* blk_nodes, int32_t blk_count, const int32_t* tasks, int32_t ntasks,
                          void* w, int32_t nrhs, hipStream_t st);
// c[i + r n] = scale[perm[i]] * src[perm[i] + r ld]  (gather, into the factor precision)
hipError_t launch_permute_in(bool fp32, int32_t n, int32_t nrhs, const int32_t* perm, const double* scale,
                             const double* src, int64_t ld, void* dst, hipStream_t st);
// dst[perm[j] + r ld] (+)= scale[perm[j]] * z[j + r n]  (scatter from the factor precision)
hipError_t launch_permute_out(bool fp32, int32_t n, int32_t nrhs, const int32_t* perm, const double* scale,
                              const void* z, double* dst, int64_t ld, int32_t accumulate, hipStream_t st);
// r = b - op(A) x (FP64), op = A (CSR) or A^T (via the column copy)
hipError_t launch_residual(int32_t n, int32_t nrhs, const int64_t* rp, const int32_t* ci, const double* av,
                           const double* b, int64_t ldb, const double* x, int64_t ldx, double* r, hipStream_t st);
// per-RHS, per-segment norms (segments: the members of a batch, seg[row] ->
// member, or one segment when seg is null), kNormSlots values each:
// out[kNormSlots (r nseg + s) + q] for q = 0 max|r|, 1 max|x|, 2 max|b|,
// 3 sum|r|, 4 sum|b|; out[kNormSlots (nrhs nseg + s)] = max row abs sum of A
constexpr int kNormSlots = 6;
hipError_t launch_norms(int32_t n, int32_t nrhs, const int64_t* rp, const double* av, const double* r,
                        const double* x, int64_t ldx, const double* b, int64_t ldb, const int32_t* seg,
                        int32_t nseg, double* out, hipStream_t st);
hipError_t launch_gather_values(int64_t nnz, const int64_t* idx, const double* src, double* dst, hipStream_t st);
// g[p] = -sum_k lam[row p, k] x[col p, k] over nrhs columns of leading dimension ld
hipError_t launch_grad(int32_t n, int32_t nrhs, int64_t ld, const int64_t* rp, const int32_t* ci, const double* lam,
                       const double* x, double* g, hipStream_t st);

}  // namespace hylu
