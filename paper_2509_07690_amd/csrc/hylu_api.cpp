// C ABI of the MI355X HYLU solver: handle life cycle, preprocessing on the
// host (Sec. 2.1), level-scheduled numerical factorisation (Sec. 2.2, 2.2.1),
// substitution with refinement (Sec. 2.3) and the repeated-solve path
// (Sec. 3.2) replayed from a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <atomic>
#include <array>
#include <vector>

#include <chrono>

#include "../../include/hylu.h"
#include "analysis.hpp"
#include "kernels.hpp"

using namespace hylu;

// Scratch of hylu_solve_noalloc: a fixed device array (each GPU the library
// runs on holds its own copy until the process ends).  Host code never passes
// its name to a kernel: the address on a device comes from
// hipGetSymbolAddress, taken once per device at set-up (scratch_setup).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int32_t kNoallocRhs = 64;     // right-hand sides per call of hylu_solve_noalloc
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the address of this device's scratch (the current device must be `dev`)
hipError_t scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
    return hipSuccess;
}

void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// per-launch timing used by hylu_profile: when active, every launch of the
// factor and solve sequences is bracketed by events and attributed to a class
struct Profiler {
    bool on = false;
    hipStream_t st = nullptr;
    struct Rec { int cls; hipEvent_t a, b; double bytes, flops; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipEvent_t ev() {
        if (used == pool.size()) { hipEvent_t e; if (hipEventCreate(&e) != hipSuccess) return nullptr; pool.push_back(e); }
        return pool[used++];
    }
};

struct LevelTasks {
    std::vector<int64_t> row_ptr;     // per level into rows
    std::vector<int32_t> maxW;        // per level
    std::vector<int64_t> sn_ptr;      // per level into snodes
    std::vector<int32_t> maxm;
    std::vector<int32_t> rows, snodes;
    std::vector<int32_t> row_nt, sn_nt;  // per level: threads per row / per supernode (0: built-in rule)
    std::vector<int32_t> row_stage;      // per level: source entries staged per batch by the row kernel
    std::vector<int32_t> row_cap;        // per level: widest row whose accumulator sits in LDS
    std::vector<int64_t> tile_ptr;        // per level into tiles (pairs: node, first local row)
    std::vector<int32_t> tiles;
    std::vector<int64_t> rrange;          // per entry of rows: its first and one-past-last source
    int32_t tune_rows = 0, tune_sn = 0;  // when nonzero, every level uses this (autotuner trials)
    // pipeline mode: the levels with chain_lev[l] set run as chain launches
    // (runs of consecutive narrow levels); chain_start[l]: the first launch
    // of the run starting at level l, else -1
    std::vector<char> chain_lev;
    std::vector<int32_t> chain_start;
    struct Chain {
        int32_t l0, l1;               // its levels
        int64_t t0, t1;               // its nodes in ctask
        int32_t nw, cap;              // wavefronts of the chain workgroup, widest row kept in LDS
    };
    std::vector<Chain> chains;
    // the launches' tasks in order: a row (>= 0) or the block LU of supernode
    // v (-(v + 1)); the bulk staging size of their level
    std::vector<int32_t> ctask, ctask_sthr;
    std::vector<int32_t> chain_of, chain_idx; // per node: its chain launch (-1: none), the task completing it there
    std::vector<int64_t> lvrows;              // per chain level: the rows a bulk launch of it would take
    std::vector<int32_t> node_level;  // execution level of every node
};

// work vectors of a solve with refinement: y, z (n x nrhs, factor precision),
// r, bc, xbest (n x nrhs, FP64), the norms of the residual test on the device
// and their pinned host copy
struct SolveWs {
    void* y = nullptr;
    void* z = nullptr;
    double* r = nullptr;
    double* bc = nullptr;                   // copy of b when refining in place
    double* xbest = nullptr;                // best refinement iterate so far
    double* norms = nullptr;
    double* h_norms = nullptr;              // pinned
};

// one launch of the blocked dense LU of a view (a large supernode or the tail)
struct DenseOp {
    int32_t kind = 0;                 // 0 panel, 1 TRSM, 2 trailing GEMM
    int32_t a[8] = {};                // panel: p0 p1 c0 c1 | TRSM: p0 p1 c1 kb0 kof | GEMM: kb0 K rb re cg0 mstep gp0 gnp
    int32_t kb[kGroup + 1] = {};      // GEMM: K offsets of the group's panels
    int64_t list = -1;                // offset of its tile / block list; -1: every tile
    int32_t count = 0;
    double elems = 0.0, flops = 0.0;  // algorithmic traffic (values) and flops
};

}  // namespace

struct hylu_handle_s {
    hylu_allocator alloc{};
    bool has_alloc = false;
    hipStream_t cap_stream = nullptr;
    int device = 0;
    // analysis
    hylu_options opt{};
    bool analyzed = false, factorized = false, sticky_error = false, uploaded = false;
    int32_t n = 0;
    int64_t nnz = 0;
    Csr A;                                  // pattern (values from analyze)
    std::vector<int32_t> perm_r, perm_c;
    std::vector<double> dr, dc;
    Symbolic sym;
    Nodes nodes;
    Layout lay;
    LevelTasks ft;
    double tau = 0.0;
    int32_t max_sn = 0;
    bool fp32 = false;
    // device memory
    std::vector<void*> blocks;
    DevLayout D{};
    void* vals = nullptr;                   // factor panels (double or float)
    int64_t* d_amap = nullptr;
    double *d_asr = nullptr, *d_asc = nullptr;
    int32_t *d_rows = nullptr, *d_snodes = nullptr, *d_tiles = nullptr;
    int64_t* d_rrange = nullptr;
    int32_t* d_lev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    TailView TV{};
    int32_t *d_ctask = nullptr, *d_csthr = nullptr;   // the chain launches' nodes and staging sizes
    // large supernodes outside the tail, factored by the blocked dense kernels
    struct DenseSn {
        int32_t v, level;
        TailView TV;
        std::vector<Layout::Panel> panels, spanels;
        std::vector<DenseOp> ops;
        int32_t* d_sp = nullptr;            // solve panels (p0, p1 pairs)
        void* d_inv = nullptr;              // inverses of their diagonal blocks (L and U, 64 x 64 each)
    };
    std::vector<DenseOp> tail_ops;          // the dense tail's launches, block-sparse when its masks are known
    std::vector<uint32_t> tail_list;        // their tile / block lists
    uint32_t* d_tail_list = nullptr;
    int32_t* d_tsp = nullptr;               // the tail's solve panels (p0, p1 pairs)
    void* d_tinv = nullptr;                 // inverses of their diagonal blocks (L and U, 64 x 64 each)
    double tail_flops = 0.0;
    int32_t tail_groups = 0, sn_groups = 0;  // panel groups (of more than one panel) of the tail / the large supernodes
    std::vector<DenseSn> dsn;
    // the large supernodes of a level whose launches are shared: per level the
    // steps (panels of all of them, then their TRSMs, then their GEMMs, panel by
    // panel; then all their inverses), each one launch over a range of jobs
    struct ViewStep { int32_t kind; int64_t j0; int32_t nj; size_t lds; double elems, flops; };
    std::vector<std::vector<ViewStep>> vsteps;
    std::vector<std::vector<int32_t>> vshared;   // per level: the dense views in its shared steps
    std::vector<ViewJob> vjobs;
    ViewJob* d_vjobs = nullptr;
    ViewDesc* d_vdesc = nullptr;
    std::vector<int32_t> dsn_ptr;           // per factor level into dsn
    std::vector<std::vector<int32_t>> dsn_l, dsn_u;   // per L-solve / U-solve level: dsn indices
    // per forward (0) / backward (1) solve level (offsets into the lists,
    // levels + 1 each): its supernodes of kLsolveSnMin..64 rows solved whole
    // by the four-wavefront kernel, those whose sums over their L region (U
    // columns past the block) are split over workgroups by rows (tasks: node,
    // first row), and whether it has a node for the per-row kernel
    struct SolveLists {
        std::vector<int32_t> sn_ptr, sp_ptr, task_ptr, sn_nodes, sp_nodes, tasks;
        std::vector<uint8_t> small;
        int32_t *d_sn = nullptr, *d_sp = nullptr, *d_tasks = nullptr;
    } sl[2];
    // the same for the transposed U^T (0) / L^T (1) solve levels: sn = the
    // nodes solved column by column, sp = those of kLsolveSnMin rows or more
    // (outside sums split by columns, then the block)
    SolveLists tl[2];
    // per forward (0) / backward (1) solve level with two or more large
    // supernodes (solve_split): their gathers in one launch (ext jobs [e0,
    // e1)) and their panel steps together, step k of every supernode that has
    // one in the k-th launch (job ranges)
    struct ViewSolve {
        int64_t e0 = 0, e1 = 0;
        std::vector<std::pair<int64_t, int64_t>> steps;
    };
    std::vector<ViewSolve> vsolve[2];
    std::vector<int32_t> vext_jobs;
    std::vector<SolveJob> vstep_jobs;
    int32_t* d_vext = nullptr;
    SolveJob* d_vstep = nullptr;
    // per solve graph (4: L, 1: U): for every level that starts a chain of
    // narrow levels solved in one launch, the end of the chain (else -1)
    std::vector<int32_t> chain_end[5];
    int32_t* d_lev_ptr[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    std::vector<int64_t> inv_off;           // per node: offset of its block inverse, or -1
    int64_t inv_total = 0;
    std::vector<int64_t> inv_ptr;           // per factor level into inv_nodes
    std::vector<int32_t> inv_nodes, inv_maxm;
    int64_t* d_inv_off = nullptr;
    // compact rows of the dense-tail nodes (see build_compact_rows) and the
    // relative maps with their sources' entries rewritten to list indices
    std::vector<int32_t> cw, cpos, crel;
    std::vector<int64_t> cpos_off;
    std::vector<uint8_t> snfuse;            // per node: its block LU done by its level's row launch
    int32_t* d_inv_nodes = nullptr;
    void* d_uinv = nullptr;
    static constexpr int kSide = 4;         // side streams for independent supernodes of a level
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *d_perm_r = nullptr, *d_perm_c = nullptr;
    double *d_dr = nullptr, *d_dc = nullptr;
    int64_t* d_arp = nullptr;
    int32_t* d_aci = nullptr;
    double* d_aval = nullptr;               // copy of the values of the last (re)factorisation
    int64_t* d_atp = nullptr;               // A^T as CSR: pointers, columns, value positions
    int32_t* d_atc = nullptr;
    int64_t* d_atq = nullptr;
    double* d_atv = nullptr;
    bool tlists = false;
    int32_t* d_pert = nullptr;              // [0] perturbed pivots, [1] a pipelined wait gave up
    int32_t* h_pert = nullptr;              // pinned copy of d_pert
    hipEvent_t fact_done = nullptr;
    int32_t last_pert = 0;
    bool pert_known = false;
    // solve workspace
    int32_t ws_nrhs = 0;
    SolveWs ws;                             // of hylu_solve (handle memory)
    double* h_norms_fixed = nullptr;        // pinned norms of hylu_solve_noalloc (kNoallocRhs right-hand sides)
    // batch of matrices on one handle (block diagonal); one member otherwise
    std::vector<int64_t> member_row_off{0}, member_nnz_off{0};
    int32_t* d_seg = nullptr;               // member of every row (null for one member)
    // graphs
    std::map<const double*, GraphEntry> refac_graphs;
    std::map<std::tuple<const double*, double*, int32_t, int64_t, int32_t>, GraphEntry> solve_graphs;
    // last solve (or hylu_residual)
    int32_t ir_iters = 0;
    double berr = 0.0, resid1 = 0.0;
    // analysis: time of the symbolic step (host or GPU) and a hash of its result
    double sym_ms = 0.0, sym_kernel_ms = 0.0;
    uint64_t sym_hash = 0;
    bool berr_known = false;
    // measurement
    Profiler prof;
    std::vector<double> lvl_bytes, lvl_flops;   // per factor level: row-kernel value entries and flops
    std::vector<int32_t> pert_rows;              // standalone rows without sources: pivot check only
    int32_t* d_pert_rows = nullptr;
    // algorithmic traffic per factor level, as value entries (times the
    // factor precision's size) and index bytes, and flops: row kernel, row
    // tiles, block inverses
    std::vector<double> lvl_idx;
    std::vector<double> tile_bytes, tile_idx, tile_flops;
    std::vector<double> inv_bytes, inv_flops;
    std::vector<double> chain_snlu_bytes, chain_snlu_flops;  // per chain launch: its block LUs (value entries)
    // one right-hand side: exact factor entries consumed by the L solve and
    // the U solve of the rows before the dense tail and by the tail's rows
    // (both solves), each with the count of those in standalone rows
    std::array<double, 6> solve_units{};
};

static const char* kClassNames[] = {"rows", "snlu", "tail_panel", "tail_trsm", "tail_gemm", "lsolve", "usolve",
                                    "tail_solve", "scatter", "other_solve", "sup_tile", "sn_inverse", "tail_dinv",
                                    "pipelined"};
enum { C_ROWS, C_SNLU, C_PANEL, C_TRSM, C_GEMM, C_LSOLVE, C_USOLVE, C_TSOLVE, C_SCATTER, C_OSOLVE, C_TILE, C_SNINV,
       C_DINV, C_PIPE, C_N };

namespace {

// HYLU_LOG=1 prints the duration of each preprocessing step to stderr
struct PhaseLog {
    bool on = std::getenv("HYLU_LOG") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void operator()(const char* what) {
        auto now = std::chrono::steady_clock::now();
        if (on) std::fprintf(stderr, "hylu: %-10s %8.3f s\n", what, std::chrono::duration<double>(now - t).count());
        t = now;
    }
};

#define HIPCHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) {                        \
        std::fprintf(stderr, "hylu: %s (line %d)\n", hipGetErrorString(e_), __LINE__);     \
        h->sticky_error = true; return HYLU_ERR_DEVICE; } } while (0)

// launch `x` and, when profiling, bracket it with events attributed to class `c`
#define LAUNCH(c, by, fl, x) do {                                                          \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;                                            \
        if (h->prof.on) { ea_ = h->prof.ev(); eb_ = h->prof.ev(); HIPCHK(hipEventRecord(ea_, st)); } \
        HIPCHK(x);                                                                          \
        if (h->prof.on) { HIPCHK(hipEventRecord(eb_, st)); h->prof.recs.push_back({(c), ea_, eb_, (double)(by), (double)(fl)}); } \
    } while (0)

void* dalloc(hylu_handle h, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    if (h->has_alloc) {
        p = h->alloc.alloc(h->alloc.ctx, bytes, nullptr);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) h->blocks.push_back(p);
    return p;
}

void free_device(hylu_handle h)
{
    for (auto& kv : h->refac_graphs) { hipGraphExecDestroy(kv.second.exec); hipGraphDestroy(kv.second.graph); }
    for (auto& kv : h->solve_graphs) { hipGraphExecDestroy(kv.second.exec); hipGraphDestroy(kv.second.graph); }
    h->refac_graphs.clear();
    h->solve_graphs.clear();
    if (!h->blocks.empty()) hipDeviceSynchronize();
    for (void* p : h->blocks) {
        if (h->has_alloc) h->alloc.free(h->alloc.ctx, p, nullptr);
        else hipFree(p);
    }
    h->blocks.clear();
    h->vals = nullptr;
    h->ws_nrhs = 0;
    h->tlists = false;
    h->uploaded = false;
}

template <typename T>
hylu_status upload(hylu_handle h, T*& dst, const std::vector<T>& src)
{
    dst = (T*)dalloc(h, sizeof(T) * std::max<size_t>(src.size(), 1));
    if (!dst) return HYLU_ERR_OOM;
    if (!src.empty()) {
        hipError_t e = hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            std::fprintf(stderr, "hylu: upload of %zu bytes: %s\n", sizeof(T) * src.size(), hipGetErrorString(e));
            return HYLU_ERR_DEVICE;
        }
    }
    return HYLU_OK;
}

#define UP(dst, src) do { hylu_status s_ = upload(h, dst, src); if (s_ != HYLU_OK) return s_; } while (0)

hylu_status validate_csr(int32_t n, const int64_t* rp, const int32_t* ci, const double* v)
{
    if (rp[0] != 0) return HYLU_ERR_CSR;
    for (int32_t i = 0; i < n; i++) {
        if (rp[i + 1] < rp[i]) return HYLU_ERR_CSR;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < 0 || ci[p] >= n) return HYLU_ERR_CSR;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return HYLU_ERR_CSR;
            if (!std::isfinite(v[p])) return HYLU_ERR_NONFINITE;
        }
    }
    return HYLU_OK;
}

// symmetric adjacency of the pattern of M + M^T without the diagonal
void symmetrize(int32_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                std::vector<int64_t>& xadj, std::vector<int32_t>& adj)
{
    std::vector<int64_t> cnt(n + 1, 0);
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) { cnt[i + 1]++; cnt[ci[p] + 1]++; }
    for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    std::vector<int32_t> tmp(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) { tmp[fill[i]++] = ci[p]; tmp[fill[ci[p]]++] = i; }
    xadj.assign(n + 1, 0);
    adj.clear();
    adj.reserve(tmp.size());
    for (int32_t i = 0; i < n; i++) {
        std::sort(tmp.begin() + cnt[i], tmp.begin() + cnt[i + 1]);
        int32_t last = -1;
        for (int64_t p = cnt[i]; p < cnt[i + 1]; p++)
            if (tmp[p] != last) { adj.push_back(tmp[p]); last = tmp[p]; }
        xadj[i + 1] = (int64_t)adj.size();
    }
}

hylu_status ensure_workspace(hylu_handle h, int32_t nrhs)
{
    if (h->ws_nrhs >= nrhs) return HYLU_OK;
    // captured solves refer to the old workspace
    for (auto& kv : h->solve_graphs) { hipGraphExecDestroy(kv.second.exec); hipGraphDestroy(kv.second.graph); }
    h->solve_graphs.clear();
    size_t es = h->fp32 ? sizeof(float) : sizeof(double);
    size_t nn = (size_t)h->n * nrhs;
    SolveWs& w = h->ws;
    w.y = dalloc(h, es * nn);
    w.z = dalloc(h, es * nn);
    w.r = (double*)dalloc(h, sizeof(double) * nn);
    w.bc = (double*)dalloc(h, sizeof(double) * nn);
    w.xbest = (double*)dalloc(h, sizeof(double) * nn);
    const size_t nseg = h->member_row_off.size() - 1;
    w.norms = (double*)dalloc(h, sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * nseg);
    if (!w.y || !w.z || !w.r || !w.bc || !w.xbest || !w.norms) return HYLU_ERR_OOM;
    if (w.h_norms) hipHostFree(w.h_norms);
    w.h_norms = nullptr;
    if (hipHostMalloc((void**)&w.h_norms, sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * nseg) != hipSuccess)
        return HYLU_ERR_OOM;
    h->ws_nrhs = nrhs;
    return HYLU_OK;
}

// scratch bytes hylu_solve_noalloc carves for nrhs right-hand sides (each
// vector rounded up to 256 bytes): the work vectors of SolveWs
size_t noalloc_bytes(hylu_handle h, int32_t nrhs)
{
    auto r = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t es = h->fp32 ? sizeof(float) : sizeof(double);
    const size_t nn = (size_t)h->n * nrhs;
    const size_t nseg = h->member_row_off.size() - 1;
    return 2 * r(es * nn) + 3 * r(sizeof(double) * nn) + r(sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * nseg);
}

// column lists of the T and L regions for the transposed solves (built on first use)
hylu_status ensure_tlists(hylu_handle h)
{
    if (h->tlists) return HYLU_OK;
    const Layout& L = h->lay;
    const int32_t n = h->n;
    std::vector<int64_t> uptr(n + 1, 0), lptr(n + 1, 0);
    // entries of the dense tail are handled by the tail kernels
    auto lend = [&](int32_t v) { return v >= L.tail_node0 ? L.lext[v] : L.lw[v]; };
    auto ubeg = [&](int32_t v) { return v >= L.tail_node0 ? L.W[v] : L.lw[v] + L.m[v]; };
    for (int32_t v = 0; v < L.nnodes; v++) {
        const int32_t* c = L.cols.data() + L.coff[v];
        for (int32_t t = 0; t < lend(v); t++) lptr[c[t] + 1] += L.m[v];
        for (int32_t t = ubeg(v); t < L.W[v]; t++) uptr[c[t] + 1] += L.m[v];
    }
    for (int32_t i = 0; i < n; i++) { uptr[i + 1] += uptr[i]; lptr[i + 1] += lptr[i]; }
    std::vector<int64_t> uslot(uptr[n]), lslot(lptr[n]);
    std::vector<int32_t> urow(uptr[n]), lrow(lptr[n]);
    std::vector<int64_t> uf(uptr.begin(), uptr.end() - 1), lf(lptr.begin(), lptr.end() - 1);
    for (int32_t v = 0; v < L.nnodes; v++) {
        const int32_t* c = L.cols.data() + L.coff[v];
        for (int32_t b = 0; b < L.m[v]; b++) {
            int64_t base = L.voff[v] + (int64_t)b * L.W[v];
            for (int32_t t = 0; t < lend(v); t++) { int64_t q = lf[c[t]]++; lslot[q] = base + t; lrow[q] = L.r0[v] + b; }
            for (int32_t t = ubeg(v); t < L.W[v]; t++) { int64_t q = uf[c[t]]++; uslot[q] = base + t; urow[q] = L.r0[v] + b; }
        }
    }
    int64_t* p1; int64_t* p2; int32_t* p3; int64_t* p4; int64_t* p5; int32_t* p6;
    UP(p1, uptr); UP(p2, uslot); UP(p3, urow); UP(p4, lptr); UP(p5, lslot); UP(p6, lrow);
    h->D.ut_ptr = p1; h->D.ut_slot = p2; h->D.ut_row = p3;
    h->D.lt_ptr = p4; h->D.lt_slot = p5; h->D.lt_row = p6;
    // A^T for the transposed residual
    const Csr& A = h->A;
    std::vector<int64_t> tp(n + 1, 0), tq(A.nnz());
    std::vector<int32_t> tc(A.nnz());
    for (int64_t p = 0; p < A.nnz(); p++) tp[A.ci[p] + 1]++;
    for (int32_t j = 0; j < n; j++) tp[j + 1] += tp[j];
    std::vector<int64_t> f(tp.begin(), tp.end() - 1);
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++) { int64_t q = f[A.ci[p]]++; tc[q] = i; tq[q] = p; }
    UP(h->d_atp, tp); UP(h->d_atc, tc); UP(h->d_atq, tq);
    h->d_atv = (double*)dalloc(h, sizeof(double) * std::max<int64_t>(A.nnz(), 1));
    if (!h->d_atv) return HYLU_ERR_OOM;
    h->tlists = true;
    return HYLU_OK;
}

// blocked right-looking LU of a dense view, one row panel at a time; panels
// go in groups while at least group_min_rows rows remain below them (option,
// default kGroupMinRows), and a block-sparse tail of at least group_tail_rows
// rows (default kGroupTailRows) still takes panel groups
constexpr int32_t kGroupMinRows = 2048;
constexpr int32_t kGroupTailRows = 16384;
// a factor level of fewer rows than this counts as narrow: deferred rows may
// join its launch on the CUs it leaves idle
constexpr int32_t kSideNarrowRows = 256;
// row accumulators in LDS: up to this width by default, wider in narrow levels
constexpr int32_t kRowCapSmall = 4096, kRowCapBig = 10240;
// supernodes of at least this many rows (and at most 64) take the
// four-wavefront forward-solve kernel
constexpr int32_t kLsolveSnMin = 8;
// a run of at least kChainMin solve levels of at most kChainNodes nodes is
// solved by one workgroup in one launch (one wavefront per node), if no node
// has more than kChainWork entries in its L (U) part; a supernode with more
// takes workgroups by groups of rows in the forward solve
constexpr int32_t kChainMin = 3, kChainNodes = 16;
constexpr int64_t kChainWork = 8192, kSplitWork = 8192;
// pipeline mode: nodes per chain launch (one LDS flag each), staging values
// per wavefront (at least the largest supernode with a block inverse), polls
// before a wait gives up (tens of milliseconds, far beyond any real wait), and
// the largest supernode a chain wavefront factors
constexpr int32_t kChainTasksMax = 1024;
constexpr int32_t kChainSw = kInvMax;
constexpr int32_t kChainSpin = 1 << 21;
constexpr int32_t kChainSnMax = 64;
constexpr int32_t kChainRunMin = 3;   // shortest run of narrow levels taken by chain launches
// a supernode of at most this many rows whose rows are row tasks of a narrow
// level has its block LU done by the last of those row tasks (the row
// launch's LDS holds its work)
constexpr int32_t kFuseSnMax = 64;
// The launch sequence of a view: groups of up to kGroup panels (left-looking
// inside the group, one trailing update per group).  With the tail's masks M
// every GEMM gets the list of its tiles that have a nonzero product, each with
// the group panels that contribute, in XCD order, and every TRSM the list of
// its blocks that hold entries (row blocks without multipliers only write
// zeros to lbuf); the rest is exactly zero and is skipped.
int32_t plan_dense(const std::vector<Layout::Panel>& panels, int32_t mT, int32_t nc, const TailMasks* M, bool group,
                   int32_t group_min_rows, std::vector<DenseOp>& ops, std::vector<uint32_t>& lists)
{
    ops.clear();
    int32_t ngroups = 0;          // groups of more than one panel
    const int32_t wd = M ? M->words : 0;
    auto bits = [&](const std::vector<uint64_t>& v, int32_t row, int32_t g0, int32_t nk) -> uint32_t {
        const uint64_t* w = v.data() + (size_t)row * wd;
        const int32_t q = g0 >> 6, o = g0 & 63;
        uint64_t x = w[q] >> o;
        if (o && q + 1 < wd) x |= w[q + 1] << (64 - o);
        return (uint32_t)(x & ((1ull << nk) - 1));
    };
    auto gemm = [&](int32_t g0, int32_t nk, const int32_t* kofs, int32_t kb0, int32_t rb, int32_t re, int32_t cg0,
                    int32_t mstep, int32_t gp0, int32_t gnp, int32_t w0, int32_t w1) {
        const int32_t K = kofs[nk];
        const int32_t rows = re - rb, cols = gnp > 0 ? gnp : nc - cg0;
        if (K <= 0 || rows <= 0 || cols <= 0) return;
        DenseOp o;
        o.kind = 2;
        const int32_t a[8] = {kb0, K, rb, re, cg0, mstep, gp0, gnp};
        std::copy(a, a + 8, o.a);
        for (int j = 0; j <= kGroup; j++) o.kb[j] = j <= nk ? kofs[j] : K;
        const int32_t gy = (rows + 63) / 64, gx = gnp > 0 ? 1 : (cols + 63) / 64;
        if (!M || gx > 4095 || gy > 65535) {
            o.elems = 2.0 * rows * cols + (double)K * (rows + cols);
            o.flops = 2.0 * K * rows * (double)cols;
            ops.push_back(o);
            return;
        }
        std::vector<uint32_t> rm(gy, 0), cm(gx, 0);
        for (int32_t r = rb; r < re; r++) rm[(r - rb) >> 6] |= bits(M->lbits, r, g0, nk);
        if (gnp > 0) {
            for (int32_t c = w0; c < w1; c++) cm[0] |= bits(M->ubits, c, g0, nk);
        } else {
            for (int32_t c = cg0; c < nc; c++) cm[(c - cg0) >> 6] |= bits(M->ubits, c, g0, nk);
        }
        std::vector<uint32_t> t;
        for (int32_t ty = 0; ty < gy; ty++)
            for (int32_t tx = 0; tx < gx; tx++) {
                const uint32_t m = rm[ty] & cm[tx];
                if (!m) continue;
                t.push_back(((uint32_t)ty << 16) | ((uint32_t)tx << 4) | m);
                double ka = 0;
                for (int j = 0; j < nk; j++)
                    if ((m >> j) & 1) ka += kofs[j + 1] - kofs[j];
                const double tr = std::min(64, rows - 64 * ty), tc = std::min(64, cols - 64 * tx);
                o.flops += 2.0 * tr * tc * ka;
                o.elems += 2.0 * tr * tc + ka * (tr + tc);
            }
        if (t.empty()) return;                     // every product is zero
        // XCD order: workgroup i runs on XCD i % 8; split the row-major tiles
        // into four bands of rows, each into two halves of columns, with equal
        // counts, and give each of the eight parts one XCD
        std::vector<uint32_t> out;
        if (t.size() >= 32) {
            const size_t n = t.size();
            std::vector<std::vector<uint32_t>> part(8);
            for (int b = 0; b < 4; b++) {
                std::vector<uint32_t> band(t.begin() + n * b / 4, t.begin() + n * (b + 1) / 4);
                std::stable_sort(band.begin(), band.end(), [](uint32_t x, uint32_t y) {
                    return ((x >> 4) & 0xFFF) < ((y >> 4) & 0xFFF);
                });
                const size_t h2 = band.size() / 2;
                part[2 * b].assign(band.begin(), band.begin() + h2);
                part[2 * b + 1].assign(band.begin() + h2, band.end());
            }
            size_t len = 0;
            for (auto& q : part) len = std::max(len, q.size());
            out.assign(8 * len, kTileNone);
            for (int c = 0; c < 8; c++)
                for (size_t i = 0; i < part[c].size(); i++) out[i * 8 + c] = part[c][i];
        } else {
            out = t;
        }
        o.list = (int64_t)lists.size();
        o.count = (int32_t)out.size();
        lists.insert(lists.end(), out.begin(), out.end());
        ops.push_back(o);
    };
    auto trsm = [&](int32_t j, const Layout::Panel& P, int32_t kb0, int32_t kof) {
        DenseOp o;
        o.kind = 1;
        const int32_t a[5] = {P.p0, P.p1, P.c1, kb0, kof};
        std::copy(a, a + 5, o.a);
        const double np = P.p1 - P.p0;
        const int32_t colsA = std::max(nc - P.c1, 0), rows = std::max(mT - P.p1, 0);
        const int32_t nA = (colsA + 63) / 64, nB = (rows + 63) / 64;
        if (!M) {
            o.elems = 2.0 * np * colsA + 3.0 * np * rows + np * np;
            o.flops = np * np * ((double)colsA + rows);
            ops.push_back(o);
            return;
        }
        std::vector<uint32_t> bl;
        double ca = 0, rr = 0;
        for (int32_t b = 0; b < nA; b++) {
            const int32_t c0 = P.c1 + 64 * b, c1 = std::min(nc, c0 + 64);
            bool any = false;
            for (int32_t c = c0; c < c1 && !any; c++) any = M->ubit(c, j);
            if (any) { bl.push_back((uint32_t)b); ca += c1 - c0; }
        }
        for (int32_t b = 0; b < nB; b++) {
            const int32_t r0 = P.p1 + 64 * b, r1 = std::min(mT, r0 + 64);
            bool any = false;
            for (int32_t r = r0; r < r1 && !any; r++) any = M->lbit(r, j);
            if (any) { bl.push_back((uint32_t)(nA + b)); rr += r1 - r0; }
            else bl.push_back((uint32_t)(nA + b) | (uint32_t)kTrsmZero);
        }
        o.elems = 2.0 * np * ca + 3.0 * np * rr + np * np + np * (rows - rr);
        o.flops = np * np * (ca + rr);
        o.list = (int64_t)lists.size();
        o.count = (int32_t)bl.size();
        lists.insert(lists.end(), bl.begin(), bl.end());
        ops.push_back(o);
    };
    for (size_t i = 0; i < panels.size();) {
        // grouping pays where the trailing matrix is large and mostly dense;
        // near the end, or where block sparsity leaves small per-panel
        // updates, its extra launches cost more than the saved passes
        const bool big = group && mT - panels[i].p1 >= group_min_rows;
        const size_t g1 = std::min(i + (size_t)(big ? kGroup : 1), panels.size());
        if (g1 - i > 1) ngroups++;
        const int32_t kb0 = panels[i].p0, cg = panels[i].cg0;
        int32_t kofs[kGroup + 1] = {0, 0, 0, 0, 0};
        for (size_t j = i; j < g1; j++) {
            const Layout::Panel& P = panels[j];
            const int32_t nk = (int32_t)(j - i);
            // this panel's rows, from the group so far
            gemm((int32_t)i, nk, kofs, kb0, P.p0, P.p1, cg, P.p0, 0, 0, 0, 0);
            DenseOp o;
            o.kind = 0;
            const int32_t a[4] = {P.p0, P.p1, P.c0, P.c1};
            std::copy(a, a + 4, o.a);
            o.elems = 2.0 * (P.p1 - P.p0) * (P.c1 - P.c0);
            o.flops = (double)(P.p1 - P.p0) * (P.p1 - P.p0) * (P.c1 - P.c0);
            ops.push_back(o);
            // the rows below at this panel's pivot columns, from the group so far
            gemm((int32_t)i, nk, kofs, kb0, P.p1, mT, 0, 0, P.p0, P.p1 - P.p0, P.c0, P.c1);
            trsm((int32_t)j, P, kb0, kofs[nk]);
            kofs[nk + 1] = kofs[nk] + (P.p1 - P.p0);
        }
        const Layout::Panel& Q = panels[g1 - 1];
        gemm((int32_t)i, (int32_t)(g1 - i), kofs, kb0, Q.p1, mT, cg, Q.p1, 0, 0, 0, 0);   // everything below the group
        i = g1;
    }
    return ngroups;
}

hylu_status enqueue_dense(hylu_handle h, const TailView& TV, const std::vector<DenseOp>& ops, const uint32_t* d_list,
                          bool search, hipStream_t st)
{
    const double es = h->fp32 ? 4.0 : 8.0;
    for (const DenseOp& o : ops) {
        const int32_t* a = o.a;
        if (o.kind == 0) {
            LAUNCH(C_PANEL, es * o.elems, o.flops,
                   launch_tail_panel(h->fp32, h->D, TV, h->vals, a[0], a[1], a[2], a[3], h->tau, h->d_pert, search ? 1 : 0, st));
        } else if (o.kind == 1) {
            const int32_t* bl = o.list >= 0 ? reinterpret_cast<const int32_t*>(d_list + o.list) : nullptr;
            LAUNCH(C_TRSM, es * o.elems, o.flops,
                   launch_tail_trsm(h->fp32, TV, h->vals, a[0], a[1], a[2], a[3], a[4], bl, o.count, st));
        } else {
            const uint32_t* tl = o.list >= 0 ? d_list + o.list : nullptr;
            LAUNCH(C_GEMM, es * o.elems, o.flops,
                   launch_tail_gemm(h->fp32, TV, h->vals, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], tl, o.count, o.kb, st));
        }
    }
    return HYLU_OK;
}

// the large supernodes of level l, spread over the side streams (forked from
// and joined back into st; under capture they become parallel graph branches)
// a large supernode's blocked LU, then the inverses of its solve panels'
// diagonal blocks (used by its forward and backward solve steps)
// Shared launches for the large supernodes of a level (Sec. 2.2: their internal
// factorisations are independent): views whose plan is the plain one-panel
// sequence (panel, TRSM, every-tile GEMM per 16-row panel) and whose panels
// fit the wide-window kernel with the window in LDS take step k of all of
// them in three launches; the same kernels on the same arguments, so the
// factors are those of the per-view launches.
void plan_shared_views(hylu_handle h)
{
    h->vsteps.assign(h->dsn_ptr.size() > 0 ? h->dsn_ptr.size() - 1 : 0, {});
    h->vshared.assign(h->vsteps.size(), {});
    h->vjobs.clear();
    const double es = h->fp32 ? 4.0 : 8.0;
    for (size_t l = 0; l < h->vsteps.size(); l++) {
        struct Step { const DenseOp* op[3]; };
        std::vector<int32_t> qs;
        std::vector<std::vector<Step>> steps;
        for (int32_t q = h->dsn_ptr[l]; q < h->dsn_ptr[l + 1]; q++) {
            const hylu_handle_s::DenseSn& d = h->dsn[q];
            const int32_t m = h->lay.m[d.v];
            std::vector<Step> st;
            bool ok = !d.ops.empty();
            for (size_t i = 0; ok && i < d.ops.size();) {
                const DenseOp& p = d.ops[i];
                if (p.kind != 0 || p.a[2] != 0 || p.a[3] != m || tail_panel_wide_lds(h->fp32, p.a[1] - p.a[0], m) == 0) {
                    ok = false;
                    break;
                }
                Step x{{&p, nullptr, nullptr}};
                i++;
                if (i < d.ops.size() && d.ops[i].kind == 1) {
                    const DenseOp& t = d.ops[i];
                    if (t.a[0] != p.a[0] || t.a[1] != p.a[1] || t.list >= 0) { ok = false; break; }
                    x.op[1] = &t;
                    i++;
                }
                if (i < d.ops.size() && d.ops[i].kind == 2) {
                    const DenseOp& g = d.ops[i];
                    if (g.a[0] != p.a[0] || g.a[1] != p.a[1] - p.a[0] || g.a[2] != p.a[1] || g.a[7] != 0 ||
                        g.list >= 0 || g.kb[1] != g.a[1]) { ok = false; break; }
                    x.op[2] = &g;
                    i++;
                }
                st.push_back(x);
            }
            if (!ok) continue;
            qs.push_back(q);
            steps.push_back(std::move(st));
        }
        if (qs.size() < 2) continue;
        h->vshared[l] = qs;
        size_t nk = 0;
        for (const auto& st : steps) nk = std::max(nk, st.size());
        auto begin = [&](int32_t kind) {
            hylu_handle_s::ViewStep vs{kind, (int64_t)h->vjobs.size(), 0, 0, 0.0, 0.0};
            return vs;
        };
        auto finish = [&](hylu_handle_s::ViewStep& vs) {
            vs.nj = (int32_t)((int64_t)h->vjobs.size() - vs.j0);
            if (vs.nj > 0) h->vsteps[l].push_back(vs);
        };
        for (size_t k = 0; k < nk; k++) {
            for (int kind = 0; kind < 3; kind++) {
                hylu_handle_s::ViewStep vs = begin(kind);
                for (size_t w = 0; w < qs.size(); w++) {
                    if (k >= steps[w].size() || !steps[w][k].op[kind]) continue;
                    const DenseOp& o = *steps[w][k].op[kind];
                    const hylu_handle_s::DenseSn& d = h->dsn[qs[w]];
                    const int32_t m = h->lay.m[d.v], nc = h->lay.W[d.v] - h->lay.lw[d.v];
                    vs.elems += es * o.elems;
                    vs.flops += o.flops;
                    ViewJob j{};
                    j.v = qs[w];
                    if (kind == 0) {
                        const int32_t a[6] = {o.a[0], o.a[1], o.a[2], o.a[3], 0, 0};
                        std::copy(a, a + 6, j.a);
                        vs.lds = std::max(vs.lds, tail_panel_wide_lds(h->fp32, o.a[1] - o.a[0], m));
                        h->vjobs.push_back(j);
                    } else if (kind == 1) {
                        const int32_t nA = (std::max(nc - o.a[2], 0) + 63) / 64, nB = (std::max(m - o.a[1], 0) + 63) / 64;
                        const int32_t a[6] = {o.a[0], o.a[1], o.a[2], nA, o.a[3], o.a[4]};
                        std::copy(a, a + 6, j.a);
                        for (int32_t b = 0; b < nA + nB; b++) { j.blk = b; h->vjobs.push_back(j); }
                    } else {
                        const int32_t rb = o.a[2], re = o.a[3], cg0 = o.a[4];
                        const int32_t gy = (re - rb + 63) / 64, gx = (nc - cg0 + 63) / 64;
                        const int32_t a[6] = {o.a[0], o.a[1], rb, re, cg0, o.a[5]};
                        std::copy(a, a + 6, j.a);
                        for (int32_t ty = 0; ty < gy; ty++)
                            for (int32_t tx = 0; tx < gx; tx++) { j.blk = (ty << 16) | tx; h->vjobs.push_back(j); }
                    }
                }
                finish(vs);
            }
        }
        hylu_handle_s::ViewStep vs = begin(3);
        for (int32_t q : qs) {
            const int32_t ns = (int32_t)h->dsn[q].spanels.size();
            vs.elems += es * ns * 3.0 * kNB * kNB;
            vs.flops += ns * 2.0 * kNB * kNB * kNB / 3.0;
            for (int32_t b = 0; b < 2 * ns; b++) {
                ViewJob j{};
                j.v = q;
                j.blk = b;
                h->vjobs.push_back(j);
            }
        }
        finish(vs);
    }
    if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2) {
        size_t nv = 0, ns = 0, nops = 0;
        for (size_t l = 0; l < h->vsteps.size(); l++) {
            nv += h->vshared[l].size();
            ns += h->vsteps[l].size();
            for (int32_t q : h->vshared[l]) nops += h->dsn[q].ops.size() + 1;
        }
        std::fprintf(stderr, "hylu: shared dense-view steps: %zu views, %zu launches for their %zu, %zu jobs\n", nv, ns,
                     nops, h->vjobs.size());
    }
}

hylu_status enqueue_dsn(hylu_handle h, const hylu_handle_s::DenseSn& q, bool search, hipStream_t st)
{
    if (search) HIPCHK(launch_tail_init(q.TV, st));
    hylu_status s = enqueue_dense(h, q.TV, q.ops, nullptr, search, st);
    if (s != HYLU_OK) return s;
    const double ns = (double)q.spanels.size();
    LAUNCH(C_DINV, (h->fp32 ? 4.0 : 8.0) * ns * 3.0 * kNB * kNB, ns * 2.0 * kNB * kNB * kNB / 3.0,
           launch_tail_dinv(h->fp32, q.TV, h->vals, q.d_sp, (int32_t)q.spanels.size(), q.d_inv, st));
    return HYLU_OK;
}

hylu_status enqueue_level_dense(hylu_handle h, int32_t l, bool search, hipStream_t st)
{
    const int32_t d0 = h->dsn_ptr[l], d1 = h->dsn_ptr[l + 1];
    if (d1 == d0) return HYLU_OK;
    // the views of the level's shared steps first, on st
    std::vector<char> shared(d1 - d0, 0);
    if ((size_t)l < h->vshared.size() && !h->vshared[l].empty()) {
        for (int32_t q : h->vshared[l]) {
            shared[q - d0] = 1;
            if (search) HIPCHK(launch_tail_init(h->dsn[q].TV, st));
        }
        for (const hylu_handle_s::ViewStep& vs : h->vsteps[l]) {
            const ViewJob* jb = h->d_vjobs + vs.j0;
            if (vs.kind == 0)
                LAUNCH(C_PANEL, vs.elems, vs.flops,
                       launch_tail_panel_views(h->fp32, h->D, h->d_vdesc, h->vals, jb, vs.nj, vs.lds, h->tau, h->d_pert,
                                               search ? 1 : 0, st));
            else if (vs.kind == 1)
                LAUNCH(C_TRSM, vs.elems, vs.flops, launch_tail_trsm_views(h->fp32, h->d_vdesc, h->vals, jb, vs.nj, st));
            else if (vs.kind == 2)
                LAUNCH(C_GEMM, vs.elems, vs.flops, launch_tail_gemm_views(h->fp32, h->d_vdesc, h->vals, jb, vs.nj, st));
            else
                LAUNCH(C_DINV, vs.elems, vs.flops, launch_tail_dinv_views(h->fp32, h->d_vdesc, h->vals, jb, vs.nj, st));
        }
    }
    int32_t rest = 0;
    for (int32_t q = d0; q < d1; q++) rest += !shared[q - d0];
    if (rest == 0) return HYLU_OK;
    if (h->prof.on || rest == 1) {             // one supernode, or measuring: stay on st
        for (int32_t q = d0; q < d1; q++) {
            if (shared[q - d0]) continue;
            hylu_status s = enqueue_dsn(h, h->dsn[q], search, st);
            if (s != HYLU_OK) return s;
        }
        return HYLU_OK;
    }
    const int k = std::min<int>(hylu_handle_s::kSide, rest);
    HIPCHK(hipEventRecord(h->ev_fork, st));
    for (int j = 0; j < k; j++) HIPCHK(hipStreamWaitEvent(h->side[j], h->ev_fork, 0));
    // largest first, each to the least loaded stream
    std::vector<double> load(k, 0.0);
    for (int32_t q = d0; q < d1; q++) {
        if (shared[q - d0]) continue;
        int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        const TailView& TV = h->dsn[q].TV;
        load[j] += (double)TV.mT * TV.mT * TV.nc;
        hylu_status s = enqueue_dsn(h, h->dsn[q], search, h->side[j]);
        if (s != HYLU_OK) return s;
    }
    for (int j = 0; j < k; j++) {
        HIPCHK(hipEventRecord(h->ev_join[j], h->side[j]));
        HIPCHK(hipStreamWaitEvent(st, h->ev_join[j], 0));
    }
    return HYLU_OK;
}

// the level loop of the numerical factorisation
hylu_status enqueue_factor(hylu_handle h, const double* d_val, bool search, hipStream_t st)
{
    const double es = h->fp32 ? 4.0 : 8.0;
    HIPCHK(launch_zero(h->d_pert, 2 * sizeof(int32_t), st));
    LAUNCH(C_SCATTER, es * h->lay.nvals, 0, launch_zero(h->vals, h->lay.nvals * (h->fp32 ? 4 : 8), st));
    LAUNCH(C_SCATTER, 40.0 * h->nnz, 2.0 * h->nnz,
           launch_scatter(h->fp32, d_val, h->d_amap, h->d_asr, h->d_asc, h->nnz, h->vals, h->d_aval, st));
    if (search) HIPCHK(launch_tail_init(h->TV, st));
    if (!h->pert_rows.empty())
        LAUNCH(C_SCATTER, 2.0 * es * h->pert_rows.size(), 0.0,
               launch_perturb_rows(h->fp32, h->D, h->vals, h->d_pert_rows, (int32_t)h->pert_rows.size(), h->tau,
                                   h->d_pert, st));
    const LevelTasks& T = h->ft;
    int32_t nl = (int32_t)T.maxW.size();
    for (int32_t l = 0; l < nl; l++) {
        if (!T.chain_lev.empty() && T.chain_lev[l]) {
            // pipeline mode over the run of narrow levels from l: its chain launches
            if (T.chain_start[l] < 0) return HYLU_ERR_INTERNAL;
            size_t c = (size_t)T.chain_start[l];
            int32_t lend = l;
            for (; c < T.chains.size() && T.chains[c].l0 == lend; c++) {
                const LevelTasks::Chain& ch = T.chains[c];
                lend = ch.l1;
                double by = h->chain_snlu_bytes[c] * es, fl = h->chain_snlu_flops[c];
                for (int32_t q = ch.l0; q < ch.l1; q++) { by += h->lvl_bytes[q] * es + h->lvl_idx[q]; fl += h->lvl_flops[q]; }
                LAUNCH(C_PIPE, by, fl,
                       launch_factor_chain(h->fp32, h->D, h->vals, h->d_ctask + ch.t0, h->d_csthr + ch.t0,
                                           (int32_t)(ch.t1 - ch.t0), ch.nw, ch.cap, kChainSw, h->tau, h->d_pert,
                                           search ? 1 : 0, h->d_inv_off,
                                           h->opt.pipeline_spin > 0 ? h->opt.pipeline_spin : kChainSpin, st));
            }
            l = lend - 1;
            continue;
        }
        int64_t r0 = T.row_ptr[l], r1 = T.row_ptr[l + 1];
        LAUNCH(C_ROWS, h->lvl_bytes[l] * es + h->lvl_idx[l], h->lvl_flops[l],
               launch_factor_rows(h->fp32, h->D, h->vals, h->d_rows + r0, h->d_rrange + 2 * r0, (int32_t)(r1 - r0),
                                  T.maxW[l], h->tau, h->d_pert,
                                  T.tune_rows ? T.tune_rows : T.row_nt[l], T.row_stage[l], T.row_cap[l],
                                  search ? 1 : 0, h->d_inv_off, st));
        if (T.tile_ptr[l + 1] > T.tile_ptr[l])
            LAUNCH(C_TILE, h->tile_bytes[l] * es + h->tile_idx[l], h->tile_flops[l],
                   launch_factor_tile(h->fp32, h->D, h->vals, h->d_tiles + 2 * T.tile_ptr[l],
                                      (int32_t)(T.tile_ptr[l + 1] - T.tile_ptr[l]), st));
        int64_t s0 = T.sn_ptr[l], s1 = T.sn_ptr[l + 1];
        if (s1 > s0) {
            double by = 0, fl = 0;
            for (int64_t q = s0; q < s1; q++) {
                int32_t v = T.snodes[q];
                double m = h->lay.m[v], wc = h->lay.W[v] - h->lay.lw[v];
                by += 2.0 * es * m * wc;
                fl += 2.0 * m * m * m / 3.0 + m * m * (wc - m);
                if (h->inv_off[v] >= 0) { by += 2.0 * es * m * m; fl += m * m * m / 3.0; }   // its block inverse
            }
            LAUNCH(C_SNLU, by, fl, launch_factor_snlu(h->fp32, h->D, h->vals, h->d_snodes + s0, (int32_t)(s1 - s0), T.maxm[l],
                                                      h->tau, h->d_pert, search ? 1 : 0,
                                                      T.tune_sn ? T.tune_sn : T.sn_nt[l], h->d_inv_off, st));
        }
        hylu_status sd = enqueue_level_dense(h, l, search, st);
        if (sd != HYLU_OK) return sd;
        if (h->inv_ptr[l + 1] > h->inv_ptr[l])
            LAUNCH(C_SNINV, h->inv_bytes[l] * es, h->inv_flops[l],
                   launch_sn_inverse(h->fp32, h->D, h->vals, h->d_inv_nodes + h->inv_ptr[l],
                                     (int32_t)(h->inv_ptr[l + 1] - h->inv_ptr[l]), h->inv_maxm[l], h->d_inv_off,
                                     h->d_uinv, st));
    }
    // dense tail: blocked right-looking LU, one row panel at a time, then the
    // inverses of the solve panels' diagonal blocks
    hylu_status sd = enqueue_dense(h, h->TV, h->tail_ops, h->d_tail_list, search, st);
    if (sd != HYLU_OK || h->lay.mT == 0) return sd;
    const double ns = (double)h->lay.spanels.size();
    LAUNCH(C_DINV, es * ns * 3.0 * kNB * kNB, ns * 2.0 * kNB * kNB * kNB / 3.0,
           launch_tail_dinv(h->fp32, h->TV, h->vals, h->d_tsp, (int32_t)h->lay.spanels.size(), h->d_tinv, st));
    return HYLU_OK;
}

// base solve in the factor precision: x = A^{-1} b (transpose 0) or A^{-T} b
hylu_status enqueue_solve(hylu_handle h, const SolveWs& w, const double* b, int64_t ldb, double* x, int64_t ldx, int32_t nrhs,
                          int32_t transpose, int32_t accumulate, hipStream_t st)
{
    const Layout& L = h->lay;
    const int32_t n = h->n;
    const bool f = h->fp32;
    // level launches of solve graph g; after each level, its large supernodes
    // (forward and backward solves) through the dense-view kernels
    auto levels = [&](int g, auto&& fn) -> hylu_status {
        for (size_t l = 0; l + 1 < L.xlev_ptr[g].size(); l++) {
            int32_t a = L.xlev_ptr[g][l], c = L.xlev_ptr[g][l + 1] - a;
            int cls = g == 4 ? C_LSOLVE : g == 1 ? C_USOLVE : C_OSOLVE;
            if ((g == 4 || g == 1) && l < h->chain_end[g].size() && h->chain_end[g][l] > (int32_t)l) {
                // a chain of narrow levels in one launch
                const int32_t e = h->chain_end[g][l];
                if (g == 4)
                    LAUNCH(cls, 0, 0, launch_lsolve_chain(f, h->D, h->vals, h->d_lev_ptr[4], h->d_lev[4], (int32_t)l, e,
                                                          w.y, nrhs, st));
                else
                    LAUNCH(cls, 0, 0, launch_usolve_chain(f, h->D, h->vals, h->d_lev_ptr[1], h->d_lev[1], (int32_t)l, e,
                                                          w.y, w.z, nrhs, st));
                l = e - 1;
                continue;
            }
            if (c > 0) LAUNCH(cls, 0, 0, fn(h->d_lev[g] + a, c, l));
            const std::vector<std::vector<int32_t>>* dl = g == 4 ? &h->dsn_l : g == 1 ? &h->dsn_u : nullptr;
            if (!dl || l >= dl->size()) continue;
            const std::vector<hylu_handle_s::ViewSolve>& VS = h->vsolve[g == 4 ? 0 : 1];
            if (l < VS.size() && !VS[l].steps.empty()) {
                // the level's large supernodes together: gathers, then each step
                const hylu_handle_s::ViewSolve& V = VS[l];
                LAUNCH(cls, 0, 0, launch_sn_ext_views(f, h->D, h->vals, h->d_vext + 2 * V.e0, (int32_t)(V.e1 - V.e0), w.y,
                                                      g == 4 ? nullptr : w.z, nrhs, g == 4 ? 0 : 1, st));
                for (const auto& J : V.steps)
                    LAUNCH(cls, 0, 0, launch_view_steps(f, h->d_vdesc, h->d_vstep + J.first, (int32_t)(J.second - J.first),
                                                        h->vals, n, w.y, g == 4 ? w.y : w.z, nrhs, g == 4 ? 0 : 1, st));
                continue;
            }
            for (int32_t q : (*dl)[l]) {
                const hylu_handle_s::DenseSn& d = h->dsn[q];
                // one launch per solve panel with the diagonal blocks' inverses
                const std::vector<Layout::Panel>& SP = d.spanels;
                const int32_t ns = (int32_t)SP.size();
                const size_t esz = f ? 4 : 8;
                auto inv = [&](int32_t k, int kind) {
                    return (const void*)((const char*)d.d_inv + ((size_t)2 * k + kind) * kNB * kNB * esz);
                };
                if (g == 4) {
                    LAUNCH(cls, 0, 0, launch_sn_lext(f, h->D, d.TV, h->vals, d.v, w.y, nrhs, st));
                    LAUNCH(cls, 0, 0, launch_tail_step(f, d.TV, h->vals, 0, 0, SP[0].p0, SP[0].p1, inv(0, 0), n, w.y,
                                                       w.y, nrhs, 0, st));
                    for (int32_t k = 0; k + 1 < ns; k++)
                        LAUNCH(cls, 0, 0, launch_tail_step(f, d.TV, h->vals, SP[k].p0, SP[k].p1, SP[k + 1].p0,
                                                           SP[k + 1].p1, inv(k + 1, 0), n, w.y, w.y, nrhs, 0, st));
                } else {
                    LAUNCH(cls, 0, 0, launch_sn_utext(f, h->D, d.TV, h->vals, d.v, w.y, w.z, nrhs, st));
                    LAUNCH(cls, 0, 0, launch_tail_step(f, d.TV, h->vals, 0, 0, SP[ns - 1].p0, SP[ns - 1].p1,
                                                       inv(ns - 1, 1), n, w.y, w.z, nrhs, 1, st));
                    for (int32_t k = ns - 1; k > 0; k--)
                        LAUNCH(cls, 0, 0, launch_tail_step(f, d.TV, h->vals, SP[k].p0, SP[k].p1, SP[k - 1].p0,
                                                           SP[k - 1].p1, inv(k - 1, 1), n, w.y, w.z, nrhs, 1, st));
                }
            }
        }
        return HYLU_OK;
    };
    hylu_status s;
    if (!transpose) {
        HIPCHK(launch_permute_in(f, n, nrhs, h->d_perm_r, h->d_dr, b, ldb, w.y, st));
        s = levels(4, [&](const int32_t* nodes, int32_t c, size_t l) {
            const hylu_handle_s::SolveLists& S = h->sl[0];
            const int32_t s0 = S.sn_ptr[l], p0 = S.sp_ptr[l], k0 = S.task_ptr[l];
            return launch_lsolve(f, h->D, h->vals, nodes, S.small[l] ? c : 0, S.d_sn + s0, S.sn_ptr[l + 1] - s0,
                                 S.d_sp + p0, S.sp_ptr[l + 1] - p0, S.d_tasks + 2 * (int64_t)k0,
                                 S.task_ptr[l + 1] - k0, w.y, nrhs, kLsolveSnMin, st);
        });
        if (s != HYLU_OK) return s;
        if (L.mT > 0) {
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_lext(f, h->D, h->vals, L.tail_node0, L.t0, w.y, nrhs, st));
            // one launch per solve panel: its contribution to the rows after it
            // and the next panel's diagonal solve (with the block inverses)
            const std::vector<Layout::Panel>& SP = L.spanels;
            const int32_t ns = (int32_t)SP.size();
            const size_t es = f ? 4 : 8;
            auto inv = [&](int32_t k, int kind) {
                return (const void*)((const char*)h->d_tinv + ((size_t)2 * k + kind) * kNB * kNB * es);
            };
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, 0, 0, SP[0].p0, SP[0].p1, inv(0, 0), n, w.y,
                                                    w.y, nrhs, 0, st));
            for (int32_t k = 0; k + 1 < ns; k++)
                LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, SP[k].p0, SP[k].p1, SP[k + 1].p0, SP[k + 1].p1,
                                                        inv(k + 1, 0), n, w.y, w.y, nrhs, 0, st));
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, 0, 0, SP[ns - 1].p0, SP[ns - 1].p1, inv(ns - 1, 1), n,
                                                    w.y, w.z, nrhs, 1, st));
            for (int32_t k = ns - 1; k > 0; k--)
                LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, SP[k].p0, SP[k].p1, SP[k - 1].p0, SP[k - 1].p1,
                                                        inv(k - 1, 1), n, w.y, w.z, nrhs, 1, st));
        }
        s = levels(1, [&](const int32_t* nodes, int32_t c, size_t l) {
            const hylu_handle_s::SolveLists& S = h->sl[1];
            const int32_t s0 = S.sn_ptr[l], p0 = S.sp_ptr[l], k0 = S.task_ptr[l];
            return launch_usolve(f, h->D, h->vals, nodes, S.small[l] ? c : 0, S.d_sn + s0, S.sn_ptr[l + 1] - s0,
                                 S.d_sp + p0, S.sp_ptr[l + 1] - p0, S.d_tasks + 2 * (int64_t)k0,
                                 S.task_ptr[l + 1] - k0, w.y, w.z, nrhs, kLsolveSnMin, st);
        });
        if (s != HYLU_OK) return s;
        HIPCHK(launch_permute_out(f, n, nrhs, h->d_perm_c, h->d_dc, w.z, x, ldx, accumulate, st));
    } else {
        HIPCHK(launch_permute_in(f, n, nrhs, h->d_perm_c, h->d_dc, b, ldb, w.y, st));
        s = levels(2, [&](const int32_t*, int32_t, size_t l) {
            const hylu_handle_s::SolveLists& S = h->tl[0];
            const int32_t s0 = S.sn_ptr[l], p0 = S.sp_ptr[l], k0 = S.task_ptr[l];
            return launch_utsolve(f, h->D, h->vals, S.d_sn + s0, S.sn_ptr[l + 1] - s0, S.d_sp + p0,
                                  S.sp_ptr[l + 1] - p0, S.d_tasks + 2 * (int64_t)k0, S.task_ptr[l + 1] - k0, w.y, w.z,
                                  nrhs, st);
        });
        if (s != HYLU_OK) return s;
        if (L.mT > 0) {
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_utext(f, h->D, h->TV, h->vals, w.y, w.z, nrhs, st));
            // U^T ascending, then L^T descending: one launch per solve panel
            // with the transposed inverses of the diagonal blocks
            const std::vector<Layout::Panel>& SP = L.spanels;
            const int32_t ns = (int32_t)SP.size();
            const size_t esz = f ? 4 : 8;
            auto inv = [&](int32_t k, int kind) {
                return (const void*)((const char*)h->d_tinv + ((size_t)2 * k + kind) * kNB * kNB * esz);
            };
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, 0, 0, SP[0].p0, SP[0].p1, inv(0, 1), n, w.y,
                                                    w.z, nrhs, 2, st));
            for (int32_t k = 0; k + 1 < ns; k++)
                LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, SP[k].p0, SP[k].p1, SP[k + 1].p0, SP[k + 1].p1,
                                                        inv(k + 1, 1), n, w.y, w.z, nrhs, 2, st));
            LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, 0, 0, SP[ns - 1].p0, SP[ns - 1].p1, inv(ns - 1, 0), n,
                                                    w.z, w.z, nrhs, 3, st));
            for (int32_t k = ns - 1; k > 0; k--)
                LAUNCH(C_TSOLVE, 0, 0, launch_tail_step(f, h->TV, h->vals, SP[k].p0, SP[k].p1, SP[k - 1].p0, SP[k - 1].p1,
                                                        inv(k - 1, 0), n, w.z, w.z, nrhs, 3, st));
        }
        s = levels(3, [&](const int32_t*, int32_t, size_t l) {
            const hylu_handle_s::SolveLists& S = h->tl[1];
            const int32_t s0 = S.sn_ptr[l], p0 = S.sp_ptr[l], k0 = S.task_ptr[l];
            return launch_ltsolve(f, h->D, h->vals, S.d_sn + s0, S.sn_ptr[l + 1] - s0, S.d_sp + p0,
                                  S.sp_ptr[l + 1] - p0, S.d_tasks + 2 * (int64_t)k0, S.task_ptr[l + 1] - k0, w.z, nrhs,
                                  st);
        });
        if (s != HYLU_OK) return s;
        HIPCHK(launch_permute_out(f, n, nrhs, h->d_perm_r, h->d_dr, w.z, x, ldx, accumulate, st));
    }
    return HYLU_OK;
}

hylu_status run_graph(hylu_handle h, GraphEntry& g, bool fresh, hipStream_t st,
                      const std::function<hylu_status(hipStream_t)>& body)
{
    if (fresh) {
        HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        hylu_status s = body(h->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
        if (s != HYLU_OK) { if (graph) hipGraphDestroy(graph); return s; }
        if (e != hipSuccess) { h->sticky_error = true; return HYLU_ERR_DEVICE; }
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(graph);
            h->sticky_error = true;
            return HYLU_ERR_DEVICE;
        }
        g.graph = graph;
        g.exec = exec;
    }
    HIPCHK(hipGraphLaunch(g.exec, st));
    return HYLU_OK;
}

// Graphs are cached per buffer address.  Callers that hand in fresh buffers on
// every call (autograd, allocators without reuse) would grow the cache without
// bound, so past a fixed size it is emptied after the device has drained.
constexpr size_t kGraphCache = 16;

template <typename Map>
void trim_graphs(Map& m)
{
    if (m.size() < kGraphCache) return;
    hipDeviceSynchronize();
    for (auto& kv : m) { hipGraphExecDestroy(kv.second.exec); hipGraphDestroy(kv.second.graph); }
    m.clear();
}

// a chain node v waits on source node s when s is a node of the same chain
// launch: the flag index of s there, else -1 (complete before the launch)
inline int32_t chain_source(const LevelTasks& T, int32_t v, int32_t s)
{
    if (T.chain_of.empty() || T.chain_of[v] < 0 || T.chain_of[s] != T.chain_of[v]) return -1;
    return T.chain_idx[s];
}

// device tables of the layout, uploaded on the first factorisation so the
// analysis itself needs no GPU
hylu_status upload_device(hylu_handle h)
{
    const Layout& L = h->lay;
    const Nodes& nd = h->nodes;
    const Csr& A = h->A;
    const LevelTasks& T = h->ft;
    const int32_t n = h->n;
    try {
        HIPCHK(hipGetDevice(&h->device));
        HIPCHK(scratch_setup(h->device));
        if (!h->h_norms_fixed) {
            const size_t nseg = h->member_row_off.size() - 1;
            if (hipHostMalloc((void**)&h->h_norms_fixed, sizeof(double) * kNormSlots * (kNoallocRhs + 1) * nseg) !=
                hipSuccess)
                return HYLU_ERR_OOM;
        }
        if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        if (!h->fact_done) HIPCHK(hipEventCreateWithFlags(&h->fact_done, hipEventDisableTiming));
        if (!h->h_pert && hipHostMalloc((void**)&h->h_pert, 2 * sizeof(int32_t)) != hipSuccess) return HYLU_ERR_OOM;
        std::vector<EdgeDesc> ed(L.esrc.size());
        for (int32_t v = 0; v < L.nnodes; v++)
            for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
                int32_t s = L.esrc[e];
                EdgeDesc& d = ed[e];
                d.uoff = L.voff[s] + L.lw[s];
                d.roff = L.eroff[e];
                d.Ws = L.W[s];
                d.ms = L.m[s];
                d.ws = L.W[s] - L.lw[s] - L.m[s];
                d.lp = L.elpos[e];
                d.r0s = L.r0[s];
                d.srcp = chain_source(T, v, s);
                d.ioff = h->inv_off[s];
            }
        std::vector<double> asr(h->nnz), asc(h->nnz);
        for (int32_t i = 0; i < n; i++)
            for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++) { asr[p] = h->dr[i]; asc[p] = h->dc[A.ci[p]]; }
        DevLayout& D = h->D;
        D = DevLayout();
        D.n = n; D.nnodes = L.nnodes; D.tail_node0 = L.tail_node0;
        int32_t *r0, *m, *lw, *W, *cols, *rel, *row_node, *pl, *qinv;
        int64_t *voff, *coff, *eptr;
        EdgeDesc* edges;
        UP(r0, L.r0); UP(m, L.m); UP(lw, L.lw); UP(W, L.W); UP(voff, L.voff); UP(coff, L.coff);
        UP(cols, L.cols); UP(eptr, L.eptr); UP(edges, ed); UP(rel, L.rel); UP(row_node, nd.of_row);
        std::vector<int32_t> zeros(n, 0);
        UP(pl, zeros); UP(qinv, zeros);
        D.r0 = r0; D.m = m; D.lw = lw; D.W = W; D.voff = voff; D.coff = coff; D.cols = cols;
        D.eptr = eptr; D.edges = edges; D.rel = rel; D.row_node = row_node; D.pl = pl; D.qinv = qinv;
        {
            int32_t *cw, *cpos, *crel;
            int64_t* cpoff;
            UP(cw, h->cw); UP(cpos, h->cpos); UP(cpoff, h->cpos_off);
            if (h->cpos.empty()) crel = rel;
            else UP(crel, h->crel);
            D.cw = cw; D.cpos = cpos; D.cpos_off = cpoff; D.crel = crel;
            uint8_t* snf;
            int32_t* sncnt;
            std::vector<int32_t> zn(std::max(L.nnodes, 1), 0);
            UP(snf, h->snfuse); UP(sncnt, zn);
            D.snfuse = snf; D.sncnt = sncnt;
        }
        UP(h->d_amap, L.amap); UP(h->d_asr, asr); UP(h->d_asc, asc);
        UP(h->d_rows, T.rows); UP(h->d_snodes, T.snodes); UP(h->d_tiles, T.tiles);
        UP(h->d_rrange, T.rrange);
        UP(h->d_inv_off, h->inv_off); UP(h->d_inv_nodes, h->inv_nodes);
        UP(h->d_tail_list, h->tail_list);
        UP(h->d_pert_rows, h->pert_rows);
        {
            std::vector<int32_t> sp;
            for (const Layout::Panel& P : L.spanels) { sp.push_back(P.p0); sp.push_back(P.p1); }
            UP(h->d_tsp, sp);
            h->d_tinv = dalloc(h, (size_t)std::max<size_t>(L.spanels.size(), 1) * 2 * kNB * kNB * (h->fp32 ? 4 : 8));
            if (!h->d_tinv) return HYLU_ERR_OOM;
        }
        h->d_uinv = dalloc(h, (size_t)std::max<int64_t>(h->inv_total, 1) * (h->fp32 ? 4 : 8));
        if (!h->d_uinv) return HYLU_ERR_OOM;
        D.uinv = h->d_uinv;
        for (int g = 0; g < 5; g++) UP(h->d_lev[g], L.xlev_nodes[g]);
        for (hylu_handle_s::SolveLists& S : h->sl) { UP(S.d_sn, S.sn_nodes); UP(S.d_sp, S.sp_nodes); UP(S.d_tasks, S.tasks); }
        for (hylu_handle_s::SolveLists& S : h->tl) { UP(S.d_sn, S.sn_nodes); UP(S.d_sp, S.sp_nodes); UP(S.d_tasks, S.tasks); }
        for (int g : {4, 1}) UP(h->d_lev_ptr[g], L.xlev_ptr[g]);
        {
            TailView& TVw = h->TV;
            TVw = TailView();
            TVw.mT = L.mT; TVw.t0 = L.t0; TVw.nc = L.mT;
            int64_t* trow; int32_t *tlo, *thi, *tpiv, *tstep;
            std::vector<int32_t> zt(std::max(L.mT, 1), 0);
            UP(trow, L.trow); UP(tlo, L.tlo); UP(thi, L.thi); UP(tpiv, zt); UP(tstep, zt);
            TVw.trow = trow; TVw.tlo = tlo; TVw.thi = thi; TVw.tpiv = tpiv; TVw.tstep = tstep;
            TVw.lbuf = dalloc(h, (size_t)64 * kGroup * std::max(L.mT, 1) * (h->fp32 ? 4 : 8));
            if (!TVw.lbuf) return HYLU_ERR_OOM;
        }
        for (hylu_handle_s::DenseSn& q : h->dsn) {
            const int32_t v = q.v, m = L.m[v], nc = L.W[v] - L.lw[v];
            std::vector<int64_t> tr(m);
            std::vector<int32_t> lo(m, 0), hi(m, m), z(std::max(m, nc), 0);
            for (int32_t a = 0; a < m; a++) tr[a] = L.voff[v] + (int64_t)a * L.W[v] + L.lw[v];
            int64_t* trow; int32_t *tlo, *thi, *tpiv, *tstep;
            UP(trow, tr); UP(tlo, lo); UP(thi, hi);
            std::vector<int32_t> zm(m, 0), zc(nc, 0);
            UP(tpiv, zm); UP(tstep, zc);
            q.TV = TailView();
            q.TV.mT = m; q.TV.nc = nc; q.TV.t0 = L.r0[v];
            q.TV.trow = trow; q.TV.tlo = tlo; q.TV.thi = thi; q.TV.tpiv = tpiv; q.TV.tstep = tstep;
            q.TV.lbuf = dalloc(h, (size_t)64 * kGroup * m * (h->fp32 ? 4 : 8));
            if (!q.TV.lbuf) return HYLU_ERR_OOM;
            std::vector<int32_t> sp;
            for (const Layout::Panel& P : q.spanels) { sp.push_back(P.p0); sp.push_back(P.p1); }
            UP(q.d_sp, sp);
            q.d_inv = dalloc(h, std::max<size_t>(q.spanels.size(), 1) * 2 * kNB * kNB * (h->fp32 ? 4 : 8));
            if (!q.d_inv) return HYLU_ERR_OOM;
        }
        UP(h->d_vext, h->vext_jobs);
        UP(h->d_vstep, h->vstep_jobs);
        if (!h->vjobs.empty() || !h->vstep_jobs.empty()) {
            std::vector<ViewDesc> vd(h->dsn.size());
            for (size_t q = 0; q < h->dsn.size(); q++) {
                vd[q].TV = h->dsn[q].TV;
                vd[q].sp = h->dsn[q].d_sp;
                vd[q].inv = h->dsn[q].d_inv;
            }
            UP(h->d_vdesc, vd);
            if (!h->vjobs.empty()) UP(h->d_vjobs, h->vjobs);
        }
        if (!h->dsn.empty()) {
            std::vector<uint8_t> fl(L.nnodes, 0);
            for (const hylu_handle_s::DenseSn& q : h->dsn) fl[q.v] = 1;
            uint8_t* d_fl;
            UP(d_fl, fl);
            h->D.dense_sn = d_fl;
        }
        if (!h->dsn.empty() && !h->side[0]) {
            for (int j = 0; j < hylu_handle_s::kSide; j++) {
                HIPCHK(hipStreamCreateWithFlags(&h->side[j], hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&h->ev_join[j], hipEventDisableTiming));
            }
            HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        }
        UP(h->d_perm_r, h->perm_r); UP(h->d_perm_c, h->perm_c);
        UP(h->d_dr, h->dr); UP(h->d_dc, h->dc);
        UP(h->d_arp, A.rp); UP(h->d_aci, A.ci); UP(h->d_aval, A.v);
        h->d_seg = nullptr;
        if (h->member_row_off.size() > 2) {
            std::vector<int32_t> seg(n);
            for (size_t k = 0; k + 1 < h->member_row_off.size(); k++)
                for (int64_t i = h->member_row_off[k]; i < h->member_row_off[k + 1]; i++) seg[i] = (int32_t)k;
            UP(h->d_seg, seg);
        }
        UP(h->d_ctask, T.ctask);
        UP(h->d_csthr, T.ctask_sthr);
        // [0]: perturbed pivots; [1]: a chain wait gave up (device error)
        int32_t* pert;
        std::vector<int32_t> one(2, 0);
        UP(pert, one);
        h->d_pert = pert;
        h->vals = dalloc(h, (size_t)std::max<int64_t>(L.nvals, 1) * (h->fp32 ? 4 : 8));
        if (!h->vals) return HYLU_ERR_OOM;
        h->uploaded = true;
    } catch (const std::bad_alloc&) {
        return HYLU_ERR_OOM;
    }
    return HYLU_OK;
}

// static pivoting and scaling (Sec. 2.1), then the fill-reducing ordering of
// the matched pattern: B = R A C with R = P_r D_r, C = D_c P_c
hylu_status order_matrix(const Csr& A, const hylu_options& opt, std::vector<int32_t>& perm_r,
                         std::vector<int32_t>& perm_c, std::vector<double>& dr, std::vector<double>& dc)
{
    const int32_t n = A.n;
    // ---- static pivoting and scaling (Sec. 2.1)
    std::vector<int32_t> match(n);
    dr.assign(n, 1.0);
    dc.assign(n, 1.0);
    if (opt.static_pivot) {
        if (!mc64_match_scale(A, match, dr, dc)) return HYLU_ERR_STRUCT_SINGULAR;
    } else {
        for (int32_t i = 0; i < n; i++) match[i] = i;
        // a row or column without entries is singular in any case
        std::vector<char> rowhas(n, 0), colhas(n, 0);
        for (int32_t i = 0; i < n; i++)
            for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++) { rowhas[i] = 1; colhas[A.ci[p]] = 1; }
        for (int32_t i = 0; i < n; i++) if (!rowhas[i] || !colhas[i]) return HYLU_ERR_STRUCT_SINGULAR;
    }
    // ---- fill-reducing ordering on the pattern of B0 + B0^T, B0 = matched A
    std::vector<int32_t> q(n);
    if (opt.ordering == 2) {
        for (int32_t i = 0; i < n; i++) q[i] = i;
    } else if (opt.ordering == 3) {
        std::vector<char> seen(n, 0);
        for (int32_t i = 0; i < n; i++) {
            int32_t x = opt.user_perm[i];
            if (x < 0 || x >= n || seen[x]) return HYLU_ERR_ARG;
            seen[x] = 1;
            q[i] = x;
        }
    } else {
        std::vector<int64_t> b0p(n + 1, 0);
        std::vector<int32_t> b0c;
        b0c.reserve(A.rp[n]);
        for (int32_t j = 0; j < n; j++) {
            int32_t r = match[j];
            for (int64_t p = A.rp[r]; p < A.rp[r + 1]; p++) b0c.push_back(A.ci[p]);
            b0p[j + 1] = (int64_t)b0c.size();
        }
        std::vector<int64_t> xadj;
        std::vector<int32_t> adj;
        symmetrize(n, b0p, b0c, xadj, adj);
        const double ad = opt.amd_dense > 0 ? opt.amd_dense : 0.0;
        q = opt.ordering == 0 ? amd_order(n, xadj, adj, ad)
                              : nd_order(n, xadj, adj, std::max(opt.nd_leaf, 8), ad, opt.ordering == 4);
        if ((int32_t)q.size() != n) return HYLU_ERR_INTERNAL;
    }
    perm_c = q;
    perm_r.resize(n);
    for (int32_t k = 0; k < n; k++) perm_r[k] = match[q[k]];
    return HYLU_OK;
}

// Compact rows: a dense-tail row's panel spans its outside sources' slots and
// every tail column, but its outside updates touch only the slots and the
// columns those sources' U rows reach.  Per tail node with sources, the sorted
// positions touched (the slots first, so a slot keeps its index) are listed
// when there are at most kCompactMax of them, with a copy of the relative maps
// whose entries for its sources index that list.  The row kernel takes the
// compact row where the whole row does not fit the launch's LDS row capacity
// and the compact one does (instead of accumulating in global memory).
constexpr int32_t kCompactMax = kRowCapBig;
void build_compact_rows(hylu_handle h)
{
    const Layout& L = h->lay;
    h->cw.assign(L.nnodes, 0);
    h->cpos_off.assign(L.nnodes + 1, 0);
    h->cpos.clear();
    h->crel = L.rel;
    int32_t wmax = 0;
    for (int32_t v = L.tail_node0; v < L.nnodes; v++) wmax = std::max(wmax, L.W[v]);
    std::vector<int32_t> idx(std::max(wmax, 1), -1);
    std::vector<int32_t> touched;
    for (int32_t v = 0; v < L.nnodes; v++) {
        h->cpos_off[v + 1] = h->cpos_off[v];
        if (v < L.tail_node0 || L.eptr[v + 1] == L.eptr[v]) continue;
        touched.clear();
        for (int32_t j = 0; j < L.lw[v]; j++) { idx[j] = 0; touched.push_back(j); }
        for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
            const int32_t s = L.esrc[e];
            const int32_t ws = L.W[s] - L.lw[s] - L.m[s];
            for (int32_t t = 0; t < ws; t++) {
                const int32_t r = L.rel[L.eroff[e] + t];
                if (idx[r] < 0) { idx[r] = 0; touched.push_back(r); }
            }
        }
        std::sort(touched.begin(), touched.end());
        const bool compact = (int32_t)touched.size() <= kCompactMax && (int32_t)touched.size() < L.W[v];
        for (size_t k = 0; k < touched.size(); k++) idx[touched[k]] = (int32_t)k;
        if (compact) {
            h->cw[v] = (int32_t)touched.size();
            h->cpos.insert(h->cpos.end(), touched.begin(), touched.end());
            h->cpos_off[v + 1] = (int64_t)h->cpos.size();
            for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
                const int32_t s = L.esrc[e];
                const int32_t ws = L.W[s] - L.lw[s] - L.m[s];
                for (int32_t t = 0; t < ws; t++) h->crel[L.eroff[e] + t] = idx[L.rel[L.eroff[e] + t]];
            }
        }
        for (int32_t r : touched) idx[r] = -1;
    }
    if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2) {
        int64_t nc = 0, wc = 0, wf = 0, nt = 0;
        for (int32_t v = L.tail_node0; v < L.nnodes; v++) {
            if (L.eptr[v + 1] == L.eptr[v]) continue;
            nt++;
            wf += (int64_t)L.W[v] * L.m[v];
            if (h->cw[v] > 0) { nc++; wc += (int64_t)h->cw[v] * L.m[v]; }
        }
        std::fprintf(stderr, "hylu: compact rows: %lld of %lld tail nodes with sources, %lld of %lld row entries\n",
                     (long long)nc, (long long)nt, (long long)wc, (long long)wf);
    }
}

// The chain launches of pipeline mode, checked on the host against the rule
// the device relies on: each launch covers consecutive chain levels, the
// launches take the chain levels in order, every node of a chain level is the
// node of exactly one launch, in level order; a chain node only takes sources
// that are complete before its launch (lower levels, not in a later launch)
// or nodes of its own launch with a lower index.  Then no wait can deadlock:
// the lowest unfinished node of a launch always has its sources, and its
// wavefront (which takes its nodes in increasing index) is working on it.
hylu_status check_chains(hylu_handle h)
{
    const LevelTasks& T = h->ft;
    const Layout& L = h->lay;
    const Nodes& nd = h->nodes;
    const int32_t nl = (int32_t)T.maxW.size();
    if (T.chains.empty()) return T.ctask.empty() ? HYLU_OK : HYLU_ERR_INTERNAL;
    if ((int32_t)T.chain_lev.size() != nl || (int32_t)T.chain_start.size() != nl) return HYLU_ERR_INTERNAL;
    std::vector<char> seen(L.nnodes, 0);
    std::vector<char> covered(nl, 0);
    int64_t tnext = 0;
    int32_t lprev = 0;
    for (size_t c = 0; c < T.chains.size(); c++) {
        const LevelTasks::Chain& ch = T.chains[c];
        if (ch.l0 < lprev || ch.l1 <= ch.l0 || ch.l1 > nl || ch.t0 != tnext || ch.t1 <= ch.t0 ||
            ch.t1 - ch.t0 > kChainTasksMax)
            return HYLU_ERR_INTERNAL;
        const bool first = c == 0 || T.chains[c - 1].l1 != ch.l0;
        if (first != (T.chain_start[ch.l0] == (int32_t)c)) return HYLU_ERR_INTERNAL;
        for (int32_t l = ch.l0; l < ch.l1; l++) {
            if (!T.chain_lev[l] || covered[l]) return HYLU_ERR_INTERNAL;
            covered[l] = 1;
        }
        int32_t prev_level = ch.l0;
        for (int64_t t = ch.t0; t < ch.t1; t++) {
            const int32_t x = T.ctask[t];
            const int64_t ti = t - ch.t0;
            const bool lu = x < 0;
            const int32_t v = lu ? -x - 1 : nd.of_row[x];
            if (v < 0 || v >= L.nnodes) return HYLU_ERR_INTERNAL;
            const int32_t lv = T.node_level[v];
            if (seen[v] || lv < prev_level || lv >= ch.l1 || v >= L.tail_node0 || L.m[v] > kChainSnMax ||
                T.chain_of[v] != (int32_t)c)
                return HYLU_ERR_INTERNAL;
            prev_level = lv;
            const bool last = lu || L.m[v] == 1;
            if ((T.chain_idx[v] == ti) != last || (lu && L.m[v] < 2)) return HYLU_ERR_INTERNAL;
            if (last) seen[v] = 1;
            if (lu) {
                // its row tasks just before it, in order (when it has sources)
                if (L.eptr[v + 1] > L.eptr[v])
                    for (int32_t a = 0; a < L.m[v]; a++) {
                        const int64_t q = t - L.m[v] + a;
                        if (q < ch.t0 || T.ctask[q] != L.r0[v] + a) return HYLU_ERR_INTERNAL;
                    }
                continue;
            }
            for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
                const int32_t s = L.esrc[e];
                const bool before = T.node_level[s] < ch.l0 && T.chain_of[s] < (int32_t)c;
                const bool earlier = T.chain_of[s] == (int32_t)c && T.chain_idx[s] < ti;
                if (!before && !earlier) {
                    std::fprintf(stderr, "hylu: pipelined schedule: row %d takes node %d before it is complete\n", x, s);
                    return HYLU_ERR_INTERNAL;
                }
            }
        }
        lprev = ch.l1;
        tnext = ch.t1;
    }
    if (tnext != (int64_t)T.ctask.size()) return HYLU_ERR_INTERNAL;
    for (int32_t l = 0; l < nl; l++)
        if (T.chain_lev[l] && !covered[l]) return HYLU_ERR_INTERNAL;
    for (int32_t v = 0; v < L.nnodes; v++)
        if (T.chain_lev[T.node_level[v]] && !seen[v]) return HYLU_ERR_INTERNAL;
    return HYLU_OK;
}

// device memory of the analysis (GPU symbolic factorisation), freed before it returns
void* analysis_alloc(void* ctx, size_t bytes)
{
    hylu_handle h = static_cast<hylu_handle>(ctx);
    void* p = nullptr;
    if (h->has_alloc) p = h->alloc.alloc(h->alloc.ctx, bytes, nullptr);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    return p;
}

void analysis_free(void* ctx, void* p)
{
    hylu_handle h = static_cast<hylu_handle>(ctx);
    if (h->has_alloc) h->alloc.free(h->alloc.ctx, p, nullptr);
    else (void)hipFree(p);
}

// FNV-1a over the compressed structure and the level sets
uint64_t structure_hash(const Symbolic& s, const Nodes& nd)
{
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t bytes) {
        const unsigned char* c = static_cast<const unsigned char*>(p);
        for (size_t k = 0; k < bytes; k++) { x ^= c[k]; x *= 1099511628211ull; }
    };
    auto vec = [&](const auto& v) { mix(v.data(), v.size() * sizeof(v[0])); };
    vec(s.lp); vec(s.lint); vec(s.run_of); vec(s.run_start); vec(s.run_up); vec(s.run_u);
    vec(s.lcount); vec(s.ucount);
    mix(&s.flops, sizeof(s.flops));
    vec(nd.ptr); vec(nd.is_sn);
    for (int t = 0; t < 4; t++) vec(nd.level[t]);
    return x;
}

hylu_status analyze_structure(hylu_handle h, PhaseLog& plog)
{
    const int32_t n = h->n;
    const hylu_options& opt = h->opt;
    const Csr& A = h->A;
    // ---- B = R A C (pattern, sorted) and the source position of each entry
    std::vector<int32_t> pcinv(n);
    for (int32_t k = 0; k < n; k++) pcinv[h->perm_c[k]] = k;
    Csr B;
    B.n = n;
    B.rp.assign(n + 1, 0);
    B.ci.resize(h->nnz);
    std::vector<int64_t> bsrc(h->nnz);
    {
        std::vector<std::pair<int32_t, int64_t>> rowbuf;
        int64_t q0 = 0;
        for (int32_t i = 0; i < n; i++) {
            int32_t r = h->perm_r[i];
            rowbuf.clear();
            for (int64_t p = A.rp[r]; p < A.rp[r + 1]; p++) rowbuf.push_back({pcinv[A.ci[p]], p});
            std::sort(rowbuf.begin(), rowbuf.end());
            for (auto& e : rowbuf) { B.ci[q0] = e.first; bsrc[q0] = e.second; q0++; }
            B.rp[i + 1] = q0;
        }
    }
    // ---- symbolic factorisation, flops, supernodes, levels (Sec. 2.1, 2.2, 2.2.1)
    plog("permute");
    int32_t sn_min = opt.sn_min, sn_max = opt.sn_max;
    if (opt.kernel_mode == 1) sn_min = std::numeric_limits<int32_t>::max();
    const auto ts = std::chrono::steady_clock::now();
    h->sym_kernel_ms = 0.0;
    if (opt.gpu_symbolic) {
        DeviceAlloc da{h, analysis_alloc, analysis_free};
        GpuSymStats gs;
        std::string e;
        if (!gpu_symbolic_levels(B, h->member_row_off, sn_min, sn_max, da, h->sym, h->nodes, gs, e)) {
            std::fprintf(stderr, "hylu: %s\n", e.c_str());
            return e.find("1 << 20") != std::string::npos ? HYLU_ERR_ARG : HYLU_ERR_DEVICE;
        }
        h->sym_kernel_ms = gs.ms_structure + gs.ms_levels;
        plog("symbolic, nodes and levels on the GPU");
    } else {
        if (!symbolic_factor(B, h->sym)) return HYLU_ERR_INTERNAL;
        plog("symbolic");
        make_nodes(h->sym, sn_min, sn_max, h->nodes);
        make_levels(h->sym, h->nodes);
        plog("nodes");
    }
    h->sym_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ts).count();
    h->sym_hash = structure_hash(h->sym, h->nodes);
    std::string err;
    int32_t tail_node0 = choose_tail(h->sym, h->nodes, opt.dense_tail, std::max(opt.tail_min, 1),
                                     opt.tail_max > 0 ? opt.tail_max : 32768);
    if (!build_layout(B, h->sym, h->nodes, tail_node0, 64, h->lay, bsrc, err)) {
        std::fprintf(stderr, "hylu: %s\n", err.c_str());
        return HYLU_ERR_INTERNAL;
    }
    plog("layout");
    // ---- perturbation threshold
    double bmax = 0.0;
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = A.rp[i]; p < A.rp[i + 1]; p++)
            bmax = std::max(bmax, std::fabs(h->dr[i] * A.v[p] * h->dc[A.ci[p]]));
    // the threshold belongs to the FP64 problem: FP32 factors perturb the same
    // pivots as FP64 ones (sqrt of the FP32 epsilon, 3.45e-4, would replace
    // pivots that FP32 represents well and stall the refinement)
    double eps = std::numeric_limits<double>::epsilon();
    h->tau = (opt.pivot_tau > 0 ? opt.pivot_tau : std::sqrt(eps)) * (bmax > 0 ? bmax : 1.0);
    // ---- level task lists of the factorisation
    build_compact_rows(h);
    const Layout& L = h->lay;
    const Nodes& nd = h->nodes;
    LevelTasks& T = h->ft;
    T = LevelTasks();
    // factor levels; the dense tail's rows take their outside updates in one
    // extra level after all others: nothing outside the tail depends on them,
    // so they need not sit on the chain of narrow levels (nor need the other
    // nodes that feed nobody)
    std::vector<std::vector<int32_t>> lvnodes;
    std::vector<std::pair<int32_t, int32_t>> late_nodes;      // (level by its sources, node) of the deferred ones
    {
        const int32_t nx = (int32_t)L.xlev_ptr[0].size() - 1;
        lvnodes.resize(nx);
        std::vector<int32_t> tailn;
        // a node no other node takes updates from can run as late as the tail
        // rows do; with a tail present such nodes join that final level
        std::vector<char> feeds(L.nnodes, 0);
        for (int32_t v = 0; v < L.nnodes; v++)
            for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) feeds[L.esrc[e]] = 1;
        const bool tail = L.tail_node0 < L.nnodes;
        for (int32_t l = 0; l < nx; l++)
            for (int32_t t = L.xlev_ptr[0][l]; t < L.xlev_ptr[0][l + 1]; t++) {
                const int32_t v = L.xlev_nodes[0][t];
                const bool late = v >= L.tail_node0 || (tail && l > 0 && !feeds[v]);
                (late ? tailn : lvnodes[l]).push_back(v);
                if (late) late_nodes.push_back({l, v});
            }
        while (!lvnodes.empty() && lvnodes.back().empty()) lvnodes.pop_back();
        if (!tailn.empty()) lvnodes.push_back(std::move(tailn));
        else late_nodes.clear();
    }
    int32_t nl = (int32_t)lvnodes.size();
    std::vector<std::vector<std::array<int64_t, 3>>> lvpieces(nl);   // per level: (row, first, end source)
    // pipeline mode (Sec. 2.2.1): every run of at least kChainRunMin
    // consecutive levels (before the deferred final one, after level 0) of at
    // most pipeline_rows rows, whose nodes are standalone rows or supernodes of
    // at most kChainSnMax rows that no blocked or tile kernel takes, runs as
    // chain launches; every other level stays a bulk launch
    std::vector<char> chain_lev(nl, 0);
    if (opt.pipeline_rows > 0 && nl > 0) {
        const int32_t nmain = late_nodes.empty() ? nl : nl - 1;
        const int32_t big_ = opt.sn_dense > 0 ? opt.sn_dense : std::numeric_limits<int32_t>::max();
        const int32_t tile_ = opt.sn_tile > 0 ? opt.sn_tile : std::numeric_limits<int32_t>::max();
        const int64_t maxrows = std::min<int64_t>(opt.pipeline_rows, kChainTasksMax / 2);   // tasks <= 2 rows
        auto ok = [&](int32_t l) {
            int64_t r = 0;
            for (int32_t v : lvnodes[l]) {
                r += L.m[v];
                if (v >= L.tail_node0 || L.m[v] > kChainSnMax) return false;
                if (nd.is_sn[v] && (L.m[v] >= big_ || L.m[v] >= tile_)) return false;
            }
            return r <= maxrows;
        };
        for (int32_t l = 1; l < nmain;) {
            int32_t e = l;
            while (e < nmain && ok(e)) e++;
            if (e - l >= kChainRunMin)
                for (int32_t q = l; q < e; q++) chain_lev[q] = 1;
            l = std::max(e, l + 1);
        }
    }
    // deferred standalone rows and tail rows join the launches of the narrow
    // levels (fewer than kSideNarrowRows rows) once their sources are
    // complete: one row per idle CU, and only where the level's own longest
    // row is estimated to take at least as long (sources applied one after
    // the other, plus the update volume), so the level does not get longer.
    // The rest stay in the final level.
    if (opt.side_rows && !late_nodes.empty()) {
        const int32_t nmain = nl - 1;
        auto cost = [&](int32_t v) {
            double c = 0;
            for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
                const int32_t u = L.esrc[e];
                c += 1.0 + (double)L.m[u] * (L.W[u] - L.lw[u]) / 2048.0;
            }
            // (a row accumulator in global memory when it does not fit in LDS)
            return (h->cw[v] == 0 && L.W[v] > kRowCapBig) ? 3.0 * c : c;
        };
        std::vector<int64_t> nrow(nmain, 0), room(nmain, 0);
        std::vector<double> lmax(nmain, 0.0);
        for (int32_t l = 0; l < nmain; l++)
            for (int32_t v : lvnodes[l]) { nrow[l] += L.m[v]; lmax[l] = std::max(lmax[l], cost(v)); }
        for (int32_t l = 0; l < nmain; l++) room[l] = nrow[l] < kSideNarrowRows ? kSideNarrowRows - nrow[l] : 0;
        for (int32_t l = 0; l < nmain; l++) if (chain_lev[l]) room[l] = 0;     // not into chain launches
        std::vector<char> moved(L.nnodes, 0);
        std::vector<std::pair<int32_t, int32_t>> order(late_nodes);
        std::sort(order.begin(), order.end());
        for (const auto& q : order) {
            const int32_t v = q.second;
            if (!(L.m[v] == 1 || v >= L.tail_node0)) continue;
            const double c = cost(v);
            for (int32_t l = std::max(q.first, 0); l < nmain; l++) {
                if (room[l] < L.m[v] || lmax[l] < c) continue;
                lvnodes[l].push_back(v);
                room[l] -= L.m[v];
                moved[v] = 1;
                break;
            }
        }
        // a tail node too long for any narrow level takes its sources in
        // pieces: in order, each piece in a later narrow level than the one
        // before, once its sources are complete and while its estimated cost
        // stays within the level's; the rest in the final level
        std::vector<int32_t> lev_of(L.nnodes, -1);
        for (int32_t l = 0; l < nmain; l++)
            for (int32_t v : lvnodes[l]) lev_of[v] = l;
        for (const auto& q : order) {
            const int32_t v = q.second;
            if (moved[v] || v < L.tail_node0 || L.eptr[v + 1] == L.eptr[v]) continue;
            // (pieces are held to half the level's estimate: a piece also
            // loads and stores the whole row)
            const double mult = 2.0 * ((h->cw[v] == 0 && L.W[v] > kRowCapBig) ? 3.0 : 1.0);
            int64_t e = L.eptr[v];
            const int64_t e1 = L.eptr[v + 1];
            std::vector<std::array<int64_t, 3>> pieces;     // (level, first, end)
            for (int32_t l = std::max(q.first, 0); l < nmain && e < e1; l++) {
                if (room[l] < L.m[v]) continue;
                const int64_t e0 = e;
                double c = 0;
                while (e < e1) {
                    const int32_t u = L.esrc[e];
                    if (lev_of[u] < 0 || lev_of[u] >= l) break;
                    const double cu = mult * (1.0 + (double)L.m[u] * (L.W[u] - L.lw[u]) / 2048.0);
                    if (c + cu > lmax[l]) break;
                    c += cu;
                    e++;
                }
                if (e > e0) { pieces.push_back({l, e0, e}); room[l] -= L.m[v]; }
            }
            if (pieces.empty()) continue;
            if (e < e1) pieces.push_back({nl - 1, e, e1});
            for (const auto& pc : pieces)
                for (int32_t r = L.r0[v]; r < L.r0[v] + L.m[v]; r++) lvpieces[pc[0]].push_back({r, pc[1], pc[2]});
            moved[v] = 1;
        }
        auto& fin = lvnodes[nl - 1];
        fin.erase(std::remove_if(fin.begin(), fin.end(), [&](int32_t v) { return moved[v] != 0; }), fin.end());
    }
    T.row_ptr.assign(1, 0); T.sn_ptr.assign(1, 0);
    h->max_sn = 0;
    h->dsn.clear();
    h->dsn_ptr.assign(1, 0);
    h->sn_groups = h->tail_groups = 0;
    const int32_t big = opt.sn_dense > 0 ? opt.sn_dense : std::numeric_limits<int32_t>::max();
    const int32_t gmin = opt.group_min_rows > 0 ? opt.group_min_rows : kGroupMinRows;
    const int32_t tile_min = opt.sn_tile > 0 ? opt.sn_tile : std::numeric_limits<int32_t>::max();
    T.tile_ptr.assign(1, 0);
    T.rrange.clear();
    h->pert_rows.clear();
    T.lvrows.assign(nl, 0);
    h->snfuse.assign(L.nnodes, 0);
    for (int32_t l = 0; l < nl; l++) {
        int32_t mw = 0, mm = 0;
        // a narrow level's row launch also factors its small supernodes (one
        // launch fewer); a wide level keeps a launch of its own for them, where
        // every supernode has a full workgroup
        int64_t lrows = (int64_t)lvpieces[l].size();
        for (int32_t v : lvnodes[l]) lrows += L.m[v];
        const bool narrow = lrows <= kSideNarrowRows;
        for (int32_t v : lvnodes[l]) {
            if (chain_lev[l]) {
                // a node of a chain launch: its rows and block LU there; the
                // level's width and rows as a bulk launch would have them
                if (L.eptr[v + 1] > L.eptr[v]) { mw = std::max(mw, L.W[v]); T.lvrows[l] += L.m[v]; }
                continue;
            }
            if (L.eptr[v + 1] == L.eptr[v]) {
                // no sources: nothing to apply; a standalone row outside the
                // tail only has its pivot checked (one small launch for all)
                if (L.m[v] == 1 && v < L.tail_node0) h->pert_rows.push_back(L.r0[v]);
            } else if (nd.is_sn[v] && v < L.tail_node0 && L.m[v] >= tile_min) {
                // outside updates of a large supernode target by 16-row tiles
                for (int32_t a = 0; a < L.m[v]; a += kTileRowsHost) { T.tiles.push_back(v); T.tiles.push_back(a); }
            } else {
                for (int32_t r = L.r0[v]; r < L.r0[v] + L.m[v]; r++) {
                    T.rows.push_back(r);
                    T.rrange.push_back(L.eptr[v]);
                    T.rrange.push_back(L.eptr[v + 1]);
                }
                mw = std::max(mw, L.W[v]);
            }
            if (!nd.is_sn[v] || v >= L.tail_node0) continue;
            if (L.m[v] >= big) {
                // blocked LU on the supernode's panel: kWideChunk-row panels, the
                // whole block as pivot window, T columns updated by TRSM/GEMM
                hylu_handle_s::DenseSn q;
                q.v = v;
                q.level = l;
                for (int32_t k = 0; k < L.m[v]; k += kWideChunk)
                    q.panels.push_back({k, std::min(k + kWideChunk, L.m[v]), 0, L.m[v], 0});
                for (int32_t k = 0; k < L.m[v]; k += 64)
                    q.spanels.push_back({k, std::min(k + 64, L.m[v]), 0, L.m[v], 0});
                std::vector<uint32_t> none;
                h->sn_groups += plan_dense(q.panels, L.m[v], L.W[v] - L.lw[v], nullptr, true, gmin, q.ops, none);
                h->dsn.push_back(std::move(q));
            } else if (narrow && L.eptr[v + 1] > L.eptr[v] && L.m[v] < tile_min && L.m[v] <= kFuseSnMax) {
                // its rows are this level's row tasks: the last of them factors it
                h->snfuse[v] = 1;
            } else {
                T.snodes.push_back(v);
                mm = std::max(mm, L.m[v]);
            }
        }
        for (const auto& pc : lvpieces[l]) {
            T.rows.push_back((int32_t)pc[0]);
            T.rrange.push_back(pc[1]);
            T.rrange.push_back(pc[2]);
            mw = std::max(mw, L.W[nd.of_row[pc[0]]]);
        }
        h->dsn_ptr.push_back((int32_t)h->dsn.size());
        T.row_ptr.push_back((int64_t)T.rows.size());
        T.tile_ptr.push_back((int64_t)T.tiles.size() / 2);
        T.sn_ptr.push_back((int64_t)T.snodes.size());
        T.maxW.push_back(mw);
        T.maxm.push_back(mm);
        h->max_sn = std::max(h->max_sn, mm);
    }
    // HYLU_LOG=2: the row tasks of every factor level (3: and each row of the last one)
    if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2) {
        for (int32_t l = 0; l < nl; l++) {
            int64_t maxsrc = 0, sumsrc = 0, tailr = 0;
            for (int64_t t = T.row_ptr[l]; t < T.row_ptr[l + 1]; t++) {
                const int64_t ns = T.rrange[2 * t + 1] - T.rrange[2 * t];
                maxsrc = std::max(maxsrc, ns);
                sumsrc += ns;
                if (nd.of_row[T.rows[t]] >= L.tail_node0) tailr++;
            }
            std::fprintf(stderr, "hylu: level %d row tasks %lld (tail %lld) sources max %lld sum %lld maxW %d\n", l,
                         (long long)(T.row_ptr[l + 1] - T.row_ptr[l]), (long long)tailr, (long long)maxsrc,
                         (long long)sumsrc, T.maxW[l]);
            if (std::atoi(lg) >= 3 && l == nl - 1)
                for (int64_t t = T.row_ptr[l]; t < T.row_ptr[l + 1]; t++)
                    std::fprintf(stderr, "hylu:   row %d sources %lld W %d\n", T.rows[t],
                                 (long long)(T.rrange[2 * t + 1] - T.rrange[2 * t]), L.W[nd.of_row[T.rows[t]]]);
        }
    }
    // the dense tail's launches, block-sparse by its structural masks
    h->tail_ops.clear();
    h->tail_list.clear();
    h->tail_flops = 0.0;
    if (L.mT > 0) {
        TailMasks M;
        tail_masks(h->sym, nd, L, M);
        // panel groups for a large tail (each pass over its trailing matrix
        // is costly: 27-point 64^3, 32786 rows, 4.68 vs 4.89 s) or where the
        // block-sparse plan keeps more than half of the dense work; not for a
        // small sparse tail (circuit, 8315 rows: 29.4 vs 30.7 ms).  The choice
        // does not depend on tail_sparse, so both plans sum in the same order.
        bool group = L.mT >= (opt.group_tail_rows > 0 ? opt.group_tail_rows : kGroupTailRows);
        if (!group) {
            std::vector<DenseOp> probe;
            std::vector<uint32_t> plist;
            plan_dense(L.panels, L.mT, L.mT, &M, false, gmin, probe, plist);
            double fl = 0.0;
            for (const DenseOp& o : probe) fl += o.flops;
            const double mTd = L.mT;
            group = fl > 0.5 * (2.0 * mTd * mTd * mTd / 3.0);
        }
        h->tail_groups = plan_dense(L.panels, L.mT, L.mT, opt.tail_sparse ? &M : nullptr, group, gmin, h->tail_ops,
                                    h->tail_list);
        for (const DenseOp& o : h->tail_ops) h->tail_flops += o.flops;
    }
    plan_shared_views(h);
    plog("tail plan");
    T.row_nt.assign(nl, 0);
    // a level of few rows runs one row per CU at most: its rows may take
    // the large staging buffer, so wide standalone sources are loaded in
    // batches rather than one after the other
    // and hold wider rows in LDS (first the row, then as large a stage as fits)
    T.row_stage.assign(nl, kStageSmall);
    T.row_cap.assign(nl, kRowCapSmall);
    for (int32_t l = 0; l < nl; l++) {
        if (T.row_ptr[l + 1] - T.row_ptr[l] + T.lvrows[l] > kSideNarrowRows) continue;
        const int32_t cap = std::min(std::max(T.maxW[l], kRowCapSmall), kRowCapBig);
        int32_t stage = kStageMax;
        while (stage > kStageSmall && factor_rows_lds(h->fp32, stage, cap) > kLdsMax) stage -= 256;
        if (factor_rows_lds(h->fp32, stage, cap) > kLdsMax) continue;
        T.row_stage[l] = stage;
        T.row_cap[l] = cap;
        // one long row per CU: eight wavefronts share its staging and updates
        if (T.maxW[l] > 1024) T.row_nt[l] = 1024;
    }
    T.sn_nt.assign(nl, 0);
    T.node_level.assign(L.nnodes, 0);
    for (int32_t l = 0; l < nl; l++)
        for (int32_t v : lvnodes[l]) T.node_level[v] = l;
    // block inverses of the supernodes outside the tail with 2..kInvMax rows,
    // computed in the level of their factorisation
    h->inv_off.assign(L.nnodes, -1);
    h->inv_total = 0;
    h->inv_ptr.assign(1, 0);
    h->inv_nodes.clear();
    h->inv_maxm.clear();
    for (int32_t l = 0; l < nl; l++) {
        int32_t mm = 0;
        if (opt.sn_inverse)
            for (int32_t v : lvnodes[l]) {
                if (!nd.is_sn[v] || v >= L.tail_node0 || L.m[v] < 2 || L.m[v] > kInvMax) continue;
                h->inv_off[v] = h->inv_total;
                h->inv_total += (int64_t)L.m[v] * L.m[v];
                // the supernode-LU kernel inverts its own nodes; the large
                // supernodes' dense views take a launch after the level
                if (L.m[v] < big) continue;
                h->inv_nodes.push_back(v);
                mm = std::max(mm, L.m[v]);
            }
        h->inv_ptr.push_back((int64_t)h->inv_nodes.size());
        h->inv_maxm.push_back(mm);
    }
    // the forward and backward solve levels' supernodes of kLsolveSnMin..64
    // rows: whole, or split by rows when their L region (the U columns past
    // their block) is long
    {
        std::vector<uint8_t> dense(L.nnodes, 0);
        for (const hylu_handle_s::DenseSn& q : h->dsn) dense[q.v] = 1;
        for (int k = 0; k < 2; k++) {
            const int g = k == 0 ? 4 : 1;
            hylu_handle_s::SolveLists& S = h->sl[k];
            S.sn_ptr.assign(1, 0); S.sp_ptr.assign(1, 0); S.task_ptr.assign(1, 0);
            S.sn_nodes.clear(); S.sp_nodes.clear(); S.tasks.clear(); S.small.clear();
            for (size_t l = 0; l + 1 < L.xlev_ptr[g].size(); l++) {
                uint8_t small = 0;
                for (int32_t t = L.xlev_ptr[g][l]; t < L.xlev_ptr[g][l + 1]; t++) {
                    const int32_t v = L.xlev_nodes[g][t], m = L.m[v];
                    if (dense[v]) continue;
                    if (m < kLsolveSnMin || m > 64) { small = 1; continue; }
                    const int64_t len = k == 0 ? L.lw[v] : L.W[v] - L.lw[v] - m;
                    if (!opt.solve_split || (int64_t)m * len < kSplitWork) { S.sn_nodes.push_back(v); continue; }
                    S.sp_nodes.push_back(v);
                    for (int32_t g0 = 0; g0 < m; g0 += kSplitRows) { S.tasks.push_back(v); S.tasks.push_back(g0); }
                }
                S.small.push_back(small);
                S.sn_ptr.push_back((int32_t)S.sn_nodes.size());
                S.sp_ptr.push_back((int32_t)S.sp_nodes.size());
                S.task_ptr.push_back((int32_t)S.tasks.size() / 2);
            }
        }
        for (int k = 0; k < 2; k++) {
            const int g = k == 0 ? 2 : 3;
            hylu_handle_s::SolveLists& S = h->tl[k];
            S.sn_ptr.assign(1, 0); S.sp_ptr.assign(1, 0); S.task_ptr.assign(1, 0);
            S.sn_nodes.clear(); S.sp_nodes.clear(); S.tasks.clear(); S.small.clear();
            for (size_t l = 0; l + 1 < L.xlev_ptr[g].size(); l++) {
                for (int32_t t = L.xlev_ptr[g][l]; t < L.xlev_ptr[g][l + 1]; t++) {
                    const int32_t v = L.xlev_nodes[g][t], m = L.m[v];
                    if (!opt.solve_split || m < kLsolveSnMin) { S.sn_nodes.push_back(v); continue; }
                    S.sp_nodes.push_back(v);
                    for (int32_t g0 = 0; g0 < m; g0 += kSplitRows) { S.tasks.push_back(v); S.tasks.push_back(g0); }
                }
                S.sn_ptr.push_back((int32_t)S.sn_nodes.size());
                S.sp_ptr.push_back((int32_t)S.sp_nodes.size());
                S.task_ptr.push_back((int32_t)S.tasks.size() / 2);
            }
        }
    }
    // the large supernodes' places in the L-solve and U-solve level sequences
    {
        std::vector<int32_t> dix(L.nnodes, -1);
        for (size_t q = 0; q < h->dsn.size(); q++) dix[h->dsn[q].v] = (int32_t)q;
        h->vext_jobs.clear();
        h->vstep_jobs.clear();
        for (int g : {4, 1}) {
            auto& out = g == 4 ? h->dsn_l : h->dsn_u;
            out.assign(L.xlev_ptr[g].size() > 0 ? L.xlev_ptr[g].size() - 1 : 0, {});
            for (size_t l = 0; l + 1 < L.xlev_ptr[g].size(); l++)
                for (int32_t t = L.xlev_ptr[g][l]; t < L.xlev_ptr[g][l + 1]; t++)
                    if (dix[L.xlev_nodes[g][t]] >= 0) out[l].push_back(dix[L.xlev_nodes[g][t]]);
            // the levels' large supernodes launched together (solve_split)
            auto& VS = h->vsolve[g == 4 ? 0 : 1];
            VS.assign(out.size(), {});
            for (size_t l = 0; opt.solve_split && l < out.size(); l++) {
                if (out[l].size() < 2) continue;
                hylu_handle_s::ViewSolve& V = VS[l];
                V.e0 = (int64_t)h->vext_jobs.size() / 2;
                size_t nsmax = 0;
                for (int32_t q : out[l]) {
                    const hylu_handle_s::DenseSn& d = h->dsn[q];
                    for (int32_t b = 0; b < (L.m[d.v] + 3) / 4; b++) { h->vext_jobs.push_back(d.v); h->vext_jobs.push_back(b); }
                    nsmax = std::max(nsmax, d.spanels.size());
                }
                V.e1 = (int64_t)h->vext_jobs.size() / 2;
                for (size_t k = 0; k < nsmax; k++) {
                    const int64_t j0 = (int64_t)h->vstep_jobs.size();
                    for (int32_t q : out[l]) {
                        const hylu_handle_s::DenseSn& d = h->dsn[q];
                        const std::vector<Layout::Panel>& SP = d.spanels;
                        const int32_t ns = (int32_t)SP.size(), mT = L.m[d.v];
                        if ((int32_t)k >= ns) continue;
                        // the arguments launch_tail_step gets for this step
                        SolveJob J{};
                        J.view = q;
                        if (g == 4) {
                            const int32_t c = (int32_t)k;          // solved panel
                            J.q0 = SP[c].p0; J.q1 = SP[c].p1; J.inv = 2 * c;
                            if (c > 0) { J.p0 = SP[c - 1].p0; J.p1 = SP[c - 1].p1; J.first = J.q1; J.count = mT - J.q1; }
                        } else {
                            const int32_t c = ns - 1 - (int32_t)k;
                            J.q0 = SP[c].p0; J.q1 = SP[c].p1; J.inv = 2 * c + 1;
                            if (c < ns - 1) { J.p0 = SP[c + 1].p0; J.p1 = SP[c + 1].p1; J.first = 0; J.count = J.q0; }
                        }
                        const int32_t nb = 1 + (J.count + 3) / 4;
                        for (int32_t b = 0; b < nb; b++) { J.blk = b; h->vstep_jobs.push_back(J); }
                    }
                    V.steps.push_back({j0, (int64_t)h->vstep_jobs.size()});
                }
            }
            // HYLU_LOG=2: the large supernodes per solve level
            if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2) {
                size_t lv = 0, nv = 0, mx = 0;
                for (const auto& q : out) if (!q.empty()) { lv++; nv += q.size(); mx = std::max(mx, q.size()); }
                std::fprintf(stderr, "hylu: %s solve: %zu large supernodes in %zu levels (at most %zu in one)\n",
                             g == 4 ? "forward" : "backward", nv, lv, mx);
            }
        }
    }
    // chains of narrow solve levels (Sec. 2.3): maximal runs of at least
    // kChainMin consecutive levels with at most kChainNodes nodes, each of at
    // most kChainRows rows and without a dense view
    for (int g : {4, 1}) {
        const auto& dl = g == 4 ? h->dsn_l : h->dsn_u;
        const int32_t nlv = L.xlev_ptr[g].size() > 0 ? (int32_t)L.xlev_ptr[g].size() - 1 : 0;
        h->chain_end[g].assign(nlv, -1);
        if (!opt.solve_chain) continue;
        auto ok = [&](int32_t l) {
            const int32_t a = L.xlev_ptr[g][l], b = L.xlev_ptr[g][l + 1];
            if (b - a > kChainNodes || (l < (int32_t)dl.size() && !dl[l].empty())) return false;
            for (int32_t t = a; t < b; t++) {
                const int32_t v = L.xlev_nodes[g][t];
                if (L.m[v] > kChainRows) return false;
                if ((int64_t)L.m[v] * (g == 4 ? L.lw[v] : L.W[v] - L.lw[v]) > kChainWork) return false;
            }
            return true;
        };
        for (int32_t l = 0; l < nlv;) {
            int32_t e = l;
            while (e < nlv && ok(e)) e++;
            if (e - l >= kChainMin) h->chain_end[g][l] = e;
            l = std::max(e, l + 1);
        }
        // HYLU_LOG=2: every solve chain with its factor entries (the L or U
        // part of its nodes' rows)
        if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2)
            for (int32_t l = 0; l < nlv; l++) {
                if (h->chain_end[g][l] <= l) continue;
                int64_t nodes = 0, sum = 0, mx = 0;
                for (int32_t t = L.xlev_ptr[g][l]; t < L.xlev_ptr[g][h->chain_end[g][l]]; t++) {
                    const int32_t v = L.xlev_nodes[g][t];
                    const int64_t e = (int64_t)L.m[v] * (g == 4 ? L.lw[v] : L.W[v] - L.lw[v]);
                    nodes++;
                    sum += e;
                    mx = std::max(mx, e);
                }
                std::fprintf(stderr, "hylu: %s solve chain levels [%d, %d) nodes %lld entries %lld max/node %lld\n",
                             g == 4 ? "L" : "U", l, h->chain_end[g][l], (long long)nodes, (long long)sum, (long long)mx);
            }
    }
    T.chain_lev = chain_lev;
    T.chain_start.assign(nl, -1);
    T.chains.clear();
    T.ctask.clear();
    T.ctask_sthr.clear();
    T.chain_of.assign(L.nnodes, -1);
    T.chain_idx.assign(L.nnodes, -1);
    for (int32_t l = 0; l < nl;) {
        if (!chain_lev[l]) { l++; continue; }
        // whole levels of the run, at most kChainTasksMax nodes per launch
        if (l == 0 || !chain_lev[l - 1]) T.chain_start[l] = (int32_t)T.chains.size();
        LevelTasks::Chain ch{};
        ch.l0 = l;
        ch.t0 = (int64_t)T.ctask.size();
        int32_t maxw = 1;
        auto ntasks = [&](int32_t q) {
            int64_t k = 0;
            for (int32_t v : lvnodes[q]) k += L.m[v] == 1 ? 1 : (L.eptr[v + 1] > L.eptr[v] ? L.m[v] : 0) + 1;
            return k;
        };
        while (l < nl && chain_lev[l] && (int64_t)T.ctask.size() - ch.t0 + ntasks(l) <= kChainTasksMax) {
            for (int32_t v : lvnodes[l]) {
                T.chain_of[v] = (int32_t)T.chains.size();
                // its rows' outside updates (a standalone row: always, for its
                // pivot check), then a supernode's block LU
                if (L.m[v] == 1 || L.eptr[v + 1] > L.eptr[v])
                    for (int32_t r = L.r0[v]; r < L.r0[v] + L.m[v]; r++) {
                        T.ctask.push_back(r);
                        T.ctask_sthr.push_back(T.row_stage[l]);
                    }
                if (L.m[v] > 1) {
                    T.ctask.push_back(-v - 1);
                    T.ctask_sthr.push_back(T.row_stage[l]);
                }
                T.chain_idx[v] = (int32_t)((int64_t)T.ctask.size() - 1 - ch.t0);
                maxw = std::max(maxw, L.W[v]);
            }
            l++;
        }
        if (l == ch.l0) return HYLU_ERR_INTERNAL;     // a level wider than a launch (excluded above)
        ch.l1 = l;
        ch.t1 = (int64_t)T.ctask.size();
        // as many wavefronts as fit with every row of the launch in LDS, at
        // least four (rows wider than their room then work in global memory)
        const int32_t nt = (int32_t)(ch.t1 - ch.t0);
        ch.nw = 0;
        for (int32_t w : {kChainThreads / 64, 6, 4})
            if (chain_lds(h->fp32, nt, w, maxw, kChainSw) <= kLdsMax) { ch.nw = w; ch.cap = maxw; break; }
        if (ch.nw == 0) {
            ch.nw = 4;
            ch.cap = maxw;
            while (ch.cap > 0 && chain_lds(h->fp32, nt, 4, ch.cap, kChainSw) > kLdsMax) ch.cap -= 64;
            ch.cap = std::max(ch.cap, 0);
        }
        T.chains.push_back(ch);
    }
    if (const char* lg = std::getenv("HYLU_LOG"); lg && std::atoi(lg) >= 2)
        for (const LevelTasks::Chain& ch : T.chains)
            std::fprintf(stderr, "hylu: chain launch levels [%d, %d) tasks %lld wavefronts %d row cap %d\n", ch.l0, ch.l1,
                         (long long)(ch.t1 - ch.t0), ch.nw, ch.cap);
    {
        const hylu_status sp = check_chains(h);
        if (sp != HYLU_OK) return sp;
    }
    // algorithmic traffic and flops of every row-kernel and tile launch, from
    // the unit costs of the update kinds (Sec. 2.2) on the exact structure:
    //  row-row (target row i, standalone source k with L(i,k) != 0):
    //      12 u_k + 8 bytes (U(k,:) values and columns, the multiplier), 1 + 2 u_k flops;
    //  sup-row (standalone target row i, source supernode s it has entries in):
    //      8 m_s (m_s + w_s) + 4 w_s + 8 (m_s + w_s) bytes, m_s^2 + 2 m_s w_s flops;
    //  sup-sup (target supernode t, source supernode s one of its rows has entries in):
    //      8 [m_s (m_s + w_s) + 2 m_t (m_s + w_s)] bytes, m_t m_s^2 + 2 m_t m_s w_s flops
    // (m_s rows of the source, w_s its columns past its block).  Padded slots and
    // the dense tail's width are not counted: they are the kernels' choice.
    h->lvl_bytes.assign(nl, 0.0);
    h->lvl_idx.assign(nl, 0.0);
    h->lvl_flops.assign(nl, 0.0);
    h->tile_bytes.assign(nl, 0.0);
    h->tile_idx.assign(nl, 0.0);
    h->tile_flops.assign(nl, 0.0);
    {
        const Symbolic& S = h->sym;
        std::vector<int64_t> mark(L.nnodes, -1), seen(L.nnodes, -1);
        int64_t stamp = 0;
        // units of target node v's rows [ra, rb) over its sources e0..e1
        // by: value entries moved, ix: index bytes, fl: flops
        auto units = [&](int32_t v, int32_t ra, int32_t rb, int64_t e0, int64_t e1, double& by, double& ix,
                         double& fl) {
            const int64_t sm = ++stamp;
            for (int64_t e = e0; e < e1; e++) mark[L.esrc[e]] = sm;
            const bool tsn = nd.is_sn[v] != 0;
            const double mt = L.m[v];
            for (int32_t i = ra; i < rb; i++) {
                const int64_t si = tsn ? sm : ++stamp;      // a supernode target counts (t, s) once
                for (int64_t q = S.lp[i]; q < S.lp[i + 1]; q++)
                    for (int32_t k = S.lint[2 * q]; k <= S.lint[2 * q + 1]; k++) {
                        const int32_t u = nd.of_row[k];
                        if (mark[u] != sm) continue;
                        if (!nd.is_sn[u]) {
                            const double uk = (double)S.ucount[k];
                            by += uk + 1.0;
                            ix += 4.0 * uk;
                            fl += 1.0 + 2.0 * uk;
                        } else if (seen[u] != si) {
                            seen[u] = si;
                            const double ms = L.m[u], ws = L.W[u] - L.lw[u] - L.m[u];
                            if (tsn) {
                                by += ms * (ms + ws) + 2.0 * mt * (ms + ws);
                                fl += mt * ms * ms + 2.0 * mt * ms * ws;
                            } else {
                                by += ms * (ms + ws) + (ms + ws);
                                ix += 4.0 * ws;
                                fl += ms * ms + 2.0 * ms * ws;
                            }
                        }
                    }
            }
        };
        for (int32_t l = 0; l < nl; l++)
            for (int32_t v : lvnodes[l]) {
                if (L.eptr[v + 1] == L.eptr[v]) continue;
                const bool tiled = nd.is_sn[v] && v < L.tail_node0 && L.m[v] >= tile_min;
                double by = 0, ix = 0, fl = 0;
                units(v, L.r0[v], L.r0[v] + L.m[v], L.eptr[v], L.eptr[v + 1], by, ix, fl);
                (tiled ? h->tile_bytes : h->lvl_bytes)[l] += by;
                (tiled ? h->tile_idx : h->lvl_idx)[l] += ix;
                (tiled ? h->tile_flops : h->lvl_flops)[l] += fl;
            }
        // pieces: every row of the node takes the same source range in a level
        for (int32_t l = 0; l < nl; l++) {
            std::map<std::tuple<int32_t, int64_t, int64_t>, std::pair<int32_t, int32_t>> byrange;
            for (const auto& pc : lvpieces[l]) {
                const int32_t v = nd.of_row[pc[0]];
                auto key = std::make_tuple(v, pc[1], pc[2]);
                auto it = byrange.find(key);
                if (it == byrange.end()) byrange[key] = {(int32_t)pc[0], (int32_t)pc[0] + 1};
                else { it->second.first = std::min(it->second.first, (int32_t)pc[0]);
                       it->second.second = std::max(it->second.second, (int32_t)pc[0] + 1); }
            }
            for (const auto& kv : byrange) {
                double by = 0, ix = 0, fl = 0;
                units(std::get<0>(kv.first), kv.second.first, kv.second.second, std::get<1>(kv.first),
                      std::get<2>(kv.first), by, ix, fl);
                h->lvl_bytes[l] += by;
                h->lvl_idx[l] += ix;
                h->lvl_flops[l] += fl;
            }
        }
        // the block LUs (and inverses) that row launches do
        for (int32_t l = 0; l < nl; l++)
            for (int32_t v : lvnodes[l]) {
                if (!h->snfuse[v]) continue;
                const double m = L.m[v], wc = L.W[v] - L.lw[v];
                h->lvl_bytes[l] += 2.0 * m * wc;
                h->lvl_flops[l] += 2.0 * m * m * m / 3.0 + m * m * (wc - m);
                if (h->inv_off[v] >= 0) { h->lvl_bytes[l] += 2.0 * m * m; h->lvl_flops[l] += m * m * m / 3.0; }
            }
        // the block LUs (and inverses) inside the chain launches
        h->chain_snlu_bytes.assign(T.chains.size(), 0.0);
        h->chain_snlu_flops.assign(T.chains.size(), 0.0);
        for (size_t c = 0; c < T.chains.size(); c++)
            for (int64_t t = T.chains[c].t0; t < T.chains[c].t1; t++) {
                if (T.ctask[t] >= 0) continue;
                const int32_t v = -T.ctask[t] - 1;
                const double m = L.m[v], w = L.W[v] - L.lw[v] - L.m[v];
                h->chain_snlu_bytes[c] += 2.0 * m * (m + w);
                h->chain_snlu_flops[c] += 2.0 * m * m * m / 3.0 + m * m * w;
                if (h->inv_off[v] >= 0) { h->chain_snlu_bytes[c] += 2.0 * m * m; h->chain_snlu_flops[c] += m * m * m / 3.0; }
            }
        // the block inverses: read and write the m x m block, m^3 / 3 flops
        h->inv_bytes.assign(nl, 0.0);
        h->inv_flops.assign(nl, 0.0);
        for (int32_t l = 0; l < nl; l++)
            for (int64_t q = h->inv_ptr[l]; q < h->inv_ptr[l + 1]; q++) {
                const double m = L.m[h->inv_nodes[q]];
                h->inv_bytes[l] += 2.0 * m * m;
                h->inv_flops[l] += m * m * m / 3.0;
            }
        // one right-hand side through the solves: 2 flops and one value per
        // exact factor entry, plus a 4-byte column index in standalone rows
        // (supernode rows share their column list)
        h->solve_units.fill(0.0);
        for (int32_t i = 0; i < n; i++) {
            double nl_i = 0;
            for (int64_t q = S.lp[i]; q < S.lp[i + 1]; q++) nl_i += S.lint[2 * q + 1] - S.lint[2 * q] + 1;
            const double nu_i = (double)S.ucount[i] + 1.0;
            const double sa = nd.is_sn[nd.of_row[i]] ? 0.0 : 1.0;
            if (i >= L.t0 && L.mT > 0) {
                h->solve_units[4] += nl_i + nu_i;
                h->solve_units[5] += sa * (nl_i + nu_i);
            } else {
                h->solve_units[0] += nl_i;
                h->solve_units[1] += sa * nl_i;
                h->solve_units[2] += nu_i;
                h->solve_units[3] += sa * nu_i;
            }
        }
    }
    plog("tasks");
    h->analyzed = true;
    return HYLU_OK;
}

// the matrix of the FP64 residual: A itself, or A^T through its column copy
// (the values of the last (re)factorisation gathered into column order)
hylu_status residual_operator(hylu_handle h, int32_t transpose, hipStream_t st, const double*& av,
                              const int64_t*& rp, const int32_t*& ci)
{
    av = h->d_aval; rp = h->d_arp; ci = h->d_aci;
    if (transpose) {
        HIPCHK(launch_gather_values(h->nnz, h->d_atq, h->d_aval, h->d_atv, st));
        av = h->d_atv; rp = h->d_atp; ci = h->d_atc;
    }
    return HYLU_OK;
}

// r = b - op(A) x in FP64, then on the host the normwise backward error
// ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) (largest over the right-hand
// sides and the members of a batch) and the accuracy measure of Sec. 3.3,
// ||r||_1 / ||b||_1 (largest likewise).  Synchronises the stream.
hylu_status measure_residual(hylu_handle h, const SolveWs& w, const int64_t* rp, const int32_t* ci, const double* av,
                             const double* b, int64_t ldb, const double* x, int64_t ldx, int32_t nrhs, hipStream_t st,
                             double& eta, double& res1)
{
    const int32_t n = h->n;
    const int32_t nseg = (int32_t)h->member_row_off.size() - 1;
    HIPCHK(launch_residual(n, nrhs, rp, ci, av, b, ldb, x, ldx, w.r, st));
    HIPCHK(launch_norms(n, nrhs, rp, av, w.r, x, ldx, b, ldb, h->d_seg, nseg, w.norms, st));
    HIPCHK(hipMemcpyAsync(w.h_norms, w.norms, sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * nseg,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    eta = 0.0;
    res1 = 0.0;
    for (int32_t sg = 0; sg < nseg; sg++) {
        const double anorm = w.h_norms[kNormSlots * ((size_t)nrhs * nseg + sg)];
        for (int32_t k = 0; k < nrhs; k++) {
            const double* q = w.h_norms + kNormSlots * ((size_t)k * nseg + sg);
            const double den = anorm * q[1] + q[2];
            eta = std::max(eta, den > 0 ? q[0] / den : (q[0] > 0 ? std::numeric_limits<double>::infinity() : 0.0));
            res1 = std::max(res1, q[4] > 0 ? q[3] / q[4] : (q[3] > 0 ? std::numeric_limits<double>::infinity() : 0.0));
        }
    }
    return HYLU_OK;
}

// forward-backward substitution with refinement on work vectors w; the base
// solve replays a cached graph (graphs = true) or is enqueued directly
hylu_status solve_impl(hylu_handle h, const SolveWs& w, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                       int32_t transpose, hipStream_t st, bool graphs)
{
    const int32_t n = h->n;
    // does refinement run?  (perturbed pivots, or FP32 factors).  After a
    // refactorisation the count of perturbed pivots is read only once the
    // base solve is queued behind it, so the device goes from one to the
    // other without waiting for the host
    const bool pert_pending = !h->pert_known;
    bool refine = h->fp32 || (!pert_pending && h->last_pert > 0);
    // b is needed after x is written when refining in place (or when that is
    // not known yet)
    const double* b = d_b;
    bool bcopy = (refine || pert_pending) && d_b == d_x;
    if (bcopy) {
        HIPCHK(hipMemcpy2DAsync(w.bc, sizeof(double) * (size_t)n, d_b, sizeof(double) * ld, sizeof(double) * (size_t)n,
                                nrhs, hipMemcpyDeviceToDevice, st));
        b = w.bc;
    }
    int64_t ldb = bcopy ? n : ld;
    hylu_status s;
    if (graphs) {
        auto key = std::make_tuple(b, d_x, nrhs, ld, transpose);
        if (h->solve_graphs.find(key) == h->solve_graphs.end()) trim_graphs(h->solve_graphs);
        auto it = h->solve_graphs.find(key);
        bool fresh = it == h->solve_graphs.end();
        GraphEntry& g = h->solve_graphs[key];
        s = run_graph(h, g, fresh, st, [&](hipStream_t cs) { return enqueue_solve(h, w, b, ldb, d_x, ld, nrhs, transpose, 0, cs); });
        if (s != HYLU_OK) { if (fresh) h->solve_graphs.erase(key); return s; }
    } else {
        s = enqueue_solve(h, w, b, ldb, d_x, ld, nrhs, transpose, 0, st);
        if (s != HYLU_OK) return s;
    }
    if (pert_pending) {
        HIPCHK(hipEventSynchronize(h->fact_done));
        h->last_pert = h->h_pert[0];
        h->pert_known = true;
        if (h->h_pert[1]) { h->sticky_error = true; return HYLU_ERR_DEVICE; }
        refine = h->fp32 || h->last_pert > 0;
    }
    h->ir_iters = 0;
    h->berr = h->resid1 = 0.0;
    h->berr_known = false;
    if (!refine) return HYLU_OK;
    // FP64 iterative refinement on the original matrix (Sec. 2.3); the
    // returned x is the iterate with the smallest backward error
    const double* av = nullptr;
    const int64_t* rp = nullptr;
    const int32_t* ci = nullptr;
    s = residual_operator(h, transpose, st, av, rp, ci);
    if (s != HYLU_OK) return s;
    int32_t maxit = h->opt.ir_maxit > 0 ? h->opt.ir_maxit : (h->fp32 ? 30 : 10);
    double tol = h->opt.ir_tol > 0 ? h->opt.ir_tol : 1e-12;
    double eta_prev = std::numeric_limits<double>::infinity();
    double best = std::numeric_limits<double>::infinity(), best_res1 = 0.0;
    double eta = 0.0, res1 = 0.0;
    const size_t colb = sizeof(double) * (size_t)n;
    for (int32_t it2 = 0;; it2++) {
        s = measure_residual(h, w, rp, ci, av, b, ldb, d_x, ld, nrhs, st, eta, res1);
        if (s != HYLU_OK) return s;
        const bool improved = eta < best;
        if (improved) { best = eta; best_res1 = res1; }
        if (eta <= tol || it2 >= maxit || eta > eta_prev / 2) {
            // a correction that did not improve on the saved iterate is undone
            if (!improved)
                HIPCHK(hipMemcpy2DAsync(d_x, sizeof(double) * ld, w.xbest, colb, colb, nrhs,
                                        hipMemcpyDeviceToDevice, st));
            break;
        }
        HIPCHK(hipMemcpy2DAsync(w.xbest, colb, d_x, sizeof(double) * ld, colb, nrhs, hipMemcpyDeviceToDevice, st));
        eta_prev = eta;
        s = enqueue_solve(h, w, w.r, n, d_x, ld, nrhs, transpose, 1, st);
        if (s != HYLU_OK) return s;
        h->ir_iters++;
    }
    h->berr = best;
    h->resid1 = best_res1;
    h->berr_known = true;
    return best <= tol ? HYLU_OK : HYLU_WARN_IR_NOT_CONVERGED;
}

}  // namespace

extern "C" {

hylu_status hylu_default_options(hylu_options* o)
{
    if (!o) return HYLU_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    o->ordering = 0;
    o->user_perm = nullptr;
    o->static_pivot = 1;
    o->precision = 0;
    o->pivot_tau = 0.0;
    o->ir_tol = 1e-12;
    o->ir_maxit = 0;
    o->sn_min = 2;
    o->sn_max = 1 << 30;
    o->kernel_mode = 0;
    o->repeated = 1;
    o->nd_leaf = 256;
    o->amd_dense = 0.0;
    o->dense_tail = 0.5;
    o->tail_min = 64;
    o->tail_max = 32768;
    o->sn_dense = 64;
    o->sn_tile = 0;
    o->sn_inverse = 1;
    o->tail_sparse = 1;
    o->side_rows = 1;
    o->pipeline_rows = 0;
    o->solve_chain = 1;
    o->gpu_symbolic = 0;
    o->pipeline_spin = 0;
    o->solve_split = 1;
    o->group_min_rows = kGroupMinRows;
    o->group_tail_rows = kGroupTailRows;
    return HYLU_OK;
}

const char* hylu_status_string(hylu_status s)
{
    switch (s) {
    case HYLU_OK: return "ok";
    case HYLU_ERR_ARG: return "invalid argument";
    case HYLU_ERR_CSR: return "invalid CSR structure";
    case HYLU_ERR_STRUCT_SINGULAR: return "structurally singular matrix";
    case HYLU_ERR_NOT_ANALYZED: return "not analyzed";
    case HYLU_ERR_NOT_FACTORIZED: return "not factorized";
    case HYLU_ERR_OOM: return "out of memory";
    case HYLU_ERR_DEVICE: return "device error";
    case HYLU_ERR_NONFINITE: return "non-finite value";
    case HYLU_ERR_INTERNAL: return "internal error";
    case HYLU_ERR_SCRATCH: return "problem larger than the fixed scratch of hylu_solve_noalloc";
    case HYLU_WARN_IR_NOT_CONVERGED: return "refinement did not reach the tolerance";
    }
    return "unknown status";
}

hylu_status hylu_create(hylu_handle* out, const hylu_allocator* alloc)
{
    if (!out) return HYLU_ERR_ARG;
    *out = nullptr;
    hylu_handle h = new (std::nothrow) hylu_handle_s();
    if (!h) return HYLU_ERR_OOM;
    if (alloc) {
        if (!alloc->alloc || !alloc->free) { delete h; return HYLU_ERR_ARG; }
        h->alloc = *alloc;
        h->has_alloc = true;
    }
    hylu_default_options(&h->opt);
    *out = h;
    return HYLU_OK;
}

hylu_status hylu_destroy(hylu_handle h)
{
    if (!h) return HYLU_ERR_ARG;
    free_device(h);
    for (hipEvent_t e : h->prof.pool) hipEventDestroy(e);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    if (h->fact_done) hipEventDestroy(h->fact_done);
    if (h->h_pert) hipHostFree(h->h_pert);
    if (h->ws.h_norms) hipHostFree(h->ws.h_norms);
    if (h->h_norms_fixed) hipHostFree(h->h_norms_fixed);
    for (int j = 0; j < hylu_handle_s::kSide; j++) {
        if (h->side[j]) hipStreamDestroy(h->side[j]);
        if (h->ev_join[j]) hipEventDestroy(h->ev_join[j]);
    }
    if (h->ev_fork) hipEventDestroy(h->ev_fork);
    delete h;
    return HYLU_OK;
}

hylu_status hylu_analyze(hylu_handle h, int32_t n, const int64_t* row_ptr, const int32_t* col,
                         const double* val, const hylu_options* opt_in)
{
    if (!h || n <= 0 || !row_ptr || !col || !val) return HYLU_ERR_ARG;
    hylu_options opt;
    if (opt_in) opt = *opt_in; else hylu_default_options(&opt);
    if (opt.ordering < 0 || opt.ordering > 4 || (opt.ordering == 3 && !opt.user_perm)) return HYLU_ERR_ARG;
    if (opt.precision < 0 || opt.precision > 1 || opt.kernel_mode < 0 || opt.kernel_mode > 2) return HYLU_ERR_ARG;
    if (opt.pipeline_rows < 0 || opt.gpu_symbolic < 0 || opt.gpu_symbolic > 1) return HYLU_ERR_ARG;
    hylu_status st = validate_csr(n, row_ptr, col, val);
    if (st != HYLU_OK) return st;
    try {
        free_device(h);
        h->analyzed = h->factorized = h->uploaded = false;
        h->sticky_error = false;
        h->pert_known = false;
        h->opt = opt;
        h->n = n;
        h->nnz = row_ptr[n];
        h->fp32 = opt.precision == 1;
        PhaseLog plog;
        Csr& A = h->A;
        A.n = n;
        A.rp.assign(row_ptr, row_ptr + n + 1);
        A.ci.assign(col, col + h->nnz);
        A.v.assign(val, val + h->nnz);
        h->member_row_off = {0, (int64_t)n};
        h->member_nnz_off = {0, h->nnz};
        {
            hylu_status so = order_matrix(A, opt, h->perm_r, h->perm_c, h->dr, h->dc);
            if (so != HYLU_OK) return so;
        }
        plog("matching and ordering");
        hylu_status s2 = analyze_structure(h, plog);
        if (s2 != HYLU_OK) return s2;
    } catch (const std::bad_alloc&) {
        return HYLU_ERR_OOM;
    } catch (...) {
        return HYLU_ERR_INTERNAL;
    }
    return HYLU_OK;
}

hylu_status hylu_analyze_batch(hylu_handle h, int32_t count, const int32_t* n_k, const int64_t* const* row_ptr_k,
                               const int32_t* const* col_k, const double* const* val_k, const hylu_options* opt_in)
{
    if (!h || count <= 0 || !n_k || !row_ptr_k || !col_k || !val_k) return HYLU_ERR_ARG;
    hylu_options opt;
    if (opt_in) opt = *opt_in; else hylu_default_options(&opt);
    if (opt.ordering < 0 || opt.ordering > 4 || opt.ordering == 3) return HYLU_ERR_ARG;   // no user permutation for a batch
    if (opt.precision < 0 || opt.precision > 1 || opt.kernel_mode < 0 || opt.kernel_mode > 2) return HYLU_ERR_ARG;
    if (opt.pipeline_rows < 0 || opt.gpu_symbolic < 0 || opt.gpu_symbolic > 1) return HYLU_ERR_ARG;
    opt.dense_tail = 0.0;   // members are independent: the levels of all of them share the launches instead
    int64_t ntot = 0, nnztot = 0;
    for (int32_t k = 0; k < count; k++) {
        if (n_k[k] <= 0 || !row_ptr_k[k] || !col_k[k] || !val_k[k]) return HYLU_ERR_ARG;
        hylu_status st = validate_csr(n_k[k], row_ptr_k[k], col_k[k], val_k[k]);
        if (st != HYLU_OK) return st;
        ntot += n_k[k];
        nnztot += row_ptr_k[k][n_k[k]];
    }
    if (ntot > std::numeric_limits<int32_t>::max()) return HYLU_ERR_ARG;
    try {
        free_device(h);
        h->analyzed = h->factorized = h->uploaded = false;
        h->sticky_error = false;
        h->pert_known = false;
        h->opt = opt;
        h->n = (int32_t)ntot;
        h->nnz = nnztot;
        h->fp32 = opt.precision == 1;
        PhaseLog plog;
        h->member_row_off.assign(count + 1, 0);
        h->member_nnz_off.assign(count + 1, 0);
        for (int32_t k = 0; k < count; k++) {
            h->member_row_off[k + 1] = h->member_row_off[k] + n_k[k];
            h->member_nnz_off[k + 1] = h->member_nnz_off[k] + row_ptr_k[k][n_k[k]];
        }
        // the block-diagonal union
        Csr& A = h->A;
        A.n = (int32_t)ntot;
        A.rp.assign(ntot + 1, 0);
        A.ci.resize(nnztot);
        A.v.resize(nnztot);
        for (int32_t k = 0; k < count; k++) {
            const int64_t r0 = h->member_row_off[k], q0 = h->member_nnz_off[k];
            for (int32_t i = 0; i < n_k[k]; i++) A.rp[r0 + i + 1] = q0 + row_ptr_k[k][i + 1];
            for (int64_t p = 0; p < row_ptr_k[k][n_k[k]]; p++) {
                A.ci[q0 + p] = (int32_t)(col_k[k][p] + r0);
                A.v[q0 + p] = val_k[k][p];
            }
        }
        // every member matched, scaled and ordered on its own, on host threads
        h->perm_r.assign(ntot, 0);
        h->perm_c.assign(ntot, 0);
        h->dr.assign(ntot, 1.0);
        h->dc.assign(ntot, 1.0);
        std::vector<hylu_status> res(count, HYLU_OK);
        std::atomic<int32_t> next{0};
        auto worker = [&]() {
            for (;;) {
                const int32_t k = next.fetch_add(1);
                if (k >= count) return;
                try {
                    Csr M;
                    M.n = n_k[k];
                    M.rp.assign(row_ptr_k[k], row_ptr_k[k] + n_k[k] + 1);
                    M.ci.assign(col_k[k], col_k[k] + M.rp[M.n]);
                    M.v.assign(val_k[k], val_k[k] + M.rp[M.n]);
                    std::vector<int32_t> pr, pc;
                    std::vector<double> dr, dc;
                    res[k] = order_matrix(M, opt, pr, pc, dr, dc);
                    if (res[k] != HYLU_OK) continue;
                    const int64_t r0 = h->member_row_off[k];
                    for (int32_t i = 0; i < M.n; i++) {
                        h->perm_r[r0 + i] = (int32_t)(pr[i] + r0);
                        h->perm_c[r0 + i] = (int32_t)(pc[i] + r0);
                        h->dr[r0 + i] = dr[i];
                        h->dc[r0 + i] = dc[i];
                    }
                } catch (const std::bad_alloc&) {
                    res[k] = HYLU_ERR_OOM;
                } catch (...) {
                    res[k] = HYLU_ERR_INTERNAL;
                }
            }
        };
        unsigned nth = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
        nth = std::min<unsigned>(nth, (unsigned)count);
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nth; t++) pool.emplace_back(worker);
        worker();
        for (auto& t : pool) t.join();
        for (int32_t k = 0; k < count; k++) if (res[k] != HYLU_OK) return res[k];
        plog("matching and ordering (members)");
        hylu_status s2 = analyze_structure(h, plog);
        if (s2 != HYLU_OK) return s2;
    } catch (const std::bad_alloc&) {
        return HYLU_ERR_OOM;
    } catch (...) {
        return HYLU_ERR_INTERNAL;
    }
    return HYLU_OK;
}

hylu_status hylu_batch_offsets(hylu_handle h, int32_t* count, int64_t* row_off, int64_t* nnz_off)
{
    if (!h || !count) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    *count = (int32_t)h->member_row_off.size() - 1;
    if (row_off) std::memcpy(row_off, h->member_row_off.data(), sizeof(int64_t) * h->member_row_off.size());
    if (nnz_off) std::memcpy(nnz_off, h->member_nnz_off.data(), sizeof(int64_t) * h->member_nnz_off.size());
    return HYLU_OK;
}

hylu_status hylu_factorize(hylu_handle h, const double* d_val, void* stream)
{
    (void)hipGetLastError();   // an error another library left on this thread is not ours
    if (!h || !d_val) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    if (!h->uploaded) {
        hylu_status su = upload_device(h);
        if (su != HYLU_OK) { free_device(h); return su; }
    }
    HIPCHK(launch_init_pivots(h->D, st));
    hylu_status s = enqueue_factor(h, d_val, true, st);
    if (s != HYLU_OK) return s;
    HIPCHK(hipMemcpyAsync(h->h_pert, h->d_pert, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->fact_done, st));
    h->pert_known = false;
    h->factorized = true;
    return HYLU_OK;
}

hylu_status hylu_refactor(hylu_handle h, const double* d_val, void* stream)
{
    (void)hipGetLastError();   // an error another library left on this thread is not ours
    if (!h || !d_val) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    if (h->refac_graphs.find(d_val) == h->refac_graphs.end()) trim_graphs(h->refac_graphs);
    auto it = h->refac_graphs.find(d_val);
    bool fresh = it == h->refac_graphs.end();
    GraphEntry& g = h->refac_graphs[d_val];
    hylu_status s = run_graph(h, g, fresh, st, [&](hipStream_t cs) { return enqueue_factor(h, d_val, false, cs); });
    if (s != HYLU_OK) { if (fresh) h->refac_graphs.erase(d_val); return s; }
    HIPCHK(hipMemcpyAsync(h->h_pert, h->d_pert, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->fact_done, st));
    h->pert_known = false;
    return HYLU_OK;
}

hylu_status hylu_solve(hylu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld, int32_t transpose,
                       void* stream)
{
    (void)hipGetLastError();
    if (!h || !d_b || !d_x || nrhs <= 0) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    if (ld < h->n) return HYLU_ERR_ARG;
    hylu_status s = ensure_workspace(h, nrhs);
    if (s != HYLU_OK) return s;
    if (transpose) { s = ensure_tlists(h); if (s != HYLU_OK) return s; }
    return solve_impl(h, h->ws, d_b, d_x, nrhs, ld, transpose, (hipStream_t)stream, true);
}

hylu_status hylu_solve_noalloc(hylu_handle h, const double* d_b, double* d_x, int32_t nrhs, int64_t ld,
                               int32_t transpose, void* stream)
{
    (void)hipGetLastError();
    if (!h || !d_b || !d_x || nrhs <= 0) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    if (ld < h->n) return HYLU_ERR_ARG;
    // the transposed solve's column lists are handle memory built on first use
    if (transpose && !h->tlists) return HYLU_ERR_ARG;
    const int32_t nseg = (int32_t)h->member_row_off.size() - 1;
    if (nrhs > kNoallocRhs || noalloc_bytes(h, nrhs) > kScratchBytes) {
        std::fprintf(stderr, "hylu: hylu_solve_noalloc: n = %d with %d right-hand sides needs %zu bytes of scratch, "
                             "more than its fixed %zu (or more than %d right-hand sides)\n",
                     h->n, nrhs, noalloc_bytes(h, nrhs), kScratchBytes, kNoallocRhs);
        return HYLU_ERR_SCRATCH;
    }
    void* base = scratch_ptr(h->device);
    if (!base || !h->h_norms_fixed) return HYLU_ERR_DEVICE;      // set up by the first (re)factorisation
    // carve the work vectors out of this device's scratch
    SolveWs w;
    const size_t es = h->fp32 ? sizeof(float) : sizeof(double);
    const size_t nn = (size_t)h->n * nrhs;
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) { void* q = p; p += (bytes + 255) & ~size_t(255); return q; };
    w.y = take(es * nn);
    w.z = take(es * nn);
    w.r = static_cast<double*>(take(sizeof(double) * nn));
    w.bc = static_cast<double*>(take(sizeof(double) * nn));
    w.xbest = static_cast<double*>(take(sizeof(double) * nn));
    w.norms = static_cast<double*>(take(sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * nseg));
    w.h_norms = h->h_norms_fixed;
    return solve_impl(h, w, d_b, d_x, nrhs, ld, transpose, (hipStream_t)stream, false);
}

hylu_status hylu_residual(hylu_handle h, const double* d_b, const double* d_x, int32_t nrhs, int64_t ld,
                          int32_t transpose, void* stream, double* berr, double* resid1)
{
    (void)hipGetLastError();
    if (!h || !d_b || !d_x || nrhs <= 0) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    if (ld < h->n) return HYLU_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    hylu_status s = ensure_workspace(h, nrhs);
    if (s != HYLU_OK) return s;
    if (transpose) { s = ensure_tlists(h); if (s != HYLU_OK) return s; }
    const double* av = nullptr;
    const int64_t* rp = nullptr;
    const int32_t* ci = nullptr;
    s = residual_operator(h, transpose, st, av, rp, ci);
    if (s != HYLU_OK) return s;
    double eta = 0.0, res1 = 0.0;
    s = measure_residual(h, h->ws, rp, ci, av, d_b, ld, d_x, ld, nrhs, st, eta, res1);
    if (s != HYLU_OK) return s;
    h->berr = eta;
    h->resid1 = res1;
    h->berr_known = true;
    if (berr) *berr = eta;
    if (resid1) *resid1 = res1;
    return HYLU_OK;
}

hylu_status hylu_grad_values(hylu_handle h, const double* d_lambda, const double* d_x, int32_t nrhs, int64_t ld,
                             double* d_gval, void* stream)
{
    if (!h || !d_lambda || !d_x || !d_gval || nrhs <= 0) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    if (ld < h->n) return HYLU_ERR_ARG;
    HIPCHK(launch_grad(h->n, nrhs, ld, h->d_arp, h->d_aci, d_lambda, d_x, d_gval, (hipStream_t)stream));
    return HYLU_OK;
}

hylu_status hylu_get_info(hylu_handle h, hylu_info* o)
{
    if (!h || !o) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    std::memset(o, 0, sizeof(*o));
    o->n = h->n;
    o->nnz_a = h->nnz;
    o->nnz_l = h->sym.nnz_l;
    o->nnz_u = h->sym.nnz_u;
    o->flops = h->sym.flops;
    o->flops_padded = h->nodes.flops_padded;
    o->factor_entries = h->lay.nvals;
    o->n_nodes = h->nodes.count;
    for (int32_t v = 0; v < h->nodes.count; v++)
        if (h->nodes.is_sn[v]) {
            int32_t m = h->nodes.ptr[v + 1] - h->nodes.ptr[v];
            o->n_supernodes++;
            o->rows_in_supernodes += m;
            o->max_supernode = std::max(o->max_supernode, m);
        }
    for (int t = 0; t < 4; t++) o->n_levels[t] = h->nodes.nlevels[t];
    if (h->factorized) {
        if (!h->pert_known) {
            if (hipEventSynchronize(h->fact_done) != hipSuccess) return HYLU_ERR_DEVICE;
            h->last_pert = h->h_pert[0];
            h->pert_known = true;
            if (h->h_pert[1]) { h->sticky_error = true; return HYLU_ERR_DEVICE; }
        }
        o->n_perturbed = h->last_pert;
    }
    o->ir_iters = h->ir_iters;
    o->berr = h->berr_known ? h->berr : -1.0;
    o->resid_1 = h->berr_known ? h->resid1 : -1.0;
    o->n_dense_sn = (int32_t)h->dsn.size();
    for (int g : {4, 1})
        for (size_t l = 0; l < h->chain_end[g].size(); l++)
            if (h->chain_end[g][l] > (int32_t)l) o->chain_levels += h->chain_end[g][l] - (int32_t)l;
    o->split_sn = (int32_t)(h->sl[0].sp_nodes.size() + h->sl[1].sp_nodes.size() + h->tl[0].sp_nodes.size() +
                            h->tl[1].sp_nodes.size());
    o->pipe_tasks = (int32_t)h->ft.ctask.size();
    o->sn_groups = h->sn_groups;
    o->tail_groups = h->tail_groups;
    o->sym_ms = h->sym_ms;
    o->sym_kernel_ms = h->sym_kernel_ms;
    o->sym_hash = h->sym_hash;
    o->pivot_tau = h->tau;
    o->tail_rows = h->lay.mT;
    o->tail_panels = (int32_t)h->lay.panels.size();
    // the dense tail counts with the products its block-sparse plan issues
    const double mT = h->lay.mT;
    o->flops_issued = h->lay.flops_kernel - (uint64_t)(2.0 * mT * mT * mT / 3.0) + (uint64_t)h->tail_flops;
    return HYLU_OK;
}

hylu_status hylu_export_symbolic(hylu_handle h, const hylu_symbolic_view* v)
{
    if (!h || !v) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    const int32_t n = h->n, nn = h->nodes.count;
    if (v->perm_r) std::memcpy(v->perm_r, h->perm_r.data(), sizeof(int32_t) * n);
    if (v->perm_c) std::memcpy(v->perm_c, h->perm_c.data(), sizeof(int32_t) * n);
    if (v->dr) std::memcpy(v->dr, h->dr.data(), sizeof(double) * n);
    if (v->dc) std::memcpy(v->dc, h->dc.data(), sizeof(double) * n);
    if (v->node_ptr) std::memcpy(v->node_ptr, h->nodes.ptr.data(), sizeof(int32_t) * (nn + 1));
    if (v->is_sn) std::memcpy(v->is_sn, h->nodes.is_sn.data(), nn);
    if (v->levels)
        for (int t = 0; t < 4; t++) std::memcpy(v->levels + (size_t)t * nn, h->nodes.level[t].data(), sizeof(int32_t) * nn);
    return HYLU_OK;
}

hylu_status hylu_autotune(hylu_handle h, const double* d_val, void* stream, int32_t reps, double* ms_default,
                          double* ms_tuned)
{
    (void)hipGetLastError();
    if (!h || !d_val) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    LevelTasks& T = h->ft;
    const int32_t nl = (int32_t)T.maxW.size();
    constexpr int kTrials = 4;
    static const int32_t kRowNT[kTrials] = {64, 128, 256, 1024};
    static const int32_t kSnNT[kTrials] = {64, 256, 256, 256};
    // best[l][t]: shortest time of level l's row launch (snlu launch) under trial t
    std::vector<std::array<double, kTrials>> trow(nl), tsn(nl);
    for (auto& a : trow) a.fill(std::numeric_limits<double>::infinity());
    for (auto& a : tsn) a.fill(std::numeric_limits<double>::infinity());
    // the levels with a row launch (not the chain launches of pipeline mode)
    std::vector<int32_t> row_levels, sn_levels;
    for (int32_t l = 0; l < nl; l++)
        if (T.chain_lev.empty() || !T.chain_lev[l]) {
            row_levels.push_back(l);
            if (T.sn_ptr[l + 1] > T.sn_ptr[l]) sn_levels.push_back(l);
        }
    reps = std::max(reps, 1);
    hylu_status s = HYLU_OK;
    for (int32_t rep = 0; rep < reps && s == HYLU_OK; rep++)
        for (int t = 0; t < kTrials && s == HYLU_OK; t++) {
            T.tune_rows = kRowNT[t];
            T.tune_sn = kSnNT[t];
            h->prof.on = true;
            h->prof.recs.clear();
            h->prof.used = 0;
            s = enqueue_factor(h, d_val, false, st);
            h->prof.on = false;
            if (s != HYLU_OK) break;
            if (hipStreamSynchronize(st) != hipSuccess) { s = HYLU_ERR_DEVICE; break; }
            // one row launch per level and one supernode-LU launch per level
            // that has small supernodes, in level order
            int32_t lr = 0;
            size_t ls = 0;
            for (const Profiler::Rec& r : h->prof.recs) {
                if (r.cls == C_ROWS) lr++;
                else if (r.cls == C_SNLU) ls++;
            }
            if ((size_t)lr != row_levels.size() || ls != sn_levels.size()) { s = HYLU_ERR_INTERNAL; break; }
            lr = 0;
            ls = 0;
            for (const Profiler::Rec& r : h->prof.recs) {
                float ms = 0.f;
                if (r.cls != C_ROWS && r.cls != C_SNLU) continue;
                if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) { s = HYLU_ERR_DEVICE; break; }
                if (r.cls == C_ROWS) { trow[row_levels[lr]][t] = std::min(trow[row_levels[lr]][t], (double)ms); lr++; }
                else { tsn[sn_levels[ls]][t] = std::min(tsn[sn_levels[ls]][t], (double)ms); ls++; }
            }
        }
    T.tune_rows = T.tune_sn = 0;
    if (s != HYLU_OK) { h->sticky_error = true; return s; }
    double before = 0.0, after = 0.0;
    for (int32_t l : row_levels) {
        // the built-in shape: 1024 threads for long rows of narrow levels, 256
        // for other long rows, 64 otherwise
        const bool narrow = T.row_ptr[l + 1] - T.row_ptr[l] <= kSideNarrowRows;
        const int def = T.maxW[l] > 1024 ? (narrow ? 3 : 2) : 0;
        int best = 0;
        for (int t = 1; t < kTrials; t++) if (trow[l][t] < trow[l][best]) best = t;
        T.row_nt[l] = kRowNT[best];
        before += trow[l][def];
        after += trow[l][best];
        if (T.sn_ptr[l + 1] > T.sn_ptr[l]) {
            const double t256 = std::min(std::min(tsn[l][1], tsn[l][2]), tsn[l][3]);
            const int sb = tsn[l][0] < t256 ? 0 : 1;
            T.sn_nt[l] = kSnNT[sb];
            before += t256;
            after += sb ? t256 : tsn[l][0];
        }
    }
    // graphs captured with the old choices are stale
    for (auto& kv : h->refac_graphs) { hipGraphExecDestroy(kv.second.exec); hipGraphDestroy(kv.second.graph); }
    h->refac_graphs.clear();
    if (ms_default) *ms_default = before;
    if (ms_tuned) *ms_tuned = after;
    // every trial was a complete refactorisation of d_val with identical results
    h->pert_known = false;
    HIPCHK(hipMemcpyAsync(h->h_pert, h->d_pert, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->fact_done, st));
    return HYLU_OK;
}

hylu_status hylu_profile(hylu_handle h, const double* d_val, const double* d_b, double* d_x, void* stream,
                         hylu_kernel_stats* stats, int32_t max_classes, int32_t* count)
{
    (void)hipGetLastError();
    if (!h || !d_val || !d_b || !d_x || !stats || !count || max_classes <= 0) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    if (h->sticky_error) return HYLU_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    hylu_status s = ensure_workspace(h, 1);
    if (s != HYLU_OK) return s;
    h->prof.on = true;
    h->prof.recs.clear();
    h->prof.used = 0;
    s = enqueue_factor(h, d_val, false, st);
    if (s == HYLU_OK) s = enqueue_solve(h, h->ws, d_b, h->n, d_x, h->n, 1, 0, 0, st);
    h->prof.on = false;
    if (s != HYLU_OK) return s;
    HIPCHK(hipStreamSynchronize(st));
    std::vector<hylu_kernel_stats> acc(C_N);
    for (int c = 0; c < C_N; c++) { std::memset(&acc[c], 0, sizeof(acc[c])); std::snprintf(acc[c].name, 32, "%s", kClassNames[c]); }
    for (const Profiler::Rec& r : h->prof.recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        acc[r.cls].launches++;
        acc[r.cls].ms += ms;
        acc[r.cls].bytes += r.bytes;
        acc[r.cls].flops += r.flops;
    }
    // the solve classes take the exact entries they consume (one right-hand side)
    const double es = h->fp32 ? 4.0 : 8.0;
    const int scls[3] = {C_LSOLVE, C_USOLVE, C_TSOLVE};
    for (int q = 0; q < 3; q++)
        if (acc[scls[q]].launches) {
            acc[scls[q]].bytes = es * h->solve_units[2 * q] + 4.0 * h->solve_units[2 * q + 1];
            acc[scls[q]].flops = 2.0 * h->solve_units[2 * q];
        }
    int32_t k = 0;
    for (int c = 0; c < C_N && k < max_classes; c++)
        if (acc[c].launches > 0) stats[k++] = acc[c];
    *count = k;
    h->pert_known = false;
    HIPCHK(hipMemcpyAsync(h->h_pert, h->d_pert, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->fact_done, st));
    return HYLU_OK;
}

hylu_status hylu_export_sizes(hylu_handle h, int64_t* ncols_total)
{
    if (!h || !ncols_total) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    *ncols_total = (int64_t)h->lay.cols.size();
    return HYLU_OK;
}

hylu_status hylu_export_factors(hylu_handle h, double* vals, int64_t* node_voff, int32_t* node_lw, int32_t* node_W,
                                int64_t* node_coff, int32_t* cols, int32_t* piv)
{
    if (!h) return HYLU_ERR_ARG;
    if (!h->analyzed) return HYLU_ERR_NOT_ANALYZED;
    if (!h->factorized) return HYLU_ERR_NOT_FACTORIZED;
    const Layout& L = h->lay;
    if (hipDeviceSynchronize() != hipSuccess) return HYLU_ERR_DEVICE;
    if (vals) {
        if (h->fp32) {
            std::vector<float> tmp(L.nvals);
            if (hipMemcpy(tmp.data(), h->vals, sizeof(float) * L.nvals, hipMemcpyDeviceToHost) != hipSuccess) return HYLU_ERR_DEVICE;
            for (int64_t i = 0; i < L.nvals; i++) vals[i] = tmp[i];
        } else if (hipMemcpy(vals, h->vals, sizeof(double) * L.nvals, hipMemcpyDeviceToHost) != hipSuccess) {
            return HYLU_ERR_DEVICE;
        }
    }
    if (node_voff) std::memcpy(node_voff, L.voff.data(), sizeof(int64_t) * (L.nnodes + 1));
    if (node_lw) std::memcpy(node_lw, L.lw.data(), sizeof(int32_t) * L.nnodes);
    if (node_W) std::memcpy(node_W, L.W.data(), sizeof(int32_t) * L.nnodes);
    if (node_coff) std::memcpy(node_coff, L.coff.data(), sizeof(int64_t) * (L.nnodes + 1));
    if (cols) std::memcpy(cols, L.cols.data(), sizeof(int32_t) * L.cols.size());
    if (piv) {
        std::vector<int32_t> pl(h->n);
        if (hipMemcpy(pl.data(), h->D.pl, sizeof(int32_t) * h->n, hipMemcpyDeviceToHost) != hipSuccess) return HYLU_ERR_DEVICE;
        for (int32_t v = 0; v < L.nnodes; v++)
            for (int32_t a = 0; a < L.m[v]; a++) piv[L.r0[v] + a] = L.r0[v] + pl[L.r0[v] + a];
    }
    return HYLU_OK;
}

}  // extern "C"
