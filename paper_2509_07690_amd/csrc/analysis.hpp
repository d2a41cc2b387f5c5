// Host-side preprocessing of HYLU (arXiv 2509.07690, Sec. 2.1) and the data
// layout the gfx950 kernels consume.  Everything here runs on the CPU once per
// sparsity pattern; the numerical phases only read the tables it produces.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hylu {

struct Csr {
    int32_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

// ---------------------------------------------------------------- ordering
// Static pivoting and scaling by a maximum-product matching (Sec. 2.1):
// row_of_col[j] is the row matched to column j; dr/dc make the matched entries
// +-1 and every other entry at most 1 in magnitude.  Returns false when the
// pattern is structurally singular.
bool mc64_match_scale(const Csr& a, std::vector<int32_t>& row_of_col,
                      std::vector<double>& dr, std::vector<double>& dc);

// Symmetric fill-reducing orderings of an undirected graph given as CSR
// adjacency without self loops.  Both return perm[new] = old.  dense_alpha
// sets AMD's dense-row threshold (<= 0: relative to the mean degree).
std::vector<int32_t> amd_order(int32_t n, const std::vector<int64_t>& xadj,
                               const std::vector<int32_t>& adj, double dense_alpha = 0.0);
// multilevel = false: separators from breadth-first level structures; true:
// from multilevel edge bisections (smaller separators on meshes)
std::vector<int32_t> nd_order(int32_t n, const std::vector<int64_t>& xadj,
                              const std::vector<int32_t>& adj, int32_t leaf_size, double dense_alpha = 0.0,
                              bool multilevel = false);

// ---------------------------------------------------------------- symbolic
// Exact, unpivoted structure of the factors of B in compressed form:
//  * L(i,:) as a list of row intervals [lo, hi] (inclusive), each inside one
//    chain run of rows with identical U structure;
//  * U of every run [r, last]: rows r..last share the columns past `last`,
//    stored once as the strict upper structure of row r (run_u), whose first
//    (last - r) entries are r+1..last.
struct Symbolic {
    int32_t n = 0;
    std::vector<int64_t> lp;            // n+1, into lint (pairs)
    std::vector<int32_t> lint;          // 2 ints per interval
    std::vector<int32_t> run_of;        // row -> run id
    std::vector<int32_t> run_start;     // run id -> first row (runs+1 entries)
    std::vector<int64_t> run_up;        // run id -> offset into run_u (runs+1)
    std::vector<int32_t> run_u;         // strict upper structure of each run's first row
    std::vector<int64_t> lcount;        // l_k: rows i > k with L(i,k) != 0
    std::vector<int64_t> ucount;        // u_k: |U(k,>k)|
    int64_t nnz_l = 0, nnz_u = 0;       // exact, U includes the diagonal
    uint64_t flops = 0;                 // F = sum_k l_k (1 + 2 u_k)
    int32_t nruns() const { return (int32_t)run_start.size() - 1; }
};

bool symbolic_factor(const Csr& b, Symbolic& s);
// lcount, nnz_l, nnz_u and flops from the intervals and ucount
void symbolic_counts(Symbolic& s);

// ---------------------------------------------------------------- nodes
// Supernodes (Sec. 2.2: consecutive rows with identical U structure) and
// standalone rows, plus the level sets of the task graphs (Sec. 2.2.1).
struct Nodes {
    int32_t count = 0;
    std::vector<int32_t> ptr;           // count+1 row boundaries
    std::vector<int32_t> of_row;        // row -> node
    std::vector<uint8_t> is_sn;         // node -> supernode flag
    // level of every node in the four task graphs:
    // 0 factor / forward (L) solve, 1 backward (U) solve, 2 U^T solve, 3 L^T solve
    std::vector<int32_t> level[4];
    int32_t nlevels[4] = {0, 0, 0, 0};
    uint64_t flops_padded = 0;          // work with every row padded to whole source nodes
};

void make_nodes(const Symbolic& s, int32_t sn_min, int32_t sn_max, Nodes& nd);
void make_levels(const Symbolic& s, Nodes& nd);

// ---------------------------------------------------------------- on the GPU
// Schedule of the GPU symbolic factorisation: the elimination tree of the
// pattern of B + B^T cut into chains (a row with one child continues the
// child's chain), chains levelled by height (a chain above all chains of its
// children's subtrees), rows ascending inside a chain.
struct EtreeChains {
    std::vector<int32_t> parent;        // per row, -1 for a root
    std::vector<int64_t> lev_ptr;       // chain levels -> chains
    std::vector<int64_t> cptr;          // chains -> rows in crow
    std::vector<int32_t> crow;
    std::vector<int32_t> cbase;         // per chain: first row of its independent block
    int64_t width = 0;                  // widest block
};
// blocks: row offsets of independent diagonal blocks (0, ..., n)
void elimination_chains(const Csr& b, const std::vector<int64_t>& blocks, EtreeChains& ec);

struct DeviceAlloc {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes);
    void (*free)(void* ctx, void* p);
};
struct GpuSymStats {
    double ms_structure = 0, ms_levels = 0;   // kernel time (event pairs)
    int32_t chain_levels = 0, retries = 0;
    int64_t chains = 0;
};
// symbolic_factor + make_nodes + make_levels with the structure and the level
// sets computed by kernels: the same Symbolic and Nodes to the bit.  Blocks
// of at most 1 << 20 rows; false with err set otherwise or on a device error.
bool gpu_symbolic_levels(const Csr& b, const std::vector<int64_t>& blocks, int32_t sn_min, int32_t sn_max,
                         const DeviceAlloc& da, Symbolic& s, Nodes& nd, GpuSymStats& stats, std::string& err);

// ---------------------------------------------------------------- layout
// Every node v (a supernode of m rows, or a standalone row with m = 1) owns a
// dense row-major panel of m x W values: [L region | diagonal block | T],
// with one shared sorted column list.  The L region holds the multipliers for
// whole source nodes (one slot per source row), the diagonal block holds the
// node's own L\U in pivoted column order, T the columns of U past the block.
// rows per factorisation panel inside a node wider than one panel
constexpr int32_t kWideChunk = 16;
// rows per tile of the supernode-target update kernel
constexpr int32_t kTileRowsHost = 16;

struct Layout {
    int32_t n = 0, nnodes = 0;
    std::vector<int32_t> r0, m, lw, W;  // per node
    std::vector<int64_t> voff, coff;    // value / column-list offsets
    std::vector<int32_t> cols;          // concatenated column lists
    int64_t nvals = 0;
    // per target node: its sources in ascending order
    std::vector<int64_t> eptr;          // nnodes+1
    std::vector<int32_t> esrc, elpos;   // source node, slot of its first row in the target
    std::vector<int64_t> eroff;         // offset of the relative map of the source's T
    std::vector<int32_t> rel;           // relative positions, concatenated
    // value map: entry q of B (CSR order of A) lands in slot amap[p]
    std::vector<int64_t> amap;          // per A entry p -> value slot
    // dense tail: rows [t0, n) factored as one dense block (same factors: the
    // padding stays exactly zero and each row still pivots inside its node)
    int32_t tail_node0 = 0, t0 = 0, mT = 0;
    std::vector<int32_t> lext;          // per node: width of the L part from sources outside the tail
    std::vector<int64_t> trow;          // per tail row: value offset of its dense part (column t0)
    std::vector<int32_t> tlo, thi;      // per tail row: tail-local block range of its node
    struct Panel { int32_t p0, p1, c0, c1, cg0; };
    std::vector<Panel> panels;          // row panels of the dense tail LU
    std::vector<Panel> spanels;         // row panels of the dense tail solves (whole nodes or 64-row chunks)
    // execution level lists (node ids by level, then index):
    // 0 factor updates (every node; tail nodes take their outside sources only)
    // 1 U solve, 2 U^T solve, 3 L^T solve, 4 L solve (nodes before the tail)
    std::vector<int32_t> xlev_ptr[5], xlev_nodes[5];
    uint64_t flops_kernel = 0;          // flops the kernels issue (padding and dense tail included)
};

// First node of the dense tail: the smallest node start t such that the exact
// factors restricted to rows and columns [t, n) have at least `density` of
// their entries nonzero (and at least min_rows rows); nd.count if none.
int32_t choose_tail(const Symbolic& s, const Nodes& nd, double density, int32_t min_rows, int32_t max_rows);

bool build_layout(const Csr& b, const Symbolic& s, const Nodes& nd, int32_t tail_node0, int32_t panel_rows,
                  Layout& L, const std::vector<int64_t>& bsrc, std::string& err);

// Structural block masks of the dense tail over its factorisation panels
// (L.panels).  lbits: per tail row, the panels whose pivot columns the row has
// L entries in; ubits: per tail column, the panels with a row that has a U
// entry in that column.  Node-padded (a row with an entry anywhere in a node's
// block counts for every panel of that node; a row's U covers its whole
// block), so every entry outside the masks stays exactly zero through the
// dense factorisation whatever pivots the blocks take: the trailing updates
// and triangular solves of those blocks can be skipped with no change to any
// result.  words: 64-bit words per row / column.
struct TailMasks {
    int32_t words = 0;
    std::vector<uint64_t> lbits, ubits;
    bool lbit(int32_t a, int32_t j) const { return (lbits[(size_t)a * words + (j >> 6)] >> (j & 63)) & 1; }
    bool ubit(int32_t c, int32_t j) const { return (ubits[(size_t)c * words + (j >> 6)] >> (j & 63)) & 1; }
};
void tail_masks(const Symbolic& s, const Nodes& nd, const Layout& L, TailMasks& M);

}  // namespace hylu
