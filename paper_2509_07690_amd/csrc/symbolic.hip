// Symbolic factorisation and task-graph levels on the GPU (HYLU Sec. 2.1 last
// step and Sec. 2.2.1), with the same results as symbolic_factor and
// make_levels on the host.
//
// Structure.  Row i of the factors is the closure of row i of B under "k < i
// in the row brings the strict upper structure of row k".  The closure does
// not depend on the order in which the k are taken, and every k it takes is a
// descendant of i in the elimination tree of the pattern of B + B^T (the
// unsymmetric factors lie inside the Cholesky factor of that pattern).  So the
// rows of one tree level are independent: the tree is cut into chains (a row
// with one child continues its child's chain), chains are levelled by height,
// one launch per level runs one workgroup per chain, and the workgroup takes
// the chain's rows in ascending order.
//
// A workgroup holds row i as a bitmap over its block of rows in LDS.  Sources
// k < i are taken window by window (32768 positions) in ascending position; a
// window's candidates are taken together (a thread each for their run data,
// then all threads over all their column lists), and what they add to the same
// window is taken in another round.  A source k of run R (rows with identical
// structure past the run: the supernode definition) brings the run's rows
// k..last and the run's shared columns.  (The host's pruning, which adds only
// the first of those columns when the rest lie in its row, saves column work
// but chains the sources one after the other; here the rounds cost more.)
// The row's U list is read off the bitmap in column order; the row extends the
// run of row i-1 when U(i-1, >i-1) is i followed by its own list (then no list
// is stored: the run's first row holds it); its L part is stored as
// intervals, maximal runs of set bits cut at run starts, which are the host's
// intervals.
//
// Levels.  A node's sources, and the nodes owning the columns past its block,
// are its descendants and ancestors in the same tree, so one pass over the
// chain levels upward (factor DAG levels by pulling, U^T levels by pushing)
// and one downward (U levels by pulling, L^T levels by pushing) give the four
// longest-path level sets, each node taken at its last row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "analysis.hpp"

namespace hylu {
namespace {

constexpr int kSymQueue = 512;               // sources taken per round
constexpr int kSymWinWords = 1024;           // bitmap words per scan window (32768 positions)
constexpr int kSymNarrow = 64;               // chain levels of at most this many chains take 1024 threads a chain
constexpr int64_t kSymLdsMax = 150 * 1024;   // bitmap + fixed LDS of one workgroup

// a run of rows with one shared structure past it, kept at its first row
struct RunRec {
    int32_t last;               // its last row so far
    int32_t len;                // |U(first, >first)|
    int64_t off;                // that list in upool (-1: no room)
};

struct SymDev {
    const int64_t* rp;          // B (rows sorted)
    const int32_t* ci;
    const int32_t* parent;      // elimination tree of B + B^T (-1: root)
    const int32_t* crow;        // chain rows, chains by level, each ascending
    const int64_t* cptr;        // chain c: crow[cptr[c] .. cptr[c + 1])
    const int32_t* cbase;       // chain c: first row of its block (bit 0 of the bitmap)
    int32_t* head;              // row -> first row of its run
    RunRec* run;                // first row of a run -> the run's record
    int32_t* ulen;              // row -> |U(i, >i)|
    int64_t* ioff;              // row -> its intervals in ipool (pairs; -1: no room)
    int32_t* icnt;
    int32_t* upool;
    int32_t* ipool;
    int64_t ucap, icap;
    unsigned long long* ctr;    // [0] U entries, [1] intervals, [2] rows stored
};

__device__ __forceinline__ uint32_t bits_from(int b) { return ~0u << b; }                  // bits b..31
__device__ __forceinline__ uint32_t bits_upto(int b) { return b >= 31 ? ~0u : ((1u << (b + 1)) - 1); }  // bits 0..b

// exclusive prefix sum of v over the workgroup of NT threads; *total gets the sum
template <int NT>
__device__ __forceinline__ int32_t block_scan(int32_t v, int32_t* sc, int32_t* total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sc[wv] = x;
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int k = 0; k < NT / 64; k++) {
        if (k < wv) before += sc[k];
        all += sc[k];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_sym_rows(SymDev D, int64_t c0, int32_t words)
{
    extern __shared__ uint32_t bm[];                      // words
    __shared__ uint32_t proc[kSymWinWords];       // window positions already taken
    __shared__ int32_t queue[kSymQueue];         // bit positions of the round's sources
    __shared__ int32_t qlen[kSymQueue];          // columns each brings (< 0: pruning test pending)
    __shared__ int32_t qpre[kSymQueue];
    __shared__ int64_t qsrc[kSymQueue];          // where they start in upool
    __shared__ int32_t sc[NT / 64];
    __shared__ int32_t s_lo, s_hi, s_qn, s_carry;
    __shared__ long long s_off;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t c = c0 + blockIdx.x;
    const int32_t base = D.cbase[c];
    for (int32_t w = tid; w < words; w += NT) bm[w] = 0;
    for (int64_t r = D.cptr[c]; r < D.cptr[c + 1]; r++) {
        const int32_t i = D.crow[r];
        const int32_t li = i - base;
        if (tid == 0) { s_lo = INT_MAX; s_hi = -1; s_qn = 0; s_carry = -1; }
        __syncthreads();
        for (int64_t q = D.rp[i] + tid; q < D.rp[i + 1]; q += NT) {
            const int32_t j = D.ci[q] - base;
            if (j == li) continue;
            atomicOr(&bm[j >> 5], 1u << (j & 31));
            atomicMin(&s_lo, j);
            atomicMax(&s_hi, j);
        }
        __syncthreads();
        // ---- sources k < i, window by window
        const int32_t lo = s_lo;
        for (int32_t p = lo; p < li;) {
            const int32_t w0 = p >> 5, wl = (li - 1) >> 5;
            const int32_t nw = min(kSymWinWords, wl - w0 + 1);
            // rows of runs taken in earlier windows are taken: those runs reach
            // from there up to s_carry without a gap
            for (int32_t t = tid; t < kSymWinWords; t += NT) {
                const int32_t cw = s_carry - ((w0 + t) << 5);
                proc[t] = cw < 0 ? 0u : bits_upto(min(cw, 31));
            }
            __syncthreads();
            for (;;) {
                for (int32_t t = tid; t < nw; t += NT) {
                    uint32_t x = bm[w0 + t] & ~proc[t];
                    if (t == 0) x &= bits_from(p & 31);
                    if (w0 + t == wl) x &= bits_upto((li - 1) & 31);
                    const int cnt = __popc(x);
                    if (cnt) {
                        int pos = atomicAdd(&s_qn, cnt);
                        while (x && pos < kSymQueue) {
                            const int b = __ffs(x) - 1;
                            x &= x - 1;
                            queue[pos++] = ((w0 + t) << 5) + b;
                        }
                    }
                }
                __syncthreads();
                const int32_t qn = min(s_qn, kSymQueue);
                if (qn == 0) break;
                // A: a thread per source: the rows kl..last of its run into the
                // row (a source whose next lower row is in the row and in the
                // same run leaves that to the lower one) and where the run's
                // shared columns start
                for (int32_t q = tid; q < qn; q += NT) {
                    const int32_t kl = queue[q];
                    const int32_t h = D.head[kl + base];
                    int32_t len = 0;
                    int64_t src = 0;
                    const bool lower = kl - 1 >= p && ((bm[(kl - 1) >> 5] >> ((kl - 1) & 31)) & 1u) &&
                                       D.head[kl - 1 + base] == h;
                    if (lower) {
                        atomicOr(&proc[(kl >> 5) - w0], 1u << (kl & 31));
                    } else {
                        const RunRec rr = D.run[h];
                        const int32_t last = rr.last;           // < i: the run's rows below i are done
                        const int32_t lastl = last - base;
                        atomicMax(&s_carry, lastl);
                        for (int32_t w = kl >> 5; w <= (lastl >> 5); w++) {
                            uint32_t m = ~0u;
                            if (w == (kl >> 5)) m &= bits_from(kl & 31);
                            if (w == (lastl >> 5)) m &= bits_upto(lastl & 31);
                            atomicOr(&bm[w], m);
                            const int32_t pw = w - w0;
                            if (pw >= 0 && pw < nw) atomicOr(&proc[pw], m);
                        }
                        const int32_t off = last - h;
                        if (off < rr.len && rr.off >= 0) {
                            len = rr.len - off;
                            src = rr.off + off;
                        }
                    }
                    qlen[q] = len;
                    qsrc[q] = src;
                }
                __syncthreads();
                // B: the shared columns of every source, all threads over all of them
                int32_t tot = 0;
                {
                    const int32_t q0 = 2 * tid;
                    const int32_t a0 = q0 < qn ? qlen[q0] : 0, a1 = q0 + 1 < qn ? qlen[q0 + 1] : 0;
                    const int32_t ex = block_scan<NT>(a0 + a1, sc, &tot);
                    if (q0 < qn) qpre[q0] = ex;
                    if (q0 + 1 < qn) qpre[q0 + 1] = ex + a0;
                }
                __syncthreads();
                int32_t mx = -1;
                if (tid < tot) {
                    int32_t a = 0;                      // source of position t: the last starting at or before it
                    {
                        int32_t b = qn - 1;
                        while (a < b) {
                            const int32_t mid = (a + b + 1) >> 1;
                            if (qpre[mid] <= tid) a = mid; else b = mid - 1;
                        }
                    }
                    // four positions per step, their loads issued before the bitmap updates
                    for (int32_t t = tid; t < tot; t += 4 * NT) {
                        int32_t j[4];
#pragma unroll
                        for (int u2 = 0; u2 < 4; u2++) {
                            const int32_t tt = t + u2 * NT;
                            j[u2] = -1;
                            if (tt < tot) {
                                while (a + 1 < qn && qpre[a + 1] <= tt) a++;
                                j[u2] = D.upool[qsrc[a] + (tt - qpre[a])] - base;
                            }
                        }
#pragma unroll
                        for (int u2 = 0; u2 < 4; u2++)
                            if (j[u2] >= 0) {
                                atomicOr(&bm[j[u2] >> 5], 1u << (j[u2] & 31));
                                mx = max(mx, j[u2]);
                            }
                    }
                }
                if (mx >= 0) atomicMax(&s_hi, mx);
                __syncthreads();
                if (tid == 0) s_qn = 0;
                __syncthreads();
            }
            p = (w0 + nw) << 5;
        }
        __syncthreads();
        const int32_t hi = s_hi;
        // ---- U(i, >i): the bits (li, hi], a contiguous word range per thread
        int32_t ws0 = 0, ws1 = 0, myc = 0;
        const int32_t wa = (li + 1) >> 5, wb = hi >> 5;
        if (hi > li) {
            const int32_t per = (wb - wa + 1 + NT - 1) / NT;
            ws0 = wa + tid * per;
            ws1 = min(ws0 + per, wb + 1);
            for (int32_t w = ws0; w < ws1; w++) myc += __popc(w == wa ? bm[w] & bits_from((li + 1) & 31) : bm[w]);
        }
        int32_t u = 0;
        const int32_t upre = block_scan<NT>(myc, sc, &u);
        // ---- does row i extend the run of row i - 1 (U(i-1, >i-1) = {i} + U(i, >i))?
        bool chain = li >= 1 && D.parent[i - 1] == i;
        int32_t hp = -1;
        if (chain) {
            hp = D.head[i - 1];
            const int64_t ub = D.run[hp].off;
            const int32_t pos = (i - 1) - hp;
            chain = ub >= 0 && D.ulen[i - 1] == u + 1 && D.upool[ub + pos] == i;
            if (chain) {
                const int32_t* P = D.upool + ub + pos + 1;
                bool ok = true;
                for (int32_t t = tid; t < u; t += NT) {
                    const int32_t j = P[t] - base;
                    if (!((bm[j >> 5] >> (j & 31)) & 1u)) ok = false;
                }
                chain = __syncthreads_and(ok) != 0;
            }
        }
        if (chain) {
            if (tid == 0) {
                D.head[i] = hp;
                D.run[hp].last = i;
            }
        } else {
            if (tid == 0) {
                const unsigned long long o = atomicAdd(&D.ctr[0], (unsigned long long)u);
                s_off = (long long)o + u <= D.ucap ? (long long)o : -1;
                D.head[i] = i;
                D.run[i] = RunRec{i, u, (int64_t)s_off};
            }
            __syncthreads();
            const long long o = s_off;
            if (o >= 0 && hi > li) {
                int32_t* dst = D.upool + o + upre;
                for (int32_t w = ws0; w < ws1; w++) {
                    uint32_t x = w == wa ? bm[w] & bits_from((li + 1) & 31) : bm[w];
                    while (x) {
                        const int b = __ffs(x) - 1;
                        x &= x - 1;
                        *dst++ = (w << 5) + b + base;
                    }
                }
            }
        }
        if (tid == 0) D.ulen[i] = u;
        // ---- L(i, :): maximal runs of set bits in [lo, li), cut at run starts
        int32_t ns = 0, ne = 0, wl0 = 0, wl1 = 0;
        if (lo < li) {
            const int32_t a = lo >> 5, b = (li - 1) >> 5;
            const int32_t per = (b - a + 1 + NT - 1) / NT;
            wl0 = a + tid * per;
            wl1 = min(wl0 + per, b + 1);
            for (int32_t w = wl0; w < wl1; w++) {
                uint32_t x = w == b ? bm[w] & bits_upto((li - 1) & 31) : bm[w];
                while (x) {
                    const int bb = __ffs(x) - 1;
                    x &= x - 1;
                    const int32_t t = (w << 5) + bb;
                    const bool st = t == lo || !((bm[(t - 1) >> 5] >> ((t - 1) & 31)) & 1u) || D.head[t + base] == t + base;
                    const bool en = t == li - 1 || !((bm[(t + 1) >> 5] >> ((t + 1) & 31)) & 1u) ||
                                    D.head[t + 1 + base] == t + 1 + base;
                    ns += st;
                    ne += en;
                }
            }
        }
        int32_t nint = 0, nint_e = 0;
        const int32_t spre = block_scan<NT>(ns, sc, &nint);
        const int32_t epre = block_scan<NT>(ne, sc, &nint_e);
        if (tid == 0) {
            const unsigned long long o = nint > 0 ? atomicAdd(&D.ctr[1], (unsigned long long)nint) : 0ull;
            s_off = nint == 0 ? 0 : ((long long)o + nint <= D.icap ? (long long)o : -1);
            D.ioff[i] = s_off;
            D.icnt[i] = nint;
        }
        __syncthreads();
        const long long io = s_off;
        if (io >= 0 && nint > 0 && nint == nint_e) {
            int32_t* dst = D.ipool + 2 * io;
            int32_t ks = spre, ke = epre;
            const int32_t b = (li - 1) >> 5;
            for (int32_t w = wl0; w < wl1; w++) {
                uint32_t x = w == b ? bm[w] & bits_upto((li - 1) & 31) : bm[w];
                while (x) {
                    const int bb = __ffs(x) - 1;
                    x &= x - 1;
                    const int32_t t = (w << 5) + bb;
                    const bool st = t == lo || !((bm[(t - 1) >> 5] >> ((t - 1) & 31)) & 1u) || D.head[t + base] == t + base;
                    const bool en = t == li - 1 || !((bm[(t + 1) >> 5] >> ((t + 1) & 31)) & 1u) ||
                                    D.head[t + 1 + base] == t + 1 + base;
                    if (st) dst[2 * (ks++)] = t + base;
                    if (en) dst[2 * (ke++) + 1] = t + base;
                }
            }
        }
        if (tid == 0 && nint != nint_e) D.ioff[i] = -2;     // cannot happen; reported as an internal error
        __syncthreads();
        // ---- clear the bits this row set (all within [lo, hi])
        const int32_t clo = min(lo, li), chi = max(hi, li - 1);
        if (clo <= chi && chi >= 0)
            for (int32_t w = (max(clo, 0) >> 5) + tid; w <= (chi >> 5); w += NT) bm[w] = 0;
        __syncthreads();
    }
}

struct LevDev {
    int32_t n;
    const int32_t* crow;
    const int64_t* cptr;
    const int32_t* of_row;      // row -> node
    const int32_t* nptr;        // node -> first row
    const int32_t* head;
    const int32_t* ulen;
    const RunRec* run;
    const int32_t* upool;
    const int64_t* ioff;
    const int32_t* icnt;
    const int32_t* ipool;
    int32_t* lev;               // 4 x nnodes: factor, U, U^T, L^T
    int32_t nn;
};

__device__ __forceinline__ int32_t ld_lev(const int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ __forceinline__ int32_t wave_max(int32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// upward pass over one chain level: one wavefront per chain, rows ascending;
// a node is taken at its last row: its factor level from its sources (pull),
// then its U^T level pushed to the nodes owning the columns past its block
__global__ __launch_bounds__(64) void k_sym_lev_up(LevDev G, int64_t c0)
{
    const int lane = threadIdx.x;
    const int64_t c = c0 + blockIdx.x;
    int32_t* l0 = G.lev;
    int32_t* l2 = G.lev + 2 * (int64_t)G.nn;
    for (int64_t r = G.cptr[c]; r < G.cptr[c + 1]; r++) {
        const int32_t row = G.crow[r];
        const int32_t v = G.of_row[row];
        if (row + 1 < G.n && G.of_row[row + 1] == v) continue;
        int32_t best = 0;
        for (int32_t i = G.nptr[v]; i <= row; i++) {
            const int64_t io = G.ioff[i];
            for (int32_t q = lane; q < G.icnt[i]; q += 64) {
                const int32_t a = G.ipool[2 * (io + q)], b = G.ipool[2 * (io + q) + 1];
                for (int32_t u = G.of_row[a]; u <= G.of_row[b]; u++)
                    if (u != v) best = max(best, ld_lev(l0 + u) + 1);
            }
        }
        best = wave_max(best);
        if (lane == 0) __hip_atomic_store(l0 + v, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t h = G.head[row];
        const int32_t* U = G.upool + G.run[h].off + (row - h);
        const int32_t lv = ld_lev(l2 + v) + 1;
        for (int32_t t = lane; t < G.ulen[row]; t += 64) {
            const int32_t u = G.of_row[U[t]];
            if (u != v) atomicMax(l2 + u, lv);
        }
        __threadfence();
    }
}

// downward pass: chain levels from the top, rows descending; a node's U level
// from the nodes owning its columns (pull), then its L^T level pushed to its
// sources
__global__ __launch_bounds__(64) void k_sym_lev_down(LevDev G, int64_t c0)
{
    const int lane = threadIdx.x;
    const int64_t c = c0 + blockIdx.x;
    int32_t* l1 = G.lev + (int64_t)G.nn;
    int32_t* l3 = G.lev + 3 * (int64_t)G.nn;
    for (int64_t r = G.cptr[c + 1] - 1; r >= G.cptr[c]; r--) {
        const int32_t row = G.crow[r];
        const int32_t v = G.of_row[row];
        if (row + 1 < G.n && G.of_row[row + 1] == v) continue;
        const int32_t h = G.head[row];
        const int32_t* U = G.upool + G.run[h].off + (row - h);
        int32_t best = 0;
        for (int32_t t = lane; t < G.ulen[row]; t += 64) {
            const int32_t u = G.of_row[U[t]];
            if (u != v) best = max(best, ld_lev(l1 + u) + 1);
        }
        best = wave_max(best);
        if (lane == 0) __hip_atomic_store(l1 + v, best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t lv = ld_lev(l3 + v) + 1;
        for (int32_t i = G.nptr[v]; i <= row; i++) {
            const int64_t io = G.ioff[i];
            for (int32_t q = lane; q < G.icnt[i]; q += 64) {
                const int32_t a = G.ipool[2 * (io + q)], b = G.ipool[2 * (io + q) + 1];
                for (int32_t u = G.of_row[a]; u <= G.of_row[b]; u++)
                    if (u != v) atomicMax(l3 + u, lv);
            }
        }
        __threadfence();
    }
}

// ---------------------------------------------------------------- host side

struct Buf {
    const DeviceAlloc* da = nullptr;
    std::vector<void*> ptrs;
    void* get(size_t bytes)
    {
        void* p = da->alloc(da->ctx, std::max<size_t>(bytes, 16));
        if (p) ptrs.push_back(p);
        return p;
    }
    ~Buf()
    {
        if (!ptrs.empty()) (void)hipDeviceSynchronize();
        for (void* p : ptrs) da->free(da->ctx, p);
    }
};

template <typename T>
T* put(Buf& B, const std::vector<T>& v, std::string& err)
{
    T* d = (T*)B.get(sizeof(T) * v.size());
    if (!d) { err = "device allocation failed"; return nullptr; }
    if (!v.empty() && hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        err = "host to device copy failed";
        return nullptr;
    }
    return d;
}

template <typename T>
bool get(std::vector<T>& v, const T* d, size_t count, std::string& err)
{
    v.resize(count);
    if (count && hipMemcpy(v.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost) != hipSuccess) {
        err = "device to host copy failed";
        return false;
    }
    return true;
}

}  // namespace

void elimination_chains(const Csr& b, const std::vector<int64_t>& blocks, EtreeChains& ec)
{
    const int32_t n = b.n;
    ec = EtreeChains();
    // entries k < i of row i of B + B^T: row i of B below the diagonal, and
    // column i of B above it
    std::vector<int64_t> lp(n + 1, 0);
    for (int32_t r = 0; r < n; r++)
        for (int64_t q = b.rp[r]; q < b.rp[r + 1]; q++) {
            const int32_t c = b.ci[q];
            if (c < r) lp[r + 1]++;
            else if (c > r) lp[c + 1]++;
        }
    for (int32_t i = 0; i < n; i++) lp[i + 1] += lp[i];
    std::vector<int32_t> lk(lp[n]);
    std::vector<int64_t> fill(lp.begin(), lp.end() - 1);
    for (int32_t r = 0; r < n; r++)
        for (int64_t q = b.rp[r]; q < b.rp[r + 1]; q++) {
            const int32_t c = b.ci[q];
            if (c < r) lk[fill[r]++] = c;
            else if (c > r) lk[fill[c]++] = r;
        }
    // elimination tree with path compression
    ec.parent.assign(n, -1);
    std::vector<int32_t> anc(n, -1);
    for (int32_t i = 0; i < n; i++)
        for (int64_t q = lp[i]; q < lp[i + 1]; q++)
            for (int32_t j = lk[q]; j != -1 && j < i;) {
                const int32_t nx = anc[j];
                anc[j] = i;
                if (nx == -1) ec.parent[j] = i;
                j = nx;
            }
    // chains: a row with exactly one child continues that child's chain
    std::vector<int32_t> nch(n, 0), child(n, -1), chain(n), lev(n), maxc(n, -1);
    for (int32_t k = 0; k < n; k++)
        if (ec.parent[k] >= 0) { nch[ec.parent[k]]++; child[ec.parent[k]] = k; }
    int32_t nc = 0, nl = 0;
    std::vector<int32_t> clev;
    for (int32_t t = 0; t < n; t++) {
        if (nch[t] == 1) {
            chain[t] = chain[child[t]];
            lev[t] = lev[child[t]];
        } else {
            chain[t] = nc++;
            lev[t] = maxc[t] + 1;
            clev.push_back(lev[t]);
        }
        nl = std::max(nl, lev[t] + 1);
        if (ec.parent[t] >= 0) maxc[ec.parent[t]] = std::max(maxc[ec.parent[t]], lev[t]);
    }
    // chains ordered by level, rows ascending inside a chain
    std::vector<int32_t> corder(nc), cpos(nc);
    ec.lev_ptr.assign(nl + 1, 0);
    for (int32_t k = 0; k < nc; k++) ec.lev_ptr[clev[k] + 1]++;
    for (int32_t l = 0; l < nl; l++) ec.lev_ptr[l + 1] += ec.lev_ptr[l];
    {
        std::vector<int64_t> f(ec.lev_ptr.begin(), ec.lev_ptr.end() - 1);
        for (int32_t k = 0; k < nc; k++) { cpos[k] = (int32_t)f[clev[k]]++; corder[cpos[k]] = k; }
    }
    std::vector<int64_t> clen(nc, 0);
    for (int32_t t = 0; t < n; t++) clen[cpos[chain[t]]]++;
    ec.cptr.assign(nc + 1, 0);
    for (int32_t k = 0; k < nc; k++) ec.cptr[k + 1] = ec.cptr[k] + clen[k];
    ec.crow.resize(n);
    ec.cbase.assign(nc, 0);
    {
        std::vector<int64_t> f(ec.cptr.begin(), ec.cptr.end() - 1);
        for (int32_t t = 0; t < n; t++) {
            const int32_t k = cpos[chain[t]];
            if (f[k] == ec.cptr[k]) {
                const size_t bi = std::upper_bound(blocks.begin(), blocks.end(), (int64_t)t) - blocks.begin() - 1;
                ec.cbase[k] = (int32_t)blocks[bi];
            }
            ec.crow[f[k]++] = t;
        }
    }
    ec.width = 0;
    for (size_t k = 0; k + 1 < blocks.size(); k++) ec.width = std::max<int64_t>(ec.width, blocks[k + 1] - blocks[k]);
}

bool gpu_symbolic_levels(const Csr& b, const std::vector<int64_t>& blocks, int32_t sn_min, int32_t sn_max,
                         const DeviceAlloc& da, Symbolic& s, Nodes& nd, GpuSymStats& stats, std::string& err)
{
    const int32_t n = b.n;
    stats = GpuSymStats();
    EtreeChains ec;
    elimination_chains(b, blocks, ec);
    const int32_t words = (int32_t)((ec.width + 31) / 32);
    const size_t lds = sizeof(uint32_t) * (size_t)words;
    if ((int64_t)lds + 8 * 1024 > kSymLdsMax) {
        err = "GPU symbolic factorisation: a block of more than 1 << 20 rows";
        return false;
    }
    const int32_t nl = (int32_t)ec.lev_ptr.size() - 1;
    const int64_t nchains = ec.cptr.size() - 1;
    stats.chain_levels = nl;
    stats.chains = nchains;
    Buf B;
    B.da = &da;
    SymDev D{};
    D.rp = put(B, b.rp, err);
    D.ci = put(B, b.ci, err);
    D.parent = put(B, ec.parent, err);
    D.crow = put(B, ec.crow, err);
    D.cptr = put(B, ec.cptr, err);
    D.cbase = put(B, ec.cbase, err);
    if (!D.rp || !D.ci || !D.parent || !D.crow || !D.cptr || !D.cbase) return false;
    D.head = (int32_t*)B.get(sizeof(int32_t) * n);
    D.run = (RunRec*)B.get(sizeof(RunRec) * n);
    D.ulen = (int32_t*)B.get(sizeof(int32_t) * n);
    D.ioff = (int64_t*)B.get(sizeof(int64_t) * n);
    D.icnt = (int32_t*)B.get(sizeof(int32_t) * n);
    D.ctr = (unsigned long long*)B.get(sizeof(unsigned long long) * 4);
    if (!D.head || !D.run || !D.ulen || !D.ioff || !D.icnt || !D.ctr) {
        err = "device allocation failed";
        return false;
    }
    const int64_t nnzb = b.nnz();
    int64_t ucap = 16 * nnzb + 4 * (int64_t)n, icap = 8 * nnzb + 2 * (int64_t)n;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { err = "event"; return false; }
    std::vector<unsigned long long> ctr(4);
    for (int attempt = 0;; attempt++) {
        D.upool = (int32_t*)B.get(sizeof(int32_t) * ucap);
        D.ipool = (int32_t*)B.get(sizeof(int32_t) * 2 * icap);
        if (!D.upool || !D.ipool) { err = "device allocation failed"; return false; }
        D.ucap = ucap;
        D.icap = icap;
        if (hipMemset(D.ctr, 0, sizeof(unsigned long long) * 4) != hipSuccess) { err = "memset"; return false; }
        (void)hipEventRecord(e0, 0);
        for (int32_t l = 0; l < nl; l++) {
            const int64_t g = ec.lev_ptr[l + 1] - ec.lev_ptr[l];
            if (g <= 0) continue;
            if (g <= kSymNarrow)
                hipLaunchKernelGGL(k_sym_rows<1024>, dim3((uint32_t)g), dim3(1024), lds, 0, D, (int64_t)ec.lev_ptr[l], words);
            else
                hipLaunchKernelGGL(k_sym_rows<256>, dim3((uint32_t)g), dim3(256), lds, 0, D, (int64_t)ec.lev_ptr[l], words);
        }
        (void)hipEventRecord(e1, 0);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            err = "GPU symbolic factorisation: launch failed";
            return false;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        stats.ms_structure += ms;
        if (hipMemcpy(ctr.data(), D.ctr, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            err = "device to host copy failed";
            return false;
        }
        if ((int64_t)ctr[0] <= ucap && (int64_t)ctr[1] <= icap) break;
        if (attempt > 0) { err = "GPU symbolic factorisation: pools"; return false; }
        // too small: once more with the sizes the first pass counted
        stats.retries++;
        ucap = std::max<int64_t>(ucap, (int64_t)ctr[0]);
        icap = std::max<int64_t>(icap, (int64_t)ctr[1]);
    }
    std::vector<int32_t> head, ulen, icnt, upool, ipool;
    std::vector<int64_t> ioff;
    std::vector<RunRec> run;
    if (!get(head, D.head, n, err) || !get(ulen, D.ulen, n, err) || !get(run, D.run, n, err) ||
        !get(ioff, D.ioff, n, err) || !get(icnt, D.icnt, n, err) || !get(upool, D.upool, ctr[0], err) ||
        !get(ipool, D.ipool, 2 * ctr[1], err))
        return false;
    // ---- the compressed structure, in row order
    s = Symbolic();
    s.n = n;
    s.lp.assign(n + 1, 0);
    s.run_of.assign(n, -1);
    s.ucount.assign(n, 0);
    s.run_up.push_back(0);
    for (int32_t i = 0; i < n; i++) {
        if (head[i] == i) {
            const int64_t uo = run[i].off;
            if (uo < 0 || run[i].len != ulen[i]) { err = "GPU symbolic factorisation: run list missing"; return false; }
            s.run_start.push_back(i);
            s.run_u.insert(s.run_u.end(), upool.begin() + uo, upool.begin() + uo + ulen[i]);
            s.run_up.push_back((int64_t)s.run_u.size());
        } else if (i == 0 || head[i] != head[i - 1]) {
            err = "GPU symbolic factorisation: run not contiguous";
            return false;
        }
        s.run_of[i] = (int32_t)s.run_start.size() - 1;
        s.ucount[i] = ulen[i];
        if (icnt[i] > 0) {
            if (ioff[i] < 0) { err = "GPU symbolic factorisation: intervals missing"; return false; }
            s.lint.insert(s.lint.end(), ipool.begin() + 2 * ioff[i], ipool.begin() + 2 * (ioff[i] + icnt[i]));
        }
        s.lp[i + 1] = (int64_t)s.lint.size() / 2;
    }
    s.run_start.push_back(n);
    symbolic_counts(s);
    // ---- nodes on the host (a pass over the runs), levels on the device
    make_nodes(s, sn_min, sn_max, nd);
    const int32_t nn = nd.count;
    LevDev G{};
    G.n = n;
    G.nn = nn;
    G.crow = D.crow;
    G.cptr = D.cptr;
    G.of_row = put(B, nd.of_row, err);
    G.nptr = put(B, nd.ptr, err);
    if (!G.of_row || !G.nptr) return false;
    G.head = D.head;
    G.ulen = D.ulen;
    G.run = D.run;
    G.upool = D.upool;
    G.ioff = D.ioff;
    G.icnt = D.icnt;
    G.ipool = D.ipool;
    G.lev = (int32_t*)B.get(sizeof(int32_t) * 4 * (size_t)std::max(nn, 1));
    if (!G.lev || hipMemset(G.lev, 0, sizeof(int32_t) * 4 * (size_t)std::max(nn, 1)) != hipSuccess) {
        err = "device allocation failed";
        return false;
    }
    (void)hipEventRecord(e0, 0);
    for (int32_t l = 0; l < nl; l++) {
        const int64_t g = ec.lev_ptr[l + 1] - ec.lev_ptr[l];
        if (g > 0) hipLaunchKernelGGL(k_sym_lev_up, dim3((uint32_t)g), dim3(64), 0, 0, G, (int64_t)ec.lev_ptr[l]);
    }
    for (int32_t l = nl - 1; l >= 0; l--) {
        const int64_t g = ec.lev_ptr[l + 1] - ec.lev_ptr[l];
        if (g > 0) hipLaunchKernelGGL(k_sym_lev_down, dim3((uint32_t)g), dim3(64), 0, 0, G, (int64_t)ec.lev_ptr[l]);
    }
    (void)hipEventRecord(e1, 0);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        err = "GPU level sets: launch failed";
        return false;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    stats.ms_levels = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<int32_t> lev;
    if (!get(lev, G.lev, 4 * (size_t)nn, err)) return false;
    for (int t = 0; t < 4; t++) {
        nd.level[t].assign(lev.begin() + (size_t)t * nn, lev.begin() + (size_t)(t + 1) * nn);
        int32_t mx = -1;
        for (int32_t v = 0; v < nn; v++) mx = std::max(mx, nd.level[t][v]);
        nd.nlevels[t] = mx + 1;
    }
    return true;
}

}  // namespace hylu
