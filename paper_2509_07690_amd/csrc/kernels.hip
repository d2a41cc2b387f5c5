// gfx950 kernels of HYLU's numerical factorisation (Sec. 2.2) and
// forward-backward substitution (Sec. 2.3).
//
// Storage (per node v with m rows, panel m x W, row-major):
//   [ L region (lw) | diagonal block (m) | T (W - lw - m) ]
// The diagonal block keeps its natural column order.  Row a of a supernode
// pivots on block column pl[r0 + a] (the largest entry of its row in the
// block, Sec. 2.2); its multiplier for an earlier row b of the same node is
// stored at the pivot column of b, and its U values at the columns not yet
// pivoted.  A target's L-region slots for a source node follow the same rule:
// the multiplier of source row b sits at the slot of b's pivot column.  No
// column is ever moved, so a level never waits on a permutation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"

namespace hylu {

namespace {

template <typename T> __device__ __forceinline__ T tabs(T x) { return x < T(0) ? -x : x; }

// value of v in lane l (l the same in every lane), all lanes active
__device__ __forceinline__ double rlane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float rlane(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
// magnitude for the pivot search: a NaN ranks above every number, so a search
// over a non-empty set of columns always returns one of them
template <typename T> __device__ __forceinline__ T pmag(T x)
{
    const T y = tabs(x);
    return y == y ? y : static_cast<T>(__builtin_huge_valf());
}

// barrier policies of the row-update device functions: a whole workgroup
// works on one task (bulk mode), or one wavefront does (the pipelined launch,
// whose other wavefronts run other tasks).  The wavefront barrier orders its
// lanes' LDS and global accesses as a block barrier does (same fences, no
// s_barrier).
struct BlockSync { static __device__ __forceinline__ void bar() { __syncthreads(); } };
struct WaveSync {
    static __device__ __forceinline__ void bar()
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
};

constexpr int kStage = 1024;   // staged source entries per batch (values + relative indices), default
constexpr int kSnSolveRows = 64;   // largest supernode of the four-wavefront forward solve

// ----------------------------------------------------------------------------
// value scatter: B = R A C into the panels (fill slots are zero)
// ----------------------------------------------------------------------------

__global__ void k_zero(uint64_t* __restrict__ p, int64_t n64)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n64; i += stride) p[i] = 0;
}

__global__ void k_zero_bytes(uint8_t* __restrict__ p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// also keeps a copy of A's values for the FP64 residual of the refinement
template <typename T>
__global__ void k_scatter(const double* __restrict__ aval, const int64_t* __restrict__ amap,
                          const double* __restrict__ asr, const double* __restrict__ asc, int64_t nnz,
                          T* __restrict__ vals, double* __restrict__ acopy)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) {
        double a = aval[p];
        acopy[p] = a;
        vals[amap[p]] = (T)((asr[p] * a) * asc[p]);
    }
}

__global__ void k_init_pivots(int32_t n, const int32_t* __restrict__ row_node, const int32_t* __restrict__ r0,
                              int32_t* __restrict__ pl, int32_t* __restrict__ qinv)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        // standalone rows pivot on their own column; supernode rows are set by the block LU
        (void)row_node; (void)r0;
        pl[i] = 0;
        qinv[i] = i;
    }
}

// ----------------------------------------------------------------------------
// row updates: one wavefront per target row.  Every source node (a standalone
// row: row-row kernel; a supernode: sup-row kernel) is applied in ascending
// order: the multipliers come from a triangular solve with the source block in
// its pivot order, then the source's T part is subtracted through the relative
// map.  The row's accumulator sits in LDS when it fits.
// ----------------------------------------------------------------------------

// a source with its own pivot order (a supernode; also a standalone source too
// large for the stage): triangular solve with its block in pivot order, then
// the update of the columns past the block.  The pivot order, and the block
// when small, are first copied to LDS; the update reads the source rows with
// independent loads (unrolled over source rows).
// stage: LDS room of sbuf / ibuf; sthr: the bulk launch's staging size,
// which decides between the inverse and the substitution (the arithmetic must
// not depend on where a task runs)
template <typename T, int NT, class Sync = BlockSync>
__device__ void apply_source_direct(const DevLayout& D, const T* __restrict__ vals, T* xs, const EdgeDesc& ed,
                                    int tid, T* sbuf, int32_t* ibuf, int stage, int sthr, const int32_t* relb)
{
    const T* Us = vals + ed.uoff;
    const int32_t* rl = relb + ed.roff;
    const int lp = ed.lp, ms = ed.ms, Ws = ed.Ws, ws = ed.ws;
    const bool pl_lds = ms <= stage;
    const int32_t* pls = pl_lds ? ibuf : D.pl + ed.r0s;
    if (pl_lds) for (int b = tid; b < ms; b += NT) ibuf[b] = D.pl[ed.r0s + b];
    if (ed.ioff >= 0 && ms <= sthr && ms <= stage) {
        // multipliers from the inverse: l_c = sum_{b <= c} x_p[b] Uinv[b][c],
        // every c at once (x_p staged in LDS first)
        const T* Ui = reinterpret_cast<const T*>(D.uinv) + ed.ioff;
        Sync::bar();
        for (int b = tid; b < ms; b += NT) sbuf[b] = xs[lp + pls[b]];
        Sync::bar();
        for (int c = tid; c < ms; c += NT) {
            T acc0 = T(0), acc1 = T(0);
            int b = 0;
            // sixteen loads in flight per step
            for (; b + 16 <= c + 1; b += 16) {
                T u[16];
#pragma unroll
                for (int k = 0; k < 16; k++) u[k] = Ui[(int64_t)(b + k) * ms + c];
#pragma unroll
                for (int k = 0; k < 16; k += 2) {
                    acc0 += sbuf[b + k] * u[k];
                    acc1 += sbuf[b + k + 1] * u[k + 1];
                }
            }
            for (; b + 2 <= c + 1; b += 2) {
                acc0 += sbuf[b] * Ui[(int64_t)b * ms + c];
                acc1 += sbuf[b + 1] * Ui[(int64_t)(b + 1) * ms + c];
            }
            if (b <= c) acc0 += sbuf[b] * Ui[(int64_t)b * ms + c];
            xs[lp + pls[c]] = acc0 + acc1;
        }
        Sync::bar();
    } else {
    const bool blk_lds = ms * ms <= stage;
    if (blk_lds)
        for (int idx = tid; idx < ms * ms; idx += NT) sbuf[idx] = Us[(int64_t)(idx / ms) * Ws + idx % ms];
    Sync::bar();
    for (int b = 0; b < ms; b++) {
        const int pb = pls[b];
        const T ub = blk_lds ? sbuf[b * ms + pb] : Us[(int64_t)b * Ws + pb];
        const T lb = xs[lp + pb] / ub;
        Sync::bar();
        if (tid == 0) xs[lp + pb] = lb;
        for (int bb = b + 1 + tid; bb < ms; bb += NT) {
            const int pc = pls[bb];
            xs[lp + pc] -= lb * (blk_lds ? sbuf[b * ms + pc] : Us[(int64_t)b * Ws + pc]);
        }
        Sync::bar();
    }
    }
    const T* Ut = Us + ms;
    // wide T regions (4 NT columns or more): two columns per thread, each
    // summed as by one column alone in the loop below (even rows of the
    // source into the first partial sum, odd ones into the second, in
    // ascending order, the last ms mod 4 rows into the first), eight rows of
    // both columns loaded per step
    if (ws >= 4 * NT) {
        for (int j0 = tid; j0 < ws; j0 += 2 * NT) {
            const int j1 = j0 + NT;
            const bool two = j1 < ws;
            T a0 = T(0), a1 = T(0), c0 = T(0), c1 = T(0);
            int b = 0;
            for (; b + 8 <= ms; b += 8) {
                T u[8], w[8];
#pragma unroll
                for (int k = 0; k < 8; k++) u[k] = Ut[(int64_t)(b + k) * Ws + j0];
#pragma unroll
                for (int k = 0; k < 8; k++) w[k] = two ? Ut[(int64_t)(b + k) * Ws + j1] : T(0);
#pragma unroll
                for (int k = 0; k < 8; k += 2) {
                    const T x0 = xs[lp + pls[b + k]], x1 = xs[lp + pls[b + k + 1]];
                    a0 += x0 * u[k];
                    a1 += x1 * u[k + 1];
                    c0 += x0 * w[k];
                    c1 += x1 * w[k + 1];
                }
            }
            for (; b + 4 <= ms; b += 4) {
                T u[4], w[4];
#pragma unroll
                for (int k = 0; k < 4; k++) u[k] = Ut[(int64_t)(b + k) * Ws + j0];
#pragma unroll
                for (int k = 0; k < 4; k++) w[k] = two ? Ut[(int64_t)(b + k) * Ws + j1] : T(0);
#pragma unroll
                for (int k = 0; k < 4; k += 2) {
                    const T x0 = xs[lp + pls[b + k]], x1 = xs[lp + pls[b + k + 1]];
                    a0 += x0 * u[k];
                    a1 += x1 * u[k + 1];
                    c0 += x0 * w[k];
                    c1 += x1 * w[k + 1];
                }
            }
            for (; b < ms; b++) {
                const T x0 = xs[lp + pls[b]];
                a0 += x0 * Ut[(int64_t)b * Ws + j0];
                if (two) c0 += x0 * Ut[(int64_t)b * Ws + j1];
            }
            xs[rl[j0]] -= a0 + a1;
            if (two) xs[rl[j1]] -= c0 + c1;
        }
    } else {
        for (int j = tid; j < ws; j += NT) {
            T acc0 = T(0), acc1 = T(0);
            const int rj = rl[j];
            int b = 0;
            // sixteen loads in flight per step
            for (; b + 16 <= ms; b += 16) {
                T u[16];
#pragma unroll
                for (int k = 0; k < 16; k++) u[k] = Ut[(int64_t)(b + k) * Ws + j];
#pragma unroll
                for (int k = 0; k < 16; k += 2) {
                    acc0 += xs[lp + pls[b + k]] * u[k];
                    acc1 += xs[lp + pls[b + k + 1]] * u[k + 1];
                }
            }
            for (; b + 4 <= ms; b += 4) {
                const T u0 = Ut[(int64_t)(b + 0) * Ws + j];
                const T u1 = Ut[(int64_t)(b + 1) * Ws + j];
                const T u2 = Ut[(int64_t)(b + 2) * Ws + j];
                const T u3 = Ut[(int64_t)(b + 3) * Ws + j];
                acc0 += xs[lp + pls[b + 0]] * u0;
                acc1 += xs[lp + pls[b + 1]] * u1;
                acc0 += xs[lp + pls[b + 2]] * u2;
                acc1 += xs[lp + pls[b + 3]] * u3;
            }
            for (; b < ms; b++) acc0 += xs[lp + pls[b]] * Ut[(int64_t)b * Ws + j];
            xs[rj] -= acc0 + acc1;
        }
    }
    Sync::bar();
}

// row updates of target row i by a block of NT threads.  Every source node (a
// standalone row: row-row kernel; a supernode: sup-row kernel) is applied in
// ascending order.  Standalone sources are staged in batches in LDS (pivot,
// the source's U values and their relative positions in the target), then
// applied one after the other from LDS.  The row's accumulator sits in LDS
// when it fits.
template <typename T, int NT>
__device__ void row_task(const DevLayout& D, T* __restrict__ vals, int i, int32_t lds_cap, T tau,
                         int32_t* __restrict__ pert, unsigned char* smem_raw, int stage,
                         int64_t eb = -1, int64_t ee = -1)
{
    T* sval = reinterpret_cast<T*>(smem_raw);                                   // stage
    int32_t* sidx = reinterpret_cast<int32_t*>(sval + stage);                  // stage
    int32_t* eoff = sidx + stage;                                               // 65 (padded to 66)
    int32_t* elp = eoff + 66;                                                   // 64
    int64_t* eu = reinterpret_cast<int64_t*>(elp + 64);                         // 64, 8-byte aligned
    int64_t* er = eu + 64;                                                      // 64
    T* xsl = reinterpret_cast<T*>(er + 64);                                     // lds_cap
    __shared__ int s_nb, s_total;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int v = D.row_node[i];
    const int W = D.W[v];
    const int a = i - D.r0[v];
    T* X = vals + D.voff[v] + (int64_t)a * W;
    // a compact row (a dense-tail row too wide for LDS whose touched
    // positions fit): the accumulator holds only the positions its outside
    // sources touch, cp[j] for entry j, and the sources' compact relative maps
    // index that list (a row that fits whole keeps its plain contiguous loads)
    const int Wc = D.cw ? D.cw[v] : 0;
    const bool compact = Wc > 0 && Wc <= lds_cap && W > lds_cap;
    const int32_t* cp = compact ? D.cpos + D.cpos_off[v] : nullptr;
    const int32_t* relb = compact ? D.crel : D.rel;
    const int Wl = compact ? Wc : W;
    const bool in_lds = Wl <= lds_cap;
    T* xs = in_lds ? xsl : X;
    if (in_lds) {
        // eight loads per thread in flight before their LDS stores (a wave
        // issues in order and would otherwise wait on every load)
        for (int j0 = tid; j0 < Wl; j0 += 8 * NT) {
            T t[8];
            int pj[8];
#pragma unroll
            for (int u = 0; u < 8; u++) { const int j = j0 + u * NT; pj[u] = j < Wl ? (cp ? cp[j] : j) : 0; }
#pragma unroll
            for (int u = 0; u < 8; u++) { const int j = j0 + u * NT; t[u] = j < Wl ? X[pj[u]] : T(0); }
#pragma unroll
            for (int u = 0; u < 8; u++) { const int j = j0 + u * NT; if (j < Wl) xs[j] = t[u]; }
        }
    }
    __syncthreads();
    // the sources [eb, ee) of the row's list (all of them by default: a long
    // row may take its sources in several launches, in order)
    const int64_t eall = D.eptr[v + 1];
    const int64_t e1 = ee >= 0 ? ee : eall;
    int64_t e = eb >= 0 ? eb : D.eptr[v];
    while (e < e1) {
        // wave 0 plans a batch: one descriptor per lane; standalone sources are staged
        if (tid < 64) {
            const int64_t my = e + lane;
            EdgeDesc ed;
            int cost = 0x3fffffff;
            if (my < e1) {
                ed = D.edges[my];
                if (ed.ms == 1) cost = ed.ws + 1;
            }
            int pre = cost;
            for (int off = 1; off < 64; off <<= 1) {
                int o = __shfl_up(pre, off, 64);
                if (lane >= off) pre = (pre > 0x3fffffff - o) ? 0x3fffffff : pre + o;
            }
            const unsigned long long fits = __ballot(pre <= stage && my < e1);
            const int nb = (fits == ~0ull) ? 64 : __builtin_ctzll(~fits);
            if (lane < nb) {
                eoff[lane] = pre - cost;
                elp[lane] = ed.lp;
                eu[lane] = ed.uoff;
                er[lane] = ed.roff;
            }
            if (lane == 0) {
                s_nb = nb;
                s_total = nb > 0 ? 0 : -1;
            }
            if (nb > 0 && lane == nb - 1) { eoff[nb] = pre; s_total = pre; }
        }
        __syncthreads();
        const int nb = s_nb, total = s_total;
        if (nb == 0) {
            // a supernode source (or an oversized standalone one)
            const EdgeDesc e0 = D.edges[e];
            apply_source_direct<T, NT>(D, vals, xs, e0, tid, sval, sidx, stage, stage, relb);
            e += 1;
            continue;
        }
        // eight entries per thread at a time: their loads are all issued
        // before the first LDS store
        for (int i0 = tid; i0 < total; i0 += 8 * NT) {
            T sv[8];
            int32_t si[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int idx = i0 + u * NT;
                sv[u] = T(0);
                si[u] = 0;
                if (idx < total) {
                    int lo = 0, hi = nb - 1;         // edge j with eoff[j] <= idx < eoff[j+1]
                    while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (eoff[mid] <= idx) lo = mid; else hi = mid - 1; }
                    const int tt = idx - eoff[lo];
                    sv[u] = vals[eu[lo] + tt];       // pivot, then the T values
                    if (tt > 0) si[u] = relb[er[lo] + tt - 1];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int idx = i0 + u * NT;
                if (idx < total) { sval[idx] = sv[u]; sidx[idx] = si[u]; }
            }
        }
        __syncthreads();
        // sequential part: every source needs the multipliers of the earlier ones
        for (int j = 0; j < nb; j++) {
            const int off = eoff[j];
            const int ws = eoff[j + 1] - off - 1;
            const int lp = elp[j];
            // every thread forms l; the multiplier is stored after the barrier
            // below (no later source of the batch touches this position: its
            // columns lie right of its own pivot, so right of this one)
            const T l = xs[lp] / sval[off];
            // the accumulator values first, then the updates (distinct
            // positions within one source)
            for (int q0 = tid; q0 < ws; q0 += 4 * NT) {
                T xv[4];
                int ix[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int q = q0 + u * NT;
                    ix[u] = q < ws ? sidx[off + 1 + q] : 0;
                    xv[u] = q < ws ? xs[ix[u]] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int q = q0 + u * NT;
                    if (q < ws) xs[ix[u]] = xv[u] - l * sval[off + 1 + q];
                }
            }
            __syncthreads();
            if (tid == 0) xs[lp] = l;
        }
        __syncthreads();
        e += nb;
    }
    if (D.m[v] == 1 && v < D.tail_node0 && e1 == eall && tid == 0) {
        // standalone row: no pivot search (Sec. 2.2), perturbation only
        T d = xs[D.lw[v]];
        if (tabs(d) < tau) {
            xs[D.lw[v]] = d < T(0) ? -tau : tau;
            atomicAdd(pert, 1);
        }
    }
    __syncthreads();
    if (in_lds) {
        for (int j = tid; j < Wl; j += NT) X[cp ? cp[j] : j] = xs[j];
    }
}

// standalone rows without sources: their pivot is checked (and perturbed)
// in place, one thread per row
template <typename T>
__global__ __launch_bounds__(256) void k_perturb_rows(DevLayout D, T* __restrict__ vals, const int32_t* __restrict__ rows,
                                                      int32_t count, T tau, int32_t* __restrict__ pert)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    const int v = D.row_node[rows[q]];
    T* d = vals + D.voff[v] + D.lw[v];
    const T x = *d;
    if (tabs(x) < tau) {
        *d = x < T(0) ? -tau : tau;
        atomicAdd(pert, 1);
    }
}

// ----------------------------------------------------------------------------
// inverse of a supernode's block in pivot order, once its LU is complete: one
// workgroup per supernode, thread j solving U_pp x = e_j by back substitution
// for column j of the inverse (U_pp staged in LDS when it fits)
// inverse of a supernode's block in pivot order, U_pp(i, k) = U(i, pl_k)
// (upper triangular), X = U_pp^{-1} row-major m x m: a wavefront per column
// j of X.  Lane l holds x[l + 64 u]; from i = j down to 0 the lane holding
// x_i divides it by U_pp(i, i) and every lane takes x_i (a lane read) off its
// entries above i, with column i of U_pp loaded one step ahead.
template <typename T>
__global__ __launch_bounds__(256) void k_sn_inverse(DevLayout D, const T* __restrict__ vals,
                                                    const int32_t* __restrict__ nodes, const int64_t* __restrict__ inv_off,
                                                    T* __restrict__ uinv, int32_t cpb)
{
    static_assert(kInvMax <= 256, "four entries per lane");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v = nodes[blockIdx.x / cpb];
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int j = (blockIdx.x % cpb) * 4 + wv;
    if (j >= m) return;
    const T* P = vals + D.voff[v] + lw;
    const int32_t* pl = D.pl + r0;
    T* X = uinv + inv_off[v];
    T x[4], uc[4], un[4];
#pragma unroll
    for (int u = 0; u < 4; u++) x[u] = lane + 64 * u == j ? T(1) : T(0);
    // column i of U_pp, rows 0..i: U(k, pl_i) for the lane's k
    auto load_col = [&](int i, T* dst) {
        const int pc = pl[i];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = lane + 64 * u;
            dst[u] = k <= i ? P[(int64_t)k * W + pc] : T(0);
        }
    };
    load_col(j, uc);
    for (int i = j; i >= 0; i--) {
        if (i > 0) load_col(i - 1, un);
        const int ui = i >> 6, li = i & 63;
        // the owner of x_i divides by the diagonal; everyone reads it
        T xi = T(0), di = T(0);
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (u == ui) { xi = x[u]; di = uc[u]; }
        xi = xi / di;
        const T q = rlane(xi, li);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = lane + 64 * u;
            if (k == i) x[u] = q;
            else if (k < i) x[u] -= uc[u] * q;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) uc[u] = un[u];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int k = lane + 64 * u;
        if (k < m) X[(int64_t)k * m + j] = k <= j ? x[u] : T(0);
    }
}

// ----------------------------------------------------------------------------
// internal factorisation of a supernode once every external update is in:
// dense LU of the m x (m + w) block+T part, row by row, each row pivoting on
// the largest entry among its block columns not yet taken (ties: lowest
// column), perturbing small pivots, then eliminating the rows below.
// ----------------------------------------------------------------------------

template <typename T, int NT, class Sync = BlockSync>
__device__ void snlu_node(const DevLayout& D, T* __restrict__ vals, int v, T tau, int32_t* __restrict__ pert,
                          int search, T* lrow, uint8_t* taken, T* red_v, int* red_i, int* s_p, int tid)
{
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int wc = W - lw;                     // block + T columns
    T* P = vals + D.voff[v] + lw;              // row a, column c at P[a*W + c]
    int32_t* pl = D.pl + r0;
    for (int c = tid; c < m; c += NT) taken[c] = 0;
    Sync::bar();
    for (int a = 0; a < m; a++) {
        T* Pa = P + (int64_t)a * W;
        int p;
        if (search) {
            T best = T(-1);
            int bi = m;
            for (int c = tid; c < m; c += NT) {
                if (taken[c]) continue;
                T x = pmag(Pa[c]);
                if (x > best || (x == best && c < bi)) { best = x; bi = c; }
            }
            red_v[tid] = best; red_i[tid] = bi;
            Sync::bar();
            for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
                if (tid < s2) {
                    T x = red_v[tid + s2]; int xi = red_i[tid + s2];
                    if (x > red_v[tid] || (x == red_v[tid] && xi < red_i[tid])) { red_v[tid] = x; red_i[tid] = xi; }
                }
                Sync::bar();
            }
            p = red_i[0];
        } else {
            p = pl[a];
        }
        if (tid == 0) {
            T d = Pa[p];
            if (tabs(d) < tau) {
                Pa[p] = d < T(0) ? -tau : tau;
                atomicAdd(pert, 1);
            }
            pl[a] = p;
            D.qinv[r0 + p] = r0 + a;
            taken[p] = 1;
            *s_p = p;
        }
        Sync::bar();
        p = *s_p;
        const T d = Pa[p];
        for (int r = a + 1 + tid; r < m; r += NT) {
            T* Pr = P + (int64_t)r * W;
            T l = Pr[p] / d;
            Pr[p] = l;
            lrow[r] = l;
        }
        Sync::bar();
        for (int c = tid; c < wc; c += NT) {
            if (c < m && taken[c]) continue;
            const T u = Pa[c];
            for (int r = a + 1; r < m; r++) P[(int64_t)r * W + c] -= lrow[r] * u;
        }
        Sync::bar();
    }
}

// The same LU for a supernode of at most kSnLds rows, its block in LDS: the
// block is factored as above (the same operations in the same order), then
// every column c past the block is finished by one thread with the forward
// substitution x_r = B_rc - sum_{a < r} l_ra x_a in a = 0, 1, .., which is the
// sequence of updates the row-by-row elimination applies to that column; the
// panel is read and written once instead of once per pivot step.  blk, lm:
// m x m each (lm: the multipliers in pivot order), lrow m, pls m, taken m.
constexpr int kSnLds = 64;
template <typename T, int NT>
__device__ void snlu_node_lds(const DevLayout& D, T* __restrict__ vals, int v, T tau, int32_t* __restrict__ pert,
                              int search, T* blk, T* lm, T* lrow, int* pls, uint8_t* taken, T* red_v, int* red_i,
                              int* s_p, int tid)
{
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int wc = W - lw;                     // block + T columns
    T* P = vals + D.voff[v] + lw;              // row a, column c at P[a*W + c]
    int32_t* pl = D.pl + r0;
    for (int idx = tid; idx < m * m; idx += NT) blk[idx] = P[(int64_t)(idx / m) * W + idx % m];
    for (int c = tid; c < m; c += NT) taken[c] = 0;
    __syncthreads();
    for (int a = 0; a < m; a++) {
        T* Ba = blk + a * m;
        int p;
        if (search) {
            T best = T(-1);
            int bi = m;
            for (int c = tid; c < m; c += NT) {
                if (taken[c]) continue;
                T x = pmag(Ba[c]);
                if (x > best || (x == best && c < bi)) { best = x; bi = c; }
            }
            red_v[tid] = best; red_i[tid] = bi;
            __syncthreads();
            for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
                if (tid < s2) {
                    T x = red_v[tid + s2]; int xi = red_i[tid + s2];
                    if (x > red_v[tid] || (x == red_v[tid] && xi < red_i[tid])) { red_v[tid] = x; red_i[tid] = xi; }
                }
                __syncthreads();
            }
            p = red_i[0];
        } else {
            p = pl[a];
        }
        if (tid == 0) {
            T d = Ba[p];
            if (tabs(d) < tau) {
                Ba[p] = d < T(0) ? -tau : tau;
                atomicAdd(pert, 1);
            }
            pl[a] = p;
            D.qinv[r0 + p] = r0 + a;
            taken[p] = 1;
            pls[a] = p;
            *s_p = p;
        }
        __syncthreads();
        p = *s_p;
        const T d = Ba[p];
        for (int r = a + 1 + tid; r < m; r += NT) {
            const T l = blk[r * m + p] / d;
            blk[r * m + p] = l;
            lrow[r] = l;
        }
        __syncthreads();
        for (int idx = tid; idx < (m - a - 1) * m; idx += NT) {
            const int r = a + 1 + idx / m, c = idx % m;
            if (taken[c]) continue;
            blk[r * m + c] -= lrow[r] * Ba[c];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < m * m; idx += NT) {
        const int r = idx / m, a = idx % m;
        P[(int64_t)r * W + a] = blk[idx];
        lm[idx] = a < r ? blk[r * m + pls[a]] : T(0);
    }
    __syncthreads();
    for (int c = m + tid; c < wc; c += NT) {
        T x[kSnLds];
#pragma unroll
        for (int r = 0; r < kSnLds; r++) x[r] = r < m ? P[(int64_t)r * W + c] : T(0);
#pragma unroll
        for (int r = 1; r < kSnLds; r++) {
            if (r < m) {
                T acc = x[r];
#pragma unroll
                for (int a = 0; a < r; a++) acc -= lm[r * m + a] * x[a];
                x[r] = acc;
            }
        }
#pragma unroll
        for (int r = 1; r < kSnLds; r++)
            if (r < m) P[(int64_t)r * W + c] = x[r];
    }
}

// inverse of node v's block in pivot order after its LU (the rule of
// k_sn_inverse, the block read from its panel): thread j solves U_pp x = e_j
template <typename T, int NT>
__device__ void sn_inverse_node(const DevLayout& D, const T* __restrict__ vals, int v, T* __restrict__ X, int tid)
{
    const int m = D.m[v], W = D.W[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v] + D.lw[v];
    const int32_t* pl = D.pl + r0;
    for (int j = tid; j < m; j += NT) {
        for (int i = j + 1; i < m; i++) X[(int64_t)i * m + j] = T(0);
        X[(int64_t)j * m + j] = T(1) / P[(int64_t)j * W + pl[j]];
        for (int i = j - 1; i >= 0; i--) {
            const T* Pi = P + (int64_t)i * W;
            T acc = T(0);
            for (int k = i + 1; k <= j; k++) acc += Pi[pl[k]] * X[(int64_t)k * m + j];
            X[(int64_t)i * m + j] = -acc / Pi[pl[i]];
        }
    }
}

// inv_off (optional): per node, the offset of its block inverse in D.uinv, or
// -1; a node with one gets it right after its LU, in the same workgroup
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_factor_snlu(DevLayout D, T* __restrict__ vals,
                                                    const int32_t* __restrict__ nodes, int32_t count,
                                                    T tau, int32_t* __restrict__ pert, int32_t search,
                                                    const int64_t* __restrict__ inv_off)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red_v[NT];
    __shared__ int red_i[NT];
    __shared__ int s_p;
    const int v = nodes[blockIdx.x];
    const int m = D.m[v];
    if (m <= kSnLds) {
        T* blk = reinterpret_cast<T*>(smem_raw);                    // m x m
        T* lm = blk + m * m;                                        // m x m
        T* lrow = lm + m * m;                                       // m
        int* pls = reinterpret_cast<int*>(lrow + m);                // m
        uint8_t* taken = reinterpret_cast<uint8_t*>(pls + m);       // m
        snlu_node_lds<T, NT>(D, vals, v, tau, pert, search, blk, lm, lrow, pls, taken, red_v, red_i, &s_p,
                             threadIdx.x);
    } else {
        T* lrow = reinterpret_cast<T*>(smem_raw);                   // m multipliers
        uint8_t* taken = smem_raw + sizeof(T) * (size_t)m;         // m flags
        snlu_node<T, NT>(D, vals, v, tau, pert, search, lrow, taken, red_v, red_i, &s_p, threadIdx.x);
    }
    if (inv_off && inv_off[v] >= 0) {
        __syncthreads();        // the block and its pivot order are complete
        sn_inverse_node<T, NT>(D, vals, v, reinterpret_cast<T*>(const_cast<void*>(D.uinv)) + inv_off[v], threadIdx.x);
    }
}

// one row task per workgroup (bulk mode)
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_factor_rows(DevLayout D, T* __restrict__ vals,
                                                    const int32_t* __restrict__ rows, const int64_t* __restrict__ ranges,
                                                    int32_t nrows, int32_t lds_cap, T tau, int32_t* __restrict__ pert,
                                                    int32_t stage, int32_t search, const int64_t* __restrict__ inv_off,
                                                    int32_t xc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_last, s_p;
    // xc > 0: workgroups go to the eight XCDs in turn, so workgroup b takes
    // task ((b/8)/xc * 8 + b%8) * xc + (b/8)%xc: every XCD gets runs of xc
    // consecutive tasks (rows of one node, which share their sources, share
    // an L2) and the runs alternate between XCDs (the grid is a multiple of
    // 8 xc; the workgroups past the last task leave)
    int t = blockIdx.x;
    if (xc > 0) {
        const int x = t & 7, slot = t >> 3;
        t = ((slot / xc) * 8 + x) * xc + slot % xc;
    }
    if (t >= nrows) return;
    const int64_t eb = ranges ? ranges[2 * t] : -1, ee = ranges ? ranges[2 * t + 1] : -1;
    const int i = rows[t];
    row_task<T, NT>(D, vals, i, lds_cap, tau, pert, smem_raw, stage, eb, ee);
    const int v = D.row_node[i];
    if (!D.snfuse || !D.snfuse[v]) return;
    // a small supernode of this launch: the workgroup that finishes its last
    // row factors its block (and inverse).  Every row's stores are made
    // visible at device scope before its count; the last one acquires them.
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(D.sncnt + v, 1) == D.m[v] - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int m = D.m[v];
    T* red_v = reinterpret_cast<T*>(smem_raw);                      // NT
    T* lrow = red_v + NT;                                           // m
    int* red_i = reinterpret_cast<int*>(lrow + m);                  // NT
    uint8_t* taken = reinterpret_cast<uint8_t*>(red_i + NT);        // m
    snlu_node<T, NT>(D, vals, v, tau, pert, search, lrow, taken, red_v, red_i, &s_p, threadIdx.x);
    if (inv_off && inv_off[v] >= 0) {
        __syncthreads();        // the block and its pivot order are complete
        sn_inverse_node<T, NT>(D, vals, v, reinterpret_cast<T*>(const_cast<void*>(D.uinv)) + inv_off[v], threadIdx.x);
    }
    if (threadIdx.x == 0) D.sncnt[v] = 0;       // ready for the next factorisation
}

// ----------------------------------------------------------------------------
// pipeline mode (Sec. 2.2.1): the narrow levels that follow the wide ones run
// as one launch.  Workgroup 0 runs the chain: its wavefronts take the nodes of
// those levels in (level, index) order, node t by wavefront t mod nw, and a
// row waits for a source node of the launch only when it is about to apply
// it, on a flag in LDS that the source's wavefront sets once that node is
// complete (its stores released at workgroup scope first).  A row thus
// applies the sources it already has while the nodes it still needs are being
// factored, instead of waiting for their whole level.  Every wait is on a node
// of lower index, so the lowest unfinished node always has its sources and
// proceeds (every wavefront of a workgroup is resident).  A wait gives up
// after `spin` polls, raising an error flag in LDS that ends every other wait
// and a global one that the host reports: the launch always ends.  The other
// workgroups run row tasks whose sources were complete before the launch, as
// the bulk row kernel does.
// ----------------------------------------------------------------------------

struct ChainCtl {
    int32_t* flag;      // LDS: per node of the chain, nonzero once complete
    int32_t* err;       // LDS: a wait gave up
    int32_t* gerr;      // global: the same, for the host
    int32_t spin;
};

// the whole wavefront waits for chain node s (wave-uniform; < 0: nothing)
__device__ __forceinline__ void chain_wait(const ChainCtl& C, int s)
{
    if (s < 0) return;
    int it = 0;
    while (__hip_atomic_load(C.flag + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
        if (__hip_atomic_load(C.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0) break;
        if (++it > C.spin) {
            __hip_atomic_store(C.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(C.gerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// is chain node s (wave-uniform; < 0: outside the launch) complete?  A
// positive answer is followed by an acquire, as after a wait
__device__ __forceinline__ bool chain_ready(const ChainCtl& C, int s)
{
    if (s < 0) return true;
    const bool r = __hip_atomic_load(C.flag + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
    if (r) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return r;
}

// ordering of one wavefront's LDS accesses: its LDS instructions execute in
// program order, so only the compiler must keep them in place (no wait on
// loads in flight, which would stall the prefetch of the next source)
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// target row i, sources [eb, ee), by one wavefront: the operations of
// row_task, source by source in the same order with the same arithmetic (a
// standalone source that the bulk launch stages, 1 + ws <= sthr, as
// x_j - l u_j with its values read straight from global memory; any other
// source through apply_source_direct).  The row sits in xsl (LDS) when
// W <= cap.  While a standalone source is applied, the pivot and first 256
// values of the next one are already being loaded when that source is
// complete.
template <typename T>
__device__ void row_task_wave(const DevLayout& D, T* __restrict__ vals, int i, int64_t eb, int64_t ee, T* xsl,
                              int cap, T* sbuf, int32_t* ibuf, int sw, int sthr, T tau, int32_t* __restrict__ pert,
                              const ChainCtl& C, int lane)
{
    const int v = D.row_node[i];
    const int W = D.W[v];
    T* X = vals + D.voff[v] + (int64_t)(i - D.r0[v]) * W;
    const bool in_lds = W <= cap;
    T* xs = in_lds ? xsl : X;
    if (in_lds) {
        for (int j0 = lane; j0 < W; j0 += 8 * 64) {
            T t[8];
#pragma unroll
            for (int u = 0; u < 8; u++) { const int j = j0 + u * 64; t[u] = j < W ? X[j] : T(0); }
#pragma unroll
            for (int u = 0; u < 8; u++) { const int j = j0 + u * 64; if (j < W) xs[j] = t[u]; }
        }
    }
    WaveSync::bar();
    bool have = false;                  // the current source's pivot and first chunk are loaded
    T cpiv = T(0), cu[4];
    int cix[4];
    EdgeDesc ed;
    if (eb < ee) ed = D.edges[eb];
    for (int64_t e = eb; e < ee; e++) {
        if (!have) chain_wait(C, ed.srcp);
        if (ed.ms == 1 && ed.ws + 1 <= sthr) {
            const T* U = vals + ed.uoff;          // pivot, then the T values
            const int32_t* rl = D.rel + ed.roff;
            const int ws = ed.ws, lp = ed.lp;
            if (!have) {
                cpiv = U[0];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int q = lane + 64 * k;
                    cu[k] = q < ws ? U[1 + q] : T(0);
                    cix[k] = q < ws ? rl[q] : 0;
                }
            }
            // the next source: its descriptor, and its first values when it
            // is a staged standalone source that is complete already
            have = false;
            T npiv = T(0), nu[4];
            int nix[4];
            if (e + 1 < ee) {
                const EdgeDesc nx = D.edges[e + 1];
                if (nx.ms == 1 && nx.ws + 1 <= sthr && chain_ready(C, nx.srcp)) {
                    const T* Un = vals + nx.uoff;
                    const int32_t* rn = D.rel + nx.roff;
                    npiv = Un[0];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int q = lane + 64 * k;
                        nu[k] = q < nx.ws ? Un[1 + q] : T(0);
                        nix[k] = q < nx.ws ? rn[q] : 0;
                    }
                    have = true;
                }
                ed = nx;
            }
            const T l = xs[lp] / cpiv;
            {
                T xv[4];
#pragma unroll
                for (int k = 0; k < 4; k++) xv[k] = lane + 64 * k < ws ? xs[cix[k]] : T(0);
#pragma unroll
                for (int k = 0; k < 4; k++)
                    if (lane + 64 * k < ws) xs[cix[k]] = xv[k] - l * cu[k];
            }
            for (int q0 = lane + 4 * 64; q0 < ws; q0 += 4 * 64) {
                T u[4], xv[4];
                int ix[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int q = q0 + 64 * k;
                    u[k] = q < ws ? U[1 + q] : T(0);
                    ix[k] = q < ws ? rl[q] : 0;
                }
#pragma unroll
                for (int k = 0; k < 4; k++) xv[k] = q0 + 64 * k < ws ? xs[ix[k]] : T(0);
#pragma unroll
                for (int k = 0; k < 4; k++)
                    if (q0 + 64 * k < ws) xs[ix[k]] = xv[k] - l * u[k];
            }
            if (in_lds) {
                wave_lds_order();
                if (lane == 0) xs[lp] = l;
                wave_lds_order();
            } else {
                WaveSync::bar();
                if (lane == 0) xs[lp] = l;
                WaveSync::bar();
            }
            if (have) {
                cpiv = npiv;
#pragma unroll
                for (int k = 0; k < 4; k++) { cu[k] = nu[k]; cix[k] = nix[k]; }
            }
        } else {
            apply_source_direct<T, 64, WaveSync>(D, vals, xs, ed, lane, sbuf, ibuf, sw, sthr, D.rel);
            have = false;
            if (e + 1 < ee) ed = D.edges[e + 1];
        }
    }
    if (D.m[v] == 1 && v < D.tail_node0 && ee == D.eptr[v + 1] && lane == 0) {
        // standalone row: no pivot search (Sec. 2.2), perturbation only
        T d = xs[D.lw[v]];
        if (tabs(d) < tau) {
            xs[D.lw[v]] = d < T(0) ? -tau : tau;
            atomicAdd(pert, 1);
        }
    }
    WaveSync::bar();
    if (in_lds)
        for (int j = lane; j < W; j += 64) X[j] = xs[j];
    WaveSync::bar();
}

// LDS of the chain workgroup: the flags (ntask + 4 ints, 16-byte multiple),
// then per wavefront its row (cap values), sbuf (sw values), the reduction
// values (64), ibuf (sw ints), the reduction indices (64) and one int
__host__ __device__ inline size_t chain_hdr_bytes(int ntask) { return (((size_t)ntask + 4) * 4 + 15) / 16 * 16; }
__host__ __device__ inline size_t chain_wave_bytes(size_t es, int cap, int sw)
{
    return ((size_t)(cap + sw + 64) * es + (size_t)(sw + 64) * 4 + 16 + 15) / 16 * 16;
}

// tasks[t] >= 0: the outside updates of row tasks[t]; tasks[t] = -(v + 1):
// the block LU (and inverse) of supernode v, whose row tasks (when it has
// sources) are the m tasks just before it.  A node is complete with its
// last task (the row task of a standalone row, the LU task of a supernode),
// whose index is what its targets wait on.
template <typename T>
__global__ __launch_bounds__(kChainThreads) void k_factor_chain(DevLayout D, T* __restrict__ vals,
                                                       const int32_t* __restrict__ tasks,
                                                       const int32_t* __restrict__ sthr_of, int32_t ntask, int32_t nw,
                                                       int32_t cap, int32_t sw, T tau, int32_t* __restrict__ pert,
                                                       int32_t search, const int64_t* __restrict__ inv_off, int32_t spin)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int32_t* flag = reinterpret_cast<int32_t*>(smem_raw);
    int32_t* err = flag + ntask;
    for (int t = threadIdx.x; t < ntask + 4; t += kChainThreads) flag[t] = 0;
    __syncthreads();        // the only block barrier: the wavefronts then run apart
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wv >= nw) return;
    unsigned char* base = smem_raw + chain_hdr_bytes(ntask) + (size_t)wv * chain_wave_bytes(sizeof(T), cap, sw);
    T* xs = reinterpret_cast<T*>(base);
    T* sbuf = xs + cap;
    T* red_v = sbuf + sw;
    int32_t* ibuf = reinterpret_cast<int32_t*>(red_v + 64);
    int32_t* red_i = ibuf + sw;
    int32_t* s_p = red_i + 64;
    const ChainCtl C{flag, err, pert + 1, spin};
    T* uinv = reinterpret_cast<T*>(const_cast<void*>(D.uinv));
    for (int t = wv; t < ntask; t += nw) {
        const int x = tasks[t];
        if (x >= 0) {
            const int v = D.row_node[x];
            row_task_wave<T>(D, vals, x, D.eptr[v], D.eptr[v + 1], xs, cap, sbuf, ibuf, sw, sthr_of[t], tau, pert, C,
                             lane);
        } else {
            const int v = -x - 1;
            const int m = D.m[v];
            if (D.eptr[v + 1] > D.eptr[v])
                for (int a = 0; a < m; a++) chain_wait(C, t - m + a);
            snlu_node<T, 64, WaveSync>(D, vals, v, tau, pert, search, sbuf, reinterpret_cast<uint8_t*>(ibuf), red_v,
                                       red_i, s_p, lane);
            if (inv_off && inv_off[v] >= 0) {
                WaveSync::bar();
                sn_inverse_node<T, 64>(D, vals, v, uinv + inv_off[v], lane);
            }
        }
        // publish: the task's stores, then its flag
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) __hip_atomic_store(flag + t, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// ----------------------------------------------------------------------------
// triangular solves, one wavefront per node of a level
// ----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return __shfl(x, 0, 64);
}

// broadcast of a lane's value (the lane index must be wave-uniform)
__device__ __forceinline__ double bcast(double x, int l)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bcast(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// sum over t = lane, lane + 64, .. < len of P[t] * y[qinv[cols[t]]]: four
// entries per lane at a time, each dependent load issued for all four before
// the next (a wave waits on a load at its first use)
template <typename T, int S = 64>
__device__ __forceinline__ T gather_lq(const T* __restrict__ P, const int32_t* __restrict__ cols,
                                       const int32_t* __restrict__ qinv, const T* __restrict__ y, int len, int lane)
{
    T acc = T(0);
    for (int t0 = lane; t0 < len; t0 += 4 * S) {
        int c[4];
        T p[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int t = t0 + S * u;
            c[u] = t < len ? cols[t] : 0;
            p[u] = t < len ? P[t] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = t0 + S * u < len ? qinv[c[u]] : 0;
#pragma unroll
        for (int u = 0; u < 4; u++) x[u] = t0 + S * u < len ? y[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) acc += p[u] * x[u];
    }
    return acc;
}

// the same with a direct index: P[t] * x[cols[t]]
template <typename T, int S = 64>
__device__ __forceinline__ T gather_x(const T* __restrict__ P, const int32_t* __restrict__ cols, const T* __restrict__ x,
                                      int len, int lane)
{
    T acc = T(0);
    for (int t0 = lane; t0 < len; t0 += 4 * S) {
        int c[4];
        T p[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int t = t0 + S * u;
            c[u] = t < len ? cols[t] : 0;
            p[u] = t < len ? P[t] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) xv[u] = t0 + S * u < len ? x[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) acc += p[u] * xv[u];
    }
    return acc;
}

// chunk staging for the node solves: out[t] = y[qinv[cols[t]]] (forward) or
// x[cols[t]] (backward), t < len, NT threads, four loads per thread in flight
constexpr int kSolveChunk = 1024;
constexpr int kChainChunk = 256;     // per wavefront in the solve chains
template <typename T, int NT>
__device__ __forceinline__ void stage_lq(const int32_t* __restrict__ cols, const int32_t* __restrict__ qinv,
                                         const T* __restrict__ y, int len, int tid, T* out)
{
    for (int t0 = tid; t0 < len; t0 += 4 * NT) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = t0 + NT * u < len ? cols[t0 + NT * u] : 0;
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = t0 + NT * u < len ? qinv[c[u]] : 0;
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = t0 + NT * u < len ? y[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) if (t0 + NT * u < len) out[t0 + NT * u] = v[u];
    }
}
template <typename T, int NT>
__device__ __forceinline__ void stage_x(const int32_t* __restrict__ cols, const T* __restrict__ x, int len, int tid,
                                        T* out)
{
    for (int t0 = tid; t0 < len; t0 += 4 * NT) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = t0 + NT * u < len ? cols[t0 + NT * u] : 0;
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = t0 + NT * u < len ? x[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 4; u++) if (t0 + NT * u < len) out[t0 + NT * u] = v[u];
    }
}

// sum over q = q0 + lane, .. < q1 (stride S) of vals[slot[q]] * w[row[q]],
// four entries per lane at a time with their dependent loads issued together
template <typename T, int S>
__device__ __forceinline__ T gather_sr(const T* __restrict__ vals, const int64_t* __restrict__ slot,
                                       const int32_t* __restrict__ row, const T* __restrict__ w, int64_t q0, int64_t q1,
                                       int lane)
{
    T acc = T(0);
    for (int64_t b = q0 + lane; b < q1; b += 4 * S) {
        int64_t sl[4];
        int32_t rw[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t q = b + S * u;
            sl[u] = q < q1 ? slot[q] : 0;
            rw[u] = q < q1 ? row[q] : 0;
        }
        T p[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const bool ok = b + S * u < q1;
            p[u] = ok ? vals[sl[u]] : T(0);
            x[u] = ok ? w[rw[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) acc += p[u] * x[u];
    }
    return acc;
}

// forward: y_i = c_i - sum_k L(i,k) y_k (unit L), rows of a node in order
template <typename T>
__global__ __launch_bounds__(64) void k_lsolve(DevLayout D, const T* __restrict__ vals,
                                               const int32_t* __restrict__ nodes, int32_t count,
                                               T* __restrict__ y, int32_t nrhs, int32_t sn_min)
{
    const int v = nodes[blockIdx.x];
    if (D.dense_sn && D.dense_sn[v]) return;     // solved by the dense-view kernels
    const int lane = threadIdx.x;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    if (sn_min > 0 && m >= sn_min && m <= kSnSolveRows) return;   // solved by k_lsolve_sn
    const T* P = vals + D.voff[v];
    const int32_t* cols = D.cols + D.coff[v];
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n;
        for (int a = 0; a < m; a++) {
            const T* Pa = P + (int64_t)a * W;
            T acc = gather_lq(Pa, cols, D.qinv, yr, lw, lane);
            for (int b = lane; b < a; b += 64) acc += Pa[lw + pl[b]] * yr[r0 + b];
            acc = wave_sum(acc);
            if (lane == 0) yr[r0 + a] -= acc;
            __syncthreads();
        }
    }
}

// forward solve of a supernode with at least sn_min rows on four wavefronts:
// the rows' gathers over the L region are independent and run first, spread
// over the wavefronts; the unit-lower block (row a's multiplier for an earlier
// row b at b's pivot column) is then swept column by column on wavefront 0,
// one lane per row, with the block staged in LDS.  pre = 1: the outside sums
// were already subtracted from y by k_lsolve_out (only the block is swept)
template <typename T>
__global__ __launch_bounds__(256) void k_lsolve_sn(DevLayout D, const T* __restrict__ vals,
                                                   const int32_t* __restrict__ nodes, int32_t count,
                                                   T* __restrict__ y, int32_t nrhs, int32_t sn_min, int32_t pre)
{
    __shared__ T Lb[kSnSolveRows][kSnSolveRows + 1];   // Lb[r][b] = L(r, b), b < r
    __shared__ T ys[kSnSolveRows];
    __shared__ T ychunk[kSolveChunk];
    const int v = nodes[blockIdx.x];
    if (D.dense_sn && D.dense_sn[v]) return;
    const int m = D.m[v];
    if (m < sn_min || m > kSnSolveRows) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int lwo = pre ? 0 : lw;        // columns of the outside sums done here
    const T* P = vals + D.voff[v];
    const int32_t* cols = D.cols + D.coff[v];
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int idx = tid; idx < m * m; idx += 256) {
        const int r = idx / m, b = idx - (idx / m) * m;
        Lb[r][b] = b < r ? P[(int64_t)r * W + lw + pl[b]] : T(0);
    }
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n;
        // the outside values every row of the node multiplies, y at the rows
        // pivoting on its L columns, staged once per chunk (each lane still
        // sums its entries t = lane + 64 k in ascending order)
        T acc[kSnSolveRows / 4];
#pragma unroll
        for (int i = 0; i < kSnSolveRows / 4; i++) acc[i] = T(0);
        for (int c0 = 0; c0 < lwo; c0 += kSolveChunk) {
            const int nc = min(kSolveChunk, lwo - c0);
            stage_lq<T, 256>(cols + c0, D.qinv, yr, nc, tid, ychunk);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kSnSolveRows / 4; i++) {
                const int a = wv + 4 * i;
                if (a < m) {
                    const T* Pa = P + (int64_t)a * W + c0;
                    for (int t = lane; t < nc; t += 64) acc[i] += Pa[t] * ychunk[t];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kSnSolveRows / 4; i++) {
            const int a = wv + 4 * i;
            if (a < m) {
                const T s = wave_sum(acc[i]);
                if (lane == 0) ys[a] = yr[r0 + a] - s;
            }
        }
        __syncthreads();
        if (wv == 0) {
            T va = lane < m ? ys[lane] : T(0);
            for (int b = 0; b < m; b++) {
                const T yb = bcast(va, b);
                if (lane > b && lane < m) va -= Lb[lane][b] * yb;
            }
            if (lane < m) yr[r0 + lane] = va;
        }
        __syncthreads();
    }
}

// the outside sums of the forward solve of a supernode with a long L region,
// spread over workgroups by groups of kSplitRows rows (task: node, first
// row), two rows per wavefront: row a subtracts sum_k L(a,k) y_k from y_a in
// place, each lane summing its entries t = lane + 64 j in ascending order as
// k_lsolve_sn does, so that k_lsolve_sn (pre = 1) finishing the block gives
// the same values to the bit
template <typename T>
__global__ __launch_bounds__(256) void k_lsolve_out(DevLayout D, const T* __restrict__ vals,
                                                    const int32_t* __restrict__ tasks, int32_t count,
                                                    T* __restrict__ y, int32_t nrhs)
{
    __shared__ T ychunk[kSolveChunk];
    const int v = tasks[2 * blockIdx.x], g0 = tasks[2 * blockIdx.x + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v];
    const int32_t* cols = D.cols + D.coff[v];
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n;
        T acc[kSplitRows / 4];
#pragma unroll
        for (int i = 0; i < kSplitRows / 4; i++) acc[i] = T(0);
        for (int c0 = 0; c0 < lw; c0 += kSolveChunk) {
            const int nc = min(kSolveChunk, lw - c0);
            stage_lq<T, 256>(cols + c0, D.qinv, yr, nc, tid, ychunk);
            __syncthreads();
            // four entries of each row per lane loaded before they are used
            for (int t0 = lane; t0 < nc; t0 += 256) {
                T p[kSplitRows / 4][4];
#pragma unroll
                for (int i = 0; i < kSplitRows / 4; i++) {
                    const int a = g0 + wv + 4 * i;
                    const T* Pa = P + (int64_t)min(a, m - 1) * W + c0;
#pragma unroll
                    for (int u = 0; u < 4; u++) p[i][u] = a < m && t0 + 64 * u < nc ? Pa[t0 + 64 * u] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (t0 + 64 * u >= nc) break;
                    const T yv = ychunk[t0 + 64 * u];
#pragma unroll
                    for (int i = 0; i < kSplitRows / 4; i++) acc[i] += p[i][u] * yv;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kSplitRows / 4; i++) {
            const int a = g0 + wv + 4 * i;
            if (a < m) {
                const T s = wave_sum(acc[i]);
                if (lane == 0) yr[r0 + a] -= s;
            }
        }
    }
}

// The long chain of narrow levels of the big triangle, solved sequentially
// (Sec. 2.3, Fig. 3) in one launch: one workgroup walks the levels [l0, l1)
// in order with a barrier between consecutive levels; inside a level every
// wavefront takes a node (nodes of at most kChainRows rows), its rows in order
// with the node's solved values kept in LDS, written out at the end.
// forward: y_i = c_i - sum_k L(i,k) y_k
template <typename T>
__global__ __launch_bounds__(64 * kChainWaves) void k_lsolve_chain(DevLayout D, const T* __restrict__ vals,
                                                                   const int32_t* __restrict__ lev_ptr,
                                                                   const int32_t* __restrict__ nodes, int32_t l0,
                                                                   int32_t l1, T* __restrict__ y, int32_t nrhs)
{
    __shared__ T ys[kChainWaves][kChainRows];
    __shared__ T yc[kChainWaves][kChainChunk];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = D.n;
    for (int l = l0; l < l1; l++) {
        const int q1 = lev_ptr[l + 1];
        for (int q = lev_ptr[l] + wv; q < q1; q += kChainWaves) {
            const int v = nodes[q];
            const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
            const T* P = vals + D.voff[v];
            const int32_t* cols = D.cols + D.coff[v];
            const int32_t* pl = D.pl + r0;
            const int myp = lane < m ? pl[lane] : 0;
            for (int r = 0; r < nrhs; r++) {
                T* yr = y + (int64_t)r * n;
                // a node of several rows: the outside values its rows share
                // staged once per chunk, eight rows' sums at a time (each lane
                // in the same order as the direct gather)
                for (int g0 = 0; g0 < m; g0 += 8) {
                    T acc[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) acc[i] = T(0);
                    if (m == 1) {
                        acc[0] = gather_lq(P, cols, D.qinv, yr, lw, lane);
                    } else {
                        for (int c0 = 0; c0 < lw; c0 += kChainChunk) {
                            const int nc = min(kChainChunk, lw - c0);
                            stage_lq<T, 64>(cols + c0, D.qinv, yr, nc, lane, yc[wv]);
                            __builtin_amdgcn_wave_barrier();
#pragma unroll
                            for (int i = 0; i < 8; i++) {
                                if (g0 + i < m) {
                                    const T* Pa = P + (int64_t)(g0 + i) * W + c0;
                                    for (int t = lane; t < nc; t += 64) acc[i] += Pa[t] * yc[wv][t];
                                }
                            }
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        const int a = g0 + i;
                        if (a >= m) break;
                        const T* Pa = P + (int64_t)a * W;
                        T s = acc[i];
                        if (lane < a) s += Pa[lw + myp] * ys[wv][lane];
                        s = wave_sum(s);
                        if (lane == 0) ys[wv][a] = yr[r0 + a] - s;
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                if (lane < m) yr[r0 + lane] = ys[wv][lane];
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    }
}

// backward: x[piv a] = (y_a - sum_{j != piv a} U_st(a,j) x_j) / U_st(a, piv a),
// the node's rows from the last, its values by local column in LDS
template <typename T>
__global__ __launch_bounds__(64 * kChainWaves) void k_usolve_chain(DevLayout D, const T* __restrict__ vals,
                                                                   const int32_t* __restrict__ lev_ptr,
                                                                   const int32_t* __restrict__ nodes, int32_t l0,
                                                                   int32_t l1, const T* __restrict__ y,
                                                                   T* __restrict__ x, int32_t nrhs)
{
    __shared__ T xs[kChainWaves][kChainRows];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = D.n;
    for (int l = l0; l < l1; l++) {
        const int q1 = lev_ptr[l + 1];
        for (int q = lev_ptr[l] + wv; q < q1; q += kChainWaves) {
            const int v = nodes[q];
            const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
            const int w = W - lw - m;
            const T* P = vals + D.voff[v] + lw;
            const int32_t* tc = D.cols + D.coff[v] + lw + m;
            const int32_t* pl = D.pl + r0;
            const int myp = lane < m ? pl[lane] : 0;
            for (int r = 0; r < nrhs; r++) {
                const T* yr = y + (int64_t)r * n;
                T* xr = x + (int64_t)r * n;
                for (int a = m - 1; a >= 0; a--) {
                    const T* Pa = P + (int64_t)a * W;
                    T acc = gather_x(Pa + m, tc, xr, w, lane);
                    if (lane > a && lane < m) acc += Pa[myp] * xs[wv][myp];
                    acc = wave_sum(acc);
                    if (lane == 0) {
                        const int c = pl[a];
                        xs[wv][c] = (yr[r0 + a] - acc) / Pa[c];
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                if (lane < m) xr[r0 + lane] = xs[wv][lane];
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    }
}

// backward: x[piv a] = (y_a - sum_{j != piv a} U_st(a,j) x_j) / U_st(a, piv a);
// the four wavefronts of the workgroup share each row's gather
template <typename T>
__global__ __launch_bounds__(256) void k_usolve(DevLayout D, const T* __restrict__ vals,
                                                const int32_t* __restrict__ nodes, int32_t count,
                                                const T* __restrict__ y, T* __restrict__ x, int32_t nrhs, int32_t sn_min)
{
    __shared__ T part[4];
    const int v = nodes[blockIdx.x];
    if (D.dense_sn && D.dense_sn[v]) return;     // solved by the dense-view kernels
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    if (sn_min > 0 && m >= sn_min && m <= kSnSolveRows) return;   // solved by k_usolve_sn
    const int w = W - lw - m;
    const T* P = vals + D.voff[v] + lw;
    const int32_t* tc = D.cols + D.coff[v] + lw + m;
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        const T* yr = y + (int64_t)r * n;
        T* xr = x + (int64_t)r * n;
        for (int a = m - 1; a >= 0; a--) {
            const T* Pa = P + (int64_t)a * W;
            T acc = gather_x<T, 256>(Pa + m, tc, xr, w, tid);
            for (int b = a + 1 + tid; b < m; b += 256) { int c = pl[b]; acc += Pa[c] * xr[r0 + c]; }
            acc = wave_sum(acc);
            if (lane == 0) part[wv] = acc;
            __syncthreads();
            if (tid == 0) {
                const int c = pl[a];
                xr[r0 + c] = (yr[r0 + a] - ((part[0] + part[1]) + (part[2] + part[3]))) / Pa[c];
            }
            __syncthreads();
        }
    }
}

// backward solve of a supernode with sn_min..64 rows on four wavefronts: the
// rows' gathers over the shared T columns do not depend on the block and run
// first, spread over the wavefronts; the block (U_st(a, piv b), b >= a, in
// pivot order, staged in LDS) is then swept column by column from the last
// one on wavefront 0, one lane per row.  pre = 1: the gathers' sums were
// already subtracted from y by k_usolve_out (only the block is swept)
template <typename T>
__global__ __launch_bounds__(256) void k_usolve_sn(DevLayout D, const T* __restrict__ vals,
                                                   const int32_t* __restrict__ nodes, int32_t count,
                                                   const T* __restrict__ y, T* __restrict__ x, int32_t nrhs,
                                                   int32_t sn_min, int32_t pre)
{
    __shared__ T Ub[kSnSolveRows][kSnSolveRows + 1];
    __shared__ T ys[kSnSolveRows];
    __shared__ int pls[kSnSolveRows];
    __shared__ T ychunk[kSolveChunk];
    const int v = nodes[blockIdx.x];
    if (D.dense_sn && D.dense_sn[v]) return;
    const int m = D.m[v];
    if (m < sn_min || m > kSnSolveRows) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int w = pre ? 0 : W - lw - m;          // columns of the gathers done here
    const T* P = vals + D.voff[v] + lw;
    const int32_t* tc = D.cols + D.coff[v] + lw + m;
    const int n = D.n;
    if (tid < m) pls[tid] = D.pl[r0 + tid];
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += 256) {
        const int a = idx / m, b = idx - (idx / m) * m;
        Ub[a][b] = b >= a ? P[(int64_t)a * W + pls[b]] : T(0);
    }
    for (int r = 0; r < nrhs; r++) {
        const T* yr = y + (int64_t)r * n;
        T* xr = x + (int64_t)r * n;
        // x at the node's columns past its block, staged once per chunk
        T acc[kSnSolveRows / 4];
#pragma unroll
        for (int i = 0; i < kSnSolveRows / 4; i++) acc[i] = T(0);
        for (int c0 = 0; c0 < w; c0 += kSolveChunk) {
            const int nc = min(kSolveChunk, w - c0);
            stage_x<T, 256>(tc + c0, xr, nc, tid, ychunk);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kSnSolveRows / 4; i++) {
                const int a = wv + 4 * i;
                if (a < m) {
                    const T* Pa = P + (int64_t)a * W + m + c0;
                    for (int t = lane; t < nc; t += 64) acc[i] += Pa[t] * ychunk[t];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kSnSolveRows / 4; i++) {
            const int a = wv + 4 * i;
            if (a < m) {
                const T s = wave_sum(acc[i]);
                if (lane == 0) ys[a] = yr[r0 + a] - s;
            }
        }
        __syncthreads();
        if (wv == 0) {
            T va = lane < m ? ys[lane] : T(0);
            T xv = T(0);
            for (int b = m - 1; b >= 0; b--) {
                const T xb = bcast(va, b) / Ub[b][b];
                if (lane == b) xv = xb;
                if (lane < b) va -= Ub[lane][b] * xb;
            }
            if (lane < m) xr[r0 + pls[lane]] = xv;
        }
        __syncthreads();
    }
}

// the gathers of the backward solve of a supernode with many columns past its
// block, spread over workgroups of kSplitRows rows (task: node, first row),
// two rows per wavefront: row a subtracts sum_j U(a,j) x_j over those
// columns from its y_a in place (y is the solve's work vector, read by no
// one else afterwards), each lane in k_usolve_sn's order
template <typename T>
__global__ __launch_bounds__(256) void k_usolve_out(DevLayout D, const T* __restrict__ vals,
                                                    const int32_t* __restrict__ tasks, int32_t count,
                                                    T* __restrict__ y, const T* __restrict__ x, int32_t nrhs)
{
    __shared__ T xchunk[kSolveChunk];
    const int v = tasks[2 * blockIdx.x], g0 = tasks[2 * blockIdx.x + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const int w = W - lw - m;
    const T* P = vals + D.voff[v] + lw + m;
    const int32_t* tc = D.cols + D.coff[v] + lw + m;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n;
        const T* xr = x + (int64_t)r * n;
        T acc[kSplitRows / 4];
#pragma unroll
        for (int i = 0; i < kSplitRows / 4; i++) acc[i] = T(0);
        for (int c0 = 0; c0 < w; c0 += kSolveChunk) {
            const int nc = min(kSolveChunk, w - c0);
            stage_x<T, 256>(tc + c0, xr, nc, tid, xchunk);
            __syncthreads();
            for (int t0 = lane; t0 < nc; t0 += 256) {
                T p[kSplitRows / 4][4];
#pragma unroll
                for (int i = 0; i < kSplitRows / 4; i++) {
                    const int a = g0 + wv + 4 * i;
                    const T* Pa = P + (int64_t)min(a, m - 1) * W + c0;
#pragma unroll
                    for (int u = 0; u < 4; u++) p[i][u] = a < m && t0 + 64 * u < nc ? Pa[t0 + 64 * u] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (t0 + 64 * u >= nc) break;
                    const T xv = xchunk[t0 + 64 * u];
#pragma unroll
                    for (int i = 0; i < kSplitRows / 4; i++) acc[i] += p[i][u] * xv;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kSplitRows / 4; i++) {
            const int a = g0 + wv + 4 * i;
            if (a < m) {
                const T s = wave_sum(acc[i]);
                if (lane == 0) yr[r0 + a] -= s;
            }
        }
    }
}

// U_st^T w = h: w_a = (h[piv a] - sum_{k<a} U_st(k, piv a) w_k) / U_st(a, piv a)
template <typename T>
__global__ __launch_bounds__(256) void k_utsolve(DevLayout D, const T* __restrict__ vals,
                                                 const int32_t* __restrict__ nodes, int32_t count,
                                                 const T* __restrict__ h, T* __restrict__ w, int32_t nrhs)
{
    __shared__ T part[4];
    const int v = nodes[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v] + lw;
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        const T* hr = h + (int64_t)r * n;
        T* wr = w + (int64_t)r * n;
        for (int a = 0; a < m; a++) {
            const int c = r0 + pl[a];
            T acc = gather_sr<T, 256>(vals, D.ut_slot, D.ut_row, wr, D.ut_ptr[c], D.ut_ptr[c + 1], tid);
            for (int b = tid; b < a; b += 256) acc += P[(int64_t)b * W + pl[a]] * wr[r0 + b];
            acc = wave_sum(acc);
            if (lane == 0) part[wv] = acc;
            __syncthreads();
            if (tid == 0)
                wr[r0 + a] = (hr[c] - ((part[0] + part[1]) + (part[2] + part[3]))) / P[(int64_t)a * W + pl[a]];
            __syncthreads();
        }
    }
}

// L^T u = w in place: u_k = w_k - sum_{i>k} L(i,k) u_i, rows of a node in reverse
template <typename T>
__global__ __launch_bounds__(256) void k_ltsolve(DevLayout D, const T* __restrict__ vals,
                                                 const int32_t* __restrict__ nodes, int32_t count,
                                                 T* __restrict__ w, int32_t nrhs)
{
    __shared__ T part[4];
    const int v = nodes[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v] + lw;
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* wr = w + (int64_t)r * n;
        for (int a = m - 1; a >= 0; a--) {
            const int c = r0 + pl[a];          // L(i, r0+a) sits at the slot of column c
            T acc = gather_sr<T, 256>(vals, D.lt_slot, D.lt_row, wr, D.lt_ptr[c], D.lt_ptr[c + 1], tid);
            for (int b = a + 1 + tid; b < m; b += 256) acc += P[(int64_t)b * W + pl[a]] * wr[r0 + b];
            acc = wave_sum(acc);
            if (lane == 0) part[wv] = acc;
            __syncthreads();
            if (tid == 0) wr[r0 + a] -= (part[0] + part[1]) + (part[2] + part[3]);
            __syncthreads();
        }
    }
}

// Transposed solves of a node of at least 8 rows in two launches.  First the
// sums over the entries outside the node, which only need solved values of
// other nodes: for each of the node's columns c_a = r0 + piv a, by
// workgroups of kSplitRows columns (task: node, first column), two per
// wavefront, gathered through the transposed index (U^T: the entries of
// column c_a in rows of earlier nodes, against w; L^T: in rows of later
// nodes, against u) and subtracted in place (U^T: from h[c_a], h being the
// solve's work vector; L^T: from w[r0 + a]).  Then the node's own
// triangular block, 64 columns at a time (k_utsolve_blk, k_ltsolve_blk).
template <typename T, bool UT>
__global__ __launch_bounds__(256) void k_tsolve_out(DevLayout D, const T* __restrict__ vals,
                                                    const int32_t* __restrict__ tasks, int32_t count,
                                                    T* __restrict__ h, const T* __restrict__ w, int32_t nrhs)
{
    const int v = tasks[2 * blockIdx.x], g0 = tasks[2 * blockIdx.x + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = D.m[v], r0 = D.r0[v];
    const int32_t* pl = D.pl + r0;
    const int64_t* ptr = UT ? D.ut_ptr : D.lt_ptr;
    const int64_t* slot = UT ? D.ut_slot : D.lt_slot;
    const int32_t* row = UT ? D.ut_row : D.lt_row;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* hr = h + (int64_t)r * n;
        const T* wr = w + (int64_t)r * n;
#pragma unroll
        for (int i = 0; i < kSplitRows / 4; i++) {
            const int a = g0 + wv + 4 * i;
            if (a >= m) break;
            const int c = r0 + pl[a];
            T s = gather_sr<T, 64>(vals, slot, row, wr, ptr[c], ptr[c + 1], lane);
            s = wave_sum(s);
            if (lane == 0) hr[UT ? c : r0 + a] -= s;
        }
    }
}

// U^T w = h on a node's block after k_tsolve_out: columns in ascending blocks
// of 64; in a block, wavefront 0 sweeps w_a = h[c_a] / U(a, c_a) and takes
// U(a, c_k) w_a off the later columns k of the block (one lane each); the
// whole workgroup then takes the block's products off the node's later
// columns
template <typename T>
__global__ __launch_bounds__(256) void k_utsolve_blk(DevLayout D, const T* __restrict__ vals,
                                                     const int32_t* __restrict__ nodes, int32_t count,
                                                     T* __restrict__ h, T* __restrict__ w, int32_t nrhs)
{
    __shared__ T Ub[64][65];          // Ub[i][k] = U(a0+i, c_{a0+k}), k >= i
    __shared__ T wb[64];
    const int v = nodes[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v] + lw;
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    for (int r = 0; r < nrhs; r++) {
        T* hr = h + (int64_t)r * n;
        T* wr = w + (int64_t)r * n;
        for (int a0 = 0; a0 < m; a0 += 64) {
            const int mb = min(64, m - a0);
            for (int idx = tid; idx < mb * mb; idx += 256) {
                const int i = idx / mb, k = idx - (idx / mb) * mb;
                Ub[i][k] = k >= i ? P[(int64_t)(a0 + i) * W + pl[a0 + k]] : T(0);
            }
            __syncthreads();
            if (wv == 0) {
                T va = lane < mb ? hr[r0 + pl[a0 + lane]] : T(0);
                T wv0 = T(0);
                for (int i = 0; i < mb; i++) {
                    const T wi = bcast(va, i) / Ub[i][i];
                    if (lane == i) wv0 = wi;
                    if (lane > i && lane < mb) va -= Ub[i][lane] * wi;
                }
                if (lane < mb) {
                    wb[lane] = wv0;
                    wr[r0 + a0 + lane] = wv0;
                }
            }
            __syncthreads();
            for (int k = a0 + mb + tid; k < m; k += 256) {
                const int pk = pl[k];
                T acc = T(0);
                for (int i = 0; i < mb; i++) acc += P[(int64_t)(a0 + i) * W + pk] * wb[i];
                hr[r0 + pk] -= acc;
            }
            __syncthreads();
        }
    }
}

// L^T u = w on a node's block after k_tsolve_out (in place): columns in
// descending blocks of 64; in a block, wavefront 0 sweeps from the last
// column, taking L(a, k) u_a off the earlier columns k of the block; the
// whole workgroup then takes the block's products off the node's earlier
// columns
template <typename T>
__global__ __launch_bounds__(256) void k_ltsolve_blk(DevLayout D, const T* __restrict__ vals,
                                                     const int32_t* __restrict__ nodes, int32_t count,
                                                     T* __restrict__ w, int32_t nrhs)
{
    __shared__ T Lb[64][65];          // Lb[i][k] = L(a0+i, a0+k) at column piv(a0+k), k < i
    __shared__ T ub[64];
    const int v = nodes[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = D.m[v], W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* P = vals + D.voff[v] + lw;
    const int32_t* pl = D.pl + r0;
    const int n = D.n;
    const int nb = (m + 63) / 64;
    for (int r = 0; r < nrhs; r++) {
        T* wr = w + (int64_t)r * n;
        for (int jb = nb - 1; jb >= 0; jb--) {
            const int a0 = jb * 64, mb = min(64, m - a0);
            for (int idx = tid; idx < mb * mb; idx += 256) {
                const int i = idx / mb, k = idx - (idx / mb) * mb;
                Lb[i][k] = k < i ? P[(int64_t)(a0 + i) * W + pl[a0 + k]] : T(0);
            }
            __syncthreads();
            if (wv == 0) {
                T va = lane < mb ? wr[r0 + a0 + lane] : T(0);
                for (int i = mb - 1; i >= 0; i--) {
                    const T ui = bcast(va, i);
                    if (lane < i) va -= Lb[i][lane] * ui;
                }
                if (lane < mb) {
                    ub[lane] = va;
                    wr[r0 + a0 + lane] = va;
                }
            }
            __syncthreads();
            for (int k = tid; k < a0; k += 256) {
                const int pk = pl[k];
                T acc = T(0);
                for (int i = 0; i < mb; i++) acc += P[(int64_t)(a0 + i) * W + pk] * ub[i];
                wr[r0 + k] -= acc;
            }
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------
// permutation / scaling, FP64 residual and norms, gradient
// ----------------------------------------------------------------------------

template <typename T>
__global__ void k_permute_in(int32_t n, int32_t nrhs, const int32_t* __restrict__ perm,
                             const double* __restrict__ scale, const double* __restrict__ src, int64_t ld,
                             T* __restrict__ dst)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * nrhs) return;
    int r = (int)(idx / n), i = (int)(idx % n);
    int o = perm[i];
    dst[idx] = (T)(scale[o] * src[o + (int64_t)r * ld]);
}

template <typename T>
__global__ void k_permute_out(int32_t n, int32_t nrhs, const int32_t* __restrict__ perm,
                              const double* __restrict__ scale, const T* __restrict__ z, double* __restrict__ dst,
                              int64_t ld, int32_t acc)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * nrhs) return;
    int r = (int)(idx / n), j = (int)(idx % n);
    int o = perm[j];
    double val = scale[o] * (double)z[idx];
    if (acc) dst[o + (int64_t)r * ld] += val; else dst[o + (int64_t)r * ld] = val;
}

__global__ void k_residual(int32_t n, int32_t nrhs, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ av, const double* __restrict__ b, int64_t ldb,
                           const double* __restrict__ x, int64_t ldx, double* __restrict__ r)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * nrhs) return;
    int k = (int)(idx / n), i = (int)(idx % n);
    const double* xk = x + (int64_t)k * ldx;
    double s = b[i + (int64_t)k * ldb];
    for (int64_t p = rp[i]; p < rp[i + 1]; p++) s -= av[p] * xk[ci[p]];
    r[idx] = s;
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// per right-hand side and per segment of rows (the members of a batch; one
// segment when seg is null), kNormSlots values at out[kNormSlots (k nseg + s)]:
// 0 max|r|, 1 max|x|, 2 max|b|, 3 sum|r|, 4 sum|b|; and at
// out[kNormSlots (nrhs nseg + s)] the largest row abs sum of A in segment s
__global__ void k_norms(int32_t n, int32_t nrhs, const int64_t* __restrict__ rp, const double* __restrict__ av,
                        const double* __restrict__ r, const double* __restrict__ x, int64_t ldx,
                        const double* __restrict__ b, int64_t ldb, const int32_t* __restrict__ seg, int32_t nseg,
                        double* __restrict__ out)
{
    __shared__ double sm[5][256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int first = blockIdx.x * blockDim.x;
    const int last = min(first + (int)blockDim.x, n) - 1;
    // a block whose rows all lie in one segment reduces in LDS first
    const int s_first = seg ? seg[first] : 0;
    const bool uniform = !seg || seg[last] == s_first;
    const int si = (i < n && seg) ? seg[i] : 0;
    for (int k = 0; k <= nrhs; k++) {
        double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
        if (i < n) {
            if (k < nrhs) {
                m0 = fabs(r[i + (int64_t)k * n]);
                m1 = fabs(x[i + (int64_t)k * ldx]);
                m2 = fabs(b[i + (int64_t)k * ldb]);
                m3 = m0;
                m4 = m2;
            } else {
                for (int64_t p = rp[i]; p < rp[i + 1]; p++) m0 += fabs(av[p]);
            }
        }
        double* o = out + kNormSlots * ((int64_t)k * nseg);
        if (!uniform) {
            if (i < n) {
                double* q = o + kNormSlots * si;
                atomic_max_nonneg(q + 0, m0);
                if (k < nrhs) {
                    atomic_max_nonneg(q + 1, m1);
                    atomic_max_nonneg(q + 2, m2);
                    atomicAdd(q + 3, m3);
                    atomicAdd(q + 4, m4);
                }
            }
            continue;
        }
        sm[0][threadIdx.x] = m0; sm[1][threadIdx.x] = m1; sm[2][threadIdx.x] = m2;
        sm[3][threadIdx.x] = m3; sm[4][threadIdx.x] = m4;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) {
                for (int q = 0; q < 3; q++) sm[q][threadIdx.x] = fmax(sm[q][threadIdx.x], sm[q][threadIdx.x + st]);
                for (int q = 3; q < 5; q++) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double* q = o + kNormSlots * s_first;
            atomic_max_nonneg(q + 0, sm[0][0]);
            if (k < nrhs) {
                atomic_max_nonneg(q + 1, sm[1][0]);
                atomic_max_nonneg(q + 2, sm[2][0]);
                atomicAdd(q + 3, sm[3][0]);
                atomicAdd(q + 4, sm[4][0]);
            }
        }
        __syncthreads();
    }
}

__global__ void k_gather(int64_t nnz, const int64_t* __restrict__ idx, const double* __restrict__ src,
                         double* __restrict__ dst)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nnz) dst[q] = src[idx[q]];
}

// g[p] = -sum_k lam[i, k] x[ci[p], k] over the nrhs columns (leading dimension ld)
__global__ void k_grad(int32_t n, int32_t nrhs, int64_t ld, const int64_t* __restrict__ rp,
                       const int32_t* __restrict__ ci, const double* __restrict__ lam, const double* __restrict__ x,
                       double* __restrict__ g)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
        const int64_t c = ci[p];
        double s = 0.0;
        for (int k = 0; k < nrhs; k++) s += lam[i + k * ld] * x[c + k * ld];
        g[p] = -s;
    }
}

// ----------------------------------------------------------------------------
// dense tail: blocked right-looking LU of the trailing block [t0, n) with the
// same pivot rule (each row searches only its own node's block columns, a
// standalone row keeps its diagonal).  A column c is still unpivoted at row a
// iff tstep[c] > a.  Per row panel [p0, p1):
//   k_tail_panel: the panel rows on their pivot window [c0, c1) (one block);
//   k_tail_trsm:  the panel rows' U right of the window (column-parallel)
//                 and the trailing rows' multipliers (row-parallel);
//   k_tail_gemm:  the trailing update of every still-unpivoted column.
// ----------------------------------------------------------------------------


__global__ void k_tail_init(int32_t mT, int32_t* __restrict__ tstep)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < mT) tstep[c] = 0x7fffffff;
}

// panel factorisation; with stage = true the panel's pivot window lives in LDS
// (np x wc values and the window's tstep entries), else it is updated in place
template <typename T, bool stage>
__global__ __launch_bounds__(256) void k_tail_panel(DevLayout D, TailView TV, T* __restrict__ vals, int p0, int p1,
                                                    int c0, int c1, T tau, int32_t* __restrict__ pert, int search)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T lrow[kNB];
    __shared__ T red_v[256];
    __shared__ int red_i[256];
    __shared__ int s_p;
    __shared__ int64_t rowoff[kNB];
    const int tid = threadIdx.x;
    const int wc = c1 - c0, np = p1 - p0;
    T* Xw = reinterpret_cast<T*>(smem_raw);                         // np x wc (stage only)
    int* tsw = reinterpret_cast<int*>(Xw + (stage ? np * wc : 0));  // wc (stage only)
    for (int r = tid; r < np; r += 256) rowoff[r] = TV.trow[p0 + r];
    __syncthreads();
    if (stage) {
        for (int idx = tid; idx < np * wc; idx += 256) {
            int r = idx / wc, c = idx % wc;
            Xw[idx] = vals[rowoff[r] + c0 + c];
        }
        for (int c = tid; c < wc; c += 256) tsw[c] = TV.tstep[c0 + c];
        __syncthreads();
    }
    // element (panel row r, tail column c) and the step that pivots column c
    auto X = [&](int r, int c) -> T& { return stage ? Xw[(r - p0) * wc + (c - c0)] : vals[rowoff[r - p0] + c]; };
    auto step = [&](int c) -> int { return stage ? tsw[c - c0] : TV.tstep[c]; };
    for (int a = p0; a < p1; a++) {
        const int lo = TV.tlo[a], hi = TV.thi[a];
        int p;
        if (!search) {
            p = TV.tpiv[a];
        } else if (hi - lo == 1) {
            p = a;
        } else {
            T best = T(-1);
            int bi = hi;
            for (int c = lo + tid; c < hi; c += 256) {
                if (step(c) <= a) continue;
                T x = pmag(X(a, c));
                if (x > best || (x == best && c < bi)) { best = x; bi = c; }
            }
            red_v[tid] = best; red_i[tid] = bi;
            __syncthreads();
            for (int s2 = 128; s2 > 0; s2 >>= 1) {
                if (tid < s2) {
                    T x = red_v[tid + s2]; int xi = red_i[tid + s2];
                    if (x > red_v[tid] || (x == red_v[tid] && xi < red_i[tid])) { red_v[tid] = x; red_i[tid] = xi; }
                }
                __syncthreads();
            }
            p = red_i[0];
        }
        if (tid == 0) {
            T d = X(a, p);
            if (tabs(d) < tau) {
                X(a, p) = d < T(0) ? -tau : tau;
                atomicAdd(pert, 1);
            }
            TV.tpiv[a] = p;
            TV.tstep[p] = a;
            if (stage) tsw[p - c0] = a;
            D.pl[TV.t0 + a] = p - lo;
            D.qinv[TV.t0 + p] = TV.t0 + a;
            s_p = p;
        }
        __syncthreads();
        p = s_p;
        const T d = X(a, p);
        for (int r = a + 1 + tid; r < p1; r += 256) {
            T l = X(r, p) / d;
            X(r, p) = l;
            lrow[r - p0] = l;
        }
        __syncthreads();
        const int rows_left = p1 - a - 1;
        for (int idx = tid; idx < rows_left * wc; idx += 256) {
            int r = a + 1 + idx / wc;
            int c = c0 + idx % wc;
            if (step(c) <= a) continue;
            X(r, c) -= lrow[r - p0] * X(a, c);
        }
        __syncthreads();
    }
    if (stage) {
        for (int idx = tid; idx < np * wc; idx += 256) {
            int r = idx / wc, c = idx % wc;
            vals[rowoff[r] + c0 + c] = Xw[idx];
        }
    }
}

// panel factorisation for a wide pivot window (wc > 64) on one workgroup of
// NT threads.  Thread t owns window columns t, t+NT, ...; per panel row the
// pivot is a block argmax over the unpivoted window columns (ties: lowest
// column), the multipliers of the later panel rows are formed by one thread
// each, and every thread eliminates its own columns down the panel.  The next
// row's candidate is taken while that row is updated, so each step makes one
// pass.  The window's pivot steps sit in LDS; STAGE also stages the window.
template <typename T, int NT, bool STAGE>
__global__ __launch_bounds__(NT) void k_tail_panel_wide(DevLayout D, TailView TVp, T* __restrict__ vals, int p0,
                                                        int p1, int c0, int c1, T tau, int32_t* __restrict__ pert,
                                                        int search, const ViewDesc* __restrict__ vd,
                                                        const ViewJob* __restrict__ jobs)
{
    TailView TV = TVp;
    if (jobs) {                 // one panel of several views' launch
        const ViewJob j = jobs[blockIdx.x];
        TV = vd[j.v].TV;
        p0 = j.a[0]; p1 = j.a[1]; c0 = j.a[2]; c1 = j.a[3];
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int64_t rowoff[kNB];
    __shared__ int rlo[kNB], rhi[kNB], rpiv[kNB];      // per panel row: block range, known pivot
    __shared__ T lrow[kNB];
    __shared__ T red_v[NT / 64];
    __shared__ int red_i[NT / 64];
    __shared__ int s_p;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wc = c1 - c0, np = p1 - p0;
    int* tsw = reinterpret_cast<int*>(smem_raw);                              // wc: step pivoting the column
    T* Xs = reinterpret_cast<T*>(smem_raw + (((size_t)wc * 4 + 15) & ~(size_t)15));   // STAGE: np x wc
    for (int r = tid; r < np; r += NT) {
        rowoff[r] = TV.trow[p0 + r];
        rlo[r] = TV.tlo[p0 + r];
        rhi[r] = TV.thi[p0 + r];
        rpiv[r] = search ? 0 : TV.tpiv[p0 + r];
    }
    for (int c = tid; c < wc; c += NT) tsw[c] = TV.tstep[c0 + c];
    __syncthreads();
    if (STAGE) {
        // eight loads per thread in flight before their LDS stores
        for (int i0 = tid; i0 < np * wc; i0 += 8 * NT) {
            T t[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * NT;
                t[u] = i < np * wc ? vals[rowoff[i / wc] + c0 + i % wc] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int i = i0 + u * NT;
                if (i < np * wc) Xs[i] = t[u];
            }
        }
        __syncthreads();
    }
    auto X = [&](int r, int c) -> T& {   // panel-local row r, window-local column c
        return STAGE ? Xs[r * wc + c] : vals[rowoff[r] + c0 + c];
    };
    // candidate of panel row 0
    T cv = T(-1);
    int ci = wc;
    if (search) {
        const int lo0 = rlo[0] - c0, hi0 = rhi[0] - c0;
        for (int c = tid; c < wc; c += NT) {
            if (tsw[c] <= p0 || c < lo0 || c >= hi0) continue;
            const T x = pmag(X(0, c));
            if (x > cv) { cv = x; ci = c; }     // ascending c: the first maximum is the lowest column
        }
    }
    for (int a = 0; a < np; a++) {
        const int ga = p0 + a;
        const int lo = rlo[a], hi = rhi[a];
        int p;
        if (!search) {
            p = rpiv[a] - c0;
        } else if (hi - lo == 1) {
            p = lo - c0;
        } else {
            // block argmax of (cv, ci): larger value, then lower column
            T bv = cv;
            int bi = ci;
            for (int off = 32; off > 0; off >>= 1) {
                const T ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < NT / 64; w++)
                    if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) { bv = red_v[w]; bi = red_i[w]; }
                s_p = bi;
            }
            __syncthreads();
            p = s_p;
        }
        if (tid == 0) {
            T d = X(a, p);
            if (tabs(d) < tau) {
                X(a, p) = d < T(0) ? -tau : tau;
                atomicAdd(pert, 1);
            }
            TV.tpiv[ga] = c0 + p;
            TV.tstep[c0 + p] = ga;
            tsw[p] = ga;
            D.pl[TV.t0 + ga] = c0 + p - lo;
            D.qinv[TV.t0 + c0 + p] = TV.t0 + ga;
        }
        __syncthreads();
        const T d = X(a, p);
        if (tid > a && tid < np) {
            const T l = X(tid, p) / d;
            X(tid, p) = l;
            lrow[tid] = l;
        }
        __syncthreads();
        cv = T(-1);
        ci = wc;
        const int nlo = a + 1 < np ? rlo[a + 1] - c0 : 0, nhi = a + 1 < np ? rhi[a + 1] - c0 : 0;
        for (int c = tid; c < wc; c += NT) {
            if (tsw[c] <= ga) continue;             // pivoted (this step's pivot included)
            const T u = X(a, c);
            if (a + 1 < np) {
                const T x1 = X(a + 1, c) - lrow[a + 1] * u;
                X(a + 1, c) = x1;
                if (pmag(x1) > cv && c >= nlo && c < nhi) { cv = pmag(x1); ci = c; }
            }
#pragma unroll 4
            for (int r = a + 2; r < np; r++) X(r, c) -= lrow[r] * u;
        }
        __syncthreads();
    }
    if (STAGE) {
        for (int r = 0; r < np; r++)
            for (int c = tid; c < wc; c += NT) vals[rowoff[r] + c0 + c] = Xs[r * wc + c];
    }
}

// panel factorisation with the window (<= 64 columns) in LDS: lanes own
// window columns; for every panel row the pivot is a wave reduction on
// wavefront 0, the multipliers are formed one thread per row, and NW
// wavefronts share the elimination, the rows dealt round robin.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_tail_panel_lds4(DevLayout D, TailView TV, T* __restrict__ vals, int p0,
                                                             int p1, int c0, int c1, T tau, int32_t* __restrict__ pert,
                                                             int search)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int64_t rowoff[kNB];
    __shared__ T lrow[kNB];
    __shared__ int spiv[kNB], slo[kNB], shi[kNB];
    __shared__ int s_p;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wc = c1 - c0, np = p1 - p0;
    int npert = 0;
    T* Xw = reinterpret_cast<T*>(smem_raw);          // np x wc
    if (tid < np) {
        rowoff[tid] = TV.trow[p0 + tid];
        slo[tid] = TV.tlo[p0 + tid];
        shi[tid] = TV.thi[p0 + tid];
        spiv[tid] = search ? 0 : TV.tpiv[p0 + tid];
    }
    int mystep = lane < wc ? TV.tstep[c0 + lane] : -1;   // the step that pivots my column
    __syncthreads();
    if (lane < wc) {
        T tmp[kNB / NW];
#pragma unroll
        for (int q = 0; q < kNB / NW; q++) {
            const int r = wv + NW * q;
            tmp[q] = r < np ? vals[rowoff[r] + c0 + lane] : T(0);
        }
#pragma unroll
        for (int q = 0; q < kNB / NW; q++) {
            const int r = wv + NW * q;
            if (r < np) Xw[r * wc + lane] = tmp[q];
        }
    }
    __syncthreads();
    for (int ar = 0; ar < np; ar++) {
        const int a = p0 + ar;
        const int lo = slo[ar], hi = shi[ar];
        T* Xa = Xw + ar * wc;
        int p;
        if (!search) {
            p = spiv[ar];
        } else if (hi - lo == 1) {
            p = a;
        } else {
            if (wv == 0) {
                T best = T(-1);
                int bi = 0x7fffffff;
                const int c = c0 + lane;
                if (lane < wc && c >= lo && c < hi && mystep > a) { best = pmag(Xa[lane]); bi = c; }
                for (int off = 32; off > 0; off >>= 1) {
                    T ob = __shfl_xor(best, off, 64);
                    int oi = __shfl_xor(bi, off, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (lane == 0) s_p = bi;
            }
            __syncthreads();
            p = s_p;
        }
        const int pc = p - c0;
        T d = Xa[pc];
        if (tabs(d) < tau) d = d < T(0) ? -tau : tau;
        if (lane == pc) mystep = a;
        // multipliers of the remaining rows, one thread per row
        const int rl = np - ar - 1;
        if (tid < rl) {
            T* Xr = Xw + (ar + 1 + tid) * wc;
            const T l = Xr[pc] / d;
            Xr[pc] = l;
            lrow[ar + 1 + tid] = l;
        }
        __syncthreads();
        if (tid == 0) {
            if (Xa[pc] != d) { Xa[pc] = d; npert++; }
            spiv[ar] = p;
        }
        if (lane < wc && mystep > a) {              // my column is still unpivoted
            const T u = Xa[lane];
            // rows ar+1.. dealt round robin: this wavefront takes r = wv mod NW
            int r = ar + 1 + ((wv - (ar + 1)) & (NW - 1));
            for (; r + 3 * NW < np; r += 4 * NW) {
                const T x0 = Xw[r * wc + lane], x1 = Xw[(r + NW) * wc + lane];
                const T x2 = Xw[(r + 2 * NW) * wc + lane], x3 = Xw[(r + 3 * NW) * wc + lane];
                Xw[r * wc + lane] = x0 - lrow[r] * u;
                Xw[(r + NW) * wc + lane] = x1 - lrow[r + NW] * u;
                Xw[(r + 2 * NW) * wc + lane] = x2 - lrow[r + 2 * NW] * u;
                Xw[(r + 3 * NW) * wc + lane] = x3 - lrow[r + 3 * NW] * u;
            }
            for (; r < np; r += NW) Xw[r * wc + lane] -= lrow[r] * u;
        }
        __syncthreads();
    }
    if (lane < wc) {
        for (int r = wv; r < np; r += NW) vals[rowoff[r] + c0 + lane] = Xw[r * wc + lane];
    }
    if (tid < np) {
        const int a = p0 + tid, p = spiv[tid];
        TV.tpiv[a] = p;
        TV.tstep[p] = a;
        D.pl[TV.t0 + a] = p - slo[tid];
        D.qinv[TV.t0 + p] = TV.t0 + a;
    }
    if (tid == 0 && npert > 0) atomicAdd(pert, npert);
}


// refactorisation of a panel whose pivot window is its own rows (pivots
// known): one wavefront, lane r holding row r of the window in registers in
// pivot order.  At step a every lane reads row a's values by readlane (all
// lanes active) and the rows below form their multiplier and update their
// copy: the operations of k_tail_panel_lds4 in the same order, without a
// block barrier per step.
template <typename T>
__global__ __launch_bounds__(64) void k_tail_panel_reg(DevLayout D, TailView TV, T* __restrict__ vals, int p0, int p1,
                                                       T tau, int32_t* __restrict__ pert)
{
    const int lane = threadIdx.x;
    const int np = p1 - p0;
    const bool mine = lane < np;
    const int64_t ro = mine ? TV.trow[p0 + lane] : 0;
    T x[kNB];
#pragma unroll
    for (int j = 0; j < kNB; j++) x[j] = (mine && j < np) ? vals[ro + TV.tpiv[p0 + j]] : T(0);
    int npert = 0;
#pragma unroll
    for (int a = 0; a < kNB; a++) {
        if (a < np) {
            T d = rlane(x[a], a);
            if (tabs(d) < tau) d = d < T(0) ? -tau : tau;
            if (lane == a && x[a] != d) { x[a] = d; npert++; }
            // rows above a (and lanes past the panel) take l = 0: their values
            // stay as they are (up to the sign of a zero), with no select per
            // update
            const bool act = mine && lane > a;
            const T l = act ? x[a] / d : T(0);
#pragma unroll
            for (int j = a + 1; j < kNB; j++) {
                const T u = rlane(x[j], a);
                x[j] -= l * u;
            }
            if (act) x[a] = l;
        }
    }
    if (mine) {
#pragma unroll
        for (int j = 0; j < kNB; j++)
            if (j < np) vals[ro + TV.tpiv[p0 + j]] = x[j];
        const int a = p0 + lane, p = TV.tpiv[a];
        TV.tstep[p] = a;
        D.pl[TV.t0 + a] = p - TV.tlo[a];
        D.qinv[TV.t0 + p] = TV.t0 + a;
    }
    if (npert > 0) atomicAdd(pert, npert);
}

// blocks [0, nA): panel rows' U for columns >= c1 (one thread per column);
// blocks [nA, ...): trailing rows' multipliers (one thread per row)
template <typename T>
__global__ __launch_bounds__(64) void k_tail_trsm(TailView TVp, T* __restrict__ vals, int p0, int p1, int c1, int nA,
                                                  int kb0, int kof, const int32_t* __restrict__ bl,
                                                  const ViewDesc* __restrict__ vd, const ViewJob* __restrict__ jobs)
{
    TailView TV = TVp;
    int jblk = -1;
    if (jobs) {                 // a block of several views' launch
        const ViewJob j = jobs[blockIdx.x];
        TV = vd[j.v].TV;
        p0 = j.a[0]; p1 = j.a[1]; c1 = j.a[2]; nA = j.a[3]; kb0 = j.a[4]; kof = j.a[5];
        jblk = j.blk;
    }
    __shared__ T M[kNB][kNB + 1];       // M[i][j] = X_{p0+i}[tpiv[p0+j]]
    __shared__ int64_t rowoff[kNB];
    __shared__ int piv[kNB];
    const int np = p1 - p0, tid = threadIdx.x;
    // block list (structurally sparse tail): column blocks of U that hold
    // entries, and every row block, flagged when its multipliers are all zero
    int blk = jblk >= 0 ? jblk : (int)blockIdx.x;
    if (bl) {
        const int e = bl[blockIdx.x];
        blk = e & ~kTrsmZero;
        if (e & kTrsmZero) {
            const int r = p1 + (blk - nA) * 64 + tid;
            if (r < TV.mT) {
                T* lb = reinterpret_cast<T*>(TV.lbuf);
                for (int b = 0; b < np; b++) lb[(int64_t)(kof + b) * TV.mT + r] = T(0);
            }
            return;
        }
    }
    for (int i = tid; i < np; i += 64) { rowoff[i] = TV.trow[p0 + i]; piv[i] = TV.tpiv[p0 + i]; }
    __syncthreads();
    if (tid < np) {                          // column tid of M: one independent load per panel row
        const int pc = piv[tid];
        T tmp[kNB];
#pragma unroll
        for (int i = 0; i < kNB; i++) tmp[i] = i < np ? vals[rowoff[i] + pc] : T(0);
#pragma unroll
        for (int i = 0; i < kNB; i++) M[i][tid] = tmp[i];
    }
    __syncthreads();
    if (blk < nA) {
        const int c = c1 + blk * 64 + tid;
        if (c >= TV.nc) return;
        // the column's values first (independent loads), then the forward
        // substitution in place
        T colv[kNB];
#pragma unroll
        for (int a = 0; a < kNB; a++) colv[a] = a < np ? vals[rowoff[a] + c] : T(0);
#pragma unroll
        for (int a = 0; a < kNB; a++) {
            if (a < np) {
                T acc = colv[a];
#pragma unroll
                for (int b = 0; b < a; b++) acc -= M[a][b] * colv[b];
                colv[a] = acc;
                vals[rowoff[a] + c] = acc;
            }
        }
    } else {
        const int r = p1 + (blk - nA) * 64 + tid;
        if (r >= TV.mT) return;
        T* Xr = vals + TV.trow[r];
        T* lb = reinterpret_cast<T*>(TV.lbuf);
        T y[kNB];
#pragma unroll
        for (int b = 0; b < kNB; b++) y[b] = b < np ? Xr[piv[b]] : T(0);
#pragma unroll
        for (int b = 0; b < kNB; b++) {
            if (b < np) {
                const T l = y[b] / M[b][b];
                y[b] = l;
#pragma unroll
                for (int bb = b + 1; bb < kNB; bb++) y[bb] -= l * M[b][bb];
            }
        }
#pragma unroll
        for (int b = 0; b < kNB; b++) {
            if (b < np) Xr[piv[b]] = y[b];
            lb[(int64_t)(kof + b) * TV.mT + r] = b < np ? y[b] : T(0);   // k-major copy for the trailing update
        }
    }
}

// trailing update X[r][c] -= sum_k L[r][k] X[kb0+k][c] on 16x16x4 MFMA tiles:
// a workgroup computes a 64 x 64 tile (four wavefronts of 32 x 32); operand
// fragments come straight from global memory (lbuf is k-major, the panel rows
// row-major, so 16 lanes read 16 consecutive values); the outputs are read
// before the K loop.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // output item v of lane l: row (l / 16) + 4 v, column l % 16
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // output item v of lane l: row 4 (l / 16) + v, column l % 16
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_tail_gemm(TailView TVp, T* __restrict__ vals, int kb0, int K, int rb, int re,
                                                   int cg0, int mstep, int gx, int gy, int swz, int gp0, int gnp,
                                                   const uint32_t* __restrict__ tl, int kb1, int kb2, int kb3,
                                                   const ViewDesc* __restrict__ vd, const ViewJob* __restrict__ jobs)
{
    typedef typename Mfma<T>::v4 v4;
    static_assert(kGroup == 4, "the K ranges below assume four panels per group");
    TailView TV = TVp;
    int jblk = -1;
    if (jobs) {                 // a tile of several views' launch: one panel, every tile
        const ViewJob j = jobs[blockIdx.x];
        TV = vd[j.v].TV;
        kb0 = j.a[0]; K = j.a[1]; rb = j.a[2]; re = j.a[3]; cg0 = j.a[4]; mstep = j.a[5];
        gp0 = 0; gnp = 0; kb1 = kb2 = kb3 = K;
        jblk = j.blk;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int mT = re, nc = TV.nc, lds = TV.mT;
    // tile of this workgroup.  Workgroups go to the 8 XCDs round robin by
    // index; with swz each XCD takes a quarter of the tile rows and half of
    // the tile columns, so the operand tiles it reads fit its own L2.  With a
    // tile list (structurally sparse tail) the list is already in that order
    // and each entry carries the group panels whose products are nonzero.
    int tx, ty, pmask = 0xF;
    {
        const int L = blockIdx.x;
        if (jblk >= 0) {
            ty = jblk >> 16;
            tx = jblk & 0xFFFF;
        } else if (tl) {
            const uint32_t e = tl[L];
            if (e == kTileNone) return;
            ty = (int)(e >> 16);
            tx = (int)((e >> 4) & 0xFFF);
            pmask = (int)(e & 0xF);
        } else if (swz) {
            const int xcd = L & 7, k = L >> 3;
            const int rb0 = (xcd >> 1) * gy / 4, rb1 = ((xcd >> 1) + 1) * gy / 4;
            const int cb0 = (xcd & 1) * gx / 2, cb1 = ((xcd & 1) + 1) * gx / 2;
            const int nr = rb1 - rb0, ncl = cb1 - cb0;
            if (k >= nr * ncl) return;
            ty = rb0 + k / ncl;
            tx = cb0 + k % ncl;
        } else {
            if (L >= gx * gy) return;
            ty = L / gx;
            tx = L % gx;
        }
    }
    // value offsets of the K panel rows, staged once (the B operand's row
    // pointers would otherwise be a dependent load in every K step)
    __shared__ int64_t trk[kNB * kGroup];
    for (int k = threadIdx.x; k < K; k += 256) trk[k] = TV.trow[kb0 + k];
    __syncthreads();
    // block tile 64 x 64, four wavefronts of 32 x 32 (2 x 2 MFMA blocks each)
    const int r0 = rb + ty * 64 + (wv >> 1) * 32, c0 = cg0 + tx * 64 + (wv & 1) * 32;
    const T* lb = reinterpret_cast<const T*>(TV.lbuf);
    const int li = lane & 15, lk = lane >> 4;
    const bool rok0 = r0 + li < mT, rok1 = r0 + 16 + li < mT;
    // gnp > 0: the columns are the pivot columns of panel rows gp0.., in order
    int cb = c0 + li, cb1 = cb + 16;
    bool cok0 = cb < nc, cok1 = cb1 < nc;
    if (gnp > 0) {
        cok0 = cb < gnp;
        cok1 = cb1 < gnp;
        cb = cok0 ? TV.tpiv[gp0 + cb] : 0;
        cb1 = cok1 ? TV.tpiv[gp0 + cb1] : 0;
    }
    const bool cm0 = cok0 && (gnp > 0 || TV.tstep[cb] >= mstep), cm1 = cok1 && (gnp > 0 || TV.tstep[cb1] >= mstep);
    // the output values are read before the K loop so their latency overlaps it
    T cold[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int r = r0 + 16 * i + Mfma<T>::row(lane, v);
            const T* Xr = vals + (r < mT ? TV.trow[r] : 0);
            cold[i][0][v] = (r < mT && cm0) ? Xr[cb] : T(0);
            cold[i][1][v] = (r < mT && cm1) ? Xr[cb1] : T(0);
        }
    v4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = v4{T(0), T(0), T(0), T(0)};
    const T* arow = lb + (int64_t)lk * lds + r0 + li;
    // K in the group's panel ranges [kbnd[j], kbnd[j+1]) whose bit is set, in
    // steps of 4 from 0 as in the dense sweep, so the products summed are the
    // same: a skipped step has only exact zeros (rows without L entries in the
    // panel, or columns without U entries)
    const int kbnd[kGroup + 1] = {0, kb1, kb2, kb3, K};
    unsigned long long kact = 0;          // bit ks: K step [4 ks, 4 ks + 4) is summed
#pragma unroll
    for (int j = 0; j < kGroup; j++) {
        if (!((pmask >> j) & 1)) continue;
        const int s0 = kbnd[j] >> 2, s1 = (kbnd[j + 1] + 3) >> 2;
        if (s1 > s0) kact |= (s1 - s0 >= 64 ? ~0ull : ((1ull << (s1 - s0)) - 1)) << s0;
    }
    // eight K steps per round, all their loads issued before the first MFMA;
    // a step outside the summed ones within a round contributes exact zeros
    const int nks = (K + 3) >> 2;
    for (int c0 = 0; c0 < nks; c0 += 8) {
        const unsigned cm = (unsigned)(kact >> c0) & 0xFFu;
        if (!cm) continue;
        T a0[8], a1[8], b0[8], b1[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int ks = c0 + u, k = ks * 4 + lk;
            const bool kok = ((cm >> u) & 1u) && k < K;
            const T* ap = arow + (int64_t)ks * 4 * lds;
            a0[u] = (kok && rok0) ? ap[0] : T(0);
            a1[u] = (kok && rok1) ? ap[16] : T(0);
            const T* bp = vals + (kok ? trk[k] : 0);
            b0[u] = (kok && cok0) ? bp[cb] : T(0);
            b1[u] = (kok && cok1) ? bp[cb1] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            acc[0][0] = Mfma<T>::mma(a0[u], b0[u], acc[0][0]);
            acc[0][1] = Mfma<T>::mma(a0[u], b1[u], acc[0][1]);
            acc[1][0] = Mfma<T>::mma(a1[u], b0[u], acc[1][0]);
            acc[1][1] = Mfma<T>::mma(a1[u], b1[u], acc[1][1]);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int r = r0 + 16 * i + Mfma<T>::row(lane, v);
            if (r >= mT) continue;
            T* Xr = vals + TV.trow[r];
            if (cm0) Xr[cb] = cold[i][0][v] - acc[i][0][v];
            if (cm1) Xr[cb1] = cold[i][1][v] - acc[i][1][v];
        }
}

// ---- row tiles of supernode targets (sup-sup on MFMA)
//
// One workgroup takes kTileRows consecutive rows of a target supernode and
// applies every source in ascending order, as the row kernel does for one
// row, so each source's panel is read once per tile instead of once per row.
// Standalone source: multipliers l_r = X[r][lp] / pivot, then a rank-1 update
// through the relative map, each wavefront on its own four rows.  Supernode
// source s (ms rows): the tile's block columns of s (staged in LDS when
// ms <= kTileMs) times the inverse of U_ss in s's pivot order, on MFMA over the
// four wavefronts, when s has that inverse (else a blocked triangular solve on
// one wavefront), then X[:, rel(T_s)] -= L (tile x ms) * U_s,T on 16x16x4 MFMA,
// 16-column blocks per wavefront, scattered through rel.
constexpr int kTileRows = 16;
constexpr int kTileMs = 448;

template <typename T>
__global__ __launch_bounds__(256) void k_factor_tile(DevLayout D, T* __restrict__ vals,
                                                     const int32_t* __restrict__ tiles, int32_t ntiles)
{
    typedef typename Mfma<T>::v4 v4;
    __shared__ T Xs[kTileRows][kTileMs + 1];
    __shared__ int pls[kTileMs];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int v = tiles[2 * blockIdx.x], a0 = tiles[2 * blockIdx.x + 1];
    const int m = D.m[v], W = D.W[v];
    const int R = min(kTileRows, m - a0);
    T* X0 = vals + D.voff[v] + (int64_t)a0 * W;
    const int64_t e1 = D.eptr[v + 1];
    for (int64_t e = D.eptr[v]; e < e1; e++) {
        const EdgeDesc ed = D.edges[e];
        const T* Us = vals + ed.uoff;
        const int32_t* rl = D.rel + ed.roff;
        const int lp = ed.lp, ms = ed.ms, Ws = ed.Ws, ws = ed.ws;
        if (ms == 1) {
            // standalone source: wavefront w updates rows w, w+4, w+8, w+12 on
            // its own, so runs of standalone sources need no block barrier
            for (int r = wv; r < R; r += 4) {
                T* Xr = X0 + (int64_t)r * W;
                const T l = Xr[lp] / Us[0];
                for (int j = lane; j < ws; j += 64) Xr[rl[j]] -= l * Us[1 + j];
                if (lane == 0) Xr[lp] = l;
            }
            __threadfence_block();
            continue;
        }
        __syncthreads();     // the standalone updates of every wavefront are in
        const int32_t* plg = D.pl + ed.r0s;
        const bool in_lds = ms <= kTileMs;
        // the tile's block columns of s in s's pivot order: XP(r, b) = X[r][lp + pl_b]
        if (in_lds) {
            for (int b = tid; b < ms; b += 256) pls[b] = plg[b];
            __syncthreads();
            for (int idx = tid; idx < kTileRows * ms; idx += 256) {
                const int r = idx / ms, c = idx - (idx / ms) * ms;
                Xs[r][c] = r < R ? X0[(int64_t)r * W + lp + pls[c]] : T(0);
            }
        }
        __syncthreads();
        auto PL = [&](int b) -> int { return in_lds ? pls[b] : plg[b]; };
        auto XP = [&](int r, int b) -> T& { return in_lds ? Xs[r][b] : X0[(int64_t)r * W + lp + PL(b)]; };
        if (ed.ioff >= 0 && in_lds && ms <= 4 * 4 * 16) {
            // L = XP U_pp^{-1} with the inverse of the source's block (upper
            // triangular, row-major ms x ms): a tile x ms by ms x ms product on
            // MFMA, the 16-column blocks of L spread over the four wavefronts
            const T* Ui = reinterpret_cast<const T*>(D.uinv) + ed.ioff;
            const int li = lane & 15, lk = lane >> 4;
            const int nblk = (ms + 15) / 16;
            v4 acc[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                acc[t] = v4{T(0), T(0), T(0), T(0)};
                const int jb = wv + 4 * t;
                if (jb < nblk) {
                    const int c = jb * 16 + li;
                    const int kend = min(ms, jb * 16 + 16);      // Ui[k][c] = 0 for k > c
                    // eight K steps per round, their loads before the MFMAs
                    for (int k0 = 0; k0 < kend; k0 += 32) {
                        T av[8], bv[8];
#pragma unroll
                        for (int u = 0; u < 8; u++) {
                            const int k = k0 + 4 * u + lk;
                            const bool ok = k0 + 4 * u < kend && k < ms;
                            av[u] = ok ? Xs[li][k] : T(0);
                            bv[u] = (ok && c < ms) ? Ui[(int64_t)k * ms + c] : T(0);
                        }
#pragma unroll
                        for (int u = 0; u < 8; u++)
                            if (k0 + 4 * u < kend) acc[t] = Mfma<T>::mma(av[u], bv[u], acc[t]);
                    }
                }
            }
            __syncthreads();          // every wavefront has read XP
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int jb = wv + 4 * t;
                const int c = jb * 16 + li;
                if (jb < nblk && c < ms)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = Mfma<T>::row(lane, q);
                        if (r < R) Xs[r][c] = acc[t][q];
                    }
            }
        } else if (wv == 0) {
        // L = XP U_pp^{-1}, U_pp(b, b') = U(b, pl_b') upper triangular in pivot
        // order; blocked by 16 columns on wavefront 0: the block's update from
        // the solved columns on MFMA, then its 16 x 16 triangle, one lane per row
            const int li = lane & 15;
            for (int kb0 = 0; kb0 < ms; kb0 += 16) {
                const int nb = min(16, ms - kb0);
                if (kb0 > 0) {
                    v4 acc = v4{T(0), T(0), T(0), T(0)};
                    const int bc = kb0 + li;
                    const int pc = bc < ms ? PL(bc) : 0;
                    for (int k0 = 0; k0 < kb0; k0 += 4) {
                        const int k = k0 + (lane >> 4);
                        const T av = li < R ? XP(li, k) : T(0);
                        const T bv = bc < ms ? Us[(int64_t)k * Ws + pc] : T(0);
                        acc = Mfma<T>::mma(av, bv, acc);
                    }
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = Mfma<T>::row(lane, q);
                        if (r < R && bc < ms) XP(r, bc) -= acc[q];
                    }
                    __threadfence_block();
                }
                if (lane < R) {
                    for (int b = kb0; b < kb0 + nb; b++) {
                        const T l = XP(lane, b) / Us[(int64_t)b * Ws + PL(b)];
                        XP(lane, b) = l;
                        for (int b2 = b + 1; b2 < kb0 + nb; b2++) XP(lane, b2) -= l * Us[(int64_t)b * Ws + PL(b2)];
                    }
                }
                __threadfence_block();
            }
        }
        __syncthreads();
        if (in_lds) {
            for (int idx = tid; idx < R * ms; idx += 256) {
                const int r = idx / ms, c = idx - (idx / ms) * ms;
                X0[(int64_t)r * W + lp + pls[c]] = Xs[r][c];
            }
        }
        // X[:, rel(T_s)] -= L * U_s,T  (A: tile rows x source rows, B: source rows x T)
        const T* Ut = Us + ms;
        const int li = lane & 15, lk = lane >> 4;
        for (int j0 = wv * 16; j0 < ws; j0 += 64) {
            v4 acc = v4{T(0), T(0), T(0), T(0)};
            const int jc = j0 + li;
            // eight K steps per round, their loads before the MFMAs
            for (int k0 = 0; k0 < ms; k0 += 32) {
                T a[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int k = k0 + 4 * u + lk;
                    a[u] = (k < ms && li < R) ? XP(li, k) : T(0);
                    bv[u] = (k < ms && jc < ws) ? Ut[(int64_t)k * Ws + jc] : T(0);
                }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (k0 + 4 * u < ms) acc = Mfma<T>::mma(a[u], bv[u], acc);
            }
            if (jc < ws) {
                const int c = rl[jc];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int r = Mfma<T>::row(lane, q);
                    if (r < R) X0[(int64_t)r * W + c] -= acc[q];
                }
            }
        }
        __syncthreads();
    }
}

// ---- dense tail solves (tail-local row/column a is global t0 + a)

// forward, outside part: y_i -= sum over the L columns from outside the tail
template <typename T>
__global__ __launch_bounds__(256) void k_tail_lext(DevLayout D, const T* __restrict__ vals, int t0, T* __restrict__ y,
                                                   int nrhs)
{
    const int lane = threadIdx.x & 63;
    const int i = t0 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= D.n) return;
    const int v = D.row_node[i];
    const int W = D.W[v];
    const T* P = vals + D.voff[v] + (int64_t)(i - D.r0[v]) * W;
    const int32_t* cols = D.cols + D.coff[v];
    // outside sources come first in the column list and are the only columns
    // < t0: the L region's first lw - (r0 - t0) entries
    const int next = D.lw[v] - (D.r0[v] - t0);
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * D.n;
        T acc = gather_lq<T, 64>(P, cols, D.qinv, yr, next, lane);
        acc = wave_sum(acc);
        if (lane == 0) yr[i] -= acc;
    }
}

// U^T, outside part: h[c] -= sum_k U_st(k, c) w_k over rows k before the tail
template <typename T>
__global__ __launch_bounds__(256) void k_tail_utext(DevLayout D, TailView TV, const T* __restrict__ vals,
                                                    T* __restrict__ h, const T* __restrict__ w, int nrhs)
{
    const int lane = threadIdx.x & 63;
    const int c = TV.t0 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= D.n) return;
    for (int r = 0; r < nrhs; r++) {
        const T* wr = w + (int64_t)r * D.n;
        // four entries per lane at a time: slots and rows, then values
        T acc = T(0);
        const int64_t q1 = D.ut_ptr[c + 1];
        for (int64_t q0 = D.ut_ptr[c] + lane; q0 < q1; q0 += 4 * 64) {
            int64_t sl[4];
            int32_t rw[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int64_t q = q0 + 64 * u;
                sl[u] = q < q1 ? D.ut_slot[q] : 0;
                rw[u] = q < q1 ? D.ut_row[q] : 0;
            }
            T pv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const bool ok = q0 + 64 * u < q1;
                pv[u] = ok ? vals[sl[u]] : T(0);
                xv[u] = ok ? wr[rw[u]] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 4; u++) acc += pv[u] * xv[u];
        }
        acc = wave_sum(acc);
        if (lane == 0) h[(int64_t)r * D.n + c] -= acc;
    }
}

// inverses of the diagonal blocks of the solve panels: for panel s = [p0, p1)
// with M[i][j] = X_{p0+i}[tpiv[p0+j]] (L strictly below the diagonal, U_st on
// and above it, both in pivot order), kind 0 writes (I + L)^-1 and kind 1
// U^-1, column-major 64 x 64 at out + (2 s + kind) * 64 * 64.  Thread j
// substitutes for column j.
template <typename T>
__global__ __launch_bounds__(64) void k_tail_dinv(TailView TVp, const T* __restrict__ vals, const int32_t* __restrict__ spp,
                                                  T* __restrict__ outp, const ViewDesc* __restrict__ vd,
                                                  const ViewJob* __restrict__ jobs)
{
    __shared__ T M[kNB][kNB + 1];
    __shared__ T X[kNB][kNB + 1];
    __shared__ int piv[kNB];
    __shared__ int64_t ro[kNB];
    TailView TV = TVp;
    const int32_t* sp = spp;
    T* out = outp;
    int bid = blockIdx.x;
    if (jobs) {                 // an inverse of several views' launch
        const ViewJob j = jobs[blockIdx.x];
        TV = vd[j.v].TV;
        sp = vd[j.v].sp;
        out = reinterpret_cast<T*>(vd[j.v].inv);
        bid = j.blk;
    }
    const int s = bid >> 1, kind = bid & 1;
    const int p0 = sp[2 * s], np = sp[2 * s + 1] - p0;
    const int lane = threadIdx.x;
    if (lane < np) { piv[lane] = TV.tpiv[p0 + lane]; ro[lane] = TV.trow[p0 + lane]; }
    __syncthreads();
    if (lane < np) {
        const int pc = piv[lane];
        T tmp[kNB];
#pragma unroll
        for (int i = 0; i < kNB; i++) tmp[i] = i < np ? vals[ro[i] + pc] : T(0);
#pragma unroll
        for (int i = 0; i < kNB; i++) M[i][lane] = tmp[i];
    }
    __syncthreads();
    const int j = lane;
    for (int i = 0; i < kNB; i++) X[i][j] = T(0);
    if (j < np) {
        if (kind == 0) {
            X[j][j] = T(1);
            for (int i = j + 1; i < np; i++) {
                T acc = T(0);
                for (int k = j; k < i; k++) acc += M[i][k] * X[k][j];
                X[i][j] = -acc;
            }
        } else {
            X[j][j] = T(1) / M[j][j];
            for (int i = j - 1; i >= 0; i--) {
                T acc = T(0);
                for (int k = i + 1; k <= j; k++) acc += M[i][k] * X[k][j];
                X[i][j] = -acc / M[i][i];
            }
        }
    }
    __syncthreads();
    T* O = out + ((int64_t)2 * s + kind) * kNB * kNB;
    for (int idx = lane; idx < kNB * kNB; idx += 64) O[idx] = X[idx & (kNB - 1)][idx >> 6];
}

// one launch per solve panel of a dense view: the targets past the next panel
// take the current panel [p0, p1)'s contribution (one wavefront each, its
// lanes over the panel's 64 columns), and workgroup 0 brings the next panel [q0, q1)'s targets up to
// date and solves its diagonal block with its inverse inv (column-major;
// transposed for modes 2 and 3).  mode 0: L, ascending, y in place; mode 1: U,
// descending, the solution to x at the pivot columns; mode 2: U^T, ascending,
// h in y, w to x; mode 3: L^T, descending, w in place in x.  A target is a row
// (modes 0, 1, 3) or a column (mode 2: only those pivoted after the next
// panel).  p0 == p1: the next panel's diagonal solve only.
template <typename T>
__device__ __forceinline__ void tail_step_body(const TailView& TV, const T* __restrict__ vals, int p0, int p1, int q0,
                                               int q1, const T* __restrict__ inv, int n, T* __restrict__ y,
                                               T* __restrict__ x, int nrhs, int mode, int first, int count, int blk)
{
    __shared__ T ys[kNB];
    __shared__ T part[4][kNB];
    __shared__ int64_t rowq[kNB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int np = p1 - p0, nq = q1 - q0, t0 = TV.t0;
    const bool tr = mode >= 2;
    const int b = p0 + lane;
    const int pb = lane < np ? TV.tpiv[b] : 0;
    const int64_t rb = (tr && lane < np) ? TV.trow[b] : 0;    // row b of the current panel
    // coefficient of target e for the current panel's lane b:
    //   modes 0, 1: X_e[piv b];  mode 2: X_b[e];  mode 3: X_b[piv e]
    if (blk == 0) {
        // every load of a phase is issued before its first use: wavefront w
        // takes the next panel's targets w, w+4, ..; the inverse's columns are
        // split the same way and the four partial sums combined in LDS
        const int t = threadIdx.x;
        if (t < nq) rowq[t] = mode <= 1 ? TV.trow[q0 + t] : (int64_t)TV.tpiv[q0 + t];
        __syncthreads();
        T c[kNB / 4], iv[kNB / 4];
#pragma unroll
        for (int q = 0; q < kNB / 4; q++) {
            const int i = wv + 4 * q;
            c[q] = (i < nq && lane < np) ? (mode <= 1 ? vals[rowq[i] + pb] : vals[rb + rowq[i]]) : T(0);
            iv[q] = (i < nq && lane < nq) ? (tr ? inv[lane * kNB + i] : inv[i * kNB + lane]) : T(0);
        }
        for (int r = 0; r < nrhs; r++) {
            T* yr = y + (int64_t)r * n + t0;
            T* xr = x + (int64_t)r * n + t0;
            const T v = lane < np ? (mode == 0 ? yr[b] : mode == 1 ? xr[pb] : xr[b]) : T(0);
            if (t < nq) ys[t] = mode <= 1 ? yr[q0 + t] : mode == 2 ? yr[rowq[t]] : xr[q0 + t];
            __syncthreads();
            if (np > 0) {
#pragma unroll
                for (int q = 0; q < kNB / 4; q++) {
                    const int i = wv + 4 * q;
                    if (i >= nq) break;
                    const T acc = wave_sum(c[q] * v);
                    if (lane == 0) ys[i] -= acc;
                }
            }
            __syncthreads();
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < kNB / 4; q++) {
                const int jj = wv + 4 * q;
                if (jj < nq) acc += iv[q] * ys[jj];
            }
            part[wv][lane] = acc;
            __syncthreads();
            if (t < nq) {
                const T o = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
                if (mode == 0) yr[q0 + t] = o;
                else if (mode == 1) xr[TV.tpiv[q0 + t]] = o;
                else xr[q0 + t] = o;
            }
            __syncthreads();
        }
        return;
    }
    const int k = (blk - 1) * 4 + wv;
    if (k >= count) return;
    const int e = first + k;
    if (mode == 2 && TV.tstep[e] < q1) return;             // a column solved at or before the next panel
    T coef = T(0);
    if (lane < np) {
        if (mode <= 1) coef = vals[TV.trow[e] + pb];
        else if (mode == 2) coef = vals[rb + e];
        else coef = vals[rb + TV.tpiv[e]];
    }
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n + t0;
        T* xr = x + (int64_t)r * n + t0;
        const T v = lane < np ? (mode == 0 ? yr[b] : mode == 1 ? xr[pb] : xr[b]) : T(0);
        const T acc = wave_sum(coef * v);
        if (lane == 0) {
            if (mode == 3) xr[e] -= acc;
            else yr[e] -= acc;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tail_step(TailView TV, const T* __restrict__ vals, int p0, int p1, int q0, int q1,
                                                   const T* __restrict__ inv, int n, T* __restrict__ y,
                                                   T* __restrict__ x, int nrhs, int mode, int first, int count)
{
    tail_step_body<T>(TV, vals, p0, p1, q0, q1, inv, n, y, x, nrhs, mode, first, count, blockIdx.x);
}

// the same step of several large supernodes of one solve level in one
// launch: a job per workgroup (its view, that view's step and the
// workgroup's block within it), each block doing what k_tail_step's does
template <typename T>
__global__ __launch_bounds__(256) void k_view_steps(const ViewDesc* __restrict__ vd, const SolveJob* __restrict__ jobs,
                                                    const T* __restrict__ vals, int n, T* __restrict__ y,
                                                    T* __restrict__ x, int nrhs, int mode)
{
    const SolveJob J = jobs[blockIdx.x];
    const ViewDesc& V = vd[J.view];
    const T* inv = reinterpret_cast<const T*>(V.inv) + (int64_t)J.inv * kNB * kNB;
    tail_step_body<T>(V.TV, vals, J.p0, J.p1, J.q0, J.q1, inv, n, y, x, nrhs, mode, J.first, J.count, J.blk);
}

// one wavefront per row of a large supernode: the gathers outside its block
template <typename T>
__device__ __forceinline__ void sn_ext_body(const DevLayout& D, const T* __restrict__ vals, int v,
                                            T* __restrict__ y, const T* __restrict__ x, int nrhs, int upper, int blk)
{
    const int lane = threadIdx.x & 63;
    const int m = D.m[v];
    const int a = blk * 4 + (threadIdx.x >> 6);
    if (a >= m) return;
    const int W = D.W[v], lw = D.lw[v], r0 = D.r0[v];
    const T* Pa = vals + D.voff[v] + (int64_t)a * W;
    const int32_t* cols = D.cols + D.coff[v];
    const int n = D.n;
    const int t0 = upper ? lw + m : 0, t1 = upper ? W : lw;
    for (int r = 0; r < nrhs; r++) {
        T* yr = y + (int64_t)r * n;
        const T* xr = upper ? x + (int64_t)r * n : nullptr;
        // the grouped gathers of the level solves (four entries per lane in flight)
        T acc = upper ? gather_x<T, 64>(Pa + t0, cols + t0, xr, t1 - t0, lane)
                      : gather_lq<T, 64>(Pa, cols, D.qinv, yr, t1, lane);
        acc = wave_sum(acc);
        if (lane == 0) yr[r0 + a] -= acc;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_sn_ext(DevLayout D, const T* __restrict__ vals, int v,
                                                T* __restrict__ y, const T* __restrict__ x, int nrhs, int upper)
{
    sn_ext_body<T>(D, vals, v, y, x, nrhs, upper, blockIdx.x);
}
// several large supernodes' gathers in one launch (jobs: node, block pairs)
template <typename T>
__global__ __launch_bounds__(256) void k_sn_ext_views(DevLayout D, const T* __restrict__ vals,
                                                      const int32_t* __restrict__ jobs, T* __restrict__ y,
                                                      const T* __restrict__ x, int nrhs, int upper)
{
    sn_ext_body<T>(D, vals, jobs[2 * blockIdx.x], y, x, nrhs, upper, jobs[2 * blockIdx.x + 1]);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st)
{
    if (bytes <= 0) return hipSuccess;
    int64_t n64 = bytes / 8;
    if (n64 > 0) {
        unsigned g = (unsigned)std::min<int64_t>(nblk(n64, 256), 65536);
        hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, st, (uint64_t*)p, n64);
    }
    int64_t rem = bytes - n64 * 8;
    if (rem > 0) hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, st, (uint8_t*)p + n64 * 8, rem);
    return hipGetLastError();
}

hipError_t launch_factor_tile(bool fp32, const DevLayout& D, void* vals, const int32_t* tiles, int32_t ntiles,
                              hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_factor_tile<float>, dim3(ntiles), dim3(256), 0, st, D, (float*)vals, tiles, ntiles);
    else hipLaunchKernelGGL(k_factor_tile<double>, dim3(ntiles), dim3(256), 0, st, D, (double*)vals, tiles, ntiles);
    return hipGetLastError();
}

hipError_t launch_sn_lext(bool fp32, const DevLayout& D, const TailView& TV, const void* vals, int32_t v, void* y,
                          int32_t nrhs, hipStream_t st)
{
    if (TV.mT <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_sn_ext<float>, dim3(nblk(TV.mT, 4)), dim3(256), 0, st, D, (const float*)vals, v, (float*)y, (const float*)nullptr, nrhs, 0);
    else hipLaunchKernelGGL(k_sn_ext<double>, dim3(nblk(TV.mT, 4)), dim3(256), 0, st, D, (const double*)vals, v, (double*)y, (const double*)nullptr, nrhs, 0);
    return hipGetLastError();
}

hipError_t launch_sn_utext(bool fp32, const DevLayout& D, const TailView& TV, const void* vals, int32_t v, void* y,
                           const void* x, int32_t nrhs, hipStream_t st)
{
    if (TV.mT <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_sn_ext<float>, dim3(nblk(TV.mT, 4)), dim3(256), 0, st, D, (const float*)vals, v, (float*)y, (const float*)x, nrhs, 1);
    else hipLaunchKernelGGL(k_sn_ext<double>, dim3(nblk(TV.mT, 4)), dim3(256), 0, st, D, (const double*)vals, v, (double*)y, (const double*)x, nrhs, 1);
    return hipGetLastError();
}

hipError_t launch_sn_ext_views(bool fp32, const DevLayout& D, const void* vals, const int32_t* jobs, int32_t njobs,
                               void* y, const void* x, int32_t nrhs, int32_t upper, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_sn_ext_views<float>, dim3(njobs), dim3(256), 0, st, D, (const float*)vals, jobs, (float*)y, (const float*)x, nrhs, upper);
    else hipLaunchKernelGGL(k_sn_ext_views<double>, dim3(njobs), dim3(256), 0, st, D, (const double*)vals, jobs, (double*)y, (const double*)x, nrhs, upper);
    return hipGetLastError();
}

hipError_t launch_view_steps(bool fp32, const ViewDesc* vd, const SolveJob* jobs, int32_t njobs, const void* vals,
                             int32_t n, void* y, void* x, int32_t nrhs, int32_t mode, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (mode < 0 || mode > 1) return hipErrorInvalidValue;
    if (fp32) hipLaunchKernelGGL(k_view_steps<float>, dim3(njobs), dim3(256), 0, st, vd, jobs, (const float*)vals, n, (float*)y, (float*)x, nrhs, mode);
    else hipLaunchKernelGGL(k_view_steps<double>, dim3(njobs), dim3(256), 0, st, vd, jobs, (const double*)vals, n, (double*)y, (double*)x, nrhs, mode);
    return hipGetLastError();
}

hipError_t launch_scatter(bool fp32, const double* aval, const int64_t* amap, const double* asr,
                          const double* asc, int64_t nnz, void* vals, double* acopy, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_scatter<float>, dim3(nblk(nnz, 256)), dim3(256), 0, st, aval, amap, asr, asc, nnz, (float*)vals, acopy);
    else hipLaunchKernelGGL(k_scatter<double>, dim3(nblk(nnz, 256)), dim3(256), 0, st, aval, amap, asr, asc, nnz, (double*)vals, acopy);
    return hipGetLastError();
}

hipError_t launch_init_pivots(const DevLayout& D, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_pivots, dim3(nblk(D.n, 256)), dim3(256), 0, st, D.n, D.row_node, D.r0, D.pl, D.qinv);
    return hipGetLastError();
}

static const int32_t kRowLdsCap = 4096;   // row accumulator in LDS up to this width
static const int32_t kXcdChunk = 16, kXcdMin = 2048;

size_t factor_rows_lds(bool fp32, int32_t stage, int32_t cap)
{
    const size_t fixed = (size_t)stage * 4 + 129 * 4 + 4 + 128 * 8;   // indices, edge tables (8-byte aligned)
    return (fp32 ? sizeof(float) : sizeof(double)) * ((size_t)stage + (size_t)std::max(cap, 1)) + fixed;
}

hipError_t launch_factor_rows(bool fp32, const DevLayout& D, void* vals, const int32_t* rows, const int64_t* ranges,
                              int32_t nrows, int32_t maxW, double tau, int32_t* pert, int32_t nt, int32_t stage,
                              int32_t lds_cap, int32_t search, const int64_t* inv_off, hipStream_t st)
{
    if (nrows <= 0) return hipSuccess;
    if (stage < kStage || stage > kStageMax || stage % 64) return hipErrorInvalidValue;
    const int32_t cap = std::min(maxW, lds_cap > 0 ? lds_cap : kRowLdsCap);
    if (nt == 0) nt = maxW > 1024 ? 256 : 64;                      // default: 4 waves per row for long rows
    // (room for the block LU of a supernode of up to 64 rows done in this launch)
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    const size_t sh = std::max(factor_rows_lds(fp32, stage, cap), (size_t)nt * (es + 4) + 64 * (es + 1) + 16);
    if (sh > kLdsMax) return hipErrorInvalidValue;
    // launches of many rows: runs of kXcdChunk consecutive rows per XCD
    const int32_t xc = nrows >= kXcdMin ? kXcdChunk : 0;
    const dim3 g(xc ? (unsigned)((nrows + 8 * xc - 1) / (8 * xc) * (8 * xc)) : (unsigned)nrows);
#define ROWS_LAUNCH(TT, NTT) hipLaunchKernelGGL((k_factor_rows<TT, NTT>), g, dim3(NTT), sh, st, D, (TT*)vals, rows, ranges, nrows, cap, (TT)tau, pert, stage, search, inv_off, xc)
    if (fp32) {
        if (nt == 1024) ROWS_LAUNCH(float, 1024);
        else if (nt == 512) ROWS_LAUNCH(float, 512);
        else if (nt == 256) ROWS_LAUNCH(float, 256);
        else if (nt == 128) ROWS_LAUNCH(float, 128);
        else if (nt == 64) ROWS_LAUNCH(float, 64);
        else return hipErrorInvalidValue;
    } else {
        if (nt == 1024) ROWS_LAUNCH(double, 1024);
        else if (nt == 512) ROWS_LAUNCH(double, 512);
        else if (nt == 256) ROWS_LAUNCH(double, 256);
        else if (nt == 128) ROWS_LAUNCH(double, 128);
        else if (nt == 64) ROWS_LAUNCH(double, 64);
        else return hipErrorInvalidValue;
    }
#undef ROWS_LAUNCH
    return hipGetLastError();
}

hipError_t launch_perturb_rows(bool fp32, const DevLayout& D, void* vals, const int32_t* rows, int32_t count,
                               double tau, int32_t* pert, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_perturb_rows<float>, dim3(nblk(count, 256)), dim3(256), 0, st, D, (float*)vals, rows, count, (float)tau, pert);
    else hipLaunchKernelGGL(k_perturb_rows<double>, dim3(nblk(count, 256)), dim3(256), 0, st, D, (double*)vals, rows, count, tau, pert);
    return hipGetLastError();
}

hipError_t launch_factor_chain(bool fp32, const DevLayout& D, void* vals, const int32_t* tasks, const int32_t* sthr,
                               int32_t ntask, int32_t nw, int32_t cap, int32_t sw, double tau, int32_t* pert,
                               int32_t search, const int64_t* inv_off, int32_t spin, hipStream_t st)
{
    if (ntask <= 0) return hipSuccess;
    if (nw < 1 || nw > kChainThreads / 64 || cap < 0 || sw < kInvMax || spin <= 0) return hipErrorInvalidValue;
    const size_t sh = chain_lds(fp32, ntask, nw, cap, sw);
    if (sh > kLdsMax) return hipErrorInvalidValue;
    if (fp32)
        hipLaunchKernelGGL(k_factor_chain<float>, dim3(1), dim3(kChainThreads), sh, st, D, (float*)vals, tasks, sthr, ntask, nw,
                           cap, sw, (float)tau, pert, search, inv_off, spin);
    else
        hipLaunchKernelGGL(k_factor_chain<double>, dim3(1), dim3(kChainThreads), sh, st, D, (double*)vals, tasks, sthr, ntask,
                           nw, cap, sw, tau, pert, search, inv_off, spin);
    return hipGetLastError();
}

size_t chain_lds(bool fp32, int32_t ntask, int32_t nw, int32_t cap, int32_t sw)
{
    return chain_hdr_bytes(ntask) + (size_t)nw * chain_wave_bytes(fp32 ? 4 : 8, cap, sw);
}

hipError_t launch_sn_inverse(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                             int32_t maxm, const int64_t* inv_off, void* uinv, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (maxm > kInvMax || maxm < 1) return hipErrorInvalidValue;
    const int cpb = (maxm + 3) / 4;                // workgroups per node: four columns each
    if (fp32) hipLaunchKernelGGL(k_sn_inverse<float>, dim3(count * cpb), dim3(256), 0, st, D, (const float*)vals, nodes, inv_off, (float*)uinv, cpb);
    else hipLaunchKernelGGL(k_sn_inverse<double>, dim3(count * cpb), dim3(256), 0, st, D, (const double*)vals, nodes, inv_off, (double*)uinv, cpb);
    return hipGetLastError();
}

hipError_t launch_factor_snlu(bool fp32, const DevLayout& D, void* vals, const int32_t* nodes, int32_t count,
                              int32_t maxm, double tau, int32_t* pert, int32_t search, int32_t nt,
                              const int64_t* inv_off, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    size_t sh = (size_t)maxm * (es + 1) + 16;
    if (sh > 60 * 1024) return hipErrorInvalidValue;   // larger blocks need the tiled path
    // blocks of at most kSnLds rows in LDS (two m x m buffers)
    const size_t sl = (size_t)std::min(maxm, kSnLds);
    sh = std::max(sh, 2 * sl * sl * es + sl * (es + 4 + 1) + 16);
    if (nt == 0) nt = 256;
    if (nt != 64 && nt != 256) return hipErrorInvalidValue;
    if (fp32) {
        if (nt == 64) hipLaunchKernelGGL((k_factor_snlu<float, 64>), dim3(count), dim3(64), sh, st, D, (float*)vals, nodes, count, (float)tau, pert, search, inv_off);
        else hipLaunchKernelGGL((k_factor_snlu<float, 256>), dim3(count), dim3(256), sh, st, D, (float*)vals, nodes, count, (float)tau, pert, search, inv_off);
    } else {
        if (nt == 64) hipLaunchKernelGGL((k_factor_snlu<double, 64>), dim3(count), dim3(64), sh, st, D, (double*)vals, nodes, count, tau, pert, search, inv_off);
        else hipLaunchKernelGGL((k_factor_snlu<double, 256>), dim3(count), dim3(256), sh, st, D, (double*)vals, nodes, count, tau, pert, search, inv_off);
    }
    return hipGetLastError();
}

hipError_t launch_lsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                         const int32_t* sn_nodes, int32_t sn_count, const int32_t* split_nodes, int32_t split_count,
                         const int32_t* tasks, int32_t ntasks, void* y, int32_t nrhs, int32_t sn_min, hipStream_t st)
{
    if (sn_min <= 0 || sn_min > kSnSolveRows) sn_min = 0;    // every node by k_lsolve
    if (count > 0) {
        if (fp32) hipLaunchKernelGGL(k_lsolve<float>, dim3(count), dim3(64), 0, st, D, (const float*)vals, nodes, count, (float*)y, nrhs, sn_min);
        else hipLaunchKernelGGL(k_lsolve<double>, dim3(count), dim3(64), 0, st, D, (const double*)vals, nodes, count, (double*)y, nrhs, sn_min);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (sn_min <= 0) return hipSuccess;
    if (sn_count > 0) {
        if (fp32) hipLaunchKernelGGL(k_lsolve_sn<float>, dim3(sn_count), dim3(256), 0, st, D, (const float*)vals, sn_nodes, sn_count, (float*)y, nrhs, sn_min, 0);
        else hipLaunchKernelGGL(k_lsolve_sn<double>, dim3(sn_count), dim3(256), 0, st, D, (const double*)vals, sn_nodes, sn_count, (double*)y, nrhs, sn_min, 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (split_count <= 0 || ntasks <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_lsolve_out<float>, dim3(ntasks), dim3(256), 0, st, D, (const float*)vals, tasks, ntasks, (float*)y, nrhs);
    else hipLaunchKernelGGL(k_lsolve_out<double>, dim3(ntasks), dim3(256), 0, st, D, (const double*)vals, tasks, ntasks, (double*)y, nrhs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fp32) hipLaunchKernelGGL(k_lsolve_sn<float>, dim3(split_count), dim3(256), 0, st, D, (const float*)vals, split_nodes, split_count, (float*)y, nrhs, sn_min, 1);
    else hipLaunchKernelGGL(k_lsolve_sn<double>, dim3(split_count), dim3(256), 0, st, D, (const double*)vals, split_nodes, split_count, (double*)y, nrhs, sn_min, 1);
    return hipGetLastError();
}

hipError_t launch_usolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                         const int32_t* sn_nodes, int32_t sn_count, const int32_t* split_nodes, int32_t split_count,
                         const int32_t* tasks, int32_t ntasks, void* y, void* x, int32_t nrhs, int32_t sn_min,
                         hipStream_t st)
{
    if (sn_min <= 0 || sn_min > kSnSolveRows) sn_min = 0;    // every node by k_usolve
    if (count > 0) {
        if (fp32) hipLaunchKernelGGL(k_usolve<float>, dim3(count), dim3(256), 0, st, D, (const float*)vals, nodes, count, (const float*)y, (float*)x, nrhs, sn_min);
        else hipLaunchKernelGGL(k_usolve<double>, dim3(count), dim3(256), 0, st, D, (const double*)vals, nodes, count, (const double*)y, (double*)x, nrhs, sn_min);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (sn_min <= 0) return hipSuccess;
    if (sn_count > 0) {
        if (fp32) hipLaunchKernelGGL(k_usolve_sn<float>, dim3(sn_count), dim3(256), 0, st, D, (const float*)vals, sn_nodes, sn_count, (const float*)y, (float*)x, nrhs, sn_min, 0);
        else hipLaunchKernelGGL(k_usolve_sn<double>, dim3(sn_count), dim3(256), 0, st, D, (const double*)vals, sn_nodes, sn_count, (const double*)y, (double*)x, nrhs, sn_min, 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (split_count <= 0 || ntasks <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_usolve_out<float>, dim3(ntasks), dim3(256), 0, st, D, (const float*)vals, tasks, ntasks, (float*)y, (const float*)x, nrhs);
    else hipLaunchKernelGGL(k_usolve_out<double>, dim3(ntasks), dim3(256), 0, st, D, (const double*)vals, tasks, ntasks, (double*)y, (const double*)x, nrhs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fp32) hipLaunchKernelGGL(k_usolve_sn<float>, dim3(split_count), dim3(256), 0, st, D, (const float*)vals, split_nodes, split_count, (const float*)y, (float*)x, nrhs, sn_min, 1);
    else hipLaunchKernelGGL(k_usolve_sn<double>, dim3(split_count), dim3(256), 0, st, D, (const double*)vals, split_nodes, split_count, (const double*)y, (double*)x, nrhs, sn_min, 1);
    return hipGetLastError();
}

hipError_t launch_lsolve_chain(bool fp32, const DevLayout& D, const void* vals, const int32_t* lev_ptr,
                               const int32_t* nodes, int32_t l0, int32_t l1, void* y, int32_t nrhs, hipStream_t st)
{
    if (l1 <= l0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_lsolve_chain<float>, dim3(1), dim3(64 * kChainWaves), 0, st, D, (const float*)vals, lev_ptr, nodes, l0, l1, (float*)y, nrhs);
    else hipLaunchKernelGGL(k_lsolve_chain<double>, dim3(1), dim3(64 * kChainWaves), 0, st, D, (const double*)vals, lev_ptr, nodes, l0, l1, (double*)y, nrhs);
    return hipGetLastError();
}

hipError_t launch_usolve_chain(bool fp32, const DevLayout& D, const void* vals, const int32_t* lev_ptr,
                               const int32_t* nodes, int32_t l0, int32_t l1, const void* y, void* x, int32_t nrhs,
                               hipStream_t st)
{
    if (l1 <= l0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_usolve_chain<float>, dim3(1), dim3(64 * kChainWaves), 0, st, D, (const float*)vals, lev_ptr, nodes, l0, l1, (const float*)y, (float*)x, nrhs);
    else hipLaunchKernelGGL(k_usolve_chain<double>, dim3(1), dim3(64 * kChainWaves), 0, st, D, (const double*)vals, lev_ptr, nodes, l0, l1, (const double*)y, (double*)x, nrhs);
    return hipGetLastError();
}

hipError_t launch_utsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                          const int32_t* blk_nodes, int32_t blk_count, const int32_t* tasks, int32_t ntasks,
                          void* h, void* w, int32_t nrhs, hipStream_t st)
{
    if (count > 0) {
        if (fp32) hipLaunchKernelGGL(k_utsolve<float>, dim3(count), dim3(256), 0, st, D, (const float*)vals, nodes, count, (const float*)h, (float*)w, nrhs);
        else hipLaunchKernelGGL(k_utsolve<double>, dim3(count), dim3(256), 0, st, D, (const double*)vals, nodes, count, (const double*)h, (double*)w, nrhs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (blk_count <= 0) return hipSuccess;
    if (ntasks > 0) {
        if (fp32) hipLaunchKernelGGL((k_tsolve_out<float, true>), dim3(ntasks), dim3(256), 0, st, D, (const float*)vals, tasks, ntasks, (float*)h, (const float*)w, nrhs);
        else hipLaunchKernelGGL((k_tsolve_out<double, true>), dim3(ntasks), dim3(256), 0, st, D, (const double*)vals, tasks, ntasks, (double*)h, (const double*)w, nrhs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (fp32) hipLaunchKernelGGL(k_utsolve_blk<float>, dim3(blk_count), dim3(256), 0, st, D, (const float*)vals, blk_nodes, blk_count, (float*)h, (float*)w, nrhs);
    else hipLaunchKernelGGL(k_utsolve_blk<double>, dim3(blk_count), dim3(256), 0, st, D, (const double*)vals, blk_nodes, blk_count, (double*)h, (double*)w, nrhs);
    return hipGetLastError();
}

hipError_t launch_ltsolve(bool fp32, const DevLayout& D, const void* vals, const int32_t* nodes, int32_t count,
                          const int32_t* blk_nodes, int32_t blk_count, const int32_t* tasks, int32_t ntasks,
                          void* w, int32_t nrhs, hipStream_t st)
{
    if (count > 0) {
        if (fp32) hipLaunchKernelGGL(k_ltsolve<float>, dim3(count), dim3(256), 0, st, D, (const float*)vals, nodes, count, (float*)w, nrhs);
        else hipLaunchKernelGGL(k_ltsolve<double>, dim3(count), dim3(256), 0, st, D, (const double*)vals, nodes, count, (double*)w, nrhs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (blk_count <= 0) return hipSuccess;
    if (ntasks > 0) {
        if (fp32) hipLaunchKernelGGL((k_tsolve_out<float, false>), dim3(ntasks), dim3(256), 0, st, D, (const float*)vals, tasks, ntasks, (float*)w, (const float*)w, nrhs);
        else hipLaunchKernelGGL((k_tsolve_out<double, false>), dim3(ntasks), dim3(256), 0, st, D, (const double*)vals, tasks, ntasks, (double*)w, (const double*)w, nrhs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (fp32) hipLaunchKernelGGL(k_ltsolve_blk<float>, dim3(blk_count), dim3(256), 0, st, D, (const float*)vals, blk_nodes, blk_count, (float*)w, nrhs);
    else hipLaunchKernelGGL(k_ltsolve_blk<double>, dim3(blk_count), dim3(256), 0, st, D, (const double*)vals, blk_nodes, blk_count, (double*)w, nrhs);
    return hipGetLastError();
}

hipError_t launch_permute_in(bool fp32, int32_t n, int32_t nrhs, const int32_t* perm, const double* scale,
                             const double* src, int64_t ld, void* dst, hipStream_t st)
{
    int64_t tot = (int64_t)n * nrhs;
    if (tot <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_permute_in<float>, dim3(nblk(tot, 256)), dim3(256), 0, st, n, nrhs, perm, scale, src, ld, (float*)dst);
    else hipLaunchKernelGGL(k_permute_in<double>, dim3(nblk(tot, 256)), dim3(256), 0, st, n, nrhs, perm, scale, src, ld, (double*)dst);
    return hipGetLastError();
}

hipError_t launch_permute_out(bool fp32, int32_t n, int32_t nrhs, const int32_t* perm, const double* scale,
                              const void* z, double* dst, int64_t ld, int32_t accumulate, hipStream_t st)
{
    int64_t tot = (int64_t)n * nrhs;
    if (tot <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_permute_out<float>, dim3(nblk(tot, 256)), dim3(256), 0, st, n, nrhs, perm, scale, (const float*)z, dst, ld, accumulate);
    else hipLaunchKernelGGL(k_permute_out<double>, dim3(nblk(tot, 256)), dim3(256), 0, st, n, nrhs, perm, scale, (const double*)z, dst, ld, accumulate);
    return hipGetLastError();
}

hipError_t launch_residual(int32_t n, int32_t nrhs, const int64_t* rp, const int32_t* ci, const double* av,
                           const double* b, int64_t ldb, const double* x, int64_t ldx, double* r, hipStream_t st)
{
    int64_t tot = (int64_t)n * nrhs;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual, dim3(nblk(tot, 256)), dim3(256), 0, st, n, nrhs, rp, ci, av, b, ldb, x, ldx, r);
    return hipGetLastError();
}

hipError_t launch_norms(int32_t n, int32_t nrhs, const int64_t* rp, const double* av, const double* r,
                        const double* x, int64_t ldx, const double* b, int64_t ldb, const int32_t* seg,
                        int32_t nseg, double* out, hipStream_t st)
{
    hipError_t e = launch_zero(out, sizeof(double) * kNormSlots * ((size_t)nrhs + 1) * (size_t)nseg, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms, dim3(nblk(n, 256)), dim3(256), 0, st, n, nrhs, rp, av, r, x, ldx, b, ldb, seg, nseg, out);
    return hipGetLastError();
}

hipError_t launch_gather_values(int64_t nnz, const int64_t* idx, const double* src, double* dst, hipStream_t st)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nblk(nnz, 256)), dim3(256), 0, st, nnz, idx, src, dst);
    return hipGetLastError();
}

hipError_t launch_grad(int32_t n, int32_t nrhs, int64_t ld, const int64_t* rp, const int32_t* ci, const double* lam,
                       const double* x, double* g, hipStream_t st)
{
    hipLaunchKernelGGL(k_grad, dim3(nblk(n, 256)), dim3(256), 0, st, n, nrhs, ld, rp, ci, lam, x, g);
    return hipGetLastError();
}

hipError_t launch_tail_init(const TailView& T, hipStream_t st)
{
    if (T.mT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tail_init, dim3(nblk(T.nc, 256)), dim3(256), 0, st, T.nc, T.tstep);
    return hipGetLastError();
}

hipError_t launch_tail_panel(bool fp32, const DevLayout& D, const TailView& T, void* vals, int32_t p0, int32_t p1,
                             int32_t c0, int32_t c1, double tau, int32_t* pert, int32_t search, hipStream_t st)
{
    if (p1 - p0 > kNB || p1 <= p0) return hipErrorInvalidValue;
    size_t es = fp32 ? sizeof(float) : sizeof(double);
    size_t sh = (size_t)(p1 - p0) * (c1 - c0) * es;
    if (!search && c0 == p0 && c1 == p1) {
        if (fp32) hipLaunchKernelGGL(k_tail_panel_reg<float>, dim3(1), dim3(64), 0, st, D, T, (float*)vals, p0, p1, (float)tau, pert);
        else hipLaunchKernelGGL(k_tail_panel_reg<double>, dim3(1), dim3(64), 0, st, D, T, (double*)vals, p0, p1, tau, pert);
    } else if (c1 - c0 <= 64) {
        if (fp32) hipLaunchKernelGGL((k_tail_panel_lds4<float, 8>), dim3(1), dim3(512), sh, st, D, T, (float*)vals, p0, p1, c0, c1, (float)tau, pert, search);
        else hipLaunchKernelGGL((k_tail_panel_lds4<double, 8>), dim3(1), dim3(512), sh, st, D, T, (double*)vals, p0, p1, c0, c1, tau, pert, search);
    } else {
        // wide window: steps in LDS, the window itself too when it fits
        const size_t tsz = ((size_t)(c1 - c0) * 4 + 15) & ~(size_t)15;
        const size_t stg = tsz + sh;
        if (stg <= 60 * 1024) {
            if (fp32) hipLaunchKernelGGL((k_tail_panel_wide<float, 256, true>), dim3(1), dim3(256), stg, st, D, T, (float*)vals, p0, p1, c0, c1, (float)tau, pert, search, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
            else hipLaunchKernelGGL((k_tail_panel_wide<double, 256, true>), dim3(1), dim3(256), stg, st, D, T, (double*)vals, p0, p1, c0, c1, tau, pert, search, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
        } else if (tsz <= 60 * 1024) {
            if (fp32) hipLaunchKernelGGL((k_tail_panel_wide<float, 1024, false>), dim3(1), dim3(1024), tsz, st, D, T, (float*)vals, p0, p1, c0, c1, (float)tau, pert, search, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
            else hipLaunchKernelGGL((k_tail_panel_wide<double, 1024, false>), dim3(1), dim3(1024), tsz, st, D, T, (double*)vals, p0, p1, c0, c1, tau, pert, search, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
        } else {
            if (fp32) hipLaunchKernelGGL((k_tail_panel<float, false>), dim3(1), dim3(256), 0, st, D, T, (float*)vals, p0, p1, c0, c1, (float)tau, pert, search);
            else hipLaunchKernelGGL((k_tail_panel<double, false>), dim3(1), dim3(256), 0, st, D, T, (double*)vals, p0, p1, c0, c1, tau, pert, search);
        }
    }
    return hipGetLastError();
}

hipError_t launch_tail_trsm(bool fp32, const TailView& T, void* vals, int32_t p0, int32_t p1, int32_t c1, int32_t kb0,
                            int32_t kof, const int32_t* blocks, int32_t nblocks, hipStream_t st)
{
    int nA = (int)nblk(std::max(T.nc - c1, 0), 64);
    int nB = (int)nblk(std::max(T.mT - p1, 0), 64);
    const int grid = blocks ? nblocks : nA + nB;
    if (grid <= 0) return hipSuccess;
    if (kof < 0 || kof + (p1 - p0) > kNB * kGroup) return hipErrorInvalidValue;
    if (fp32) hipLaunchKernelGGL(k_tail_trsm<float>, dim3(grid), dim3(64), 0, st, T, (float*)vals, p0, p1, c1, nA, kb0, kof, blocks, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    else hipLaunchKernelGGL(k_tail_trsm<double>, dim3(grid), dim3(64), 0, st, T, (double*)vals, p0, p1, c1, nA, kb0, kof, blocks, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    return hipGetLastError();
}

hipError_t launch_tail_gemm(bool fp32, const TailView& T, void* vals, int32_t kb0, int32_t K, int32_t rb, int32_t re,
                            int32_t cg0, int32_t mstep, int32_t gp0, int32_t gnp, const uint32_t* tiles,
                            int32_t ntiles, const int32_t* kbnd, hipStream_t st)
{
    int gx = gnp > 0 ? (int)nblk(gnp, 64) : (int)nblk(std::max(T.nc - cg0, 0), 64);
    int gy = (int)nblk(std::max(re - rb, 0), 64);
    if (gx == 0 || gy == 0 || K <= 0) return hipSuccess;
    if (K > kNB * kGroup || re > T.mT || gnp > kNB) return hipErrorInvalidValue;
    int kb1 = K, kb2 = K, kb3 = K;
    if (kbnd) {
        kb1 = kbnd[1]; kb2 = kbnd[2]; kb3 = kbnd[3];
        if (kbnd[0] != 0 || kb1 < 0 || kb1 > kb2 || kb2 > kb3 || kb3 > K) return hipErrorInvalidValue;
    }
    const int swz = gy >= 8 && gx >= 4;
    unsigned grid = swz ? 8u * (unsigned)((gy + 3) / 4) * (unsigned)((gx + 1) / 2) : (unsigned)(gx * gy);
    if (tiles) {
        if (ntiles <= 0) return hipSuccess;
        grid = (unsigned)ntiles;
    }
    if (fp32) hipLaunchKernelGGL(k_tail_gemm<float>, dim3(grid), dim3(256), 0, st, T, (float*)vals, kb0, K, rb, re, cg0, mstep, gx, gy, swz, gp0, gnp, tiles, kb1, kb2, kb3, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    else hipLaunchKernelGGL(k_tail_gemm<double>, dim3(grid), dim3(256), 0, st, T, (double*)vals, kb0, K, rb, re, cg0, mstep, gx, gy, swz, gp0, gnp, tiles, kb1, kb2, kb3, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    return hipGetLastError();
}

hipError_t launch_tail_lext(bool fp32, const DevLayout& D, const void* vals, int32_t tail_node0, int32_t t0,
                            void* y, int32_t nrhs, hipStream_t st)
{
    (void)tail_node0;
    int mT = D.n - t0;
    if (mT <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_tail_lext<float>, dim3(nblk(mT, 4)), dim3(256), 0, st, D, (const float*)vals, t0, (float*)y, nrhs);
    else hipLaunchKernelGGL(k_tail_lext<double>, dim3(nblk(mT, 4)), dim3(256), 0, st, D, (const double*)vals, t0, (double*)y, nrhs);
    return hipGetLastError();
}

hipError_t launch_tail_utext(bool fp32, const DevLayout& D, const TailView& T, const void* vals, void* h,
                             const void* w, int32_t nrhs, hipStream_t st)
{
    if (T.mT <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_tail_utext<float>, dim3(nblk(T.mT, 4)), dim3(256), 0, st, D, T, (const float*)vals, (float*)h, (const float*)w, nrhs);
    else hipLaunchKernelGGL(k_tail_utext<double>, dim3(nblk(T.mT, 4)), dim3(256), 0, st, D, T, (const double*)vals, (double*)h, (const double*)w, nrhs);
    return hipGetLastError();
}

hipError_t launch_tail_dinv(bool fp32, const TailView& T, const void* vals, const int32_t* spanels, int32_t nsp,
                            void* out, hipStream_t st)
{
    if (nsp <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_tail_dinv<float>, dim3(2 * nsp), dim3(64), 0, st, T, (const float*)vals, spanels, (float*)out, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    else hipLaunchKernelGGL(k_tail_dinv<double>, dim3(2 * nsp), dim3(64), 0, st, T, (const double*)vals, spanels, (double*)out, (const ViewDesc*)nullptr, (const ViewJob*)nullptr);
    return hipGetLastError();
}

size_t tail_panel_wide_lds(bool fp32, int32_t np, int32_t wc)
{
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    const size_t tsz = ((size_t)wc * 4 + 15) & ~(size_t)15;
    const size_t stg = tsz + (size_t)np * wc * es;
    return (wc > 64 && np <= kNB && stg <= 60 * 1024) ? stg : 0;
}

hipError_t launch_tail_panel_views(bool fp32, const DevLayout& D, const ViewDesc* vd, void* vals, const ViewJob* jobs,
                                   int32_t njobs, size_t lds, double tau, int32_t* pert, int32_t search, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (!vd || !jobs || lds == 0 || lds > 60 * 1024) return hipErrorInvalidValue;
    const TailView none{};
    if (fp32) hipLaunchKernelGGL((k_tail_panel_wide<float, 256, true>), dim3(njobs), dim3(256), lds, st, D, none, (float*)vals, 0, 0, 0, 0, (float)tau, pert, search, vd, jobs);
    else hipLaunchKernelGGL((k_tail_panel_wide<double, 256, true>), dim3(njobs), dim3(256), lds, st, D, none, (double*)vals, 0, 0, 0, 0, tau, pert, search, vd, jobs);
    return hipGetLastError();
}

hipError_t launch_tail_trsm_views(bool fp32, const ViewDesc* vd, void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (!vd || !jobs) return hipErrorInvalidValue;
    const TailView none{};
    if (fp32) hipLaunchKernelGGL(k_tail_trsm<float>, dim3(njobs), dim3(64), 0, st, none, (float*)vals, 0, 0, 0, 0, 0, 0, (const int32_t*)nullptr, vd, jobs);
    else hipLaunchKernelGGL(k_tail_trsm<double>, dim3(njobs), dim3(64), 0, st, none, (double*)vals, 0, 0, 0, 0, 0, 0, (const int32_t*)nullptr, vd, jobs);
    return hipGetLastError();
}

hipError_t launch_tail_gemm_views(bool fp32, const ViewDesc* vd, void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (!vd || !jobs) return hipErrorInvalidValue;
    const TailView none{};
    if (fp32) hipLaunchKernelGGL(k_tail_gemm<float>, dim3(njobs), dim3(256), 0, st, none, (float*)vals, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, (const uint32_t*)nullptr, 0, 0, 0, vd, jobs);
    else hipLaunchKernelGGL(k_tail_gemm<double>, dim3(njobs), dim3(256), 0, st, none, (double*)vals, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, (const uint32_t*)nullptr, 0, 0, 0, vd, jobs);
    return hipGetLastError();
}

hipError_t launch_tail_dinv_views(bool fp32, const ViewDesc* vd, const void* vals, const ViewJob* jobs, int32_t njobs,
                                  hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    if (!vd || !jobs) return hipErrorInvalidValue;
    const TailView none{};
    if (fp32) hipLaunchKernelGGL(k_tail_dinv<float>, dim3(njobs), dim3(64), 0, st, none, (const float*)vals, (const int32_t*)nullptr, (float*)nullptr, vd, jobs);
    else hipLaunchKernelGGL(k_tail_dinv<double>, dim3(njobs), dim3(64), 0, st, none, (const double*)vals, (const int32_t*)nullptr, (double*)nullptr, vd, jobs);
    return hipGetLastError();
}

hipError_t launch_tail_step(bool fp32, const TailView& T, const void* vals, int32_t p0, int32_t p1, int32_t q0, int32_t q1,
                            const void* inv, int32_t n, void* y, void* x, int32_t nrhs, int32_t mode, hipStream_t st)
{
    const int np = p1 - p0, nq = q1 - q0;
    if (np < 0 || np > kNB || nq <= 0 || nq > kNB || mode < 0 || mode > 3) return hipErrorInvalidValue;
    const bool asc = mode == 0 || mode == 2;
    if (np > 0 && (asc ? q0 != p1 : q1 != p0)) return hipErrorInvalidValue;
    if (q0 < 0 || q1 > T.mT) return hipErrorInvalidValue;
    if (mode == 2 && T.nc != T.mT) return hipErrorInvalidValue;   // columns of the tail only
    int first = 0, count = 0;
    if (np > 0) {
        if (mode == 0) { first = q1; count = T.mT - q1; }
        else if (mode == 2) { first = 0; count = T.mT; }
        else { first = 0; count = q0; }
    }
    const unsigned grid = 1u + nblk(count, 4);
    if (fp32) hipLaunchKernelGGL(k_tail_step<float>, dim3(grid), dim3(256), 0, st, T, (const float*)vals, p0, p1, q0, q1,
                                 (const float*)inv, n, (float*)y, (float*)x, nrhs, mode, first, count);
    else hipLaunchKernelGGL(k_tail_step<double>, dim3(grid), dim3(256), 0, st, T, (const double*)vals, p0, p1, q0, q1,
                            (const double*)inv, n, (double*)y, (double*)x, nrhs, mode, first, count);
    return hipGetLastError();
}

}  // namespace hylu
