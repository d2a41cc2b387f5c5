// Symbolic factorisation, supernode detection, task-graph levels and the
// panel layout (HYLU Sec. 2.1 last step, Sec. 2.2 supernode definition,
// Sec. 2.2.1 levelisation).
//
// The symbolic step forms the exact structure of every row of L and U in
// row order (the up-looking order of Sec. 2.2): row i is the union of row i
// of B and, for every k < i met so far in ascending order, the strict upper
// structure of row k.  Consecutive rows whose U structures agree once the
// leading row is dropped form a chain run (the supernode definition); all rows
// of a run share the columns past the run, so when the smallest k of a run
// enters row i the whole rest of the run and its shared columns enter
// together and the other rows of the run need no visit.  Runs are what keeps
// this pass far below the O(flops) cost of the row-by-row union.
#include <algorithm>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <vector>

#include "analysis.hpp"

namespace hylu {

// Is the strict upper structure of run R's last row, less its first entry p,
// contained in U(p, >p)?  (Both sorted; p's run may still be open.)  Then a
// row that takes run R as a source and also takes p needs nothing else of R.
static bool run_covered_by(const Symbolic& s, int32_t R, int32_t p, int32_t open_run, int32_t open_start,
                           const std::vector<int32_t>& open_u)
{
    const int32_t rs = s.run_start[R], last = s.run_start[R + 1] - 1;
    const int32_t* a = s.run_u.data() + s.run_up[R] + (last - rs);
    const int64_t na = s.run_up[R + 1] - s.run_up[R] - (last - rs);
    const int32_t Rp = s.run_of[p];
    const int32_t* b;
    int64_t nb;
    if (Rp == open_run) {
        b = open_u.data() + (p - open_start);
        nb = (int64_t)open_u.size() - (p - open_start);
    } else {
        const int32_t rsp = s.run_start[Rp];
        b = s.run_u.data() + s.run_up[Rp] + (p - rsp);
        nb = s.run_up[Rp + 1] - s.run_up[Rp] - (p - rsp);
    }
    int64_t q = 0;
    for (int64_t t = 1; t < na; t++) {
        while (q < nb && b[q] < a[t]) q++;
        if (q == nb || b[q] != a[t]) return false;
    }
    return true;
}

bool symbolic_factor(const Csr& b, Symbolic& s)
{
    const int32_t n = b.n;
    s = Symbolic();
    s.n = n;
    s.lp.assign(n + 1, 0);
    s.run_of.assign(n, -1);
    s.ucount.assign(n, 0);
    s.run_up.push_back(0);
    std::vector<int32_t> mark(n, -1), done(n, -1);
    std::vector<int8_t> covered(n + 1, -1);            // per run: pruning test result (-1 not yet known)
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
    std::vector<int32_t> ubuf, open_u;                 // open_u: strict U of the open run's first row
    int32_t open_run = -1, open_start = 0;
    for (int32_t i = 0; i < n; i++) {
        ubuf.clear();
        mark[i] = i;
        for (int64_t q = b.rp[i]; q < b.rp[i + 1]; q++) {
            int32_t j = b.ci[q];
            if (mark[j] == i) continue;
            mark[j] = i;
            if (j < i) heap.push(j); else ubuf.push_back(j);
        }
        while (!heap.empty()) {
            int32_t k = heap.top();
            heap.pop();
            if (done[k] == i) continue;
            int32_t R = s.run_of[k];
            int32_t rs, last;
            const int32_t* ul;
            int64_t ulen;
            if (R == open_run) {
                rs = open_start; last = i - 1;
                ul = open_u.data(); ulen = (int64_t)open_u.size();
            } else {
                rs = s.run_start[R]; last = s.run_start[R + 1] - 1;
                ul = s.run_u.data() + s.run_up[R]; ulen = s.run_up[R + 1] - s.run_up[R];
            }
            s.lint.push_back(k);
            s.lint.push_back(last);
            for (int32_t t = k; t <= last; t++) { done[t] = i; mark[t] = i; }
            // pruning: when the run's structure past its first entry p (< i)
            // lies inside U(p, >p), the source p (taken later, p > last)
            // brings all of it; only p is queued here
            if (R != open_run && last - rs < ulen) {
                const int32_t pj = ul[last - rs];
                if (pj < i) {
                    if (covered[R] < 0) covered[R] = run_covered_by(s, R, pj, open_run, open_start, open_u) ? 1 : 0;
                    if (covered[R] == 1) {
                        if (mark[pj] != i) { mark[pj] = i; heap.push(pj); }
                        continue;
                    }
                }
            }
            for (int64_t t = last - rs; t < ulen; t++) {
                int32_t j = ul[t];
                if (mark[j] == i) continue;
                mark[j] = i;
                if (j < i) heap.push(j); else ubuf.push_back(j);
            }
        }
        s.lp[i + 1] = (int64_t)s.lint.size() / 2;
        std::sort(ubuf.begin(), ubuf.end());
        s.ucount[i] = (int64_t)ubuf.size();
        // does row i extend the open run?  U(i-1,:) \ {i-1, i} == U(i,:) \ {i}
        bool chain = false;
        if (open_run >= 0) {
            int64_t off = (i - 1) - open_start;       // U(i-1, > i-1) = open_u[off:]
            int64_t plen = (int64_t)open_u.size() - off;
            if (plen >= 1 && open_u[off] == i && plen - 1 == (int64_t)ubuf.size())
                chain = std::equal(ubuf.begin(), ubuf.end(), open_u.begin() + off + 1);
        }
        if (chain) {
            s.run_of[i] = open_run;
        } else {
            if (open_run >= 0) {
                s.run_u.insert(s.run_u.end(), open_u.begin(), open_u.end());
                s.run_up.push_back((int64_t)s.run_u.size());
            }
            open_run = (int32_t)s.run_start.size();
            s.run_start.push_back(i);
            open_start = i;
            open_u = ubuf;
            s.run_of[i] = open_run;
        }
    }
    if (open_run >= 0) {
        s.run_u.insert(s.run_u.end(), open_u.begin(), open_u.end());
        s.run_up.push_back((int64_t)s.run_u.size());
    }
    s.run_start.push_back(n);
    symbolic_counts(s);
    return true;
}

void symbolic_counts(Symbolic& s)
{
    const int32_t n = s.n;
    s.nnz_l = s.nnz_u = 0;
    // l_k from the intervals, F = sum_k l_k (1 + 2 u_k)
    std::vector<int64_t> diff(n + 1, 0);
    for (int64_t t = 0; t < s.lp[n]; t++) {
        diff[s.lint[2 * t]]++;
        diff[s.lint[2 * t + 1] + 1]--;
        s.nnz_l += s.lint[2 * t + 1] - s.lint[2 * t] + 1;
    }
    s.lcount.assign(n, 0);
    int64_t acc = 0;
    uint64_t F = 0;
    for (int32_t k = 0; k < n; k++) {
        acc += diff[k];
        s.lcount[k] = acc;
        F += (uint64_t)acc * (1 + 2 * (uint64_t)s.ucount[k]);
        s.nnz_u += 1 + s.ucount[k];
    }
    s.flops = F;
}

// strict upper structure of row k: a suffix of its run's stored list
static inline void row_upper(const Symbolic& s, int32_t k, const int32_t*& p, int64_t& len)
{
    int32_t R = s.run_of[k];
    int64_t base = s.run_up[R] + (k - s.run_start[R]);
    p = s.run_u.data() + base;
    len = s.run_up[R + 1] - base;
}

void make_nodes(const Symbolic& s, int32_t sn_min, int32_t sn_max, Nodes& nd)
{
    const int32_t n = s.n;
    if (sn_min < 2) sn_min = 2;
    if (sn_max < 1) sn_max = 1;
    nd = Nodes();
    nd.ptr.push_back(0);
    nd.of_row.assign(n, 0);
    for (int32_t R = 0; R < s.nruns(); R++) {
        int32_t rs = s.run_start[R], re = s.run_start[R + 1];
        for (int32_t c0 = rs; c0 < re;) {
            int32_t c = std::min(re - c0, sn_max);
            if (c >= sn_min) {
                for (int32_t t = c0; t < c0 + c; t++) nd.of_row[t] = nd.count;
                nd.is_sn.push_back(1);
                nd.ptr.push_back(c0 + c);
                nd.count++;
            } else {
                for (int32_t t = c0; t < c0 + c; t++) {
                    nd.of_row[t] = nd.count;
                    nd.is_sn.push_back(0);
                    nd.ptr.push_back(t + 1);
                    nd.count++;
                }
            }
            c0 += c;
        }
    }
    // padded work: every source row of a supernode source, and the own
    // supernode's earlier rows, cost 1 + 2 u_k each
    std::vector<uint64_t> rowcost(n), pre(n + 1, 0);
    for (int32_t k = 0; k < n; k++) { rowcost[k] = 1 + 2 * (uint64_t)s.ucount[k]; pre[k + 1] = pre[k] + rowcost[k]; }
    uint64_t fp = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t v = nd.of_row[i];
        for (int64_t t = s.lp[i]; t < s.lp[i + 1]; t++) {
            int32_t lo = s.lint[2 * t], hi = s.lint[2 * t + 1];
            for (int32_t u = nd.of_row[lo]; u <= nd.of_row[hi]; u++) {
                if (u == v) continue;
                if (nd.is_sn[u]) fp += pre[nd.ptr[u + 1]] - pre[nd.ptr[u]];
                else {
                    int32_t k = nd.ptr[u];
                    if (k >= lo && k <= hi) fp += rowcost[k];
                }
            }
        }
        if (nd.is_sn[v]) fp += pre[i] - pre[nd.ptr[v]];
    }
    nd.flops_padded = fp;
}

void make_levels(const Symbolic& s, Nodes& nd)
{
    const int32_t nn = nd.count;
    for (int t = 0; t < 4; t++) nd.level[t].assign(nn, 0);
    // factor / forward solve: v waits for the nodes covering L(i,:), i in v
    std::vector<int32_t>& l0 = nd.level[0];
    std::vector<int32_t>& l3 = nd.level[3];
    for (int32_t v = 0; v < nn; v++)
        for (int32_t i = nd.ptr[v]; i < nd.ptr[v + 1]; i++)
            for (int64_t t = s.lp[i]; t < s.lp[i + 1]; t++)
                for (int32_t u = nd.of_row[s.lint[2 * t]]; u <= nd.of_row[s.lint[2 * t + 1]]; u++)
                    if (u != v && l0[u] + 1 > l0[v]) l0[v] = l0[u] + 1;
    for (int32_t v = nn - 1; v >= 0; v--)
        for (int32_t i = nd.ptr[v]; i < nd.ptr[v + 1]; i++)
            for (int64_t t = s.lp[i]; t < s.lp[i + 1]; t++)
                for (int32_t u = nd.of_row[s.lint[2 * t]]; u <= nd.of_row[s.lint[2 * t + 1]]; u++)
                    if (u != v && l3[v] + 1 > l3[u]) l3[u] = l3[v] + 1;
    // backward solve: v waits for the nodes owning the columns past its block
    std::vector<int32_t>& l1 = nd.level[1];
    std::vector<int32_t>& l2 = nd.level[2];
    for (int32_t v = nn - 1; v >= 0; v--) {
        const int32_t* up; int64_t ul;
        row_upper(s, nd.ptr[v + 1] - 1, up, ul);
        for (int64_t t = 0; t < ul; t++) {
            int32_t u = nd.of_row[up[t]];
            if (u != v && l1[u] + 1 > l1[v]) l1[v] = l1[u] + 1;
        }
    }
    for (int32_t v = 0; v < nn; v++) {
        const int32_t* up; int64_t ul;
        row_upper(s, nd.ptr[v + 1] - 1, up, ul);
        for (int64_t t = 0; t < ul; t++) {
            int32_t u = nd.of_row[up[t]];
            if (u != v && l2[v] + 1 > l2[u]) l2[u] = l2[v] + 1;
        }
    }
    for (int t = 0; t < 4; t++) {
        int32_t mx = -1;
        for (int32_t v = 0; v < nn; v++) mx = std::max(mx, nd.level[t][v]);
        nd.nlevels[t] = mx + 1;
    }
}

int32_t choose_tail(const Symbolic& s, const Nodes& nd, double density, int32_t min_rows, int32_t max_rows)
{
    const int32_t n = s.n;
    if (density <= 0.0 || n == 0) return nd.count;
    // entries of L and U with min(row, col) = t
    std::vector<int64_t> diff(n + 1, 0);
    for (int64_t t = 0; t < s.lp[n]; t++) { diff[s.lint[2 * t]]++; diff[s.lint[2 * t + 1] + 1]--; }
    std::vector<double> cnt(n);
    int64_t acc = 0;
    for (int32_t k = 0; k < n; k++) { acc += diff[k]; cnt[k] = (double)acc + 1.0 + (double)s.ucount[k]; }
    double suf = 0.0;
    int32_t best = n;
    for (int32_t t = n - 1; t >= 0; t--) {
        suf += cnt[t];
        double m = (double)(n - t);
        if (n - t > max_rows) break;
        if (suf >= density * m * m && n - t >= min_rows) best = t;
    }
    if (best >= n) return nd.count;
    return nd.of_row[best];
}

void tail_masks(const Symbolic& s, const Nodes& nd, const Layout& L, TailMasks& M)
{
    const int32_t mT = L.mT, t0 = L.t0, np = (int32_t)L.panels.size();
    M = TailMasks();
    if (mT <= 0 || np == 0) return;
    const int32_t wd = (np + 63) / 64;
    M.words = wd;
    M.lbits.assign((size_t)mT * wd, 0);
    M.ubits.assign((size_t)mT * wd, 0);
    // panels whose pivot window holds tail-local column c: [pf[c], pl[c]]
    // (one panel, or every chunk of a node cut into chunks)
    std::vector<int32_t> pf(mT, np), pl(mT, -1), prow(mT, 0);
    for (int32_t j = 0; j < np; j++) {
        const Layout::Panel& P = L.panels[j];
        for (int32_t c = P.c0; c < P.c1; c++) { pf[c] = std::min(pf[c], j); pl[c] = std::max(pl[c], j); }
        for (int32_t a = P.p0; a < P.p1; a++) prow[a] = j;
    }
    auto set_range = [&](uint64_t* w, int32_t j0, int32_t j1) {      // bits j0..j1 inclusive
        for (int32_t j = j0; j <= j1;) {
            if ((j & 63) == 0 && j + 63 <= j1) { w[j >> 6] = ~0ull; j += 64; }
            else { w[j >> 6] |= 1ull << (j & 63); j++; }
        }
    };
    for (int32_t a = 0; a < mT; a++) {
        const int32_t i = t0 + a;
        const int32_t v = nd.of_row[i];
        const int32_t b0 = nd.ptr[v] - t0, b1 = nd.ptr[v + 1] - t0;
        uint64_t* lw = M.lbits.data() + (size_t)a * wd;
        // L entries in the tail (intervals of strictly-lower columns), widened
        // to whole windows; the row's own node counts whole
        for (int64_t t = s.lp[i]; t < s.lp[i + 1]; t++) {
            int32_t lo = std::max(s.lint[2 * t], t0), hi = s.lint[2 * t + 1];
            if (hi < lo) continue;
            set_range(lw, pf[lo - t0], pl[hi - t0]);
        }
        set_range(lw, pf[b0], pl[b1 - 1]);
        // U entries: the whole block and the strict upper structure
        const int32_t j = prow[a];
        const uint64_t bit = 1ull << (j & 63);
        for (int32_t c = b0; c < b1; c++) M.ubits[(size_t)c * wd + (j >> 6)] |= bit;
        const int32_t* up; int64_t ul;
        row_upper(s, i, up, ul);
        for (int64_t t = 0; t < ul; t++) M.ubits[(size_t)(up[t] - t0) * wd + (j >> 6)] |= bit;
    }
}

bool build_layout(const Csr& b, const Symbolic& s, const Nodes& nd, int32_t tail_node0, int32_t panel_rows,
                  Layout& L, const std::vector<int64_t>& bsrc, std::string& err)
{
    const int32_t n = s.n, nn = nd.count;
    L = Layout();
    L.n = n; L.nnodes = nn;
    L.tail_node0 = tail_node0;
    L.t0 = tail_node0 < nn ? nd.ptr[tail_node0] : n;
    L.mT = n - L.t0;
    const int32_t t0 = L.t0;
    L.r0.resize(nn); L.m.resize(nn); L.lw.resize(nn); L.W.resize(nn); L.lext.resize(nn);
    L.voff.resize(nn + 1); L.coff.resize(nn + 1);
    L.eptr.assign(nn + 1, 0);
    std::vector<int32_t> stamp(nn, -1), srcs;
    std::vector<int32_t> colstamp(n, -1), colpos(n, 0);
    std::vector<int32_t> flev(nn, 0);
    int64_t voff = 0;
    for (int32_t v = 0; v < nn; v++) {
        const bool tail = v >= tail_node0;
        int32_t v0 = nd.ptr[v], v1 = nd.ptr[v + 1], m = v1 - v0;
        // source nodes: union over the node's rows of the nodes covering L(i,:)
        // (for a tail node only those before the tail: the rest is dense)
        srcs.clear();
        for (int32_t i = v0; i < v1; i++)
            for (int64_t t = s.lp[i]; t < s.lp[i + 1]; t++) {
                int32_t lo = s.lint[2 * t], hi = s.lint[2 * t + 1];
                for (int32_t u = nd.of_row[lo]; u <= nd.of_row[hi]; u++) {
                    if (u == v || stamp[u] == v || (tail && u >= tail_node0)) continue;
                    stamp[u] = v;
                    srcs.push_back(u);
                }
            }
        std::sort(srcs.begin(), srcs.end());
        // column list: source rows | block | columns past the block; a tail node
        // lists its outside sources, then every column of the tail
        L.coff[v] = (int64_t)L.cols.size();
        for (int32_t u : srcs)
            for (int32_t k = nd.ptr[u]; k < nd.ptr[u + 1]; k++) L.cols.push_back(k);
        int32_t lext = (int32_t)(L.cols.size() - L.coff[v]);
        int32_t lw;
        if (tail) {
            for (int32_t k = t0; k < n; k++) L.cols.push_back(k);
            lw = lext + (v0 - t0);
        } else {
            lw = lext;
            for (int32_t k = v0; k < v1; k++) L.cols.push_back(k);
            const int32_t* up; int64_t ul;
            row_upper(s, v1 - 1, up, ul);
            for (int64_t t = 0; t < ul; t++) L.cols.push_back(up[t]);
        }
        int32_t W = (int32_t)(L.cols.size() - L.coff[v]);
        L.r0[v] = v0; L.m[v] = m; L.lw[v] = lw; L.W[v] = W; L.lext[v] = lext;
        L.voff[v] = voff;
        voff += (int64_t)m * W;
        for (int32_t t = 0; t < W; t++) { int32_t c = L.cols[L.coff[v] + t]; colstamp[c] = v; colpos[c] = t; }
        // edges with relative maps of the source's T into this node
        int32_t lpos = 0;
        for (int32_t u : srcs) {
            L.esrc.push_back(u);
            L.elpos.push_back(lpos);
            lpos += nd.ptr[u + 1] - nd.ptr[u];
            L.eroff.push_back((int64_t)L.rel.size());
            const int32_t* uu; int64_t uul;
            row_upper(s, nd.ptr[u + 1] - 1, uu, uul);
            int32_t mu = nd.ptr[u + 1] - nd.ptr[u];
            for (int64_t t = 0; t < uul; t++) {
                int32_t c = uu[t];
                if (colstamp[c] != v) { err = "layout: source column outside target structure"; return false; }
                L.rel.push_back(colpos[c]);
            }
            L.flops_kernel += (uint64_t)m * mu * (mu + 2 * (uint64_t)uul);
            flev[v] = std::max(flev[v], flev[u] + 1);
        }
        L.eptr[v + 1] = (int64_t)L.esrc.size();
        if (nd.is_sn[v] && !tail) L.flops_kernel += (uint64_t)m * m * (uint64_t)(2 * (W - lw) - m);
        // value map for B's entries of these rows
        if (L.amap.empty()) L.amap.assign(bsrc.size(), -1);
        for (int32_t i = v0; i < v1; i++)
            for (int64_t q = b.rp[i]; q < b.rp[i + 1]; q++) {
                int32_t c = b.ci[q];
                if (colstamp[c] != v) { err = "layout: entry of B outside the structure"; return false; }
                L.amap[bsrc[q]] = L.voff[v] + (int64_t)(i - v0) * W + colpos[c];
            }
    }
    L.voff[nn] = voff;
    L.coff[nn] = (int64_t)L.cols.size();
    L.nvals = voff;
    if (L.amap.empty()) L.amap.assign(bsrc.size(), -1);
    for (int64_t p = 0; p < (int64_t)L.amap.size(); p++)
        if (L.amap[p] < 0 || L.amap[p] >= L.nvals) { err = "layout: value map entry out of range"; return false; }
    for (int32_t v = 0; v < nn; v++)
        for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
            int32_t s2 = L.esrc[e];
            int32_t ws2 = L.W[s2] - L.lw[s2] - L.m[s2];
            if (L.elpos[e] + L.m[s2] > L.lext[v]) { err = "layout: source block outside the L region"; return false; }
            for (int32_t t = 0; t < ws2; t++)
                if (L.rel[L.eroff[e] + t] < 0 || L.rel[L.eroff[e] + t] >= L.W[v]) { err = "layout: relative index out of range"; return false; }
        }
    // ---- dense tail tables
    const int32_t mT = L.mT;
    if (mT > 0) {
        L.trow.resize(mT); L.tlo.resize(mT); L.thi.resize(mT);
        for (int32_t v = tail_node0; v < nn; v++)
            for (int32_t a = 0; a < L.m[v]; a++) {
                int32_t r = L.r0[v] + a - t0;
                L.trow[r] = L.voff[v] + (int64_t)a * L.W[v] + L.lext[v];
                L.tlo[r] = L.r0[v] - t0;
                L.thi[r] = L.r0[v] + L.m[v] - t0;
            }
        // panels: whole nodes up to panel_rows rows; a larger node is cut into
        // chunks that share its block as pivot window.  The factorisation cuts
        // such nodes into chunks of kWideChunk rows: the panel kernel of a wide
        // window runs on one workgroup and its traffic grows with the chunk
        // height, while the trailing update runs chip-wide.  The solves keep
        // panel_rows-row chunks.
        const int32_t NB = std::max(panel_rows, 1);
        auto build = [&](std::vector<Layout::Panel>& out, int32_t chunk) {
            int32_t cp0 = -1, cp1 = -1;
            auto flush = [&]() { if (cp0 >= 0) out.push_back({cp0, cp1, cp0, cp1, cp1}); cp0 = cp1 = -1; };
            for (int32_t v = tail_node0; v < nn; v++) {
                int32_t a0 = L.r0[v] - t0, m = L.m[v];
                if (m > NB) {
                    flush();
                    for (int32_t k = 0; k < m; k += chunk)
                        out.push_back({a0 + k, std::min(a0 + k + chunk, a0 + m), a0, a0 + m, a0});
                } else {
                    if (cp0 >= 0 && cp1 - cp0 + m > NB) flush();
                    if (cp0 < 0) cp0 = a0;
                    cp1 = a0 + m;
                }
            }
            flush();
        };
        build(L.panels, std::min(NB, kWideChunk));
        build(L.spanels, NB);
        L.flops_kernel += (uint64_t)(2.0 * (double)mT * mT * mT / 3.0);
    }
    // ---- execution level lists
    std::vector<int32_t> lv[5];
    for (int g = 0; g < 5; g++) lv[g].assign(nn, -1);
    for (int32_t v = 0; v < nn; v++) lv[0][v] = flev[v];
    for (int32_t v = 0; v < tail_node0; v++) lv[4][v] = flev[v];
    // backward solve: the tail is solved first, so only nodes before it order the rest
    for (int32_t v = tail_node0 - 1; v >= 0; v--) {
        int32_t l = 0;
        const int32_t* tc = L.cols.data() + L.coff[v] + L.lw[v] + L.m[v];
        for (int32_t t = 0; t < L.W[v] - L.lw[v] - L.m[v]; t++) {
            int32_t u = nd.of_row[tc[t]];
            if (u < tail_node0) l = std::max(l, lv[1][u] + 1);
        }
        lv[1][v] = l;
    }
    for (int32_t v = 0; v < tail_node0; v++) lv[2][v] = std::max(lv[2][v], 0);
    for (int32_t v = 0; v < tail_node0; v++) {
        const int32_t* tc = L.cols.data() + L.coff[v] + L.lw[v] + L.m[v];
        for (int32_t t = 0; t < L.W[v] - L.lw[v] - L.m[v]; t++) {
            int32_t u = nd.of_row[tc[t]];
            if (u < tail_node0) lv[2][u] = std::max(lv[2][u], lv[2][v] + 1);
        }
    }
    for (int32_t v = 0; v < tail_node0; v++) lv[3][v] = std::max(lv[3][v], 0);
    for (int32_t v = tail_node0 - 1; v >= 0; v--)
        for (int64_t e = L.eptr[v]; e < L.eptr[v + 1]; e++) {
            int32_t u = L.esrc[e];
            lv[3][u] = std::max(lv[3][u], lv[3][v] + 1);
        }
    for (int g = 0; g < 5; g++) {
        int32_t nl = 0;
        for (int32_t v = 0; v < nn; v++) nl = std::max(nl, lv[g][v] + 1);
        L.xlev_ptr[g].assign(nl + 1, 0);
        for (int32_t v = 0; v < nn; v++) if (lv[g][v] >= 0) L.xlev_ptr[g][lv[g][v] + 1]++;
        for (int32_t l = 0; l < nl; l++) L.xlev_ptr[g][l + 1] += L.xlev_ptr[g][l];
        L.xlev_nodes[g].resize(L.xlev_ptr[g][nl]);
        std::vector<int32_t> fill(L.xlev_ptr[g].begin(), L.xlev_ptr[g].end() - 1);
        for (int32_t v = 0; v < nn; v++) if (lv[g][v] >= 0) L.xlev_nodes[g][fill[lv[g][v]]++] = v;
    }
    return true;
}

}  // namespace hylu
