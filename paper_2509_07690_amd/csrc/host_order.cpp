// Static pivoting / scaling and fill-reducing orderings (HYLU Sec. 2.1).
//
// * mc64_match_scale: maximum-product bipartite matching with the dual
//   variables that give the scaling (Duff & Koster's weighted matching): the
//   cost of entry (i,j) is c_ij = log(max_k |a_kj|) - log|a_ij| >= 0, a
//   minimum-cost perfect matching is found by successive shortest augmenting
//   paths (Dijkstra on reduced costs c_ij - u_i - v_j >= 0), and
//   dr_i = exp(u_i), dc_j = exp(v_j) / max_k |a_kj| make the matched entries
//   +-1 and all others at most 1 in magnitude.
// * amd_order: approximate minimum degree (Amestoy, Davis & Duff) on the
//   quotient graph: elements absorb the elements they cover, degrees are the
//   approximate external degrees, indistinguishable variables are merged into
//   supervariables found by hashing, and variables whose only neighbour is the
//   new element are eliminated with it.
// * nd_order: nested dissection by recursive vertex-separator bisection, the
//   parts below a size limit ordered by AMD.  Two separator methods: the
//   middle level of a breadth-first level structure from a pseudo-peripheral
//   node (thinned to the nodes next to the upper side), or a multilevel
//   bisection:
//   the graph is coarsened by heavy-edge matching, the coarsest graph is split
//   by greedy graph growing from several seeds, the split is refined by
//   Fiduccia-Mattheyses passes on every level while it is projected back, and
//   the vertex separator is the smaller boundary of the final edge cut.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <queue>
#include <random>
#include <vector>

#include "analysis.hpp"

namespace hylu {

// =========================================================================
// maximum-product matching + scaling
// =========================================================================

bool mc64_match_scale(const Csr& a, std::vector<int32_t>& row_of_col,
                      std::vector<double>& dr, std::vector<double>& dc)
{
    const int32_t n = a.n;
    const double INF = std::numeric_limits<double>::infinity();
    // column-major copy of the nonzero entries with costs
    std::vector<int64_t> cp(n + 1, 0);
    for (int64_t p = 0; p < a.nnz(); p++)
        if (a.v[p] != 0.0) cp[a.ci[p] + 1]++;
    for (int32_t j = 0; j < n; j++) cp[j + 1] += cp[j];
    std::vector<int32_t> ri(cp[n]);
    std::vector<double> cc(cp[n]);
    std::vector<double> cmax(n, 0.0);
    {
        std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
        for (int32_t i = 0; i < n; i++)
            for (int64_t p = a.rp[i]; p < a.rp[i + 1]; p++) {
                double av = std::fabs(a.v[p]);
                if (av == 0.0) continue;
                int32_t j = a.ci[p];
                ri[fill[j]] = i;
                cc[fill[j]] = av;
                fill[j]++;
                cmax[j] = std::max(cmax[j], av);
            }
    }
    for (int32_t j = 0; j < n; j++) {
        if (cmax[j] == 0.0) return false;                 // empty column
        double lm = std::log(cmax[j]);
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) cc[p] = lm - std::log(cc[p]);
    }
    // initial duals: u_i = min_j c_ij, v_j = min_i (c_ij - u_i)
    std::vector<double> u(n, INF), v(n, INF);
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) u[ri[p]] = std::min(u[ri[p]], cc[p]);
    for (int32_t i = 0; i < n; i++) if (u[i] == INF) return false;   // empty row
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) v[j] = std::min(v[j], cc[p] - u[ri[p]]);
    auto rc = [&](int64_t p, int32_t j) { double r = cc[p] - u[ri[p]] - v[j]; return r > 0.0 ? r : 0.0; };
    // greedy matching on tight edges
    std::vector<int32_t> mrow(n, -1), mcol(n, -1);       // mrow[i] = column, mcol[j] = row
    for (int32_t j = 0; j < n; j++)
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) {
            int32_t i = ri[p];
            if (mrow[i] < 0 && rc(p, j) == 0.0) { mrow[i] = j; mcol[j] = i; break; }
        }
    // shortest augmenting paths from every free column
    std::vector<double> d(n, INF);
    std::vector<int32_t> pred(n, -1), done(n, -1);
    std::vector<int32_t> touched, popped;
    typedef std::pair<double, int32_t> item;
    for (int32_t j0 = 0; j0 < n; j0++) {
        if (mcol[j0] >= 0) continue;
        std::priority_queue<item, std::vector<item>, std::greater<item>> pq;
        touched.clear(); popped.clear();
        for (int64_t p = cp[j0]; p < cp[j0 + 1]; p++) {
            int32_t i = ri[p];
            double nd = rc(p, j0);
            if (nd < d[i]) { if (d[i] == INF) touched.push_back(i); d[i] = nd; pred[i] = j0; pq.push({nd, i}); }
        }
        int32_t found = -1;
        double D = 0.0;
        while (!pq.empty()) {
            item it = pq.top(); pq.pop();
            int32_t i = it.second;
            if (done[i] == j0 || it.first > d[i]) continue;
            done[i] = j0;
            popped.push_back(i);
            if (mrow[i] < 0) { found = i; D = it.first; break; }
            int32_t j = mrow[i];
            double dj = it.first;
            for (int64_t p = cp[j]; p < cp[j + 1]; p++) {
                int32_t k = ri[p];
                if (done[k] == j0) continue;
                double nd = dj + rc(p, j);
                if (nd < d[k]) { if (d[k] == INF) touched.push_back(k); d[k] = nd; pred[k] = j; pq.push({nd, k}); }
            }
        }
        if (found < 0) return false;                        // structurally singular
        // dual update keeps reduced costs >= 0 and the new matched edges tight
        for (int32_t i : popped) {
            if (i == found || d[i] >= D) continue;
            u[i] += d[i] - D;
            v[mrow[i]] += D - d[i];
        }
        v[j0] += D;
        // augment
        int32_t i = found;
        for (;;) {
            int32_t j = pred[i];
            int32_t iprev = mcol[j];
            mcol[j] = i; mrow[i] = j;
            if (j == j0) break;
            i = iprev;
        }
        for (int32_t t : touched) d[t] = INF;
    }
    row_of_col.assign(mcol.begin(), mcol.end());
    dr.resize(n); dc.resize(n);
    for (int32_t i = 0; i < n; i++) dr[i] = std::exp(u[i]);
    for (int32_t j = 0; j < n; j++) dc[j] = std::exp(v[j]) / cmax[j];
    return true;
}

// =========================================================================
// approximate minimum degree
// =========================================================================

namespace {

enum : uint8_t { VAR = 0, ELEM = 1, ABSORBED = 2, MERGED = 3, DENSE = 4 };

struct Amd {
    int32_t n;
    std::vector<int32_t> iw;
    int64_t pfree = 0;
    std::vector<int64_t> pe;
    std::vector<int32_t> len, elen, nv;
    std::vector<int64_t> deg, esize, w, mark;
    std::vector<uint8_t> kind;
    std::vector<int32_t> head, dnext, dprev;
    std::vector<int32_t> mfirst, mlast, mnext;     // member chains for the output order

    void dl_insert(int32_t i, int64_t d) {
        dprev[i] = -1; dnext[i] = head[d];
        if (head[d] >= 0) dprev[head[d]] = i;
        head[d] = i;
    }
    void dl_remove(int32_t i) {
        int64_t d = deg[i];
        if (dprev[i] >= 0) dnext[dprev[i]] = dnext[i]; else head[d] = dnext[i];
        if (dnext[i] >= 0) dprev[dnext[i]] = dprev[i];
        dprev[i] = dnext[i] = -1;
    }
    void members_append(int32_t to, int32_t from) {      // from and its members join to's list
        int32_t f = from, l = mlast[from] >= 0 ? mlast[from] : from;
        mnext[l] = -1;
        // chain: from -> members(from)
        if (mfirst[from] >= 0) { mnext[from] = mfirst[from]; } else { mnext[from] = -1; l = from; }
        if (mfirst[to] < 0) mfirst[to] = f; else mnext[mlast[to]] = f;
        mlast[to] = l;
        mfirst[from] = mlast[from] = -1;
    }
    // make room for `need` more entries at the tail, compacting live lists if needed
    void reserve(int64_t need) {
        if (pfree + need <= (int64_t)iw.size()) return;
        std::vector<int32_t> live;
        for (int32_t i = 0; i < n; i++)
            if ((kind[i] == VAR || kind[i] == ELEM) && pe[i] >= 0) live.push_back(i);
        int64_t total = 0;
        for (int32_t i : live) total += len[i];
        std::vector<int32_t> nw((size_t)std::max<int64_t>(2 * (total + need) + n, 1024));
        int64_t q = 0;
        for (int32_t i : live) {
            std::copy(iw.begin() + pe[i], iw.begin() + pe[i] + len[i], nw.begin() + q);
            pe[i] = q; q += len[i];
        }
        iw.swap(nw);
        pfree = q;
    }
};

}  // namespace

std::vector<int32_t> amd_order(int32_t n, const std::vector<int64_t>& xadj,
                               const std::vector<int32_t>& adj, double dense_alpha)
{
    std::vector<int32_t> order;
    order.reserve(n);
    if (n == 0) return order;
    Amd A;
    A.n = n;
    A.pe.assign(n, -1); A.len.assign(n, 0); A.elen.assign(n, 0); A.nv.assign(n, 1);
    A.deg.assign(n, 0); A.esize.assign(n, 0); A.w.assign(n, 0); A.mark.assign(n, 0);
    A.kind.assign(n, VAR);
    A.head.assign(n + 1, -1); A.dnext.assign(n, -1); A.dprev.assign(n, -1);
    A.mfirst.assign(n, -1); A.mlast.assign(n, -1); A.mnext.assign(n, -1);
    // dense rows are ordered last: more than max(16, alpha sqrt(n)) entries,
    // or with alpha <= 0 more than max(16, min(10 sqrt(n), 6 x the mean
    // degree)), which also catches the hub rows of power-law patterns
    int64_t dense;
    if (dense_alpha > 0) {
        dense = std::max<int64_t>(16, (int64_t)(dense_alpha * std::sqrt((double)n)));
    } else {
        const double mean = (double)xadj[n] / n;
        dense = std::max<int64_t>(16, (int64_t)std::min(10.0 * std::sqrt((double)n), 6.0 * mean));
    }
    std::vector<int32_t> dense_nodes;
    for (int32_t i = 0; i < n; i++)
        if (xadj[i + 1] - xadj[i] > dense && n > 2 * dense) { A.kind[i] = DENSE; dense_nodes.push_back(i); }
    int64_t total = 0;
    for (int32_t i = 0; i < n; i++) if (A.kind[i] == VAR) total += xadj[i + 1] - xadj[i];
    A.iw.resize((size_t)(total + total / 5 + 2 * (int64_t)n + 1024));
    int32_t nlive = 0;
    for (int32_t i = 0; i < n; i++) {
        if (A.kind[i] != VAR) continue;
        nlive++;
        A.pe[i] = A.pfree;
        for (int64_t p = xadj[i]; p < xadj[i + 1]; p++) {
            int32_t j = adj[p];
            if (j != i && A.kind[j] != DENSE) A.iw[A.pfree++] = j;
        }
        A.len[i] = (int32_t)(A.pfree - A.pe[i]);
        A.deg[i] = A.len[i];
        A.dl_insert(i, A.deg[i]);
    }
    int64_t nel = 0, tag = 1, wflg = 2;
    int64_t mindeg = 0;
    std::vector<int32_t> Lp, ekeep, vkeep, mass;
    std::vector<int64_t> dpart(n, 0);
    std::vector<uint64_t> hsh(n, 0);
    std::vector<std::pair<uint64_t, int32_t>> buckets;
    std::vector<int64_t> cmpmark(n, 0);
    int64_t cmptag = 0;
    while (nel < nlive) {
        while (mindeg <= n && A.head[mindeg] < 0) mindeg++;
        int32_t p = A.head[mindeg];
        A.dl_remove(p);
        // ---- new element L_p = (A_p u L_e for e in E_p) \ {p}
        tag++;
        A.mark[p] = tag;
        Lp.clear();
        for (int32_t t = 0; t < A.len[p]; t++) {
            int32_t x = A.iw[A.pe[p] + t];
            if (t < A.elen[p]) {
                if (A.kind[x] != ELEM) continue;
                for (int32_t s = 0; s < A.len[x]; s++) {
                    int32_t j = A.iw[A.pe[x] + s];
                    if (A.kind[j] == VAR && A.mark[j] != tag) { A.mark[j] = tag; Lp.push_back(j); A.dl_remove(j); }
                }
                A.kind[x] = ABSORBED;
            } else if (A.kind[x] == VAR && A.mark[x] != tag) {
                A.mark[x] = tag; Lp.push_back(x); A.dl_remove(x);
            }
        }
        A.kind[p] = ELEM;
        nel += A.nv[p];
        A.reserve((int64_t)Lp.size());
        A.pe[p] = A.pfree;
        int64_t es = 0;
        for (int32_t j : Lp) { A.iw[A.pfree++] = j; es += A.nv[j]; }
        A.len[p] = (int32_t)Lp.size();
        A.elen[p] = 0;
        A.esize[p] = es;
        // ---- |L_e \ L_p| for elements next to L_p
        for (int32_t i : Lp)
            for (int32_t t = 0; t < A.elen[i]; t++) {
                int32_t e = A.iw[A.pe[i] + t];
                if (A.kind[e] != ELEM || e == p) continue;
                if (A.w[e] < wflg) A.w[e] = A.esize[e] + wflg;
                A.w[e] -= A.nv[i];
            }
        // ---- clean adjacency, partial degrees, hashes, mass elimination
        mass.clear();
        buckets.clear();
        for (int32_t i : Lp) {
            ekeep.clear(); vkeep.clear();
            int64_t dp = 0;
            uint64_t h = 0;
            int64_t base = A.pe[i];
            for (int32_t t = 0; t < A.elen[i]; t++) {
                int32_t e = A.iw[base + t];
                if (A.kind[e] != ELEM || e == p) continue;
                int64_t we = A.w[e] - wflg;
                if (we <= 0) { A.kind[e] = ABSORBED; continue; }   // L_e inside L_p
                dp += we; ekeep.push_back(e); h += (uint64_t)e;
            }
            for (int32_t t = A.elen[i]; t < A.len[i]; t++) {
                int32_t j = A.iw[base + t];
                if (A.kind[j] != VAR || A.mark[j] == tag) continue;
                dp += A.nv[j]; vkeep.push_back(j); h += (uint64_t)j;
            }
            int32_t nl = 1 + (int32_t)ekeep.size() + (int32_t)vkeep.size();
            if (nl > A.len[i]) {                                  // no room in place: move to the tail
                A.reserve(nl);
                base = A.pe[i] = A.pfree;
                A.pfree += nl;
            }
            int64_t q = base;
            A.iw[q++] = p;
            for (int32_t e : ekeep) A.iw[q++] = e;
            for (int32_t j : vkeep) A.iw[q++] = j;
            A.len[i] = nl;
            A.elen[i] = 1 + (int32_t)ekeep.size();
            if (ekeep.empty() && vkeep.empty()) {
                mass.push_back(i);
            } else {
                dpart[i] = dp;
                hsh[i] = h;
                buckets.push_back({h, i});
            }
        }
        for (int32_t i : mass) {
            A.kind[i] = MERGED;
            A.esize[p] -= A.nv[i];
            nel += A.nv[i];
            A.nv[p] += A.nv[i];
            A.nv[i] = 0;
            A.members_append(p, i);
        }
        // ---- supervariables: same element and variable lists
        std::sort(buckets.begin(), buckets.end());
        for (size_t s = 0; s < buckets.size();) {
            size_t e = s;
            while (e < buckets.size() && buckets[e].first == buckets[s].first) e++;
            for (size_t x = s; x < e; x++) {
                int32_t i = buckets[x].second;
                if (A.kind[i] != VAR) continue;
                cmptag++;
                for (int32_t t = 0; t < A.len[i]; t++) cmpmark[A.iw[A.pe[i] + t]] = cmptag;
                for (size_t y = x + 1; y < e; y++) {
                    int32_t j = buckets[y].second;
                    if (A.kind[j] != VAR || A.len[j] != A.len[i] || A.elen[j] != A.elen[i]) continue;
                    bool same = true;
                    for (int32_t t = 0; t < A.len[j] && same; t++) same = cmpmark[A.iw[A.pe[j] + t]] == cmptag;
                    if (!same) continue;
                    A.nv[i] += A.nv[j];
                    A.nv[j] = 0;
                    A.kind[j] = MERGED;
                    A.members_append(i, j);
                }
            }
            s = e;
        }
        // ---- approximate external degrees
        int64_t degme = A.esize[p];
        for (int32_t i : Lp) {
            if (A.kind[i] != VAR) continue;
            int64_t lp_ext = degme - A.nv[i];
            int64_t d = std::min(dpart[i] + lp_ext, A.deg[i] + lp_ext);
            d = std::min<int64_t>(d, (int64_t)nlive - nel - A.nv[i]);
            if (d < 0) d = 0;
            A.deg[i] = d;
            A.dl_insert(i, d);
            if (d < mindeg) mindeg = d;
        }
        // ---- L_p keeps principal variables only
        {
            int64_t q = A.pe[p];
            for (int32_t t = 0; t < A.len[p]; t++) {
                int32_t j = A.iw[A.pe[p] + t];
                if (A.kind[j] == VAR) A.iw[q++] = j;
            }
            A.len[p] = (int32_t)(q - A.pe[p]);
        }
        order.push_back(p);
        for (int32_t m = A.mfirst[p]; m >= 0; m = A.mnext[m]) order.push_back(m);
        wflg += (int64_t)nlive + 2;
    }
    for (int32_t i : dense_nodes) order.push_back(i);
    return order;
}

// =========================================================================
// nested dissection
// =========================================================================

namespace {

// BFS level structure restricted to nodes with part[x] == id.
static int32_t bfs_levels(const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                          const std::vector<int32_t>& nodes, const std::vector<int32_t>& part, int32_t id,
                          int32_t root, std::vector<int32_t>& level, std::vector<int32_t>& queue)
{
    for (int32_t x : nodes) level[x] = -1;
    queue.clear();
    queue.push_back(root);
    level[root] = 0;
    int32_t maxl = 0;
    for (size_t h = 0; h < queue.size(); h++) {
        int32_t x = queue[h];
        for (int64_t p = xadj[x]; p < xadj[x + 1]; p++) {
            int32_t y = adj[p];
            if (part[y] != id || level[y] >= 0) continue;
            level[y] = level[x] + 1;
            maxl = std::max(maxl, level[y]);
            queue.push_back(y);
        }
    }
    return maxl;
}

// ---- multilevel edge bisection ---------------------------------------------

// a graph with vertex and edge weights (local numbering, no self loops)
struct WGraph {
    int32_t n = 0;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj, ew, vw;
    int64_t total() const { int64_t t = 0; for (int32_t w : vw) t += w; return t; }
};

// heavy-edge matching: every vertex (in a random order) pairs with its
// unmatched neighbour of largest edge weight; cmap[x] is x's coarse vertex
static void coarsen(const WGraph& g, std::mt19937& rng, std::vector<int32_t>& cmap, WGraph& c)
{
    const int32_t n = g.n;
    std::vector<int32_t> order(n), match(n, -1);
    std::iota(order.begin(), order.end(), 0);
    std::shuffle(order.begin(), order.end(), rng);
    for (int32_t x : order) {
        if (match[x] >= 0) continue;
        int32_t best = -1, bw = -1;
        for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) {
            const int32_t y = g.adj[p];
            if (match[y] < 0 && g.ew[p] > bw) { bw = g.ew[p]; best = y; }
        }
        if (best >= 0) { match[x] = best; match[best] = x; } else match[x] = x;
    }
    cmap.assign(n, -1);
    int32_t nc = 0;
    for (int32_t x : order)
        if (cmap[x] < 0) { cmap[x] = nc; cmap[match[x]] = nc; nc++; }
    c.n = nc;
    c.vw.assign(nc, 0);
    std::vector<std::vector<int32_t>> members(nc);
    for (int32_t x = 0; x < n; x++) { c.vw[cmap[x]] += g.vw[x]; members[cmap[x]].push_back(x); }
    c.xadj.assign(nc + 1, 0);
    c.adj.clear();
    c.ew.clear();
    std::vector<int32_t> slot(nc, -1);
    for (int32_t u = 0; u < nc; u++) {
        const size_t base = c.adj.size();
        for (int32_t x : members[u])
            for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) {
                const int32_t v = cmap[g.adj[p]];
                if (v == u) continue;
                if (slot[v] < 0) { slot[v] = (int32_t)c.adj.size(); c.adj.push_back(v); c.ew.push_back(0); }
                c.ew[slot[v]] += g.ew[p];
            }
        for (size_t q = base; q < c.adj.size(); q++) slot[c.adj[q]] = -1;
        c.xadj[u + 1] = (int64_t)c.adj.size();
    }
}

static int64_t cut_weight(const WGraph& g, const std::vector<uint8_t>& side)
{
    int64_t cut = 0;
    for (int32_t x = 0; x < g.n; x++)
        for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++)
            if (side[x] != side[g.adj[p]]) cut += g.ew[p];
    return cut / 2;
}

// Fiduccia-Mattheyses passes: move the vertex of largest gain (cut weight
// removed) to the other side while both sides stay within [lo, hi] weight,
// each vertex at most once per pass, and keep the best prefix of moves
static void fm_refine(const WGraph& g, std::vector<uint8_t>& side, int64_t lo, int64_t hi, int passes)
{
    const int32_t n = g.n;
    std::vector<int64_t> gain(n);
    std::vector<uint8_t> moved(n);
    int64_t w[2] = {0, 0};
    for (int32_t x = 0; x < n; x++) w[side[x]] += g.vw[x];
    for (int pass = 0; pass < passes; pass++) {
        for (int32_t x = 0; x < n; x++) {
            int64_t gx = 0;
            for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) gx += side[g.adj[p]] != side[x] ? g.ew[p] : -g.ew[p];
            gain[x] = gx;
        }
        std::fill(moved.begin(), moved.end(), 0);
        // max-heap of (gain, vertex), lazily invalidated; boundary vertices only
        std::priority_queue<std::pair<int64_t, int32_t>> heap;
        for (int32_t x = 0; x < n; x++) {
            bool bnd = false;
            for (int64_t p = g.xadj[x]; p < g.xadj[x + 1] && !bnd; p++) bnd = side[g.adj[p]] != side[x];
            if (bnd) heap.push({gain[x], x});
        }
        std::vector<int32_t> seq;
        int64_t cur = 0, best = 0;
        size_t best_len = 0;
        int32_t since_best = 0;
        while (!heap.empty() && since_best < 200) {
            auto [gx, x] = heap.top();
            heap.pop();
            if (moved[x] || gx != gain[x]) continue;
            const int s0 = side[x], s1 = 1 - s0;
            if (w[s1] + g.vw[x] > hi || w[s0] - g.vw[x] < lo) continue;
            moved[x] = 1;
            side[x] = (uint8_t)s1;
            w[s0] -= g.vw[x];
            w[s1] += g.vw[x];
            cur += gx;
            seq.push_back(x);
            for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) {
                const int32_t y = g.adj[p];
                if (moved[y]) continue;
                gain[y] += side[y] == s1 ? -2 * g.ew[p] : 2 * g.ew[p];
                heap.push({gain[y], y});
            }
            if (cur > best) { best = cur; best_len = seq.size(); since_best = 0; } else since_best++;
        }
        // undo the moves after the best prefix
        for (size_t q = seq.size(); q-- > best_len;) {
            const int32_t x = seq[q];
            const int s1 = side[x], s0 = 1 - s1;
            side[x] = (uint8_t)s0;
            w[s1] -= g.vw[x];
            w[s0] += g.vw[x];
        }
        if (best <= 0) break;
    }
}

// greedy graph growing from `seed`: the part grows by the boundary vertex
// that adds the least cut, until it holds half of the weight
static void grow(const WGraph& g, int32_t seed, std::vector<uint8_t>& side)
{
    const int32_t n = g.n;
    side.assign(n, 1);
    const int64_t half = g.total() / 2;
    int64_t w0 = 0;
    std::vector<int64_t> conn(n, 0);          // edge weight into part 0
    std::vector<int64_t> deg(n, 0);
    for (int32_t x = 0; x < n; x++)
        for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) deg[x] += g.ew[p];
    std::priority_queue<std::pair<int64_t, int32_t>> heap;   // key: 2 conn - deg (cut removed)
    heap.push({0, seed});
    std::vector<uint8_t> in(n, 0);
    while (w0 < half) {
        int32_t x = -1;
        while (!heap.empty()) {
            auto [k, y] = heap.top();
            heap.pop();
            if (!in[y] && k == 2 * conn[y] - deg[y]) { x = y; break; }
        }
        if (x < 0) {                            // the part's component is used up: any vertex
            for (int32_t y = 0; y < n && x < 0; y++) if (!in[y]) x = y;
            if (x < 0) break;
        }
        in[x] = 1;
        side[x] = 0;
        w0 += g.vw[x];
        for (int64_t p = g.xadj[x]; p < g.xadj[x + 1]; p++) {
            const int32_t y = g.adj[p];
            if (in[y]) continue;
            conn[y] += g.ew[p];
            heap.push({2 * conn[y] - deg[y], y});
        }
    }
}

// two-way split of g minimising the cut weight with both sides within 10% of
// half the weight: coarsen to about 100 vertices, grow from eight seeds,
// refine, project back level by level with refinement
static std::vector<uint8_t> multilevel_bisect(const WGraph& g0, uint32_t seed)
{
    std::mt19937 rng(seed);
    std::vector<WGraph> gs;
    std::vector<std::vector<int32_t>> maps;
    gs.push_back(g0);
    while (gs.back().n > 100) {
        WGraph c;
        std::vector<int32_t> cmap;
        coarsen(gs.back(), rng, cmap, c);
        if (c.n > 0.9 * gs.back().n) break;        // no longer shrinking (e.g. a star)
        maps.push_back(std::move(cmap));
        gs.push_back(std::move(c));
    }
    auto bounds = [](const WGraph& g, int64_t& lo, int64_t& hi) {
        const int64_t t = g.total();
        int64_t maxv = 0;
        for (int32_t w : g.vw) maxv = std::max<int64_t>(maxv, w);
        lo = std::min<int64_t>((int64_t)(0.45 * t), t / 2 - maxv);
        hi = std::max<int64_t>((int64_t)(0.55 * t) + 1, t / 2 + maxv);
    };
    const WGraph& cg = gs.back();
    int64_t lo, hi;
    bounds(cg, lo, hi);
    std::vector<uint8_t> best;
    int64_t best_cut = INT64_MAX;
    std::uniform_int_distribution<int32_t> pick(0, std::max(cg.n - 1, 0));
    for (int t = 0; t < 8; t++) {
        std::vector<uint8_t> side;
        grow(cg, pick(rng), side);
        fm_refine(cg, side, lo, hi, 4);
        const int64_t c = cut_weight(cg, side);
        if (c < best_cut) { best_cut = c; best = side; }
    }
    for (size_t l = gs.size() - 1; l-- > 0;) {
        const WGraph& g = gs[l];
        std::vector<uint8_t> side(g.n);
        for (int32_t x = 0; x < g.n; x++) side[x] = best[maps[l][x]];
        bounds(g, lo, hi);
        fm_refine(g, side, lo, hi, 4);
        best.swap(side);
    }
    return best;
}

}  // namespace

std::vector<int32_t> nd_order(int32_t n, const std::vector<int64_t>& xadj,
                              const std::vector<int32_t>& adj, int32_t leaf_size, double dense_alpha, bool multilevel)
{
    // part[x]: id of the sub-problem node x belongs to, or -1 once numbered
    std::vector<int32_t> part(n, 0), level(n, -1), queue;
    std::vector<int32_t> local(n, -1);
    int32_t next_id = 1;
    struct Job { int32_t id; std::vector<int32_t> nodes; };
    std::vector<Job> stack;
    {
        Job j0; j0.id = 0;
        j0.nodes.resize(n);
        std::iota(j0.nodes.begin(), j0.nodes.end(), 0);
        stack.push_back(std::move(j0));
    }
    std::vector<std::vector<int32_t>> leaves;
    std::vector<std::vector<int32_t>> seps_rev;   // separators in the order they are found
    while (!stack.empty()) {
        Job job = std::move(stack.back());
        stack.pop_back();
        std::vector<int32_t>& nodes = job.nodes;
        if ((int32_t)nodes.size() <= leaf_size) { leaves.push_back(nodes); continue; }
        // connected components first
        int32_t root = nodes[0];
        int32_t maxl = bfs_levels(xadj, adj, nodes, part, job.id, root, level, queue);
        if (queue.size() < nodes.size()) {
            std::vector<int32_t> comp(queue.begin(), queue.end()), rest;
            for (int32_t x : nodes) if (level[x] < 0) rest.push_back(x);
            int32_t a = next_id++, b = next_id++;
            for (int32_t x : comp) part[x] = a;
            for (int32_t x : rest) part[x] = b;
            stack.push_back({b, rest});
            stack.push_back({a, comp});
            continue;
        }
        std::vector<int32_t> sep, lower, upper;
        if (multilevel) {
            // multilevel edge bisection of the part, then the smaller of the two
            // boundaries as the vertex separator
            const int32_t m = (int32_t)nodes.size();
            for (int32_t t = 0; t < m; t++) local[nodes[t]] = t;
            WGraph g;
            g.n = m;
            g.xadj.assign(m + 1, 0);
            g.vw.assign(m, 1);
            for (int32_t t = 0; t < m; t++) {
                const int32_t x = nodes[t];
                for (int64_t p = xadj[x]; p < xadj[x + 1]; p++) {
                    const int32_t y = adj[p];
                    if (y != x && part[y] == job.id) { g.adj.push_back(local[y]); g.ew.push_back(1); }
                }
                g.xadj[t + 1] = (int64_t)g.adj.size();
            }
            const std::vector<uint8_t> side = multilevel_bisect(g, 0x9e3779b9u ^ (uint32_t)m);
            int64_t nb[2] = {0, 0};
            std::vector<uint8_t> bnd(m, 0);
            for (int32_t t = 0; t < m; t++)
                for (int64_t p = g.xadj[t]; p < g.xadj[t + 1]; p++)
                    if (side[g.adj[p]] != side[t]) { bnd[t] = 1; nb[side[t]]++; break; }
            const int ss = nb[0] <= nb[1] ? 0 : 1;      // the separator's side
            for (int32_t t = 0; t < m; t++) {
                const int32_t x = nodes[t];
                if (side[t] == ss && bnd[t]) sep.push_back(x);
                else if (side[t] == 0) lower.push_back(x);
                else upper.push_back(x);
            }
            for (int32_t t = 0; t < m; t++) local[nodes[t]] = -1;
            if (sep.empty() || lower.empty() || upper.empty()) { leaves.push_back(nodes); continue; }
        } else {
            // pseudo-peripheral root: repeat BFS from the farthest node of the smallest degree
            for (int it = 0; it < 6; it++) {
                int32_t best = -1;
                int64_t bestdeg = INT64_MAX;
                for (int32_t x : nodes)
                    if (level[x] == maxl) {
                        int64_t dgx = xadj[x + 1] - xadj[x];
                        if (dgx < bestdeg) { bestdeg = dgx; best = x; }
                    }
                int32_t ml2 = bfs_levels(xadj, adj, nodes, part, job.id, best, level, queue);
                if (ml2 <= maxl) { if (ml2 == maxl) root = best; bfs_levels(xadj, adj, nodes, part, job.id, root, level, queue); break; }
                root = best; maxl = ml2;
            }
            if (maxl < 2) { leaves.push_back(nodes); continue; }
            // level sizes; choose the level near the middle (by count) with the fewest nodes
            std::vector<int64_t> cnt(maxl + 1, 0);
            for (int32_t x : nodes) cnt[level[x]]++;
            int64_t half = (int64_t)nodes.size() / 2, acc = 0;
            int32_t mid = 1;
            for (int32_t l = 0; l <= maxl; l++) { acc += cnt[l]; if (acc >= half) { mid = l; break; } }
            mid = std::max(1, std::min(mid, maxl - 1));
            int32_t best = mid;
            // search a window around the middle for a smaller separator with balance >= 1/3
            int64_t below = 0;
            for (int32_t l = 0; l <= maxl; l++) {
                if (l >= 1 && l <= maxl - 1) {
                    int64_t above = (int64_t)nodes.size() - below - cnt[l];
                    if (3 * std::min(below, above) >= (int64_t)nodes.size() - cnt[l] &&
                        cnt[l] < cnt[best]) best = l;
                }
                below += cnt[l];
            }
            // separator = level `best`, thinned: keep only nodes adjacent to the upper side
            for (int32_t x : nodes) {
                if (level[x] < best) lower.push_back(x);
                else if (level[x] > best) upper.push_back(x);
                else {
                    bool touches_upper = false;
                    for (int64_t p = xadj[x]; p < xadj[x + 1] && !touches_upper; p++)
                        touches_upper = part[adj[p]] == job.id && level[adj[p]] == best + 1;
                    if (touches_upper) sep.push_back(x); else lower.push_back(x);
                }
            }
        }
        for (int32_t x : sep) part[x] = -1;
        seps_rev.push_back(sep);
        int32_t a = next_id++, b = next_id++;
        for (int32_t x : lower) part[x] = a;
        for (int32_t x : upper) part[x] = b;
        if (!upper.empty()) stack.push_back({b, upper});
        if (!lower.empty()) stack.push_back({a, lower});
    }
    // number leaves first (each by AMD on its induced subgraph), then separators
    // from the last one found (deepest) to the first (the top separator is last)
    std::vector<int32_t> result;
    result.reserve(n);
    for (auto& leaf : leaves) {
        int32_t m = (int32_t)leaf.size();
        for (int32_t t = 0; t < m; t++) local[leaf[t]] = t;
        std::vector<int64_t> lx(m + 1, 0);
        std::vector<int32_t> la;
        for (int32_t t = 0; t < m; t++) {
            int32_t x = leaf[t];
            for (int64_t p = xadj[x]; p < xadj[x + 1]; p++) {
                int32_t y = adj[p];
                if (y != x && local[y] >= 0 && part[y] == part[x]) la.push_back(local[y]);
            }
            lx[t + 1] = (int64_t)la.size();
        }
        std::vector<int32_t> lo = amd_order(m, lx, la, dense_alpha);
        for (int32_t t : lo) result.push_back(leaf[t]);
        for (int32_t t = 0; t < m; t++) local[leaf[t]] = -1;
    }
    // separators are numbered from the end in the order they were found, so
    // every separator follows all nodes of the two parts it splits
    std::vector<int32_t> seps_num;
    for (size_t s = seps_rev.size(); s-- > 0;) seps_num.insert(seps_num.end(), seps_rev[s].begin(), seps_rev[s].end());
    result.insert(result.end(), seps_num.begin(), seps_num.end());
    return result;
}

}  // namespace hylu
