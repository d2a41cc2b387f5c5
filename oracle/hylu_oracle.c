/*
 * Plain, slow, single-threaded FP64 oracle for HYLU's numerical
 * factorisation and forward-backward substitution (arXiv 2509.07690).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP path is
 * checked against.  It shares no code, header, table or helper with the
 * library under paper_2509_07690_amd/; only tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * What it computes, in the paper's order:
 *   O-3  B = R A C with R, C from the static pivoting / scaling and the
 *        fill-reducing ordering (Sec. 2.1).  The permutations and scalings
 *        are heuristics' outputs and are taken as data; orc_check_matching
 *        certifies the property Sec. 2.1 states for them (unit diagonal,
 *        off-diagonals bounded by one).
 *   O-4  exact, unpivoted symbolic structure of L and U (Sec. 2.1, last
 *        step; Sec. 2.2 up-looking order): row i of the factors is the
 *        union of row i of B and, for every k < i already in the row (in
 *        ascending order, the set grows), the strict upper structure of row k.
 *   O-5  flop count F = sum_k l_k (1 + 2 u_k) (Sec. 2.1 computes it during
 *        symbolic factorisation; the formula is the standard one).
 *   O-6  supernodes: maximal runs of consecutive rows with identical U
 *        structure (Sec. 2.2 definition).
 *   O-7  task graph and levels (Sec. 2.2.1): nodes are supernodes and
 *        standalone rows, edges come from the structure of L; a node's level
 *        is one more than the deepest level among its predecessors.  Three
 *        further level sets are built the same way for the backward solve and
 *        the two transposed solves.
 *   O-8  up-looking numerical factorisation (Sec. 2.2): each row is formed
 *        from its sources in ascending order; supernode sources are used in
 *        full (the dense sub-blocks of the supernodal kernels); within a
 *        supernode the largest entry of the diagonal block is pivoted to the
 *        diagonal and standalone rows are not pivoted; small pivots are
 *        perturbed (Sec. 2.2 pivoting paragraph).
 *   O-9  forward-backward substitution (Sec. 2.3).
 *   O-10 iterative refinement after perturbation (Sec. 2.3, last paragraph).
 *   O-11 transposed solve and the gradient of a loss through x = A^{-1} b.
 *
 * Storage conventions of the results (all 0-based, in B's index space):
 *   exact L  : CSR (Lp, Li), strict lower part, sorted columns;
 *   exact U  : CSR (Up, Ui), diagonal included, sorted columns;
 *   factors  : L as CSR over the padded source list of every row (Fp, Fi, Fv),
 *              U stored in B's column order ("U_st", B = L * U_st) as CSR
 *              (Sp, Si, Sv) with sorted columns, and piv[i] = column holding
 *              row i's pivot.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_OOM -2
#define ORC_ERR_STATE -3
#define ORC_ERR_MATCH -4

typedef struct {
    int32_t n;
    /* original A */
    int64_t *arp;
    int32_t *aci;
    double *av;
    /* static pivoting + ordering as data */
    int32_t *pr, *pc;       /* new row/col -> original row/col */
    double *dr, *dc;        /* scaling by original row / col */
    /* B = R A C in new indices, sorted CSR */
    int64_t *brp;
    int32_t *bci;
    double *bv;
    int64_t *bsrc;          /* CSR position of A that produced each entry of B */
    /* exact symbolic structure */
    int64_t *Lp, *Up;
    int32_t *Li, *Ui;
    uint64_t flops, flops_padded;
    /* partition */
    int32_t nnodes;
    int32_t *node_ptr;      /* nnodes+1 row boundaries */
    int32_t *node_of;       /* row -> node */
    int32_t *is_sn;         /* node -> 1 if supernode */
    /* levels per node: 0 factor / L-solve, 1 U-solve, 2 U^T-solve, 3 L^T-solve */
    int32_t *lev[4];
    int32_t nlev[4];
    /* numeric factors */
    int64_t *Fp, *Sp;
    int32_t *Fi, *Si, *piv;
    double *Fv, *Sv;
    double *upiv;           /* value of row i's pivot */
    int32_t nperturbed;
    int factored;
} orc;

static void *xmalloc(size_t n) { return malloc(n ? n : 1); }
static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s ? s : 1); }

void orc_destroy(orc *o)
{
    if (!o) return;
    free(o->arp); free(o->aci); free(o->av);
    free(o->pr); free(o->pc); free(o->dr); free(o->dc);
    free(o->brp); free(o->bci); free(o->bv); free(o->bsrc);
    free(o->Lp); free(o->Up); free(o->Li); free(o->Ui);
    free(o->node_ptr); free(o->node_of); free(o->is_sn);
    for (int t = 0; t < 4; t++) free(o->lev[t]);
    free(o->Fp); free(o->Sp); free(o->Fi); free(o->Si); free(o->piv);
    free(o->Fv); free(o->Sv); free(o->upiv);
    free(o);
}

/* ------------------------------------------------------------------------ */
/* O-3: B = R A C, entry (i', j') = dr[pr[i']] * A(pr[i'], pc[j']) * dc[pc[j']] */
/* ------------------------------------------------------------------------ */

static int form_b(orc *o)
{
    int32_t n = o->n;
    int64_t nnz = o->arp[n];
    int32_t *pcinv = xmalloc(sizeof(int32_t) * n);
    if (!pcinv) return ORC_ERR_OOM;
    for (int32_t j = 0; j < n; j++) pcinv[o->pc[j]] = j;
    free(o->brp); free(o->bci); free(o->bv); free(o->bsrc);
    o->brp = xmalloc(sizeof(int64_t) * (n + 1));
    o->bci = xmalloc(sizeof(int32_t) * nnz);
    o->bv = xmalloc(sizeof(double) * nnz);
    o->bsrc = xmalloc(sizeof(int64_t) * nnz);
    if (!o->brp || !o->bci || !o->bv || !o->bsrc) { free(pcinv); return ORC_ERR_OOM; }
    o->brp[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t r = o->pr[i];
        int64_t base = o->brp[i], len = o->arp[r + 1] - o->arp[r];
        o->brp[i + 1] = base + len;
        /* insertion sort by new column (rows are short) */
        for (int64_t t = 0; t < len; t++) {
            int64_t p = o->arp[r] + t;
            int32_t j = pcinv[o->aci[p]];
            double v = (o->dr[r] * o->av[p]) * o->dc[o->aci[p]];
            int64_t q = base + t;
            while (q > base && o->bci[q - 1] > j) {
                o->bci[q] = o->bci[q - 1]; o->bv[q] = o->bv[q - 1]; o->bsrc[q] = o->bsrc[q - 1];
                q--;
            }
            o->bci[q] = j; o->bv[q] = v; o->bsrc[q] = p;
        }
    }
    free(pcinv);
    return ORC_OK;
}

orc *orc_create(int32_t n, const int64_t *rp, const int32_t *ci, const double *v,
                const int32_t *pr, const int32_t *pc, const double *dr, const double *dc)
{
    if (n <= 0 || !rp || !ci || !v) return NULL;
    orc *o = xcalloc(1, sizeof(orc));
    if (!o) return NULL;
    o->n = n;
    int64_t nnz = rp[n];
    o->arp = xmalloc(sizeof(int64_t) * (n + 1));
    o->aci = xmalloc(sizeof(int32_t) * nnz);
    o->av = xmalloc(sizeof(double) * nnz);
    o->pr = xmalloc(sizeof(int32_t) * n);
    o->pc = xmalloc(sizeof(int32_t) * n);
    o->dr = xmalloc(sizeof(double) * n);
    o->dc = xmalloc(sizeof(double) * n);
    if (!o->arp || !o->aci || !o->av || !o->pr || !o->pc || !o->dr || !o->dc) { orc_destroy(o); return NULL; }
    memcpy(o->arp, rp, sizeof(int64_t) * (n + 1));
    memcpy(o->aci, ci, sizeof(int32_t) * nnz);
    memcpy(o->av, v, sizeof(double) * nnz);
    for (int32_t i = 0; i < n; i++) {
        o->pr[i] = pr ? pr[i] : i;
        o->pc[i] = pc ? pc[i] : i;
        o->dr[i] = dr ? dr[i] : 1.0;
        o->dc[i] = dc ? dc[i] : 1.0;
    }
    if (form_b(o) != ORC_OK) { orc_destroy(o); return NULL; }
    return o;
}

/* New values of A on the same pattern (the repeated-solve scenario, Sec. 3.2). */
int orc_set_values(orc *o, const double *v)
{
    if (!o || !v) return ORC_ERR_ARG;
    memcpy(o->av, v, sizeof(double) * o->arp[o->n]);
    for (int32_t i = 0; i < o->n; i++) {
        int32_t r = o->pr[i];
        for (int64_t q = o->brp[i]; q < o->brp[i + 1]; q++) {
            int64_t p = o->bsrc[q];
            o->bv[q] = (o->dr[r] * o->av[p]) * o->dc[o->aci[p]];
        }
    }
    o->factored = 0;
    return ORC_OK;
}

void orc_copy_b(const orc *o, int64_t *rp, int32_t *ci, double *v)
{
    memcpy(rp, o->brp, sizeof(int64_t) * (o->n + 1));
    memcpy(ci, o->bci, sizeof(int32_t) * o->brp[o->n]);
    memcpy(v, o->bv, sizeof(double) * o->brp[o->n]);
}

/* O-1: the scaled, matched matrix has |b_ii| = 1 and |b_ij| <= 1 (Sec. 2.1).
 * Returns 0 if the certificate holds within tol, else ORC_ERR_MATCH.
 * Also checks that pr and pc are permutations. */
int orc_check_matching(const orc *o, double tol)
{
    int32_t n = o->n;
    char *seen = xcalloc(n, 1);
    char *seen2 = xcalloc(n, 1);
    int bad = 0;
    for (int32_t i = 0; i < n && !bad; i++) {
        if (o->pr[i] < 0 || o->pr[i] >= n || seen[o->pr[i]]) bad = 1; else seen[o->pr[i]] = 1;
        if (o->pc[i] < 0 || o->pc[i] >= n || seen2[o->pc[i]]) bad = 1; else seen2[o->pc[i]] = 1;
    }
    free(seen); free(seen2);
    if (bad) return ORC_ERR_MATCH;
    for (int32_t i = 0; i < n; i++) {
        int diag = 0;
        for (int64_t q = o->brp[i]; q < o->brp[i + 1]; q++) {
            double a = fabs(o->bv[q]);
            if (o->bci[q] == i) { diag = 1; if (fabs(a - 1.0) > tol) return ORC_ERR_MATCH; }
            else if (a > 1.0 + tol) return ORC_ERR_MATCH;
        }
        if (!diag) return ORC_ERR_MATCH;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O-4 / O-5: exact symbolic structure and flop count                        */
/* ------------------------------------------------------------------------ */

/* binary min-heap of int32 */
typedef struct { int32_t *a; int64_t n, cap; } heap;
static int heap_push(heap *h, int32_t v)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 64;
        int32_t *na = realloc(h->a, sizeof(int32_t) * nc);
        if (!na) return ORC_ERR_OOM;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->n++;
    h->a[i] = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p] <= h->a[i]) break;
        int32_t t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t; i = p;
    }
    return ORC_OK;
}
static int32_t heap_pop(heap *h)
{
    int32_t top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->n && h->a[l] < h->a[s]) s = l;
        if (r < h->n && h->a[r] < h->a[s]) s = r;
        if (s == i) break;
        int32_t t = h->a[s]; h->a[s] = h->a[i]; h->a[i] = t; i = s;
    }
    return top;
}

typedef struct { int32_t *a; int64_t n, cap; } ivec;
static int ivec_push(ivec *v, int32_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int32_t *na = realloc(v->a, sizeof(int32_t) * nc);
        if (!na) return ORC_ERR_OOM;
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
    return ORC_OK;
}
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int orc_symbolic(orc *o)
{
    int32_t n = o->n;
    int32_t *mark = xmalloc(sizeof(int32_t) * n);
    int32_t *rowbuf = xmalloc(sizeof(int32_t) * n);
    heap h = {0};
    ivec L = {0}, U = {0};
    free(o->Lp); free(o->Up); free(o->Li); free(o->Ui);
    o->Li = NULL; o->Ui = NULL;
    o->Lp = xmalloc(sizeof(int64_t) * (n + 1));
    o->Up = xmalloc(sizeof(int64_t) * (n + 1));
    if (!mark || !rowbuf || !o->Lp || !o->Up) goto oom;
    for (int32_t i = 0; i < n; i++) mark[i] = -1;
    o->Lp[0] = o->Up[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        int64_t nu = 0;
        /* S = struct(B(i,:)) u {i} */
        mark[i] = i;
        rowbuf[nu++] = i;
        for (int64_t q = o->brp[i]; q < o->brp[i + 1]; q++) {
            int32_t j = o->bci[q];
            if (mark[j] == i) continue;
            mark[j] = i;
            if (j < i) { if (heap_push(&h, j)) goto oom; }
            else rowbuf[nu++] = j;
        }
        /* visit k < i in ascending order; the set grows */
        while (h.n > 0) {
            int32_t k = heap_pop(&h);
            if (ivec_push(&L, k)) goto oom;
            for (int64_t q = o->Up[k]; q < o->Up[k + 1]; q++) {
                int32_t j = o->Ui[q];
                if (j == k || mark[j] == i) continue;
                mark[j] = i;
                if (j < i) { if (heap_push(&h, j)) goto oom; }
                else rowbuf[nu++] = j;
            }
        }
        qsort(rowbuf, (size_t)nu, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < nu; t++) if (ivec_push(&U, rowbuf[t])) goto oom;
        o->Lp[i + 1] = L.n;
        o->Up[i + 1] = U.n;
        /* Ui is read while later rows are built: keep the pointer current */
        o->Ui = U.a;
    }
    o->Li = L.a; L.a = NULL;
    o->Ui = U.a; U.a = NULL;
    /* O-5: F = sum_k l_k (1 + 2 u_k) */
    {
        int64_t *lcount = xcalloc(n, sizeof(int64_t));
        if (!lcount) goto oom;
        for (int64_t q = 0; q < o->Lp[n]; q++) lcount[o->Li[q]]++;
        uint64_t F = 0;
        for (int32_t k = 0; k < n; k++) {
            uint64_t uk = (uint64_t)(o->Up[k + 1] - o->Up[k] - 1);
            F += (uint64_t)lcount[k] * (1 + 2 * uk);
        }
        o->flops = F;
        free(lcount);
    }
    free(mark); free(rowbuf); free(h.a);
    return ORC_OK;
oom:
    free(mark); free(rowbuf); free(h.a); free(L.a); free(U.a);
    o->Ui = NULL;
    return ORC_ERR_OOM;
}

/* ------------------------------------------------------------------------ */
/* O-6: supernode partition (Sec. 2.2 definition)                            */
/* ------------------------------------------------------------------------ */

/* rows r and r+1 chain when (r+1) is in U(r,:) and U(r,:)\{r,r+1} == U(r+1,:)\{r+1} */
static int chains(const orc *o, int32_t r)
{
    int64_t a0 = o->Up[r], a1 = o->Up[r + 1], b0 = o->Up[r + 1], b1 = o->Up[r + 2];
    /* U(r,:) sorted starts with r, so (r+1) in U(r,:) iff the second entry is r+1 */
    if (a1 - a0 < 2 || o->Ui[a0 + 1] != r + 1) return 0;
    /* compare U(r,:) minus its first two entries with U(r+1,:) minus its first */
    if ((a1 - a0 - 2) != (b1 - b0 - 1)) return 0;
    for (int64_t t = 0; t < a1 - a0 - 2; t++)
        if (o->Ui[a0 + 2 + t] != o->Ui[b0 + 1 + t]) return 0;
    return 1;
}

int orc_partition(orc *o, int32_t sn_min, int32_t sn_max)
{
    if (!o->Up) return ORC_ERR_STATE;
    int32_t n = o->n;
    if (sn_min < 2) sn_min = 2;
    if (sn_max < 1) sn_max = 1;
    free(o->node_ptr); free(o->node_of); free(o->is_sn);
    o->node_ptr = xmalloc(sizeof(int32_t) * (n + 1));
    o->node_of = xmalloc(sizeof(int32_t) * n);
    o->is_sn = xmalloc(sizeof(int32_t) * n);
    if (!o->node_ptr || !o->node_of || !o->is_sn) return ORC_ERR_OOM;
    int32_t nn = 0;
    int32_t r = 0;
    o->node_ptr[0] = 0;
    while (r < n) {
        int32_t e = r + 1;                 /* maximal run [r, e) */
        while (e < n && chains(o, e - 1)) e++;
        int32_t s = r;
        while (s < e) {                    /* chunks of sn_max from the top */
            int32_t c = e - s < sn_max ? e - s : sn_max;
            if (c >= sn_min) {
                o->is_sn[nn] = 1;
                for (int32_t t = s; t < s + c; t++) o->node_of[t] = nn;
                o->node_ptr[++nn] = s + c;
            } else {
                for (int32_t t = s; t < s + c; t++) {
                    o->is_sn[nn] = 0;
                    o->node_of[t] = nn;
                    o->node_ptr[++nn] = t + 1;
                }
            }
            s += c;
        }
        r = e;
    }
    o->nnodes = nn;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O-7: task graphs and levels (Sec. 2.2.1)                                  */
/* ------------------------------------------------------------------------ */

int orc_levels(orc *o)
{
    if (!o->node_of) return ORC_ERR_STATE;
    int32_t n = o->n, nn = o->nnodes;
    for (int t = 0; t < 4; t++) {
        free(o->lev[t]);
        o->lev[t] = xcalloc(nn, sizeof(int32_t));
        if (!o->lev[t]) return ORC_ERR_OOM;
    }
    int32_t *lv;
    /* factor / L-solve: v waits for every node u holding a k in L(i,:), i in v */
    lv = o->lev[0];
    for (int32_t i = 0; i < n; i++) {
        int32_t v = o->node_of[i];
        for (int64_t q = o->Lp[i]; q < o->Lp[i + 1]; q++) {
            int32_t u = o->node_of[o->Li[q]];
            if (u != v && lv[u] + 1 > lv[v]) lv[v] = lv[u] + 1;
        }
    }
    /* U-solve (backward): v waits for every node u holding a column of U(i,:), i in v */
    lv = o->lev[1];
    for (int32_t i = n - 1; i >= 0; i--) {
        int32_t v = o->node_of[i];
        for (int64_t q = o->Up[i]; q < o->Up[i + 1]; q++) {
            int32_t u = o->node_of[o->Ui[q]];
            if (u != v && lv[u] + 1 > lv[v]) lv[v] = lv[u] + 1;
        }
    }
    /* U^T-solve: reverse of the U graph */
    lv = o->lev[2];
    for (int32_t i = 0; i < n; i++) {
        int32_t v = o->node_of[i];
        for (int64_t q = o->Up[i]; q < o->Up[i + 1]; q++) {
            int32_t u = o->node_of[o->Ui[q]];
            if (u != v && lv[v] + 1 > lv[u]) lv[u] = lv[v] + 1;
        }
    }
    /* L^T-solve: reverse of the L graph */
    lv = o->lev[3];
    for (int32_t i = n - 1; i >= 0; i--) {
        int32_t v = o->node_of[i];
        for (int64_t q = o->Lp[i]; q < o->Lp[i + 1]; q++) {
            int32_t u = o->node_of[o->Li[q]];
            if (u != v && lv[v] + 1 > lv[u]) lv[u] = lv[v] + 1;
        }
    }
    for (int t = 0; t < 4; t++) {
        int32_t m = -1;
        for (int32_t v = 0; v < nn; v++) if (o->lev[t][v] > m) m = o->lev[t][v];
        o->nlev[t] = m + 1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O-8: up-looking numerical factorisation with supernode diagonal pivoting  */
/* and pivot perturbation (Sec. 2.2)                                         */
/* ------------------------------------------------------------------------ */

/* Perturbation threshold of Sec. 2.2 (the paper names the technique, not its
 * value): rel * max |b_ij| over this oracle's own B, 1 when B is all zero.
 * With rel = sqrt(eps) and B scaled to max |b_ij| = 1 by the static pivoting
 * this is the usual tiny-pivot replacement level.  Read on the values B holds
 * when it is called: for a refactorisation the threshold of the analysed
 * values is taken before orc_set_values. */
double orc_pivot_tau(const orc *o, double rel)
{
    double m = 0.0;
    for (int64_t q = 0; q < o->brp[o->n]; q++)
        if (fabs(o->bv[q]) > m) m = fabs(o->bv[q]);
    return rel * (m > 0 ? m : 1.0);
}

/* pivot_search = 1: choose pivots; 0: reuse piv_in (refactorisation). */
int orc_numeric(orc *o, double tau, int pivot_search, const int32_t *piv_in)
{
    if (!o->lev[0] || !o->node_of) return ORC_ERR_STATE;
    if (!pivot_search && !piv_in) return ORC_ERR_ARG;
    int32_t n = o->n;
    /* padded source list of every row: whole supernodes, own supernode's earlier rows */
    free(o->Fp); free(o->Fi); free(o->Fv);
    free(o->Sp); free(o->Si); free(o->Sv); free(o->piv); free(o->upiv);
    o->Fp = xmalloc(sizeof(int64_t) * (n + 1));
    o->Sp = xmalloc(sizeof(int64_t) * (n + 1));
    o->piv = xmalloc(sizeof(int32_t) * n);
    o->upiv = xmalloc(sizeof(double) * n);
    double *x = xcalloc(n, sizeof(double));
    char *used = xcalloc(n, 1);        /* block columns already pivoted (own supernode) */
    ivec F = {0};
    if (!o->Fp || !o->Sp || !o->piv || !o->upiv || !x || !used) goto oom;
    o->Fp[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t v = o->node_of[i];
        int32_t last = -1;
        for (int64_t q = o->Lp[i]; q < o->Lp[i + 1]; q++) {
            int32_t u = o->node_of[o->Li[q]];
            if (u == v) continue;
            if (o->is_sn[u]) {
                if (u == last) continue;
                for (int32_t k = o->node_ptr[u]; k < o->node_ptr[u + 1]; k++) if (ivec_push(&F, k)) goto oom;
            } else {
                if (ivec_push(&F, o->Li[q])) goto oom;
            }
            last = u;
        }
        if (o->is_sn[v]) for (int32_t k = o->node_ptr[v]; k < i; k++) if (ivec_push(&F, k)) goto oom;
        o->Fp[i + 1] = F.n;
    }
    o->Fi = F.a; F.a = NULL;
    o->Fv = xmalloc(sizeof(double) * o->Fp[n]);
    o->Si = xmalloc(sizeof(int32_t) * o->Up[n]);
    o->Sv = xmalloc(sizeof(double) * o->Up[n]);
    if (!o->Fv || !o->Si || !o->Sv) goto oom;
    memcpy(o->Sp, o->Up, sizeof(int64_t) * (n + 1));
    o->nperturbed = 0;
    uint64_t fpad = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t v = o->node_of[i];
        int32_t t0 = o->node_ptr[v], t1 = o->node_ptr[v + 1];
        /* scatter B(i,:) into the dense work vector */
        for (int64_t q = o->brp[i]; q < o->brp[i + 1]; q++) x[o->bci[q]] = o->bv[q];
        /* sources in ascending order */
        for (int64_t q = o->Fp[i]; q < o->Fp[i + 1]; q++) {
            int32_t k = o->Fi[q];
            int32_t pk = o->piv[k];
            double l = x[pk] / o->upiv[k];
            o->Fv[q] = l;
            x[pk] = 0.0;
            for (int64_t s = o->Sp[k]; s < o->Sp[k + 1]; s++) {
                int32_t j = o->Si[s];
                if (j != pk) x[j] -= l * o->Sv[s];
            }
            fpad += 1 + 2 * (uint64_t)(o->Sp[k + 1] - o->Sp[k] - 1);
        }
        /* pivot */
        int32_t p = i;
        if (o->is_sn[v]) {
            if (pivot_search) {
                double best = -1.0;
                for (int32_t c = t0; c < t1; c++) {
                    if (used[c]) continue;
                    if (fabs(x[c]) > best) { best = fabs(x[c]); p = c; }
                }
            } else {
                p = piv_in[i];
            }
            used[p] = 1;
        }
        o->piv[i] = p;
        if (fabs(x[p]) < tau) {
            x[p] = (x[p] < 0.0) ? -tau : tau;
            o->nperturbed++;
        }
        o->upiv[i] = x[p];
        /* U_st(i,:): unpivoted block columns then the columns past the block */
        int64_t s = o->Sp[i];
        if (o->is_sn[v]) {
            /* candidates are block columns not pivoted by rows t0..i-1 (p included) */
            for (int32_t c = t0; c < t1; c++) {
                if (used[c] && c != p) continue;
                o->Si[s] = c; o->Sv[s] = x[c]; s++; x[c] = 0.0;
            }
            for (int64_t q = o->Up[i]; q < o->Up[i + 1]; q++) {
                int32_t j = o->Ui[q];
                if (j < t1) continue;
                o->Si[s] = j; o->Sv[s] = x[j]; s++; x[j] = 0.0;
            }
            if (i == t1 - 1) for (int32_t c = t0; c < t1; c++) used[c] = 0;
        } else {
            for (int64_t q = o->Up[i]; q < o->Up[i + 1]; q++) {
                int32_t j = o->Ui[q];
                o->Si[s] = j; o->Sv[s] = x[j]; s++; x[j] = 0.0;
            }
        }
        if (s != o->Sp[i + 1]) goto oom; /* cannot happen: sizes agree by construction */
        /* every L column was zeroed when its source was applied */
    }
    o->flops_padded = fpad;
    free(x); free(used);
    o->factored = 1;
    return ORC_OK;
oom:
    free(x); free(used); free(F.a);
    return ORC_ERR_OOM;
}

/* ------------------------------------------------------------------------ */
/* O-9: forward-backward substitution (Sec. 2.3)                             */
/* ------------------------------------------------------------------------ */

/* Solve A x = b for one right-hand side given in the original index space. */
int orc_solve(const orc *o, const double *b, double *xout)
{
    if (!o->factored) return ORC_ERR_STATE;
    int32_t n = o->n;
    double *y = xmalloc(sizeof(double) * n);
    double *z = xmalloc(sizeof(double) * n);
    if (!y || !z) { free(y); free(z); return ORC_ERR_OOM; }
    for (int32_t i = 0; i < n; i++) y[i] = o->dr[o->pr[i]] * b[o->pr[i]];   /* c = R b */
    for (int32_t i = 0; i < n; i++) {                                          /* L y = c */
        double s = y[i];
        for (int64_t q = o->Fp[i]; q < o->Fp[i + 1]; q++) s -= o->Fv[q] * y[o->Fi[q]];
        y[i] = s;
    }
    for (int32_t i = n - 1; i >= 0; i--) {                                     /* U_st z = y */
        double s = y[i];
        int32_t p = o->piv[i];
        for (int64_t q = o->Sp[i]; q < o->Sp[i + 1]; q++)
            if (o->Si[q] != p) s -= o->Sv[q] * z[o->Si[q]];
        z[p] = s / o->upiv[i];
    }
    for (int32_t j = 0; j < n; j++) xout[o->pc[j]] = o->dc[o->pc[j]] * z[j];  /* x = C z */
    free(y); free(z);
    return ORC_OK;
}

/* Solve A^T lambda = g (O-11): lambda = R^T L^{-T} U_st^{-T} C^T g. */
int orc_solve_transposed(const orc *o, const double *g, double *lam)
{
    if (!o->factored) return ORC_ERR_STATE;
    int32_t n = o->n;
    double *h = xmalloc(sizeof(double) * n);
    double *w = xmalloc(sizeof(double) * n);
    if (!h || !w) { free(h); free(w); return ORC_ERR_OOM; }
    for (int32_t j = 0; j < n; j++) h[j] = o->dc[o->pc[j]] * g[o->pc[j]];     /* C^T g */
    /* U_st^T v = h, rows ascending: v_i = h[piv i] / U_st(i,piv i), then push */
    for (int32_t i = 0; i < n; i++) {
        int32_t p = o->piv[i];
        double vi = h[p] / o->upiv[i];
        w[i] = vi;
        for (int64_t q = o->Sp[i]; q < o->Sp[i + 1]; q++)
            if (o->Si[q] != p) h[o->Si[q]] -= o->Sv[q] * vi;
    }
    /* L^T u = v, rows descending: u_i final, then push into its sources */
    for (int32_t i = n - 1; i >= 0; i--) {
        double ui = w[i];
        for (int64_t q = o->Fp[i]; q < o->Fp[i + 1]; q++) w[o->Fi[q]] -= o->Fv[q] * ui;
    }
    for (int32_t i = 0; i < n; i++) lam[o->pr[i]] = o->dr[o->pr[i]] * w[i];  /* R^T u */
    free(h); free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O-10: backward error and iterative refinement (Sec. 2.3, Sec. 3.3)        */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated sum helper */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v; else k->c += (v - t) + k->s;
    k->s = t;
}

/* r = b - A x with compensated row sums (original A). */
void orc_residual(const orc *o, const double *b, const double *x, double *r)
{
    for (int32_t i = 0; i < o->n; i++) {
        ksum k = {b[i], 0.0};
        for (int64_t p = o->arp[i]; p < o->arp[i + 1]; p++) kadd(&k, -o->av[p] * x[o->aci[p]]);
        r[i] = k.s + k.c;
    }
}

/* Normwise backward error ||b-Ax||_inf / (||A||_inf ||x||_inf + ||b||_inf) and
 * the paper's accuracy measure ||Ax-b||_1 / ||b||_1 (Sec. 3.3). */
void orc_backward_error(const orc *o, const double *b, const double *x, double *eta, double *res1)
{
    int32_t n = o->n;
    double *r = xmalloc(sizeof(double) * n);
    orc_residual(o, b, x, r);
    double rinf = 0, xinf = 0, binf = 0, ainf = 0;
    ksum r1 = {0, 0}, b1 = {0, 0};
    for (int32_t i = 0; i < n; i++) {
        double ra = 0;
        for (int64_t p = o->arp[i]; p < o->arp[i + 1]; p++) ra += fabs(o->av[p]);
        if (ra > ainf) ainf = ra;
        if (fabs(r[i]) > rinf) rinf = fabs(r[i]);
        if (fabs(x[i]) > xinf) xinf = fabs(x[i]);
        if (fabs(b[i]) > binf) binf = fabs(b[i]);
        kadd(&r1, fabs(r[i]));
        kadd(&b1, fabs(b[i]));
    }
    double den = ainf * xinf + binf;
    *eta = den > 0 ? rinf / den : 0.0;
    double bb = b1.s + b1.c;
    *res1 = bb > 0 ? (r1.s + r1.c) / bb : 0.0;
    free(r);
}

/* Solve with refinement: stop at eta <= tol, on stagnation (eta_new > eta_old/2)
 * or after maxit corrections; returns the number of corrections applied and
 * keeps the best iterate. */
int orc_solve_ir(const orc *o, const double *b, double *x, double tol, int maxit, double *eta_out)
{
    int32_t n = o->n;
    double *r = xmalloc(sizeof(double) * n), *d = xmalloc(sizeof(double) * n);
    double *best = xmalloc(sizeof(double) * n);
    if (!r || !d || !best) { free(r); free(d); free(best); return ORC_ERR_OOM; }
    int rc = orc_solve(o, b, x);
    if (rc) { free(r); free(d); free(best); return rc; }
    double eta, res1, eta_best;
    orc_backward_error(o, b, x, &eta, &res1);
    eta_best = eta;
    memcpy(best, x, sizeof(double) * n);
    int it = 0;
    while (eta > tol && it < maxit) {
        orc_residual(o, b, x, r);
        orc_solve(o, r, d);
        for (int32_t i = 0; i < n; i++) x[i] += d[i];
        it++;
        double e2;
        orc_backward_error(o, b, x, &e2, &res1);
        if (e2 < eta_best) { eta_best = e2; memcpy(best, x, sizeof(double) * n); }
        if (e2 > eta / 2) break;
        eta = e2;
    }
    memcpy(x, best, sizeof(double) * n);
    if (eta_out) *eta_out = eta_best;
    free(r); free(d); free(best);
    return it;
}

/* Gradient of a loss through x = A^{-1} b given lambda = A^{-T} dL/dx (O-11):
 * dL/dA(p) = -lambda[row p] * x[col p] on the pattern, dL/db = lambda. */
void orc_gradient_values(const orc *o, const double *lam, const double *x, double *gval)
{
    for (int32_t i = 0; i < o->n; i++)
        for (int64_t p = o->arp[i]; p < o->arp[i + 1]; p++) gval[p] = -lam[i] * x[o->aci[p]];
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                 */
/* ------------------------------------------------------------------------ */

/* sizes[0..11] = n, nnz(A), nnz(L exact), nnz(U exact), F (as int64), F_padded,
 * nnodes, n supernodes, rows in supernodes, nnz of padded L, nperturbed, factored */
void orc_sizes(const orc *o, int64_t *sizes)
{
    memset(sizes, 0, sizeof(int64_t) * 12);
    sizes[0] = o->n;
    sizes[1] = o->arp[o->n];
    if (o->Lp) sizes[2] = o->Lp[o->n];
    if (o->Up) sizes[3] = o->Up[o->n];
    sizes[4] = (int64_t)o->flops;
    sizes[5] = (int64_t)o->flops_padded;
    sizes[6] = o->nnodes;
    if (o->is_sn) {
        for (int32_t v = 0; v < o->nnodes; v++) if (o->is_sn[v]) {
            sizes[7]++;
            sizes[8] += o->node_ptr[v + 1] - o->node_ptr[v];
        }
    }
    if (o->Fp) sizes[9] = o->Fp[o->n];
    sizes[10] = o->nperturbed;
    sizes[11] = o->factored;
}

void orc_copy_symbolic(const orc *o, int64_t *Lp, int32_t *Li, int64_t *Up, int32_t *Ui)
{
    memcpy(Lp, o->Lp, sizeof(int64_t) * (o->n + 1));
    memcpy(Li, o->Li, sizeof(int32_t) * o->Lp[o->n]);
    memcpy(Up, o->Up, sizeof(int64_t) * (o->n + 1));
    memcpy(Ui, o->Ui, sizeof(int32_t) * o->Up[o->n]);
}

void orc_copy_partition(const orc *o, int32_t *node_ptr, int32_t *is_sn)
{
    memcpy(node_ptr, o->node_ptr, sizeof(int32_t) * (o->nnodes + 1));
    memcpy(is_sn, o->is_sn, sizeof(int32_t) * o->nnodes);
}

void orc_copy_levels(const orc *o, int32_t *lev4)
{
    for (int t = 0; t < 4; t++) memcpy(lev4 + (int64_t)t * o->nnodes, o->lev[t], sizeof(int32_t) * o->nnodes);
}

void orc_copy_factors(const orc *o, int64_t *Fp, int32_t *Fi, double *Fv,
                      int64_t *Sp, int32_t *Si, double *Sv, int32_t *piv)
{
    int32_t n = o->n;
    memcpy(Fp, o->Fp, sizeof(int64_t) * (n + 1));
    memcpy(Fi, o->Fi, sizeof(int32_t) * o->Fp[n]);
    memcpy(Fv, o->Fv, sizeof(double) * o->Fp[n]);
    memcpy(Sp, o->Sp, sizeof(int64_t) * (n + 1));
    memcpy(Si, o->Si, sizeof(int32_t) * o->Sp[n]);
    memcpy(Sv, o->Sv, sizeof(double) * o->Sp[n]);
    memcpy(piv, o->piv, sizeof(int32_t) * n);
}
