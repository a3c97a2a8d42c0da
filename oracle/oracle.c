/*
 * CPU oracle for butterfly counting, tip decomposition and wing
 * decomposition of a simple bipartite graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * Everything here is plain and slow on purpose: each routine is the
 * textbook definition or the paper's sequential bottom-up peeling
 * (Section 2.2, Algorithm 2), with none of PBNG's two-phase machinery,
 * priority relabelling or BE-Index.  Peeling is sequential.  The counting
 * definitions of Section 2.1 are independent per start vertex, so counting
 * may hand whole start vertices to several host threads (orc_set_threads;
 * one thread by default): each start's sums are still formed by one thread
 * in the same order, so the results do not depend on the thread count.
 *
 * Graph input: U-side CSR.  row_ptr[n_u+1] (int64), col[m] (int32) with the
 * V ids of every row strictly increasing.  Edge id = CSR slot.
 * All supports and entity numbers are uint64.
 *
 * Return codes: 0 ok, -1 bad argument, -2 malformed graph, -3 out of memory,
 * -9 stopped early on the work budget (outputs partial).
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef int32_t i32;

/* ---------------------------------------------------------------------- */
/* Graph validation and the V-side adjacency (transpose).                  */
/* ---------------------------------------------------------------------- */

int orc_validate(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col)
{
    if (n_u < 0 || n_v < 0 || !row_ptr) return -1;
    if (row_ptr[0] != 0) return -2;
    for (i64 u = 0; u < n_u; ++u) {
        if (row_ptr[u + 1] < row_ptr[u]) return -2;
        for (i64 j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            if (col[j] < 0 || col[j] >= n_v) return -2;
            if (j > row_ptr[u] && col[j] <= col[j - 1]) return -2; /* unsorted or duplicate */
        }
    }
    return 0;
}

/* V-side CSR by counting sort: vptr[n_v+1], vadj[m] = U ids ascending,
 * veid[m] = edge id of (vadj[k], v).                                        */
static int transpose(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col,
                     i64 **vptr_o, i32 **vadj_o, i64 **veid_o)
{
    i64 m = row_ptr[n_u];
    i64 *vptr = calloc((size_t)n_v + 1, sizeof(i64));
    i32 *vadj = malloc((size_t)(m ? m : 1) * sizeof(i32));
    i64 *veid = malloc((size_t)(m ? m : 1) * sizeof(i64));
    i64 *fill = malloc((size_t)(n_v ? n_v : 1) * sizeof(i64));
    if (!vptr || !vadj || !veid || !fill) { free(vptr); free(vadj); free(veid); free(fill); return -3; }
    for (i64 e = 0; e < m; ++e) vptr[col[e] + 1]++;
    for (i64 v = 0; v < n_v; ++v) vptr[v + 1] += vptr[v];
    for (i64 v = 0; v < n_v; ++v) fill[v] = vptr[v];
    for (i64 u = 0; u < n_u; ++u)
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            i64 k = fill[col[e]]++;
            vadj[k] = (i32)u;
            veid[k] = e;
        }
    free(fill);
    *vptr_o = vptr; *vadj_o = vadj; *veid_o = veid;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Counting (Section 2.1 definitions, not Algorithm 1's priority scheme).   */
/*                                                                          */
/* For a vertex u, c(u,u') = |N_u ∩ N_u'| is found by walking every wedge   */
/* u -> v -> u'.  Then                                                       */
/*   support(u)     = sum over u' != u of C(c(u,u'), 2)                      */
/*   support(u, v)  = sum over u' in N_v, u' != u, of (c(u,u') - 1)          */
/* (each butterfly through edge (u,v) is one (u', v') with v' in both        */
/* N_u and N_u', v' != v).                                                  */
/* ---------------------------------------------------------------------- */

static u64 choose2(u64 c) { return c * (c - 1) / 2; }

/* Host threads used by counting (start vertices split among them). */
static int g_threads = 1;

int orc_set_threads(int n)
{
    g_threads = n > 0 ? n : 1;
    return g_threads;
}

/* Per-vertex supports of the rows of a CSR (the "left" side), using the
 * transposed lists for the 2-hop walk.                                     */
static int count_left(i64 n_l, const i64 *lptr, const i32 *ladj,
                      const i64 *rptr, const i32 *radj, u64 *out_vertex,
                      u64 *out_edge /* optional, indexed by left CSR slot */)
{
    int rc = 0;
#pragma omp parallel num_threads(g_threads)
    {
        /* each thread: its own counter array and touched list */
        u64 *cnt = calloc((size_t)(n_l ? n_l : 1), sizeof(u64));
        i32 *touched = malloc((size_t)(n_l ? n_l : 1) * sizeof(i32));
        if (!cnt || !touched) {
#pragma omp atomic write
            rc = -3;
        }
#pragma omp barrier
        if (rc == 0) {
#pragma omp for schedule(dynamic, 64)
            for (i64 u = 0; u < n_l; ++u) {
                i64 nt = 0;
                for (i64 j = lptr[u]; j < lptr[u + 1]; ++j) {
                    i32 v = ladj[j];
                    for (i64 k = rptr[v]; k < rptr[v + 1]; ++k) {
                        i32 w = radj[k];
                        if (w == u) continue;
                        if (cnt[w] == 0) touched[nt++] = w;
                        cnt[w]++;
                    }
                }
                if (out_vertex) {
                    u64 s = 0;
                    for (i64 t = 0; t < nt; ++t) s += choose2(cnt[touched[t]]);
                    out_vertex[u] = s;
                }
                if (out_edge) {
                    for (i64 j = lptr[u]; j < lptr[u + 1]; ++j) {
                        i32 v = ladj[j];
                        u64 s = 0;
                        for (i64 k = rptr[v]; k < rptr[v + 1]; ++k) {
                            i32 w = radj[k];
                            if (w == u) continue;
                            s += cnt[w] - 1;
                        }
                        out_edge[j] = s;
                    }
                }
                for (i64 t = 0; t < nt; ++t) cnt[touched[t]] = 0;
            }
        }
        free(cnt);
        free(touched);
    }
    return rc;
}

/* Per-vertex butterfly counts of both sides: out_u[n_u], out_v[n_v]
 * (either may be NULL).                                                    */
int orc_count_vertex(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col,
                     u64 *out_u, u64 *out_v)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    if (out_u) rc = count_left(n_u, row_ptr, col, vptr, vadj, out_u, NULL);
    if (!rc && out_v) rc = count_left(n_v, vptr, vadj, row_ptr, col, out_v, NULL);
    free(vptr); free(vadj); free(veid);
    return rc;
}

/* Per-edge butterfly counts: out_e[m] in edge-id order.                    */
int orc_count_edge(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col, u64 *out_e)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    if (!out_e) return -1;
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    rc = count_left(n_u, row_ptr, col, vptr, vadj, NULL, out_e);
    free(vptr); free(vadj); free(veid);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Indexed binary min-heap over vertex ids ordered by (key[id], id): each    */
/* vertex sits in the heap once; a lowered key moves it up (keys only       */
/* decrease while peeling), so memory stays O(n).                           */
/* ---------------------------------------------------------------------- */

typedef struct { i64 *a; i64 *pos; const u64 *key; i64 n; } iheap;

static int ih_less(const iheap *h, i64 x, i64 y)
{
    return h->key[x] < h->key[y] || (h->key[x] == h->key[y] && x < y);
}

static void ih_place(iheap *h, i64 i, i64 x) { h->a[i] = x; h->pos[x] = i; }

static void ih_up(iheap *h, i64 i)
{
    i64 x = h->a[i];
    while (i > 0) {
        i64 p = (i - 1) / 2;
        if (!ih_less(h, x, h->a[p])) break;
        ih_place(h, i, h->a[p]);
        i = p;
    }
    ih_place(h, i, x);
}

static i64 ih_pop(iheap *h)
{
    i64 top = h->a[0];
    h->pos[top] = -1;
    i64 x = h->a[--h->n];
    if (h->n == 0) return top;
    i64 i = 0;
    for (;;) {
        i64 l = 2 * i + 1, r = l + 1, s = -1;
        if (l < h->n && ih_less(h, h->a[l], x)) s = l;
        if (r < h->n && ih_less(h, h->a[r], s < 0 ? x : h->a[l])) s = r;
        if (s < 0) break;
        ih_place(h, i, h->a[s]);
        i = s;
    }
    ih_place(h, i, x);
    return top;
}

/* ---------------------------------------------------------------------- */
/* Tip decomposition by sequential bottom-up peeling (Section 2.2, the      */
/* vertex form of Algorithm 2).  Only the rows of the CSR are peeled; the    */
/* other side is never removed (Definition 2: a k-tip keeps all of V).       */
/*                                                                          */
/* Repeatedly take an unpeeled vertex u of minimum support, record          */
/* theta_u = support(u), remove u, and for every unpeeled u' sharing c >= 1 */
/* neighbours with u set support(u') = max(theta_u, support(u') - C(c,2)).  */
/*                                                                          */
/* stats[0] = wedges walked (u -> v -> u', u' != u, dead u' included, i.e.  */
/*            no dynamic graph updates), stats[1] = vertices peeled.         */
/* wedge_budget > 0 stops once that many wedges were walked (returns -9).   */
/* order (optional, int64[n_l]) receives the peel order.                    */
/* ---------------------------------------------------------------------- */

static int tip_left(i64 n_l, const i64 *lptr, const i32 *ladj, const i64 *rptr,
                    const i32 *radj, u64 *theta, u64 *stats, u64 wedge_budget, i64 *order)
{
    u64 *sup = malloc((size_t)(n_l ? n_l : 1) * sizeof(u64));
    u64 *cnt = calloc((size_t)(n_l ? n_l : 1), sizeof(u64));
    i32 *touched = malloc((size_t)(n_l ? n_l : 1) * sizeof(i32));
    unsigned char *alive = malloc((size_t)(n_l ? n_l : 1));
    iheap h = {0};
    h.a = malloc((size_t)(n_l ? n_l : 1) * sizeof(i64));
    h.pos = malloc((size_t)(n_l ? n_l : 1) * sizeof(i64));
    h.key = sup;
    int rc = 0;
    if (!sup || !cnt || !touched || !alive || !h.a || !h.pos) { rc = -3; goto out; }
    rc = count_left(n_l, lptr, ladj, rptr, radj, sup, NULL);
    if (rc) goto out;
    for (i64 u = 0; u < n_l; ++u) {
        alive[u] = 1;
        ih_place(&h, h.n, u);
        ih_up(&h, h.n++);
    }
    u64 wedges = 0, peeled = 0;
    while (h.n > 0) {
        i64 u = ih_pop(&h);
        u64 k = sup[u];
        theta[u] = k;
        alive[u] = 0;
        if (order) order[peeled] = u;
        peeled++;
        i64 nt = 0;
        for (i64 j = lptr[u]; j < lptr[u + 1]; ++j) {
            i32 v = ladj[j];
            for (i64 q = rptr[v]; q < rptr[v + 1]; ++q) {
                i32 w = radj[q];
                if (w == u) continue;
                wedges++;
                if (!alive[w]) continue;
                if (cnt[w] == 0) touched[nt++] = w;
                cnt[w]++;
            }
        }
        for (i64 t = 0; t < nt; ++t) {
            i32 w = touched[t];
            u64 c = cnt[w];
            cnt[w] = 0;
            if (c < 2) continue;
            u64 d = choose2(c);
            u64 nv = sup[w] > d ? sup[w] - d : 0;
            if (nv < k) nv = k;
            if (nv != sup[w]) {
                sup[w] = nv;
                ih_up(&h, h.pos[w]);
            }
        }
        if (wedge_budget && wedges >= wedge_budget) { rc = -9; break; }
    }
    if (stats) { stats[0] = wedges; stats[1] = peeled; }
out:
    free(sup); free(cnt); free(touched); free(alive); free(h.a); free(h.pos);
    return rc;
}

/* side 0: peel U; side 1: peel V.  theta has n_u or n_v entries.           */
int orc_tip(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col, int side,
            u64 *theta, u64 *stats, u64 wedge_budget, i64 *order)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    if (!theta || (side != 0 && side != 1)) return -1;
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    if (side == 0) rc = tip_left(n_u, row_ptr, col, vptr, vadj, theta, stats, wedge_budget, order);
    else           rc = tip_left(n_v, vptr, vadj, row_ptr, col, theta, stats, wedge_budget, order);
    free(vptr); free(vadj); free(veid);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Wing decomposition by sequential bottom-up peeling (Algorithm 2).        */
/*                                                                          */
/* Support of an edge is below m (each butterfly through e = (u,v) is named */
/* by its opposite edge (u',v')), and peeling changes a support by exactly  */
/* one per removed butterfly, so a dense bucket queue in the Batagelj-      */
/* Zaversnik arrangement holds the edges sorted by support: each decrement  */
/* moves an edge to the front of its bucket and shifts the bucket start.    */
/*                                                                          */
/* Peeling e = (u,v) with support k: every butterfly {(u,v),(u,v'),(u',v),  */
/* (u',v')} whose other three edges are unpeeled is removed, and each of    */
/* those three edges with support above k loses one (the max(k, s-1) of     */
/* Algorithm 2).  The butterflies are found from whichever endpoint's       */
/* 2-hop walk is shorter in the input graph (either walk finds all of them).*/
/*                                                                          */
/* stats[0] = wedges walked, stats[1] = support updates applied.            */
/* ---------------------------------------------------------------------- */

typedef struct {
    u64 *sup;      /* support per edge                                  */
    i64 *vert;     /* edges sorted by support                            */
    i64 *pos;      /* position of each edge in vert                      */
    i64 *bin;      /* start of each support bucket in vert               */
} bucketq;

static void bq_dec(bucketq *q, i64 e)
{
    u64 s = q->sup[e];
    i64 pe = q->pos[e];
    i64 pw = q->bin[s];          /* first slot of bucket s */
    i64 w = q->vert[pw];
    if (w != e) {
        q->vert[pe] = w; q->pos[w] = pe;
        q->vert[pw] = e; q->pos[e] = pw;
    }
    q->bin[s]++;
    q->sup[e] = s - 1;
}

int orc_wing(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col, u64 *theta,
             u64 *stats, u64 wedge_budget, i64 *order)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    if (!theta && row_ptr[n_u] > 0) return -1;
    i64 m = row_ptr[n_u];
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    bucketq q = {0};
    i64 *mark_u = NULL, *mark_v = NULL;   /* edge id of (u, v') / (u', v) marked, -1 if none */
    unsigned char *alive = NULL;
    u64 *cost_u = NULL, *cost_v = NULL;
    i64 *eu = NULL;
    q.sup = malloc((size_t)(m ? m : 1) * sizeof(u64));
    q.vert = malloc((size_t)(m ? m : 1) * sizeof(i64));
    q.pos = malloc((size_t)(m ? m : 1) * sizeof(i64));
    q.bin = calloc((size_t)m + 2, sizeof(i64));
    mark_v = malloc((size_t)(n_v ? n_v : 1) * sizeof(i64));
    mark_u = malloc((size_t)(n_u ? n_u : 1) * sizeof(i64));
    alive = malloc((size_t)(m ? m : 1));
    cost_u = calloc((size_t)(n_u ? n_u : 1), sizeof(u64));
    cost_v = calloc((size_t)(n_v ? n_v : 1), sizeof(u64));
    eu = malloc((size_t)(m ? m : 1) * sizeof(i64));
    if (!q.sup || !q.vert || !q.pos || !q.bin || !mark_u || !mark_v || !alive || !cost_u || !cost_v || !eu) { rc = -3; goto out; }
    rc = count_left(n_u, row_ptr, col, vptr, vadj, NULL, q.sup);
    if (rc) goto out;
    for (i64 u = 0; u < n_u; ++u)
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) eu[e] = u;
    /* walk lengths: from u, sum of d(v') over v' in N_u; from v, sum of d(u') */
    for (i64 u = 0; u < n_u; ++u)
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            i32 v = col[e];
            cost_u[u] += (u64)(vptr[v + 1] - vptr[v]);
            cost_v[v] += (u64)(row_ptr[u + 1] - row_ptr[u]);
        }
    for (i64 v = 0; v < n_v; ++v) mark_v[v] = -1;
    for (i64 u = 0; u < n_u; ++u) mark_u[u] = -1;
    /* bucket sort by support */
    for (i64 e = 0; e < m; ++e) q.bin[q.sup[e] + 1]++;
    for (i64 s = 0; s <= m; ++s) q.bin[s + 1] += q.bin[s];
    {
        i64 *fill = malloc((size_t)(m + 1) * sizeof(i64));
        if (!fill) { rc = -3; goto out; }
        memcpy(fill, q.bin, (size_t)(m + 1) * sizeof(i64));
        for (i64 e = 0; e < m; ++e) { i64 p = fill[q.sup[e]]++; q.vert[p] = e; q.pos[e] = p; }
        free(fill);
    }
    for (i64 e = 0; e < m; ++e) alive[e] = 1;
    u64 wedges = 0, updates = 0;
    for (i64 i = 0; i < m; ++i) {
        i64 e = q.vert[i];
        u64 k = q.sup[e];
        theta[e] = k;
        if (order) order[i] = e;
        alive[e] = 0;
        i64 u = eu[e];
        i32 v = col[e];
        if (cost_u[u] <= cost_v[v]) {
            /* mark the other endpoints u' of v's live edges, walk v' in N_u */
            for (i64 t = vptr[v]; t < vptr[v + 1]; ++t)
                if (alive[veid[t]]) mark_u[vadj[t]] = veid[t];
            for (i64 j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                i64 e1 = j;                          /* (u, v') */
                if (!alive[e1]) continue;
                i32 vp = col[j];
                for (i64 t = vptr[vp]; t < vptr[vp + 1]; ++t) {
                    i32 up = vadj[t];
                    if (up == u) continue;
                    wedges++;
                    i64 e3 = veid[t];                /* (u', v') */
                    i64 e2 = mark_u[up];             /* (u', v)  */
                    if (e2 < 0 || !alive[e3]) continue;
                    if (q.sup[e1] > k) { bq_dec(&q, e1); updates++; }
                    if (q.sup[e2] > k) { bq_dec(&q, e2); updates++; }
                    if (q.sup[e3] > k) { bq_dec(&q, e3); updates++; }
                }
            }
            for (i64 t = vptr[v]; t < vptr[v + 1]; ++t) mark_u[vadj[t]] = -1;
        } else {
            /* mark the other endpoints v' of u's live edges, walk u' in N_v */
            for (i64 j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
                if (alive[j]) mark_v[col[j]] = j;
            for (i64 t = vptr[v]; t < vptr[v + 1]; ++t) {
                i64 e2 = veid[t];                    /* (u', v) */
                if (!alive[e2]) continue;
                i32 up = vadj[t];
                for (i64 j = row_ptr[up]; j < row_ptr[up + 1]; ++j) {
                    i32 vp = col[j];
                    if (vp == v) continue;
                    wedges++;
                    i64 e3 = j;                      /* (u', v') */
                    i64 e1 = mark_v[vp];             /* (u, v')  */
                    if (e1 < 0 || !alive[e3]) continue;
                    if (q.sup[e1] > k) { bq_dec(&q, e1); updates++; }
                    if (q.sup[e2] > k) { bq_dec(&q, e2); updates++; }
                    if (q.sup[e3] > k) { bq_dec(&q, e3); updates++; }
                }
            }
            for (i64 j = row_ptr[u]; j < row_ptr[u + 1]; ++j) mark_v[col[j]] = -1;
        }
        if (wedge_budget && wedges >= wedge_budget) { rc = -9; break; }
    }
    if (stats) { stats[0] = wedges; stats[1] = updates; }
out:
    free(q.sup); free(q.vert); free(q.pos); free(q.bin); free(mark_u); free(mark_v);
    free(alive); free(cost_u); free(cost_v); free(eu);
    free(vptr); free(vadj); free(veid);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* k-tips and k-wings from entity numbers (Section 2.2, Definitions 1-2).   */
/*                                                                          */
/* The k-tips of side U are the butterfly-connected components of the U     */
/* vertices with tip number >= k (with all of V): two such vertices are     */
/* joined when they share at least two neighbours (they lie in a common     */
/* butterfly).  The k-wings are the butterfly-connected components of the   */
/* edges with wing number >= k: two edges are joined when some butterfly of */
/* that edge set holds both.  Components are named by their smallest        */
/* member id; entities below k get -1.  Union-find with union by smaller    */
/* root, so every root is its component's smallest id.                      */
/* ---------------------------------------------------------------------- */

static i64 uf_find(i64 *p, i64 x)
{
    while (p[x] != x) x = p[x];
    return x;
}

static void uf_union(i64 *p, i64 a, i64 b)
{
    a = uf_find(p, a);
    b = uf_find(p, b);
    if (a == b) return;
    if (a < b) p[b] = a; else p[a] = b;
}

/* side 0: components of U vertices, side 1: of V vertices.                 */
int orc_tip_components(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col, int side,
                       const u64 *theta, u64 k, i64 *comp)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    if (side != 0 && side != 1) return -1;
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    i64 n_l = side == 0 ? n_u : n_v;
    const i64 *lptr = side == 0 ? row_ptr : vptr;
    const i32 *ladj = side == 0 ? col : vadj;
    const i64 *rptr = side == 0 ? vptr : row_ptr;
    const i32 *radj = side == 0 ? vadj : col;
    i64 *p = malloc((size_t)(n_l ? n_l : 1) * sizeof(i64));
    u64 *cnt = calloc((size_t)(n_l ? n_l : 1), sizeof(u64));
    i64 *touched = malloc((size_t)(n_l ? n_l : 1) * sizeof(i64));
    if (!p || !cnt || !touched) { rc = -3; goto out; }
    for (i64 u = 0; u < n_l; ++u) p[u] = u;
    for (i64 u = 0; u < n_l; ++u) {
        if (theta[u] < k) continue;
        i64 nt = 0;
        for (i64 j = lptr[u]; j < lptr[u + 1]; ++j) {
            i32 v = ladj[j];
            for (i64 q = rptr[v]; q < rptr[v + 1]; ++q) {
                i32 w = radj[q];
                if (w == u || theta[w] < k) continue;
                if (cnt[w] == 0) touched[nt++] = w;
                cnt[w]++;
            }
        }
        for (i64 t = 0; t < nt; ++t) {
            i64 w = touched[t];
            if (cnt[w] >= 2) uf_union(p, u, w);
            cnt[w] = 0;
        }
    }
    for (i64 u = 0; u < n_l; ++u) comp[u] = theta[u] >= k ? uf_find(p, u) : -1;
out:
    free(p); free(cnt); free(touched);
    free(vptr); free(vadj); free(veid);
    return rc;
}

int orc_wing_components(i64 n_u, i64 n_v, const i64 *row_ptr, const i32 *col, const u64 *theta, u64 k,
                        i64 *comp)
{
    int rc = orc_validate(n_u, n_v, row_ptr, col);
    if (rc) return rc;
    i64 m = row_ptr[n_u];
    i64 *vptr; i32 *vadj; i64 *veid;
    rc = transpose(n_u, n_v, row_ptr, col, &vptr, &vadj, &veid);
    if (rc) return rc;
    i64 *p = malloc((size_t)(m ? m : 1) * sizeof(i64));
    i64 *mark = malloc((size_t)(n_v ? n_v : 1) * sizeof(i64));  /* edge id of (u, v) or -1 */
    if (!p || !mark) { rc = -3; goto out; }
    for (i64 e = 0; e < m; ++e) p[e] = e;
    for (i64 v = 0; v < n_v; ++v) mark[v] = -1;
    /* every butterfly {(u,v),(u,v'),(u',v),(u',v')} of the edges with wing
       number >= k, found from its smaller U vertex u, joins its four edges */
    for (i64 u = 0; u < n_u; ++u) {
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (theta[e] >= k) mark[col[e]] = e;
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            if (theta[e] < k) continue;
            i32 v = col[e];
            for (i64 q = vptr[v]; q < vptr[v + 1]; ++q) {
                i32 w = vadj[q];                 /* u' */
                i64 f = veid[q];                 /* (u', v) */
                if (w <= u || theta[f] < k) continue;
                for (i64 g2 = row_ptr[w]; g2 < row_ptr[w + 1]; ++g2) {
                    i32 v2 = col[g2];            /* v' */
                    if (v2 <= v || theta[g2] < k || mark[v2] < 0) continue;
                    uf_union(p, e, f);
                    uf_union(p, e, mark[v2]);
                    uf_union(p, e, g2);
                }
            }
        }
        for (i64 e = row_ptr[u]; e < row_ptr[u + 1]; ++e) mark[col[e]] = -1;
    }
    for (i64 e = 0; e < m; ++e) comp[e] = theta[e] >= k ? uf_find(p, e) : -1;
out:
    free(p); free(mark);
    free(vptr); free(vadj); free(veid);
    return rc;
}
