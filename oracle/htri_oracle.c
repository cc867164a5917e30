/*
 * CPU oracle for hyper-triangle counting -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never calls it
 * and shares no code, header, table or helper with it.
 *
 * It is the plain two-step algorithm of Yin et al., "Efficient Computation of
 * Hyper-triangles on Hypergraphs" (PVLDB 18(3), 2024), written for
 * obviousness, not speed:
 *
 *   normalise   Def. 2.1 (a hyperedge is a non-empty vertex SET) and the
 *               Section 2 assumption that no two hyperedges hold the same
 *               vertex set (the experiments deduplicate, Section 6.1).
 *   step 1      Algorithm 2 ("Preprocess"): the per-vertex hyperedge lists
 *               E_v in ascending id order, then for every e_i the hyperedges
 *               e_j (j > i) that share a vertex, their common-vertex count
 *               omega_ij and their type (inclusion iff omega_ij equals
 *               min(|e_i|,|e_j|), intersection otherwise; Def. 2.3).
 *   step 2      Algorithm 3 generalised to every class as "Exact-adv" does
 *               (Section 6.1): each hyperwedge (i,j), i<j, is closed by every
 *               k > j adjacent to both; a triple is therefore met exactly once,
 *               at its two smallest ids -- the hyperwedge order O of Section 2
 *               and the i<min{j,k} rule of Algorithm 1.
 *   classify    the seven regions a..g of Section 2 (Def. 2.4 and the text
 *               after it), with g = |e_i & e_j & e_k| taken as |Omega_ij & e_k|
 *               (Omega_ij, the common vertices of the hyperwedge (Def. 2.2),
 *               listed once per hyperwedge by merging the two sorted member
 *               lists, then merged with e_k); classes with inclusion
 *               hyperwedges follow the rules of Algorithm 5 (Count-CCC,
 *               Count-TCC, Count-TTC), the intersection-only class (TTT) is
 *               numbered from which regions are empty.
 *
 * Pattern numbers 1-8 are fixed by Algorithm 5's arithmetic, 5 by the e-mail
 * case study (Fig. 7) and 10 and 12 by the co-authorship case study (Fig. 6).
 * The figure that numbers the rest is not available; 9, 11 and 13-20 follow
 * the order (pair regions non-empty, then private regions non-empty,
 * ascending) -- parity unpinned against the paper for those numbers only.
 *
 * Counts are int64.  Multithreading (pthreads over owners i, per-thread
 * arrays summed in thread order) mirrors the paper's Par-adv decomposition
 * (Section 3.4) and keeps every result deterministic.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID -1
#define ORC_E_RANGE -2
#define ORC_E_EMPTY_EDGE -3
#define ORC_E_DUPLICATE_EDGE -4
#define ORC_E_OOM -5
#define ORC_E_STATE -8

typedef struct {
    /* normalised hypergraph: ids 0..m-1 are the surviving input hyperedges in
     * input order */
    int64_t m;
    int32_t n;
    int64_t *off;      /* m+1 */
    int32_t *mem;      /* sorted, distinct members */
    int64_t *orig;     /* normalised id -> input index */
    int64_t removed;   /* duplicate hyperedges dropped */
    /* step 1 */
    int have_wedges;
    int64_t *vptr;     /* n+1: E_v lists */
    int32_t *vadj;
    int64_t nw;        /* number of hyperwedges (i<j) */
    int64_t *wptr;     /* m+1: wedges of owner i are [wptr[i], wptr[i+1]) */
    int32_t *wj;       /* partner j (> i), ascending within an owner */
    int32_t *wom;      /* omega_ij */
    int64_t *nptr;     /* m+1: symmetric adjacency N(x), ascending */
    int32_t *nadj;
    int32_t *nom;
    int64_t n_incl, n_inter;
} orc_graph;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* lexicographic comparison of two hyperedges' sorted member lists; ties are
 * broken by input index so that the first occurrence sorts first */
static const int64_t *g_cmp_off;
static const int32_t *g_cmp_mem;
static int cmp_edge(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    int64_t lx = g_cmp_off[x + 1] - g_cmp_off[x], ly = g_cmp_off[y + 1] - g_cmp_off[y];
    int64_t l = lx < ly ? lx : ly;
    for (int64_t t = 0; t < l; t++) {
        int32_t u = g_cmp_mem[g_cmp_off[x] + t], v = g_cmp_mem[g_cmp_off[y] + t];
        if (u != v) return (u > v) - (u < v);
    }
    if (lx != ly) return (lx > ly) - (lx < ly);
    return (x > y) - (x < y);
}

static int same_edge(const int64_t *off, const int32_t *mem, int64_t x, int64_t y) {
    int64_t lx = off[x + 1] - off[x];
    if (lx != off[y + 1] - off[y]) return 0;
    return memcmp(mem + off[x], mem + off[y], (size_t)lx * sizeof(int32_t)) == 0;
}

void orc_free(void *h) {
    orc_graph *g = (orc_graph *)h;
    if (!g) return;
    free(g->off); free(g->mem); free(g->orig);
    free(g->vptr); free(g->vadj); free(g->wptr); free(g->wj); free(g->wom);
    free(g->nptr); free(g->nadj); free(g->nom);
    free(g);
}

/* Normalise (Def. 2.1 + the distinct-hyperedge assumption).
 * dedupe != 0: keep the first occurrence of each vertex set; else fail on a
 * duplicate. */
int orc_normalize(const int64_t *off_in, int64_t m_in, const int32_t *mem_in, int32_t n,
                  int dedupe, void **out) {
    *out = NULL;
    if (m_in < 0 || n < 0 || !off_in || off_in[0] != 0) return ORC_E_INVALID;
    for (int64_t x = 0; x < m_in; x++)
        if (off_in[x + 1] < off_in[x]) return ORC_E_INVALID;
    int64_t nnz_in = off_in[m_in];
    for (int64_t t = 0; t < nnz_in; t++)
        if (mem_in[t] < 0 || mem_in[t] >= n) return ORC_E_RANGE;

    /* 1. sort each hyperedge's members and drop repeated vertex ids */
    int64_t *off1 = malloc(sizeof(int64_t) * (m_in + 1));
    int32_t *mem1 = malloc(sizeof(int32_t) * (nnz_in ? nnz_in : 1));
    if (!off1 || !mem1) { free(off1); free(mem1); return ORC_E_OOM; }
    off1[0] = 0;
    for (int64_t x = 0; x < m_in; x++) {
        int64_t b = off_in[x], l = off_in[x + 1] - b;
        int32_t *dst = mem1 + off1[x];
        memcpy(dst, mem_in + b, (size_t)l * sizeof(int32_t));
        qsort(dst, (size_t)l, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t t = 0; t < l; t++)
            if (u == 0 || dst[t] != dst[u - 1]) dst[u++] = dst[t];
        if (u == 0) { free(off1); free(mem1); return ORC_E_EMPTY_EDGE; }
        off1[x + 1] = off1[x] + u;
    }

    /* 2. duplicates: sort hyperedge indices by member list, compare runs */
    int64_t *idx = malloc(sizeof(int64_t) * (m_in ? m_in : 1));
    char *keep = malloc((size_t)(m_in ? m_in : 1));
    if (!idx || !keep) { free(off1); free(mem1); free(idx); free(keep); return ORC_E_OOM; }
    for (int64_t x = 0; x < m_in; x++) { idx[x] = x; keep[x] = 1; }
    g_cmp_off = off1; g_cmp_mem = mem1;
    qsort(idx, (size_t)m_in, sizeof(int64_t), cmp_edge);
    int64_t removed = 0;
    for (int64_t t = 1; t < m_in; t++) {
        if (same_edge(off1, mem1, idx[t - 1], idx[t])) {
            if (!dedupe) { free(off1); free(mem1); free(idx); free(keep); return ORC_E_DUPLICATE_EDGE; }
            keep[idx[t]] = 0;  /* idx[t] > idx[t-1]: a later occurrence */
            removed++;
        }
    }
    free(idx);

    /* 3. renumber survivors 0..m-1 in input order */
    orc_graph *g = calloc(1, sizeof(orc_graph));
    if (!g) { free(off1); free(mem1); free(keep); return ORC_E_OOM; }
    g->n = n;
    g->m = m_in - removed;
    g->removed = removed;
    g->off = malloc(sizeof(int64_t) * (g->m + 1));
    g->orig = malloc(sizeof(int64_t) * (g->m ? g->m : 1));
    g->mem = malloc(sizeof(int32_t) * (off1[m_in] ? off1[m_in] : 1));
    if (!g->off || !g->orig || !g->mem) { free(off1); free(mem1); free(keep); orc_free(g); return ORC_E_OOM; }
    g->off[0] = 0;
    int64_t y = 0;
    for (int64_t x = 0; x < m_in; x++) {
        if (!keep[x]) continue;
        int64_t l = off1[x + 1] - off1[x];
        memcpy(g->mem + g->off[y], mem1 + off1[x], (size_t)l * sizeof(int32_t));
        g->off[y + 1] = g->off[y] + l;
        g->orig[y] = x;
        y++;
    }
    free(off1); free(mem1); free(keep);
    *out = g;
    return ORC_OK;
}

int64_t orc_num_edges(void *h) { return ((orc_graph *)h)->m; }
int64_t orc_nnz(void *h) { orc_graph *g = h; return g->off[g->m]; }
int64_t orc_removed(void *h) { return ((orc_graph *)h)->removed; }
void orc_get_csr(void *h, int64_t *off, int32_t *mem, int64_t *orig) {
    orc_graph *g = h;
    memcpy(off, g->off, sizeof(int64_t) * (g->m + 1));
    memcpy(mem, g->mem, sizeof(int32_t) * g->off[g->m]);
    memcpy(orig, g->orig, sizeof(int64_t) * g->m);
}

static inline int64_t esize(const orc_graph *g, int64_t x) { return g->off[x + 1] - g->off[x]; }

int orc_build_vertex_lists(void *h);

/* Step 1 (Algorithm 2).  E_v lists ascending by hyperedge id; for every e_i
 * the partners j > i with omega_ij, found by counting, for each v in e_i,
 * the hyperedges of E_v after e_i (the same multiset Algorithm 2's merge
 * over the E_v lists walks).  Also the symmetric adjacency N(x).
 *
 * Owners are independent (the paper's Par-adv runs step 1 with threads over
 * hyperedges): a count pass gives each owner's number of partners, a prefix
 * sum their offsets, and a fill pass writes each owner's sorted partners at
 * its offset.  Threads claim owners in chunks; every owner's output depends
 * on that owner alone, so the result is the same for any thread count. */
typedef struct {
    orc_graph *g;
    int pass;                  /* 0: count partners, 1: fill them */
    atomic_llong next;
    atomic_int err;
} wedge_job;

static void *wedge_worker(void *p) {
    wedge_job *job = p;
    orc_graph *g = job->g;
    int64_t m = g->m;
    int32_t *cnt = calloc((size_t)(m ? m : 1), sizeof(int32_t));
    int32_t *touched = malloc(sizeof(int32_t) * (m ? m : 1));
    if (!cnt || !touched) { free(cnt); free(touched); atomic_store(&job->err, ORC_E_OOM); return NULL; }
    const int64_t chunk = 256;
    for (;;) {
        int64_t i0 = atomic_fetch_add(&job->next, chunk);
        if (i0 >= m) break;
        int64_t i1 = i0 + chunk < m ? i0 + chunk : m;
        for (int64_t i = i0; i < i1; i++) {
            int64_t nt = 0;
            for (int64_t t = g->off[i]; t < g->off[i + 1]; t++) {
                int32_t v = g->mem[t];
                for (int64_t r = g->vptr[v]; r < g->vptr[v + 1]; r++) {
                    int32_t j = g->vadj[r];
                    if (j <= i) continue;
                    if (cnt[j]++ == 0) touched[nt++] = j;
                }
            }
            if (job->pass == 0) {
                g->wptr[i + 1] = nt;
            } else {
                qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
                int64_t b = g->wptr[i];
                for (int64_t q = 0; q < nt; q++) {
                    g->wj[b + q] = touched[q];
                    g->wom[b + q] = cnt[touched[q]];
                }
            }
            for (int64_t q = 0; q < nt; q++) cnt[touched[q]] = 0;
        }
    }
    free(cnt); free(touched);
    return NULL;
}

static int run_wedge_pass(orc_graph *g, int pass, int nthreads) {
    wedge_job job;
    job.g = g;
    job.pass = pass;
    atomic_init(&job.next, 0);
    atomic_init(&job.err, ORC_OK);
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    if (!th) return ORC_E_OOM;
    for (int q = 0; q < nthreads; q++) pthread_create(&th[q], NULL, wedge_worker, &job);
    for (int q = 0; q < nthreads; q++) pthread_join(th[q], NULL);
    free(th);
    return atomic_load(&job.err);
}

int orc_build_wedges_threads(void *h, int nthreads) {
    orc_graph *g = h;
    if (g->have_wedges) return ORC_OK;
    if (nthreads < 1) nthreads = 1;
    int64_t m = g->m;
    int rc0 = orc_build_vertex_lists(h);
    if (rc0 != ORC_OK) return rc0;

    g->wptr = calloc((size_t)m + 1, sizeof(int64_t));
    if (!g->wptr) return ORC_E_OOM;
    int rc = run_wedge_pass(g, 0, nthreads);
    if (rc != ORC_OK) return rc;
    for (int64_t i = 0; i < m; i++) g->wptr[i + 1] += g->wptr[i];
    g->nw = g->wptr[m];
    g->wj = malloc(sizeof(int32_t) * (g->nw ? g->nw : 1));
    g->wom = malloc(sizeof(int32_t) * (g->nw ? g->nw : 1));
    if (!g->wj || !g->wom) return ORC_E_OOM;
    rc = run_wedge_pass(g, 1, nthreads);
    if (rc != ORC_OK) return rc;

    /* types (Def. 2.3, Algorithm 2's final test) */
    g->n_incl = g->n_inter = 0;
    for (int64_t i = 0; i < m; i++)
        for (int64_t q = g->wptr[i]; q < g->wptr[i + 1]; q++) {
            int64_t j = g->wj[q];
            int64_t mn = esize(g, i) < esize(g, j) ? esize(g, i) : esize(g, j);
            if (g->wom[q] == mn) g->n_incl++; else g->n_inter++;
        }

    /* symmetric adjacency: appending in wedge order keeps each list sorted */
    g->nptr = calloc((size_t)m + 1, sizeof(int64_t));
    g->nadj = malloc(sizeof(int32_t) * (g->nw > 0 ? 2 * g->nw : 1));
    g->nom = malloc(sizeof(int32_t) * (g->nw > 0 ? 2 * g->nw : 1));
    int64_t *nf = malloc(sizeof(int64_t) * (m ? m : 1));
    if (!g->nptr || !g->nadj || !g->nom || !nf) { free(nf); return ORC_E_OOM; }
    for (int64_t i = 0; i < m; i++)
        for (int64_t q = g->wptr[i]; q < g->wptr[i + 1]; q++) {
            g->nptr[i + 1]++;
            g->nptr[g->wj[q] + 1]++;
        }
    for (int64_t x = 0; x < m; x++) g->nptr[x + 1] += g->nptr[x];
    memcpy(nf, g->nptr, sizeof(int64_t) * m);
    for (int64_t i = 0; i < m; i++)
        for (int64_t q = g->wptr[i]; q < g->wptr[i + 1]; q++) {
            int32_t j = g->wj[q];
            g->nadj[nf[i]] = j; g->nom[nf[i]++] = g->wom[q];
            g->nadj[nf[j]] = (int32_t)i; g->nom[nf[j]++] = g->wom[q];
        }
    free(nf);
    g->have_wedges = 1;
    return ORC_OK;
}

int orc_build_wedges(void *h) { return orc_build_wedges_threads(h, 1); }

int64_t orc_num_wedges(void *h) { return ((orc_graph *)h)->nw; }

/* summary: [0]=|wedges| [1]=|intersection| [2]=|inclusion| [3]=W=sum_x C(deg_x,2)
 *          [4]=max omega [5]=m */
void orc_summary(void *h, int64_t out[6]) {
    orc_graph *g = h;
    int64_t W = 0, mx = 0;
    for (int64_t x = 0; x < g->m; x++) {
        int64_t d = g->nptr[x + 1] - g->nptr[x];
        W += d * (d - 1) / 2;
    }
    for (int64_t q = 0; q < g->nw; q++) if (g->wom[q] > mx) mx = g->wom[q];
    out[0] = g->nw; out[1] = g->n_inter; out[2] = g->n_incl; out[3] = W; out[4] = mx; out[5] = g->m;
}

void orc_get_wedges(void *h, int32_t *wi, int32_t *wj, int32_t *wom) {
    orc_graph *g = h;
    for (int64_t i = 0; i < g->m; i++)
        for (int64_t q = g->wptr[i]; q < g->wptr[i + 1]; q++) {
            wi[q] = (int32_t)i; wj[q] = g->wj[q]; wom[q] = g->wom[q];
        }
}

void orc_get_degrees(void *h, int64_t *deg) {
    orc_graph *g = h;
    for (int64_t x = 0; x < g->m; x++) deg[x] = g->nptr[x + 1] - g->nptr[x];
}

/* |e_i & e_j & e_k| by a three-way merge of sorted member lists */
static int64_t triple_common(const orc_graph *g, int64_t i, int64_t j, int64_t k) {
    const int32_t *a = g->mem + g->off[i], *ae = g->mem + g->off[i + 1];
    const int32_t *b = g->mem + g->off[j], *be = g->mem + g->off[j + 1];
    const int32_t *c = g->mem + g->off[k], *ce = g->mem + g->off[k + 1];
    int64_t r = 0;
    while (a < ae && b < be && c < ce) {
        if (*a == *b && *b == *c) { r++; a++; b++; c++; continue; }
        int32_t mx = *a;
        if (*b > mx) mx = *b;
        if (*c > mx) mx = *c;
        if (*a < mx) a++;
        if (*b < mx) b++;
        if (*c < mx) c++;
    }
    return r;
}

/* Pattern of the hyper-triangle {e_i, e_j, e_k} from the sizes and the
 * pairwise / triple common-vertex counts. */
static int classify(int64_t si, int64_t sj, int64_t sk, int64_t wij, int64_t wik,
                    int64_t wjk, int64_t g) {
    /* inclusion hyperwedges: omega equals the smaller size (Def. 2.3) */
    int cij = wij == (si < sj ? si : sj);
    int cik = wik == (si < sk ? si : sk);
    int cjk = wjk == (sj < sk ? sj : sk);
    int nc = cij + cik + cjk;
    if (nc == 3) return 1;                           /* CCC: a chain */
    if (nc == 2) {
        /* TCC: x is the hyperedge in both inclusion hyperwedges, y and z
         * form the intersection hyperwedge */
        int64_t sx, wxy, wxz, wyz;
        if (!cjk) { sx = si; wxy = wij; wxz = wik; wyz = wjk; }
        else if (!cik) { sx = sj; wxy = wij; wxz = wjk; wyz = wik; }
        else { sx = sk; wxy = wik; wxz = wjk; wyz = wij; }
        if (wxy == sx) {
            /* x lies inside both y and z (Count-TCC, first inner loop) */
            return wyz > sx ? 3 : 2;
        }
        /* x contains both y and z (second inner loop): x = y u z exactly? */
        return (wxy + wxz - wyz == sx) ? 4 : 5;
    }
    if (nc == 1) {
        /* TTC: the inclusion hyperwedge holds the larger L and the smaller S
         * (S inside L); X is the third hyperedge (Count-TTC). */
        int64_t sL, wLS, wLX, wSX;
        if (cij) {
            if (si > sj) { sL = si; wLS = wij; wLX = wik; wSX = wjk; }
            else { sL = sj; wLS = wij; wLX = wjk; wSX = wik; }
        } else if (cik) {
            if (si > sk) { sL = si; wLS = wik; wLX = wij; wSX = wjk; }
            else { sL = sk; wLS = wik; wLX = wjk; wSX = wij; }
        } else {
            if (sj > sk) { sL = sj; wLS = wjk; wLX = wij; wSX = wik; }
            else { sL = sk; wLS = wjk; wLX = wik; wSX = wij; }
        }
        if (wLX == wSX) return 6;
        if (wLS + wLX - wSX == sL) return 7;
        return 8;
    }
    /* TTT: regions by inclusion-exclusion */
    int64_t a = si - wij - wik + g, b = sj - wij - wjk + g, c = sk - wik - wjk + g;
    int64_t d = wij - g, e = wjk - g, f = wik - g;
    int s = (a > 0) + (b > 0) + (c > 0);            /* non-empty private regions */
    int q = (d > 0) + (e > 0) + (f > 0);            /* non-empty pair regions */
    if (g == 0) return 17 + s;                       /* SparseTTT */
    /* DenseTTT, numbered by (q, s) ascending */
    if (q == 0) return 9;                            /* s == 3 */
    if (q == 1) return 10;                           /* s == 3 */
    if (q == 2) return s == 2 ? 11 : 12;
    return 13 + s;                                   /* q == 3 */
}

int orc_classify(int64_t si, int64_t sj, int64_t sk, int64_t wij, int64_t wik, int64_t wjk,
                 int64_t g) {
    return classify(si, sj, sk, wij, wik, wjk, g);
}

/* ---------------------------------------------------------------- step 2 */

typedef struct {
    orc_graph *g;
    atomic_llong next;
    atomic_int err;
    int64_t end;               /* owners [next at start, end) are counted */
    int nthreads;
    uint32_t edge_mask;        /* bit p: count pattern p into per-edge counts */
    int64_t *H;                /* nthreads x 21 */
    int64_t *t;                /* nthreads x m, or NULL */
    int32_t *cw;               /* per-wedge forward closure count, or NULL */
} count_job;

typedef struct { count_job *job; int tid; } count_arg;

/* the sorted common vertices of e_i and e_j (Omega_ij of Def. 2.2) */
static int64_t common_vertices(const orc_graph *g, int64_t i, int64_t j, int32_t *out) {
    const int32_t *a = g->mem + g->off[i], *ae = g->mem + g->off[i + 1];
    const int32_t *b = g->mem + g->off[j], *be = g->mem + g->off[j + 1];
    int64_t n = 0;
    while (a < ae && b < be) {
        if (*a < *b) a++;
        else if (*b < *a) b++;
        else { out[n++] = *a; a++; b++; }
    }
    return n;
}

/* |Omega & e_k| for a sorted vertex list Omega, by a merge with e_k; with
 * Omega = e_i & e_j this is g = |e_i & e_j & e_k| */
static int64_t common_with(const orc_graph *g, const int32_t *om, int64_t n, int64_t k) {
    const int32_t *c = g->mem + g->off[k], *ce = g->mem + g->off[k + 1];
    int64_t q = 0, r = 0;
    while (q < n && c < ce) {
        if (om[q] < *c) q++;
        else if (*c < om[q]) c++;
        else { r++; q++; c++; }
    }
    return r;
}

static void *count_worker(void *p) {
    count_arg *arg = p;
    count_job *job = arg->job;
    orc_graph *g = job->g;
    int64_t *H = job->H + 21 * arg->tid;
    int64_t *t = job->t ? job->t + g->m * arg->tid : NULL;
    int64_t maxs = 1;
    for (int64_t x = 0; x < g->m; x++) if (esize(g, x) > maxs) maxs = esize(g, x);
    int32_t *om = malloc(sizeof(int32_t) * (size_t)maxs);
    if (!om) { atomic_store(&job->err, ORC_E_OOM); return NULL; }
    const int64_t chunk = 64;
    for (;;) {
        int64_t i0 = atomic_fetch_add(&job->next, chunk);
        if (i0 >= job->end) break;
        int64_t i1 = i0 + chunk < job->end ? i0 + chunk : job->end;
        for (int64_t i = i0; i < i1; i++) {
            int64_t si = esize(g, i);
            for (int64_t q = g->wptr[i]; q < g->wptr[i + 1]; q++) {
                int64_t j = g->wj[q], wij = g->wom[q], sj = esize(g, j);
                int32_t closed = 0;
                int64_t nom = common_vertices(g, i, j, om);   /* Omega_ij, nom == wij */
                /* merge N(i) and N(j), keeping k > j */
                int64_t a = g->nptr[i], ae = g->nptr[i + 1];
                int64_t b = g->nptr[j], be = g->nptr[j + 1];
                while (a < ae && g->nadj[a] <= j) a++;
                while (b < be && g->nadj[b] <= j) b++;
                while (a < ae && b < be) {
                    if (g->nadj[a] < g->nadj[b]) { a++; continue; }
                    if (g->nadj[a] > g->nadj[b]) { b++; continue; }
                    int64_t k = g->nadj[a];
                    int64_t wik = g->nom[a], wjk = g->nom[b];
                    int64_t gg = common_with(g, om, nom, k);
                    int p = classify(si, sj, esize(g, k), wij, wik, wjk, gg);
                    H[p]++;
                    closed++;
                    if (t && ((job->edge_mask >> p) & 1u)) { t[i]++; t[j]++; t[k]++; }
                    a++; b++;
                }
                if (job->cw) job->cw[q] = closed;
            }
        }
    }
    free(om);
    return NULL;
}

/* The count below restricted to the owners i in [i0, i1): every hyper-
 * triangle whose smallest id lies in the range, counted exactly as the full
 * count does.  Summing the results over ranges that tile [0, m) gives the
 * full count's H and t (each triangle is met at its smallest id only). */
int orc_count_range(void *h, int64_t i0, int64_t i1, int nthreads, uint32_t edge_mask,
                    int64_t H_out[21], int64_t *t_out, int32_t *cw_out) {
    orc_graph *g = h;
    if (!g->have_wedges) return ORC_E_STATE;
    if (i0 < 0 || i1 < i0 || i1 > g->m) return ORC_E_INVALID;
    if (nthreads < 1) nthreads = 1;
    count_job job;
    job.g = g;
    atomic_init(&job.next, i0);
    atomic_init(&job.err, ORC_OK);
    job.end = i1;
    job.nthreads = nthreads;
    job.edge_mask = edge_mask;
    job.H = calloc((size_t)nthreads * 21, sizeof(int64_t));
    job.t = t_out ? calloc((size_t)nthreads * (size_t)(g->m ? g->m : 1), sizeof(int64_t)) : NULL;
    job.cw = cw_out;
    if (!job.H || (t_out && !job.t)) { free(job.H); free(job.t); return ORC_E_OOM; }
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    count_arg *args = malloc(sizeof(count_arg) * nthreads);
    for (int q = 0; q < nthreads; q++) {
        args[q].job = &job; args[q].tid = q;
        pthread_create(&th[q], NULL, count_worker, &args[q]);
    }
    for (int q = 0; q < nthreads; q++) pthread_join(th[q], NULL);
    if (atomic_load(&job.err) != ORC_OK) {
        free(job.H); free(job.t); free(th); free(args);
        return atomic_load(&job.err);
    }
    memset(H_out, 0, 21 * sizeof(int64_t));
    for (int q = 0; q < nthreads; q++)
        for (int p = 1; p <= 20; p++) H_out[p] += job.H[21 * q + p];
    for (int p = 1; p <= 20; p++) H_out[0] += H_out[p];
    if (t_out) {
        memset(t_out, 0, sizeof(int64_t) * g->m);
        for (int q = 0; q < nthreads; q++)
            for (int64_t x = 0; x < g->m; x++) t_out[x] += job.t[g->m * q + x];
    }
    free(job.H); free(job.t); free(th); free(args);
    return ORC_OK;
}

/* Exact count of every pattern.  H[0] = total, H[p] for p = 1..20.
 * t (may be NULL): per-hyperedge count of the triangles whose pattern bit is
 * set in edge_mask.  cw (may be NULL): per-wedge forward closure count in the
 * wedge order of orc_get_wedges. */
int orc_count(void *h, int nthreads, uint32_t edge_mask, int64_t H_out[21], int64_t *t_out,
              int32_t *cw_out) {
    orc_graph *g = h;
    return orc_count_range(h, 0, g->m, nthreads, edge_mask, H_out, t_out, cw_out);
}

/* ------------------------------------------------ on-demand neighbourhoods
 * For graphs too large for orc_build_wedges: only the E_v lists are built,
 * and the neighbourhood N(x) with omega of any single hyperedge is computed
 * on demand by counting over the E_v lists of its vertices (the same
 * counting as step 1, without the j > i restriction). */

int orc_build_vertex_lists(void *h) {
    orc_graph *g = h;
    if (g->vptr) return ORC_OK;
    int64_t n = g->n, m = g->m, nnz = g->off[m];
    g->vptr = calloc((size_t)n + 1, sizeof(int64_t));
    g->vadj = malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (n ? n : 1));
    if (!g->vptr || !g->vadj || !fill) { free(fill); return ORC_E_OOM; }
    for (int64_t t = 0; t < nnz; t++) g->vptr[g->mem[t] + 1]++;
    for (int64_t v = 0; v < n; v++) g->vptr[v + 1] += g->vptr[v];
    memcpy(fill, g->vptr, sizeof(int64_t) * n);
    for (int64_t x = 0; x < m; x++)
        for (int64_t t = g->off[x]; t < g->off[x + 1]; t++)
            g->vadj[fill[g->mem[t]]++] = (int32_t)x;
    free(fill);
    return ORC_OK;
}

typedef struct { int32_t *nb; int32_t *om; int64_t len; } nlist;

/* N(x) sorted by id, with omega; cnt must be a zeroed int32[m] scratch */
static int neighbourhood(const orc_graph *g, int64_t x, int32_t *cnt, nlist *out) {
    int64_t cap = 0;
    for (int64_t t = g->off[x]; t < g->off[x + 1]; t++) {
        int32_t v = g->mem[t];
        cap += g->vptr[v + 1] - g->vptr[v];
    }
    out->nb = malloc(sizeof(int32_t) * (cap ? cap : 1));
    out->om = malloc(sizeof(int32_t) * (cap ? cap : 1));
    if (!out->nb || !out->om) return ORC_E_OOM;
    int64_t nt = 0;
    for (int64_t t = g->off[x]; t < g->off[x + 1]; t++) {
        int32_t v = g->mem[t];
        for (int64_t r = g->vptr[v]; r < g->vptr[v + 1]; r++) {
            int32_t y = g->vadj[r];
            if (y == x) continue;
            if (cnt[y]++ == 0) out->nb[nt++] = y;
        }
    }
    qsort(out->nb, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int64_t q = 0; q < nt; q++) { out->om[q] = cnt[out->nb[q]]; cnt[out->nb[q]] = 0; }
    out->len = nt;
    return ORC_OK;
}

static void nfree(nlist *l) { free(l->nb); free(l->om); l->nb = l->om = NULL; }

/* Per-wedge closure under an arbitrary hyperedge order: rank (int64[m], a
 * permutation; NULL = id order).  For each wedge (i, j) with
 * rank[i] < rank[j], out[w*21 + p] counts the third hyperedges k adjacent to
 * both with rank[k] > rank[j], by pattern; out[w*21] is their total. */
int orc_wedge_closure_ranked(void *h, const int64_t *rank, const int32_t *wi, const int32_t *wj,
                             int64_t nw, int64_t *out) {
    orc_graph *g = h;
    int rc = orc_build_vertex_lists(h);
    if (rc != ORC_OK) return rc;
    int32_t *cnt = calloc((size_t)(g->m ? g->m : 1), sizeof(int32_t));
    if (!cnt) return ORC_E_OOM;
    for (int64_t w = 0; w < nw; w++) {
        int64_t i = wi[w], j = wj[w];
        int64_t *o = out + 21 * w;
        memset(o, 0, 21 * sizeof(int64_t));
        if (i < 0 || j < 0 || i >= g->m || j >= g->m || i == j) { free(cnt); return ORC_E_INVALID; }
        int64_t ri = rank ? rank[i] : i, rj = rank ? rank[j] : j;
        if (ri >= rj) { free(cnt); return ORC_E_INVALID; }
        nlist Ni, Nj;
        if (neighbourhood(g, i, cnt, &Ni) != ORC_OK || neighbourhood(g, j, cnt, &Nj) != ORC_OK) {
            free(cnt); return ORC_E_OOM;
        }
        int64_t wij = -1;
        for (int64_t a = 0; a < Ni.len; a++) if (Ni.nb[a] == j) { wij = Ni.om[a]; break; }
        if (wij < 0) { nfree(&Ni); nfree(&Nj); free(cnt); return ORC_E_INVALID; }
        int64_t a = 0, b = 0;
        while (a < Ni.len && b < Nj.len) {
            if (Ni.nb[a] < Nj.nb[b]) { a++; continue; }
            if (Ni.nb[a] > Nj.nb[b]) { b++; continue; }
            int64_t k = Ni.nb[a];
            int64_t rk = rank ? rank[k] : k;
            if (rk > rj) {
                int p = classify(esize(g, i), esize(g, j), esize(g, k), wij, Ni.om[a], Nj.om[b],
                                 triple_common(g, i, j, k));
                o[p]++;
                o[0]++;
            }
            a++; b++;
        }
        nfree(&Ni); nfree(&Nj);
    }
    free(cnt);
    return ORC_OK;
}

/* Triangles containing each listed hyperedge x, restricted to the patterns
 * of edge_mask: half the sum over y in N(x) of the triangles {x, y, z},
 * z in N(x) & N(y). */
int orc_edge_triangles(void *h, const int32_t *xs, int64_t n, uint32_t edge_mask, int64_t *out) {
    orc_graph *g = h;
    int rc = orc_build_vertex_lists(h);
    if (rc != ORC_OK) return rc;
    int32_t *cnt = calloc((size_t)(g->m ? g->m : 1), sizeof(int32_t));
    if (!cnt) return ORC_E_OOM;
    for (int64_t q = 0; q < n; q++) {
        int64_t x = xs[q];
        if (x < 0 || x >= g->m) { free(cnt); return ORC_E_INVALID; }
        nlist Nx;
        if (neighbourhood(g, x, cnt, &Nx) != ORC_OK) { free(cnt); return ORC_E_OOM; }
        int64_t twice = 0;
        for (int64_t u = 0; u < Nx.len; u++) {
            int64_t y = Nx.nb[u];
            nlist Ny;
            if (neighbourhood(g, y, cnt, &Ny) != ORC_OK) { nfree(&Nx); free(cnt); return ORC_E_OOM; }
            int64_t a = 0, b = 0;
            while (a < Nx.len && b < Ny.len) {
                if (Nx.nb[a] < Ny.nb[b]) { a++; continue; }
                if (Nx.nb[a] > Ny.nb[b]) { b++; continue; }
                int64_t z = Nx.nb[a];
                int p = classify(esize(g, x), esize(g, y), esize(g, z), Nx.om[u], Nx.om[a], Ny.om[b],
                                 triple_common(g, x, y, z));
                if ((edge_mask >> p) & 1u) twice++;
                a++; b++;
            }
            nfree(&Ny);
        }
        out[q] = twice / 2;
        nfree(&Nx);
    }
    free(cnt);
    return ORC_OK;
}

/* Per-wedge closure split by pattern for an arbitrary list of hyperwedges
 * (i, j), i<j: out[w*21 + p] = #{k > j : k adjacent to i and j, pattern p},
 * out[w*21] = their total.  Works one wedge at a time so that sampled
 * wedges of a graph too large for orc_count can be checked. */
int orc_wedge_closure(void *h, const int32_t *wi, const int32_t *wj, int64_t nw, int64_t *out) {
    orc_graph *g = h;
    if (!g->have_wedges) return ORC_E_STATE;
    for (int64_t w = 0; w < nw; w++) {
        int64_t i = wi[w], j = wj[w];
        int64_t *o = out + 21 * w;
        memset(o, 0, 21 * sizeof(int64_t));
        if (i < 0 || j < 0 || i >= g->m || j >= g->m || i >= j) return ORC_E_INVALID;
        /* omega_ij from i's list */
        int64_t wij = -1;
        for (int64_t a = g->nptr[i]; a < g->nptr[i + 1]; a++)
            if (g->nadj[a] == j) { wij = g->nom[a]; break; }
        if (wij < 0) return ORC_E_INVALID;   /* not a hyperwedge */
        int64_t a = g->nptr[i], ae = g->nptr[i + 1], b = g->nptr[j], be = g->nptr[j + 1];
        while (a < ae && g->nadj[a] <= j) a++;
        while (b < be && g->nadj[b] <= j) b++;
        while (a < ae && b < be) {
            if (g->nadj[a] < g->nadj[b]) { a++; continue; }
            if (g->nadj[a] > g->nadj[b]) { b++; continue; }
            int64_t k = g->nadj[a];
            int p = classify(esize(g, i), esize(g, j), esize(g, k), wij, g->nom[a], g->nom[b],
                             triple_common(g, i, j, k));
            o[p]++;
            o[0]++;
            a++; b++;
        }
    }
    return ORC_OK;
}

/* The plain two-step count restricted to a list of owners, from the E_v
 * lists alone (neighbourhoods built on demand, step 1 per owner and per
 * partner): for each listed owner i, every hyperwedge (i, j), j > i, is
 * closed by the k > j adjacent to both.  Used to time the oracle on a
 * bounded sample of a large workload.  H_out[21] and the number of
 * hyperwedges closed (*nwedges) cover the listed owners only. */
typedef struct {
    orc_graph *g;
    const int32_t *owners;
    int64_t n;
    atomic_llong next;
    int64_t *H;        /* nthreads x 21 */
    int64_t *nw;       /* nthreads */
    atomic_int err;
} sample_job;

typedef struct { sample_job *job; int tid; } sample_arg;

static void *sample_worker(void *p) {
    sample_arg *arg = p;
    sample_job *job = arg->job;
    orc_graph *g = job->g;
    int64_t *H = job->H + 21 * arg->tid;
    int32_t *cnt = calloc((size_t)(g->m ? g->m : 1), sizeof(int32_t));
    if (!cnt) { atomic_store(&job->err, ORC_E_OOM); return NULL; }
    for (;;) {
        int64_t q = atomic_fetch_add(&job->next, 1);
        if (q >= job->n) break;
        int64_t i = job->owners[q];
        nlist Ni;
        if (neighbourhood(g, i, cnt, &Ni) != ORC_OK) { atomic_store(&job->err, ORC_E_OOM); break; }
        for (int64_t u = 0; u < Ni.len; u++) {
            int64_t j = Ni.nb[u];
            if (j <= i) continue;
            job->nw[arg->tid]++;
            nlist Nj;
            if (neighbourhood(g, j, cnt, &Nj) != ORC_OK) { atomic_store(&job->err, ORC_E_OOM); break; }
            int64_t a = u + 1, b = 0;
            while (b < Nj.len && Nj.nb[b] <= j) b++;
            while (a < Ni.len && b < Nj.len) {
                if (Ni.nb[a] < Nj.nb[b]) { a++; continue; }
                if (Ni.nb[a] > Nj.nb[b]) { b++; continue; }
                int64_t k = Ni.nb[a];
                int p = classify(esize(g, i), esize(g, j), esize(g, k), Ni.om[u], Ni.om[a], Nj.om[b],
                                 triple_common(g, i, j, k));
                H[p]++;
                a++; b++;
            }
            nfree(&Nj);
        }
        nfree(&Ni);
    }
    free(cnt);
    return NULL;
}

int orc_count_owner_sample(void *h, const int32_t *owners, int64_t n, int nthreads, int64_t H_out[21],
                           int64_t *nwedges) {
    orc_graph *g = h;
    int rc = orc_build_vertex_lists(h);
    if (rc != ORC_OK) return rc;
    if (nthreads < 1) nthreads = 1;
    for (int64_t q = 0; q < n; q++)
        if (owners[q] < 0 || owners[q] >= g->m) return ORC_E_INVALID;
    sample_job job;
    job.g = g; job.owners = owners; job.n = n;
    atomic_init(&job.next, 0);
    atomic_init(&job.err, ORC_OK);
    job.H = calloc((size_t)nthreads * 21, sizeof(int64_t));
    job.nw = calloc((size_t)nthreads, sizeof(int64_t));
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    sample_arg *args = malloc(sizeof(sample_arg) * nthreads);
    if (!job.H || !job.nw || !th || !args) { free(job.H); free(job.nw); free(th); free(args); return ORC_E_OOM; }
    for (int t = 0; t < nthreads; t++) {
        args[t].job = &job; args[t].tid = t;
        pthread_create(&th[t], NULL, sample_worker, &args[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    memset(H_out, 0, 21 * sizeof(int64_t));
    *nwedges = 0;
    for (int t = 0; t < nthreads; t++) {
        for (int p = 1; p <= 20; p++) H_out[p] += job.H[21 * t + p];
        *nwedges += job.nw[t];
    }
    for (int p = 1; p <= 20; p++) H_out[0] += H_out[p];
    rc = atomic_load(&job.err);
    free(job.H); free(job.nw); free(th); free(args);
    return rc;
}
