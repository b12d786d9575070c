/*
 * CPU oracle for balanced-butterfly counting in a signed bipartite graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no code, header or table with the HIP library.
 *
 * What is computed (paper: Section 2, Problem Definition):
 *   * a butterfly is a 4-cycle u1-v1-u2-v2 with u1 != u2 in U, v1 != v2 in V and
 *     all four edges present (Definition 1);
 *   * it is balanced when it holds an even number of negative edges
 *     (Definition 2), i.e. when the product of its four signs is +1;
 *   * the answer is the number of balanced butterflies (problem statement).
 *
 * Functions (all plain loops, deliberately unoptimised):
 *   bbo_brute_force  O0: every pair {u1,u2} x every pair {v1,v2}, on a dense
 *                    sign matrix; the definition read literally.
 *   bbo_pairs        O1: for every same-side pair {x,z} the common neighbours y
 *                    carry t_y = sign(x,y) * sign(z,y); a butterfly on {x,z}
 *                    with middles {y1,y2} is balanced iff t_y1 == t_y2 (the
 *                    product of its four signs is t_y1 * t_y2).  So the pair
 *                    holds C(l,2) + C(m,2) balanced and l*m unbalanced
 *                    butterflies, l = #{t=+1}, m = #{t=-1} (the counting fact
 *                    behind Lemma 2 of Section 4).  Every butterfly has exactly
 *                    one U pair and one V pair, so side U and side V must agree.
 *   bbo_per_vertex   c_x = number of balanced butterflies containing x: the same
 *                    pair sums without the z > x restriction (Section 5.1, the
 *                    per-vertex count; the end vertex z is taken != x).
 *   bbo_wedges       W = number of wedges (u,v,w) with p(v) < p(u) and
 *                    p(w) < p(u) under the vertex priority of Definition 4
 *                    (degree, then id; ids are global: U first, then V) -- the
 *                    number of innermost iterations of the bucket algorithm
 *                    (Algorithm 2, Section 4.1).
 *   bbo_bucket       the bucket method itself (Algorithm 2 in the paper's
 *                    order, starts in parallel as in Algorithm 4): balanced,
 *                    unbalanced and W; a third route to the same totals.
 *
 * Every function validates its input like the library must: ids in range, sign
 * in {+1,-1}, no (u,v) pair twice (E is a set of pairs, Section 2).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum {
    BBO_OK = 0,
    BBO_ERR_INVALID_ARG = -1,
    BBO_ERR_VERTEX_RANGE = -2,
    BBO_ERR_BAD_SIGN = -3,
    BBO_ERR_DUPLICATE_EDGE = -4,
    BBO_ERR_OVERFLOW = -6,
    BBO_ERR_OUT_OF_MEMORY = -7,
};

/* ------------------------------------------------------------------------ */
/* Input checks and adjacency lists (by vertex id, unsorted).                 */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int check_input(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu,
                       const int32_t* ev, const int8_t* sg) {
    if (n_u < 0 || n_v < 0 || m < 0) return BBO_ERR_INVALID_ARG;
    if (m > 0 && (!eu || !ev || !sg)) return BBO_ERR_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i) {
        if (eu[i] < 0 || eu[i] >= n_u || ev[i] < 0 || ev[i] >= n_v) return BBO_ERR_VERTEX_RANGE;
        if (sg[i] != 1 && sg[i] != -1) return BBO_ERR_BAD_SIGN;
    }
    if (m > 1) {
        uint64_t* keys = (uint64_t*)malloc((size_t)m * sizeof(uint64_t));
        if (!keys) return BBO_ERR_OUT_OF_MEMORY;
        for (int64_t i = 0; i < m; ++i) keys[i] = (uint64_t)eu[i] * (uint64_t)n_v + (uint64_t)ev[i];
        qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);
        int dup = 0;
        for (int64_t i = 1; i < m && !dup; ++i) dup = keys[i] == keys[i - 1];
        free(keys);
        if (dup) return BBO_ERR_DUPLICATE_EDGE;
    }
    return BBO_OK;
}

/* Adjacency of one side: for vertex x, entries nbr[off[x] .. off[x+1]) with signs. */
typedef struct {
    int64_t* off;
    int32_t* nbr;
    int8_t* sgn;
} adj_t;

static void adj_free(adj_t* a) {
    free(a->off);
    free(a->nbr);
    free(a->sgn);
}

/* from_u != 0: rows are U vertices, neighbours are V ids; else the reverse. */
static int adj_build(adj_t* a, int32_t n_rows, int64_t m, const int32_t* eu, const int32_t* ev,
                     const int8_t* sg, int from_u) {
    a->off = (int64_t*)calloc((size_t)n_rows + 1, sizeof(int64_t));
    a->nbr = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    a->sgn = (int8_t*)malloc((size_t)(m > 0 ? m : 1));
    int64_t* fill = (int64_t*)calloc((size_t)n_rows + 1, sizeof(int64_t));
    if (!a->off || !a->nbr || !a->sgn || !fill) {
        free(fill);
        adj_free(a);
        return BBO_ERR_OUT_OF_MEMORY;
    }
    for (int64_t i = 0; i < m; ++i) a->off[(from_u ? eu[i] : ev[i]) + 1]++;
    for (int32_t x = 0; x < n_rows; ++x) a->off[x + 1] += a->off[x];
    for (int64_t i = 0; i < m; ++i) {
        int32_t r = from_u ? eu[i] : ev[i];
        int64_t at = a->off[r] + fill[r]++;
        a->nbr[at] = from_u ? ev[i] : eu[i];
        a->sgn[at] = sg[i];
    }
    free(fill);
    return BBO_OK;
}

static uint64_t choose2(uint64_t k) { return k < 2 ? 0 : k * (k - 1) / 2; }

/* ------------------------------------------------------------------------ */
/* O0: brute force over all pairs of pairs (Definitions 1 and 2).            */

int bbo_brute_force(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                    const int8_t* sg, uint64_t* out_balanced, uint64_t* out_total) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    if ((int64_t)n_u * (int64_t)n_v > (int64_t)1 << 26) return BBO_ERR_INVALID_ARG;
    int8_t* s = (int8_t*)calloc((size_t)n_u * (size_t)n_v + 1, 1);
    if (!s) return BBO_ERR_OUT_OF_MEMORY;
    for (int64_t i = 0; i < m; ++i) s[(size_t)eu[i] * n_v + ev[i]] = sg[i];
    uint64_t bal = 0, tot = 0;
    for (int32_t u1 = 0; u1 < n_u; ++u1)
        for (int32_t u2 = u1 + 1; u2 < n_u; ++u2)
            for (int32_t v1 = 0; v1 < n_v; ++v1)
                for (int32_t v2 = v1 + 1; v2 < n_v; ++v2) {
                    int a = s[(size_t)u1 * n_v + v1], b = s[(size_t)u1 * n_v + v2];
                    int c = s[(size_t)u2 * n_v + v1], d = s[(size_t)u2 * n_v + v2];
                    if (a == 0 || b == 0 || c == 0 || d == 0) continue; /* not a butterfly */
                    tot++;
                    if (a * b * c * d > 0) bal++; /* even number of negative edges */
                }
    free(s);
    *out_balanced = bal;
    *out_total = tot;
    return BBO_OK;
}

/* ------------------------------------------------------------------------ */
/* O1 and the per-vertex count: same-side pairs and their common neighbours. */

typedef struct {
    const adj_t* ax; /* rows: side X, neighbours in Y */
    const adj_t* ay; /* rows: side Y, neighbours in X */
    int32_t nx;
    int32_t x0, x1;     /* this thread's rows of X */
    int all_partners;   /* 0: only partners z > x (each pair once); 1: every z != x */
    u128 bal, unb;      /* totals over this thread's pairs (all_partners == 0) */
    uint64_t* per_x;    /* all_partners == 1: balanced butterflies containing x */
    int err;
} pair_job;

static void* pair_worker(void* arg) {
    pair_job* j = (pair_job*)arg;
    uint32_t* same = (uint32_t*)calloc((size_t)j->nx + 1, sizeof(uint32_t));
    uint32_t* opp = (uint32_t*)calloc((size_t)j->nx + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(((size_t)j->nx + 1) * sizeof(int32_t));
    if (!same || !opp || !touched) {
        j->err = BBO_ERR_OUT_OF_MEMORY;
        free(same);
        free(opp);
        free(touched);
        return NULL;
    }
    for (int32_t x = j->x0; x < j->x1; ++x) {
        int32_t nt = 0;
        for (int64_t e = j->ax->off[x]; e < j->ax->off[x + 1]; ++e) {
            int32_t y = j->ax->nbr[e];
            int s1 = j->ax->sgn[e];
            for (int64_t f = j->ay->off[y]; f < j->ay->off[y + 1]; ++f) {
                int32_t z = j->ay->nbr[f];
                if (z == x) continue;
                if (!j->all_partners && z < x) continue;
                if (same[z] == 0 && opp[z] == 0) touched[nt++] = z;
                if (s1 * j->ay->sgn[f] > 0)
                    same[z]++; /* t_y = +1 */
                else
                    opp[z]++; /* t_y = -1 */
            }
        }
        u128 bx = 0;
        for (int32_t i = 0; i < nt; ++i) {
            int32_t z = touched[i];
            bx += (u128)choose2(same[z]) + (u128)choose2(opp[z]);
            j->unb += (u128)same[z] * (u128)opp[z];
            same[z] = 0;
            opp[z] = 0;
        }
        if (j->all_partners)
            j->per_x[x] = (uint64_t)bx;
        else
            j->bal += bx;
    }
    free(same);
    free(opp);
    free(touched);
    return NULL;
}

static int run_pairs(const adj_t* ax, const adj_t* ay, int32_t nx, int nthreads, int all_partners,
                     u128* bal, u128* unb, uint64_t* per_x) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pair_job jobs[256];
    pthread_t th[256];
    /* Each thread takes one contiguous block of rows. */
    int32_t per = nx / nthreads + 1;
    for (int t = 0; t < nthreads; ++t) {
        int64_t a = (int64_t)t * per, b = (int64_t)(t + 1) * per;
        jobs[t] = (pair_job){ax, ay, nx, (int32_t)(a > nx ? nx : a), (int32_t)(b > nx ? nx : b),
                             all_partners, 0, 0, per_x, 0};
        pthread_create(&th[t], NULL, pair_worker, &jobs[t]);
    }
    int err = 0;
    *bal = 0;
    *unb = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].err) err = jobs[t].err;
        *bal += jobs[t].bal;
        *unb += jobs[t].unb;
    }
    return err;
}

/* Pairs on one side (side 0: pairs of U vertices, side 1: pairs of V
 * vertices).  out[0] = balanced, out[1] = unbalanced butterflies. */
int bbo_pairs(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
              const int8_t* sg, int side, int nthreads, uint64_t* out) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    adj_t au, av;
    if ((rc = adj_build(&au, n_u, m, eu, ev, sg, 1))) return rc;
    if ((rc = adj_build(&av, n_v, m, eu, ev, sg, 0))) {
        adj_free(&au);
        return rc;
    }
    u128 bal, unb;
    if (side == 0)
        rc = run_pairs(&au, &av, n_u, nthreads, 0, &bal, &unb, NULL);
    else
        rc = run_pairs(&av, &au, n_v, nthreads, 0, &bal, &unb, NULL);
    adj_free(&au);
    adj_free(&av);
    if (rc) return rc;
    if ((bal >> 64) || (unb >> 64)) return BBO_ERR_OVERFLOW;
    out[0] = (uint64_t)bal;
    out[1] = (uint64_t)unb;
    return BBO_OK;
}

/* Same as bbo_pairs but for a subset of the rows of side X only: rows
 * [x0, x1) each summed over their partners z > x, split over nthreads threads.
 * Summing the results of consecutive row blocks that cover the whole side
 * gives bbo_pairs.  Used to time a bounded sample of the full computation. */
int bbo_pairs_rows(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                   const int8_t* sg, int side, int32_t x0, int32_t x1, int nthreads,
                   uint64_t* out) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    adj_t au, av;
    if ((rc = adj_build(&au, n_u, m, eu, ev, sg, 1))) return rc;
    if ((rc = adj_build(&av, n_v, m, eu, ev, sg, 0))) {
        adj_free(&au);
        return rc;
    }
    int32_t nx = side == 0 ? n_u : n_v;
    if (x0 < 0) x0 = 0;
    if (x1 > nx) x1 = nx;
    if (x1 < x0) x1 = x0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pair_job jobs[256];
    pthread_t th[256];
    int32_t per = (x1 - x0) / nthreads + 1;
    for (int t = 0; t < nthreads; ++t) {
        int64_t a = (int64_t)x0 + (int64_t)t * per, b = a + per;
        jobs[t] = (pair_job){side == 0 ? &au : &av, side == 0 ? &av : &au, nx,
                             (int32_t)(a > x1 ? x1 : a), (int32_t)(b > x1 ? x1 : b), 0, 0, 0, NULL, 0};
        pthread_create(&th[t], NULL, pair_worker, &jobs[t]);
    }
    u128 bal = 0, unb = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].err) rc = jobs[t].err;
        bal += jobs[t].bal;
        unb += jobs[t].unb;
    }
    adj_free(&au);
    adj_free(&av);
    if (rc) return rc;
    if ((bal >> 64) || (unb >> 64)) return BBO_ERR_OVERFLOW;
    out[0] = (uint64_t)bal;
    out[1] = (uint64_t)unb;
    return BBO_OK;
}

/* Balanced butterflies containing each vertex: out[0 .. n_u) for U, then
 * out[n_u .. n_u + n_v) for V. */
int bbo_per_vertex(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
                   const int8_t* sg, int nthreads, uint64_t* out) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    adj_t au, av;
    if ((rc = adj_build(&au, n_u, m, eu, ev, sg, 1))) return rc;
    if ((rc = adj_build(&av, n_v, m, eu, ev, sg, 0))) {
        adj_free(&au);
        return rc;
    }
    u128 bal, unb;
    rc = run_pairs(&au, &av, n_u, nthreads, 1, &bal, &unb, out);
    if (!rc) rc = run_pairs(&av, &au, n_v, nthreads, 1, &bal, &unb, out + n_u);
    adj_free(&au);
    adj_free(&av);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* W: wedges kept by the vertex-priority filter (Definition 4, Algorithm 2).  */

typedef struct {
    const int64_t* off; /* global adjacency: ids 0..n_u-1 are U, n_u.. are V */
    const int32_t* nbr;
    const int64_t* deg;
    int32_t g0, g1;
    uint64_t w;
} wedge_job;

/* p(a) < p(b): lower degree, or equal degree and lower id (Definition 4). */
static int prio_less(const int64_t* deg, int32_t a, int32_t b) {
    return deg[a] < deg[b] || (deg[a] == deg[b] && a < b);
}

static void* wedge_worker(void* arg) {
    wedge_job* j = (wedge_job*)arg;
    uint64_t w = 0;
    for (int32_t u = j->g0; u < j->g1; ++u)
        for (int64_t e = j->off[u]; e < j->off[u + 1]; ++e) {
            int32_t v = j->nbr[e];
            if (!prio_less(j->deg, v, u)) continue;
            for (int64_t f = j->off[v]; f < j->off[v + 1]; ++f)
                if (prio_less(j->deg, j->nbr[f], u)) w++;
        }
    j->w = w;
    return NULL;
}

int bbo_wedges(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
               const int8_t* sg, int nthreads, uint64_t* out_w) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    int32_t n = n_u + n_v;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* nbr = (int32_t*)malloc((size_t)(2 * m + 1) * sizeof(int32_t));
    if (!off || !deg || !fill || !nbr) {
        free(off);
        free(deg);
        free(fill);
        free(nbr);
        return BBO_ERR_OUT_OF_MEMORY;
    }
    for (int64_t i = 0; i < m; ++i) {
        deg[eu[i]]++;
        deg[n_u + ev[i]]++;
    }
    for (int32_t x = 0; x < n; ++x) off[x + 1] = off[x] + deg[x];
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = eu[i], b = n_u + ev[i];
        nbr[off[a] + fill[a]++] = b;
        nbr[off[b] + fill[b]++] = a;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    wedge_job jobs[256];
    pthread_t th[256];
    int32_t per = n / nthreads + 1;
    uint64_t w = 0;
    for (int t = 0; t < nthreads; ++t) {
        int64_t a = (int64_t)t * per, b = (int64_t)(t + 1) * per;
        jobs[t] = (wedge_job){off, nbr, deg, (int32_t)(a > n ? n : a), (int32_t)(b > n ? n : b), 0};
        pthread_create(&th[t], NULL, wedge_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        w += jobs[t].w;
    }
    free(off);
    free(deg);
    free(fill);
    free(nbr);
    *out_w = w;
    return BBO_OK;
}

/* ------------------------------------------------------------------------ */
/* The bucket method itself on the CPU (Section 4.1, Algorithm 2; run with
 * the parallel loop over start vertices of Section 5.2, Algorithm 4).
 *
 * A third, independent way to the same totals, and the paper's own method
 * timed on host cores.  Steps, in the paper's order:
 *   1. the priority p(x) of every vertex: degree, then global id
 *      (Definition 4; ids are U = 0..n_u-1, V = n_u..n-1);
 *   2. every neighbour list sorted by ascending priority;
 *   3. for every start u: for every neighbour v with p(v) < p(u) (a prefix of
 *      the sorted list), for every neighbour w of v with p(w) < p(u) (a prefix
 *      too), the wedge u-v-w goes to bucket B1[w] when sign(u,v) == sign(v,w)
 *      (symmetric, Definition 5) and to B2[w] otherwise (asymmetric,
 *      Definition 6);
 *   4. then every touched w adds C(B1[w],2) + C(B2[w],2) balanced butterflies
 *      (Lemma 2) and B1[w] * B2[w] unbalanced ones; the buckets are emptied
 *      before the next start (they belong to one start; Algorithm 2 declares
 *      them once, but a bucket shared by two starts would pair wedges with
 *      different ends).
 * out[0] = balanced, out[1] = unbalanced, out[2] = wedges enumerated (W).
 * Threads take starts from a shared counter, a few at a time. */

typedef struct {
    const int64_t* off;  /* neighbour list of x: nbr[off[x] .. off[x+1]), by priority */
    const int32_t* nbr;  /* neighbour ids (global) */
    const int8_t* sgn;
    const int32_t* prio; /* p(x) as a rank: 0 = lowest priority */
    int32_t n;
    int64_t* next;       /* shared: next start to take */
    u128 bal, unb;
    uint64_t w;
    int err;
} bucket_job;

static const int32_t* g_sort_prio; /* comparator context (only set while sorting) */

static int cmp_by_prio(const void* a, const void* b) {
    int32_t x = g_sort_prio[((const int64_t*)a)[0]], y = g_sort_prio[((const int64_t*)b)[0]];
    return x < y ? -1 : (x > y ? 1 : 0);
}

static const int64_t* g_sort_deg;

static int cmp_vertex_prio(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    if (g_sort_deg[x] != g_sort_deg[y]) return g_sort_deg[x] < g_sort_deg[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void* bucket_worker(void* arg) {
    bucket_job* j = (bucket_job*)arg;
    uint32_t* b1 = (uint32_t*)calloc((size_t)j->n + 1, sizeof(uint32_t));
    uint32_t* b2 = (uint32_t*)calloc((size_t)j->n + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(((size_t)j->n + 1) * sizeof(int32_t));
    if (!b1 || !b2 || !touched) {
        j->err = BBO_ERR_OUT_OF_MEMORY;
        free(b1);
        free(b2);
        free(touched);
        return NULL;
    }
    for (;;) {
        int64_t u0 = __atomic_fetch_add(j->next, 16, __ATOMIC_RELAXED);
        if (u0 >= j->n) break;
        int64_t u1 = u0 + 16 > j->n ? j->n : u0 + 16;
        for (int32_t u = (int32_t)u0; u < (int32_t)u1; ++u) {
            const int32_t pu = j->prio[u];
            int32_t nt = 0;
            for (int64_t e = j->off[u]; e < j->off[u + 1]; ++e) {
                const int32_t v = j->nbr[e];
                if (j->prio[v] >= pu) break; /* sorted: the rest rank higher */
                for (int64_t f = j->off[v]; f < j->off[v + 1]; ++f) {
                    const int32_t w = j->nbr[f];
                    if (j->prio[w] >= pu) break;
                    j->w++;
                    if (b1[w] == 0 && b2[w] == 0) touched[nt++] = w;
                    if (j->sgn[e] == j->sgn[f])
                        b1[w]++;
                    else
                        b2[w]++;
                }
            }
            for (int32_t i = 0; i < nt; ++i) {
                const int32_t w = touched[i];
                j->bal += (u128)choose2(b1[w]) + (u128)choose2(b2[w]);
                j->unb += (u128)b1[w] * (u128)b2[w];
                b1[w] = 0;
                b2[w] = 0;
            }
        }
    }
    free(b1);
    free(b2);
    free(touched);
    return NULL;
}

int bbo_bucket(int32_t n_u, int32_t n_v, int64_t m, const int32_t* eu, const int32_t* ev,
               const int8_t* sg, int nthreads, uint64_t* out) {
    int rc = check_input(n_u, n_v, m, eu, ev, sg);
    if (rc) return rc;
    const int32_t n = n_u + n_v;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* byprio = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t* prio = (int32_t*)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t* tmp = (int64_t*)malloc((size_t)(2 * m + 1) * 2 * sizeof(int64_t));
    int32_t* nbr = (int32_t*)malloc((size_t)(2 * m + 1) * sizeof(int32_t));
    int8_t* sgn = (int8_t*)malloc((size_t)(2 * m + 1));
    if (!off || !deg || !fill || !byprio || !prio || !tmp || !nbr || !sgn) {
        rc = BBO_ERR_OUT_OF_MEMORY;
        goto done;
    }
    /* 1. priorities: vertices in ascending (degree, id) order */
    for (int64_t i = 0; i < m; ++i) {
        deg[eu[i]]++;
        deg[n_u + ev[i]]++;
    }
    for (int32_t x = 0; x < n; ++x) byprio[x] = x;
    g_sort_deg = deg;
    qsort(byprio, (size_t)n, sizeof(int32_t), cmp_vertex_prio);
    for (int32_t r = 0; r < n; ++r) prio[byprio[r]] = r;
    /* 2. neighbour lists (global ids), each sorted by ascending priority;
     *    tmp holds (neighbour, edge index) pairs while sorting */
    for (int32_t x = 0; x < n; ++x) off[x + 1] = off[x] + deg[x];
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = eu[i], b = n_u + ev[i];
        int64_t at = off[a] + fill[a]++;
        tmp[2 * at] = b;
        tmp[2 * at + 1] = i;
        at = off[b] + fill[b]++;
        tmp[2 * at] = a;
        tmp[2 * at + 1] = i;
    }
    g_sort_prio = prio;
    for (int32_t x = 0; x < n; ++x)
        qsort(tmp + 2 * off[x], (size_t)(off[x + 1] - off[x]), 2 * sizeof(int64_t), cmp_by_prio);
    for (int64_t k = 0; k < 2 * m; ++k) {
        nbr[k] = (int32_t)tmp[2 * k];
        sgn[k] = sg[tmp[2 * k + 1]];
    }
    /* 3-4. the starts, in parallel */
    {
        if (nthreads < 1) nthreads = 1;
        if (nthreads > 256) nthreads = 256;
        bucket_job jobs[256];
        pthread_t th[256];
        int64_t next = 0;
        for (int t = 0; t < nthreads; ++t) {
            jobs[t] = (bucket_job){off, nbr, sgn, prio, n, &next, 0, 0, 0, 0};
            pthread_create(&th[t], NULL, bucket_worker, &jobs[t]);
        }
        u128 bal = 0, unb = 0;
        uint64_t w = 0;
        for (int t = 0; t < nthreads; ++t) {
            pthread_join(th[t], NULL);
            if (jobs[t].err) rc = jobs[t].err;
            bal += jobs[t].bal;
            unb += jobs[t].unb;
            w += jobs[t].w;
        }
        if (!rc && ((bal >> 64) || (unb >> 64))) rc = BBO_ERR_OVERFLOW;
        if (!rc) {
            out[0] = (uint64_t)bal;
            out[1] = (uint64_t)unb;
            out[2] = w;
        }
    }
done:
    free(off);
    free(deg);
    free(fill);
    free(byprio);
    free(prio);
    free(tmp);
    free(nbr);
    free(sgn);
    return rc;
}
