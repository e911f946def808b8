/*
 * ORACLE -- test infrastructure only.  Not part of the product path: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * A plain, slow, obviously correct CPU definition of what an evolving-graph
 * query computes (Section 2, Section 3 of the paper):
 *
 *   - A snapshot is a SET of (src, dst, w) triples.  Snapshot i is obtained
 *     from snapshot i-1 (snapshot -1 = the base edge set) by applying batch i:
 *     its deletions first, then its additions.  Deleting an absent triple and
 *     adding a present one change nothing.
 *   - values[v][i] = Val_A(snapshot b+i, s, v) for the window [b, b+L), where
 *     Val_A is the best path value of the query over all paths s -> v
 *     (Table 2 edge functions):
 *        SSSP  path value = sum of w (saturating at 0xFFFFFFFE), best = min,
 *              source 0, unreachable 0xFFFFFFFF
 *        BFS   path value = number of edges, best = min, source 0,
 *              unreachable 0xFFFFFFFF
 *        SSWP  path value = min w along the path, best = max,
 *              source 0xFFFFFFFF, unreachable 0
 *        SSNP  path value = max w along the path, best = min, source 0,
 *              unreachable 0xFFFFFFFF
 *        VITERBI  path value = the source's 1.0 divided by each weight along
 *              the path in turn, best = max; values are IEEE single floats
 *              held as their 32-bit patterns (non-negative, so their order is
 *              the integer order): each step divides in double precision and
 *              rounds to single (to nearest even), and a quotient below the
 *              smallest normal single counts as unreachable (0.0)
 *   - The intersection graph of a window holds the triples present in every
 *     snapshot of the window; the union graph those present in any
 *     (Section 3, Step 1).
 *
 * Each snapshot is materialised on its own and solved from scratch by
 * Dijkstra's algorithm (SSSP, SSWP, SSNP, VITERBI: the path values never
 * improve when a path is extended, so settling vertices best-first is exact)
 * or by a FIFO
 * breadth-first search (BFS).  This shares no code with the GPU library.
 */
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

enum { O_SSSP = 0, O_BFS = 1, O_SSWP = 2, O_SSNP = 3, O_VIT = 4 };
#define ONE_F32 0x3F800000u /* 1.0f */
#define INF32 0xFFFFFFFFu
#define SAT32 0xFFFFFFFEu

/* ------------------------------------------------------------------ replay */

typedef struct {
    uint32_t src, dst, w;
    int16_t since;    /* snapshot the current presence started at */
    uint8_t present;
    uint8_t used;     /* 0 = free slot */
    uint64_t bits[2];
} rec_t;

typedef struct { rec_t* r; uint64_t mask; uint64_t n; } tmap;

static uint64_t hash3(uint32_t a, uint32_t b, uint32_t c) {
    uint64_t h = (uint64_t)a * 0x9E3779B97F4A7C15ULL;
    h ^= (uint64_t)b + 0x632BE59BD9B4E019ULL + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ULL;
    h ^= (uint64_t)c + 0x94D049BB133111EBULL + (h << 6) + (h >> 2);
    h ^= h >> 31;
    h *= 0x94D049BB133111EBULL;
    return h ^ (h >> 29);
}

static rec_t* tmap_find(tmap* m, uint32_t s, uint32_t d, uint32_t w, int create) {
    uint64_t i = hash3(s, d, w) & m->mask;
    for (;;) {
        rec_t* r = &m->r[i];
        if (!r->used) {
            if (!create) return NULL;
            r->used = 1; r->src = s; r->dst = d; r->w = w;
            r->present = 0; r->since = 0; r->bits[0] = r->bits[1] = 0;
            m->n++;
            return r;
        }
        if (r->src == s && r->dst == d && r->w == w) return r;
        i = (i + 1) & m->mask;
    }
}

static void set_bits(uint64_t bits[2], int from, int to) {
    for (int t = from; t < to; ++t) bits[t >> 6] |= 1ULL << (t & 63);
}

/* Which of P partitions a triple belongs to (each partition replays alone). */
static uint32_t part_of(uint32_t s, uint32_t d, uint32_t w, uint32_t P) {
    return (uint32_t)(hash3(s, d, w) >> 40) % P;
}

/*
 * Replay the batches.  Inputs are (n, 3) uint32 triples; batch i's deletions
 * are dels[del_off[i] .. del_off[i+1]) and its additions likewise.  Output:
 * every distinct triple ever present, with bit t of its two-word mask set iff
 * the triple is in snapshot t.  Returns the triple count (<= cap) or -1.
 *
 * A triple's presence depends only on its own events, so the triples are
 * split into partitions by hash and each thread replays one partition, in
 * event order, with its own map.
 */
int64_t oracle_replay(uint32_t K, const uint32_t* base, uint64_t n_base,
                      const uint32_t* dels, const uint64_t* del_off,
                      const uint32_t* adds, const uint64_t* add_off,
                      uint32_t* out_trip, uint64_t* out_bits, uint64_t cap) {
    if (K > 128) return -1;
    const uint32_t P = (uint32_t)omp_get_max_threads();
    const uint64_t total = n_base + add_off[K];
    uint64_t* counts = (uint64_t*)calloc(P + 1, sizeof(uint64_t));
    tmap* maps = (tmap*)calloc(P, sizeof(tmap));
    int err = 0;
#pragma omp parallel num_threads(P)
    {
        const uint32_t me = (uint32_t)omp_get_thread_num();
        uint64_t hcap = 16;
        while (hcap < 2 * (total / P + 1) + 16) hcap <<= 1;
        tmap m = {(rec_t*)calloc(hcap, sizeof(rec_t)), hcap - 1, 0};
        if (!m.r) {
#pragma omp atomic write
            err = 1;
        } else {
            for (uint64_t j = 0; j < n_base; ++j) {
                const uint32_t* e = base + 3 * j;
                if (part_of(e[0], e[1], e[2], P) != me) continue;
                rec_t* r = tmap_find(&m, e[0], e[1], e[2], 1);
                if (!r->present) { r->present = 1; r->since = 0; }
            }
            for (uint32_t i = 0; i < K; ++i) {
                for (uint64_t j = del_off[i]; j < del_off[i + 1]; ++j) {
                    const uint32_t* e = dels + 3 * j;
                    if (part_of(e[0], e[1], e[2], P) != me) continue;
                    rec_t* r = tmap_find(&m, e[0], e[1], e[2], 0);
                    if (r && r->present) { set_bits(r->bits, r->since, (int)i); r->present = 0; }
                }
                for (uint64_t j = add_off[i]; j < add_off[i + 1]; ++j) {
                    const uint32_t* e = adds + 3 * j;
                    if (part_of(e[0], e[1], e[2], P) != me) continue;
                    rec_t* r = tmap_find(&m, e[0], e[1], e[2], 1);
                    if (!r->present) { r->present = 1; r->since = (int16_t)i; }
                }
            }
            for (uint64_t i = 0; i <= m.mask; ++i)
                if (m.r[i].used && m.r[i].present) set_bits(m.r[i].bits, m.r[i].since, (int)K);
        }
        maps[me] = m;
        counts[me + 1] = m.n;
#pragma omp barrier
#pragma omp single
        {
            for (uint32_t t = 0; t < P; ++t) counts[t + 1] += counts[t];
        }
        if (!err && counts[P] <= cap) {
            uint64_t n = counts[me];
            for (uint64_t i = 0; m.r && i <= m.mask; ++i) {
                rec_t* r = &m.r[i];
                if (!r->used) continue;
                out_trip[3 * n] = r->src; out_trip[3 * n + 1] = r->dst; out_trip[3 * n + 2] = r->w;
                out_bits[2 * n] = r->bits[0]; out_bits[2 * n + 1] = r->bits[1];
                n++;
            }
        }
        free(m.r);
    }
    int64_t n = (err || counts[P] > cap) ? -1 : (int64_t)counts[P];
    free(counts);
    free(maps);
    return n;
}

/* ------------------------------------------------------------------ solves */

typedef struct { uint32_t* off; uint32_t* dst; uint32_t* w; } adj_t;

/* Adjacency (by source) of the triples selected by `keep`. */
static int build_adj(uint32_t V, uint64_t n, const uint32_t* trip, const uint8_t* keep, adj_t* a) {
    a->off = (uint32_t*)calloc((size_t)V + 1, sizeof(uint32_t));
    uint64_t m = 0;
    for (uint64_t j = 0; j < n; ++j)
        if (keep[j]) { a->off[trip[3 * j] + 1]++; m++; }
    for (uint32_t v = 0; v < V; ++v) a->off[v + 1] += a->off[v];
    a->dst = (uint32_t*)malloc((m + 1) * sizeof(uint32_t));
    a->w = (uint32_t*)malloc((m + 1) * sizeof(uint32_t));
    uint32_t* fill = (uint32_t*)malloc(((size_t)V + 1) * sizeof(uint32_t));
    if (!a->off || !a->dst || !a->w || !fill) return -1;
    memcpy(fill, a->off, ((size_t)V + 1) * sizeof(uint32_t));
    for (uint64_t j = 0; j < n; ++j)
        if (keep[j]) {
            uint32_t p = fill[trip[3 * j]]++;
            a->dst[p] = trip[3 * j + 1];
            a->w[p] = trip[3 * j + 2];
        }
    free(fill);
    return 0;
}

static void free_adj(adj_t* a) { free(a->off); free(a->dst); free(a->w); }

/* Binary min-heap of 64-bit items (priority in the high word, vertex low). */
typedef struct { uint64_t* h; uint64_t n; } heap_t;

static void heap_push(heap_t* q, uint64_t x) {
    uint64_t i = q->n++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (q->h[p] <= x) break;
        q->h[i] = q->h[p];
        i = p;
    }
    q->h[i] = x;
}

static uint64_t heap_pop(heap_t* q) {
    uint64_t top = q->h[0], x = q->h[--q->n], i = 0;
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= q->n) break;
        if (c + 1 < q->n && q->h[c + 1] < q->h[c]) c++;
        if (x <= q->h[c]) break;
        q->h[i] = q->h[c];
        i = c;
    }
    if (q->n) q->h[i] = x;
    return top;
}

/* Candidate value of the path to u extended by an edge of weight w. */
static uint32_t extend(int algo, uint32_t xu, uint32_t w) {
    switch (algo) {
    case O_SSSP: {
        if (xu == INF32) return INF32;
        uint64_t s = (uint64_t)xu + w;
        return s > SAT32 ? SAT32 : (uint32_t)s;
    }
    case O_SSWP: return xu < w ? xu : w;
    case O_SSNP: return xu == INF32 ? INF32 : (xu > w ? xu : w);
    case O_VIT: {
        if (xu == 0u) return 0u;
        float x;
        memcpy(&x, &xu, 4);
        const double q = (double)x / (double)w;
        if (q < (double)FLT_MIN) return 0u;
        const float r = (float)q;
        uint32_t out;
        memcpy(&out, &r, 4);
        return out;
    }
    }
    return INF32;
}

static int max_type(int algo) { return algo == O_SSWP || algo == O_VIT; }

/* a is a strictly better value than b */
static int better(int algo, uint32_t a, uint32_t b) { return max_type(algo) ? a > b : a < b; }

static int solve_adj(int algo, uint32_t V, const adj_t* a, uint32_t source, uint32_t* val) {
    uint32_t unreach = max_type(algo) ? 0u : INF32;
    for (uint32_t v = 0; v < V; ++v) val[v] = unreach;
    if (source >= V) return -1;
    uint64_t m = a->off[V];
    if (algo == O_BFS) {
        uint32_t* queue = (uint32_t*)malloc(((size_t)V + 1) * sizeof(uint32_t));
        uint64_t qh = 0, qt = 0;
        val[source] = 0;
        queue[qt++] = source;
        while (qh < qt) {
            uint32_t u = queue[qh++];
            for (uint32_t e = a->off[u]; e < a->off[u + 1]; ++e) {
                uint32_t x = a->dst[e];
                if (val[x] == INF32) { val[x] = val[u] + 1; queue[qt++] = x; }
            }
        }
        free(queue);
        return 0;
    }
    heap_t q = {(uint64_t*)malloc((m + 2) * sizeof(uint64_t)), 0};
    uint8_t* done = (uint8_t*)calloc(V, 1);
    val[source] = algo == O_SSWP ? INF32 : (algo == O_VIT ? ONE_F32 : 0u);
    /* the heap pops the smallest priority: priorities of max-type queries are complemented */
#define PRIO(x) ((uint64_t)(max_type(algo) ? ~(x) : (x)) << 32)
    heap_push(&q, PRIO(val[source]) | source);
    while (q.n) {
        uint64_t it = heap_pop(&q);
        uint32_t u = (uint32_t)it;
        if (done[u]) continue;
        done[u] = 1;
        for (uint32_t e = a->off[u]; e < a->off[u + 1]; ++e) {
            uint32_t x = a->dst[e];
            if (done[x]) continue;
            uint32_t c = extend(algo, val[u], a->w[e]);
            if (better(algo, c, val[x])) {
                val[x] = c;
                heap_push(&q, PRIO(c) | x);
            }
        }
    }
#undef PRIO
    free(q.h);
    free(done);
    return 0;
}

/* Solve on an explicit edge list (n triples, duplicates allowed). */
int oracle_solve(uint32_t V, uint64_t n, const uint32_t* trip, int algo, uint32_t source, uint32_t* out) {
    if (algo < 0 || algo > 4) return -1;
    uint8_t* keep = (uint8_t*)malloc(n + 1);
    memset(keep, 1, n + 1);
    adj_t a = {0, 0, 0};
    int rc = build_adj(V, n, trip, keep, &a);
    if (rc == 0) rc = solve_adj(algo, V, &a, source, out);
    free_adj(&a);
    free(keep);
    return rc;
}

static int has_bit(const uint64_t* bits, uint64_t j, uint32_t t) {
    return (int)((bits[2 * j + (t >> 6)] >> (t & 63)) & 1ULL);
}

/*
 * Per-snapshot values for the snapshots listed in `snaps` (n_snaps of them):
 * out[v * n_snaps + j] = value of v in snapshot snaps[j].  Snapshots are
 * independent, so they are solved in parallel, one per thread.
 */
int oracle_query(uint32_t V, uint64_t n, const uint32_t* trip, const uint64_t* bits, int algo,
                 uint32_t source, const uint32_t* snaps, uint32_t n_snaps, uint32_t* out, int nthreads) {
    if (algo < 0 || algo > 4 || source >= V) return -1;
    int err = 0;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t j = 0; j < (int64_t)n_snaps; ++j) {
        uint32_t t = snaps[j];
        uint8_t* keep = (uint8_t*)malloc(n + 1);
        uint32_t* val = (uint32_t*)malloc(((size_t)V + 1) * sizeof(uint32_t));
        for (uint64_t e = 0; e < n; ++e) keep[e] = (uint8_t)has_bit(bits, e, t);
        adj_t a = {0, 0, 0};
        int rc = build_adj(V, n, trip, keep, &a);
        if (rc == 0) rc = solve_adj(algo, V, &a, source, val);
        if (rc) {
#pragma omp atomic write
            err = rc;
        } else {
            for (uint32_t v = 0; v < V; ++v) out[(size_t)v * n_snaps + j] = val[v];
        }
        free_adj(&a);
        free(keep);
        free(val);
    }
    return err;
}

/*
 * Bounds of Step 1: r_cap = values on the intersection graph of the window
 * [b, b+L) (triples present in every snapshot of it), r_cup = values on the
 * union graph (triples present in at least one).
 */
int oracle_bounds(uint32_t V, uint64_t n, const uint32_t* trip, const uint64_t* bits, int algo,
                  uint32_t source, uint32_t b, uint32_t L, uint32_t* r_cap, uint32_t* r_cup) {
    if (algo < 0 || algo > 4 || source >= V || L == 0) return -1;
    uint8_t* all = (uint8_t*)malloc(n + 1);
    uint8_t* any = (uint8_t*)malloc(n + 1);
    for (uint64_t e = 0; e < n; ++e) {
        int c = 0;
        for (uint32_t t = b; t < b + L; ++t) c += has_bit(bits, e, t);
        all[e] = (uint8_t)(c == (int)L);
        any[e] = (uint8_t)(c > 0);
    }
    adj_t a1 = {0, 0, 0}, a2 = {0, 0, 0};
    int rc = build_adj(V, n, trip, all, &a1);
    if (rc == 0) rc = solve_adj(algo, V, &a1, source, r_cap);
    free_adj(&a1);
    if (rc == 0) rc = build_adj(V, n, trip, any, &a2);
    if (rc == 0) rc = solve_adj(algo, V, &a2, source, r_cup);
    free_adj(&a2);
    free(all);
    free(any);
    return rc;
}
