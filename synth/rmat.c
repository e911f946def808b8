/*
 * Seeded synthetic evolving-graph generator.
 *
 * Produces the inputs that both the HIP library and the CPU oracle consume:
 * a base edge list (a set of distinct (src, dst, w) triples drawn by R-MAT)
 * and K update batches, each a list of deletions drawn uniformly without
 * replacement from the current snapshot plus as many fresh R-MAT additions.
 * It holds none of the query arithmetic: it only draws random numbers and
 * keeps the current edge set so that deletions and additions are valid.
 *
 * Random numbers: counter-based SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Draw number i of
 * stream j under seed s is the SplitMix64 finaliser applied to
 * base(s, j) + (i + 1) * gamma, so any draw can be produced independently and
 * generation parallelises without changing the result.
 *
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each of the `scale`
 * levels picks one quadrant with probabilities a, b, c, d = 1 - a - b - c,
 * setting one bit of src (c, d quadrants) and one bit of dst (b, d quadrants),
 * most significant bit first.  No noise and no vertex permutation.
 *
 * Triples are packed into a 64-bit key (src << 40 | dst << 16 | w), which
 * limits scale to 24 and w to 65534.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
    return sm64_mix(seed * GAMMA + sm64_mix(stream + GAMMA));
}

/* Draw number `i` of the stream whose base is `base`. */
static inline uint64_t draw(uint64_t base, uint64_t i) {
    return sm64_mix(base + (i + 1) * GAMMA);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, n) by multiply-shift on the top 32 bits (Lemire). */
static inline uint64_t below(uint64_t r, uint64_t n) {
    if (n <= 0xFFFFFFFFULL) return ((r >> 32) * n) >> 32;
    return r % n;
}

uint64_t synth_draw(uint64_t seed, uint64_t stream, uint64_t i) {
    return draw(stream_base(seed, stream), i);
}

#define KEY(s, d, w) (((uint64_t)(s) << 40) | ((uint64_t)(d) << 16) | (uint64_t)(w))
#define KSRC(k) ((uint32_t)((k) >> 40))
#define KDST(k) ((uint32_t)(((k) >> 16) & 0xFFFFFFu))
#define KW(k) ((uint32_t)((k) & 0xFFFFu))

typedef struct {
    uint32_t scale;
    double a, b, c;
    uint32_t wmin, wmax;
} rmat_params;

/* One R-MAT sample: `scale` + 1 draws (one per level, then the weight). */
static inline uint64_t rmat_sample(const rmat_params* p, uint64_t base, uint64_t i) {
    uint64_t first = i * (uint64_t)(p->scale + 1);
    uint32_t src = 0, dst = 0;
    double ab = p->a + p->b, abc = p->a + p->b + p->c;
    for (uint32_t l = 0; l < p->scale; ++l) {
        double r = unit(draw(base, first + l));
        uint32_t sb, db;
        if (r < p->a) { sb = 0; db = 0; }
        else if (r < ab) { sb = 0; db = 1; }
        else if (r < abc) { sb = 1; db = 0; }
        else { sb = 1; db = 1; }
        src = (src << 1) | sb;
        dst = (dst << 1) | db;
    }
    uint32_t w = p->wmin + (uint32_t)below(draw(base, first + p->scale), (uint64_t)(p->wmax - p->wmin + 1));
    return KEY(src, dst, w);
}

/* Plain R-MAT samples (duplicates kept), as (src, dst, w) triples. */
void synth_rmat(uint32_t scale, double a, double b, double c, uint32_t wmin, uint32_t wmax,
                uint64_t seed, uint64_t stream, uint64_t n, uint32_t* out) {
    rmat_params p = {scale, a, b, c, wmin, wmax};
    uint64_t base = stream_base(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t k = rmat_sample(&p, base, (uint64_t)i);
        out[3 * i] = KSRC(k);
        out[3 * i + 1] = KDST(k);
        out[3 * i + 2] = KW(k);
    }
}

/* Parallel LSD radix sort of 64-bit keys, 8-bit digits, `bits` low bits significant. */
static void radix_sort_u64(uint64_t* a, uint64_t* tmp, uint64_t n, int bits) {
    int nt = omp_get_max_threads();
    uint64_t* cnt = (uint64_t*)calloc((size_t)nt * 256, sizeof(uint64_t));
    for (int shift = 0; shift < bits; shift += 8) {
        memset(cnt, 0, (size_t)nt * 256 * sizeof(uint64_t));
#pragma omp parallel num_threads(nt)
        {
            int t = omp_get_thread_num();
            uint64_t lo = n * (uint64_t)t / (uint64_t)nt, hi = n * (uint64_t)(t + 1) / (uint64_t)nt;
            uint64_t* c = cnt + (size_t)t * 256;
            for (uint64_t i = lo; i < hi; ++i) c[(a[i] >> shift) & 0xFF]++;
#pragma omp barrier
#pragma omp single
            {
                uint64_t run = 0;
                for (int d = 0; d < 256; ++d)
                    for (int u = 0; u < nt; ++u) {
                        uint64_t v = cnt[(size_t)u * 256 + d];
                        cnt[(size_t)u * 256 + d] = run;
                        run += v;
                    }
            }
            for (uint64_t i = lo; i < hi; ++i) tmp[c[(a[i] >> shift) & 0xFF]++] = a[i];
        }
        uint64_t* s = a; a = tmp; tmp = s;
    }
    /* an odd number of passes leaves the result in the scratch buffer */
    if (((bits + 7) / 8) & 1) memcpy(tmp, a, n * sizeof(uint64_t));
    free(cnt);
}

/* Open-addressing set of keys (stored as key + 1; 0 = empty, ~0 = removed). */
typedef struct { uint64_t* slot; uint64_t mask; } kset;

static inline uint64_t kset_h(uint64_t k) { return sm64_mix(k ^ 0x5851F42D4C957F2DULL); }

static int kset_has(const kset* s, uint64_t k) {
    uint64_t v = k + 1, i = kset_h(k) & s->mask;
    for (;;) {
        uint64_t x = s->slot[i];
        if (x == 0) return 0;
        if (x == v) return 1;
        i = (i + 1) & s->mask;
    }
}

/* Returns 1 when inserted, 0 when already present. */
static int kset_add(kset* s, uint64_t k) {
    uint64_t v = k + 1, i = kset_h(k) & s->mask;
    for (;;) {
        uint64_t x = s->slot[i];
        if (x == 0) { s->slot[i] = v; return 1; }
        if (x == v) return 0;
        i = (i + 1) & s->mask;
    }
}

static void kset_add_par(kset* s, uint64_t k) {
    uint64_t v = k + 1, i = kset_h(k) & s->mask;
    for (;;) {
        uint64_t x = __atomic_load_n(&s->slot[i], __ATOMIC_RELAXED);
        if (x == v) return;
        if (x == 0) {
            uint64_t expect = 0;
            if (__atomic_compare_exchange_n(&s->slot[i], &expect, v, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return;
            if (expect == v) return;
        }
        i = (i + 1) & s->mask;
    }
}

static void kset_del(kset* s, uint64_t k) {
    uint64_t v = k + 1, i = kset_h(k) & s->mask;
    for (;;) {
        uint64_t x = s->slot[i];
        if (x == 0) return;
        if (x == v) { s->slot[i] = ~0ULL; return; }
        i = (i + 1) & s->mask;
    }
}

/*
 * Full instance.  Streams: 0 = base samples; 1 + i = additions of batch i;
 * (1 << 20) + i = deletions of batch i.
 *   base_out : capacity n_samples triples; receives the distinct base triples
 *              sorted by (src, dst, w); the count is returned.
 *   del_out  : K * n_del triples, batch-major.  add_out : K * n_add triples.
 * Returns the number of base triples, or -1 when an argument is out of range
 * (scale > 24, wmax > 65534, wmin == 0 or wmin > wmax, or a batch deletes more
 * edges than the snapshot holds).
 */
int64_t synth_instance(uint32_t scale, double a, double b, double c, uint32_t wmin, uint32_t wmax,
                       uint64_t seed, uint64_t n_samples, uint32_t K, uint64_t n_del, uint64_t n_add,
                       uint32_t* base_out, uint32_t* del_out, uint32_t* add_out) {
    if (scale > 24 || wmax > 65534 || wmin == 0 || wmin > wmax) return -1;
    rmat_params p = {scale, a, b, c, wmin, wmax};
    uint64_t* keys = (uint64_t*)malloc(n_samples * sizeof(uint64_t) + 8);
    uint64_t* tmp = (uint64_t*)malloc(n_samples * sizeof(uint64_t) + 8);
    uint64_t sb0 = stream_base(seed, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n_samples; ++i) keys[i] = rmat_sample(&p, sb0, (uint64_t)i);
    radix_sort_u64(keys, tmp, n_samples, 64);
    uint64_t n = 0;
    for (uint64_t i = 0; i < n_samples; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[n++] = keys[i];
    for (uint64_t i = 0; i < n; ++i) {
        base_out[3 * i] = KSRC(keys[i]);
        base_out[3 * i + 1] = KDST(keys[i]);
        base_out[3 * i + 2] = KW(keys[i]);
    }
    free(tmp);

    /* current snapshot: array `cur` (order matters for deletion draws) + set */
    uint64_t cap_n = n + (uint64_t)K * n_add + 16;
    uint64_t* cur = (uint64_t*)realloc(keys, cap_n * sizeof(uint64_t));
    uint64_t hcap = 1024;
    while (hcap < 2 * cap_n) hcap <<= 1;
    kset set = {(uint64_t*)calloc(hcap, sizeof(uint64_t)), hcap - 1};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) kset_add_par(&set, cur[i]);

    uint64_t ncur = n;
    for (uint32_t bi = 0; bi < K; ++bi) {
        if (n_del > ncur) { free(cur); free(set.slot); return -1; }
        /* deletions: partial Fisher-Yates from the tail of `cur` */
        uint64_t db = stream_base(seed, (1ULL << 20) + bi);
        for (uint64_t k = 0; k < n_del; ++k) {
            uint64_t j = below(draw(db, k), ncur - k);
            uint64_t t = cur[j];
            cur[j] = cur[ncur - 1 - k];
            cur[ncur - 1 - k] = t;
        }
        uint32_t* dout = del_out + (size_t)3 * n_del * bi;
        for (uint64_t k = 0; k < n_del; ++k) {
            uint64_t key = cur[ncur - 1 - k];
            dout[3 * k] = KSRC(key); dout[3 * k + 1] = KDST(key); dout[3 * k + 2] = KW(key);
        }
        /* additions: fresh samples absent from the previous snapshot and from this batch */
        uint64_t ab = stream_base(seed, 1ULL + bi);
        uint32_t* aout = add_out + (size_t)3 * n_add * bi;
        uint64_t got = 0, att = 0;
        uint64_t* added = (uint64_t*)malloc((n_add + 1) * sizeof(uint64_t));
        while (got < n_add) {
            uint64_t key = rmat_sample(&p, ab, att++);
            if (kset_add(&set, key)) added[got++] = key;
        }
        for (uint64_t k = 0; k < n_del; ++k) kset_del(&set, cur[ncur - 1 - k]);
        ncur -= n_del;
        for (uint64_t k = 0; k < n_add; ++k) {
            cur[ncur++] = added[k];
            aout[3 * k] = KSRC(added[k]); aout[3 * k + 1] = KDST(added[k]); aout[3 * k + 2] = KW(added[k]);
        }
        free(added);
    }
    free(cur);
    free(set.slot);
    return (int64_t)n;
}
