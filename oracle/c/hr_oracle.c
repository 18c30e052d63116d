/*
 * C part of the CPU oracle (test infrastructure only; never linked by the
 * product).  Plain loops over the definitions, parallelised over independent
 * instances with pthreads (instances are independent, Sec. 1.2 of the paper:
 * the search is embarrassingly parallel over domains).
 *
 *  oracle_brute_hits      every k < N with (B - lo - k A) mod 2^64 < D, by
 *                         evaluating all k (the set behind Eq. 1).
 *  oracle_exhaustive_many the paper's phase 3 (Sec. 4.1): evaluate each
 *                         piece polynomial at every x < N by the tabulated
 *                         difference shift (Sec. 5.2, Fig. 7) in W-bit fixed
 *                         point and classify the value against the HR test.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t dist;
    uint32_t k;
} hit_t;

static int hit_cmp(const void* x, const void* y) {
    const hit_t* a = (const hit_t*)x;
    const hit_t* b = (const hit_t*)y;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return a->k < b->k ? -1 : (a->k > b->k);
}

typedef struct {
    const uint64_t *A, *B, *lo, *D;
    const uint32_t* N;
    uint64_t n;
    uint32_t* counts;
    const uint64_t* offsets; /* NULL in the counting pass */
    uint32_t* ks;
    uint64_t cap;
    int tid, nthreads;
} brute_arg;

static void* brute_worker(void* p) {
    brute_arg* g = (brute_arg*)p;
    for (uint64_t i = (uint64_t)g->tid; i < g->n; i += (uint64_t)g->nthreads) {
        const uint64_t A = g->A[i], B = g->B[i] - g->lo[i], D = g->D[i];
        const uint32_t N = g->N[i];
        if (!g->offsets) {
            uint32_t c = 0;
            for (uint64_t k = 0; k < N; ++k)
                if ((uint64_t)(B - k * A) < D) ++c;
            g->counts[i] = c;
        } else {
            uint32_t c = g->counts[i];
            if (c == 0) continue;
            hit_t* h = (hit_t*)malloc(sizeof(hit_t) * c);
            uint32_t m = 0;
            for (uint64_t k = 0; k < N; ++k) {
                uint64_t dist = B - k * A;
                if (dist < D) { h[m].dist = dist; h[m].k = (uint32_t)k; ++m; }
            }
            qsort(h, m, sizeof(hit_t), hit_cmp);
            for (uint32_t j = 0; j < m; ++j)
                if (g->offsets[i] + j < g->cap) g->ks[g->offsets[i] + j] = h[j].k;
            free(h);
        }
    }
    return NULL;
}

static void run_brute(brute_arg* base, int threads) {
    pthread_t th[256];
    brute_arg args[256];
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    for (int t = 0; t < threads; ++t) {
        args[t] = *base;
        args[t].tid = t;
        args[t].nthreads = threads;
        pthread_create(&th[t], NULL, brute_worker, &args[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
}

/* Hits of n instances (per-instance window start lo[i] and width D[i]).
 * counts[i] receives the hit count of instance i; the hits themselves are
 * written as k values, instance by instance, each instance's hits ordered by
 * (distance, k), into ks[0 .. min(total, cap)).  offsets (n entries) receives
 * the exclusive prefix sum of counts.  Returns the total number of hits. */
uint64_t oracle_brute_hits(const uint64_t* A, const uint64_t* B, const uint32_t* N,
                           const uint64_t* lo, const uint64_t* D, uint64_t n,
                           uint32_t* counts, uint64_t* offsets, uint32_t* ks,
                           uint64_t cap, int threads) {
    brute_arg g;
    memset(&g, 0, sizeof g);
    g.A = A; g.B = B; g.N = N; g.lo = lo; g.D = D; g.n = n;
    g.counts = counts; g.ks = ks; g.cap = cap;
    run_brute(&g, threads);
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; ++i) { offsets[i] = total; total += counts[i]; }
    g.offsets = offsets;
    run_brute(&g, threads);
    return total;
}

/* ---------------------------------------------------------------------- */

#define MAXL 8   /* up to 512-bit words */
#define MAXD 16

typedef struct {
    const uint64_t* rows;     /* piece p: (delta+1) words of L limbs at p*(delta+1)*L */
    const uint32_t* N;
    const uint64_t *hr_lo, *hr_hi, *rej_lo, *rej_hi;
    uint64_t n_pieces;
    int delta, L;
    uint32_t* counts;         /* per piece: HR + ambiguous values found */
    uint32_t** xs;            /* per piece scratch lists, allocated by the worker */
    uint8_t** cls;
    int tid, nthreads;
} exh_arg;

/* w += x over L limbs (mod 2^(64 L)). */
static void add_words(uint64_t* w, const uint64_t* x, int L) {
    unsigned carry = 0;
    for (int l = 0; l < L; ++l) {
        unsigned __int128 s = (unsigned __int128)w[l] + x[l] + carry;
        w[l] = (uint64_t)s;
        carry = (unsigned)(s >> 64);
    }
}

static void* exh_worker(void* p) {
    exh_arg* g = (exh_arg*)p;
    const int d = g->delta, L = g->L;
    for (uint64_t pc = (uint64_t)g->tid; pc < g->n_pieces; pc += (uint64_t)g->nthreads) {
        uint64_t v[MAXD + 1][MAXL];
        for (int j = 0; j <= d; ++j)
            memcpy(v[j], g->rows + (pc * (uint64_t)(d + 1) + (uint64_t)j) * L, sizeof(uint64_t) * L);
        uint32_t cap = 16, m = 0;
        uint32_t* xs = (uint32_t*)malloc(sizeof(uint32_t) * cap);
        uint8_t* cl = (uint8_t*)malloc(cap);
        const uint64_t hl = g->hr_lo[pc], hh = g->hr_hi[pc];
        const uint64_t rl = g->rej_lo[pc], rh = g->rej_hi[pc];
        for (uint32_t x = 0; x < g->N[pc]; ++x) {
            const uint64_t t = v[0][L - 1];
            int c = -1;
            if (t >= hl && t <= hh) c = 1;              /* certainly HR   */
            else if (!(t >= rl && t <= rh)) c = 2;      /* undecided       */
            if (c > 0) {
                if (m == cap) {
                    cap *= 2;
                    xs = (uint32_t*)realloc(xs, sizeof(uint32_t) * cap);
                    cl = (uint8_t*)realloc(cl, cap);
                }
                xs[m] = x; cl[m] = (uint8_t)c; ++m;
            }
            /* Fig. 7: Delta^{l}(x+1) = Delta^{l}(x) + Delta^{l+1}(x) */
            for (int l = 0; l < d; ++l) add_words(v[l], v[l + 1], L);
        }
        g->counts[pc] = m;
        g->xs[pc] = xs;
        g->cls[pc] = cl;
    }
    return NULL;
}

/* Exhaustive phase over n_pieces pieces.  For each piece the caller gives
 * its rows r_0..r_delta (W = 64 L bits each), N, and four thresholds on the
 * top 64 bits t of the value: HR iff hr_lo <= t <= hr_hi, rejected iff
 * rej_lo <= t <= rej_hi, undecided otherwise.  Results go to counts[] and to
 * the CSR arrays xs_out / cls_out (piece order, increasing x), at most cap
 * entries.  Returns the total. */
uint64_t oracle_exhaustive_many(const uint64_t* rows, const uint32_t* N,
                                const uint64_t* hr_lo, const uint64_t* hr_hi,
                                const uint64_t* rej_lo, const uint64_t* rej_hi,
                                uint64_t n_pieces, int delta, int L,
                                uint32_t* counts, uint32_t* xs_out, uint8_t* cls_out,
                                uint64_t cap, int threads) {
    if (delta > MAXD || L > MAXL || L < 1) return (uint64_t)-1;
    exh_arg g;
    memset(&g, 0, sizeof g);
    g.rows = rows; g.N = N; g.hr_lo = hr_lo; g.hr_hi = hr_hi;
    g.rej_lo = rej_lo; g.rej_hi = rej_hi; g.n_pieces = n_pieces;
    g.delta = delta; g.L = L; g.counts = counts;
    g.xs = (uint32_t**)calloc(n_pieces ? n_pieces : 1, sizeof(uint32_t*));
    g.cls = (uint8_t**)calloc(n_pieces ? n_pieces : 1, sizeof(uint8_t*));
    pthread_t th[256];
    exh_arg args[256];
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    for (int t = 0; t < threads; ++t) {
        args[t] = g;
        args[t].tid = t;
        args[t].nthreads = threads;
        pthread_create(&th[t], NULL, exh_worker, &args[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    uint64_t total = 0;
    for (uint64_t pc = 0; pc < n_pieces; ++pc) {
        for (uint32_t j = 0; j < counts[pc]; ++j, ++total) {
            if (total < cap) { xs_out[total] = g.xs[pc][j]; cls_out[total] = g.cls[pc][j]; }
        }
        free(g.xs[pc]);
        free(g.cls[pc]);
    }
    free(g.xs);
    free(g.cls);
    return total;
}
