/*
 * ggen.c -- seeded synthetic graph generators.  See ggen.h for the contract.
 * Host C only; holds no traversal arithmetic.
 */
#include "ggen.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ RNG -- */

/* SplitMix64 step: advance the 64-bit state by the golden-ratio increment and
 * return the mixed value (Steele, Lea & Flood 2014). */
static uint64_t splitmix64(uint64_t* x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } rng_t;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

/* xoshiro256** (Blackman & Vigna 2018). */
static inline uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* Independent generator per (seed, stream, chunk): the three words are folded
 * through SplitMix64 and the result seeds the four state words. */
static void rng_seed(rng_t* r, uint64_t seed, uint64_t stream, uint64_t chunk) {
    uint64_t x = seed;
    uint64_t h = splitmix64(&x);
    x = h ^ stream;
    h = splitmix64(&x);
    x = h ^ chunk;
    h = splitmix64(&x);
    x = h;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

/* Integer in [lo, hi] from the top 32 bits (multiply-shift). */
static inline int32_t rng_int(rng_t* r, int32_t lo, int32_t hi) {
    uint64_t span = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
    uint64_t top = rng_next(r) >> 32;
    return (int32_t)((int64_t)lo + (int64_t)((top * span) >> 32));
}

/* Uniform double in [0, 1) from 53 bits. */
static inline double rng_unit(rng_t* r) {
    return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------- thread helpers --- */

#define CHUNK_EDGES 65536

static int gen_threads(void) {
    const char* e = getenv("GGEN_THREADS");
    long t = e ? atol(e) : sysconf(_SC_NPROCESSORS_ONLN);
    if (t < 1) t = 1;
    if (t > 16) t = 16;
    return (int)t;
}

typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi, int tid);

typedef struct {
    range_fn fn;
    void* ctx;
    int64_t lo, hi;
    int tid;
} job_t;

static void* job_main(void* p) {
    job_t* j = (job_t*)p;
    j->fn(j->ctx, j->lo, j->hi, j->tid);
    return NULL;
}

/* Split [0, total) into nt contiguous ranges, one thread each. */
static void run_parallel(int nt, int64_t total, range_fn fn, void* ctx) {
    if (nt <= 1 || total < 2) {
        fn(ctx, 0, total, 0);
        return;
    }
    if ((int64_t)nt > total) nt = (int)total;
    pthread_t th[16];
    job_t jobs[16];
    for (int t = 0; t < nt; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].lo = total * t / nt;
        jobs[t].hi = total * (t + 1) / nt;
        jobs[t].tid = t;
        pthread_create(&th[t], NULL, job_main, &jobs[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------- CSR build ----- */

typedef struct {
    int32_t n;
    int64_t m;
    int nt;
    const int32_t *src, *dst, *wt;
    int32_t *row_ptr, *col, *w;
    int64_t* cnt; /* nt * n counts, then offsets */
} csr_ctx;

static void csr_count(void* p, int64_t lo, int64_t hi, int tid) {
    csr_ctx* c = (csr_ctx*)p;
    int64_t* h = c->cnt + (int64_t)tid * c->n;
    for (int64_t e = lo; e < hi; ++e) h[c->src[e]]++;
}

static void csr_scatter(void* p, int64_t lo, int64_t hi, int tid) {
    csr_ctx* c = (csr_ctx*)p;
    int64_t* off = c->cnt + (int64_t)tid * c->n;
    for (int64_t e = lo; e < hi; ++e) {
        int64_t pos = off[c->src[e]]++;
        c->col[pos] = c->dst[e];
        if (c->w) c->w[pos] = c->wt ? c->wt[e] : 1;
    }
}

int ggen_csr_from_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* wt, int32_t* row_ptr, int32_t* col, int32_t* w) {
    if (n < 1 || m < 0 || m >= ((int64_t)1 << 31) || !row_ptr || (m > 0 && (!src || !dst || !col)))
        return -1;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    int nt = gen_threads();
    /* keep the per-thread count table modest */
    while (nt > 1 && (int64_t)nt * n * 8 > ((int64_t)1 << 31)) nt /= 2;
    if (m < 4 * CHUNK_EDGES) nt = 1;
    csr_ctx c = {n, m, nt, src, dst, wt, row_ptr, col, w, NULL};
    c.cnt = (int64_t*)calloc((size_t)nt * (size_t)n, sizeof(int64_t));
    if (!c.cnt) return -3;
    run_parallel(nt, m, csr_count, &c);
    /* row_ptr and per-thread starting offsets: thread t's edges of row v
     * follow those of threads < t, which keeps generation order. */
    int64_t run = 0;
    for (int32_t v = 0; v < n; ++v) {
        row_ptr[v] = (int32_t)run;
        for (int t = 0; t < nt; ++t) {
            int64_t k = c.cnt[(int64_t)t * n + v];
            c.cnt[(int64_t)t * n + v] = run;
            run += k;
        }
    }
    row_ptr[n] = (int32_t)run;
    run_parallel(nt, m, csr_scatter, &c);
    free(c.cnt);
    return 0;
}

/* ------------------------------------------------------- raw stream ---- */

int ggen_raw(uint64_t seed, uint64_t stream, uint64_t chunk, int64_t count, uint64_t* out) {
    if (count < 0 || (count > 0 && !out)) return -1;
    rng_t r;
    rng_seed(&r, seed, stream, chunk);
    for (int64_t i = 0; i < count; ++i) out[i] = rng_next(&r);
    return 0;
}

/* ------------------------------------------------- uniform (ER) -------- */

typedef struct {
    int32_t n;
    int64_t m;
    int32_t wlo, whi;
    uint64_t seed, stream;
    int32_t *src, *dst, *wt;
    int32_t scale;
    double a, ab, abc;
} edge_ctx;

static void uniform_chunks(void* p, int64_t clo, int64_t chi, int tid) {
    (void)tid;
    edge_ctx* c = (edge_ctx*)p;
    for (int64_t ch = clo; ch < chi; ++ch) {
        rng_t r;
        rng_seed(&r, c->seed, c->stream, (uint64_t)ch);
        int64_t e0 = ch * CHUNK_EDGES, e1 = e0 + CHUNK_EDGES;
        if (e1 > c->m) e1 = c->m;
        for (int64_t e = e0; e < e1; ++e) {
            int32_t u, v;
            do {
                u = rng_int(&r, 0, c->n - 1);
                v = rng_int(&r, 0, c->n - 1);
            } while (u == v);
            c->src[e] = u;
            c->dst[e] = v;
            if (c->wt) c->wt[e] = rng_int(&r, c->wlo, c->whi);
        }
    }
}

static int finish_csr(int32_t n, int64_t m, int32_t* src, int32_t* dst, int32_t* wt,
                      int32_t* row_ptr, int32_t* col, int32_t* w) {
    int rc = ggen_csr_from_edges(n, m, src, dst, wt, row_ptr, col, w);
    free(src);
    free(dst);
    free(wt);
    return rc;
}

int ggen_uniform(int32_t n, int64_t m, int32_t wlo, int32_t whi, uint64_t seed, uint64_t stream,
                 int32_t* row_ptr, int32_t* col, int32_t* w) {
    if (n < 1 || m < 0 || m >= ((int64_t)1 << 31) || (m > 0 && n < 2) || wlo > whi || wlo < 0)
        return -1;
    edge_ctx c;
    memset(&c, 0, sizeof c);
    c.n = n;
    c.m = m;
    c.wlo = wlo;
    c.whi = whi;
    c.seed = seed;
    c.stream = stream;
    c.src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    c.dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    c.wt = w ? (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1)) : NULL;
    if (!c.src || !c.dst || (w && !c.wt)) return -3;
    int64_t nch = (m + CHUNK_EDGES - 1) / CHUNK_EDGES;
    run_parallel(gen_threads(), nch, uniform_chunks, &c);
    return finish_csr(n, m, c.src, c.dst, c.wt, row_ptr, col, w);
}

/* ------------------------------------------------------------ R-MAT ---- */

static void rmat_chunks(void* p, int64_t clo, int64_t chi, int tid) {
    (void)tid;
    edge_ctx* c = (edge_ctx*)p;
    for (int64_t ch = clo; ch < chi; ++ch) {
        rng_t r;
        rng_seed(&r, c->seed, c->stream, (uint64_t)ch);
        int64_t e0 = ch * CHUNK_EDGES, e1 = e0 + CHUNK_EDGES;
        if (e1 > c->m) e1 = c->m;
        for (int64_t e = e0; e < e1; ++e) {
            int32_t u = 0, v = 0;
            for (int lvl = 0; lvl < c->scale; ++lvl) {
                double x = rng_unit(&r);
                int32_t bit = (int32_t)1 << (c->scale - 1 - lvl);
                if (x < c->a) {
                    /* quadrant a: neither bit */
                } else if (x < c->ab) {
                    v |= bit; /* b */
                } else if (x < c->abc) {
                    u |= bit; /* c */
                } else {
                    u |= bit; /* d */
                    v |= bit;
                }
            }
            c->src[e] = u;
            c->dst[e] = v;
            if (c->wt) c->wt[e] = rng_int(&r, c->wlo, c->whi);
        }
    }
}

int ggen_rmat(int32_t scale, int64_t m, double a, double b, double c_, int32_t wlo, int32_t whi,
              uint64_t seed, uint64_t stream, int32_t* row_ptr, int32_t* col, int32_t* w) {
    if (scale < 1 || scale > 30 || m < 0 || m >= ((int64_t)1 << 31) || wlo > whi || wlo < 0 ||
        a < 0 || b < 0 || c_ < 0 || a + b + c_ > 1.0)
        return -1;
    edge_ctx c;
    memset(&c, 0, sizeof c);
    c.n = (int32_t)1 << scale;
    c.m = m;
    c.wlo = wlo;
    c.whi = whi;
    c.seed = seed;
    c.stream = stream;
    c.scale = scale;
    c.a = a;
    c.ab = a + b;
    c.abc = a + b + c_;
    c.src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    c.dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    c.wt = w ? (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1)) : NULL;
    if (!c.src || !c.dst || (w && !c.wt)) return -3;
    int64_t nch = (m + CHUNK_EDGES - 1) / CHUNK_EDGES;
    run_parallel(gen_threads(), nch, rmat_chunks, &c);
    return finish_csr(c.n, m, c.src, c.dst, c.wt, row_ptr, col, w);
}

/* ------------------------------------------------------------- grid ---- */

int64_t ggen_grid_edges(int32_t width, int32_t height, int64_t n_shortcuts) {
    if (width < 1 || height < 1 || n_shortcuts < 0) return -1;
    int64_t und = (int64_t)height * (width - 1) + (int64_t)width * (height - 1);
    return 2 * (und + n_shortcuts);
}

typedef struct {
    int32_t W, H, span, wlo, whi;
    int64_t n_short, und_grid;
    uint64_t seed, stream;
    int32_t *src, *dst, *wt;
} grid_ctx;

/* Undirected grid edges of row y, in x order: right neighbour, then down.
 * Directed slots: the undirected edge k fills 2k (u->v) and 2k+1 (v->u). */
static void grid_rows(void* p, int64_t ylo, int64_t yhi, int tid) {
    (void)tid;
    grid_ctx* g = (grid_ctx*)p;
    for (int64_t y = ylo; y < yhi; ++y) {
        rng_t r;
        rng_seed(&r, g->seed, g->stream, (uint64_t)y);
        /* undirected edges before row y: each full row contributes
         * (W-1) right edges + W down edges */
        int64_t k = y * ((int64_t)(g->W - 1) + g->W);
        for (int32_t x = 0; x < g->W; ++x) {
            int32_t u = (int32_t)(y * g->W + x);
            if (x + 1 < g->W) {
                int32_t v = u + 1, wv = rng_int(&r, g->wlo, g->whi);
                g->src[2 * k] = u; g->dst[2 * k] = v; g->wt[2 * k] = wv;
                g->src[2 * k + 1] = v; g->dst[2 * k + 1] = u; g->wt[2 * k + 1] = wv;
                ++k;
            }
            if (y + 1 < g->H) {
                int32_t v = u + g->W, wv = rng_int(&r, g->wlo, g->whi);
                g->src[2 * k] = u; g->dst[2 * k] = v; g->wt[2 * k] = wv;
                g->src[2 * k + 1] = v; g->dst[2 * k + 1] = u; g->wt[2 * k + 1] = wv;
                ++k;
            }
        }
    }
}

static void grid_shortcuts(void* p, int64_t clo, int64_t chi, int tid) {
    (void)tid;
    grid_ctx* g = (grid_ctx*)p;
    int64_t n = (int64_t)g->W * g->H;
    for (int64_t ch = clo; ch < chi; ++ch) {
        rng_t r;
        rng_seed(&r, g->seed, g->stream, ((uint64_t)1 << 40) | (uint64_t)ch);
        int64_t s0 = ch * CHUNK_EDGES, s1 = s0 + CHUNK_EDGES;
        if (s1 > g->n_short) s1 = g->n_short;
        for (int64_t s = s0; s < s1; ++s) {
            /* the whole draw (u, dx, dy) is repeated until the target lies
             * on the grid, so every accepted pair is uniform over the valid
             * ones */
            int32_t u, vx, vy;
            for (;;) {
                u = rng_int(&r, 0, (int32_t)(n - 1));
                int32_t dx = rng_int(&r, -g->span, g->span);
                int32_t dy = rng_int(&r, -g->span, g->span);
                int32_t adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
                if (adx + ady < 2) continue;
                vx = u % g->W + dx;
                vy = u / g->W + dy;
                if (vx < 0 || vx >= g->W || vy < 0 || vy >= g->H) continue;
                break;
            }
            int32_t v = vy * g->W + vx, wv = rng_int(&r, g->wlo, g->whi);
            int64_t k = g->und_grid + s;
            g->src[2 * k] = u; g->dst[2 * k] = v; g->wt[2 * k] = wv;
            g->src[2 * k + 1] = v; g->dst[2 * k + 1] = u; g->wt[2 * k + 1] = wv;
        }
    }
}

int ggen_grid(int32_t width, int32_t height, int64_t n_shortcuts, int32_t span, int32_t wlo,
              int32_t whi, uint64_t seed, uint64_t stream, int32_t* row_ptr, int32_t* col,
              int32_t* w) {
    int64_t n = (int64_t)width * height;
    int64_t m = ggen_grid_edges(width, height, n_shortcuts);
    if (m < 0 || n >= ((int64_t)1 << 31) || m >= ((int64_t)1 << 31) || wlo > whi || wlo < 0)
        return -1;
    /* some (u, dx, dy) must exist with |dx|+|dy| >= 2 and the target on the
     * grid, otherwise the redraw loop could not end */
    if (n_shortcuts > 0) {
        int ok = (span >= 2 && (width >= 3 || height >= 3)) ||
                 (span >= 1 && width >= 2 && height >= 2);
        if (!ok) return -1;
    }
    grid_ctx g;
    g.W = width;
    g.H = height;
    g.span = span;
    g.wlo = wlo;
    g.whi = whi;
    g.n_short = n_shortcuts;
    g.und_grid = (int64_t)height * (width - 1) + (int64_t)width * (height - 1);
    g.seed = seed;
    g.stream = stream;
    g.src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g.dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g.wt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    if (!g.src || !g.dst || !g.wt) return -3;
    int nt = gen_threads();
    run_parallel(nt, height, grid_rows, &g);
    run_parallel(nt, (n_shortcuts + CHUNK_EDGES - 1) / CHUNK_EDGES, grid_shortcuts, &g);
    return finish_csr((int32_t)n, m, g.src, g.dst, g.wt, row_ptr, col, w);
}

/* ------------------------------------------------------------ misc ----- */

int ggen_pick_sources(int32_t n, const int32_t* row_ptr, int32_t count, uint64_t seed,
                      uint64_t stream, int32_t* out) {
    if (n < 1 || count < 0 || !row_ptr || (count > 0 && !out)) return -1;
    if (row_ptr[n] == row_ptr[0]) return -2;
    rng_t r;
    rng_seed(&r, seed, stream, 0);
    for (int32_t i = 0; i < count; ++i) {
        int32_t v;
        do {
            v = rng_int(&r, 0, n - 1);
        } while (row_ptr[v + 1] == row_ptr[v]);
        out[i] = v;
    }
    return 0;
}

uint64_t ggen_fnv1a(const int32_t* a, int64_t count) {
    uint64_t h = 0xcbf29ce484222325ULL;
    const unsigned char* p = (const unsigned char*)a;
    for (int64_t i = 0; i < count * 4; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ULL;
    }
    return h;
}
