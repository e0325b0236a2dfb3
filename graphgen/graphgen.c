/*
 * Seeded synthetic input generators (data graphs only).
 *
 * This module produces the undirected simple graphs that stand in for the
 * paper's datasets (Section 7.1, Table 3): Chung-Lu power-law graphs and
 * R-MAT graphs.  It holds none of the enumeration method's arithmetic; both
 * the oracle and the GPU library read the CSR that it writes.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), a counter-based generator, so every
 * random draw is a pure function of (seed, stream, index) and the output does
 * not depend on the number of threads.
 *
 * Output CSR: int64 row_ptr[n+1], int32 col[nnz]; every list strictly
 * ascending, symmetric, no self-loops, no duplicates.  Vertex IDs are passed
 * through a seeded random permutation so that IDs carry no degree order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                       */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t v[4]; } gg_ctr;

static inline void gg_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static gg_ctr gg_philox(gg_ctr c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        gg_mulhilo(0xD2511F53u, c.v[0], &hi0, &lo0);
        gg_mulhilo(0xCD9E8D57u, c.v[2], &hi1, &lo1);
        gg_ctr o;
        o.v[0] = hi1 ^ c.v[1] ^ k0;
        o.v[1] = lo1;
        o.v[2] = hi0 ^ c.v[3] ^ k1;
        o.v[3] = lo0;
        c = o;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

/* Exposed for the known-answer test of the generator itself. */
void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    gg_ctr c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
    gg_ctr o = gg_philox(c, key[0], key[1]);
    memcpy(out, o.v, sizeof(o.v));
}

/* A stream of uniform draws: counter = (index lo, index hi, stream lo, stream hi). */
typedef struct {
    uint32_t k0, k1;
    uint64_t stream;
    uint64_t idx;      /* next block index */
    uint32_t buf[4];
    int left;
} gg_rng;

static void gg_rng_init(gg_rng *r, uint64_t seed, uint64_t stream) {
    r->k0 = (uint32_t)seed;
    r->k1 = (uint32_t)(seed >> 32);
    r->stream = stream;
    r->idx = 0;
    r->left = 0;
}

static inline uint32_t gg_u32(gg_rng *r) {
    if (r->left == 0) {
        gg_ctr c = {{(uint32_t)r->idx, (uint32_t)(r->idx >> 32), (uint32_t)r->stream,
                     (uint32_t)(r->stream >> 32)}};
        gg_ctr o = gg_philox(c, r->k0, r->k1);
        memcpy(r->buf, o.v, sizeof(o.v));
        r->left = 4;
        r->idx++;
    }
    return r->buf[4 - (r->left--)];
}

/* Uniform double in (0, 1): 53 random bits, never exactly 0. */
static inline double gg_unif(gg_rng *r) {
    uint64_t a = gg_u32(r) >> 5, b = gg_u32(r) >> 6;
    return ((double)((a << 26) | b) + 0.5) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* threading helpers                                                    */
/* ------------------------------------------------------------------ */
static int gg_threads(int req) {
    if (req > 0) return req;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    if (c < 1) c = 1;
    if (c > 16) c = 16;
    return (int)c;
}

typedef void (*gg_body)(void *arg, int64_t lo, int64_t hi);
typedef struct {
    gg_body fn;
    void *arg;
    int64_t n, chunk;
    int64_t *next;
    pthread_mutex_t *mu;
} gg_pool_arg;

static void *gg_pool_worker(void *p) {
    gg_pool_arg *a = (gg_pool_arg *)p;
    for (;;) {
        int64_t lo = __atomic_fetch_add(a->next, a->chunk, __ATOMIC_RELAXED);
        if (lo >= a->n) break;
        int64_t hi = lo + a->chunk < a->n ? lo + a->chunk : a->n;
        a->fn(a->arg, lo, hi);
    }
    return NULL;
}

static void gg_parallel_for(int nthreads, int64_t n, int64_t chunk, gg_body fn, void *arg) {
    int64_t next = 0;
    gg_pool_arg pa = {fn, arg, n, chunk, &next, NULL};
    pthread_t th[64];
    int t = nthreads > 64 ? 64 : nthreads;
    for (int i = 1; i < t; ++i) pthread_create(&th[i], NULL, gg_pool_worker, &pa);
    gg_pool_worker(&pa);
    for (int i = 1; i < t; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------ */
/* graph container                                                      */
/* ------------------------------------------------------------------ */
typedef struct gg_graph {
    int64_t n, nnz;
    int64_t *rp;
    int32_t *col;
} gg_graph;

int64_t gg_n(const gg_graph *g) { return g->n; }
int64_t gg_nnz(const gg_graph *g) { return g->nnz; }
void gg_copy(const gg_graph *g, int64_t *rp, int32_t *col) {
    memcpy(rp, g->rp, sizeof(int64_t) * (size_t)(g->n + 1));
    memcpy(col, g->col, sizeof(int32_t) * (size_t)g->nnz);
}
void gg_free(gg_graph *g) {
    if (!g) return;
    free(g->rp);
    free(g->col);
    free(g);
}

/* Seeded random permutation of 0..n-1 (Fisher-Yates, one stream). */
static int32_t *gg_permutation(int64_t n, uint64_t seed) {
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
    gg_rng r;
    gg_rng_init(&r, seed, 0xFFFFFFFF00000001ULL);
    for (int64_t i = n - 1; i > 0; --i) {
        uint64_t x = ((uint64_t)gg_u32(&r) << 32) | gg_u32(&r);
        int64_t j = (int64_t)(x % (uint64_t)(i + 1));
        int32_t t = p[i];
        p[i] = p[j];
        p[j] = t;
    }
    return p;
}

/*
 * Build a clean CSR from a list of undirected pairs (u, v): relabel through
 * perm, symmetrise, drop self-loops, sort and deduplicate each list.
 */
typedef struct {
    int64_t npairs;
    const int32_t *pu, *pv;
    const int32_t *perm;
    int64_t *deg;      /* atomic counters, then fill cursors */
    int64_t *rp;
    int32_t *col;
    int64_t *newdeg;
} gg_build_ctx;

static void gg_count_body(void *arg, int64_t lo, int64_t hi) {
    gg_build_ctx *c = (gg_build_ctx *)arg;
    for (int64_t i = lo; i < hi; ++i) {
        int32_t u = c->perm[c->pu[i]], v = c->perm[c->pv[i]];
        if (u == v) continue;
        __atomic_fetch_add(&c->deg[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&c->deg[v], 1, __ATOMIC_RELAXED);
    }
}

static void gg_fill_body(void *arg, int64_t lo, int64_t hi) {
    gg_build_ctx *c = (gg_build_ctx *)arg;
    for (int64_t i = lo; i < hi; ++i) {
        int32_t u = c->perm[c->pu[i]], v = c->perm[c->pv[i]];
        if (u == v) continue;
        int64_t a = __atomic_fetch_add(&c->deg[u], 1, __ATOMIC_RELAXED);
        c->col[a] = v;
        int64_t b = __atomic_fetch_add(&c->deg[v], 1, __ATOMIC_RELAXED);
        c->col[b] = u;
    }
}

static int gg_cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void gg_sort_body(void *arg, int64_t lo, int64_t hi) {
    gg_build_ctx *c = (gg_build_ctx *)arg;
    for (int64_t u = lo; u < hi; ++u) {
        int32_t *L = c->col + c->rp[u];
        int64_t d = c->rp[u + 1] - c->rp[u];
        if (d > 1) qsort(L, (size_t)d, sizeof(int32_t), gg_cmp_i32);
        int64_t w = 0;
        for (int64_t i = 0; i < d; ++i)
            if (w == 0 || L[i] != L[w - 1]) L[w++] = L[i];
        c->newdeg[u] = w;
    }
}

static gg_graph *gg_build_csr(int64_t n, int64_t npairs, const int32_t *pu, const int32_t *pv,
                              uint64_t perm_seed, int nthreads) {
    gg_build_ctx c;
    memset(&c, 0, sizeof(c));
    c.npairs = npairs;
    c.pu = pu;
    c.pv = pv;
    c.perm = gg_permutation(n, perm_seed);
    c.deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    gg_parallel_for(nthreads, npairs, 1 << 16, gg_count_body, &c);
    c.rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    c.rp[0] = 0;
    for (int64_t u = 0; u < n; ++u) c.rp[u + 1] = c.rp[u] + c.deg[u];
    int64_t tot = c.rp[n];
    c.col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    for (int64_t u = 0; u < n; ++u) c.deg[u] = c.rp[u];
    gg_parallel_for(nthreads, npairs, 1 << 16, gg_fill_body, &c);
    c.newdeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    gg_parallel_for(nthreads, n, 1024, gg_sort_body, &c);
    /* compact the deduplicated lists in place, in ascending row order */
    int64_t *rp2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    rp2[0] = 0;
    for (int64_t u = 0; u < n; ++u) rp2[u + 1] = rp2[u] + c.newdeg[u];
    for (int64_t u = 0; u < n; ++u) {
        if (rp2[u] != c.rp[u])
            memmove(c.col + rp2[u], c.col + c.rp[u], sizeof(int32_t) * (size_t)c.newdeg[u]);
    }
    gg_graph *g = (gg_graph *)malloc(sizeof(gg_graph));
    g->n = n;
    g->nnz = rp2[n];
    g->rp = rp2;
    g->col = (int32_t *)realloc(c.col, sizeof(int32_t) * (size_t)(g->nnz > 0 ? g->nnz : 1));
    free(c.rp);
    free(c.deg);
    free(c.newdeg);
    free((void *)c.perm);
    return g;
}

/* ------------------------------------------------------------------ */
/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004), no noise                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int scale;
    uint64_t seed;
    uint32_t ta, tab, tabc; /* cumulative thresholds on 32-bit uniforms */
    int32_t *pu, *pv;
} gg_rmat_ctx;

static void gg_rmat_body(void *arg, int64_t lo, int64_t hi) {
    gg_rmat_ctx *c = (gg_rmat_ctx *)arg;
    for (int64_t e = lo; e < hi; ++e) {
        gg_rng r;
        gg_rng_init(&r, c->seed, (uint64_t)e);
        uint32_t u = 0, v = 0;
        for (int l = 0; l < c->scale; ++l) {
            uint32_t x = gg_u32(&r);
            /* quadrant of x: [0,a) top-left, [a,a+b) top-right, [a+b,a+b+c)
               bottom-left, rest bottom-right; computed without branches (the
               quadrant is unpredictable, so branches cost more than the draws) */
            const uint32_t s1 = x >= c->ta, s2 = x >= c->tab, s3 = x >= c->tabc;
            const uint32_t ub = s2, vb = s1 ^ s2 ^ s3;
            u = (u << 1) | ub;
            v = (v << 1) | vb;
        }
        c->pu[e] = (int32_t)u;
        c->pv[e] = (int32_t)v;
    }
}

static uint32_t gg_thresh(double p) {
    double t = p * 4294967296.0;
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    if (t <= 0) return 0;
    return (uint32_t)t;
}

gg_graph *gg_rmat(int scale, int64_t nsamples, double a, double b, double c, uint64_t seed,
                  int nthreads) {
    if (scale < 1 || scale > 30 || nsamples < 0) return NULL;
    nthreads = gg_threads(nthreads);
    gg_rmat_ctx ctx;
    ctx.scale = scale;
    ctx.seed = seed;
    ctx.ta = gg_thresh(a);
    ctx.tab = gg_thresh(a + b);
    ctx.tabc = gg_thresh(a + b + c);
    ctx.pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsamples > 0 ? nsamples : 1));
    ctx.pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsamples > 0 ? nsamples : 1));
    gg_parallel_for(nthreads, nsamples, 1 << 14, gg_rmat_body, &ctx);
    int64_t n = (int64_t)1 << scale;
    gg_graph *g = gg_build_csr(n, nsamples, ctx.pu, ctx.pv, seed ^ 0xA5A5A5A5DEADBEEFULL, nthreads);
    free(ctx.pu);
    free(ctx.pv);
    return g;
}

/* ------------------------------------------------------------------ */
/* Chung-Lu (Chung and Lu 2002) with power-law weights                  */
/*   w_i = c (i+1)^(-1/(gamma-1)), capped at wcap, c bisected so that    */
/*   mean(w) = dbar;  p_ij = min(1, w_i w_j / sum(w)).                   */
/* exact=1: one Bernoulli draw per pair (O(n^2));                        */
/* exact=0: Miller-Hagberg skip sampling ("Efficient generation of       */
/*          networks with given expected degrees", WAW 2011), O(n + m).  */
/* ------------------------------------------------------------------ */
static void gg_cl_weights(int64_t n, double dbar, double gamma, double wcap, double *w) {
    double ex = -1.0 / (gamma - 1.0);
    double lo = 0.0, hi = dbar * 4.0 + 1.0;
    /* grow hi until the mean reaches dbar (capped weights saturate at wcap) */
    for (int it = 0; it < 200; ++it) {
        double s = 0;
        for (int64_t i = 0; i < n; ++i) {
            double x = hi * pow((double)(i + 1), ex);
            s += x < wcap ? x : wcap;
        }
        if (s / (double)n >= dbar) break;
        hi *= 2.0;
    }
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), s = 0;
        for (int64_t i = 0; i < n; ++i) {
            double x = mid * pow((double)(i + 1), ex);
            s += x < wcap ? x : wcap;
        }
        if (s / (double)n < dbar) lo = mid; else hi = mid;
    }
    double cc = 0.5 * (lo + hi);
    for (int64_t i = 0; i < n; ++i) {
        double x = cc * pow((double)(i + 1), ex);
        w[i] = x < wcap ? x : wcap;
    }
}

typedef struct {
    int64_t n;
    const double *w;
    double S;
    uint64_t seed;
    int exact;
    /* per-row output, two passes: count then fill */
    int64_t *cnt;
    int64_t *off;
    int32_t *pu, *pv;
    int fill;
} gg_cl_ctx;

static void gg_cl_row(gg_cl_ctx *c, int64_t u) {
    gg_rng r;
    gg_rng_init(&r, c->seed, (uint64_t)u);
    int64_t k = 0;
    int64_t base = c->fill ? c->off[u] : 0;
    const double *w = c->w;
    if (c->exact) {
        for (int64_t v = u + 1; v < c->n; ++v) {
            double p = w[u] * w[v] / c->S;
            if (p > 1.0) p = 1.0;
            double x = (double)gg_u32(&r) * (1.0 / 4294967296.0);
            if (x < p) {
                if (c->fill) {
                    c->pu[base + k] = (int32_t)u;
                    c->pv[base + k] = (int32_t)v;
                }
                ++k;
            }
        }
    } else {
        int64_t v = u + 1;
        double p = 1.0;
        if (v < c->n) {
            p = w[u] * w[v] / c->S;
            if (p > 1.0) p = 1.0;
        }
        while (v < c->n && p > 0) {
            if (p != 1.0) {
                double x = gg_unif(&r);
                double skip = floor(log(x) / log1p(-p));
                if (skip > (double)(c->n)) break;
                v += (int64_t)skip;
            }
            if (v < c->n) {
                double q = w[u] * w[v] / c->S;
                if (q > 1.0) q = 1.0;
                double x = gg_unif(&r);
                if (x < q / p) {
                    if (c->fill) {
                        c->pu[base + k] = (int32_t)u;
                        c->pv[base + k] = (int32_t)v;
                    }
                    ++k;
                }
                p = q;
                ++v;
            }
        }
    }
    if (!c->fill) c->cnt[u] = k;
}

static void gg_cl_body(void *arg, int64_t lo, int64_t hi) {
    gg_cl_ctx *c = (gg_cl_ctx *)arg;
    for (int64_t u = lo; u < hi; ++u) gg_cl_row(c, u);
}

gg_graph *gg_chung_lu(int64_t n, double dbar, double gamma, double wcap, int exact, uint64_t seed,
                      int nthreads) {
    if (n < 2 || n > 0x7FFFFFFF || gamma <= 1.0 || dbar <= 0) return NULL;
    nthreads = gg_threads(nthreads);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (wcap <= 0) wcap = sqrt((double)n * dbar);
    gg_cl_weights(n, dbar, gamma, wcap, w);
    double S = 0;
    for (int64_t i = 0; i < n; ++i) S += w[i];
    gg_cl_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n;
    c.w = w;
    c.S = S;
    c.seed = seed;
    c.exact = exact;
    c.cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    c.fill = 0;
    /* rows near 0 carry most pairs; small chunks keep threads balanced */
    gg_parallel_for(nthreads, n, exact ? 16 : 256, gg_cl_body, &c);
    c.off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    c.off[0] = 0;
    for (int64_t u = 0; u < n; ++u) c.off[u + 1] = c.off[u] + c.cnt[u];
    int64_t m = c.off[n];
    c.pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    c.pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    c.fill = 1;
    gg_parallel_for(nthreads, n, exact ? 16 : 256, gg_cl_body, &c);
    gg_graph *g = gg_build_csr(n, m, c.pu, c.pv, seed ^ 0x5EED5EED12345678ULL, nthreads);
    free(c.pu);
    free(c.pv);
    free(c.off);
    free(c.cnt);
    free(w);
    return g;
}

/* Erdos-Renyi G(n, p) with one Bernoulli draw per pair (small test graphs). */
gg_graph *gg_gnp(int64_t n, double p, uint64_t seed) {
    if (n < 1 || n > 100000) return NULL;
    int64_t cap = n * (n - 1) / 2;
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    int64_t m = 0;
    gg_rng r;
    gg_rng_init(&r, seed, 7);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t v = u + 1; v < n; ++v) {
            double x = (double)gg_u32(&r) * (1.0 / 4294967296.0);
            if (x < p) {
                pu[m] = (int32_t)u;
                pv[m] = (int32_t)v;
                ++m;
            }
        }
    gg_graph *g = gg_build_csr(n, m, pu, pv, seed ^ 0x0BADC0DE0BADC0DEULL, 1);
    free(pu);
    free(pv);
    return g;
}

/* Clean CSR from caller-supplied pairs (used for named test graphs). */
gg_graph *gg_from_pairs(int64_t n, int64_t m, const int32_t *pu, const int32_t *pv, uint64_t perm_seed,
                        int permute) {
    if (n < 1) return NULL;
    for (int64_t i = 0; i < m; ++i)
        if (pu[i] < 0 || pu[i] >= n || pv[i] < 0 || pv[i] >= n) return NULL;
    if (permute) return gg_build_csr(n, m, pu, pv, perm_seed, 1);
    /* identity relabel */
    gg_build_ctx c;
    memset(&c, 0, sizeof(c));
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) id[i] = (int32_t)i;
    c.npairs = m;
    c.pu = pu;
    c.pv = pv;
    c.perm = id;
    c.deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    gg_count_body(&c, 0, m);
    c.rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    c.rp[0] = 0;
    for (int64_t u = 0; u < n; ++u) c.rp[u + 1] = c.rp[u] + c.deg[u];
    int64_t tot = c.rp[n];
    c.col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    for (int64_t u = 0; u < n; ++u) c.deg[u] = c.rp[u];
    gg_fill_body(&c, 0, m);
    c.newdeg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    gg_sort_body(&c, 0, n);
    int64_t *rp2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    rp2[0] = 0;
    for (int64_t u = 0; u < n; ++u) rp2[u + 1] = rp2[u] + c.newdeg[u];
    for (int64_t u = 0; u < n; ++u)
        if (rp2[u] != c.rp[u])
            memmove(c.col + rp2[u], c.col + c.rp[u], sizeof(int32_t) * (size_t)c.newdeg[u]);
    gg_graph *g = (gg_graph *)malloc(sizeof(gg_graph));
    g->n = n;
    g->nnz = rp2[n];
    g->rp = rp2;
    g->col = c.col;
    free(c.rp);
    free(c.deg);
    free(c.newdeg);
    free(id);
    return g;
}
