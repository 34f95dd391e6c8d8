/*
 * Fast kernels of the planted-cluster input generator (sampling and CSC
 * assembly only; no clustering arithmetic).  Loaded by mclgen/planted.py.
 *
 * Random numbers: each cluster draws from its own SplitMix64 stream (Steele,
 * Lea and Flood, OOPSLA 2014) seeded from (seed, cluster id), so the output is
 * independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
typedef struct { uint64_t s; } rng_t;
static inline uint64_t rng_next(rng_t *r) { r->s += GAMMA; return mix64(r->s); }
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }
/* number of trials up to and including the first success, p in (0,1) */
static inline int64_t rng_geom(rng_t *r, double log1mp)
{
    double u = rng_u01(r);                      /* [0,1) */
    double g = floor(log1p(-u) / log1mp);       /* failures before success */
    if (g > 9.0e18) g = 9.0e18;
    return (int64_t)g + 1;
}
static inline rng_t stream(uint64_t seed, uint64_t id)
{
    rng_t r = { mix64(seed + GAMMA * (id + 1)) ^ 0x5851F42D4C957F2DULL };
    return r;
}

/* Intra-cluster edges: every unordered pair (a < b) of cluster c is an edge
 * with probability p (geometric skipping), weight U(wlo, whi).  Positions are
 * mapped to vertex ids through perm[cstart[c] + a].  If `u` is NULL only the
 * per-cluster counts are written; otherwise edges are written from offs[c]. */
void gen_intra(int64_t ncl, const int64_t *sizes, const int64_t *cstart, const int64_t *perm,
               double p, uint64_t seed, double wlo, double whi,
               int64_t *counts, const int64_t *offs, int32_t *u, int32_t *v, double *w)
{
    double log1mp = log1p(-p);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < ncl; ++c) {
        int64_t s = sizes[c];
        rng_t r = stream(seed, (uint64_t)c);
        int64_t a = 0, b = 0, cnt = 0;   /* current pair (a, b); b = a means "before row start" */
        if (s < 2) { counts[c] = 0; continue; }
        for (;;) {
            int64_t g = (p >= 1.0) ? 1 : rng_geom(&r, log1mp);
            b += g;
            while (b >= s) {                   /* spill into the next rows */
                int64_t over = b - s;
                ++a;
                if (a >= s - 1) break;
                b = a + 1 + over;
            }
            if (a >= s - 1) break;
            if (u) {
                int64_t o = offs[c] + cnt;
                u[o] = (int32_t)perm[cstart[c] + a];
                v[o] = (int32_t)perm[cstart[c] + b];
                w[o] = wlo + (whi - wlo) * rng_u01(&r);
            } else {
                (void)rng_u01(&r);             /* keep the stream identical in both passes */
            }
            ++cnt;
        }
        counts[c] = cnt;
    }
}

static int cmp_rw(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

typedef struct { int32_t row; int32_t pad; double w; } rw_t;

/* Symmetrise E undirected edges into CSC with a self-loop per column whose
 * weight is the column's largest off-diagonal weight (1.0 if none).
 * colptr must have n+1 entries; rowidx/val must hold 2E+n entries. */
void gen_assemble(int64_t n, int64_t E, const int32_t *eu, const int32_t *ev, const double *ew,
                  int64_t *colptr, int32_t *rowidx, double *val)
{
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        #pragma omp atomic
        deg[eu[e]]++;
        #pragma omp atomic
        deg[ev[e]]++;
    }
    colptr[0] = 0;
    for (int64_t j = 0; j < n; ++j) colptr[j + 1] = colptr[j] + deg[j] + 1;
    int64_t *cur = deg;
    for (int64_t j = 0; j < n; ++j) cur[j] = colptr[j];
    rw_t *tmp = (rw_t *)malloc(sizeof(rw_t) * (size_t)(colptr[n] > 0 ? colptr[n] : 1));
    /* placement inside a column depends on the thread schedule; the per-column
       sort below makes the result independent of it (rows are unique) */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        int64_t pa, pb;
        #pragma omp atomic capture
        pa = cur[eu[e]]++;
        #pragma omp atomic capture
        pb = cur[ev[e]]++;
        rw_t a = { ev[e], 0, ew[e] }, b = { eu[e], 0, ew[e] };
        tmp[pa] = a;        /* column eu[e], row ev[e] */
        tmp[pb] = b;
    }
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < n; ++j) {
        int64_t lo = colptr[j], hi = colptr[j + 1] - 1;   /* last slot: self-loop */
        double mx = 0.0;
        for (int64_t q = lo; q < hi; ++q) if (tmp[q].w > mx) mx = tmp[q].w;
        rw_t self = { (int32_t)j, 0, mx > 0.0 ? mx : 1.0 };
        tmp[hi] = self;
        qsort(tmp + lo, (size_t)(hi - lo + 1), sizeof(rw_t), cmp_rw);
        for (int64_t q = lo; q <= hi; ++q) { rowidx[q] = tmp[q].row; val[q] = tmp[q].w; }
    }
    free(tmp);
    free(deg);
}
