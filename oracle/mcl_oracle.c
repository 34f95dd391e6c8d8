/*
 * Plain FP64 CPU oracle for one Markov-clustering (MCL) iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is compared against.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code with the GPU library: the sparse product uses a dense
 * sparse-accumulator (SPA) with a touched-row list, thresholds come from full
 * per-column sorts, and sums run sequentially in ascending row order.
 *
 * Matrices are CSC: int64 colptr[ncols+1], int32 rowidx (ascending, unique
 * within a column), double val.  Every parallel loop is over independent
 * columns, so results do not depend on the thread count.
 *
 * Paper sections followed (arXiv 2002.10083):
 *   - Alg. 1 (overview of MCL): column-stochastic start, expansion B = A A,
 *     pruning with a threshold and top-k per column, inflation as a Hadamard
 *     power, loop while the matrix changes.
 *   - Section 2, "Notations": flops(AB) = sum_j sum_{i in inds(B_*j)} nnz(A_*i).
 *   - Section 5 (probabilistic memory requirement estimation): Cohen's
 *     exponential-key estimator with r keys, estimate (r-1)/sum of keys.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* column-stochastic normalisation (Alg. 1, first step)                */
/* ------------------------------------------------------------------ */
void orc_normalize(int64_t ncols, const int64_t *colptr, const double *val_in,
                   double *val_out)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < ncols; ++j) {
        double s = 0.0;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) s += val_in[p];
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p)
            val_out[p] = (s > 0.0) ? val_in[p] / s : 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* expansion: C = A B, column by column with a dense accumulator       */
/* (Alg. 1 expansion step; flops as defined in Section 2)              */
/* ------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Pass 1: per output column, the number of distinct rows and the flops. */
void orc_expand_count(int64_t a_nrows, int64_t b_ncols,
                      const int64_t *a_colptr, const int32_t *a_rowidx,
                      const int64_t *b_colptr, const int32_t *b_rowidx,
                      int64_t *nnz_out, int64_t *flops_out)
{
    #pragma omp parallel
    {
        int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(a_nrows > 0 ? a_nrows : 1));
        for (int64_t i = 0; i < a_nrows; ++i) stamp[i] = -1;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < b_ncols; ++j) {
            int64_t cnt = 0, fl = 0;
            for (int64_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
                int64_t k = b_rowidx[p];
                fl += a_colptr[k + 1] - a_colptr[k];
                for (int64_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                    int32_t i = a_rowidx[q];
                    if (stamp[i] != j) { stamp[i] = j; ++cnt; }
                }
            }
            nnz_out[j] = cnt;
            flops_out[j] = fl;
        }
        free(stamp);
    }
}

/* Pass 2: values.  For column j, the nonzeros b_kj are visited in ascending k
 * and every a_ik of column k is accumulated as spa[i] = spa[i] + a_ik * b_kj
 * (the product rounded to double, then added; the first touch of row i starts
 * from 0.0; built without floating-point contraction).  The touched rows are then
 * sorted ascending.  c_colptr must hold the exclusive prefix sum of pass 1. */
void orc_expand_fill(int64_t a_nrows, int64_t b_ncols,
                     const int64_t *a_colptr, const int32_t *a_rowidx, const double *a_val,
                     const int64_t *b_colptr, const int32_t *b_rowidx, const double *b_val,
                     const int64_t *c_colptr, int32_t *c_rowidx, double *c_val)
{
    #pragma omp parallel
    {
        size_t n = (size_t)(a_nrows > 0 ? a_nrows : 1);
        double *spa = (double *)malloc(sizeof(double) * n);
        int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * n);
        for (int64_t i = 0; i < a_nrows; ++i) stamp[i] = -1;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < b_ncols; ++j) {
            int32_t *touched = c_rowidx + c_colptr[j];
            int64_t cnt = 0;
            for (int64_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
                int64_t k = b_rowidx[p];
                double bkj = b_val[p];
                for (int64_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                    int32_t i = a_rowidx[q];
                    if (stamp[i] != j) { stamp[i] = j; spa[i] = 0.0; touched[cnt++] = i; }
                    spa[i] = spa[i] + a_val[q] * bkj;
                }
            }
            qsort(touched, (size_t)cnt, sizeof(int32_t), cmp_i32);
            for (int64_t t = 0; t < cnt; ++t) c_val[c_colptr[j] + t] = spa[touched[t]];
        }
        free(spa);
        free(stamp);
    }
}

/* ------------------------------------------------------------------ */
/* prune / recover / select (Alg. 1 prune step)                        */
/* ------------------------------------------------------------------ */
static int cmp_desc_f64(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Per column j of B (m = nnz(B_*j)):
 *   nP = #{b >= theta}, mP = sum of those, mB = sum of the column
 *   (both summed in ascending row order);
 *   recover  if R > 0 and nP < R and mP < pct * mB: t = R-th largest value
 *            (0 when m < R, i.e. the whole column is kept);
 *   select   else if S > 0 and nP > S: t = S-th largest value;
 *   threshold otherwise: t = theta.
 * Every entry with b >= t is kept, so ties at the k-th value are all kept.
 * Outputs the threshold, the mode (0 threshold, 1 recover, 2 select), the kept
 * count and the decision inputs (nP, mP, mB) per column. */
void orc_prune_plan(int64_t ncols, const int64_t *colptr, const double *val,
                    double theta, int64_t S, int64_t R, double pct,
                    double *thr_out, int32_t *mode_out, int64_t *kept_out,
                    int64_t *np_out, double *mp_out, double *mb_out)
{
    #pragma omp parallel
    {
        double *buf = NULL;
        int64_t cap = 0;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < ncols; ++j) {
            int64_t a = colptr[j], m = colptr[j + 1] - colptr[j];
            int64_t nP = 0;
            double mP = 0.0, mB = 0.0;
            for (int64_t p = 0; p < m; ++p) {
                double b = val[a + p];
                mB += b;
                if (b >= theta) { ++nP; mP += b; }
            }
            double t = theta;
            int32_t mode = 0;
            int recover = (R > 0) && (nP < R) && (mP < pct * mB);
            int select = !recover && (S > 0) && (nP > S);
            if (recover || select) {
                int64_t k = recover ? R : S;
                if (m > cap) { free(buf); cap = m; buf = (double *)malloc(sizeof(double) * (size_t)cap); }
                memcpy(buf, val + a, sizeof(double) * (size_t)m);
                qsort(buf, (size_t)m, sizeof(double), cmp_desc_f64);
                if (recover) { mode = 1; t = (m >= k) ? buf[k - 1] : 0.0; }
                else         { mode = 2; t = buf[k - 1]; }
            }
            int64_t kept = 0;
            for (int64_t p = 0; p < m; ++p) kept += (val[a + p] >= t);
            thr_out[j] = t; mode_out[j] = mode; kept_out[j] = kept;
            np_out[j] = nP; mp_out[j] = mP; mb_out[j] = mB;
        }
        free(buf);
    }
}

/* Copy the kept entries (b >= thr[j]) into C; c_colptr is the prefix sum of
 * the kept counts. */
void orc_prune_fill(int64_t ncols, const int64_t *colptr, const int32_t *rowidx,
                    const double *val, const double *thr,
                    const int64_t *c_colptr, int32_t *c_rowidx, double *c_val)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < ncols; ++j) {
        int64_t o = c_colptr[j];
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p)
            if (val[p] >= thr[j]) { c_rowidx[o] = rowidx[p]; c_val[o] = val[p]; ++o; }
    }
}

/* ------------------------------------------------------------------ */
/* inflation (Alg. 1 inflation step) followed by column re-normalisation */
/* ------------------------------------------------------------------ */
void orc_inflate(int64_t ncols, const int64_t *colptr, const double *val_in,
                 double r, double *val_out)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < ncols; ++j) {
        double s = 0.0;
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
            double c = val_in[p];
            double cr = (r == 2.0) ? c * c : pow(c, r);
            val_out[p] = cr;
            s += cr;
        }
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p)
            val_out[p] = (s > 0.0) ? val_out[p] / s : 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* change between successive iterates: max |a_new - a_old| over the     */
/* union of the two patterns, per column (the loop test of Alg. 1)      */
/* ------------------------------------------------------------------ */
void orc_delta(int64_t ncols,
               const int64_t *o_colptr, const int32_t *o_rowidx, const double *o_val,
               const int64_t *n_colptr, const int32_t *n_rowidx, const double *n_val,
               double *delta_out)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < ncols; ++j) {
        int64_t p = o_colptr[j], pe = o_colptr[j + 1];
        int64_t q = n_colptr[j], qe = n_colptr[j + 1];
        double d = 0.0;
        while (p < pe || q < qe) {
            double diff;
            if (q >= qe || (p < pe && o_rowidx[p] < n_rowidx[q])) { diff = fabs(o_val[p]); ++p; }
            else if (p >= pe || n_rowidx[q] < o_rowidx[p])       { diff = fabs(n_val[q]); ++q; }
            else { diff = fabs(n_val[q] - o_val[p]); ++p; ++q; }
            if (diff > d) d = diff;
        }
        delta_out[j] = d;
    }
}

/* ------------------------------------------------------------------ */
/* Cohen's probabilistic nnz estimator (Section 5)                      */
/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the t-th output of the
 * generator seeded with s is mix(s + (t + 1) * gamma). */
static const uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ULL;
static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static uint64_t sm_output(uint64_t seed, uint64_t t) { return sm_mix(seed + (t + 1) * SM_GAMMA); }

/* Key l of first-layer vertex (row) i in MCL iteration `iter`: the stream seed
 * is output `iter` of SplitMix64(seed), the uniform is output i*r+l of that
 * stream mapped to (0,1], and the key is -ln(U) ~ Exp(1) (lambda = 1). */
double orc_cohen_key(uint64_t seed, int64_t iter, int64_t i, int64_t l, int64_t r)
{
    uint64_t s = sm_output(seed, (uint64_t)iter);
    uint64_t x = sm_output(s, (uint64_t)i * (uint64_t)r + (uint64_t)l);
    double u = (double)((x >> 11) + 1ULL) * (1.0 / 9007199254740992.0);
    return -log(u);
}

/* est_j = (r - 1) / sum_l M_j(l) with m_k(l) = min_{i in A_*k} key(i,l) and
 * M_j(l) = min_{k in B_*j} m_k(l); columns that reach no row estimate 0. */
void orc_cohen_estimate(int64_t a_nrows, int64_t a_ncols, int64_t b_ncols,
                        const int64_t *a_colptr, const int32_t *a_rowidx,
                        const int64_t *b_colptr, const int32_t *b_rowidx,
                        int64_t r, uint64_t seed, int64_t iter, double *est_out)
{
    double *keys = (double *)malloc(sizeof(double) * (size_t)(a_nrows * r + 1));
    double *mk = (double *)malloc(sizeof(double) * (size_t)(a_ncols * r + 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < a_nrows; ++i)
        for (int64_t l = 0; l < r; ++l) keys[i * r + l] = orc_cohen_key(seed, iter, i, l, r);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < a_ncols; ++k)
        for (int64_t l = 0; l < r; ++l) {
            double m = INFINITY;
            for (int64_t q = a_colptr[k]; q < a_colptr[k + 1]; ++q) {
                double v = keys[(int64_t)a_rowidx[q] * r + l];
                if (v < m) m = v;
            }
            mk[k * r + l] = m;
        }
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < b_ncols; ++j) {
        double sum = 0.0;
        int reached = 1;
        for (int64_t l = 0; l < r; ++l) {
            double m = INFINITY;
            for (int64_t p = b_colptr[j]; p < b_colptr[j + 1]; ++p) {
                double v = mk[(int64_t)b_rowidx[p] * r + l];
                if (v < m) m = v;
            }
            if (!(m < INFINITY)) reached = 0;
            sum += m;
        }
        est_out[j] = reached ? (double)(r - 1) / sum : 0.0;
    }
    free(keys);
    free(mk);
}

/* ------------------------------------------------------------------ */
/* multiway merge of partial products (Section 4): per column a k-way   */
/* heap merge of the sorted lists; equal rows are summed in list order. */
/* ------------------------------------------------------------------ */
typedef struct { int32_t row; int32_t list; int64_t pos; } heap_item;

static int item_less(const heap_item *a, const heap_item *b)
{
    return (a->row < b->row) || (a->row == b->row && a->list < b->list);
}
static void heap_push(heap_item *h, int *n, heap_item it)
{
    int i = (*n)++;
    h[i] = it;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!item_less(&h[i], &h[p])) break;
        heap_item t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}
static heap_item heap_pop(heap_item *h, int *n)
{
    heap_item top = h[0];
    h[0] = h[--(*n)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        if (l < *n && item_less(&h[l], &h[s])) s = l;
        if (r < *n && item_less(&h[r], &h[s])) s = r;
        if (s == i) break;
        heap_item t = h[i]; h[i] = h[s]; h[s] = t; i = s;
    }
    return top;
}

/* nparts lists given as arrays of pointers.  If `fill` is 0 only the merged
 * counts are produced (c_colptr ignored); otherwise rows and values are
 * written at c_colptr. */
void orc_merge(int64_t ncols, int32_t nparts,
               const int64_t *const *colptrs, const int32_t *const *rowidxs,
               const double *const *vals, int fill,
               int64_t *count_out, const int64_t *c_colptr, int32_t *c_rowidx, double *c_val)
{
    #pragma omp parallel
    {
        heap_item *h = (heap_item *)malloc(sizeof(heap_item) * (size_t)(nparts + 1));
        #pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < ncols; ++j) {
            int n = 0;
            for (int32_t l = 0; l < nparts; ++l) {
                int64_t a = colptrs[l][j];
                if (a < colptrs[l][j + 1]) {
                    heap_item it = { rowidxs[l][a], l, a };
                    heap_push(h, &n, it);
                }
            }
            int64_t cnt = 0, o = fill ? c_colptr[j] : 0;
            int32_t last = -1;
            while (n > 0) {
                heap_item it = heap_pop(h, &n);
                double v = vals[it.list][it.pos];
                if (it.row != last) {
                    if (fill) { c_rowidx[o + cnt] = it.row; c_val[o + cnt] = v; }
                    ++cnt;
                    last = it.row;
                } else if (fill) {
                    c_val[o + cnt - 1] += v;
                }
                int64_t nx = it.pos + 1;
                if (nx < colptrs[it.list][j + 1]) {
                    heap_item nt = { rowidxs[it.list][nx], it.list, nx };
                    heap_push(h, &n, nt);
                }
            }
            count_out[j] = cnt;
        }
        free(h);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel loops (results do not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
