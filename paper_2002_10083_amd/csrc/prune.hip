// Stand-alone prune, inflation and normalisation kernels (Alg. 1 of
// arXiv 2002.10083) on explicit CSC matrices.  One wavefront per column, four
// columns per workgroup.  Sums use the same fixed tree as the fused
// iteration kernel (64-entry butterfly blocks, block sums accumulated by lane
// in order, then a butterfly over lanes), so prune decisions and inflated
// values are bit-identical to the fused path.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace mcl {

namespace {

// Fixed-tree sums over positions 0..m-1 of get(p) and of the entries >= theta,
// computed by one wave without block storage: lane (b mod 64) accumulates the
// sum of block b, in increasing b.
template <typename Get>
__device__ void wave_prune_sums(Get get, int m, double theta, double *mB, double *mP, int *nP)
{
    double accB = 0.0, accP = 0.0;
    int cnt = 0;
    const int nblk = (m + WAVE - 1) / WAVE;
    for (int b = 0; b < nblk; ++b) {
        const int p = b * WAVE + lane();
        const double v = (p < m) ? get(p) : 0.0;
        const bool ab = (p < m) && (v >= theta);
        const double sB = wave_sum(v);
        const double sP = wave_sum(ab ? v : 0.0);
        cnt += __popcll(ballot(ab));
        if (lane() == (b & (WAVE - 1))) { accB += sB; accP += sP; }
    }
    *mB = wave_sum(accB);
    *mP = wave_sum(accP);
    *nP = cnt;
}

template <typename Get>
__device__ double wave_fixed_sum(Get get, int m)
{
    double acc = 0.0;
    const int nblk = (m + WAVE - 1) / WAVE;
    for (int b = 0; b < nblk; ++b) {
        const int p = b * WAVE + lane();
        const double s = wave_sum((p < m) ? get(p) : 0.0);
        if (lane() == (b & (WAVE - 1))) acc += s;
    }
    return wave_sum(acc);
}

// Exact k-th largest of get(p), p < m (positive doubles), by an MSD radix
// select over bit patterns; `hist` is this wave's 256-int LDS histogram.
template <typename Get>
__device__ double wave_kth_largest(Get get, int m, int kth, int *hist)
{
    uint64_t prefix = 0, pmask = 0;
    int kk = kth;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = lane(); i < 256; i += WAVE) hist[i] = 0;
        group_sync<WAVE>();
        for (int p = lane(); p < m; p += WAVE) {
            const uint64_t u = (uint64_t)__double_as_longlong(get(p));
            if ((u & pmask) == prefix) atomicAdd(&hist[(u >> shift) & 255], 1);
        }
        group_sync<WAVE>();
        const int l = lane();
        const int c0 = hist[4 * l], c1 = hist[4 * l + 1], c2 = hist[4 * l + 2], c3 = hist[4 * l + 3];
        int x = c0 + c1 + c2 + c3;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int y = __shfl_down(x, d, WAVE);
            if (l + d < WAVE) x += y;
        }
        int above = __shfl_down(x, 1, WAVE);
        if (l == WAVE - 1) above = 0;
        int dsel = 0, knew = 0;
        const bool mine = above < kk && kk <= x;
        if (mine) {
            const int cs[4] = {c3, c2, c1, c0};
            int ab = above;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (ab + cs[q] >= kk) { dsel = 4 * l + 3 - q; knew = kk - ab; break; }
                ab += cs[q];
            }
        }
        const uint64_t who = ballot(mine);
        const int src = __ffsll((long long)who) - 1;
        dsel = __shfl(dsel, src, WAVE);
        kk = __shfl(knew, src, WAVE);
        prefix |= (uint64_t)dsel << shift;
        pmask |= 255ull << shift;
        group_sync<WAVE>();
    }
    return __longlong_as_double((long long)prefix);
}

}  // namespace

// Per column: branch (0 threshold, 1 recover, 2 select), threshold and kept
// count, exactly as the fused iteration decides them.
__global__ __launch_bounds__(256) void k_prune_plan(DevCSC B, PruneArgs pa, double *__restrict__ thr,
                                                    int64_t *__restrict__ kept, int8_t *__restrict__ mode)
{
    __shared__ int hist[4][256];
    const int w = threadIdx.x / WAVE;
    const int64_t j = (int64_t)blockIdx.x * 4 + w;
    if (j >= B.ncols) return;
    const int64_t s = B.colptr[j];
    const int m = (int)(B.colptr[j + 1] - s);
    const double *v = B.val + s;
    auto get = [&](int p) { return v[p]; };
    double mB, mP;
    int nP;
    wave_prune_sums(get, m, pa.theta, &mB, &mP, &nP);
    int md = 0, kth = 0;
    double t = pa.theta;
    const bool rec = pa.R > 0 && nP < pa.R && mP < pa.pct * mB;
    const bool sel = !rec && pa.S > 0 && nP > pa.S;
    if (rec) {
        md = 1;
        if (m >= pa.R) kth = pa.R; else t = 0.0;
    } else if (sel) {
        md = 2;
        kth = pa.S;
    }
    if (kth > 0) t = wave_kth_largest(get, m, kth, hist[w]);
    int c = 0;
    for (int p = lane(); p < m; p += WAVE) c += (v[p] >= t) ? 1 : 0;
    c = wave_sum_i(c);
    if (lane() == 0) {
        thr[j] = t;
        kept[j] = c;
        if (mode) mode[j] = (int8_t)md;
    }
}

void launch_prune_plan(const DevCSC &B, const PruneArgs &pa, double *thr, int64_t *kept, int8_t *mode,
                       hipStream_t st)
{
    if (B.ncols == 0) return;
    hipLaunchKernelGGL(k_prune_plan, dim3((unsigned)((B.ncols + 3) / 4)), dim3(256), 0, st, B, pa, thr,
                       kept, mode);
}

// Order-preserving copy of the entries >= thr[j].
__global__ __launch_bounds__(256) void k_prune_fill(DevCSC B, const double *__restrict__ thr,
                                                    const int64_t *__restrict__ colptr,
                                                    int32_t *__restrict__ row, double *__restrict__ val)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= B.ncols) return;
    const int64_t s = B.colptr[j], e = B.colptr[j + 1];
    const double t = thr[j];
    int64_t o = colptr[j];
    for (int64_t base = s; base < e; base += WAVE) {
        const int64_t p = base + lane();
        const bool keep = (p < e) && (B.val[p] >= t);
        const uint64_t mk = ballot(keep);
        if (keep) {
            const int64_t q = o + popc_below(mk);
            row[q] = B.rowidx[p];
            val[q] = B.val[p];
        }
        o += __popcll(mk);
    }
}

void launch_prune_fill(const DevCSC &B, const double *thr, const int64_t *colptr, int32_t *row,
                       double *val, hipStream_t st)
{
    if (B.ncols == 0) return;
    hipLaunchKernelGGL(k_prune_fill, dim3((unsigned)((B.ncols + 3) / 4)), dim3(256), 0, st, B, thr,
                       colptr, row, val);
}

// In-place inflation: c -> c^r / sum(c^r) with the fixed tree.  err (device,
// nullable) receives max_j |sum_i a_ij - 1| through an atomic max on the bit
// pattern (non-negative doubles order like their bits).
__global__ __launch_bounds__(256) void k_inflate(int64_t ncols, const int64_t *__restrict__ colptr,
                                                 double *__restrict__ val, double r,
                                                 unsigned long long *__restrict__ err)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= ncols) return;
    const int64_t s = colptr[j];
    const int m = (int)(colptr[j + 1] - s);
    double *v = val + s;
    const double sum = wave_fixed_sum([&](int p) { return inflate_pow(v[p], r); }, m);
    for (int p = lane(); p < m; p += WAVE) {
        const double c = inflate_pow(v[p], r);
        v[p] = (sum > 0.0) ? c / sum : 0.0;
    }
    if (err) {
        group_sync<WAVE>();
        const double t = wave_fixed_sum([&](int p) { return v[p]; }, m);
        const double e = (m > 0) ? fabs(t - 1.0) : 0.0;
        if (lane() == 0) atomicMax(err, (unsigned long long)__double_as_longlong(e));
    }
}

void launch_inflate(int64_t ncols, const int64_t *colptr, double *val, double r, double *err,
                    hipStream_t st)
{
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_inflate, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, st, ncols, colptr,
                       val, r, (unsigned long long *)err);
}

// In-place column normalisation: a = w / sum(w) (fixed tree).
__global__ __launch_bounds__(256) void k_normalize(int64_t ncols, const int64_t *__restrict__ colptr,
                                                   double *__restrict__ val)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= ncols) return;
    const int64_t s = colptr[j];
    const int m = (int)(colptr[j + 1] - s);
    double *v = val + s;
    const double sum = wave_fixed_sum([&](int p) { return v[p]; }, m);
    for (int p = lane(); p < m; p += WAVE) v[p] = (sum > 0.0) ? v[p] / sum : 0.0;
}

void launch_normalize(int64_t ncols, const int64_t *colptr, double *val, hipStream_t st)
{
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_normalize, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, st, ncols, colptr,
                       val);
}

}  // namespace mcl
