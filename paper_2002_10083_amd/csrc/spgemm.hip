// Expansion kernels for gfx950: symbolic pass, Cohen estimate, column binning,
// per-bin hash-table SpGEMM with a fused prune / inflate / change epilogue,
// an HBM-table variant for the heaviest columns, and compaction.
//
// Expansion (arXiv 2002.10083, Alg. 1): column j of B = A*A gathers
// b_kj * A_*k for every nonzero b_kj of the column.  With CSC operands this is
// column-wise Gustavson, which is what the paper's CSC-native formulation
// computes (Section 3, "Sparse matrix storage format").  Work per column is
// flops_j = sum_{k in B_*j} nnz(A_*k) (Section 2, "Notations").
//
// One workgroup (or one wavefront) owns one output column and a private hash
// table of S slots (int32 row key + fp64 value) in LDS.  The nonzeros of B_*j
// are visited in ascending k and, for each, all entries of A_*k are inserted
// in parallel: rows inside one A_*k are distinct, so a k-step has no
// conflicts, and k-steps are separated by a barrier (or owned by a single
// wave, whose LDS operations complete in issue order).  Every output entry is
// therefore accumulated as acc = acc + (a_ik * b_kj) (product rounded to
// double, then one rounded add) in ascending k no
// matter how the table is laid out -- results are bit-identical across table
// sizes, bins and schedules.  The column is then sorted by row (bucket count
// + in-bucket rank) and either written (expand) or pruned, inflated and
// compared with the previous iterate in LDS (fused iteration).
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace mcl {

// ---------------------------------------------------------------------------
// bins
// ---------------------------------------------------------------------------
// Temp-buffer offsets: base >= 0 is an offset in the main temp region;
// base < 0 encodes -(1 + (region << 48 | offset)) for the fallback regions.
constexpr int64_t REGION_MASK = ((int64_t)1 << 48) - 1;
// Table slots per LDS bin and the maximum number of distinct keys it accepts
// (load factor 3/4; more keys flag the column as overflowed).
__host__ __device__ constexpr int bin_slots_c(int b) { return 128 << b; }
__host__ __device__ constexpr int bin_cap_c(int b) { return (3 * (128 << b)) / 4; }
// Largest columns (bin 7) in LDS, in concurrent workgroups: up to MP_SMALL
// keys 32 waves per column with two row groups each, up to MP_NARROW 64
// waves with one group each, both with 512-slot tables per wave; up to
// MP_MAX 64 waves with 1024-slot tables (4/5 of the tables' capacity:
// headroom for an uneven spread of rows over the waves).  Larger columns use
// HBM tables.
constexpr int64_t MP_SMALL = (int64_t)32 * ((13 * 512) / 16) * 4 / 5;
constexpr int64_t MP_NARROW = (int64_t)64 * ((13 * 512) / 16) * 4 / 5;
constexpr int64_t MP_MAX = (int64_t)64 * ((13 * 1024) / 16) * 4 / 5;
// Largest row span of a dense-accumulator column (see k_numeric_dense).
constexpr int DENSE_SPAN = 8192;
__host__ __device__ constexpr bool dense_shape(int64_t flops, int64_t span)
{
    return flops > 0 && span <= DENSE_SPAN && flops >= 2 * span;
}
// Keys a column may be planned with in bin b: bins of 1024+ slots split the
// column over waves with private tables, so they keep 1/8 headroom for an
// uneven spread of rows over the waves.
__host__ __device__ constexpr int plan_cap_c(int b) { return (b >= 3) ? (bin_cap_c(b) * 7) / 8 : bin_cap_c(b); }
int lds_bin_slots(int bin) { return bin_slots_c(bin); }
int lds_bin_cap(int bin) { return bin_cap_c(bin); }

// Per-lane minima of 16 key slots reduced over the 64 lanes with a
// transposed butterfly: at each of the first four steps a lane keeps half of
// its slots and receives the partner's values for them (8+4+2+1 exchanges),
// then two plain steps finish.  Afterwards lane l holds the minimum of slot
// cohen_slot(l) (the four lanes of a quad hold the same slot).
__device__ __forceinline__ float keymin_reduce(float (&v)[16])
{
#pragma unroll
    for (int h = 8, d = 32; h >= 1; h >>= 1, d >>= 1) {
        const bool up = (lane() & d) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const float send = up ? v[i] : v[i + h];
            const float keep = up ? v[i + h] : v[i];
            v[i] = fminf(keep, __shfl_xor(send, d, WAVE));
        }
    }
    float x = v[0];
    x = fminf(x, __shfl_xor(x, 2, WAVE));
    x = fminf(x, __shfl_xor(x, 1, WAVE));
    return x;
}
__device__ __forceinline__ int cohen_slot(int l)
{
    return ((l >> 5) & 1) * 8 + ((l >> 4) & 1) * 4 + ((l >> 3) & 1) * 2 + ((l >> 2) & 1);
}

// ---------------------------------------------------------------------------
// symbolic pass: flops, row span, Cohen finish, MLP features
// ---------------------------------------------------------------------------
// One wavefront per column j of B.  For every nonzero b_kj: len = nnz(A_*k),
// first and last row of A_*k, read from the column record of k (RS floats:
// RP key minima, then first row, last row, length).  Outputs flops_j, the
// row span [lo_j, hi_j] that bounds the product column, and (RP > 0)
// Cohen's estimate from the key minima, and 12 MLP features.
template <int RP>
__global__ __launch_bounds__(256) void k_symbolic(DevCSC A, DevCSC B, int64_t *__restrict__ flops,
                                                  int32_t *__restrict__ lo, int32_t *__restrict__ hi,
                                                  const float *__restrict__ rec, int r,
                                                  float *__restrict__ est, float *__restrict__ feat,
                                                  const int64_t *__restrict__ prev_nnz, int iteration)
{
    constexpr int RS = col_rec_stride_c(RP);
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= B.ncols) return;
    const int64_t bs = B.colptr[j], be = B.colptr[j + 1];
    int64_t fl = 0, sq = 0;
    int mn = INT32_MAX, mx = -1, lmax = 0, lmin = INT32_MAX;
    double bmax = 0.0, bsq = 0.0, wl = 0.0;
    float cm[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) cm[l] = INFINITY;
    for (int64_t p = bs + lane(); p < be; p += WAVE) {
        const int k = B.rowidx[p];
        const double b = B.val[p];
        const float *rk = rec + (int64_t)k * RS;
        const int4 info = *(const int4 *)(rk + RP);
        const int len = info.z;
        fl += len;
        sq += (int64_t)len * len;
        lmax = max(lmax, len);
        lmin = min(lmin, len);
        bmax = fmax(bmax, b);
        bsq += b * b;
        wl += b * (double)len;
        if (len > 0) {
            mn = min(mn, info.x);
            mx = max(mx, info.y);
        }
        if constexpr (RP > 0) {
            const float4 *cr = (const float4 *)rk;
#pragma unroll
            for (int q = 0; q < RP / 4; ++q) {
                const float4 x = cr[q];
                cm[4 * q + 0] = fminf(cm[4 * q + 0], x.x);
                cm[4 * q + 1] = fminf(cm[4 * q + 1], x.y);
                cm[4 * q + 2] = fminf(cm[4 * q + 2], x.z);
                cm[4 * q + 3] = fminf(cm[4 * q + 3], x.w);
            }
        }
    }
    fl = wave_sum_i64(fl);
    sq = wave_sum_i64(sq);
    mn = wave_min_i(mn);
    mx = wave_max_i(mx);
    lmax = wave_max_i(lmax);
    lmin = wave_min_i(lmin);
    bmax = wave_max(bmax);
    bsq = wave_sum(bsq);
    wl = wave_sum(wl);
    float esum = 0.f;
    bool reached = true;
    if constexpr (RP > 0) {
        // column minima per key (slot cohen_slot(lane) on every lane), then
        // the sum over the r keys, added in key order on lane 0
        const float v = keymin_reduce(cm);
#pragma unroll
        for (int l = 0; l < 16; ++l) {
            if (l < r) {
                const float vl = __shfl(v, ((l >> 3) & 1) * 32 + ((l >> 2) & 1) * 16 + ((l >> 1) & 1) * 8 +
                                               (l & 1) * 4, WAVE);
                if (!(vl < INFINITY)) reached = false;
                esum += vl;
            }
        }
    }
    if (lane() == 0) {
        flops[j] = fl;
        lo[j] = (mx >= 0) ? mn : 0;
        hi[j] = (mx >= 0) ? mx : 0;
        if (RP > 0 && est) est[j] = (reached && fl > 0) ? (float)(r - 1) / esum : 0.f;
        if (feat) {
            const int m = (int)(be - bs);
            const double mean = m ? (double)fl / m : 0.0;
            const double var = m ? fmax((double)sq / m - mean * mean, 0.0) : 0.0;
            float *f = feat + j * 12;
            f[0] = log1pf((float)m);
            f[1] = log1pf((float)fl);
            f[2] = log1pf((float)lmax);
            f[3] = log1pf((float)mean);
            f[4] = log1pf((float)(m ? lmin : 0));
            f[5] = (float)iteration;
            f[6] = log1pf((float)((mx >= 0) ? (mx - mn + 1) : 0));
            f[7] = (float)bmax;
            f[8] = (float)bsq;
            f[9] = log1pf((float)sqrt(var));
            f[10] = prev_nnz ? log1pf((float)prev_nnz[j]) : 0.f;
            f[11] = log1pf((float)wl);
        }
    }
}

void launch_symbolic(const DevCSC &A, const DevCSC &B, int64_t *flops, int32_t *lo, int32_t *hi,
                     const float *rec, int r, float *est, float *feat, const int64_t *prev_nnz,
                     int iteration, hipStream_t st)
{
    if (B.ncols == 0) return;
    const dim3 grid((unsigned)((B.ncols + 3) / 4));
#define MCL_SYM(RP_)                                                                                   \
    hipLaunchKernelGGL(k_symbolic<RP_>, grid, dim3(256), 0, st, A, B, flops, lo, hi, rec, r, est, feat, \
                       prev_nnz, iteration)
    switch (r > 0 ? cohen_stride(r) : 0) {
    case 0: MCL_SYM(0); break;
    case 4: MCL_SYM(4); break;
    case 8: MCL_SYM(8); break;
    case 12: MCL_SYM(12); break;
    default: MCL_SYM(16); break;
    }
#undef MCL_SYM
}


// ---------------------------------------------------------------------------
// Cohen's estimator (Section 5): exponential keys on the first layer (rows of
// A), minimum over each column of A, then over each column of B.
// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output t of the generator
// seeded with s is mix(s + (t+1) * gamma).  The stream of MCL iteration `it`
// is seeded with output `it` of SplitMix64(seed); key (i, l) uses output
// i*r + l of that stream, mapped to U in (0, 1], key = -ln U.
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t sm64_out(uint64_t seed, uint64_t t)
{
    return sm64_mix(seed + (t + 1) * 0x9E3779B97F4A7C15ull);
}

// Key l of row i is stored at keys[i*rp + l], rp = r rounded up to 4 (so a
// row's keys are 16-byte aligned); its value depends only on (seed,
// iteration, i*r + l).  Padding entries are +inf.
__global__ __launch_bounds__(256) void k_cohen_keys(int64_t nrows, int r, int rp, uint64_t seed, int it,
                                                    float *__restrict__ keys)
{
    const uint64_t s = sm64_out(seed, (uint64_t)it);
    const int64_t n = nrows * rp;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / rp;
        const int l = (int)(q - i * rp);
        float key = INFINITY;
        if (l < r) {
            const uint64_t x = sm64_out(s, (uint64_t)(i * r + l));
            const double u = (double)((x >> 11) + 1ull) * (1.0 / 9007199254740992.0);
            key = (float)(-log(u));
        }
        keys[q] = key;
    }
}

void launch_cohen_keys(int64_t nrows, int r, uint64_t seed, int iteration, float *keys,
                       hipStream_t st)
{
    if (nrows == 0) return;
    hipLaunchKernelGGL(k_cohen_keys, dim3(2048), dim3(256), 0, st, nrows, r, cohen_stride(r), seed, iteration,
                       keys);
}

// Column record of A_*k (RS floats): rec[k*RS + l] = min over rows i of A_*k
// of key(i, l) for l < RP (+inf past r), then first row, last row and
// length of the column (as ints).  One wave per column.
template <int RP>
__global__ __launch_bounds__(256) void k_cohen_colmin(DevCSC A, const float *__restrict__ keys, int r,
                                                      float *__restrict__ rec)
{
    constexpr int RS = col_rec_stride_c(RP);
    const int64_t k = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (k >= A.ncols) return;
    const int64_t a0 = A.colptr[k], a1 = A.colptr[k + 1];
    if (lane() == 0) {
        const int len = (int)(a1 - a0);
        *(int4 *)(rec + k * RS + RP) = make_int4(len ? A.rowidx[a0] : 0, len ? A.rowidx[a1 - 1] : 0, len, 0);
    }
    float cm[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) cm[l] = INFINITY;
    for (int64_t p = a0 + lane(); p < a1; p += WAVE) {
        const float4 *kr = (const float4 *)(keys + (int64_t)A.rowidx[p] * RP);
#pragma unroll
        for (int q = 0; q < RP / 4; ++q) {
            const float4 x = kr[q];
            cm[4 * q + 0] = fminf(cm[4 * q + 0], x.x);
            cm[4 * q + 1] = fminf(cm[4 * q + 1], x.y);
            cm[4 * q + 2] = fminf(cm[4 * q + 2], x.z);
            cm[4 * q + 3] = fminf(cm[4 * q + 3], x.w);
        }
    }
    const float v = keymin_reduce(cm);
    const int slot = cohen_slot(lane());
    if ((lane() & 3) == 0 && slot < RP) rec[k * RS + slot] = (slot < r) ? v : INFINITY;
}

void launch_cohen_colmin(const DevCSC &A, const float *keys, int r, float *rec, hipStream_t st)
{
    if (A.ncols == 0) return;
    const dim3 grid((unsigned)((A.ncols + 3) / 4));
    switch (cohen_stride(r)) {
    case 4: hipLaunchKernelGGL(k_cohen_colmin<4>, grid, dim3(256), 0, st, A, keys, r, rec); break;
    case 8: hipLaunchKernelGGL(k_cohen_colmin<8>, grid, dim3(256), 0, st, A, keys, r, rec); break;
    case 12: hipLaunchKernelGGL(k_cohen_colmin<12>, grid, dim3(256), 0, st, A, keys, r, rec); break;
    default: hipLaunchKernelGGL(k_cohen_colmin<16>, grid, dim3(256), 0, st, A, keys, r, rec); break;
    }
}

// Column records without key minima: first row, last row, length.
__global__ __launch_bounds__(256) void k_col_records(DevCSC A, float *__restrict__ rec)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.ncols;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a0 = A.colptr[k], a1 = A.colptr[k + 1];
        const int len = (int)(a1 - a0);
        *(int4 *)(rec + k * 4) = make_int4(len ? A.rowidx[a0] : 0, len ? A.rowidx[a1 - 1] : 0, len, 0);
    }
}

void launch_col_records(const DevCSC &A, float *rec, hipStream_t st)
{
    if (A.ncols == 0) return;
    const int64_t blocks = std::min<int64_t>((A.ncols + 255) / 256, 4096);
    hipLaunchKernelGGL(k_col_records, dim3((unsigned)blocks), dim3(256), 0, st, A, rec);
}


// ---------------------------------------------------------------------------
// planning: per column table size and bin
// ---------------------------------------------------------------------------
// need_j = the number of distinct keys the table must accept.  Columns whose
// exact-safe bound ub_j = min(flops_j, row span_j, nrows) fits the 1024-slot
// bin use the bound (no estimate, no overflow possible).  Larger columns use
// the estimate scaled by 1.3 * est_scale (clamped to ub_j).  The bin is the
// smallest LDS table whose capacity holds need_j; beyond 8192 slots the
// column goes to the HBM-table kernel (bin 7) sized by need_j.
// Wave-aggregated reservation in one of NC counters: the active lanes with
// `valid` and class c reserve consecutive positions of counters[c] with one
// atomic per class and wave.  Returns the lane's position (0 when !valid).
template <int NC>
__device__ __forceinline__ int wave_reserve(int32_t *counters, int c, bool valid)
{
    int pos = 0;
    for (int q = 0; q < NC; ++q) {
        const uint64_t m = ballot(valid && c == q);
        if (m == 0) continue;
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane() == leader) base = atomicAdd(&counters[q], __popcll(m));
        base = readlane_i(base, leader);
        if (valid && c == q) pos = base + popc_below(m);
    }
    return pos;
}

// Workgroup-aggregated reservation: the waves first combine their counts in
// LDS (lcnt, lbase: NC ints each), then every class costs one global atomic
// per workgroup and call.  Called by all threads of the workgroup.
template <int NC>
__device__ __forceinline__ int block_reserve(int32_t *counters, int c, bool valid, int32_t *lcnt, int32_t *lbase)
{
    if (threadIdx.x < NC) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const int wpos = wave_reserve<NC>(lcnt, c, valid);
    __syncthreads();
    if (threadIdx.x < NC) lbase[threadIdx.x] = lcnt[threadIdx.x] ? atomicAdd(&counters[threadIdx.x], lcnt[threadIdx.x]) : 0;
    __syncthreads();
    return valid ? lbase[c] + wpos : 0;
}

__global__ __launch_bounds__(256) void k_plan(int64_t ncols, const int64_t *__restrict__ flops,
                                              const int32_t *__restrict__ lo, const int32_t *__restrict__ hi,
                                              const float *__restrict__ est, int est_kind,
                                              double est_scale, int64_t nrows,
                                              const uint8_t *__restrict__ col_active,
                                              int32_t *__restrict__ bin, int64_t *__restrict__ capv,
                                              int32_t *__restrict__ bin_count,
                                              unsigned long long *__restrict__ max_global)
{
    // bin counts and the largest HBM-table size are combined per workgroup
    __shared__ int32_t lcnt[NUM_LDS_BINS + 1];
    __shared__ unsigned long long lmax;
    if (threadIdx.x <= NUM_LDS_BINS) lcnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) lmax = 0;
    __syncthreads();
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x; j0 < ncols; j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        const bool act = j < ncols && !(col_active && !col_active[j]);
        if (j < ncols && !act) { bin[j] = -1; capv[j] = 0; }
        if (!act) continue;
        const int64_t fl = flops[j];
        int64_t ub = fl;
        if (fl > 0) ub = min(ub, (int64_t)(hi[j] - lo[j] + 1));
        ub = min(ub, nrows);
        int64_t need = ub;
        bool try_lds = false;
        // a column for the dense accumulator is sized by its row span (exact-safe)
        const bool dense = fl > 0 && dense_shape(fl, (int64_t)(hi[j] - lo[j] + 1));
        if (est_kind != 0 && est && ub > plan_cap_c(2) && !dense) {
            double e = ceil(1.3 * est_scale * (double)est[j]);
            if (e < 1.0) e = 1.0;
            need = min(ub, (int64_t)e);
            // an estimate near the largest LDS table still tries LDS first
            try_lds = (double)est[j] <= 1.25 * plan_cap_c(NUM_LDS_BINS - 1);
        }
        int b = 0;
        while (b < NUM_LDS_BINS && plan_cap_c(b) < need) ++b;
        if (b == NUM_LDS_BINS && try_lds) b = NUM_LDS_BINS - 1;
        bin[j] = b;
        capv[j] = (b < NUM_LDS_BINS) ? bin_cap_c(b) : need;
        wave_reserve<NUM_LDS_BINS + 1>(lcnt, b, true);
        if (b == NUM_LDS_BINS) atomicMax(&lmax, (unsigned long long)need);
    }
    __syncthreads();
    if (threadIdx.x <= NUM_LDS_BINS && lcnt[threadIdx.x]) atomicAdd(&bin_count[threadIdx.x], lcnt[threadIdx.x]);
    if (threadIdx.x == 0 && lmax) atomicMax(max_global, lmax);
}

void launch_plan(int64_t ncols, const int64_t *flops, const int32_t *lo, const int32_t *hi,
                 const float *est, int est_kind, double est_scale, int64_t nrows,
                 const uint8_t *col_active, int32_t *bin, int64_t *capv, int32_t *bin_count,
                 int64_t *max_global, hipStream_t st)
{
    if (ncols == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((ncols + 255) / 256, 1024);
    hipLaunchKernelGGL(k_plan, dim3(grid), dim3(256), 0, st, ncols, flops, lo, hi, est, est_kind,
                       est_scale, nrows, col_active, bin, capv, bin_count,
                       (unsigned long long *)max_global);
}

// One phase of a phased product: columns [c0, c1) keep their bin and get
// their temp offset relative to the phase start; all others are disabled.
__global__ __launch_bounds__(256) void k_phase_plan(int64_t n, const int32_t *__restrict__ bin,
                                                    const int64_t *__restrict__ base, int64_t c0, int64_t c1,
                                                    int32_t *__restrict__ ph_bin, int64_t *__restrict__ ph_base,
                                                    int32_t *__restrict__ counts)
{
    __shared__ int32_t lcnt[NUM_LDS_BINS + 1];
    if (threadIdx.x <= NUM_LDS_BINS) lcnt[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x; j0 < n; j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        const int b = (j >= c0 && j < c1) ? bin[j] : -1;
        if (j < n) ph_bin[j] = b;
        if (b >= 0) ph_base[j] = base[j] - base[c0];
        wave_reserve<NUM_LDS_BINS + 1>(lcnt, b, b >= 0);
    }
    __syncthreads();
    if (threadIdx.x <= NUM_LDS_BINS && lcnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], lcnt[threadIdx.x]);
}

void launch_phase_plan(int64_t n, const int32_t *bin, const int64_t *base, int64_t c0, int64_t c1,
                       int32_t *ph_bin, int64_t *ph_base, int32_t *counts, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_phase_plan, dim3(grid), dim3(256), 0, st, n, bin, base, c0, c1, ph_bin, ph_base,
                       counts);
}

// Scatter the listed columns into per-bin lists by bin[j].
__global__ __launch_bounds__(256) void k_scatter_bins_list(const int32_t *__restrict__ list, int32_t n,
                                                           const int32_t *__restrict__ bin,
                                                           BinOffsets bin_off, int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ out)
{
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool valid = i < n;
        const int j = valid ? list[i] : 0;
        const int b = valid ? bin[j] : 0;
        const int pos = wave_reserve<NUM_LDS_BINS + 1>(cursor, b, valid);
        if (valid) out[bin_off.off[b] + pos] = j;
    }
}

void launch_scatter_bins_list(const int32_t *list, int32_t n, const int32_t *bin, const BinOffsets &off,
                              int32_t *cursor, int32_t *out, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_scatter_bins_list, dim3(grid), dim3(256), 0, st, list, n, bin, off, cursor, out);
}

// est_j = min(flops_j, row span_j, nrows): the exact-safe bound as an estimate.
__global__ void k_bound_estimate(int64_t n, const int64_t *__restrict__ flops, const int32_t *__restrict__ lo,
                                 const int32_t *__restrict__ hi, int64_t nrows, float *__restrict__ est)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t u = flops[j];
        if (u > 0) u = min(u, (int64_t)(hi[j] - lo[j] + 1));
        est[j] = (float)min(u, nrows);
    }
}

void launch_bound_estimate(int64_t n, const int64_t *flops, const int32_t *lo, const int32_t *hi,
                           int64_t nrows, float *est, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_bound_estimate, dim3(grid), dim3(256), 0, st, n, flops, lo, hi, nrows, est);
}

// Re-plan of columns that overflowed the largest LDS bin, from their exact
// product size m_j: the HBM table sized for m_j.
__global__ __launch_bounds__(256) void k_replan(const int32_t *__restrict__ list, int32_t n,
                                                const int64_t *__restrict__ exact,
                                                int32_t *__restrict__ bin, int64_t *__restrict__ capv,
                                                uint8_t *__restrict__ hbm_only,
                                                int32_t *__restrict__ bin_count,
                                                unsigned long long *__restrict__ max_global)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int j = list[i];
        const int64_t need = max(exact[j], (int64_t)1);
        const int b = NUM_LDS_BINS;
        bin[j] = b;
        capv[j] = need;
        hbm_only[j] = 1;
        atomicAdd(&bin_count[b], 1);  // few columns reach this path
        atomicMax(max_global, (unsigned long long)need);
    }
}

void launch_replan(const int32_t *list, int32_t n, const int64_t *exact, int32_t *bin, int64_t *capv,
                   uint8_t *hbm_only, int32_t *bin_count, int64_t *max_global, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_replan, dim3(grid), dim3(256), 0, st, list, n, exact, bin, capv, hbm_only, bin_count,
                       (unsigned long long *)max_global);
}

// Exact-safe bound ub_j = min(flops_j, row span_j, nrows) of the listed
// columns, written to ub[j]; the maximum goes to *max_ub.
__global__ __launch_bounds__(256) void k_list_bound(const int32_t *__restrict__ list, int32_t n,
                                                    const int64_t *__restrict__ flops,
                                                    const int32_t *__restrict__ lo,
                                                    const int32_t *__restrict__ hi, int64_t nrows,
                                                    int64_t *__restrict__ ub,
                                                    unsigned long long *__restrict__ max_ub)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int j = list[i];
        int64_t u = flops[j];
        if (u > 0) u = min(u, (int64_t)(hi[j] - lo[j] + 1));
        u = min(u, nrows);
        ub[j] = u;
        atomicMax(max_ub, (unsigned long long)u);
    }
}

void launch_list_bound(const int32_t *list, int32_t n, const int64_t *flops, const int32_t *lo,
                       const int32_t *hi, int64_t nrows, int64_t *ub, int64_t *max_ub, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_list_bound, dim3(grid), dim3(256), 0, st, list, n, flops, lo, hi, nrows, ub,
                       (unsigned long long *)max_ub);
}

// Temp offsets of the listed columns after the main region: base[j] =
// -(1 + offset) into the second temp buffer (prefix of capv over the list).
__global__ void k_list_base(const int32_t *__restrict__ list, int32_t n, const int64_t *__restrict__ capv,
                            int64_t *__restrict__ base, int64_t *__restrict__ total, int region)
{
    // single wave, sequential chunks of 64 (the list is short)
    int64_t run = 0;
    for (int c = 0; c < n; c += WAVE) {
        const int i = c + lane();
        const int64_t v = (i < n) ? capv[list[i]] : 0;
        int64_t x = v;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int64_t y = __shfl_up(x, d, WAVE);
            if (lane() >= d) x += y;
        }
        if (i < n) base[list[i]] = -(1 + (((int64_t)region << 48) | (run + x - v)));
        run += __shfl(x, WAVE - 1, WAVE);
    }
    if (lane() == 0) *total = run;
}

void launch_list_base(const int32_t *list, int32_t n, const int64_t *capv, int64_t *base, int64_t *total,
                      int region, hipStream_t st)
{
    hipLaunchKernelGGL(k_list_base, dim3(1), dim3(WAVE), 0, st, list, n, capv, base, total, region);
}

// Overflowed columns move one LDS bin up (twice the table); columns that
// overflowed the largest LDS bin are flagged for an exact count (bin 7).
// With force_exact every listed column is flagged for the exact count: a
// column that overflowed twice is sized from its exact product size, so the
// overflow rounds end after at most three launches of any column.
__global__ __launch_bounds__(256) void k_bump(const int32_t *__restrict__ list, int32_t n,
                                              int32_t *__restrict__ bin, int64_t *__restrict__ capv,
                                              int32_t *__restrict__ bin_count,
                                              int32_t *__restrict__ exact_list,
                                              int32_t *__restrict__ n_exact, int to_multipass,
                                              int round, const int64_t *__restrict__ exact_cnt)
{
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool valid = i < n;
        const int j = valid ? list[i] : 0;
        const int b = valid ? bin[j] : 0;
        const int64_t ex = (valid && exact_cnt && round <= 2) ? exact_cnt[j] : -1;
        int nb = b + 1;
        bool up;
        if (ex >= 0) {
            // the split kernels counted the column's keys: the smallest LDS
            // bin that holds them, else the multi-pass kernel at that size
            nb = 0;
            while (nb < NUM_LDS_BINS && bin_cap_c(nb) < ex) ++nb;
            up = nb < NUM_LDS_BINS || (to_multipass && ex <= MP_MAX);
            if (up) {
                bin[j] = nb;
                capv[j] = (nb < NUM_LDS_BINS) ? (int64_t)bin_cap_c(nb) : max(ex, (int64_t)1);
            }
        } else {
            // LDS bins move one up; the largest LDS bin moves to the
            // multi-pass kernel at its full capacity (when available); the
            // rest go to the exact count
            up = valid && round == 1 && (b + 1 < NUM_LDS_BINS || (to_multipass && b + 1 == NUM_LDS_BINS));
            if (up) {
                bin[j] = b + 1;
                capv[j] = (b + 1 < NUM_LDS_BINS) ? (int64_t)bin_cap_c(b + 1) : MP_NARROW;
            }
        }
        wave_reserve<NUM_LDS_BINS + 1>(bin_count, nb, up);
        const int pos = wave_reserve<1>(n_exact, 0, valid && !up);
        if (valid && !up) exact_list[pos] = j;
    }
}

void launch_bump(const int32_t *list, int32_t n, int32_t *bin, int64_t *capv, int32_t *bin_count,
                 int32_t *exact_list, int32_t *n_exact, bool to_multipass, int round,
                 const int64_t *exact_cnt, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_bump, dim3(grid), dim3(256), 0, st, list, n, bin, capv, bin_count, exact_list,
                       n_exact, (int)to_multipass, round, exact_cnt);
}

// Per-bin totals of the launched columns: flops, nnz(B_*j), output count.
__global__ __launch_bounds__(256) void k_bin_sums(const int32_t *__restrict__ lists, BinOffsets off,
                                                  BinOffsets cnt, const int64_t *__restrict__ flops,
                                                  const int64_t *__restrict__ bcolptr,
                                                  const int64_t *__restrict__ out_cnt,
                                                  const int64_t *__restrict__ prod,
                                                  unsigned long long *__restrict__ acc)
{
    const int b = blockIdx.y;
    int64_t f = 0, bn = 0, o = 0, pr = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt.off[b]; i += gridDim.x * blockDim.x) {
        const int j = lists[off.off[b] + i];
        f += flops[j];
        if (bcolptr) bn += bcolptr[j + 1] - bcolptr[j];
        const int64_t oc = max(out_cnt[j], (int64_t)0);
        o += oc;
        pr += (prod && out_cnt[j] >= 0) ? prod[j] : oc;
    }
    f = wave_sum_i64(f);
    bn = wave_sum_i64(bn);
    o = wave_sum_i64(o);
    pr = wave_sum_i64(pr);
    if (lane() == 0) {
        atomicAdd(&acc[4 * b + 0], (unsigned long long)f);
        atomicAdd(&acc[4 * b + 1], (unsigned long long)bn);
        atomicAdd(&acc[4 * b + 2], (unsigned long long)o);
        atomicAdd(&acc[4 * b + 3], (unsigned long long)pr);
    }
}

void launch_bin_sums(const int32_t *lists, const BinOffsets &off, const BinOffsets &cnt,
                     const int64_t *flops, const int64_t *bcolptr, const int64_t *out_cnt,
                     const int64_t *prod, int64_t *acc,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_bin_sums, dim3(64, 8), dim3(256), 0, st, lists, off, cnt, flops, bcolptr, out_cnt,
                       prod, (unsigned long long *)acc);
}

__global__ __launch_bounds__(256) void k_scatter_bins(int64_t ncols, const int32_t *__restrict__ bin,
                                                      BinOffsets bin_off, int32_t *__restrict__ cursor,
                                                      int32_t *__restrict__ lists)
{
    __shared__ int32_t lcnt[NUM_LDS_BINS + 1], lbase[NUM_LDS_BINS + 1];
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x; j0 < ncols; j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        const int b = (j < ncols) ? bin[j] : -1;
        const int pos = block_reserve<NUM_LDS_BINS + 1>(cursor, b, b >= 0, lcnt, lbase);
        if (b >= 0) lists[bin_off.off[b] + pos] = (int32_t)j;
    }
}

void launch_scatter_bins(int64_t ncols, const int32_t *bin, const BinOffsets &bin_off, int32_t *cursor,
                         int32_t *lists, hipStream_t st)
{
    if (ncols == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((ncols + 255) / 256, 1024);
    hipLaunchKernelGGL(k_scatter_bins, dim3(grid), dim3(256), 0, st, ncols, bin, bin_off, cursor,
                       lists);
}

// ---------------------------------------------------------------------------
// numeric column kernel (shared by the LDS bins and the HBM-table variant)
// ---------------------------------------------------------------------------
template <typename IdxT>
struct Scratch {
    int32_t *key;    // S slots
    double *val;     // S slots
    IdxT *list;      // cap: bucketed slots, later the kept list
    IdxT *sorted;    // cap: slots in ascending row order
    int *bcnt;       // NB bucket offsets
    int *bcur;       // NB bucket cursors
    double *p0, *p1; // per 64-block partial sums (cap/64 + 1)
    int *ip;         // per 64-block counts
    int *hist;       // 256-bin histogram
    int *misc;       // 16 ints: [0] nkeys [1] overflow [2..] broadcast
    double *dmisc;   // 4 doubles
    int *wsum;       // NT/64 ints for scans
};

// Open-addressing table of S slots organised as S/4 buckets of four int32
// keys (16-byte aligned).  A key lives in the first bucket, starting at its
// home bucket, that had a free slot when it was inserted; one 128-bit LDS read
// fetches a whole bucket, so a lookup is normally one read and four compares,
// and an insertion one compare-and-swap.  In LDS tables probing stops after
// PROBE_MAX bucket visits: the key is then reported as not placed (-1,
// overflow flag raised) and the column is recomputed with a larger table.
// Tables in HBM are sized from the exact count and probe every bucket if
// needed, so an insertion there fails only when the table is full.
constexpr int PROBE_MAX = 32;
typedef int32_t keys4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) keys4 lds_keys4;  // tables live in LDS

// acc += x for one table value (one correctly rounded add), by the lane that
// owns the slot in this step; the read and the write of one wave apply in
// issue order.
template <bool LDS>
__device__ __forceinline__ void table_add(double *acc, double x)
{
    if constexpr (LDS) {
        auto *p = (__attribute__((address_space(3))) double *)acc;
        *p = *p + x;
    } else {
        *acc = *acc + x;
    }
}

// acc += x as a fire-and-forget LDS atomic add (one correctly rounded add).
// Only used on tables private to one wave, where lanes of one instruction
// never share a slot and successive instructions apply in issue order.
__device__ __forceinline__ void lds_atomic_add(double *acc, double x)
{
    __hip_atomic_fetch_add((__attribute__((address_space(3))) double *)acc, x, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int bucket_match(const keys4 kb, int32_t k)
{
    return (kb.x == k) ? 0 : (kb.y == k) ? 1 : (kb.z == k) ? 2 : (kb.w == k) ? 3 : -1;
}

// First free slot of the bucket, or -1 when it is full.  The slots of a
// bucket are claimed in order (an insertion takes the first free one), so
// the occupied slots form a prefix; a torn or stale view only makes the
// compare-and-swap fail and the insertion look again.
__device__ __forceinline__ int bucket_empty(const keys4 kb)
{
    const int occ = (kb.x != EMPTY_KEY ? 1 : 0) + (kb.y != EMPTY_KEY ? 1 : 0) + (kb.z != EMPTY_KEY ? 1 : 0) +
                    (kb.w != EMPTY_KEY ? 1 : 0);
    return occ < 4 ? occ : -1;
}

// Read bucket b.  LDS tables use one 128-bit LDS read; tables in HBM (the
// largest columns) read the four words as workgroup-scope atomics, so slots
// claimed by other waves of the workgroup are seen.
template <bool LDS>
__device__ __forceinline__ keys4 load_bucket(const int32_t *key, uint32_t b)
{
    if constexpr (LDS) {
        return *(volatile const lds_keys4 *)(key + 4 * b);
    } else {
        keys4 r;
        int32_t *p = const_cast<int32_t *>(key + 4 * b);
        r.x = __hip_atomic_load(p + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        r.y = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        r.z = __hip_atomic_load(p + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        r.w = __hip_atomic_load(p + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return r;
    }
}

// Insert k starting at bucket b.  `fresh` is set when this call placed k
// (exactly one caller per key does).
template <bool LDS>
__device__ __forceinline__ int insert_from(int32_t *key, int32_t k, uint32_t b, int nbmask, int *ovf, bool &fresh)
{
    const int limit = LDS ? PROBE_MAX : nbmask + 1;
#pragma unroll 1
    for (int p = 0; p < limit; ++p) {
        const keys4 kb = load_bucket<LDS>(key, b);
        const int hit = bucket_match(kb, k);
        if (hit >= 0) return (int)(4 * b) + hit;
        const int e = bucket_empty(kb);
        if (e < 0) {
            b = (b + 1) & (uint32_t)nbmask;
            continue;
        }
        const int old = atomicCAS(&key[4 * b + e], EMPTY_KEY, k);
        fresh = old == EMPTY_KEY;
        if (old == EMPTY_KEY || old == k) return (int)(4 * b) + e;
        // another key took that slot: look at the same bucket again
    }
    *ovf = 1;
    return -1;
}

template <bool LDS>
__device__ __forceinline__ int find_or_insert(int32_t *key, int32_t k, int logNB, int nbmask, int *ovf,
                                              bool &fresh)
{
    return insert_from<LDS>(key, k, hash_slot(k, logNB), nbmask, ovf, fresh);
}

// The same insertion split in two, so that the first-bucket reads of many
// keys can be in flight together: the caller reads the home bucket b of k
// (load_bucket) and place_key() finishes the insertion from it (a stale
// bucket is harmless: a slot seen empty is claimed by compare-and-swap, and
// keys never move).
template <bool LDS>
__device__ __forceinline__ int place_key(int32_t *key, int32_t k, uint32_t b, keys4 kb, int nbmask, int *ovf,
                                         bool &fresh)
{
    const int hit = bucket_match(kb, k);
    if (hit >= 0) return (int)(4 * b) + hit;
    const int e = bucket_empty(kb);
    if (e >= 0) {
        const int old = atomicCAS(&key[4 * b + e], EMPTY_KEY, k);
        fresh = old == EMPTY_KEY;
        if (old == EMPTY_KEY || old == k) return (int)(4 * b) + e;
    }
    return insert_from<LDS>(key, k, b, nbmask, ovf, fresh);
}

// Lookup after all insertions (and a barrier): plain reads suffice.
template <bool LDS>
__device__ __forceinline__ int find_from(const int32_t *key, int32_t k, uint32_t b, int nbmask)
{
    const int limit = LDS ? PROBE_MAX : nbmask + 1;
#pragma unroll 1
    for (int p = 0; p < limit; ++p) {
        keys4 kb;
        if constexpr (LDS) kb = *(const lds_keys4 *)(key + 4 * b);
        else kb = *(const keys4 *)(key + 4 * b);
        const int hit = bucket_match(kb, k);
        if (hit >= 0) return (int)(4 * b) + hit;
        if (bucket_empty(kb) >= 0) return -1;
        b = (b + 1) & (uint32_t)nbmask;
    }
    return -1;
}

template <bool LDS>
__device__ __forceinline__ int find_slot(const int32_t *key, int32_t k, int logNB, int nbmask)
{
    return find_from<LDS>(key, k, hash_slot(k, logNB), nbmask);
}

__device__ __forceinline__ int bucket_of(int32_t k, int32_t lo, uint64_t mul, int NB)
{
    const int b = (int)(((uint64_t)(uint32_t)(k - lo) * mul) >> 32);
    return min(max(b, 0), NB - 1);
}

// Exact k-th largest (kth >= 1) of m positive doubles get(p), p < m, by an
// MSD radix select over their IEEE bit patterns (monotone for positive
// values), 8 bits per pass.  Once at most 64 values share the selected
// prefix, they are gathered and one wave ranks them by comparison.  Called by
// all NT threads of the group; hist holds 256 ints (reused for the gathered
// values).
template <int NT, bool GS, typename Get>
__device__ double radix_kth_largest(Get get, int m, int kth, int *hist, int *misc, double *dmisc)
{
    const int tid = threadIdx.x % NT;
    const bool w0 = tid < WAVE;
    uint64_t prefix = 0, pmask = 0;
    int kk = kth;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = tid; i < 256; i += NT) hist[i] = 0;
        group_sync<NT, GS>();
        for (int p = tid; p < m; p += NT) {
            const uint64_t u = (uint64_t)__double_as_longlong(get(p));
            if ((u & pmask) == prefix) atomicAdd(&hist[(u >> shift) & 255], 1);
        }
        group_sync<NT, GS>();
        if (w0) {
            // lane l owns digits 4l..4l+3; find digit d with
            // count(digits > d) < kk <= count(digits >= d)
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
            if (above < kk && kk <= x) {
                int dsel = 4 * l, knew = kk, csel = 0;
                const int cs[4] = {c3, c2, c1, c0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (above + cs[q] >= kk) { dsel = 4 * l + 3 - q; knew = kk - above; csel = cs[q]; break; }
                    above += cs[q];
                }
                misc[4] = dsel;
                misc[5] = knew;
                misc[12] = csel;  // values sharing the new prefix
                misc[13] = 0;
            }
        }
        group_sync<NT, GS>();
        const int d = misc[4];
        kk = misc[5];
        const int cand = misc[12];
        prefix |= (uint64_t)d << shift;
        pmask |= 255ull << shift;
        group_sync<NT, GS>();
        if (cand <= WAVE && shift > 0) {
            // gather the candidates' bit patterns (low words in hist[0, 64),
            // high words in hist[64, 128)), then the kk-th largest of them
            for (int p = tid; p < m; p += NT) {
                const uint64_t u = (uint64_t)__double_as_longlong(get(p));
                if ((u & pmask) == prefix) {
                    const int q = atomicAdd(&misc[13], 1);
                    hist[q] = (int)(uint32_t)u;
                    hist[WAVE + q] = (int)(uint32_t)(u >> 32);
                }
            }
            group_sync<NT, GS>();
            if (w0 && lane() < cand) {
                // positive doubles order like their bit patterns
                const uint64_t v = ((uint64_t)(uint32_t)hist[WAVE + lane()] << 32) | (uint32_t)hist[lane()];
                int gt = 0, ge = 0;
                for (int q = 0; q < cand; ++q) {
                    const uint64_t c = ((uint64_t)(uint32_t)hist[WAVE + q] << 32) | (uint32_t)hist[q];
                    gt += (c > v) ? 1 : 0;
                    ge += (c >= v) ? 1 : 0;
                }
                if (gt < kk && kk <= ge) dmisc[2] = __longlong_as_double((long long)v);  // ties write the same value
            }
            group_sync<NT, GS>();
            const double r = dmisc[2];
            group_sync<NT, GS>();
            return r;
        }
    }
    return __longlong_as_double((long long)prefix);
}

// Prune decision shared by the fused kernel and the stand-alone prune: the
// fixed-tree sums of the column (mB) and of its entries >= theta (mP), the
// count nP, and the resulting branch and threshold (recover / select /
// threshold).  get(p) returns the value at sorted position p < m.
template <int NT, bool GS, typename Get>
__device__ void prune_decide(Get get, int m, const PruneArgs &pa, double *p0, double *p1, int *ip,
                             int *hist, int *misc, double *dmisc, int *out_mode, double *out_t)
{
    const int tid = threadIdx.x % NT;
    const int w = tid / WAVE;
    constexpr int NWV = (NT + WAVE - 1) / WAVE;
    const int nblk = (m + WAVE - 1) / WAVE;
    for (int b = w; b < nblk; b += NWV) {
        const int p = b * WAVE + lane();
        const double v = (p < m) ? get(p) : 0.0;
        const bool ab = (p < m) && (v >= pa.theta);
        const double sB = wave_sum(v);
        const double sP = wave_sum(ab ? v : 0.0);
        const int c = __popcll(ballot(ab));
        if (lane() == 0) { p0[b] = sB; p1[b] = sP; ip[b] = c; }
    }
    group_sync<NT, GS>();
    if (tid < WAVE) {
        const double mB = fixed_tree_finish(p0, nblk);
        const double mP = fixed_tree_finish(p1, nblk);
        int nP = 0;
        for (int b = lane(); b < nblk; b += WAVE) nP += ip[b];
        nP = wave_sum_i(nP);
        int mode = 0, kth = 0;
        double t = pa.theta;
        const bool rec = pa.R > 0 && nP < pa.R && mP < pa.pct * mB;
        const bool sel = !rec && pa.S > 0 && nP > pa.S;
        if (rec) {
            mode = 1;
            if (m >= pa.R) kth = pa.R; else t = 0.0;
        } else if (sel) {
            mode = 2;
            kth = pa.S;
        }
        if (lane() == 0) { misc[2] = mode; misc[3] = kth; dmisc[0] = t; }
    }
    group_sync<NT, GS>();
    const int mode = misc[2], kth = misc[3];
    double t = dmisc[0];
    group_sync<NT, GS>();
    if (kth > 0) t = radix_kth_largest<NT, GS>(get, m, kth, hist, misc, dmisc);
    *out_mode = mode;
    *out_t = t;
}

// Sort the m keys of a table (S slots) by row: bucket count over the row
// span [lo, lo+span), prefix sum, scatter of slot ids into bucket order, then
// the rank of every key inside its bucket by comparison.  emit(rank, slot)
// is called once per key.  Called by all NT threads of the group.
template <int NT, bool GS, typename IdxT, typename Emit>
__device__ void sort_table(const int32_t *tkey, int S, int m, int32_t lo, int64_t span, int *bcnt,
                           int *bcur, int NB, IdxT *list, int *wsum, Emit emit)
{
    const int tid = threadIdx.x % NT;
    const uint64_t mul = (span <= NB) ? (1ull << 32) : (((uint64_t)NB << 32) / (uint64_t)span);
    for (int b = tid; b < NB; b += NT) bcnt[b] = 0;
    group_sync<NT, GS>();
    for (int s = tid; s < S; s += NT) {
        const int k = tkey[s];
        if (k != EMPTY_KEY) atomicAdd(&bcnt[bucket_of(k, lo, mul, NB)], 1);
    }
    group_sync<NT, GS>();
    block_exscan<NT, GS>(bcnt, NB, wsum);
    for (int b = tid; b < NB; b += NT) bcur[b] = bcnt[b];
    group_sync<NT, GS>();
    for (int s = tid; s < S; s += NT) {
        const int k = tkey[s];
        if (k != EMPTY_KEY) {
            const int pos = atomicAdd(&bcur[bucket_of(k, lo, mul, NB)], 1);
            list[pos] = (IdxT)s;
        }
    }
    group_sync<NT, GS>();
    for (int p = tid; p < m; p += NT) {
        const int s = list[p];
        const int k = tkey[s];
        const int b = bucket_of(k, lo, mul, NB);
        const int st = bcnt[b];
        const int en = (b + 1 < NB) ? bcnt[b + 1] : m;
        int rank = st;
        for (int q = st; q < en; ++q) rank += (tkey[list[q]] < k) ? 1 : 0;
        emit(rank, s);
    }
}

// Fused-iteration epilogue on a table whose m keys are listed in row order in
// sc.sorted: prune (Alg. 1), inflation with column re-normalisation, the
// change against the previous iterate (column j of B, which is A), and the
// per-column outputs.  find(row) returns the slot of a row or -1.
// fixed_mode >= 0: the prune branch and threshold were decided by the
// caller (fixed_mode, fixed_t) and the m listed keys are the column's kept
// entries; m_prod >= 0 is then the column's unpruned entry count.
template <int NT, bool GS, typename IdxT, typename Find, typename Keys = const int32_t *>
__device__ void iterate_epilogue(const NumericArgs &a, int64_t j, int m, int64_t bs, int mj,
                                 int64_t base, Keys tkey, double *tval,
                                 const Scratch<IdxT> &sc, Find find, int m_prod = -1, int fixed_mode = -1,
                                 double fixed_t = 0.0)
{
    const int tid = threadIdx.x % NT;
    const int w = tid / WAVE;
    constexpr int NWV = (NT + WAVE - 1) / WAVE;
    // ---------------- prune (Alg. 1) ----------------
    auto getv = [&](int p) { return tval[sc.sorted[p]]; };
    int pmode = fixed_mode;
    double t = fixed_t;
    if (fixed_mode < 0)
        prune_decide<NT, GS>(getv, m, a.pa, sc.p0, sc.p1, sc.ip, sc.hist, sc.misc, sc.dmisc, &pmode, &t);

    // kept entries, in row order, into sc.list
    const int nblk = (m + WAVE - 1) / WAVE;
    for (int b = w; b < nblk; b += NWV) {
        const int p = b * WAVE + lane();
        const bool keep = (p < m) && (getv(p) >= t);
        const int c = __popcll(ballot(keep));
        if (lane() == 0) sc.ip[b] = c;
    }
    group_sync<NT, GS>();
    const int K = block_exscan<NT, GS>(sc.ip, nblk, sc.wsum);
    for (int b = w; b < nblk; b += NWV) {
        const int p = b * WAVE + lane();
        const bool keep = (p < m) && (getv(p) >= t);
        const uint64_t mk = ballot(keep);
        if (keep) sc.list[sc.ip[b] + popc_below(mk)] = sc.sorted[p];
    }
    group_sync<NT, GS>();

    // ---------------- inflation: c^r / column sum (fixed tree over kept rank) ----------------
    const double r = a.pa.r;
    const int kblk = (K + WAVE - 1) / WAVE;
    for (int b = w; b < kblk; b += NWV) {
        const int q = b * WAVE + lane();
        const double c = (q < K) ? inflate_pow(tval[sc.list[q]], r) : 0.0;
        const double bsum = wave_sum(c);
        if (lane() == 0) sc.p0[b] = bsum;
    }
    group_sync<NT, GS>();
    if (tid < WAVE) {
        const double ssum = fixed_tree_finish(sc.p0, kblk);
        if (lane() == 0) sc.dmisc[1] = ssum;
    }
    // dropped entries read as 0 in the change computation
    for (int p = tid; p < m; p += NT) {
        const int s = sc.sorted[p];
        if (tval[s] < t) tval[s] = 0.0;
    }
    group_sync<NT, GS>();
    const double ssum = sc.dmisc[1];
    for (int q = tid; q < K; q += NT) {
        const int s = sc.list[q];
        const double c = inflate_pow(tval[s], r);
        const double an = (ssum > 0.0) ? c / ssum : 0.0;
        a.out_row[base + q] = tkey[s];
        a.out_val[base + q] = an;
        tval[s] = an;
    }
    group_sync<NT, GS>();

    // ---------------- change vs the previous iterate (A_*j == B_*j) ----------------
    double dmax = 0.0;
    for (int t2 = tid; t2 < mj; t2 += NT) {
        const int k = a.B.rowidx[bs + t2];
        const double old = a.B.val[bs + t2];
        const int s = find(k);
        if (s >= 0) {
            dmax = fmax(dmax, fabs(tval[s] - old));
            tval[s] = -1.0;  // matched
        } else {
            dmax = fmax(dmax, old);
        }
    }
    group_sync<NT, GS>();
    for (int q = tid; q < K; q += NT) dmax = fmax(dmax, tval[sc.list[q]]);  // unmatched new entries
    dmax = wave_max(dmax);
    if constexpr (NT > WAVE) {
        if (lane() == 0) sc.p1[w] = dmax;
        group_sync<NT, GS>();
        if (tid == 0) {
            for (int q = 1; q < NWV; ++q) dmax = fmax(dmax, sc.p1[q]);
        }
    }
    if (tid == 0) {
        a.out_cnt[j] = K;
        if (a.nnz_prod) a.nnz_prod[j] = m_prod >= 0 ? m_prod : m;
        if (a.delta) a.delta[j] = dmax;
        if (a.mode) a.mode[j] = (int8_t)pmode;
    }
}

// columns computed by the dense-accumulator kernel (the other kernels skip them)
__device__ __forceinline__ bool dense_column(const NumericArgs &a, int64_t j) { return a.dense && a.dense[j]; }

// The numeric body for one column j, executed by NT threads.
template <int NT, int MODE, int E, int D, typename IdxT, bool GS, bool PIPE = false>
__device__ void column_body(const NumericArgs &a, int64_t j, int S, int logS, int cap, int NB,
                           const Scratch<IdxT> &sc)
{
    const int tid = threadIdx.x % NT;
    if (a.capv) cap = (int)min((int64_t)cap, a.capv[j]);
    int32_t *tkey = sc.key;
    double *tval = sc.val;

    for (int s = tid; s < S; s += NT) {
        tkey[s] = EMPTY_KEY;
        if (MODE != MODE_COUNT) tval[s] = 0.0;
    }
    if (tid == 0) { sc.misc[6] = 0; sc.misc[7] = 0; }
    group_sync<NT, GS>();

    // ---------------- accumulation ----------------
    // Step t of column j adds b_t * A_*k to the table, for the t-th nonzero
    // b_kj of B_*j.
    const int64_t bs = a.B.colptr[j];
    const int mj = (int)(a.B.colptr[j + 1] - bs);
    // Key count and overflow: each wave counts the keys it placed.  At the
    // end of every burst group the waves publish their counts and read all
    // of them back; the slots alternate between two sets by group parity,
    // so a wave that races ahead into the next group writes the other set
    // and every wave takes the same decision (misc[6 + parity] is the
    // probe-failure flag, ip[parity * NWV + w] the count of wave w).
    const int w = tid / WAVE;
    constexpr int NWV = (NT + WAVE - 1) / WAVE;
    int keys_w = 0, m = 0, par = 0;
    bool overflow = false;
    double sink = 0.0;  // sum of all products a lane saw (kept live, never used)
    for (int tb = 0; tb < mj && !overflow; tb += WAVE) {
        // lane l of every wave holds step tb + l: row/value pointers, length, b
        const int t = tb + lane();
        const int32_t *rp = nullptr;
        const double *vp = nullptr;
        int klen = 0;
        double bv = 1.0;
        if (t < mj) {
            const int k = a.B.rowidx[bs + t];
            bv = a.B.val[bs + t];
            const int64_t p0 = a.A.colptr[k];
            rp = a.A.rowidx + p0;
            vp = a.A.val + p0;
            klen = (int)(a.A.colptr[k + 1] - p0);
        }
        const int nb = min(WAVE, mj - tb);
        // Every step of the batch is cut into ceil(len/CH) chunks (at least
        // one, possibly empty); the total is known up front so the ring below
        // runs a fixed number of rounds with no early exit.
        constexpr int CH = NT * E;
        const int nchunk_l = (lane() < nb) ? max(1, (klen + CH - 1) / CH) : 0;
        const int total = wave_sum_i(nchunk_l);
        // Chunks are consumed in load order, which keeps the ascending-k
        // accumulation order.  Every load is issued unconditionally (lanes
        // past the end read a dummy word holding row -1) and the iterator
        // advances with selects, so the compiler can keep the loads
        // outstanding.
        const int32_t *dummy_r = (const int32_t *)a.dummy;
        const double *dummy_v = (const double *)a.dummy;
        int iu = 0, ioff = 0;
        auto issue = [&](int32_t(&r)[E], double(&v)[E], double &b) {
            const int ul = min(iu, WAVE - 1);
            const int32_t *rb = (const int32_t *)readlane_i64((int64_t)rp, ul);
            const double *vbp = (const double *)readlane_i64((int64_t)vp, ul);
            const int len0 = readlane_i(klen, ul);
            const int len = (iu < nb) ? len0 : 0;
            b = readlane_d(bv, ul);
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int e = ioff + tid + q * NT;
                const bool in = e < len;
                r[q] = ldg(in ? rb + e : dummy_r);
                if (MODE != MODE_COUNT) v[q] = ldg(in ? vbp + e : dummy_v);
            }
            const bool more = ioff + CH < len;
            ioff = more ? ioff + CH : 0;
            iu = more ? iu : iu + 1;
        };
        // A group is D consecutive chunks: their loads are issued back to
        // back, then the chunks are folded in order.
        auto issue_group = [&](int32_t(&r)[D][E], double(&v)[D][E], double(&b)[D]) {
#pragma unroll
            for (int i = 0; i < D; ++i) issue(r[i], v[i], b[i]);
        };
        auto fold_group = [&](int32_t(&r)[D][E], double(&v)[D][E], double(&b)[D]) {
            // 1. place every key of the group (the order of insertions does
            //    not matter): all first-bucket reads go out together
            uint32_t hb[D][E];
            keys4 kb[D][E];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int q = 0; q < E; ++q)
                {
                    hb[i][q] = hash_slot(max(r[i][q], 0), logS - 2);
                    kb[i][q] = load_bucket<!GS>(tkey, hb[i][q]);
                }
            int sl[D][E];
#pragma unroll
            for (int i = 0; i < D; ++i) {
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    // the dummy word reads as row -1; testing the loaded
                    // row (not a separate flag) keeps the load ahead of the
                    // branch, so the compiler cannot sink it into the branch
                    sl[i][q] = -1;
                    bool fresh = false;
                    if (r[i][q] >= 0)
                        sl[i][q] = place_key<!GS>(tkey, r[i][q], hb[i][q], kb[i][q], (S >> 2) - 1,
                                                  &sc.misc[6 + par], fresh);
                    keys_w += __popcll(ballot(fresh));
                }
            }
            if (NWV > 1 && lane() == 0) sc.ip[par * NWV + w] = keys_w;
            // 2. the value updates, chunk by chunk in order; a row may recur
            //    in the next chunk, so chunks are separated by a barrier
            //    (one wave: its LDS operations already apply in order)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (MODE != MODE_COUNT) {
#pragma unroll
                    for (int q = 0; q < E; ++q) {
                        // every lane folds its product into `sink`, so the
                        // value load is used outside the branch and cannot be
                        // sunk into it (idle lanes stay out of the table)
                        const double prod = v[i][q] * b[i];
                        sink += prod;
                        if (sl[i][q] >= 0) table_add<!GS>(tval + sl[i][q], prod);
                    }
                }
                if (NWV > 1 || GS || i == D - 1) group_sync<NT, GS>();
            }
            if constexpr (NWV == 1) {
                m = keys_w;
            } else {
                m = 0;
                for (int v2 = 0; v2 < NWV; ++v2) m += sc.ip[par * NWV + v2];
            }
            overflow = sc.misc[6 + par] != 0 || m > cap;
            par ^= 1;
        };
        int32_t rA[D][E];
        double vA[D][E], bA[D];
        if constexpr (!PIPE) {
            // burst groups: one memory latency per group, overlapped only by
            // the other waves and workgroups of the CU
            for (int g0 = 0; g0 < total && !overflow; g0 += D) {
                issue_group(rA, vA, bA);
                fold_group(rA, vA, bA);
            }
        } else {
            // double-buffered groups: the loads of group g+1 are in flight
            // while group g is folded (past the last chunk the iterator
            // issues dummy loads)
            int32_t rB[D][E];
            double vB[D][E], bB[D];
            const int ng = (total + D - 1) / D;
            issue_group(rA, vA, bA);
            for (int g = 0; g < ng && !overflow; g += 2) {
                issue_group(rB, vB, bB);
                fold_group(rA, vA, bA);
                if (g + 1 >= ng || overflow) break;
                issue_group(rA, vA, bA);
                fold_group(rB, vB, bB);
            }
        }
    }
    // products are >= 0 or NaN (dummy lanes), so this store never happens;
    // the compiler cannot know that and keeps `sink` (and the loads) live
    if (MODE != MODE_COUNT && sink == -1.0) sc.dmisc[3] = sink;
    group_sync<NT, GS>();
    if (overflow) {
        if (tid == 0) a.out_cnt[j] = -1;
        return;
    }
    if (MODE == MODE_COUNT) {
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }

    // ---------------- sort the m keys by row ----------------
    const int32_t lo = a.lo[j];
    const int64_t span = (int64_t)a.hi[j] - lo + 1;
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    if (MODE == MODE_EXPAND) {
        sort_table<NT, GS, IdxT>(tkey, S, m, lo, span, sc.bcnt, sc.bcur, NB, sc.list, sc.wsum,
                                 [&](int rank, int s) {
                                     a.out_row[base + rank] = tkey[s];
                                     a.out_val[base + rank] = tval[s];
                                 });
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }
    sort_table<NT, GS, IdxT>(tkey, S, m, lo, span, sc.bcnt, sc.bcur, NB, sc.list, sc.wsum,
                             [&](int rank, int s) { sc.sorted[rank] = (IdxT)s; });
    group_sync<NT, GS>();
    iterate_epilogue<NT, GS, IdxT>(a, j, m, bs, mj, base, tkey, tval, sc,
                                   [&](int32_t k) { return find_slot<!GS>(tkey, k, logS - 2, (S >> 2) - 1); });
}

// ---------------------------------------------------------------------------
// LDS-bin kernels
// ---------------------------------------------------------------------------
template <int S>
struct LdsBin {
    static constexpr int CAP = (3 * S) / 4;
    static constexpr int NB = (S / 4 < 64) ? 64 : S / 4;
    static constexpr int NBLK = CAP / WAVE + 2;
    using Idx = uint16_t;
};

template <int S, int NW, int CPW, int MODE, int E, int D, bool PIPE>
__global__ __launch_bounds__(NW * WAVE * CPW) void k_numeric_lds(NumericArgs a)
{
    using L = LdsBin<S>;
    constexpr int NT = NW * WAVE;
    struct alignas(16) Col {
        double val[S];
        int32_t key[S];
        double p0[L::NBLK], p1[L::NBLK];
        int32_t bcnt[L::NB], bcur[L::NB];
        int32_t ip[L::NBLK];
        int32_t hist[256];
        uint16_t list[L::CAP], sorted[L::CAP];
        int32_t misc[16];
        double dmisc[4];
        int32_t wsum[NW];
    };
    __shared__ Col cols[CPW] __attribute__((aligned(16)));
    const int ci = threadIdx.x / NT;
    const int64_t idx = (int64_t)blockIdx.x * CPW + ci;
    if (idx >= a.ncols) return;  // whole groups exit together
    Col &c = cols[ci];
    Scratch<uint16_t> sc{c.key, c.val, c.list, c.sorted, c.bcnt, c.bcur, c.p0, c.p1,
                         c.ip, c.hist, c.misc, c.dmisc, c.wsum};
    constexpr int logS = __builtin_ctz(S);
    if (dense_column(a, a.cols[idx])) return;  // whole column group (a workgroup when NW > 1)
    column_body<NT, MODE, E, D, uint16_t, false, PIPE>(a, a.cols[idx], S, logS, L::CAP, L::NB, sc);
}

// ---------------------------------------------------------------------------
// Sliced source layout and the sliced-table kernel for large columns.
//
// Rows are dealt to NG = 64 groups by the top six bits of their
// multiplicative hash.  The sliced copy of a source matrix keeps every column
// in place but orders its entries by group (in no particular order inside a
// group) and records the 65 group boundaries of the column.  Every kernel
// of a product reads the sliced copy: the HBM tables take their bucket from
// the top bits of the same hash, so consecutive entries also probe one region
// of an HBM table.  A workgroup of NW waves then gives wave w the groups
// [w*G, (w+1)*G), G = NG/NW, with a
// private table of SW slots: the entries of A_*k that wave w needs are one
// contiguous, exactly known run, waves never share a row, so accumulation
// needs no barrier, and a wave's LDS operations apply in issue order, which
// keeps the ascending-k order of every row.  Hashed groups spread the rows
// of a column evenly over the waves whatever the vertex numbering.
// ---------------------------------------------------------------------------
constexpr int NG = SLICE_GROUPS;
static_assert(NG == WAVE, "one group per lane in the layout pass");

__device__ __forceinline__ uint32_t row_hash(int32_t r) { return (uint32_t)r * 2654435761u; }
__device__ __forceinline__ int row_group(int32_t r) { return (int)(row_hash(r) >> 26); }
// home bucket inside a sub-table of 2^logNB buckets: the hash bits below the group bits
__device__ __forceinline__ uint32_t hash_bucket(uint32_t h, int logNB) { return (h << 6) >> (32 - logNB); }
__device__ __forceinline__ uint32_t sub_bucket(int32_t r, int logNB) { return hash_bucket(row_hash(r), logNB); }

// A record of the packed sliced copy: row, then the value's low and high
// words.  12 bytes with 4-byte alignment, so one dwordx3 load per entry and
// a run of a column is one contiguous byte range (fewer partially used
// cache lines than a row range plus a value range).
typedef uint32_t rec3 __attribute__((ext_vector_type(3), aligned(4)));

// One wave per column: group sizes (LDS counters), boundaries, then a
// scatter by LDS cursors.  The order of the entries inside a group is not
// specified (every consumer treats a run as a set of distinct rows).
__global__ __launch_bounds__(256) void k_slice_layout(DevCSC A, int32_t *__restrict__ rowo,
                                                      double *__restrict__ valo, uint32_t *__restrict__ reco,
                                                      int32_t *__restrict__ goff, uint32_t *__restrict__ poff)
{
    __shared__ int32_t ctr[4][NG];
    const int w = threadIdx.x / WAVE;
    const int64_t k = (int64_t)blockIdx.x * 4 + w;
    if (k >= A.ncols) return;  // whole wave
    int32_t *c = ctr[w];
    const int64_t p0 = A.colptr[k];
    const int len = (int)(A.colptr[k + 1] - p0);
    c[lane()] = 0;
    group_sync<WAVE>();
    for (int e = lane(); e < len; e += WAVE) atomicAdd(&c[row_group(A.rowidx[p0 + e])], 1);
    group_sync<WAVE>();
    const int cnt = c[lane()];
    const int cur = wave_incl_scan(cnt) - cnt;  // lane g: first position of group g
    goff[k * (NG + 1) + lane()] = cur;
    if (lane() == 0) goff[k * (NG + 1) + NG] = len;
    // every fourth boundary as an absolute record index (the end of the last
    // column's last run is the record count)
    if ((lane() & 3) == 0) poff[k * (NG / 4) + lane() / 4] = (uint32_t)(p0 + cur);
    if (lane() == 0 && k + 1 == A.ncols) poff[(k + 1) * (NG / 4)] = (uint32_t)(p0 + len);
    group_sync<WAVE>();
    c[lane()] = cur;
    group_sync<WAVE>();
    for (int e = lane(); e < len; e += WAVE) {
        const int32_t r = A.rowidx[p0 + e];
        const int64_t d = p0 + atomicAdd(&c[row_group(r)], 1);
        const double v = A.val[p0 + e];
        rowo[d] = r;
        valo[d] = v;
        const uint64_t vb = (uint64_t)__double_as_longlong(v);
        *(__attribute__((address_space(1))) rec3 *)(reco + d * 3) = rec3{(uint32_t)r, (uint32_t)vb,
                                                                         (uint32_t)(vb >> 32)};
    }
}

void launch_slice_layout(const DevCSC &A, int32_t *rowo, double *valo, uint32_t *reco, int32_t *goff,
                         uint32_t *poff, hipStream_t st)
{
    if (A.ncols <= 0) return;
    hipLaunchKernelGGL(k_slice_layout, dim3((unsigned)((A.ncols + 3) / 4)), dim3(256), 0, st, A, rowo, valo,
                       reco, goff, poff);
}

// One wave accumulates the row groups [g0, g1) of column j into its private
// table of SW slots (cleared here).  Returns the number of keys it placed;
// *wovf is raised when a probe fails; more than capw keys stop the
// accumulation early (the caller treats both as overflow).
// col_keys / col_cap: a counter shared by the column's waves and the
// column's key capacity; a wave stops soon after the column total exceeds it
// (the total is read with the next group's bucket reads, so no LDS round
// trip waits on it).
//
// DENSE: instead of a hash table, the wave adds into wval[row - dlo] (a
// dense accumulator over the column's row span, shared by the column's
// waves, which own disjoint rows, cleared by the caller) and marks the row
// in the bitmap dbits; wkey, wovf, col_keys and the capacities are unused
// and the return value is 0.
// NARROW: the sliced copy holds fewer than 2^32 bytes (NARROW_RECS records),
// so a record's address is a 32-bit byte offset, advanced by adds only.
constexpr uint32_t NARROW_RECS = 0xFFFFFFFFu / 12u;
template <int SW, int MODE, int D, bool DENSE = false, bool NARROW = false>
__device__ int slice_accumulate(const NumericArgs &a, int64_t j, int g0, int g1, int32_t *wkey, double *wval,
                                int *wovf, int capw, double *never, int *col_keys, int64_t col_cap,
                                int32_t dlo = 0, uint32_t *dbits = nullptr)
{
    constexpr int NBW = SW / 4;
    constexpr int LOGNBW = __builtin_ctz(NBW);
    if constexpr (!DENSE) {
        for (int s = lane(); s < SW; s += WAVE) {
            wkey[s] = EMPTY_KEY;
            if (MODE != MODE_COUNT) wval[s] = 0.0;
        }
        group_sync<WAVE>();
    }

    const int64_t bs = a.B.colptr[j];
    const int mj = (int)(a.B.colptr[j + 1] - bs);
    bool overflow = false;
    int keys_w = 0;     // keys this wave placed
    int published = 0;  // of which already added to *col_keys
    int lovf = 0;       // a probe of this lane failed
    int sinkh = 0;      // high words of the products a lane saw (kept live, never used)
    const uint32_t lane12 = 12u * (uint32_t)lane();

    // Step metadata of a batch of 64 steps (lane l: step tb + l): the row k
    // and value of b, then this wave's run in A_*k (start, length).  The next
    // batch's metadata is loaded while the current batch is folded in: its
    // step rows at the batch start, its runs after the first group.
    auto step_of = [&](int tb, int &k, double &b) {
        const int t = tb + lane();
        k = -1;
        b = 0.0;
        if (t < mj) {
            k = a.B.rowidx[bs + t];
            b = a.B.val[bs + t];
        }
    };
    // a run that starts and ends on a fourth group boundary: both ends from
    // one 64-byte block of poff (no colptr or goff line per step)
    const bool q4 = a.poff && ((g0 | g1) & 3) == 0;
    auto run_of = [&](int k, uint32_t &ws, int &len) {
        ws = 0;
        len = 0;
        if (k >= 0) {
            if (q4) {
                const uint32_t *po = a.poff + (int64_t)k * (NG / 4);
                ws = po[g0 >> 2];
                len = (int)(po[g1 >> 2] - ws);
            } else {
                const int32_t *go = a.goff + (int64_t)k * (NG + 1);
                const int r0 = go[g0], r1 = go[g1];
                ws = (uint32_t)a.A.colptr[k] + (uint32_t)r0;  // the sliced copy has fewer than 2^32 entries
                len = r1 - r0;
            }
        }
    };
    // The non-empty runs of a batch move to the low lanes, in step order
    // (forward permute; the lanes above the last non-empty run become
    // empty), so the run starts of a batch are strictly increasing and no
    // two steps start at one position.
    auto compact = [&](uint32_t &ws, int &len, double &bv) {
        const uint64_t ne = ballot(len > 0);
        if (ne == ~0ull) return;
        const int dst = (len > 0 ? popc_below(ne) : WAVE - 1) << 2;
        ws = (uint32_t)__builtin_amdgcn_ds_permute(dst, (int)ws);
        len = __builtin_amdgcn_ds_permute(dst, len);
        if (MODE != MODE_COUNT) {
            const int64_t bb = __double_as_longlong(bv);
            const int lo = __builtin_amdgcn_ds_permute(dst, (int)(uint32_t)bb);
            const int hi = __builtin_amdgcn_ds_permute(dst, (int)(bb >> 32));
            bv = __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
        }
        if (lane() >= __popcll(ne)) {
            ws = 0;
            len = 0;
            bv = 0.0;
        }
    };
    int kn, lenn;
    uint32_t wsn;
    double bvn;
    step_of(0, kn, bvn);
    run_of(kn, wsn, lenn);
    compact(wsn, lenn, bvn);
    for (int tb = 0; tb < mj && !overflow; tb += WAVE) {
        const uint32_t ws = wsn;
        const int len = lenn;
        const double bv = bvn;
        bool next_runs = tb + WAVE < mj;  // the next batch's runs are still to be loaded
        if (next_runs) step_of(tb + WAVE, kn, bvn);
        // The runs of the batch's steps are packed back to back: chunk c
        // holds entries [64c, 64c + 64) of the concatenation, usually
        // pieces of several steps.  pre = start of the lane's run.
        const int pre = wave_incl_scan(len) - len;
        const int total = readlane_i(pre + len, WAVE - 1);
        const int nchunk = (total + WAVE - 1) / WAVE;
        // Groups of D chunks: loads issued back to back, first-bucket reads
        // of all D chunks together, then insertion, then the value updates
        // chunk by chunk and, inside a chunk, step by step (atomic adds of
        // one wave apply in issue order, so every row still sees its steps
        // in ascending k).  Groups are double-buffered: the loads of group
        // g+1 are in flight while group g is folded in.
        struct Grp {
            int32_t rr[D];
            double vv[D], bb[D];
            int sub[D], nsub[D];
        };
        // lane l's run as an offset into A: entry f of the packed sequence,
        // f in [pre_l, pre_l + len_l), is A entry f + base_l
        const uint32_t basev = ws - (uint32_t)pre;  // modulo 2^32
        // NARROW: the same in bytes (12 * entry index, exact below 2^32)
        const uint32_t baseb = NARROW ? basev * 12u : 0u;
        auto issue = [&](Grp &G, int c0) {
            // two sweeps: the lane permutes of all D chunks first (one wait
            // for all of them), then the addresses and the loads
            uint32_t bu[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int F = (c0 + i) * WAVE;
                // runs are in lane order with ascending starts: lanes
                // [0, cnt0) start at or before F (cnt0 >= 1: lane 0 starts
                // at 0), the next k lanes start inside the chunk; a lane's
                // step is the last run starting at or before its entry
                // The runs starting inside the chunk mark their first entry
                // (forward permute of a 1 to lane pre - F; lanes nobody
                // writes read 0); a lane's rank among the chunk's steps is
                // the number of marks at or below it.
                const int cnt0 = __popcll(ballot(pre <= F));
                const bool starts = len > 0 && pre > F && pre < F + WAVE;
                const int mark = __builtin_amdgcn_ds_permute(starts ? (pre - F) << 2 : 0, starts ? 1 : 0);
                const uint64_t M = ballot(mark != 0);
                const int k = __popcll(M);
                const int rank = popc_below(M) + mark;
                const int u = cnt0 - 1 + rank;
                bu[i] = (uint32_t)shfl_i((int)(NARROW ? baseb : basev), u);
                if (MODE != MODE_COUNT) G.bb[i] = shfl_d(bv, u);
                G.sub[i] = rank;  // position of the lane's step among the chunk's steps
                G.nsub[i] = k + 1;
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int F = (c0 + i) * WAVE;
                // past the run ends: the sentinel entry (row -1, value 0)
                rec3 x;
                if constexpr (NARROW) {
                    const uint32_t ab = (F + lane() < total) ? bu[i] + 12u * (uint32_t)F + lane12 : a.src_end * 12u;
                    x = ldg((const rec3 *)((const char *)a.srec + ab));
                } else {
                    const uint32_t ad = (F + lane() < total) ? bu[i] + (uint32_t)(F + lane()) : a.src_end;
                    x = ldg((const rec3 *)(a.srec + (uint64_t)ad * 3));
                }
                G.rr[i] = (int32_t)x.x;
                if (MODE != MODE_COUNT) G.vv[i] = __longlong_as_double((int64_t)(((uint64_t)x.z << 32) | x.y));
            }
        };
        // The adds of one chunk (sub = the lane's step among the chunk's
        // nsub steps).  One masked atomic per step, in step order: a row met by two steps
        // of the chunk sits in two lanes, and only successive instructions
        // of a wave are documented to apply in order (lanes of one
        // instruction that share an address are applied in an unspecified
        // order).  Written as a loop with a run-time trip count, so the
        // compiler cannot merge the steps' atomics into one instruction --
        // which it may do with an unrolled form, since every lane runs
        // exactly one of them.
        auto ordered_adds = [&](int sub, int nsub, int slot, double x) {
            for (int q = 0; q < nsub; ++q)
                if (sub == q && slot >= 0) lds_atomic_add(wval + slot, x);
        };
        auto fold_dense = [&](Grp &G) {
            double prod[D];
            int sl[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                sl[i] = (G.rr[i] != EMPTY_KEY) ? G.rr[i] - dlo : -1;
                prod[i] = G.vv[i] * G.bb[i];
                sinkh |= __double2hiint(prod[i]);  // keeps the value load out of the branch
                // a touched row holds a positive sum unless every product
                // added to it underflowed to zero: only those mark the bitmap
                if (sl[i] >= 0 && prod[i] == 0.0) atomicOr(&dbits[sl[i] >> 5], 1u << (sl[i] & 31));
            }
#pragma unroll
            for (int i = 0; i < D; ++i) ordered_adds(G.sub[i], G.nsub[i], sl[i], prod[i]);
        };
        auto fold_hash = [&](Grp &G) {
            uint32_t hb[D];
            keys4 kb[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                hb[i] = sub_bucket(G.rr[i], LOGNBW);
                kb[i] = load_bucket<true>(wkey, hb[i]);
            }
            const int col_total = __hip_atomic_load((__attribute__((address_space(3))) int *)col_keys,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            int sl[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                sl[i] = -1;
                bool fresh = false;
                if (G.rr[i] != EMPTY_KEY) sl[i] = place_key<true>(wkey, G.rr[i], hb[i], kb[i], NBW - 1, &lovf, fresh);
                keys_w += __popcll(ballot(fresh));
            }
            // a column already over its capacity is recomputed elsewhere: skip
            // its value updates.  (Testing the total here, before any atomic,
            // keeps the wait for it -- and for the permutes issued before
            // it -- ahead of the atomics.)
            const bool col_over = col_total > col_cap;
            if (MODE != MODE_COUNT && !col_over) {
                double prod[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    prod[i] = G.vv[i] * G.bb[i];
                    sinkh |= __double2hiint(prod[i]);  // keeps the value load out of the branch
                }
#pragma unroll
                for (int i = 0; i < D; ++i) ordered_adds(G.sub[i], G.nsub[i], sl[i], prod[i]);
            }
            const int delta = __builtin_amdgcn_readfirstlane(keys_w - published);
            if (delta != 0) {  // new keys: publish them (no return value to wait for)
                if (lane() == 0)
                    __hip_atomic_fetch_add((__attribute__((address_space(3))) int *)col_keys, delta,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                published = keys_w;
            }
            overflow = ballot(lovf != 0) != 0 || keys_w > capw || col_over;
        };
        auto fold = [&](Grp &G) {
            if constexpr (DENSE) fold_dense(G);
            else fold_hash(G);
        };
        Grp GA, GB;
        issue(GA, 0);
        for (int c0 = 0; c0 < nchunk && !overflow; c0 += 2 * D) {
            issue(GB, c0 + D);  // past the last chunk: loads of the sentinel entry
            fold(GA);
            if (next_runs) {
                run_of(kn, wsn, lenn);
                compact(wsn, lenn, bvn);
                next_runs = false;
            }
            if (c0 + D >= nchunk || overflow) break;
            issue(GA, c0 + 2 * D);
            fold(GB);
        }
        if (next_runs) {
            run_of(kn, wsn, lenn);
            compact(wsn, lenn, bvn);
        }
    }
    if constexpr (!DENSE) {
        const bool any_ovf = ballot(lovf != 0) != 0;
        if (lane() == 0) *wovf = any_ovf ? 1 : 0;
    }
    if (MODE != MODE_COUNT && sinkh < 0) *never = 1.0;  // never: products are >= 0
    group_sync<WAVE>();
    return keys_w;
}

template <int NW, int SW, int MODE, int D>
__global__ __launch_bounds__(NW * WAVE) void k_numeric_hsplit(NumericArgs a)
{
    constexpr int NT = NW * WAVE;
    constexpr int G = NG / NW;                 // groups per wave
    constexpr int CAPW = (13 * SW) / 16;       // keys per wave table
    constexpr int NBW = SW / 4;                // buckets per wave table
    constexpr int LOGNBW = __builtin_ctz(NBW);
    constexpr int STOT = NW * SW;
    constexpr int CAPT = NW * CAPW;
    constexpr int NBS = STOT / 4;              // sort buckets
    constexpr int NBLK = CAPT / WAVE + 2;
    static_assert(NG % NW == 0 && STOT <= 65536, "layout");
    struct alignas(16) Sh {
        double val[STOT];
        int32_t key[STOT];
        double p0[NBLK], p1[NBLK];
        int32_t ip[NBLK];
        int32_t bcnt[NBS], bcur[NBS];
        int32_t hist[256];
        uint16_t list[CAPT], sorted[CAPT];
        int32_t wcnt[NW], wovf[NW];
        int32_t misc[16];
        double dmisc[4];
        int32_t wsum[NW];
    };
    __shared__ Sh sh __attribute__((aligned(16)));
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    const int64_t j = a.cols[blockIdx.x];
    if (dense_column(a, j)) return;  // whole workgroup
    if (tid == 0) sh.misc[8] = 0;
    __syncthreads();
    const int64_t col_cap = a.capv ? min((int64_t)CAPT, a.capv[j]) : (int64_t)CAPT;
    const int keys_w = a.src_end <= NARROW_RECS
        ? slice_accumulate<SW, MODE, D, false, true>(a, j, w * G, (w + 1) * G, sh.key + w * SW, sh.val + w * SW,
                                                     &sh.wovf[w], CAPW, &sh.dmisc[3], &sh.misc[8], col_cap)
        : slice_accumulate<SW, MODE, D>(a, j, w * G, (w + 1) * G, sh.key + w * SW, sh.val + w * SW,
                                                     &sh.wovf[w], CAPW, &sh.dmisc[3], &sh.misc[8], col_cap);
    if (lane() == 0) {
        sh.wcnt[w] = keys_w;
        if (keys_w > CAPW) sh.wovf[w] = 1;
    }
    __syncthreads();

    int m = 0, ovf = 0;
    for (int q = 0; q < NW; ++q) {
        m += sh.wcnt[q];
        ovf |= sh.wovf[q];
    }
    if (a.capv && m > a.capv[j]) ovf = 1;  // more keys than the column's output slot holds
    if (ovf) {
        if (tid == 0) a.out_cnt[j] = -1;
        return;
    }
    if (MODE == MODE_COUNT) {
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }
    const int64_t bs = a.B.colptr[j];
    const int mj = (int)(a.B.colptr[j + 1] - bs);
    const int32_t lo = a.lo[j];
    const int64_t span = (int64_t)a.hi[j] - lo + 1;
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    if (MODE == MODE_EXPAND) {
        sort_table<NT, false, uint16_t>(sh.key, STOT, m, lo, span, sh.bcnt, sh.bcur, NBS, sh.list, sh.wsum,
                                        [&](int rank, int s) {
                                            a.out_row[base + rank] = sh.key[s];
                                            a.out_val[base + rank] = sh.val[s];
                                        });
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }
    sort_table<NT, false, uint16_t>(sh.key, STOT, m, lo, span, sh.bcnt, sh.bcur, NBS, sh.list, sh.wsum,
                                    [&](int rank, int s) { sh.sorted[rank] = (uint16_t)s; });
    __syncthreads();
    Scratch<uint16_t> sc{sh.key, sh.val, sh.list, sh.sorted, sh.bcnt, sh.bcur, sh.p0, sh.p1,
                         sh.ip, sh.hist, sh.misc, sh.dmisc, sh.wsum};
    iterate_epilogue<NT, false, uint16_t>(a, j, m, bs, mj, base, sh.key, sh.val, sc, [&](int32_t k) {
        const int ow = row_group(k) / G;
        const int s = find_from<true>(sh.key + ow * SW, k, sub_bucket(k, LOGNBW), NBW - 1);
        return (s < 0) ? -1 : ow * SW + s;
    });
}

// ---------------------------------------------------------------------------
// Split sliced tables: the row groups of a column are divided among P
// workgroups ("parts") of NWP waves, which run concurrently and hold only
// their own waves' tables (NWP * SW slots, no epilogue arrays), so several
// parts fit on one CU.  Part p covers the groups [p*NG/P, (p+1)*NG/P); as in
// the one-workgroup kernel every row belongs to exactly one wave, which adds
// its products in ascending k.  A part appends its keys and values, unsorted,
// to the column's temp slot at an offset taken from the column's counter
// part_cnt[j]; PART_OVF in that counter marks a column that overflowed.
// k_finish_part then sorts each column by row and runs the epilogue, and
// resets the counter.  The block index keeps the P parts of a column on one
// XCD (workgroups are dealt to the 8 XCDs in turn), so the column's step
// metadata is fetched once per L2.
// ---------------------------------------------------------------------------
constexpr int32_t PART_OVF = 1 << 30;         // the column does not fit its slot
constexpr int32_t PART_INC = 1 << 29;         // ... and its key count is incomplete
constexpr int32_t PART_CNT = PART_INC - 1;    // key count bits

// Overflowed column with a complete count: record it (the overflow round
// re-plans the column at that size instead of counting it again).
__device__ __forceinline__ void note_exact(const NumericArgs &a, int64_t j, int32_t c)
{
    if (a.exact_cnt && !(c & PART_INC)) a.exact_cnt[j] = c & PART_CNT;
}

__device__ __forceinline__ bool multipass_column(const NumericArgs &a, int64_t j);


// MP: the launch holds the multi-pass columns of the largest bin together
// with HBM-table columns, which it skips; 3 = the columns of up to MP_SMALL
// keys, 1 = up to MP_NARROW, 2 = the larger ones.
template <int NWP, int SW, int P, int MODE, int D, int MP = 0>
__device__ __forceinline__ void numeric_part_body(const NumericArgs &a)
{
    constexpr int G = NG / (P * NWP);  // groups per wave
    constexpr int CAPW = (13 * SW) / 16;
    static_assert(NG % (P * NWP) == 0, "groups must divide evenly");
    struct alignas(16) Sh {
        double val[NWP * SW];
        int32_t key[NWP * SW];
        int32_t wcnt[NWP], wovf[NWP];
        int32_t misc[4];
        double dmisc[4];
    };
    __shared__ Sh sh __attribute__((aligned(16)));
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    const uint32_t b = blockIdx.x;
    const uint32_t r = b % (8 * P);
    const int p = (int)(r / 8);
    const uint32_t idx = (b / (8 * P)) * 8 + r % 8;
    if (idx >= (uint32_t)a.ncols) return;  // whole workgroup
    const int64_t j = a.cols[idx];
    if (dense_column(a, j)) return;  // whole workgroup
    if constexpr (MP != 0) {
        if (!multipass_column(a, j)) return;  // whole workgroup
        const int64_t c = a.capv[j];
        if ((c <= MP_SMALL ? 3 : c <= MP_NARROW ? 1 : 2) != MP) return;
    }
    if (tid == 0) sh.misc[0] = 0;
    __syncthreads();
    const int64_t col_cap = a.capv ? a.capv[j] : (int64_t)(P * NWP * CAPW);
    const int g0 = p * (NG / P) + w * G;
    const int keys_w = a.src_end <= NARROW_RECS
        ? slice_accumulate<SW, MODE, D, false, true>(a, j, g0, g0 + G, sh.key + w * SW, sh.val + w * SW,
                                                     &sh.wovf[w], CAPW, &sh.dmisc[3], &sh.misc[0], col_cap)
        : slice_accumulate<SW, MODE, D>(a, j, g0, g0 + G, sh.key + w * SW, sh.val + w * SW,
                                                     &sh.wovf[w], CAPW, &sh.dmisc[3], &sh.misc[0], col_cap);
    if (lane() == 0) {
        sh.wcnt[w] = keys_w;
        if (keys_w > CAPW) sh.wovf[w] = 1;
    }
    __syncthreads();
    int mp = 0, ovf = 0, pre = 0;
    for (int q = 0; q < NWP; ++q) {
        if (q < w) pre += sh.wcnt[q];
        mp += sh.wcnt[q];
        ovf |= sh.wovf[q];
    }
    if (tid == 0) {
        // every part adds its key count, so an overflowed column still gets
        // its exact count -- unless a wave table overflowed, or the part
        // alone passed the column's capacity (its waves then stop early)
        int off = -1;
        if (ovf || sh.misc[0] > col_cap) {
            atomicOr(&a.part_cnt[j], PART_OVF | PART_INC);
        } else {
            off = atomicAdd(&a.part_cnt[j], mp);
            if ((off & PART_OVF) || (int64_t)(off & PART_CNT) + mp > col_cap) {
                atomicOr(&a.part_cnt[j], PART_OVF);
                off = -1;
            }
        }
        sh.misc[1] = off;
    }
    __syncthreads();
    const int off = sh.misc[1] & PART_CNT;
    if (sh.misc[1] < 0) return;
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    const int32_t *wkey = sh.key + w * SW;
    const double *wval = sh.val + w * SW;
    int run = 0;
    for (int s0 = 0; s0 < SW; s0 += WAVE) {
        const int k = wkey[s0 + lane()];
        const uint64_t mk = ballot(k != EMPTY_KEY);
        if (k != EMPTY_KEY) {
            const int64_t d = base + off + pre + run + popc_below(mk);
            a.out_row[d] = k;
            a.out_val[d] = wval[s0 + lane()];
        }
        run += __popcll(mk);
    }
}

// Two register budgets: the compiler's choice, and 64 VGPRs (eight waves
// per SIMD when the LDS allows it).
template <int NWP, int SW, int P, int MODE, int D>
__global__ __launch_bounds__(NWP * WAVE) void k_numeric_part(NumericArgs a)
{
    numeric_part_body<NWP, SW, P, MODE, D>(a);
}

// the multi-pass columns of the largest bin: 64 waves per column, one row
// group each; 8 workgroups of 8 waves with 512-slot tables for columns of up
// to MP_NARROW keys, 16 workgroups of 4 waves with 1024-slot tables above
constexpr int MPP_NW = 8, MPP_P = 8, MPW_NW = 4, MPW_P = 16;
static_assert(MPP_NW * MPP_P == NG && MPW_NW * MPW_P == NG, "one group per wave");
template <int MODE>
__global__ __launch_bounds__(MPP_NW * WAVE) void k_numeric_mpart(NumericArgs a)
{
    numeric_part_body<MPP_NW, 512, MPP_P, MODE, 2, 1>(a);
}
template <int MODE>
__global__ __launch_bounds__(MPW_NW * WAVE) void k_numeric_mpart_wide(NumericArgs a)
{
    numeric_part_body<MPW_NW, 1024, MPW_P, MODE, 2, 2>(a);
}
// up to MP_SMALL keys: 8 workgroups of 4 waves, two row groups per wave
constexpr int MPS_NW = 4, MPS_P = 8;
template <int MODE>
__global__ __launch_bounds__(MPS_NW * WAVE) void k_numeric_mpart_small(NumericArgs a)
{
    numeric_part_body<MPS_NW, 512, MPS_P, MODE, 2, 3>(a);
}

template <int NWP, int SW, int P, int MODE, int D>
__global__ __launch_bounds__(NWP * WAVE) __attribute__((amdgpu_num_vgpr(64))) void k_numeric_part_v64(
    NumericArgs a)
{
    numeric_part_body<NWP, SW, P, MODE, D>(a);
}

// Prune decision before the sort, for an unsorted column of m entries
// (key[p], val[p]).  The column sums mB and mP (of all entries and of those
// >= theta) only decide the recovery branch (nP < R and mP < pct * mB); the
// fused epilogue forms them by a fixed tree over the sorted column.  Here
// they are summed in the unsorted order instead: a sum of m nonnegative
// values lies within m * 2^-53 times the sum of the exact one, whatever the
// order, so when |mP - pct * mB| exceeds 4 * m * 2^-53 * max(1, pct) * mB
// the branch is the one the sorted sums would take.  The branch and
// threshold then follow from nP and an order-independent selection over
// the unsorted values, the entries below the threshold are dropped (their
// keys become EMPTY_KEY) and only the kept ones need sorting -- the same
// kept set, order and values as deciding on the whole sorted column.  Returns the number of entries left to sort
// (m, with fmode = -1, when the margin is too small to decide; else fmode
// is the branch and ft the threshold).  Called by all NT threads of the
// group.
template <int NT, bool GS, typename KeyT>
__device__ int select_first(const NumericArgs &a, int m, KeyT *key, const double *val, int *wsum, double *p0,
                            double *p1, int *hist, int *misc, double *dmisc, int &fmode, double &ft)
{
    constexpr int NWV = NT / WAVE;
    static_assert(NT % WAVE == 0, "whole waves");
    const int tid = threadIdx.x % NT;
    const int w = tid / WAVE;
    const int nblk = (m + WAVE - 1) / WAVE;
    int cnt = 0;  // nP: entries >= theta
    for (int b = w; b < nblk; b += NWV) {
        const int p = b * WAVE + lane();
        cnt += __popcll(ballot(p < m && val[p] >= a.pa.theta));
    }
    if (lane() == 0) wsum[w] = cnt;
    group_sync<NT, GS>();
    int nP = 0;
    for (int q = 0; q < NWV; ++q) nP += wsum[q];
    group_sync<NT, GS>();
    fmode = -1;
    ft = 0.0;
    bool rec = false;
    if (a.pa.R > 0 && nP < a.pa.R) {
        double sb = 0.0, sp = 0.0;
        for (int b = w; b < nblk; b += NWV) {
            const int p = b * WAVE + lane();
            const double v = p < m ? val[p] : 0.0;
            sb += wave_sum(v);
            sp += wave_sum(v >= a.pa.theta ? v : 0.0);
        }
        if (lane() == 0) {  // per-wave partial sums (p0, p1 hold at least NWV entries)
            p0[w] = sb;
            p1[w] = sp;
        }
        group_sync<NT, GS>();
        double mB = 0.0, mP = 0.0;
        for (int q = 0; q < NWV; ++q) {
            mB += p0[q];
            mP += p1[q];
        }
        group_sync<NT, GS>();
        const double d = mP - a.pa.pct * mB;
        if (!(fabs(d) > 4.0 * (double)m * 0x1p-53 * fmax(1.0, a.pa.pct) * mB)) return m;  // too close to call
        rec = d < 0.0;
    }
    if (rec) {
        fmode = 1;
        ft = (m >= a.pa.R) ? radix_kth_largest<NT, GS>([&](int p) { return val[p]; }, m, a.pa.R, hist, misc, dmisc)
                           : 0.0;
    } else if (a.pa.S > 0 && nP > a.pa.S) {
        fmode = 2;
        ft = radix_kth_largest<NT, GS>([&](int p) { return val[p]; }, m, a.pa.S, hist, misc, dmisc);
    } else {
        fmode = 0;
        ft = a.pa.theta;
    }
    int kc = 0;
    for (int b = w; b < nblk; b += NWV) {
        const int p = b * WAVE + lane();
        const bool keep = p < m && val[p] >= ft;
        if (p < m && !keep) key[p] = EMPTY_KEY;
        kc += __popcll(ballot(keep));
    }
    if (lane() == 0) wsum[w] = kc;
    group_sync<NT, GS>();
    int msort = 0;
    for (int q = 0; q < NWV; ++q) msort += wsum[q];
    group_sync<NT, GS>();
    return msort;
}

// Finishing kernel of the split sliced tables: one workgroup per column
// loads the m appended entries into LDS, sorts them by row and writes them
// (expand) or runs the fused epilogue (iterate).  Several launches of
// different sizes share a bin's columns: this one takes the columns with
// mlo < m <= mhi (CAPF >= mhi bounds its LDS arrays), and the last one also
// the columns that overflowed.  A column is finished by exactly one launch,
// which resets its counter to 0 (a value only the first launch takes, with
// mlo < 0).
template <int NT, int CAPF, int MODE>
__global__ __launch_bounds__(NT) void k_finish_part(NumericArgs a, int mlo, int mhi, int last)
{
    constexpr int NBS = CAPF / 3;  // sort buckets
    constexpr int NBLK = CAPF / WAVE + 2;
    static_assert(NBLK >= NT / WAVE, "per-wave partial sums fit p0 and p1");
    struct alignas(16) Sh {
        double val[CAPF];
        int32_t key[CAPF];
        double p0[NBLK], p1[NBLK];
        int32_t ip[NBLK];
        int32_t bcnt[NBS], bcur[NBS];
        int32_t hist[256];
        uint16_t list[CAPF], sorted[CAPF];
        int32_t misc[16];
        double dmisc[4];
        int32_t wsum[NT / WAVE];
    };
    __shared__ Sh sh __attribute__((aligned(16)));
    const int tid = threadIdx.x;
    const int64_t j = a.cols[blockIdx.x];
    if (dense_column(a, j)) return;  // whole workgroup
    const int c = a.part_cnt[j];
    const bool bad = (c & PART_OVF) || c > mhi;
    if (bad ? !last : (c <= mlo || c > mhi)) return;  // another launch's column (whole workgroup)
    __syncthreads();  // every thread has read the counter before it is reset
    if (tid == 0) a.part_cnt[j] = 0;
    if (bad) {
        if (tid == 0) {
            a.out_cnt[j] = -1;
            if (c & PART_OVF) note_exact(a, j, c);
        }
        return;
    }
    const int m = c;
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    for (int q = tid; q < m; q += NT) {
        sh.key[q] = a.out_row[base + q];
        sh.val[q] = a.out_val[base + q];
    }
    __syncthreads();
    const int32_t lo = a.lo[j];
    const int64_t span = (int64_t)a.hi[j] - lo + 1;
    if (MODE == MODE_EXPAND) {
        sort_table<NT, false, uint16_t>(sh.key, m, m, lo, span, sh.bcnt, sh.bcur, NBS, sh.list, sh.wsum,
                                        [&](int rank, int s) {
                                            a.out_row[base + rank] = sh.key[s];
                                            a.out_val[base + rank] = sh.val[s];
                                        });
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }
    Scratch<uint16_t> sc{sh.key, sh.val, sh.list, sh.sorted, sh.bcnt, sh.bcur, sh.p0, sh.p1,
                         sh.ip, sh.hist, sh.misc, sh.dmisc, sh.wsum};
    const int64_t bs = a.B.colptr[j];
    const int mj = (int)(a.B.colptr[j + 1] - bs);
    int fmode;
    double ft;
    const int msort = select_first<NT, false>(a, m, sh.key, sh.val, sh.wsum, sh.p0, sh.p1, sh.hist, sh.misc, sh.dmisc,
                                                fmode, ft);
    sort_table<NT, false, uint16_t>(sh.key, m, msort, lo, span, sh.bcnt, sh.bcur, NBS, sh.list, sh.wsum,
                                    [&](int rank, int s) { sh.sorted[rank] = (uint16_t)s; });
    __syncthreads();
    iterate_epilogue<NT, false, uint16_t>(
        a, j, msort, bs, mj, base, sh.key, sh.val, sc,
        [&](int32_t k) {
            int l = 0, h = msort;  // first rank with key >= k
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (sh.key[sh.sorted[mid]] < k) l = mid + 1;
                else h = mid;
            }
            return (l < msort && sh.key[sh.sorted[l]] == k) ? (int)sh.sorted[l] : -1;
        },
        m, fmode, ft);
}

// Finishing launches of a split bin whose columns hold at most `mmax` <=
// CAPF keys, by column size: smaller columns get smaller workgroups, several
// of which share a CU.  Each launch has one workgroup per column of the bin
// and takes the columns of its size class (the others exit at once).
template <int CAPF, int MODE>
static void finish_split(const NumericArgs &a, int mmax, hipStream_t st)
{
    constexpr int NTF = CAPF >= 6144 ? 1024 : CAPF >= 3072 ? 512 : CAPF >= 768 ? 256 : 64;
    const unsigned n = (unsigned)a.ncols;
    if constexpr (CAPF >= 6144) {
        hipLaunchKernelGGL((k_finish_part<256, 2048, MODE>), dim3(n), dim3(256), 0, st, a, -1, 2048, 0);
        hipLaunchKernelGGL((k_finish_part<512, 4096, MODE>), dim3(n), dim3(512), 0, st, a, 2048, 4096, 0);
        hipLaunchKernelGGL((k_finish_part<NTF, CAPF, MODE>), dim3(n), dim3(NTF), 0, st, a, 4096, mmax, 1);
    } else if constexpr (CAPF >= 3072) {
        hipLaunchKernelGGL((k_finish_part<256, 1024, MODE>), dim3(n), dim3(256), 0, st, a, -1, 1024, 0);
        hipLaunchKernelGGL((k_finish_part<256, 2048, MODE>), dim3(n), dim3(256), 0, st, a, 1024, 2048, 0);
        hipLaunchKernelGGL((k_finish_part<NTF, CAPF, MODE>), dim3(n), dim3(NTF), 0, st, a, 2048, mmax, 1);
    } else {
        hipLaunchKernelGGL((k_finish_part<NTF, CAPF, MODE>), dim3(n), dim3(NTF), 0, st, a, -1, mmax, 1);
    }
}

template <int NWP, int SW, int P, int MODE, int D, int CAPF, int WPE>
static void launch_part(const NumericArgs &a, hipStream_t st, hipEvent_t mid)
{
    const unsigned n = (unsigned)a.ncols;
    const unsigned grid = ((n + 7) / 8) * 8 * P;
    if constexpr (WPE == 8)
        hipLaunchKernelGGL((k_numeric_part_v64<NWP, SW, P, MODE, D>), dim3(grid), dim3(NWP * WAVE), 0, st, a);
    else
        hipLaunchKernelGGL((k_numeric_part<NWP, SW, P, MODE, D>), dim3(grid), dim3(NWP * WAVE), 0, st, a);
    if (mid) (void)hipEventRecord(mid, st);
    finish_split<CAPF, MODE>(a, CAPF, st);
}

// ---------------------------------------------------------------------------
// Persistent accumulation: one launch accumulates every column of the LDS
// bins 0-6.  A work item is one wave's share of one column: part p of P owns
// the row groups [p*64/P, (p+1)*64/P) with a private 512-slot table (bins
// 0-2: P = 1, the whole column; bins 3-6: P = slots / 512) and appends its
// keys and values, unsorted, to the column's temp slot as the split kernels
// do.  Items are numbered in schedule order -- the bins in the order the
// schedule lists them, a bin's columns in list order, a column's parts one
// after another.  The columns are dealt to eight queues, one per XCD (column
// c of a bin to queue c % 8), so the parts of a column run on one XCD and
// fetch the column's step metadata into one L2; a wave takes PERSIST_BATCH
// consecutive items at a time from its XCD's queue, then from the others,
// until none is left, so the columns of every bin (and, in a batched
// iteration, of every component) share one launch with no tail between
// bins.  The waves of a workgroup never
// synchronise with each other.  The finishing launches of every bin follow.
// ---------------------------------------------------------------------------
constexpr int PERSIST_BATCH = 4;
static_assert(PERSIST_QUEUES == 8, "one work queue per XCD");

void launch_numeric_dense(NumericMode mode, const NumericArgs &a, hipStream_t st);

// One wave: part p of the 2^LG parts of column j.
template <int MODE, int LG>
__device__ __forceinline__ void part_wave(const NumericArgs &a, int64_t j, int p, int32_t *wkey, double *wval,
                                          int32_t *wmisc, double *wdm)
{
    constexpr int SW = 512;
    constexpr int CAPW = (13 * SW) / 16;
    constexpr int G = NG >> LG;
    const int64_t col_cap = a.capv[j];
    if (lane() == 0) wmisc[0] = 0;  // keys of the column placed by this wave
    group_sync<WAVE>();
    const int keys_w = a.src_end <= NARROW_RECS
        ? slice_accumulate<SW, MODE, 2, false, true>(a, j, p * G, p * G + G, wkey, wval, &wmisc[1], CAPW, wdm,
                                                     &wmisc[0], col_cap)
        : slice_accumulate<SW, MODE, 2>(a, j, p * G, p * G + G, wkey, wval, &wmisc[1], CAPW, wdm,
                                                     &wmisc[0], col_cap);
    // as in the split kernels: a complete key count is added to the
    // column's counter even when the column overflows
    int off = -1;
    if (lane() == 0) {
        if (wmisc[1] || keys_w > CAPW || wmisc[0] > col_cap) {
            atomicOr(&a.part_cnt[j], PART_OVF | PART_INC);
        } else {
            off = atomicAdd(&a.part_cnt[j], keys_w);
            if ((off & PART_OVF) || (int64_t)(off & PART_CNT) + keys_w > col_cap) {
                atomicOr(&a.part_cnt[j], PART_OVF);
                off = -1;
            }
        }
    }
    off = __builtin_amdgcn_readfirstlane(off);
    if (off < 0) return;
    off &= PART_CNT;
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    int run = 0;
    for (int s0 = 0; s0 < SW; s0 += WAVE) {
        const int k = wkey[s0 + lane()];
        const uint64_t mk = ballot(k != EMPTY_KEY);
        if (k != EMPTY_KEY) {
            const int64_t d = base + off + run + popc_below(mk);
            a.out_row[d] = k;
            a.out_val[d] = wval[s0 + lane()];
        }
        run += __popcll(mk);
    }
}

// Six waves per SIMD: the LDS of six 4-wave workgroups (24.7 KB each) fits a
// CU, and the register budget for six (80) is what the body needs with a few
// spills (measured on the batched iterations: 0.6 % faster than the
// unconstrained 92 registers at five waves).
template <int MODE>
__global__ __launch_bounds__(4 * WAVE) __attribute__((amdgpu_waves_per_eu(6))) void k_numeric_persist(
    NumericArgs a, PersistSched s, const int32_t *__restrict__ lists, uint32_t *__restrict__ next)
{
    struct alignas(16) W {
        double val[512];
        int32_t key[512];
        int32_t misc[4];
        double dm[2];
    };
    __shared__ W ws[4];
    W &me = ws[threadIdx.x / WAVE];
    // workgroups are dealt to the XCDs in turn: a wave serves the queue of
    // its own XCD first, then helps with the others
    const int x0 = (int)(blockIdx.x % PERSIST_QUEUES);
    for (int t = 0; t < PERSIST_QUEUES; ++t) {
        const int x = (x0 + t) % PERSIST_QUEUES;
        const int32_t *first = s.qfirst[x];
        const uint32_t total = (uint32_t)first[s.n];
        for (;;) {
            uint32_t i0 = 0;
            if (lane() == 0) i0 = atomicAdd(&next[x], (uint32_t)PERSIST_BATCH);
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)i0);
            if (b0 >= total) break;  // whole wave: this queue is done
            const uint32_t b1 = min(b0 + (uint32_t)PERSIST_BATCH, total);
            for (uint32_t i = b0; i < b1; ++i) {
                int e = 0;
                while (i >= (uint32_t)first[e + 1]) ++e;
                const uint32_t loc = i - (uint32_t)first[e];
                const int lg = s.parts[e];  // log2 of the parts per column
                const uint32_t cq = loc >> lg;  // the queue's cq-th column of the entry
                const int p = (int)(loc & ((1u << lg) - 1));
                const int64_t j = lists[s.off[e] + x + PERSIST_QUEUES * cq];
                if (dense_column(a, j)) continue;  // the dense kernels own it
                switch (lg) {
                case 0: part_wave<MODE, 0>(a, j, p, me.key, me.val, me.misc, me.dm); break;
                case 1: part_wave<MODE, 1>(a, j, p, me.key, me.val, me.misc, me.dm); break;
                case 2: part_wave<MODE, 2>(a, j, p, me.key, me.val, me.misc, me.dm); break;
                case 3: part_wave<MODE, 3>(a, j, p, me.key, me.val, me.misc, me.dm); break;
                default: part_wave<MODE, 4>(a, j, p, me.key, me.val, me.misc, me.dm); break;
                }
            }
        }
    }
}

// log2 of the parts per column of a bin (bins 0-2: one part)
static int split_parts_log2(int bin) { return bin <= 2 ? 0 : bin - 2; }

bool persist_fits(const int32_t counts[8])
{
    int64_t items = 0;
    for (int b = 0; b < NUM_LDS_BINS; ++b) items += (int64_t)counts[b] << split_parts_log2(b);
    return items < ((int64_t)1 << 30);  // 32-bit work counter with room for the overshoot
}

void launch_numeric_persist(NumericMode mode, const NumericArgs &a0, const int32_t *lists, const int32_t counts[8],
                            const int64_t *dense_bin, uint32_t *next, bool light_first, hipStream_t st,
                            hipEvent_t mid)
{
    NumericArgs a = a0;
    int32_t off[NUM_LDS_BINS];
    int32_t o = 0;
    for (int b = 0; b < NUM_LDS_BINS; ++b) {
        off[b] = o;
        o += counts[b];
    }
    // dense columns (bins 3-6) first: their own kernels
    for (int b = 3; b < NUM_LDS_BINS; ++b) {
        if (counts[b] == 0 || !a0.dense || (dense_bin && dense_bin[b] == 0)) continue;
        a.cols = lists + off[b];
        a.ncols = counts[b];
        launch_numeric_dense(mode, a, st);
    }
    // schedule: the heaviest bins first (or, by the policy, the lightest);
    // column c of a bin goes to queue c % PERSIST_QUEUES, whose items are
    // numbered entry by entry
    PersistSched s{};
    for (int k = 0; k < NUM_LDS_BINS; ++k) {
        const int b = light_first ? k : NUM_LDS_BINS - 1 - k;
        if (counts[b] == 0) continue;
        const int e = s.n++;
        s.bin[e] = b;
        s.parts[e] = split_parts_log2(b);
        s.off[e] = off[b];
    }
    int64_t items = 0;
    for (int x = 0; x < PERSIST_QUEUES; ++x) {
        int64_t f = 0;
        s.qfirst[x][0] = 0;
        for (int e = 0; e < s.n; ++e) {
            const int64_t cols = counts[s.bin[e]] > x ? (counts[s.bin[e]] - x + PERSIST_QUEUES - 1) / PERSIST_QUEUES : 0;
            f += cols << s.parts[e];
            s.qfirst[x][e + 1] = (int32_t)f;
        }
        for (int e = s.n + 1; e <= NUM_LDS_BINS; ++e) s.qfirst[x][e] = (int32_t)f;
        items += f;
    }
    if (s.n > 0) {
        static unsigned resident[2] = {0, 0};
        const int mi = mode == MODE_EXPAND ? 0 : 1;
        if (resident[mi] == 0) {
            int per_cu = 0, cus = 0, dev = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (mode == MODE_EXPAND)
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_numeric_persist<MODE_EXPAND>, 4 * WAVE, 0);
            else
                (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_numeric_persist<MODE_ITERATE>, 4 * WAVE,
                                                                   0);
            resident[mi] = (unsigned)std::max(1, per_cu) * (unsigned)std::max(1, cus);
        }
        const unsigned grid =
            (unsigned)std::min<int64_t>(resident[mi], (items + 4 * PERSIST_BATCH - 1) / (4 * PERSIST_BATCH));
        (void)hipMemsetAsync(next, 0, PERSIST_QUEUES * sizeof(uint32_t), st);
        if (mode == MODE_EXPAND)
            hipLaunchKernelGGL(k_numeric_persist<MODE_EXPAND>, dim3(grid), dim3(4 * WAVE), 0, st, a0, s, lists, next);
        else
            hipLaunchKernelGGL(k_numeric_persist<MODE_ITERATE>, dim3(grid), dim3(4 * WAVE), 0, st, a0, s, lists,
                               next);
    }
    if (mid) (void)hipEventRecord(mid, st);
    // finishing, bin by bin
    for (int b = 0; b < NUM_LDS_BINS; ++b) {
        if (counts[b] == 0) continue;
        a.cols = lists + off[b];
        a.ncols = counts[b];
        a.dense = (dense_bin && dense_bin[b] == 0) ? nullptr : a0.dense;
        const int cap = bin_cap_c(b);
#define MCL_FIN(CAPF_)                                                              \
    do {                                                                            \
        if (mode == MODE_EXPAND) finish_split<CAPF_, MODE_EXPAND>(a, cap, st);      \
        else finish_split<CAPF_, MODE_ITERATE>(a, cap, st);                         \
    } while (0)
        switch (b) {
        case 0: case 1: case 2: MCL_FIN(384); break;
        case 3: MCL_FIN(768); break;
        case 4: MCL_FIN(1536); break;
        case 5: MCL_FIN(3072); break;
        default: MCL_FIN(6144); break;
        }
#undef MCL_FIN
    }
}

// ---------------------------------------------------------------------------
// Dense accumulator: a column whose product rows span at most SPAN
// consecutive rows (lo_j .. hi_j from the symbolic pass) and that does at
// least two multiply-adds per row of that span is accumulated in an LDS
// array indexed by row - lo_j instead of a hash table: no probing, and the
// occupied rows come out in ascending order from a bitmap, so the column
// needs no sort.  As in the sliced-table kernels, wave w owns the rows of
// the hash groups [w*G, (w+1)*G), so a row's products arrive in ascending k
// from one wave.  The number of distinct rows is exact, so a column that
// does not fit its planned slot reports its exact count.
// ---------------------------------------------------------------------------
template <int NW, int SPAN, int MODE>
__global__ __launch_bounds__(NW * WAVE) void k_numeric_dense(NumericArgs a, int span_min)
{
    constexpr int NT = NW * WAVE;
    constexpr int G = NG / NW;
    constexpr int NWORD = SPAN / 32;
    constexpr int NBLK = SPAN / WAVE + 2;
    struct alignas(16) Sh {
        double acc[SPAN];
        uint32_t bits[NWORD];
        int32_t wcnt[NWORD];
        uint16_t sorted[SPAN], list[SPAN];
        double p0[NBLK], p1[NBLK];
        int32_t ip[NBLK];
        int32_t hist[256];
        int32_t misc[16];
        double dmisc[4];
        int32_t wsum[NW];
    };
    __shared__ Sh sh __attribute__((aligned(16)));
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    const int64_t j = a.cols[blockIdx.x];
    if (!dense_column(a, j)) return;  // whole workgroup
    const int32_t lo = a.lo[j];
    const int span = a.hi[j] - lo + 1;
    if (span > SPAN || span <= span_min) return;  // the other size's column
    const int nword = (span + 31) / 32;
    for (int s = tid; s < span; s += NT) sh.acc[s] = 0.0;
    for (int q = tid; q < nword; q += NT) sh.bits[q] = 0u;
    __syncthreads();
    slice_accumulate<512, MODE, 2, true>(a, j, w * G, (w + 1) * G, nullptr, sh.acc, nullptr, 0, &sh.dmisc[3],
                                         nullptr, 0, lo, sh.bits);
    __syncthreads();
    // occupancy: a nonzero sum, or a row whose products all underflowed;
    // each wave takes 64 consecutive slots per step (two bitmap words)
    for (int s0 = tid - lane(); s0 < span; s0 += NT) {
        const int s = s0 + lane();
        const uint64_t nz = ballot(s < span && sh.acc[s] != 0.0);
        if (lane() == 0) {
            sh.bits[s0 >> 5] |= (uint32_t)nz;
            if ((s0 >> 5) + 1 < nword) sh.bits[(s0 >> 5) + 1] |= (uint32_t)(nz >> 32);
        }
    }
    __syncthreads();
    // occupied rows in ascending order: word counts, their prefix, then the
    // set bits of every word
    for (int q = tid; q < nword; q += NT) sh.wcnt[q] = __popc(sh.bits[q]);
    __syncthreads();
    const int m = block_exscan<NT>(sh.wcnt, nword, sh.wsum);
    const int64_t cap = a.capv ? a.capv[j] : (int64_t)span;
    if (m > cap) {
        if (tid == 0) {
            a.out_cnt[j] = -1;
            if (a.exact_cnt) a.exact_cnt[j] = m;
        }
        return;
    }
    for (int q = tid; q < nword; q += NT) {
        uint32_t b = sh.bits[q];
        int pos = sh.wcnt[q];
        while (b) {
            const int t = __ffs(b) - 1;
            sh.sorted[pos++] = (uint16_t)(q * 32 + t);
            b &= b - 1;
        }
    }
    __syncthreads();
    const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
    if (MODE == MODE_EXPAND) {
        for (int i = tid; i < m; i += NT) {
            const int s = sh.sorted[i];
            a.out_row[base + i] = lo + s;
            a.out_val[base + i] = sh.acc[s];
        }
        if (tid == 0) a.out_cnt[j] = m;
        return;
    }
    struct RowOf {
        int32_t lo;
        __device__ int32_t operator[](int s) const { return lo + s; }
    };
    Scratch<uint16_t> sc{nullptr, sh.acc, sh.list, sh.sorted, nullptr, nullptr, sh.p0, sh.p1,
                         sh.ip, sh.hist, sh.misc, sh.dmisc, sh.wsum};
    const int64_t bs = a.B.colptr[j];
    const int mj = (int)(a.B.colptr[j + 1] - bs);
    iterate_epilogue<NT, false, uint16_t>(a, j, m, bs, mj, base, RowOf{lo}, sh.acc, sc, [&](int32_t k) {
        const int s = k - lo;
        return (s >= 0 && s < span && ((sh.bits[s >> 5] >> (s & 31)) & 1u)) ? s : -1;
    });
}

// Dense launches over a bin's column list: spans up to 4096 rows with 8
// waves (three workgroups per CU), up to DENSE_SPAN with 16.
void launch_numeric_dense(NumericMode mode, const NumericArgs &a, hipStream_t st)
{
    if (a.ncols <= 0 || !a.dense || !a.goff || mode == MODE_COUNT) return;
    const unsigned n = (unsigned)a.ncols;
    if (mode == MODE_EXPAND) {
        hipLaunchKernelGGL((k_numeric_dense<8, 4096, MODE_EXPAND>), dim3(n), dim3(8 * WAVE), 0, st, a, 0);
        hipLaunchKernelGGL((k_numeric_dense<16, DENSE_SPAN, MODE_EXPAND>), dim3(n), dim3(16 * WAVE), 0, st, a,
                           4096);
    } else {
        hipLaunchKernelGGL((k_numeric_dense<8, 4096, MODE_ITERATE>), dim3(n), dim3(8 * WAVE), 0, st, a, 0);
        hipLaunchKernelGGL((k_numeric_dense<16, DENSE_SPAN, MODE_ITERATE>), dim3(n), dim3(16 * WAVE), 0, st, a,
                           4096);
    }
}

// Columns for the dense kernels: planned in bin 3 or above, row span of at
// most DENSE_SPAN rows and at least two multiply-adds per row of the span
// (dense_shape; such columns are planned by their span, so they fit).
__global__ __launch_bounds__(256) void k_mark_dense(int64_t ncols, const int32_t *__restrict__ bin,
                                                    const int64_t *__restrict__ flops,
                                                    const int32_t *__restrict__ lo, const int32_t *__restrict__ hi,
                                                    uint8_t *__restrict__ dense,
                                                    unsigned long long *__restrict__ count)
{
    // count[b]: dense columns planned in bin b
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x; j0 < ncols; j0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = j0 + threadIdx.x;
        int b = -1;
        if (j < ncols) {
            const bool d = bin[j] >= 3 && dense_shape(flops[j], (int64_t)hi[j] - lo[j] + 1);
            dense[j] = d ? 1 : 0;
            if (d) b = bin[j];
        }
        for (int q = 3; q <= NUM_LDS_BINS; ++q) {
            const uint64_t m = ballot(b == q);
            if (m && lane() == __ffsll((long long)m) - 1) atomicAdd(&count[q], (unsigned long long)__popcll(m));
        }
    }
}

void launch_mark_dense(int64_t ncols, const int32_t *bin, const int64_t *flops, const int32_t *lo,
                       const int32_t *hi, uint8_t *dense, int64_t *count, hipStream_t st)
{
    if (ncols <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((ncols + 255) / 256, 8192);
    hipLaunchKernelGGL(k_mark_dense, dim3(g), dim3(256), 0, st, ncols, bin, flops, lo, hi, dense,
                       (unsigned long long *)count);
}

// ---------------------------------------------------------------------------
// Columns too large for one LDS table set (bin 7): the split kernels above
// with 64 waves per column append their keys and values, unsorted, to the
// column's output slot; the finishing kernel below sorts them and runs the
// epilogue.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool multipass_column(const NumericArgs &a, int64_t j)
{
    return a.goff && a.capv && !(a.hbm_only && a.hbm_only[j]) && a.capv[j] <= MP_MAX;
}

// Finishing pass for the multi-pass columns: copies the m appended entries
// (count and overflow flags in part_cnt, reset here) to HBM scratch, sorts
// them by row, then writes them (expand) or runs the fused epilogue on them
// (iterate).  Persistent workgroups with one scratch slab each, like the
// HBM-table kernel.
template <int MODE>
__global__ __launch_bounds__(1024) void k_finish_mpass(NumericArgs a, char *slab, size_t slab_bytes)
{
    constexpr int NT = 1024;
    constexpr int SM = (int)MP_MAX;
    constexpr int NB = SM / 4;
    constexpr int NBLK = SM / WAVE + 2;
    __shared__ int32_t hist[256];
    __shared__ int32_t misc[16];
    __shared__ double dmisc[4];
    __shared__ int32_t wsum[NT / WAVE];
    char *my = slab + (size_t)blockIdx.x * slab_bytes;
    int32_t *skey = (int32_t *)my;
    double *sval = (double *)(my + (size_t)SM * 4);
    int32_t *list = (int32_t *)(my + (size_t)SM * 12);
    int32_t *sorted = list + SM;
    int32_t *bcnt = sorted + SM;
    int32_t *bcur = bcnt + NB;
    int32_t *ip = bcur + NB;
    double *p0 = (double *)(ip + NBLK + (NBLK & 1));
    double *p1 = p0 + NBLK;
    Scratch<int32_t> sc{skey, sval, list, sorted, bcnt, bcur, p0, p1, ip, hist, misc, dmisc, wsum};
    const int tid = threadIdx.x;
    for (int64_t idx = blockIdx.x; idx < a.ncols; idx += gridDim.x) {
        const int64_t j = a.cols[idx];
        if (!multipass_column(a, j) || dense_column(a, j)) continue;
        const int c = a.part_cnt[j];
        __syncthreads();  // every thread has read the counter before it is reset
        if (tid == 0) a.part_cnt[j] = 0;
        if ((c & PART_OVF) || c > (int)MP_MAX) {
            if (tid == 0) {
                a.out_cnt[j] = -1;
                if (c & PART_OVF) note_exact(a, j, c);
            }
            continue;
        }
        const int m = c;
        const int64_t base = a.out_base[j] >= 0 ? a.out_base[j] : ((-a.out_base[j] - 1) & REGION_MASK);
        for (int q = tid; q < m; q += NT) {
            skey[q] = a.out_row[base + q];
            sval[q] = a.out_val[base + q];
        }
        __syncthreads();
        const int32_t lo = a.lo[j];
        const int64_t span = (int64_t)a.hi[j] - lo + 1;
        if (MODE == MODE_EXPAND) {
            sort_table<NT, true, int32_t>(skey, m, m, lo, span, bcnt, bcur, NB, list, wsum, [&](int rank, int s) {
                a.out_row[base + rank] = skey[s];
                a.out_val[base + rank] = sval[s];
            });
            if (tid == 0) a.out_cnt[j] = m;
        } else {
            int fmode;
            double ft;
            const int msort = select_first<NT, true>(a, m, skey, sval, wsum, p0, p1, hist, misc, dmisc, fmode, ft);
            sort_table<NT, true, int32_t>(skey, m, msort, lo, span, bcnt, bcur, NB, list, wsum,
                                          [&](int rank, int s) { sorted[rank] = s; });
            __syncthreads();
            const int64_t bs = a.B.colptr[j];
            const int mj = (int)(a.B.colptr[j + 1] - bs);
            iterate_epilogue<NT, true, int32_t>(
                a, j, msort, bs, mj, base, skey, sval, sc,
                [&](int32_t k) {
                    int l = 0, h = msort;  // first rank with key >= k
                    while (l < h) {
                        const int mid = (l + h) >> 1;
                        if (skey[sorted[mid]] < k) l = mid + 1;
                        else h = mid;
                    }
                    return (l < msort && skey[sorted[l]] == k) ? sorted[l] : -1;
                },
                m, fmode, ft);
        }
        __syncthreads();
    }
}

size_t mpass_slab_bytes()
{
    const size_t SM = (size_t)MP_MAX, NB = SM / 4, NBLK = SM / WAVE + 2;
    return ((SM * 20 + NB * 8 + (NBLK + (NBLK & 1)) * 4 + NBLK * 16) + 255) & ~(size_t)255;
}

void launch_numeric_mpass(NumericMode mode, const NumericArgs &a, void *slab, size_t slab_bytes, int nslabs,
                          hipStream_t st)
{
    if (a.ncols <= 0 || !a.goff || !a.part_cnt || mode == MODE_COUNT) return;
    launch_numeric_dense(mode, a, st);
    const int grid = std::min(nslabs, a.ncols);
    const unsigned g8 = (unsigned)(((a.ncols + 7) / 8) * 8);
    if (mode == MODE_EXPAND) {
        hipLaunchKernelGGL(k_numeric_mpart_small<MODE_EXPAND>, dim3(g8 * MPS_P), dim3(MPS_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_numeric_mpart<MODE_EXPAND>, dim3(g8 * MPP_P), dim3(MPP_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_numeric_mpart_wide<MODE_EXPAND>, dim3(g8 * MPW_P), dim3(MPW_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_finish_mpass<MODE_EXPAND>, dim3(grid), dim3(1024), 0, st, a, (char *)slab, slab_bytes);
    } else {
        hipLaunchKernelGGL(k_numeric_mpart_small<MODE_ITERATE>, dim3(g8 * MPS_P), dim3(MPS_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_numeric_mpart<MODE_ITERATE>, dim3(g8 * MPP_P), dim3(MPP_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_numeric_mpart_wide<MODE_ITERATE>, dim3(g8 * MPW_P), dim3(MPW_NW * WAVE), 0, st, a);
        hipLaunchKernelGGL(k_finish_mpass<MODE_ITERATE>, dim3(grid), dim3(1024), 0, st, a, (char *)slab,
                           slab_bytes);
    }
}

// Launch shapes per bin: (slots, waves per column, columns per workgroup,
// entries per lane per chunk, chunks per group, double-buffered groups), or
// the sliced-table kernel (waves, chunks per group; reads the sliced source
// layout).  Variant 0 is the fastest shape measured on the 1M-vertex planted
// graph; the others are alternatives the tuner may select through
// mcl_params.bin_policy (4 bits per bin).  Exact-count launches use the
// shared-table shape (shared_table_variant).
template <int MODE>
static void launch_lds_mode(int bin, int variant, const NumericArgs &a, hipStream_t st, hipEvent_t mid = nullptr)
{
    const int n = a.ncols;
    if (n <= 0) return;
#define MCL_LAUNCH(S_, NW_, CPW_, E_, D_, P_)                                               \
    hipLaunchKernelGGL((k_numeric_lds<S_, NW_, CPW_, MODE, E_, D_, P_>),                    \
                       dim3((n + CPW_ - 1) / CPW_), dim3(NW_ * WAVE * CPW_), 0, st, a)
#define MCL_SPLIT_W(NW_, SW_, D_)                                                            \
    if constexpr (MODE != MODE_COUNT)                                                        \
        hipLaunchKernelGGL((k_numeric_hsplit<NW_, SW_, MODE, D_>), dim3(n), dim3(NW_ * WAVE), 0, st, a)
#define MCL_SPLIT(NW_, D_) MCL_SPLIT_W(NW_, 512, D_)
#define MCL_PART(NWP_, SW_, P_, D_, CAPF_, WPE_)                                             \
    if constexpr (MODE != MODE_COUNT) launch_part<NWP_, SW_, P_, MODE, D_, CAPF_, WPE_>(a, st, mid)
    switch (bin * 8 + variant) {
    case 0: MCL_LAUNCH(128, 1, 4, 2, 4, false); break;
    case 1: MCL_LAUNCH(128, 1, 4, 1, 8, false); break;
    case 8: MCL_LAUNCH(256, 1, 4, 2, 4, false); break;
    case 9: MCL_LAUNCH(256, 1, 4, 1, 8, false); break;
    case 16: MCL_LAUNCH(512, 1, 4, 2, 4, false); break;
    case 17: MCL_LAUNCH(512, 1, 4, 2, 8, false); break;
    case 24: MCL_SPLIT(2, 4); break;
    case 25: MCL_LAUNCH(1024, 2, 1, 2, 4, false); break;
    case 26: MCL_LAUNCH(1024, 2, 1, 2, 4, true); break;
    case 27: MCL_LAUNCH(1024, 1, 2, 4, 4, false); break;
    case 28: MCL_PART(1, 512, 2, 2, 768, 1); break;
    case 29: MCL_PART(1, 512, 2, 2, 768, 8); break;
    case 32: MCL_SPLIT(4, 4); break;
    case 33: MCL_LAUNCH(2048, 4, 1, 2, 4, false); break;
    case 34: MCL_LAUNCH(2048, 4, 1, 2, 4, true); break;
    case 35: MCL_LAUNCH(2048, 4, 1, 1, 8, true); break;
    case 36: MCL_PART(2, 512, 2, 2, 1536, 1); break;
    case 37: MCL_PART(1, 512, 4, 2, 1536, 1); break;
    case 38: MCL_PART(1, 512, 4, 2, 1536, 8); break;
    case 40: MCL_SPLIT(8, 4); break;
    case 41: MCL_LAUNCH(4096, 8, 1, 1, 4, false); break;
    case 42: MCL_LAUNCH(4096, 8, 1, 1, 4, true); break;
    case 43: MCL_SPLIT(8, 8); break;
    case 44: MCL_LAUNCH(4096, 8, 1, 1, 8, false); break;
    case 45: MCL_PART(4, 512, 2, 2, 3072, 1); break;
    case 46: MCL_PART(2, 512, 4, 2, 3072, 1); break;
    case 47: MCL_PART(1, 512, 8, 2, 3072, 1); break;
    case 48: MCL_SPLIT(16, 4); break;
    case 49: MCL_LAUNCH(8192, 16, 1, 1, 4, false); break;
    case 50: MCL_LAUNCH(8192, 16, 1, 1, 4, true); break;
    case 51: MCL_LAUNCH(8192, 16, 1, 1, 8, true); break;
    case 52: MCL_LAUNCH(8192, 16, 1, 1, 8, false); break;
    case 53: MCL_SPLIT(16, 2); break;
    case 54: MCL_PART(2, 512, 8, 2, 6144, 1); break;
    case 55: MCL_PART(1, 512, 16, 2, 6144, 1); break;
    case 56: MCL_PART(4, 512, 4, 2, 6144, 8); break;
    case 57: MCL_PART(8, 512, 2, 2, 6144, 1); break;
    case 58: MCL_PART(2, 512, 8, 2, 6144, 8); break;
    case 59: MCL_PART(8, 512, 2, 2, 6144, 8); break;
    case 60: MCL_PART(4, 512, 4, 2, 6144, 1); break;
    case 61: MCL_PART(1, 512, 16, 2, 6144, 8); break;
    case 62: MCL_PART(4, 512, 4, 1, 6144, 8); break;
    default: launch_lds_mode<MODE>(bin, 0, a, st); break;
    }
#undef MCL_PART
#undef MCL_SPLIT
#undef MCL_SPLIT_W
#undef MCL_LAUNCH
}

bool lds_variant_sliced(int bin, int variant)
{
    return (bin >= 3 && bin <= 6 && variant == 0) || (bin == 5 && variant == 3) || lds_variant_split(bin, variant) ||
           (bin == 6 && variant == 5);
}

bool lds_variant_split(int bin, int variant)
{
    return (bin == 3 && variant >= 4) || (bin == 4 && variant >= 4) || (bin == 5 && variant >= 5) ||
           (bin == 6 && variant >= 6);
}

// Launch used by exact counts (a mode the sliced kernels do not serve): the
// shared-table shape of the bin.
static int shared_table_variant(int bin) { return (bin >= 3 && bin <= 6) ? 1 : 0; }

int lds_bin_variants(int bin)
{
    static const int nv[NUM_LDS_BINS] = {2, 2, 2, 6, 7, 8, 15};
    return (bin >= 0 && bin < NUM_LDS_BINS) ? nv[bin] : 1;
}

void launch_numeric_lds(int bin, int variant, NumericMode mode, const NumericArgs &a, hipStream_t st,
                        hipEvent_t mid)
{
    if (bin >= 3 && a.dense && mode != MODE_COUNT) launch_numeric_dense(mode, a, st);
    if (lds_variant_split(bin, variant) && !a.part_cnt) variant = 0;
    if (lds_variant_sliced(bin, variant) && !a.goff) variant = shared_table_variant(bin);
    switch (mode) {
    case MODE_COUNT: launch_lds_mode<MODE_COUNT>(bin, shared_table_variant(bin), a, st); break;
    case MODE_EXPAND: launch_lds_mode<MODE_EXPAND>(bin, variant, a, st, mid); break;
    case MODE_ITERATE: launch_lds_mode<MODE_ITERATE>(bin, variant, a, st, mid); break;
    }
}

// ---------------------------------------------------------------------------
// HBM-table kernel: persistent workgroups, each with a private slab of
// device memory holding the table and the sort scratch for one column at a
// time.  Used for columns whose table does not fit LDS and for the exact
// count of overflowed columns.
// ---------------------------------------------------------------------------
struct SlabLayout {
    size_t key, val, list, sorted, bcnt, bcur, p0, p1, ip, bytes;
};
static __host__ __device__ SlabLayout slab_layout(int S, int cap)
{
    const int NB = (S / 4 < 64) ? 64 : S / 4;
    const int NBLK = cap / WAVE + 2;
    SlabLayout L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) & ~(size_t)255; return r; };
    L.val = take((size_t)S * 8);
    L.key = take((size_t)S * 4);
    L.list = take((size_t)cap * 4);
    L.sorted = take((size_t)cap * 4);
    L.bcnt = take((size_t)NB * 4);
    L.bcur = take((size_t)NB * 4);
    L.p0 = take((size_t)NBLK * 8);
    L.p1 = take((size_t)NBLK * 8);
    L.ip = take((size_t)NBLK * 4);
    L.bytes = o;
    return L;
}
size_t global_slab_bytes(int S, int cap) { return slab_layout(S, cap).bytes; }

template <int MODE>
__global__ __launch_bounds__(1024) void k_numeric_global(NumericArgs a, int S, int cap, char *slab,
                                                         size_t slab_bytes)
{
    constexpr int NT = 1024;
    __shared__ int32_t hist[256];
    __shared__ int32_t misc[16];
    __shared__ double dmisc[4];
    __shared__ int32_t wsum[NT / WAVE];
    const SlabLayout L = slab_layout(S, cap);
    char *my = slab + (size_t)blockIdx.x * slab_bytes;
    Scratch<int32_t> sc{(int32_t *)(my + L.key), (double *)(my + L.val), (int32_t *)(my + L.list),
                        (int32_t *)(my + L.sorted), (int *)(my + L.bcnt), (int *)(my + L.bcur),
                        (double *)(my + L.p0), (double *)(my + L.p1), (int *)(my + L.ip),
                        hist, misc, dmisc, wsum};
    const int NB = (S / 4 < 64) ? 64 : S / 4;
    const int logS = __builtin_ctz((unsigned)S);
    for (int64_t idx = blockIdx.x; idx < a.ncols; idx += gridDim.x) {
        const int64_t j = a.cols[idx];
        // columns of the multi-pass LDS kernel are done there (not in count mode)
        if (MODE != MODE_COUNT && (multipass_column(a, j) || dense_column(a, j))) continue;
        column_body<NT, MODE, 1, 2, int32_t, true>(a, j, S, logS, cap, NB, sc);
        __syncthreads();
    }
}

void launch_numeric_global(NumericMode mode, const NumericArgs &a, int S, int cap, void *slab,
                           size_t slab_bytes, int nslabs, hipStream_t st)
{
    if (a.ncols <= 0) return;
    const int grid = std::min(nslabs, a.ncols);
    switch (mode) {
    case MODE_COUNT:
        hipLaunchKernelGGL((k_numeric_global<MODE_COUNT>), dim3(grid), dim3(1024), 0, st, a, S,
                           cap, (char *)slab, slab_bytes);
        break;
    case MODE_EXPAND:
        hipLaunchKernelGGL((k_numeric_global<MODE_EXPAND>), dim3(grid), dim3(1024), 0, st, a, S,
                           cap, (char *)slab, slab_bytes);
        break;
    case MODE_ITERATE:
        hipLaunchKernelGGL((k_numeric_global<MODE_ITERATE>), dim3(grid), dim3(1024), 0, st, a,
                           S, cap, (char *)slab, slab_bytes);
        break;
    }
}

// ---------------------------------------------------------------------------
// overflow list, scans, compaction, batched-mode helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_collect_overflow(const int32_t *__restrict__ cols, int32_t n,
                                                          const int64_t *__restrict__ cnt,
                                                          int32_t *__restrict__ list,
                                                          int32_t *__restrict__ count)
{
    for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
        const int i = i0 + threadIdx.x;
        const int j = (i < n) ? cols[i] : 0;
        const bool o = (i < n) && cnt[j] < 0;
        const int pos = wave_reserve<1>(count, 0, o);
        if (o) list[pos] = j;
    }
}

void launch_collect_overflow(int64_t, const int32_t *cols, int32_t n, const int64_t *cnt,
                             int32_t *ovf_list, int32_t *ovf_count, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_collect_overflow, dim3(grid), dim3(256), 0, st, cols, n, cnt, ovf_list,
                       ovf_count);
}

// Exclusive scan of int64 (three phases: per-block sums, scan of the block
// sums, add back).  out may alias in; out has n+1 entries (out[n] = total).
constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_ITEMS = 8;
constexpr int64_t SCAN_TILE = (int64_t)SCAN_BLOCK * SCAN_ITEMS;

__device__ int64_t block_incl_scan_i64(int64_t x, int64_t *ws)
{
    const int tid = threadIdx.x, w = tid / WAVE;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int64_t y = __shfl_up(x, d, WAVE);
        if (lane() >= d) x += y;
    }
    if (lane() == WAVE - 1) ws[w] = x;
    __syncthreads();
    if (w == 0) {
        int64_t v = (lane() < SCAN_BLOCK / WAVE) ? ws[lane()] : 0;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int64_t y = __shfl_up(v, d, WAVE);
            if (lane() >= d) v += y;
        }
        if (lane() < SCAN_BLOCK / WAVE) ws[lane()] = v;
    }
    __syncthreads();
    const int64_t add = (w > 0) ? ws[w - 1] : 0;
    __syncthreads();
    return x + add;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const int64_t *__restrict__ in, int64_t n,
                                                           int64_t *__restrict__ tile_sum)
{
    __shared__ int64_t ws[SCAN_BLOCK / WAVE];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = t0 + (int64_t)q * SCAN_BLOCK + threadIdx.x;
        if (i < n) s += in[i];
    }
    const int64_t inc = block_incl_scan_i64(s, ws);
    if (threadIdx.x == SCAN_BLOCK - 1) tile_sum[blockIdx.x] = inc;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(int64_t *__restrict__ tile_sum, int64_t ntiles)
{
    __shared__ int64_t ws[SCAN_BLOCK / WAVE];
    __shared__ int64_t last;
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += SCAN_BLOCK) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = (i < ntiles) ? tile_sum[i] : 0;
        const int64_t inc = block_incl_scan_i64(v, ws);
        if (i < ntiles) tile_sum[i] = carry + inc - v;  // exclusive
        if (threadIdx.x == SCAN_BLOCK - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int64_t *__restrict__ in, int64_t n,
                                                           const int64_t *__restrict__ tile_sum,
                                                           int64_t *__restrict__ out)
{
    __shared__ int64_t ws[SCAN_BLOCK / WAVE];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    // each thread owns SCAN_ITEMS consecutive elements
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = t0 + (int64_t)threadIdx.x * SCAN_ITEMS + q;
        v[q] = (i < n) ? in[i] : 0;
        s += v[q];
    }
    const int64_t inc = block_incl_scan_i64(s, ws);
    int64_t run = tile_sum[blockIdx.x] + inc - s;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = t0 + (int64_t)threadIdx.x * SCAN_ITEMS + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) out[n] = tile_sum[gridDim.x];
}

int64_t exscan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 2; }

void launch_exscan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t st)
{
    const int64_t ntiles = std::max<int64_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, st, tmp, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, st, in, n, tmp, out);
}

// Copy each column's entries from its temp slot to its final position.  One
// wave per column.
// Copy every column from its temp slot (region and offset decoded from
// base) to its final position.  Columns with bin < 0 (inactive) are skipped.
__global__ __launch_bounds__(256) void k_compact(int64_t ncols, const int32_t *__restrict__ bin,
                                                 const int64_t *__restrict__ base,
                                                 const int64_t *__restrict__ cnt,
                                                 const int64_t *__restrict__ colptr, TempRegions tr,
                                                 int32_t *__restrict__ row, double *__restrict__ val)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= ncols) return;
    if (bin && bin[j] < 0) return;
    const int64_t n = cnt[j];
    if (n <= 0) return;
    const int64_t b = base[j], d = colptr[j];
    int reg = 0;
    int64_t o = b;
    if (b < 0) {
        const int64_t v = -b - 1;
        reg = (int)(v >> 48);
        o = v & REGION_MASK;
    }
    const int32_t *sr = tr.row[reg] + o;
    const double *sv = tr.val[reg] + o;
    for (int64_t q = lane(); q < n; q += WAVE) {
        row[d + q] = sr[q];
        val[d + q] = sv[q];
    }
}

void launch_compact(int64_t ncols, const int32_t *bin, const int64_t *base, const int64_t *cnt,
                    const int64_t *colptr, const TempRegions &tr, int32_t *row, double *val,
                    hipStream_t st)
{
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, st, ncols, bin, base,
                       cnt, colptr, tr, row, val);
}

// Batched mode: the component of every column and whether it is active.
__global__ void k_col_comp(int64_t ncols, const int64_t *__restrict__ comp_ptr, int64_t ncomp,
                           int32_t *__restrict__ col_comp, const uint8_t *__restrict__ active,
                           uint8_t *__restrict__ col_active)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncomp;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t act = active ? active[c] : 1;
        for (int64_t j = comp_ptr[c]; j < comp_ptr[c + 1]; ++j) {
            col_comp[j] = (int32_t)c;
            col_active[j] = act;
        }
    }
}

void launch_col_comp(int64_t ncols, const int64_t *comp_ptr, int64_t ncomp, int32_t *col_comp,
                     const uint8_t *active, uint8_t *col_active, hipStream_t st)
{
    if (ncomp == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((ncomp + 255) / 256, 4096);
    hipLaunchKernelGGL(k_col_comp, dim3(grid), dim3(256), 0, st, ncols, comp_ptr, ncomp, col_comp,
                       active, col_active);
}

// Inactive (frozen) columns keep their previous entries: count = nnz, change 0.
__global__ void k_counts_inactive(DevCSC A, const int32_t *__restrict__ col_comp,
                                  const uint8_t *__restrict__ active, int64_t *__restrict__ cnt,
                                  double *__restrict__ delta)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < A.ncols;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (!active[col_comp[j]]) {
            cnt[j] = A.colptr[j + 1] - A.colptr[j];
            delta[j] = 0.0;
        }
    }
}

void launch_counts_inactive(const DevCSC &A, const int32_t *col_comp, const uint8_t *active,
                            int64_t *cnt, double *delta, hipStream_t st)
{
    if (A.ncols == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((A.ncols + 255) / 256, 4096);
    hipLaunchKernelGGL(k_counts_inactive, dim3(grid), dim3(256), 0, st, A, col_comp, active, cnt, delta);
}

__global__ __launch_bounds__(256) void k_copy_inactive(DevCSC A, const int32_t *__restrict__ col_comp,
                                                       const uint8_t *__restrict__ active,
                                                       const int64_t *__restrict__ colptr,
                                                       int32_t *__restrict__ row, double *__restrict__ val)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j >= A.ncols || active[col_comp[j]]) return;
    const int64_t s = A.colptr[j], n = A.colptr[j + 1] - s, d = colptr[j];
    for (int64_t q = lane(); q < n; q += WAVE) {
        row[d + q] = A.rowidx[s + q];
        val[d + q] = A.val[s + q];
    }
}

void launch_copy_inactive(const DevCSC &A, const int32_t *col_comp, const uint8_t *active,
                          const int64_t *colptr, int32_t *row, double *val, hipStream_t st)
{
    if (A.ncols == 0) return;
    hipLaunchKernelGGL(k_copy_inactive, dim3((unsigned)((A.ncols + 3) / 4)), dim3(256), 0, st, A,
                       col_comp, active, colptr, row, val);
}

// Per-component max of the per-column change.  One wave per component.
__global__ __launch_bounds__(256) void k_comp_max(int64_t ncomp, const int64_t *__restrict__ comp_ptr,
                                                  const double *__restrict__ delta, double *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (c >= ncomp) return;
    double m = 0.0;
    for (int64_t j = comp_ptr[c] + lane(); j < comp_ptr[c + 1]; j += WAVE) m = fmax(m, delta[j]);
    m = wave_max(m);
    if (lane() == 0) out[c] = m;
}

void launch_comp_max(int64_t ncomp, const int64_t *comp_ptr, const double *delta, double *out,
                     hipStream_t st)
{
    if (ncomp == 0) return;
    hipLaunchKernelGGL(k_comp_max, dim3((unsigned)((ncomp + 3) / 4)), dim3(256), 0, st, ncomp, comp_ptr,
                       delta, out);
}

// CSC invariants: colptr monotone from 0, rows in range and strictly
// ascending, values finite and > 0.  flag[0] becomes nonzero on a violation.
__global__ __launch_bounds__(256) void k_validate(DevCSC A, int32_t *__restrict__ flag)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE;
    if (j > A.ncols) return;
    if (j == A.ncols) {
        if (lane() == 0 && (A.colptr[0] != 0 || A.colptr[A.ncols] != A.nnz)) atomicOr(flag, 1);
        return;
    }
    const int64_t s = A.colptr[j], e = A.colptr[j + 1];
    bool bad = (e < s) || s < 0 || e > A.nnz;
    if (!bad) {
        for (int64_t p = s + lane(); p < e; p += WAVE) {
            const int r = A.rowidx[p];
            const double v = A.val[p];
            if (r < 0 || r >= A.nrows || !(v > 0.0) || !isfinite(v)) bad = true;
            if (p > s && A.rowidx[p - 1] >= r) bad = true;
        }
    }
    if (__ballot(bad) != 0 && lane() == 0) atomicOr(flag, 1);
}

void launch_validate(const DevCSC &A, int32_t *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((A.ncols + 1 + 3) / 4)), dim3(256), 0, st, A, flag);
}

// Totals for the stats block: acc[0] = nnz product, acc[1] = #select,
// acc[2] = #recover, acc[3] = flops; dmax[0] = max change.
__global__ __launch_bounds__(256) void k_reduce_stats(int64_t ncols, const int64_t *__restrict__ nnz_prod,
                                                      const int8_t *__restrict__ mode,
                                                      const double *__restrict__ delta,
                                                      const int64_t *__restrict__ flops,
                                                      unsigned long long *__restrict__ acc,
                                                      double *__restrict__ dmax)
{
    int64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    double dm = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ncols;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (nnz_prod) s0 += nnz_prod[j];
        if (mode) { s1 += mode[j] == 2; s2 += mode[j] == 1; }
        if (delta) dm = fmax(dm, delta[j]);
        if (flops) s3 += flops[j];
    }
    s0 = wave_sum_i64(s0);
    s1 = wave_sum_i64(s1);
    s2 = wave_sum_i64(s2);
    s3 = wave_sum_i64(s3);
    dm = wave_max(dm);
    if (lane() == 0) {
        atomicAdd(&acc[0], (unsigned long long)s0);
        atomicAdd(&acc[1], (unsigned long long)s1);
        atomicAdd(&acc[2], (unsigned long long)s2);
        atomicAdd(&acc[3], (unsigned long long)s3);
        // values are >= 0, so their bit patterns order like the values
        atomicMax((unsigned long long *)dmax, (unsigned long long)__double_as_longlong(dm));
    }
}

void launch_reduce_stats(int64_t ncols, const int64_t *nnz_prod, const int8_t *mode,
                         const double *delta, const int64_t *flops, int64_t *acc, double *dmax,
                         hipStream_t st)
{
    if (ncols == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((ncols + 255) / 256, 1024);
    hipLaunchKernelGGL(k_reduce_stats, dim3(grid), dim3(256), 0, st, ncols, nnz_prod, mode, delta, flops,
                       (unsigned long long *)acc, dmax);
}

}  // namespace mcl
