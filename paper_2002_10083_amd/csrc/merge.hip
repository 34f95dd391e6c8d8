// Sorted multiway merge of the partial products one process forms across its
// Sparse SUMMA stages (arXiv 2002.10083, Section 2 "Overview of Sparse
// SUMMA", Section 4 and Alg. 2): C = sum of P same-shape matrices whose
// columns hold strictly ascending rows.  Equal rows are summed in list order,
// ((v_p0 + v_p1) + v_p2) + ..., over the lists that hold the row.
//
// The merged sequence of a column is cut into tiles of at most MT_CAP
// elements at row boundaries (tile k starts at the smallest row r whose
// count of smaller elements over all lists reaches k * tile), so every tile
// is an independent merge of P short sorted runs that fits in LDS.  Inside a
// tile an element is the *owner* of its row when no earlier list holds the
// row; owners are exactly the output entries.  With the exclusive prefix
// count of owners over the concatenated runs, an owner's output position is
// the sum over lists q of the owners of q below the owner's row, which one
// lower_bound per list gives -- no sort and no hash table.  A count pass
// sizes the output, a fill pass writes it; both read each input once.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace mcl {

constexpr int MT_NT = 256;    // threads per tile
constexpr int MT_CAP = 2048;  // elements per tile (LDS)
constexpr int MT_WORDS = MT_CAP / 32;  // owner-flag words per tile

int merge_max_parts() { return MT_MAX_PARTS; }
int64_t merge_tile_elems(int nparts) { return (int64_t)MT_CAP - nparts; }

// first position in the ascending a[0, n) whose value is >= r
__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int n, int32_t r)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < r) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Tiles per column: ceil(merged length / tile), at least one.
__global__ __launch_bounds__(256) void k_merge_ntiles(const DevCSC *__restrict__ parts, int P, int64_t ncols,
                                                      int64_t tile, int64_t *__restrict__ ntile)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ncols;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = 0;
        for (int q = 0; q < P; ++q) m += parts[q].colptr[j + 1] - parts[q].colptr[j];
        ntile[j] = std::max<int64_t>(1, (m + tile - 1) / tile);
    }
}

// One wave per column: the column of every tile and the first row of every
// tile.  Boundary k is the smallest row value with at least k * tile
// elements below it over all lists.  With P <= 32 lists the wave probes G =
// 64 / PP row values at once (PP = P rounded up to a power of two; lane
// g * PP + q counts the elements of list q below probe g, a butterfly over
// the group's PP lanes sums them), so each round cuts the range into G + 1
// parts instead of 2; with more lists the lanes take the lists and probe
// one value per round.
__global__ __launch_bounds__(256) void k_merge_bounds(const DevCSC *__restrict__ parts, int P, int64_t nrows,
                                                      int64_t ncols, int64_t tile,
                                                      const int64_t *__restrict__ tile_ptr,
                                                      int32_t *__restrict__ tile_col,
                                                      int32_t *__restrict__ tile_row)
{
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; j < ncols; j += nw) {
        const int64_t t0 = tile_ptr[j];
        const int T = (int)(tile_ptr[j + 1] - t0);
        for (int k = lane(); k < T; k += WAVE) {
            tile_col[t0 + k] = (int32_t)j;
            if (k == 0) tile_row[t0] = 0;
        }
        const int PP = P <= 1 ? 1 : 1 << (32 - __clz(P - 1));
        if (T > 1 && PP <= WAVE / 2) {
            const int G = WAVE / PP, g = lane() / PP, q = lane() % PP;
            int64_t c0 = 0, n = 0;
            if (q < P) {
                c0 = parts[q].colptr[j];
                n = parts[q].colptr[j + 1] - c0;
            }
            for (int k = 1; k < T; ++k) {
                const int64_t target = (int64_t)k * tile;
                int64_t lo = 0, hi = nrows;
                while (lo < hi) {
                    const int64_t span = hi - lo;
                    const int64_t mid = lo + span * (g + 1) / (G + 1);  // ascending in g, inside [lo, hi)
                    int64_t c = (q < P) ? lower_bound_i32(parts[q].rowidx + c0, (int)n, (int32_t)mid) : 0;
                    for (int d = 1; d < PP; d <<= 1) c += __shfl_xor(c, d, WAVE);
                    const uint64_t ok = ballot(q == 0 && c >= target);
                    if (ok) {
                        const int gs = (__ffsll((long long)ok) - 1) / PP;  // first probe reaching the target
                        hi = lo + span * (gs + 1) / (G + 1);
                        if (gs > 0) lo = lo + span * gs / (G + 1) + 1;
                    } else {
                        lo = lo + span * G / (G + 1) + 1;
                    }
                }
                if (lane() == 0) tile_row[t0 + k] = (int32_t)lo;
            }
            continue;
        }
        for (int k = 1; k < T; ++k) {
            const int64_t target = (int64_t)k * tile;
            int64_t lo = 0, hi = nrows;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                int64_t c = 0;
                for (int q = lane(); q < P; q += WAVE) {
                    const int64_t c0 = parts[q].colptr[j], c1 = parts[q].colptr[j + 1];
                    c += lower_bound_i32(parts[q].rowidx + c0, (int)(c1 - c0), (int32_t)mid);
                }
                c = wave_sum_i64(c);
                if (c >= target) hi = mid;
                else lo = mid + 1;
            }
            if (lane() == 0) tile_row[t0 + k] = (int32_t)lo;
        }
    }
}

// One workgroup per tile.  COUNT: tile_cnt[t] = owners of the tile, and
// the owner flag of every element as a bit in obits[t * MT_WORDS ...].
// FILL: the owners' rows and summed values at tile_off[t] + their rank
// (the flags are read back, not recomputed).
template <bool FILL>
__global__ __launch_bounds__(MT_NT) void k_merge_tile(const DevCSC *__restrict__ parts, int P, int64_t nrows,
                                                      const int64_t *__restrict__ tile_ptr,
                                                      const int32_t *__restrict__ tile_col,
                                                      const int32_t *__restrict__ tile_row,
                                                      int64_t *__restrict__ tile_cnt,
                                                      const int64_t *__restrict__ tile_off,
                                                      int32_t *__restrict__ out_row, double *__restrict__ out_val,
                                                      uint32_t *__restrict__ obits, int32_t *__restrict__ err)
{
    __shared__ int32_t rows[MT_CAP];
    __shared__ int32_t pre[MT_CAP + 1];
    __shared__ int32_t segoff[MT_MAX_PARTS + 1];
    __shared__ int64_t segg[MT_MAX_PARTS];
    __shared__ int32_t wsum[MT_NT / WAVE];
    const int tid = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t j = tile_col[t];
    const bool first = t == tile_ptr[j];
    const bool last = t + 1 == tile_ptr[j + 1];
    const int32_t r0 = tile_row[t];
    const int32_t r1 = last ? (int32_t)nrows : tile_row[t + 1];
    // this tile's run of every list: rows in [r0, r1)
    for (int q = tid; q < P; q += MT_NT) {
        const int64_t c0 = parts[q].colptr[j], c1 = parts[q].colptr[j + 1];
        const int32_t *rq = parts[q].rowidx + c0;
        const int s = first ? 0 : lower_bound_i32(rq, (int)(c1 - c0), r0);
        const int e = last ? (int)(c1 - c0) : lower_bound_i32(rq, (int)(c1 - c0), r1);
        segoff[q] = e - s;
        segg[q] = c0 + s;
    }
    __syncthreads();
    const int m = block_exscan<MT_NT>(segoff, P, wsum);  // segoff[q] = start of run q
    if (m > MT_CAP) {
        // only rows that are not strictly ascending within a column can make
        // a tile longer than its bound: report malformed input
        if (tid == 0) {
            atomicOr(err, 1);
            if (!FILL) tile_cnt[t] = 0;
        }
        return;
    }
    if (tid == 0) segoff[P] = m;
    for (int q = 0; q < P; ++q) {
        const int o = segoff[q], nq = (q + 1 < P ? segoff[q + 1] : m) - o;
        const int32_t *src = parts[q].rowidx + segg[q];
        for (int i = tid; i < nq; i += MT_NT) rows[o + i] = src[i];
    }
    __syncthreads();
    uint32_t *tbits = obits + t * MT_WORDS;
    if constexpr (FILL) {
        for (int idx = tid; idx < m; idx += MT_NT) pre[idx] = (int32_t)((tbits[idx >> 5] >> (idx & 31)) & 1u);
    } else {
        // owners: no earlier list holds the row (consecutive lanes take
        // consecutive elements, so the row reads are free of bank conflicts)
        for (int i0 = 0; i0 < m; i0 += MT_NT) {
            const int idx = i0 + tid;
            bool owner = false;
            if (idx < m) {
                const int p = lower_bound_i32(segoff + 1, P, idx + 1);  // run holding idx
                const int32_t r = rows[idx];
                owner = true;
                for (int q = 0; q < p && owner; ++q) {
                    const int o = segoff[q], nq = segoff[q + 1] - o;
                    const int lb = lower_bound_i32(rows + o, nq, r);
                    owner = !(lb < nq && rows[o + lb] == r);
                }
                pre[idx] = owner ? 1 : 0;
            }
            // the wave's 64 consecutive elements: two words of flags
            const uint64_t mk = ballot(owner);
            const int w0 = (i0 + (tid & ~(WAVE - 1))) >> 5;
            if (lane() == 0 && w0 * 32 < m) {
                tbits[w0] = (uint32_t)mk;
                tbits[w0 + 1] = (uint32_t)(mk >> 32);
            }
        }
    }
    __syncthreads();
    const int owners = block_exscan<MT_NT>(pre, m, wsum);
    if (!FILL) {
        if (tid == 0) tile_cnt[t] = owners;
        return;
    }
    if (tid == 0) pre[m] = owners;
    __syncthreads();
    const int64_t base = tile_off[t];
    // an owner's rank: the owners of every run below its row; its value: the
    // values of the later runs that hold the row, added in run order
    for (int idx = tid; idx < m; idx += MT_NT) {
        if (pre[idx + 1] == pre[idx]) continue;  // not an owner
        const int p = lower_bound_i32(segoff + 1, P, idx + 1);
        const int i = idx - segoff[p];
        const int32_t r = rows[idx];
        int out = 0;
        double v = parts[p].val[segg[p] + i];
        for (int q = 0; q < P; ++q) {
            const int o = segoff[q], nq = segoff[q + 1] - o;
            const int lb = (q == p) ? i : lower_bound_i32(rows + o, nq, r);
            out += pre[o + lb] - pre[o];  // owners of list q below row r
            if (q > p && lb < nq && rows[o + lb] == r) v = v + parts[q].val[segg[q] + lb];
        }
        out_row[base + out] = r;
        out_val[base + out] = v;
    }
}

__global__ __launch_bounds__(256) void k_merge_colptr(int64_t ncols, const int64_t *__restrict__ tile_ptr,
                                                      const int64_t *__restrict__ tile_off,
                                                      int64_t *__restrict__ colptr)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= ncols;
         j += (int64_t)gridDim.x * blockDim.x)
        colptr[j] = tile_off[tile_ptr[j]];
}

void launch_merge_ntiles(const DevCSC *parts, int nparts, int64_t ncols, int64_t *ntile, hipStream_t st)
{
    if (ncols <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((ncols + 255) / 256, 8192);
    hipLaunchKernelGGL(k_merge_ntiles, dim3(g), dim3(256), 0, st, parts, nparts, ncols,
                       merge_tile_elems(nparts), ntile);
}

void launch_merge_bounds(const DevCSC *parts, int nparts, int64_t nrows, int64_t ncols, const int64_t *tile_ptr,
                         int32_t *tile_col, int32_t *tile_row, hipStream_t st)
{
    if (ncols <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((ncols + 3) / 4, 65536);
    hipLaunchKernelGGL(k_merge_bounds, dim3(g), dim3(256), 0, st, parts, nparts, nrows, ncols,
                       merge_tile_elems(nparts), tile_ptr, tile_col, tile_row);
}

int64_t merge_owner_words(int64_t ntiles) { return ntiles * MT_WORDS; }

void launch_merge_tiles(bool fill, const DevCSC *parts, int nparts, int64_t nrows, int64_t ntiles,
                        const int64_t *tile_ptr, const int32_t *tile_col, const int32_t *tile_row,
                        int64_t *tile_cnt, const int64_t *tile_off, int32_t *out_row, double *out_val,
                        uint32_t *obits, int32_t *err, hipStream_t st)
{
    if (ntiles <= 0) return;
    if (fill)
        hipLaunchKernelGGL(k_merge_tile<true>, dim3((unsigned)ntiles), dim3(MT_NT), 0, st, parts, nparts, nrows,
                           tile_ptr, tile_col, tile_row, tile_cnt, tile_off, out_row, out_val, obits, err);
    else
        hipLaunchKernelGGL(k_merge_tile<false>, dim3((unsigned)ntiles), dim3(MT_NT), 0, st, parts, nparts,
                           nrows, tile_ptr, tile_col, tile_row, tile_cnt, tile_off, out_row, out_val, obits, err);
}

void launch_merge_colptr(int64_t ncols, const int64_t *tile_ptr, const int64_t *tile_off, int64_t *colptr,
                         hipStream_t st)
{
    const unsigned g = (unsigned)std::min<int64_t>((ncols + 1 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_merge_colptr, dim3(g), dim3(256), 0, st, ncols, tile_ptr, tile_off, colptr);
}

}  // namespace mcl
