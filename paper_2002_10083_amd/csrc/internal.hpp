// Host-side interface between the C-ABI layer (api.hip) and the kernel
// launchers (spgemm.hip, prune.hip, merge.hip, mlp.hip, components.hip).
// Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcl {

struct DevCSC {
    int64_t nrows, ncols, nnz;
    const int64_t *colptr;
    const int32_t *rowidx;
    const double *val;
};

struct PruneArgs {
    double theta;   // prune threshold
    int S;          // select count (0 = off)
    int R;          // recover count (0 = off)
    double pct;     // recovery mass fraction
    double r;       // inflation power
};

enum NumericMode { MODE_COUNT = 0, MODE_EXPAND = 1, MODE_ITERATE = 2 };

// Per-column outputs of the numeric kernels.  Unused pointers may be null.
struct NumericArgs {
    DevCSC A, B;
    const int32_t *cols;      // column ids handled by this launch
    int32_t ncols;            // number of entries in cols
    const int32_t *lo, *hi;   // row span bound of every product column
    const int64_t *out_base;  // temp offset of every column (EXPAND / ITERATE)
    const int64_t *capv;      // per-column key capacity (temp slot size); may be null
    int32_t *out_row;
    double *out_val;
    int64_t *out_cnt;         // nnz written per column, -1 = table overflow
    int64_t *nnz_prod;        // exact unpruned nnz per column (ITERATE)
    double *delta;            // per-column max change (ITERATE)
    int8_t *mode;             // per-column prune branch 0/1/2 (ITERATE)
    PruneArgs pa;
    const void *dummy;        // >= 16 bytes of readable device memory (masked-off loads)
    const int32_t *goff;      // sliced layout of A: SLICE_GROUPS + 1 boundaries per column (or null)
    const uint32_t *poff;     // sliced layout of A: record index of every fourth group boundary,
                              //   SLICE_GROUPS / 4 per column, then the record count (or null)
    const uint32_t *srec;     // sliced copy of A (column ranges of A.colptr) as packed 12-byte
                              //   records {row, value low word, value high word}
    uint32_t src_end;         // sliced copy: index of the record past the last (row -1, value 0)
    const uint8_t *hbm_only;  // columns sized by an exact count: HBM-table kernel only (or null)
    int32_t *part_cnt;        // split sliced kernels: keys appended per column (all zero between launches)
    int64_t *exact_cnt;       // split sliced kernels: exact key count of an overflowed column, -1 = unknown
    const uint8_t *dense;     // columns computed by the dense-accumulator kernel (or null)
};

// ---- spgemm.hip
constexpr int SLICE_GROUPS = 64;                     // row groups of the sliced source layout
// bin_policy bits: accumulate LDS bins 0-6 in one persistent launch; with
// it, queue the lightest bins first instead of the heaviest
constexpr uint32_t POLICY_PERSIST = 1u << 28;
constexpr uint32_t POLICY_LIGHT_FIRST = 1u << 29;
// Work schedule of the persistent accumulation: entry e covers the columns
// of bin `bin[e]` (at `off[e]` in the bin lists), 2^parts[e] items per
// column.  Column c of an entry belongs to queue c % PERSIST_QUEUES; in
// queue x, items [qfirst[x][e], qfirst[x][e + 1]) belong to entry e (fewer
// than 2^30 items in all).
constexpr int PERSIST_QUEUES = 8;
struct PersistSched {
    int32_t n;
    int32_t bin[7], parts[7], off[7];
    int32_t qfirst[PERSIST_QUEUES][8];
};
// the sliced kernels index the sliced copy of A (and its sentinel) with 32-bit entry indices
constexpr int64_t SLICE_MAX_NNZ = (int64_t{1} << 32) - 2;
constexpr int NUM_LDS_BINS = 7;                      // tables of 128 .. 8192 slots
int lds_bin_slots(int bin);                          // slots of bin
int lds_bin_cap(int bin);                            // max distinct keys of bin
bool lds_variant_sliced(int bin, int variant);       // launch reads the sliced layout of A
bool lds_variant_split(int bin, int variant);        // split sliced tables (needs NumericArgs.part_cnt)
// phase [c0, c1) of a phased product: bins (-1 outside), phase-relative temp offsets, bin counts
// largest columns: multi-pass LDS accumulation + sort/epilogue in HBM scratch
size_t mpass_slab_bytes();
// whether the LDS bins' columns fit one persistent accumulation launch
bool persist_fits(const int32_t counts[8]);
// the persistent accumulation of bins 0-6 (dense launches first, finishing
// launches after; mid, nullable, is recorded after the accumulation);
// `next` points to PERSIST_QUEUES device counters (zeroed here)
void launch_numeric_persist(NumericMode mode, const NumericArgs &a, const int32_t *lists, const int32_t counts[8],
                            const int64_t *dense_bin, uint32_t *next, bool light_first, hipStream_t st,
                            hipEvent_t mid);
void launch_numeric_mpass(NumericMode mode, const NumericArgs &a, void *slab, size_t slab_bytes, int nslabs,
                          hipStream_t st);
void launch_phase_plan(int64_t n, const int32_t *bin, const int64_t *base, int64_t c0, int64_t c1,
                       int32_t *ph_bin, int64_t *ph_base, int32_t *counts, hipStream_t st);
// sliced copy of A: rows and values, each column ordered by row group, as separate arrays and
// as packed 12-byte records (same order), + group boundaries
void launch_slice_layout(const DevCSC &A, int32_t *rowo, double *valo, uint32_t *reco, int32_t *goff,
                         uint32_t *poff, hipStream_t st);
// Cohen keys per row are stored with this stride (r rounded up to 4)
inline int cohen_stride(int r) { return (r + 3) & ~3; }
// Column records of A for the symbolic pass: RP key minima (RP = padded key
// count, 0 without Cohen keys), then {first row, last row, length, 0} as
// ints; the stride in floats keeps every record inside one 128-byte line.
__host__ __device__ constexpr int col_rec_stride_c(int rp) { return rp == 0 ? 4 : rp == 4 ? 8 : rp <= 12 ? 16 : 32; }
inline int col_rec_stride(int r) { return col_rec_stride_c(r > 0 ? cohen_stride(r) : 0); }
// r = 0: records without key minima (launch_col_records), no Cohen estimate
void launch_symbolic(const DevCSC &A, const DevCSC &B, int64_t *flops, int32_t *lo, int32_t *hi,
                     const float *rec, int r, float *est, float *feat, const int64_t *prev_nnz,
                     int iteration, hipStream_t st);
void launch_cohen_keys(int64_t nrows, int r, uint64_t seed, int iteration, float *keys, hipStream_t st);
void launch_cohen_colmin(const DevCSC &A, const float *keys, int r, float *rec, hipStream_t st);
void launch_col_records(const DevCSC &A, float *rec, hipStream_t st);
// Chooses the bin of every column (bins 0..6 LDS, 7 = HBM table) and its capacity.
void launch_plan(int64_t ncols, const int64_t *flops, const int32_t *lo, const int32_t *hi,
                 const float *est, int est_kind, double est_scale, int64_t nrows,
                 const uint8_t *col_active, int32_t *bin, int64_t *capv, int32_t *bin_count,
                 int64_t *max_global, hipStream_t st);
struct BinOffsets { int32_t off[8]; };
void launch_scatter_bins(int64_t ncols, const int32_t *bin, const BinOffsets &bin_off, int32_t *cursor,
                         int32_t *lists, hipStream_t st);
void launch_scatter_bins_list(const int32_t *list, int32_t n, const int32_t *bin, const BinOffsets &off,
                              int32_t *cursor, int32_t *out, hipStream_t st);
void launch_bound_estimate(int64_t n, const int64_t *flops, const int32_t *lo, const int32_t *hi,
                           int64_t nrows, float *est, hipStream_t st);
void launch_replan(const int32_t *list, int32_t n, const int64_t *exact, int32_t *bin, int64_t *capv,
                   uint8_t *hbm_only, int32_t *bin_count, int64_t *max_global, hipStream_t st);
void launch_list_bound(const int32_t *list, int32_t n, const int64_t *flops, const int32_t *lo,
                       const int32_t *hi, int64_t nrows, int64_t *ub, int64_t *max_ub, hipStream_t st);
void launch_list_base(const int32_t *list, int32_t n, const int64_t *capv, int64_t *base, int64_t *total,
                      int region, hipStream_t st);
// round 1 and 2: columns with a known exact count (exact_cnt, nullable) are
// re-binned by it; round 1 moves the others one bin up; later rounds send
// the rest to the exact path
void launch_bump(const int32_t *list, int32_t n, int32_t *bin, int64_t *capv, int32_t *bin_count,
                 int32_t *exact_list, int32_t *n_exact, bool to_multipass, int round,
                 const int64_t *exact_cnt, hipStream_t st);
// acc: per bin {flops, nnz(B_*j), output entries, unpruned product entries (prod, or out_cnt if null)}
void launch_bin_sums(const int32_t *lists, const BinOffsets &off, const BinOffsets &cnt,
                     const int64_t *flops, const int64_t *bcolptr, const int64_t *out_cnt,
                     const int64_t *prod, int64_t *acc, hipStream_t st);
constexpr int MAX_REGIONS = 8;
struct TempRegions {
    const int32_t *row[MAX_REGIONS];
    const double *val[MAX_REGIONS];
};
// mid (nullable): recorded between the accumulation and finishing kernels of a split launch
// dense-accumulator columns: marked after planning, launched with bins 3..7
// count: 8 counters (zeroed by the caller), dense columns per planned bin
void launch_mark_dense(int64_t ncols, const int32_t *bin, const int64_t *flops, const int32_t *lo,
                       const int32_t *hi, uint8_t *dense, int64_t *count, hipStream_t st);
void launch_numeric_lds(int bin, int variant, NumericMode mode, const NumericArgs &a, hipStream_t st,
                        hipEvent_t mid = nullptr);
int lds_bin_variants(int bin);
void launch_numeric_global(NumericMode mode, const NumericArgs &a, int S, int cap, void *slab,
                           size_t slab_bytes, int nslabs, hipStream_t st);
size_t global_slab_bytes(int S, int cap);
void launch_collect_overflow(int64_t ncols, const int32_t *cols, int32_t n, const int64_t *cnt,
                             int32_t *ovf_list, int32_t *ovf_count, hipStream_t st);
void launch_exscan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *block_tmp, hipStream_t st);
int64_t exscan_tmp_elems(int64_t n);
void launch_compact(int64_t ncols, const int32_t *bin, const int64_t *base, const int64_t *cnt,
                    const int64_t *colptr, const TempRegions &tr, int32_t *row, double *val,
                    hipStream_t st);
void launch_copy_inactive(const DevCSC &A, const int32_t *col_comp, const uint8_t *active,
                          const int64_t *colptr, int32_t *row, double *val, hipStream_t st);
void launch_counts_inactive(const DevCSC &A, const int32_t *col_comp, const uint8_t *active,
                            int64_t *cnt, double *delta, hipStream_t st);
void launch_col_comp(int64_t ncols, const int64_t *comp_ptr, int64_t ncomp, int32_t *col_comp,
                     const uint8_t *active, uint8_t *col_active, hipStream_t st);
void launch_comp_max(int64_t ncomp, const int64_t *comp_ptr, const double *delta, double *out,
                     hipStream_t st);
void launch_validate(const DevCSC &A, int32_t *flag, hipStream_t st);
void launch_reduce_stats(int64_t ncols, const int64_t *nnz_prod, const int8_t *mode,
                         const double *delta, const int64_t *flops, int64_t *acc, double *dmax,
                         hipStream_t st);

// ---- prune.hip
void launch_prune_plan(const DevCSC &B, const PruneArgs &pa, double *thr, int64_t *kept,
                       int8_t *mode, hipStream_t st);
void launch_prune_fill(const DevCSC &B, const double *thr, const int64_t *colptr, int32_t *row,
                       double *val, hipStream_t st);
void launch_inflate(int64_t ncols, const int64_t *colptr, double *val, double r, double *err,
                    hipStream_t st);
void launch_normalize(int64_t ncols, const int64_t *colptr, double *val, hipStream_t st);


// ---- merge.hip: sorted multiway merge of same-shape partial products
constexpr int MT_MAX_PARTS = 256;                      // lists one merge call accepts
int merge_max_parts();
int64_t merge_tile_elems(int nparts);                  // target elements per tile
void launch_merge_ntiles(const DevCSC *parts, int nparts, int64_t ncols, int64_t *ntile, hipStream_t st);
void launch_merge_bounds(const DevCSC *parts, int nparts, int64_t nrows, int64_t ncols, const int64_t *tile_ptr,
                         int32_t *tile_col, int32_t *tile_row, hipStream_t st);
// owner-flag workspace of the count pass, read by the fill pass (uint32 words)
int64_t merge_owner_words(int64_t ntiles);
void launch_merge_tiles(bool fill, const DevCSC *parts, int nparts, int64_t nrows, int64_t ntiles,
                        const int64_t *tile_ptr, const int32_t *tile_col, const int32_t *tile_row,
                        int64_t *tile_cnt, const int64_t *tile_off, int32_t *out_row, double *out_val,
                        uint32_t *obits, int32_t *err, hipStream_t st);
void launch_merge_colptr(int64_t ncols, const int64_t *tile_ptr, const int64_t *tile_off, int64_t *colptr,
                         hipStream_t st);

// ---- components.hip
// weakly connected components of the pattern of a square A; label = smallest vertex id.
// parent: int32[nrows] scratch; nroots: one int64, cleared by the first kernel.
void launch_components(const DevCSC &A, int32_t *parent, int32_t *label, int64_t *nroots, hipStream_t st);

// ---- mlp.hip
constexpr int MLP_IN = 12, MLP_H = 64;
size_t mlp_packed_bytes();
size_t mlp_state_floats();
void launch_mlp_forward(const void *packed, const float *feat, int64_t rows, float *out,
                        hipStream_t st);
void launch_mlp_init(float *state, uint64_t seed, hipStream_t st);
void launch_expm1_inplace(float *v, int64_t n, hipStream_t st);
void launch_mlp_train_step(float *state, void *packed, const float *feat, const float *target,
                           int64_t rows, float lr, float *loss_dev, float *grad_out,
                           float *grad_tmp, hipStream_t st);
size_t mlp_train_tmp_floats(int64_t rows);

}  // namespace mcl
