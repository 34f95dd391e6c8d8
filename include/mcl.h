/*
 * mcl.h -- C ABI of the MI355X (gfx950) Markov-clustering expansion library.
 *
 * One MCL iteration (arXiv 2002.10083, Alg. 1): expansion B = A*A of a
 * column-stochastic matrix, pruning of B (threshold, then top-k selection or
 * recovery per column), inflation (Hadamard power, then column
 * re-normalisation), and the change between successive iterates.  Also the
 * merge of the partial products one process forms across its Sparse SUMMA
 * stages (Section 2 "Overview of Sparse SUMMA", Section 4 and Alg. 2), the
 * probabilistic output-size estimator (Section 5) and a learned replacement
 * for it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Matrices are CSC (`mcl_csc`): colptr int64[ncols+1], rowidx int32[nnz]
 * (strictly ascending within a column, 0 <= row < nrows), val double[nnz]
 * (finite, > 0).  nrows and ncols must be < 2^31.  Unless stated otherwise
 * every pointer inside an `mcl_csc`, and every array argument, is a DEVICE
 * pointer; `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  All work is enqueued on `stream`; calls return after the last
 * host-visible result is known (they synchronise the stream for the small
 * device-to-host copies that size their outputs).
 *
 * Memory: the library never calls hipMalloc for matrix data or workspace.
 * Every byte comes from `mcl_allocator` (stream-ordered: memory returned by
 * alloc may be used by work enqueued on `stream`; free may be called while
 * that work is still pending on the same stream).  A NULL allocator selects
 * hipMallocAsync/hipFreeAsync on `stream`.  Output matrices are filled with
 * arrays from `alloc`; the caller owns them and releases them with the same
 * allocator.  Inputs are borrowed and never written, except by
 * mcl_normalize and mcl_inflate, which work in place.
 *
 * Errors: 0 = MCL_OK, negative codes below; mcl_last_error() returns a
 * thread-local message.  On error, every allocation made by the call has
 * been released, output descriptors are zeroed and the stream is
 * synchronised.  No C++ exception crosses the ABI.
 *
 * Determinism: for the same input and parameters every entry point produces
 * bit-identical output, whatever the estimator, table sizes or batching.
 * Entries of a product column are accumulated in ascending order of the
 * inner index k as acc = acc + a_ik*b_kj, the product rounded to double
 * before the addition (no fused multiply-add).
 */
#ifndef MCL_H
#define MCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCL_OK 0
#define MCL_EINVAL (-1)   /* bad shape, pointer, parameter or malformed CSC */
#define MCL_ENOMEM (-2)   /* the allocator returned NULL */
#define MCL_EHIP (-3)     /* HIP runtime error (text in mcl_last_error) */

/* bin_policy flags: one persistent accumulation launch for LDS bins 0-6,
 * and its queue order (lightest bins first instead of heaviest) */
#define MCL_POLICY_PERSIST (1 << 28)
#define MCL_POLICY_LIGHT_FIRST (1 << 29)

/* Output-size estimator used to size the per-column hash tables. */
#define MCL_EST_BOUND 0   /* exact-safe bound min(flops_j, row span_j) */
#define MCL_EST_COHEN 1   /* Cohen's exponential-key estimate (Section 5) */
#define MCL_EST_MLP 2     /* learned estimate (mcl_mlp_forward) */

typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t *colptr;  /* int64[ncols+1] */
    int32_t *rowidx;  /* int32[nnz], ascending per column */
    double *val;      /* double[nnz] */
} mcl_csc;

typedef struct {
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
    void *ctx;
} mcl_allocator;

typedef struct {
    double prune_threshold;  /* theta: keep b >= theta (Alg. 1 prune) */
    int32_t select_num;      /* S: keep the S largest when more than S pass theta; 0 = off */
    int32_t recover_num;     /* R: keep the R largest when fewer than R pass theta and they
                                carry less than recover_pct of the column mass; 0 = off */
    double recover_pct;      /* mass fraction of the recovery test (0.9) */
    double inflation;        /* r of the Hadamard power (2.0) */
    int32_t estimator;       /* MCL_EST_* */
    int32_t cohen_keys;      /* keys per vertex for MCL_EST_COHEN (3..16) */
    uint64_t seed;           /* Cohen key seed */
    int32_t iteration;       /* MCL iteration index (fresh Cohen keys per iteration) */
    double est_scale;        /* multiplies every estimate (test knob; 1.0) */
    const void *mlp_weights; /* device pointer to the packed BF16 MLP (MCL_EST_MLP) */
    int32_t validate;        /* nonzero: check the CSC invariants of every input */
    int32_t bin_policy;      /* launch shape per table bin, 4 bits per bin (0 = default); bit 28
                                (MCL_POLICY_PERSIST): accumulate the columns of all LDS bins
                                (0-6) in one persistent launch whose waves take (column, part)
                                work items from per-XCD queues, heaviest bins first (bit 29,
                                MCL_POLICY_LIGHT_FIRST: lightest first), then finish each bin
                                (sort, epilogue) -- same results */
    float *est_out;          /* optional device float[ncols]: the estimate used per column */
    int64_t *nnz_out;        /* optional device int64[ncols]: exact nnz of each product column */
    int64_t phase_bytes;     /* mcl_iterate: bound on the product's temporary storage; when the
                                planned temp exceeds it the columns are processed in phases of
                                contiguous column ranges (same results).  0 = 40 % of the free
                                device memory at call time; < 0 = never split */
} mcl_params;

typedef struct {
    int64_t flops;            /* sum_j sum_{k in B_*j} nnz(A_*k) (multiply-adds) */
    int64_t nnz_product;      /* nnz of the unpruned product */
    int64_t nnz_kept;         /* nnz after pruning (mcl_iterate / mcl_prune) */
    int64_t n_overflow;       /* columns whose estimated table overflowed */
    int64_t n_selected;       /* columns reduced by top-k selection */
    int64_t n_recovered;      /* columns that took the recovery branch */
    int64_t n_global;         /* columns computed with an HBM-resident table */
    double t_symbolic_ms, t_estimate_ms, t_numeric_ms, t_fallback_ms, t_compact_ms, t_merge_ms,
        t_total_ms;
    double max_change;        /* max |a_new - a_old| (mcl_iterate) */
    int64_t peak_workspace_bytes;
    /* per table bin (0..6: LDS tables of 128 << b slots, 7: HBM table), first pass:
       columns, time of the bin's kernel (HIP events on `stream`), flops,
       nnz of the referenced B columns and entries written */
    int64_t bin_cols[8];
    double bin_ms[8];
    int64_t bin_flops[8];
    int64_t bin_bnnz[8];
    int64_t bin_out[8];
    int64_t n_phases;         /* column phases used by mcl_iterate (see mcl_params.phase_bytes) */
    /* bins whose columns are split over several workgroups (an accumulation
       kernel, then a kernel that sorts each column and runs the epilogue):
       time of the accumulation kernel alone (0 for other bins), and the
       unpruned product entries of every bin's columns.  With the persistent
       accumulation (bin_policy bit 28, MCL_POLICY_PERSIST) bins 0-6 share
       one accumulation launch: bin_ms[0] then holds the time of all of
       bins 0-6, bin_part_ms[0] that of the shared accumulation launch. */
    double bin_part_ms[8];
    int64_t bin_prod[8];
    int64_t n_dense;          /* columns accumulated in a dense array over their row span */
} mcl_stats;

/* Fills `p` with the defaults: theta 1e-4, S 1100, R 1400, pct 0.9, r 2,
 * MCL_EST_COHEN with 5 keys, seed 0, est_scale 1. */
void mcl_default_params(mcl_params *p);

/* Alg. 1, first step: scale every column of A (in place) to sum 1 (columns
 * summing to zero are left as zeros).  The column sum uses the fixed
 * reduction tree described at mcl_inflate. */
int mcl_normalize(mcl_csc *A, void *stream);

/* Expansion (Alg. 1): C = A*B, unpruned, A.ncols == B.nrows (A may be
 * rectangular).  C's arrays come from `alloc`.  Per column j the work is
 * flops_j = sum_{k in B_*j} nnz(A_*k) (Section 2 "Notations"). */
int mcl_expand(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, const mcl_params *params,
               const mcl_allocator *alloc, void *stream, mcl_stats *stats);

/* Prune step of Alg. 1 on an explicit matrix B, into a new matrix C:
 * with P_j = {i : b_ij >= theta}, a column is recovered (threshold = R-th
 * largest value, or 0 when the column is shorter than R) when R > 0,
 * |P_j| < R and sum(P_j) < recover_pct * sum(B_*j); otherwise it is reduced to
 * its S largest when S > 0 and |P_j| > S; otherwise thresholded at theta.
 * All entries >= the column threshold are kept (ties included). */
int mcl_prune(const mcl_csc *B, mcl_csc *C, const mcl_params *params,
              const mcl_allocator *alloc, void *stream, mcl_stats *stats);

/* Inflation (Alg. 1), in place: c -> c^r, then each column divided by its
 * sum.  Sums use a fixed tree: 64-entry blocks of consecutive positions are
 * summed by a xor-butterfly, block sums are accumulated by lane (block l,
 * l+64, ... in order) and the 64 lane sums combined by the same butterfly.
 * If colsum_err_max is not NULL it receives max_j |sum_i a_ij - 1| (host). */
int mcl_inflate(mcl_csc *C, double r, void *stream, double *colsum_err_max);

/* One fused MCL iteration -- the body of the loop of Alg. 1 (Section 2
 * "Overview of the MCL algorithm"): expansion, prune, inflation and the
 * change that the loop condition tests.  A_next = inflate(prune(A*A)),
 * bit-identical to mcl_inflate(mcl_prune(mcl_expand(A, A))).  A must be
 * square.  A_next's arrays come from `alloc` (the caller owns them).
 * max_change receives (host)
 * max_{i,j} |a_next_ij - a_ij| over the union of both patterns -- one value,
 * or one per component when comp_ptr is given.  Errors: MCL_EINVAL for a
 * non-square A, bad parameters or (with validate) a malformed A; MCL_ENOMEM
 * when the allocator fails; MCL_EHIP for a runtime error.  A column whose
 * estimated table overflows is recomputed (one bin larger, then sized by an
 * exact symbolic count), so the result never depends on the estimate.
 * Batched form: comp_ptr (device int64[ncomp+1]) splits the vertices into
 * ncomp contiguous ranges whose blocks are closed under A (block-diagonal A);
 * `active` (device uint8[ncomp]) selects the components to iterate: columns
 * of inactive components are copied unchanged.  With comp_ptr == NULL the
 * whole matrix is one component and `active` is ignored. */
int mcl_iterate(const mcl_csc *A, mcl_csc *A_next, const int64_t *comp_ptr, int64_t ncomp,
                const uint8_t *active, const mcl_params *params, const mcl_allocator *alloc,
                void *stream, mcl_stats *stats, double *max_change);

/* Clusters of Alg. 1 (its last step; Section 2 "Overview of the MCL
 * algorithm"): the connected components of the pattern of a square A,
 * treated as undirected (vertices i and j are joined when a_ij or a_ji is
 * stored; weak connectivity of the directed pattern).  labels (device
 * int32[ncols], caller-owned) receives for every vertex the smallest vertex
 * id of its component, so labels are unique for a given pattern whatever the
 * schedule.  ncomp (host, nullable) receives the number of components.
 * Values of A are not read.  Errors: MCL_EINVAL for a non-square A or NULL
 * labels with ncols > 0; MCL_ENOMEM / MCL_EHIP as elsewhere. */
int mcl_components(const mcl_csc *A, int32_t *labels, int64_t *ncomp, const mcl_allocator *alloc,
                   void *stream);

/* mcl_components for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same matrix, labels and errors as mcl_components, with no allocator: the
 * union-find parent array and the root counter live in a fixed scratch array
 * inside the library (a 256-byte header plus MCL_NOALLOC_MAX_VERTICES int32,
 * 16 MiB), one copy per GPU, held until the process ends.  The call
 * allocates nothing on the device.  A square A with more than
 * MCL_NOALLOC_MAX_VERTICES columns is rejected with MCL_EINVAL.  `stream`
 * must belong to the current device.  ncomp (host, nullable): when NULL the
 * call neither copies back nor synchronises, so it returns as soon as its
 * kernels are enqueued.  Every call on one GPU uses that GPU's one scratch
 * array, which keeps the last call's contents (each call re-initialises what
 * it reads): calls that overlap on one GPU (other host threads, other
 * streams) race and their labels are undefined. */
#define MCL_NOALLOC_MAX_VERTICES (1 << 22)
int mcl_components_noalloc(const mcl_csc *A, int32_t *labels, int64_t *ncomp, void *stream);

/* Sparse SUMMA merge (Section 2 "Overview of Sparse SUMMA", Section 4, the
 * merge step of Alg. 2): C = sum of nparts same-shape matrices (`parts` is a
 * HOST array of descriptors whose arrays are device pointers; 1 <= nparts <=
 * 256, else MCL_EINVAL).  A sorted multiway merge: each input column is read
 * as an ascending run of rows, equal rows are summed in array order,
 * (((p0 + p1) + p2) + ...), over the parts that hold the row.  Columns are
 * cut into tiles of at most 2,048 merged elements; workspace is O(ncols) plus
 * 280 bytes per tile (its bounds and the counting pass's owner flags), and
 * the output is sized by that counting pass, so the peak memory is the
 * inputs plus C plus the workspace.  stats: nnz_product = nnz_kept = nnz(C),
 * t_merge_ms, bin_cols[7] = the number of merge tiles. */
int mcl_merge_partials(const mcl_csc *parts, int32_t nparts, mcl_csc *C,
                       const mcl_allocator *alloc, void *stream, mcl_stats *stats);

/* Symbolic pass of C = A*B: flops_j = sum_{k in B_*j} nnz(A_*k) (Section 2
 * "Notations"; device int64[ncols of B]) and, when nnz_per_col is not NULL,
 * the exact nnz of every product column -- the exact symbolic SpGEMM that
 * Section 5 replaces by an estimate (insert-only hash count; device
 * int64[ncols of B]).  Both outputs are caller-owned device arrays; values of
 * A and B are not read.  Errors: MCL_EINVAL for mismatched shapes or NULL
 * flops_per_col, MCL_ENOMEM / MCL_EHIP as elsewhere. */
int mcl_symbolic(const mcl_csc *A, const mcl_csc *B, int64_t *flops_per_col,
                 int64_t *nnz_per_col, const mcl_allocator *alloc, void *stream);

/* Per-column output-size estimate (device float[B.ncols]) with the estimator
 * chosen in params (Cohen: Section 5; MLP: learned; BOUND: the exact-safe
 * bound).  Also fills the 12 MLP input features per column when `features`
 * (device float[B.ncols * 12]) is not NULL. */
int mcl_estimate(const mcl_csc *A, const mcl_csc *B, const mcl_params *params, float *est,
                 float *features, const mcl_allocator *alloc, void *stream);

/* Learned estimator: a 12 -> 64 -> 64 -> 1 ReLU MLP with BF16 weights and
 * FP32 accumulation predicting log(1 + nnz).  `weights` is the packed BF16
 * blob (mcl_mlp_packed_bytes()), `feat` device float[rows*12], `out` device
 * float[rows] = the predicted log(1 + nnz). */
size_t mcl_mlp_packed_bytes(void);
int mcl_mlp_forward(const void *weights, const float *feat, int64_t rows, float *out, void *stream);

/* One Adam step of the MLP on a batch (device arrays).  `state` is a device
 * float buffer of mcl_mlp_state_floats() floats: FP32 master weights, Adam
 * moments and the step counter; `packed` (device) receives the BF16 weights.
 * loss (host, nullable) receives the batch mean squared error of
 * log(1 + nnz); grad_out (device, nullable) receives the FP32 gradient of the
 * master weights. */
size_t mcl_mlp_state_floats(void);
int mcl_mlp_init(float *state, uint64_t seed, void *stream);
int mcl_mlp_train_step(float *state, void *packed, const float *feat, const float *target,
                       int64_t rows, float lr, float *loss, float *grad_out, void *stream);

/* Multithreaded CPU hash SpGEMM, the paper's host expansion (Section 6
 * "Faster SpGEMM on CPU"): C = A*B, unpruned, with HOST matrices.  Every
 * worker thread keeps one hash table for its lifetime (grown to the largest
 * column it has met); a column is accumulated in it, sorted by row and
 * appended to the worker's buffer, and the buffers are copied into place
 * once every column is counted (instead of a separate symbolic pass).
 * Products are accumulated in the
 * library's order (ascending k, product rounded before the addition), so C
 * is bit-identical to mcl_expand's.  nthreads <= 0 uses OMP_NUM_THREADS
 * threads when that variable holds a positive count, else every hardware
 * thread.  A, B: host arrays, read only; every call checks their structure
 * (colptr[0] == 0, non-decreasing colptr, colptr[ncols] == nnz, rows in
 * range) -- MCL_EINVAL otherwise, or for A.ncols != B.nrows.  C receives
 * malloc'd host arrays that the caller releases with mcl_host_free.  stats
 * (nullable): flops, nnz_product = nnz_kept = nnz(C), t_numeric_ms =
 * t_total_ms (the whole product); the other fields are zero.  MCL_ENOMEM when host
 * memory runs out (nothing is leaked, C is zeroed). */
int mcl_expand_host(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, int32_t nthreads, mcl_stats *stats);

/* Releases the host arrays of a matrix returned by mcl_expand_host or
 * mcl_expand_dispatch and zeroes its pointers and nnz. */
void mcl_host_free(mcl_csc *C);

/* Where a product of HOST matrices runs, chosen by its flops (Section 3
 * "Pipelined Sparse SUMMA": a multiplication with too few operations to
 * occupy the GPU stays on the CPU): flops(A*B) < gpu_min_flops runs
 * mcl_expand_host on nthreads threads; otherwise A and B are copied to the
 * device (arrays from `alloc` on `stream`), multiplied by mcl_expand with
 * `params`, and C is copied back.  gpu_min_flops <= 0 selects
 * MCL_DISPATCH_GPU_MIN_FLOPS, the crossover measured on one MI355X with its
 * host (GPU time including both copies vs 16 host threads: 3.1e6 flops on
 * planted graphs).  Either way C
 * holds malloc'd host arrays (release with mcl_host_free) and is
 * bit-identical.  where (nullable) receives 0 (CPU) or 1 (GPU); stats as in
 * mcl_expand_host or mcl_expand, with t_total_ms covering the whole call
 * (copies included).  Errors as in mcl_expand_host and mcl_expand. */
#define MCL_DISPATCH_GPU_MIN_FLOPS 3000000
int mcl_expand_dispatch(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, int64_t gpu_min_flops,
                        int32_t nthreads, const mcl_params *params, const mcl_allocator *alloc,
                        void *stream, mcl_stats *stats, int32_t *where);

/* Thread-local text of the last error. */
const char *mcl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCL_H */
