// C-ABI entry points (include/mcl.h): argument checks, workspace management
// through the caller's stream-ordered allocator, and the orchestration of the
// symbolic / estimate / plan / numeric / fallback / compaction kernels.
#include "mcl.h"
#include "host_spgemm.hpp"
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

#define HIPC(x)                                                                          \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            fail(MCL_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Workspace and output memory of one call.  Workspace is released at the end
// of the call (stream-ordered); outputs are released only on error.
struct Mem {
    const mcl_allocator *al;
    hipStream_t st;
    std::vector<void *> work, outs;
    std::vector<size_t> wsz;
    size_t cur = 0, peak = 0;

    void *raw(size_t bytes)
    {
        if (bytes == 0) bytes = 8;
        void *p = nullptr;
        if (al && al->alloc) {
            p = al->alloc(al->ctx, bytes, (void *)st);
            if (!p) fail(MCL_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMallocAsync(&p, bytes, st);
            if (e != hipSuccess || !p)
                fail(MCL_ENOMEM, "hipMallocAsync failed for " + std::to_string(bytes) + " bytes");
        }
        return p;
    }
    template <typename T>
    T *ws(int64_t n)
    {
        size_t b = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
        void *p = raw(b);
        work.push_back(p);
        wsz.push_back(b);
        cur += b;
        peak = std::max(peak, cur);
        return (T *)p;
    }
    // workspace taken after mark() can be released early with free_since()
    size_t mark() const { return work.size(); }
    void free_since(size_t m, const std::vector<void *> &keep)
    {
        std::vector<void *> kw;
        std::vector<size_t> ks;
        for (size_t i = m; i < work.size(); ++i) {
            if (std::find(keep.begin(), keep.end(), work[i]) != keep.end()) {
                kw.push_back(work[i]);
                ks.push_back(wsz[i]);
            } else {
                release(work[i]);
                cur -= wsz[i];
            }
        }
        work.resize(m);
        wsz.resize(m);
        work.insert(work.end(), kw.begin(), kw.end());
        wsz.insert(wsz.end(), ks.begin(), ks.end());
    }
    template <typename T>
    T *out(int64_t n)
    {
        size_t b = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
        void *p = raw(b);
        outs.push_back(p);
        cur += b;
        peak = std::max(peak, cur);
        return (T *)p;
    }
    void release(void *p)
    {
        if (!p) return;
        if (al && al->free) al->free(al->ctx, p, (void *)st);
        else (void)hipFreeAsync(p, st);
    }
    void free_work()
    {
        for (void *p : work) release(p);
        work.clear();
        wsz.clear();
    }
    void free_outs()
    {
        for (void *p : outs) release(p);
        outs.clear();
    }
};

struct Timer {
    hipStream_t st;
    std::vector<hipEvent_t> ev;
    void mark()
    {
        hipEvent_t e;
        if (hipEventCreate(&e) == hipSuccess) {
            (void)hipEventRecord(e, st);
            ev.push_back(e);
        }
    }
    double ms(size_t a, size_t b)
    {
        if (b >= ev.size() || a >= ev.size()) return 0.0;
        float t = 0.f;
        (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
    ~Timer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

mcl::DevCSC dev(const mcl_csc &m)
{
    return mcl::DevCSC{m.nrows, m.ncols, m.nnz, m.colptr, m.rowidx, m.val};
}

void check_csc(const mcl_csc *m, const char *name)
{
    if (!m) fail(MCL_EINVAL, std::string(name) + " is NULL");
    if (m->nrows < 0 || m->ncols < 0 || m->nnz < 0)
        fail(MCL_EINVAL, std::string(name) + ": negative dimension");
    if (m->nrows >= (int64_t)INT32_MAX || m->ncols >= (int64_t)INT32_MAX)
        fail(MCL_EINVAL, std::string(name) + ": dimensions must be < 2^31");
    if (!m->colptr) fail(MCL_EINVAL, std::string(name) + ": colptr is NULL");
    if (m->nnz > 0 && (!m->rowidx || !m->val))
        fail(MCL_EINVAL, std::string(name) + ": rowidx/val NULL with nnz > 0");
}

void validate_dev(Mem &mem, const mcl_csc *m, const char *name)
{
    int32_t *flag = mem.ws<int32_t>(1);
    HIPC(hipMemsetAsync(flag, 0, sizeof(int32_t), mem.st));
    mcl::launch_validate(dev(*m), flag, mem.st);
    int32_t h = 0;
    HIPC(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipStreamSynchronize(mem.st));
    if (h) fail(MCL_EINVAL, std::string(name) + ": malformed CSC (unsorted/out-of-range rows, "
                                                 "non-positive or non-finite values, or bad colptr)");
}

mcl::PruneArgs prune_args(const mcl_params &p)
{
    mcl::PruneArgs a;
    a.theta = p.prune_threshold;
    a.S = p.select_num;
    a.R = p.recover_num;
    a.pct = p.recover_pct;
    a.r = p.inflation;
    return a;
}

void check_params(const mcl_params &p)
{
    if (!(p.prune_threshold >= 0.0) || !std::isfinite(p.prune_threshold))
        fail(MCL_EINVAL, "prune_threshold must be finite and >= 0");
    if (p.select_num < 0 || p.recover_num < 0) fail(MCL_EINVAL, "select/recover counts must be >= 0");
    if (!(p.recover_pct >= 0.0 && p.recover_pct <= 1.0)) fail(MCL_EINVAL, "recover_pct must be in [0,1]");
    if (!(p.inflation > 0.0) || !std::isfinite(p.inflation)) fail(MCL_EINVAL, "inflation must be > 0");
    if (p.estimator < MCL_EST_BOUND || p.estimator > MCL_EST_MLP) fail(MCL_EINVAL, "unknown estimator");
    if (p.estimator == MCL_EST_COHEN && (p.cohen_keys < 2 || p.cohen_keys > 16))
        fail(MCL_EINVAL, "cohen_keys must be in [2,16]");
    if (p.estimator == MCL_EST_MLP && !p.mlp_weights) fail(MCL_EINVAL, "MLP estimator needs mlp_weights");
    if (!(p.est_scale > 0.0)) fail(MCL_EINVAL, "est_scale must be > 0");
}

int64_t next_pow2(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <typename F>
int guarded(F &&f)
{
    try {
        f();
        return MCL_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host out of memory";
        return MCL_ENOMEM;
    } catch (...) {
        g_err = "unknown internal error";
        return MCL_EHIP;
    }
}

// ---------------------------------------------------------------------------
// The product engine shared by expand, iterate, symbolic and merge.
// ---------------------------------------------------------------------------
struct ProductPlan {
    // per column (size n)
    int64_t *flops = nullptr;
    int32_t *lo = nullptr, *hi = nullptr;
    float *est = nullptr;
    int32_t *bin = nullptr;
    int64_t *capv = nullptr;
    int64_t *base = nullptr;  // n+1
    int64_t *cnt = nullptr;
    uint8_t *hbm_only = nullptr;  // columns sized by an exact count (HBM-table kernel)
    int32_t *lists = nullptr;
    int32_t counts[8] = {0};
    int64_t max_global = 0;
    int64_t temp_total = 0;
};

struct EngineOut {
    mcl::TempRegions tr{};
    int nregions = 0;
    int64_t n_overflow = 0, n_global = 0;
    double t_numeric = 0, t_fallback = 0;
    double bin_ms[8] = {0};
    double bin_part_ms[8] = {0};  // split bins: accumulation kernel alone
    int64_t bin_cols[8] = {0};
    int64_t bin_acc[32] = {0};  // per bin: flops, nnz(B_*j), output entries, unpruned entries
    int64_t n_dense = 0;        // columns computed by the dense-accumulator kernels
    int n_phases = 0;
};

mcl::BinOffsets offsets_of(const int32_t counts[8])
{
    mcl::BinOffsets off{};
    int32_t run = 0;
    for (int b = 0; b < 8; ++b) { off.off[b] = run; run += counts[b]; }
    return off;
}

// Launch every non-empty bin; per-bin times are accumulated into eo.bin_ms
// when `timed` (events around each launch, on the stream).
// dense_bin (nullable): dense-accumulator columns per bin; a bin without any
// skips the dense launches (null: every bin runs them when a.dense is set).
void run_bins(Mem &mem, mcl::NumericMode mode, mcl::NumericArgs a, const int32_t counts[8],
              const int32_t *lists, int64_t max_global, EngineOut &eo, bool timed, uint32_t policy = 0,
              const int64_t *dense_bin = nullptr)
{
    const uint8_t *dense_all = a.dense;
    int32_t off = 0;
    std::vector<hipEvent_t> ev;
    std::vector<int> evbin;
    std::vector<hipEvent_t> evmid;  // per timed bin: between the kernels of a split launch (or null)
    // persistent accumulation of the LDS bins (policy flag): one launch for
    // bins 0-6, timed as bin 0 (accumulation in bin_part_ms[0])
    const bool persist = (policy & mcl::POLICY_PERSIST) && mode != mcl::MODE_COUNT && a.goff && a.part_cnt &&
                         mcl::persist_fits(counts);
    if (persist) {
        int32_t nlds = 0;
        for (int b = 0; b < mcl::NUM_LDS_BINS; ++b) nlds += counts[b];
        if (nlds > 0) {
            hipEvent_t e0 = nullptr, e1 = nullptr, em = nullptr;
            if (timed) {
                HIPC(hipEventCreate(&e0));
                HIPC(hipEventCreate(&e1));
                HIPC(hipEventCreate(&em));
                HIPC(hipEventRecord(e0, mem.st));
            }
            uint32_t *next = mem.ws<uint32_t>(mcl::PERSIST_QUEUES);
            mcl::launch_numeric_persist(mode, a, lists, counts, dense_bin, next,
                                        (policy & mcl::POLICY_LIGHT_FIRST) != 0, mem.st, em);
            HIPC(hipGetLastError());
            if (timed) {
                HIPC(hipEventRecord(e1, mem.st));
                ev.push_back(e0);
                ev.push_back(e1);
                evbin.push_back(0);
                evmid.push_back(em);
            }
            for (int b = 0; b < mcl::NUM_LDS_BINS; ++b) eo.bin_cols[b] += counts[b];
        }
        off = nlds;
    }
    for (int b = persist ? mcl::NUM_LDS_BINS : 0; b < 8; ++b) {
        const int32_t c = counts[b];
        if (c > 0) {
            a.cols = lists + off;
            a.ncols = c;
            a.dense = (dense_bin && dense_bin[b] == 0) ? nullptr : dense_all;
            hipEvent_t e0 = nullptr, e1 = nullptr, em = nullptr;
            int variant = 0;
            if (b < mcl::NUM_LDS_BINS) {
                variant = (int)((policy >> (4 * b)) & 15u);
                if (variant >= mcl::lds_bin_variants(b)) variant = 0;
            }
            if (timed) {
                HIPC(hipEventCreate(&e0));
                HIPC(hipEventCreate(&e1));
                if (b < mcl::NUM_LDS_BINS && mcl::lds_variant_split(b, variant) && a.part_cnt &&
                    mode != mcl::MODE_COUNT)
                    HIPC(hipEventCreate(&em));
                HIPC(hipEventRecord(e0, mem.st));
            }
            if (b < mcl::NUM_LDS_BINS) {
                mcl::launch_numeric_lds(b, variant, mode, a, mem.st, em);
            } else {
                // multi-pass LDS kernel for the columns within its capacity,
                // HBM-resident tables for the rest
                if (mode != mcl::MODE_COUNT && a.goff) {
                    const size_t mslab = mcl::mpass_slab_bytes();
                    const int mslabs = std::min<int>(c, 512);
                    char *ms = mem.ws<char>((int64_t)(mslab * mslabs));
                    mcl::launch_numeric_mpass(mode, a, ms, mslab, mslabs, mem.st);
                }
                const int64_t S = next_pow2((max_global * 4) / 3 + 2);
                if (S > (int64_t)1 << 30) fail(MCL_EINVAL, "product column too large for the HBM table");
                const int cap = (int)std::min<int64_t>((S * 3) / 4, max_global);
                const size_t slab = mcl::global_slab_bytes((int)S, (int)std::max<int64_t>(cap, 1));
                const size_t budget = (size_t)4 << 30;
                int nslabs = (int)std::max<size_t>(1, std::min<size_t>(budget / slab, 1024));
                nslabs = std::min(nslabs, c);
                char *sl = mem.ws<char>((int64_t)(slab * nslabs));
                mcl::launch_numeric_global(mode, a, (int)S, cap, sl, slab, nslabs, mem.st);
                eo.n_global += c;
            }
            HIPC(hipGetLastError());
            if (timed) {
                HIPC(hipEventRecord(e1, mem.st));
                ev.push_back(e0);
                ev.push_back(e1);
                evbin.push_back(b);
                evmid.push_back(em);
            }
            eo.bin_cols[b] += c;
        }
        off += c;
    }
    if (timed && !ev.empty()) {
        HIPC(hipEventSynchronize(ev.back()));
        for (size_t i = 0; i < evbin.size(); ++i) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
            eo.bin_ms[evbin[i]] += t;
            if (evmid[i]) {
                float tp = 0.f;
                (void)hipEventElapsedTime(&tp, ev[2 * i], evmid[i]);
                eo.bin_part_ms[evbin[i]] += tp;
            }
        }
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : evmid)
        if (e) (void)hipEventDestroy(e);
}

// Column ranges of a phased product: consecutive columns whose planned temp
// (12 bytes per slot) fits `phase_bytes` (0 = 40 % of the free device
// memory, < 0 = one phase).  Returns the cut points c_0 = 0 < ... < c_P = n
// and, in cut_base, the temp offsets at the cuts.
std::vector<int64_t> phase_cuts(Mem &mem, const ProductPlan &pl, int64_t n, int64_t phase_bytes,
                                std::vector<int64_t> &cut_base)
{
    cut_base = {0, pl.temp_total};
    if (phase_bytes < 0 || n <= 1) return {0, n};
    int64_t budget = phase_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIPC(hipMemGetInfo(&fr, &tot));
        budget = (int64_t)(0.4 * (double)fr);
    }
    const int64_t slots = std::max<int64_t>(budget / 12, 1);
    if (pl.temp_total <= slots) return {0, n};
    std::vector<int64_t> hb(n + 1);
    HIPC(hipMemcpyAsync(hb.data(), pl.base, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipStreamSynchronize(mem.st));
    std::vector<int64_t> cuts{0};
    cut_base = {0};
    int64_t c0 = 0;
    while (c0 < n) {
        // largest c1 with hb[c1] - hb[c0] <= slots, at least one column
        int64_t c1 = (int64_t)(std::upper_bound(hb.begin() + c0, hb.end(), hb[c0] + slots) - hb.begin()) - 1;
        c1 = std::min(std::max(c1, c0 + 1), n);
        cuts.push_back(c1);
        cut_base.push_back(hb[c1]);
        c0 = c1;
    }
    return cuts;
}

// Sliced copy of the source matrix, read by the sliced-table and multi-pass
// kernels (every other launch accepts it too: the entries of one step stay
// distinct).
void use_sliced_source(Mem &mem, mcl::NumericArgs &a, uint32_t policy)
{
    (void)policy;  // the multi-pass kernel of the largest columns needs it too
    if (a.A.ncols <= 0 || a.A.nnz > mcl::SLICE_MAX_NNZ) return;  // larger A: shared-table kernels
    // one entry past the last holds row -1 and value 0: masked-off lanes load it
    const int64_t nz = a.A.nnz;
    int32_t *ro = mem.ws<int32_t>(nz + 1);
    double *vo = mem.ws<double>(nz + 1);
    uint32_t *rec = mem.ws<uint32_t>(3 * (nz + 1));
    int32_t *go = mem.ws<int32_t>(a.A.ncols * (mcl::SLICE_GROUPS + 1));
    uint32_t *po = mem.ws<uint32_t>(a.A.ncols * (mcl::SLICE_GROUPS / 4) + 1);
    HIPC(hipMemsetAsync(ro + nz, 0xFF, sizeof(int32_t), mem.st));
    HIPC(hipMemsetAsync(vo + nz, 0, sizeof(double), mem.st));
    HIPC(hipMemsetAsync(rec + 3 * nz, 0xFF, sizeof(uint32_t), mem.st));
    HIPC(hipMemsetAsync(rec + 3 * nz + 1, 0, 2 * sizeof(uint32_t), mem.st));
    mcl::launch_slice_layout(a.A, ro, vo, rec, go, po, mem.st);
    // every kernel reads the sliced copy (same columns, rows grouped by hash):
    // the sliced-table kernels as packed records, the others as arrays
    a.A.rowidx = ro;
    a.A.val = vo;
    a.srec = rec;
    a.goff = go;
    a.poff = po;
    a.src_end = (uint32_t)nz;
}

// Runs the numeric phase for the columns binned in `pl`, then resolves table
// overflow.  An overflowed column whose keys the split kernels counted is
// re-binned by that exact count (smallest LDS bin that holds it, else the
// multi-pass kernel at that size); any other overflowed column moves one LDS
// bin up (the largest LDS bin to the multi-pass kernel).  Both are recomputed
// into a new temp region.  A column that still overflows after its second
// launch (third, if it was re-binned by its exact count twice) gets an exact
// count and an HBM table of exactly that size, which cannot overflow.  So
// every column is launched at most four times whatever its estimate.  `a`
// carries A/B, the prune args and the per-column outputs.
void engine(Mem &mem, int64_t n, int64_t nrows, mcl::NumericMode mode, mcl::NumericArgs a,
            ProductPlan &pl, EngineOut &eo, Timer &tm, const int64_t *bcolptr = nullptr,
            uint32_t policy = 0)
{
    int32_t *trow = mem.ws<int32_t>(pl.temp_total);
    double *tval = (mode == mcl::MODE_COUNT) ? nullptr : mem.ws<double>(pl.temp_total);
    eo.tr.row[0] = trow;
    eo.tr.val[0] = tval;
    eo.nregions = 1;
    {
        mcl::BinOffsets off = offsets_of(pl.counts);
        int32_t *cursor = mem.ws<int32_t>(8);
        HIPC(hipMemsetAsync(cursor, 0, 8 * sizeof(int32_t), mem.st));
        mcl::launch_scatter_bins(n, pl.bin, off, cursor, pl.lists, mem.st);
    }
    {
        int64_t *dummy = mem.ws<int64_t>(8);
        HIPC(hipMemsetAsync(dummy, 0xFF, 8 * sizeof(int64_t), mem.st));  // row -1 (no row)
        a.dummy = dummy;
    }
    a.part_cnt = mem.ws<int32_t>(std::max<int64_t>(n, 1));
    HIPC(hipMemsetAsync(a.part_cnt, 0, std::max<int64_t>(n, 1) * sizeof(int32_t), mem.st));
    a.exact_cnt = mem.ws<int64_t>(std::max<int64_t>(n, 1));
    HIPC(hipMemsetAsync(a.exact_cnt, 0xFF, std::max<int64_t>(n, 1) * sizeof(int64_t), mem.st));  // -1
    // dense-accumulator columns, counted per bin: bins without any skip the
    // dense launches in the first pass
    a.dense = nullptr;
    int64_t dense_bin[8] = {0};
    if (a.goff && mode != mcl::MODE_COUNT && n > 0) {
        uint8_t *dn = mem.ws<uint8_t>(n);
        int64_t *dc = mem.ws<int64_t>(8);
        HIPC(hipMemsetAsync(dc, 0, 8 * sizeof(int64_t), mem.st));
        mcl::launch_mark_dense(n, pl.bin, pl.flops, pl.lo, pl.hi, dn, dc, mem.st);
        HIPC(hipMemcpyAsync(dense_bin, dc, sizeof(dense_bin), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
        for (int b = 0; b < 8; ++b) eo.n_dense += dense_bin[b];
        if (eo.n_dense > 0) a.dense = dn;
    }
    a.lo = pl.lo;
    a.hi = pl.hi;
    a.hbm_only = pl.hbm_only;
    a.out_base = pl.base;
    a.capv = pl.capv;
    a.out_row = trow;
    a.out_val = tval;
    a.out_cnt = pl.cnt;
    tm.mark();
    const size_t t0 = tm.ev.size() - 1;
    run_bins(mem, mode, a, pl.counts, pl.lists, pl.max_global, eo, true, policy, dense_bin);
    // per-bin totals of the first pass (the launch shape the timing refers to)
    {
        int64_t *acc = mem.ws<int64_t>(32);
        HIPC(hipMemsetAsync(acc, 0, 32 * sizeof(int64_t), mem.st));
        mcl::BinOffsets cnt{};
        for (int b = 0; b < 8; ++b) cnt.off[b] = pl.counts[b];
        mcl::launch_bin_sums(pl.lists, offsets_of(pl.counts), cnt, pl.flops, bcolptr, pl.cnt, a.nnz_prod, acc,
                             mem.st);
        HIPC(hipMemcpyAsync(eo.bin_acc, acc, sizeof(eo.bin_acc), hipMemcpyDeviceToHost, mem.st));
    }
    tm.mark();
    const size_t t1 = tm.ev.size() - 1;

    const int32_t *cur_list = pl.lists;
    int32_t cur_n = 0;
    for (int b = 0; b < 8; ++b) cur_n += pl.counts[b];
    int32_t *ovf = mem.ws<int32_t>(std::max<int32_t>(cur_n, 1));
    int32_t *dev_i = mem.ws<int32_t>(16);
    int64_t *dev_l = mem.ws<int64_t>(4);
    int64_t *ub = nullptr;
    for (int round = 1;; ++round) {
        HIPC(hipMemsetAsync(dev_i, 0, 16 * sizeof(int32_t), mem.st));
        mcl::launch_collect_overflow(n, cur_list, cur_n, pl.cnt, ovf, dev_i, mem.st);
        int32_t novf = 0;
        HIPC(hipMemcpyAsync(&novf, dev_i, sizeof(int32_t), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
        if (round == 1) eo.t_numeric = tm.ms(t0, t1);
        if (novf == 0) break;
        if (round == 1) eo.n_overflow = novf;
        // at most four rounds reach this point (see above); the region table
        // holds MAX_REGIONS temp regions
        if (round >= mcl::MAX_REGIONS) fail(MCL_EHIP, "table overflow did not resolve");
        // a column whose keys the split kernels counted is re-binned by that
        // count (first and second round); otherwise the first round moves it
        // one bin up (the largest LDS bin to the multi-pass kernel) and later
        // rounds send it to the exact path
        int32_t *counts_d = dev_i + 1;       // 8 counters
        int32_t *nexact_d = dev_i + 9;
        int32_t *exact = mem.ws<int32_t>(novf);
        mcl::launch_bump(ovf, novf, pl.bin, pl.capv, counts_d, exact, nexact_d,
                         mode != mcl::MODE_COUNT && a.goff, round, a.exact_cnt, mem.st);
        int32_t hc[9];
        HIPC(hipMemcpyAsync(hc, counts_d, 9 * sizeof(int32_t), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
        int32_t counts2[8];
        for (int b = 0; b < 8; ++b) counts2[b] = hc[b];
        const int32_t nexact = hc[8];
        int64_t max_need = 0;
        if (nexact > 0) {
            // exact product size with an exact-safe HBM table, then bin 7
            if (!ub) ub = mem.ws<int64_t>(n);
            HIPC(hipMemsetAsync(dev_l, 0, 4 * sizeof(int64_t), mem.st));
            mcl::launch_list_bound(exact, nexact, pl.flops, pl.lo, pl.hi, nrows, ub, dev_l, mem.st);
            int64_t max_ub = 0;
            HIPC(hipMemcpyAsync(&max_ub, dev_l, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipStreamSynchronize(mem.st));
            mcl::NumericArgs c = a;
            c.dense = nullptr;  // the exact count covers every listed column
            c.capv = nullptr;
            c.out_row = nullptr;
            c.out_val = nullptr;
            int32_t cc[8] = {0, 0, 0, 0, 0, 0, 0, nexact};
            EngineOut dummy;
            run_bins(mem, mcl::MODE_COUNT, c, cc, exact, std::max<int64_t>(max_ub, 1), dummy, false);
            HIPC(hipMemsetAsync(dev_i + 10, 0, 6 * sizeof(int32_t), mem.st));
            HIPC(hipMemsetAsync(dev_l, 0, 4 * sizeof(int64_t), mem.st));
            int32_t *bc2 = mem.ws<int32_t>(8);
            HIPC(hipMemsetAsync(bc2, 0, 8 * sizeof(int32_t), mem.st));
            mcl::launch_replan(exact, nexact, pl.cnt, pl.bin, pl.capv, pl.hbm_only, bc2, dev_l, mem.st);
            int32_t hb2[8];
            HIPC(hipMemcpyAsync(hb2, bc2, sizeof(hb2), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipMemcpyAsync(&max_need, dev_l, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipStreamSynchronize(mem.st));
            for (int b = 0; b < 8; ++b) counts2[b] += hb2[b];
        }
        // new temp region for the recomputed columns
        const int region = eo.nregions;
        mcl::launch_list_base(ovf, novf, pl.capv, pl.base, dev_l + 1, region, mem.st);
        int64_t rtotal = 0;
        HIPC(hipMemcpyAsync(&rtotal, dev_l + 1, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
        int32_t *rrow = mem.ws<int32_t>(rtotal);
        double *rval = (mode == mcl::MODE_COUNT) ? nullptr : mem.ws<double>(rtotal);
        eo.tr.row[region] = rrow;
        eo.tr.val[region] = rval;
        eo.nregions = region + 1;
        int32_t *lists2 = mem.ws<int32_t>(novf);
        {
            int32_t *cursor = mem.ws<int32_t>(8);
            HIPC(hipMemsetAsync(cursor, 0, 8 * sizeof(int32_t), mem.st));
            mcl::launch_scatter_bins_list(ovf, novf, pl.bin, offsets_of(counts2), cursor, lists2, mem.st);
        }
        a.out_row = rrow;
        a.out_val = rval;
        run_bins(mem, mode, a, counts2, lists2, std::max<int64_t>(max_need, 1), eo, false, policy);
        // the next round inspects only the recomputed columns
        int32_t *next = mem.ws<int32_t>(novf);
        HIPC(hipMemcpyAsync(next, lists2, novf * sizeof(int32_t), hipMemcpyDeviceToDevice, mem.st));
        cur_list = next;
        cur_n = novf;
    }
    tm.mark();
    HIPC(hipStreamSynchronize(mem.st));
    eo.t_fallback = tm.ms(t1, tm.ev.size() - 1);
}

void copy_bin_stats(const EngineOut &eo, mcl_stats *s)
{
    if (!s) return;
    for (int b = 0; b < 8; ++b) {
        s->bin_cols[b] = eo.bin_cols[b];
        s->bin_ms[b] = eo.bin_ms[b];
        s->bin_flops[b] = eo.bin_acc[4 * b];
        s->bin_bnnz[b] = eo.bin_acc[4 * b + 1];
        s->bin_out[b] = eo.bin_acc[4 * b + 2];
        s->bin_prod[b] = eo.bin_acc[4 * b + 3];
        s->bin_part_ms[b] = eo.bin_part_ms[b];
    }
    s->n_dense = eo.n_dense;
}

// Symbolic pass + estimate + plan for C = A*B (or the merge of parts).
void plan_product(Mem &mem, const mcl::DevCSC &A, const mcl::DevCSC &B, const mcl_params &p,
                  const uint8_t *col_active, ProductPlan &pl, Timer &tm, double *t_sym,
                  double *t_est, float *feat_out)
{
    const int64_t n = B.ncols;
    pl.flops = mem.ws<int64_t>(n);
    pl.lo = mem.ws<int32_t>(n);
    pl.hi = mem.ws<int32_t>(n);
    pl.est = mem.ws<float>(n);
    pl.bin = mem.ws<int32_t>(n);
    pl.capv = mem.ws<int64_t>(n + 1);
    pl.base = mem.ws<int64_t>(n + 1);
    pl.cnt = mem.ws<int64_t>(n);
    pl.lists = mem.ws<int32_t>(n);
    pl.hbm_only = mem.ws<uint8_t>(n);
    HIPC(hipMemsetAsync(pl.hbm_only, 0, n, mem.st));
    tm.mark();
    const size_t e0 = tm.ev.size() - 1;
    // column records of A (key minima with Cohen keys, row range and length)
    const bool cohen = p.estimator == MCL_EST_COHEN;
    const int r = cohen ? p.cohen_keys : 0;
    float *rec = mem.ws<float>(std::max<int64_t>(A.ncols, 1) * mcl::col_rec_stride(r));
    if (cohen) {
        float *keys = mem.ws<float>(A.nrows * mcl::cohen_stride(r));
        mcl::launch_cohen_keys(A.nrows, r, p.seed, p.iteration, keys, mem.st);
        mcl::launch_cohen_colmin(A, keys, r, rec, mem.st);
    } else {
        mcl::launch_col_records(A, rec, mem.st);
    }
    tm.mark();
    const size_t ea = tm.ev.size() - 1;
    float *feat = feat_out;
    if (p.estimator == MCL_EST_MLP && !feat) feat = mem.ws<float>(n * 12);
    mcl::launch_symbolic(A, B, pl.flops, pl.lo, pl.hi, rec, r, cohen ? pl.est : nullptr, feat, nullptr,
                         p.iteration, mem.st);
    tm.mark();
    const size_t e1 = tm.ev.size() - 1;
    if (p.estimator == MCL_EST_MLP) {
        mcl::launch_mlp_forward(p.mlp_weights, feat, n, pl.est, mem.st);
        mcl::launch_expm1_inplace(pl.est, n, mem.st);
    }
    if (p.est_out && p.estimator != MCL_EST_BOUND)
        HIPC(hipMemcpyAsync(p.est_out, pl.est, n * sizeof(float), hipMemcpyDeviceToDevice, mem.st));
    tm.mark();
    const size_t e2 = tm.ev.size() - 1;
    int32_t *bc = mem.ws<int32_t>(8);
    int64_t *mg = mem.ws<int64_t>(1);
    HIPC(hipMemsetAsync(bc, 0, 8 * sizeof(int32_t), mem.st));
    HIPC(hipMemsetAsync(mg, 0, sizeof(int64_t), mem.st));
    mcl::launch_plan(n, pl.flops, pl.lo, pl.hi, pl.est, p.estimator, p.est_scale, A.nrows, col_active,
                     pl.bin, pl.capv, bc, mg, mem.st);
    int64_t *tmp = mem.ws<int64_t>(mcl::exscan_tmp_elems(n));
    mcl::launch_exscan_i64(pl.capv, pl.base, n, tmp, mem.st);
    HIPC(hipMemcpyAsync(pl.counts, bc, sizeof(pl.counts), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipMemcpyAsync(&pl.max_global, mg, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipMemcpyAsync(&pl.temp_total, pl.base + n, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipStreamSynchronize(mem.st));
    // estimate time: Cohen's keys and key minima (their finish is fused into
    // the symbolic pass) or the MLP forward; symbolic time: the pass itself
    // and, without Cohen keys, the column records it reads
    if (t_sym) *t_sym = tm.ms(ea, e1) + (cohen ? 0.0 : tm.ms(e0, ea));
    if (t_est) *t_est = (cohen ? tm.ms(e0, ea) : 0.0) + tm.ms(e1, e2);
}

// colptr = exclusive scan of cnt; returns nnz (host).
int64_t scan_counts(Mem &mem, const int64_t *cnt, int64_t n, int64_t *colptr)
{
    int64_t *tmp = mem.ws<int64_t>(mcl::exscan_tmp_elems(n));
    mcl::launch_exscan_i64(cnt, colptr, n, tmp, mem.st);
    int64_t nnz = 0;
    HIPC(hipMemcpyAsync(&nnz, colptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipStreamSynchronize(mem.st));
    return nnz;
}

void zero_out(mcl_csc *C)
{
    if (C) {
        int64_t r = C->nrows, c = C->ncols;
        std::memset(C, 0, sizeof(*C));
        C->nrows = r;
        C->ncols = c;
    }
}

template <typename F>
int with_mem(const mcl_allocator *al, void *stream, mcl_csc *out, F &&f)
{
    Mem mem{al, (hipStream_t)stream};
    int rc = guarded([&] { f(mem); });
    if (rc != MCL_OK) {
        (void)hipStreamSynchronize(mem.st);
        mem.free_outs();
        zero_out(out);
    }
    mem.free_work();
    if (rc != MCL_OK) (void)hipStreamSynchronize(mem.st);
    return rc;
}

void fill_stats_totals(Mem &mem, int64_t n, const int64_t *nnz_prod, const int8_t *mode,
                       const double *delta, const int64_t *flops, mcl_stats *s, double *dmax_out)
{
    int64_t *acc = mem.ws<int64_t>(4);
    double *dm = mem.ws<double>(1);
    HIPC(hipMemsetAsync(acc, 0, 4 * sizeof(int64_t), mem.st));
    HIPC(hipMemsetAsync(dm, 0, sizeof(double), mem.st));
    mcl::launch_reduce_stats(n, nnz_prod, mode, delta, flops, acc, dm, mem.st);
    int64_t h[4];
    double hd = 0.0;
    HIPC(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipMemcpyAsync(&hd, dm, sizeof(double), hipMemcpyDeviceToHost, mem.st));
    HIPC(hipStreamSynchronize(mem.st));
    if (s) {
        if (nnz_prod) s->nnz_product = h[0];
        s->n_selected = h[1];
        s->n_recovered = h[2];
        s->flops = h[3];
        s->max_change = hd;
    }
    if (dmax_out) *dmax_out = hd;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of mcl_components_noalloc: a 256-byte header (the root counter),
// then the union-find parent array of up to MCL_NOALLOC_MAX_VERTICES
// vertices.  Every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: host code uses only the per-device address that
// hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_HEADER_BYTES = 256;
constexpr size_t NOALLOC_SCRATCH_BYTES =
    NOALLOC_HEADER_BYTES + sizeof(int32_t) * (size_t)MCL_NOALLOC_MAX_VERTICES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current and kept for the life of the process.
unsigned char *scratch_on_current_device()
{
    int d = -1;
    HIPC(hipGetDevice(&d));
    if (d < 0 || d >= NOALLOC_MAX_DEVICES) fail(MCL_EHIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[d]) {
        void *ptr = nullptr;
        HIPC(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(MCL_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_dev[d] = ptr;
    }
    return (unsigned char *)g_scratch_dev[d];
}

}  // namespace

// ===========================================================================
// exported C ABI
// ===========================================================================
extern "C" {

const char *mcl_last_error(void) { return g_err.c_str(); }

void mcl_default_params(mcl_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->prune_threshold = 1e-4;
    p->select_num = 1100;
    p->recover_num = 1400;
    p->recover_pct = 0.9;
    p->inflation = 2.0;
    p->estimator = MCL_EST_COHEN;
    p->cohen_keys = 5;
    p->seed = 0;
    p->iteration = 0;
    p->est_scale = 1.0;
}

int mcl_normalize(mcl_csc *A, void *stream)
{
    return guarded([&] {
        check_csc(A, "A");
        mcl::launch_normalize(A->ncols, A->colptr, A->val, (hipStream_t)stream);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize((hipStream_t)stream));
    });
}

int mcl_expand(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, const mcl_params *params,
               const mcl_allocator *alloc, void *stream, mcl_stats *stats)
{
    mcl_params p;
    mcl_default_params(&p);
    if (params) p = *params;
    return with_mem(alloc, stream, C, [&](Mem &mem) {
        if (!C) fail(MCL_EINVAL, "C is NULL");
        check_csc(A, "A");
        check_csc(B, "B");
        check_params(p);
        if (A->ncols != B->nrows) fail(MCL_EINVAL, "A.ncols != B.nrows");
        if (p.validate) { validate_dev(mem, A, "A"); validate_dev(mem, B, "B"); }
        Timer tm{mem.st};
        tm.mark();
        const int64_t n = B->ncols;
        const mcl::DevCSC dA = dev(*A), dB = dev(*B);
        ProductPlan pl;
        double tsym = 0, test = 0;
        plan_product(mem, dA, dB, p, nullptr, pl, tm, &tsym, &test, nullptr);
        mcl::NumericArgs a{};
        a.A = dA;
        a.B = dB;
        a.pa = prune_args(p);
        use_sliced_source(mem, a, (uint32_t)p.bin_policy);
        EngineOut eo;
        engine(mem, n, A->nrows, mcl::MODE_EXPAND, a, pl, eo, tm, B->colptr, (uint32_t)p.bin_policy);
        if (p.nnz_out) HIPC(hipMemcpyAsync(p.nnz_out, pl.cnt, n * sizeof(int64_t), hipMemcpyDeviceToDevice, mem.st));
        tm.mark();
        const size_t c0 = tm.ev.size() - 1;
        int64_t *colptr = mem.out<int64_t>(n + 1);
        const int64_t nnz = scan_counts(mem, pl.cnt, n, colptr);
        int32_t *row = mem.out<int32_t>(nnz);
        double *val = mem.out<double>(nnz);
        mcl::launch_compact(n, nullptr, pl.base, pl.cnt, colptr, eo.tr, row, val, mem.st);
        HIPC(hipGetLastError());
        tm.mark();
        fill_stats_totals(mem, n, nullptr, nullptr, nullptr, pl.flops, stats, nullptr);
        copy_bin_stats(eo, stats);
        C->nrows = A->nrows;
        C->ncols = n;
        C->nnz = nnz;
        C->colptr = colptr;
        C->rowidx = row;
        C->val = val;
        if (stats) {
            stats->nnz_product = nnz;
            stats->nnz_kept = nnz;
            stats->n_overflow = eo.n_overflow;
            stats->n_global = eo.n_global;
            stats->t_symbolic_ms = tsym;
            stats->t_estimate_ms = test;
            stats->t_numeric_ms = eo.t_numeric;
            stats->t_fallback_ms = eo.t_fallback;
            stats->t_compact_ms = tm.ms(c0, tm.ev.size() - 1);
            stats->t_total_ms = tm.ms(0, tm.ev.size() - 1);
            stats->peak_workspace_bytes = (int64_t)mem.peak;
        }
    });
}

int mcl_iterate(const mcl_csc *A, mcl_csc *A_next, const int64_t *comp_ptr, int64_t ncomp,
                const uint8_t *active, const mcl_params *params, const mcl_allocator *alloc,
                void *stream, mcl_stats *stats, double *max_change)
{
    mcl_params p;
    mcl_default_params(&p);
    if (params) p = *params;
    return with_mem(alloc, stream, A_next, [&](Mem &mem) {
        if (!A_next) fail(MCL_EINVAL, "A_next is NULL");
        check_csc(A, "A");
        check_params(p);
        if (A->nrows != A->ncols) fail(MCL_EINVAL, "mcl_iterate needs a square matrix");
        if (comp_ptr && ncomp <= 0) fail(MCL_EINVAL, "ncomp must be > 0 with comp_ptr");
        if (comp_ptr && !active) fail(MCL_EINVAL, "active is NULL");
        if (p.validate) validate_dev(mem, A, "A");
        Timer tm{mem.st};
        tm.mark();
        const int64_t n = A->ncols;
        const mcl::DevCSC dA = dev(*A);
        int32_t *col_comp = nullptr;
        uint8_t *col_active = nullptr;
        if (comp_ptr) {
            col_comp = mem.ws<int32_t>(n);
            col_active = mem.ws<uint8_t>(n);
            mcl::launch_col_comp(n, comp_ptr, ncomp, col_comp, active, col_active, mem.st);
        }
        ProductPlan pl;
        double tsym = 0, test = 0;
        plan_product(mem, dA, dA, p, col_active, pl, tm, &tsym, &test, nullptr);
        int64_t *nnzp = mem.ws<int64_t>(n);
        double *delta = mem.ws<double>(n);
        int8_t *mode = mem.ws<int8_t>(n);
        HIPC(hipMemsetAsync(nnzp, 0, n * sizeof(int64_t), mem.st));
        HIPC(hipMemsetAsync(mode, 0, n * sizeof(int8_t), mem.st));
        mcl::NumericArgs a{};
        a.A = dA;
        a.B = dA;
        a.pa = prune_args(p);
        a.nnz_prod = nnzp;
        a.delta = delta;
        a.mode = mode;
        const uint32_t policy = (uint32_t)p.bin_policy;
        use_sliced_source(mem, a, policy);
        std::vector<int64_t> cut_base;
        const std::vector<int64_t> cuts = phase_cuts(mem, pl, n, p.phase_bytes, cut_base);
        EngineOut eo;
        int64_t *colptr = mem.out<int64_t>(n + 1);
        int32_t *row = nullptr;
        double *val = nullptr;
        int64_t nnz = 0;
        size_t c0ev = 0;
        if (cuts.size() == 2) {
            engine(mem, n, A->nrows, mcl::MODE_ITERATE, a, pl, eo, tm, A->colptr, policy);
            if (comp_ptr) mcl::launch_counts_inactive(dA, col_comp, active, pl.cnt, delta, mem.st);
            if (p.nnz_out) HIPC(hipMemcpyAsync(p.nnz_out, nnzp, n * sizeof(int64_t), hipMemcpyDeviceToDevice, mem.st));
            tm.mark();
            c0ev = tm.ev.size() - 1;
            nnz = scan_counts(mem, pl.cnt, n, colptr);
            row = mem.out<int32_t>(nnz);
            val = mem.out<double>(nnz);
            mcl::launch_compact(n, pl.bin, pl.base, pl.cnt, colptr, eo.tr, row, val, mem.st);
        } else {
            // phases: contiguous column ranges, each with its own temp; the
            // kept entries of a phase are compacted into a phase buffer and
            // the temp is released before the next phase
            HIPC(hipMemsetAsync(pl.cnt, 0, n * sizeof(int64_t), mem.st));
            int32_t *phb = mem.ws<int32_t>(n);
            int64_t *phbase = mem.ws<int64_t>(n);
            int32_t *pcnt = mem.ws<int32_t>(8);
            struct PhaseOut { int64_t c0, c1; int64_t *cp; int32_t *r; double *v; };
            std::vector<PhaseOut> outs;
            for (size_t q = 0; q + 1 < cuts.size(); ++q) {
                const int64_t c0 = cuts[q], c1 = cuts[q + 1];
                const size_t mk = mem.mark();
                HIPC(hipMemsetAsync(pcnt, 0, 8 * sizeof(int32_t), mem.st));
                mcl::launch_phase_plan(n, pl.bin, pl.base, c0, c1, phb, phbase, pcnt, mem.st);
                ProductPlan ph = pl;
                ph.bin = phb;
                ph.base = phbase;
                HIPC(hipMemcpyAsync(ph.counts, pcnt, sizeof(ph.counts), hipMemcpyDeviceToHost, mem.st));
                HIPC(hipStreamSynchronize(mem.st));
                ph.temp_total = cut_base[q + 1] - cut_base[q];
                EngineOut e;
                engine(mem, n, A->nrows, mcl::MODE_ITERATE, a, ph, e, tm, A->colptr, policy);
                int64_t *pcp = mem.ws<int64_t>(c1 - c0 + 1);
                const int64_t pn = scan_counts(mem, pl.cnt + c0, c1 - c0, pcp);
                int32_t *r = mem.ws<int32_t>(pn);
                double *v = mem.ws<double>(pn);
                mcl::launch_compact(c1 - c0, phb + c0, phbase + c0, pl.cnt + c0, pcp, e.tr, r, v, mem.st);
                HIPC(hipGetLastError());
                mem.free_since(mk, {pcp, r, v});
                outs.push_back({c0, c1, pcp, r, v});
                eo.n_overflow += e.n_overflow;
                eo.n_global += e.n_global;
                eo.n_dense += e.n_dense;
                eo.t_numeric += e.t_numeric;
                eo.t_fallback += e.t_fallback;
                for (int b = 0; b < 8; ++b) {
                    eo.bin_ms[b] += e.bin_ms[b];
                    eo.bin_part_ms[b] += e.bin_part_ms[b];
                    eo.bin_cols[b] += e.bin_cols[b];
                }
                for (int b = 0; b < 32; ++b) eo.bin_acc[b] += e.bin_acc[b];
            }
            eo.n_phases = (int)outs.size();
            if (comp_ptr) mcl::launch_counts_inactive(dA, col_comp, active, pl.cnt, delta, mem.st);
            if (p.nnz_out) HIPC(hipMemcpyAsync(p.nnz_out, nnzp, n * sizeof(int64_t), hipMemcpyDeviceToDevice, mem.st));
            tm.mark();
            c0ev = tm.ev.size() - 1;
            nnz = scan_counts(mem, pl.cnt, n, colptr);
            row = mem.out<int32_t>(nnz);
            val = mem.out<double>(nnz);
            for (const PhaseOut &o : outs) {
                mcl::TempRegions tr{};
                tr.row[0] = o.r;
                tr.val[0] = o.v;
                mcl::launch_compact(o.c1 - o.c0, pl.bin + o.c0, o.cp, pl.cnt + o.c0, colptr + o.c0, tr, row, val,
                                    mem.st);
            }
        }
        if (comp_ptr) mcl::launch_copy_inactive(dA, col_comp, active, colptr, row, val, mem.st);
        HIPC(hipGetLastError());
        tm.mark();
        double dmax = 0.0;
        fill_stats_totals(mem, n, nnzp, mode, delta, pl.flops, stats, &dmax);
        copy_bin_stats(eo, stats);
        if (max_change) {
            if (comp_ptr) {
                double *cm = mem.ws<double>(ncomp);
                mcl::launch_comp_max(ncomp, comp_ptr, delta, cm, mem.st);
                HIPC(hipMemcpyAsync(max_change, cm, ncomp * sizeof(double), hipMemcpyDeviceToHost, mem.st));
                HIPC(hipStreamSynchronize(mem.st));
            } else {
                *max_change = dmax;
            }
        }
        A_next->nrows = A->nrows;
        A_next->ncols = n;
        A_next->nnz = nnz;
        A_next->colptr = colptr;
        A_next->rowidx = row;
        A_next->val = val;
        if (stats) {
            stats->nnz_kept = nnz;
            stats->n_overflow = eo.n_overflow;
            stats->n_global = eo.n_global;
            stats->t_symbolic_ms = tsym;
            stats->t_estimate_ms = test;
            stats->t_numeric_ms = eo.t_numeric;
            stats->t_fallback_ms = eo.t_fallback;
            stats->t_compact_ms = tm.ms(c0ev, tm.ev.size() - 1);
            stats->t_total_ms = tm.ms(0, tm.ev.size() - 1);
            stats->peak_workspace_bytes = (int64_t)mem.peak;
            stats->n_phases = std::max(1, eo.n_phases);
        }
    });
}

int mcl_prune(const mcl_csc *B, mcl_csc *C, const mcl_params *params, const mcl_allocator *alloc,
              void *stream, mcl_stats *stats)
{
    mcl_params p;
    mcl_default_params(&p);
    if (params) p = *params;
    return with_mem(alloc, stream, C, [&](Mem &mem) {
        if (!C) fail(MCL_EINVAL, "C is NULL");
        check_csc(B, "B");
        check_params(p);
        if (p.validate) validate_dev(mem, B, "B");
        Timer tm{mem.st};
        tm.mark();
        const int64_t n = B->ncols;
        const mcl::DevCSC dB = dev(*B);
        double *thr = mem.ws<double>(n);
        int64_t *kept = mem.ws<int64_t>(n);
        int8_t *mode = mem.ws<int8_t>(n);
        mcl::launch_prune_plan(dB, prune_args(p), thr, kept, mode, mem.st);
        int64_t *colptr = mem.out<int64_t>(n + 1);
        const int64_t nnz = scan_counts(mem, kept, n, colptr);
        int32_t *row = mem.out<int32_t>(nnz);
        double *val = mem.out<double>(nnz);
        mcl::launch_prune_fill(dB, thr, colptr, row, val, mem.st);
        HIPC(hipGetLastError());
        tm.mark();
        fill_stats_totals(mem, n, nullptr, mode, nullptr, nullptr, stats, nullptr);
        C->nrows = B->nrows;
        C->ncols = n;
        C->nnz = nnz;
        C->colptr = colptr;
        C->rowidx = row;
        C->val = val;
        if (stats) {
            stats->nnz_product = B->nnz;
            stats->nnz_kept = nnz;
            stats->flops = 0;
            stats->t_total_ms = tm.ms(0, 1);
            stats->peak_workspace_bytes = (int64_t)mem.peak;
        }
    });
}

int mcl_inflate(mcl_csc *C, double r, void *stream, double *colsum_err_max)
{
    Mem mem{nullptr, (hipStream_t)stream};
    int rc = guarded([&] {
        check_csc(C, "C");
        if (!(r > 0.0) || !std::isfinite(r)) fail(MCL_EINVAL, "inflation must be > 0");
        double *err = nullptr;
        if (colsum_err_max) {
            err = mem.ws<double>(1);
            HIPC(hipMemsetAsync(err, 0, sizeof(double), mem.st));
        }
        mcl::launch_inflate(C->ncols, C->colptr, C->val, r, err, mem.st);
        HIPC(hipGetLastError());
        if (err) HIPC(hipMemcpyAsync(colsum_err_max, err, sizeof(double), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
    });
    mem.free_work();
    return rc;
}

int mcl_merge_partials(const mcl_csc *parts, int32_t nparts, mcl_csc *C, const mcl_allocator *alloc,
                       void *stream, mcl_stats *stats)
{
    return with_mem(alloc, stream, C, [&](Mem &mem) {
        if (!C) fail(MCL_EINVAL, "C is NULL");
        if (!parts || nparts <= 0) fail(MCL_EINVAL, "need at least one part");
        if (nparts > mcl::merge_max_parts())
            fail(MCL_EINVAL, "at most " + std::to_string(mcl::merge_max_parts()) + " parts per merge");
        for (int l = 0; l < nparts; ++l) {
            check_csc(&parts[l], "part");
            if (parts[l].nrows != parts[0].nrows || parts[l].ncols != parts[0].ncols)
                fail(MCL_EINVAL, "parts must have the same shape");
        }
        Timer tm{mem.st};
        tm.mark();
        const int64_t n = parts[0].ncols, nrows = parts[0].nrows;
        std::vector<mcl::DevCSC> h(nparts);
        for (int l = 0; l < nparts; ++l) h[l] = dev(parts[l]);
        mcl::DevCSC *dparts = mem.ws<mcl::DevCSC>(nparts);
        HIPC(hipMemcpyAsync(dparts, h.data(), nparts * sizeof(mcl::DevCSC), hipMemcpyHostToDevice, mem.st));
        if (stats) std::memset(stats, 0, sizeof(*stats));
        int64_t *colptr = mem.out<int64_t>(n + 1);
        int64_t nnz = 0, ntiles = 0;
        int32_t *row = nullptr;
        double *val = nullptr;
        if (n == 0) {
            HIPC(hipMemsetAsync(colptr, 0, sizeof(int64_t), mem.st));
        } else {
            // tiles per column, their columns and first rows
            int64_t *ntile = mem.ws<int64_t>(n);
            int64_t *tile_ptr = mem.ws<int64_t>(n + 1);
            mcl::launch_merge_ntiles(dparts, nparts, n, ntile, mem.st);
            int64_t *tmp = mem.ws<int64_t>(mcl::exscan_tmp_elems(n));
            mcl::launch_exscan_i64(ntile, tile_ptr, n, tmp, mem.st);
            HIPC(hipMemcpyAsync(&ntiles, tile_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipStreamSynchronize(mem.st));
            int32_t *tile_col = mem.ws<int32_t>(ntiles);
            int32_t *tile_row = mem.ws<int32_t>(ntiles);
            int64_t *tile_cnt = mem.ws<int64_t>(ntiles);
            int64_t *tile_off = mem.ws<int64_t>(ntiles + 1);
            int32_t *err = mem.ws<int32_t>(1);
            uint32_t *obits = mem.ws<uint32_t>(mcl::merge_owner_words(ntiles));
            HIPC(hipMemsetAsync(err, 0, sizeof(int32_t), mem.st));
            mcl::launch_merge_bounds(dparts, nparts, nrows, n, tile_ptr, tile_col, tile_row, mem.st);
            // count pass, output offsets, fill pass
            mcl::launch_merge_tiles(false, dparts, nparts, nrows, ntiles, tile_ptr, tile_col, tile_row, tile_cnt,
                                    nullptr, nullptr, nullptr, obits, err, mem.st);
            int64_t *tmp2 = mem.ws<int64_t>(mcl::exscan_tmp_elems(ntiles));
            mcl::launch_exscan_i64(tile_cnt, tile_off, ntiles, tmp2, mem.st);
            int32_t herr = 0;
            HIPC(hipMemcpyAsync(&nnz, tile_off + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, mem.st));
            HIPC(hipStreamSynchronize(mem.st));
            if (herr) fail(MCL_EINVAL, "part: rows are not strictly ascending within a column");
            row = mem.out<int32_t>(nnz);
            val = mem.out<double>(nnz);
            mcl::launch_merge_colptr(n, tile_ptr, tile_off, colptr, mem.st);
            mcl::launch_merge_tiles(true, dparts, nparts, nrows, ntiles, tile_ptr, tile_col, tile_row, nullptr,
                                    tile_off, row, val, obits, err, mem.st);
        }
        HIPC(hipGetLastError());
        tm.mark();
        HIPC(hipStreamSynchronize(mem.st));
        C->nrows = nrows;
        C->ncols = n;
        C->nnz = nnz;
        C->colptr = colptr;
        C->rowidx = row;
        C->val = val;
        if (stats) {
            stats->nnz_product = nnz;
            stats->nnz_kept = nnz;
            stats->t_merge_ms = tm.ms(0, tm.ev.size() - 1);
            stats->t_total_ms = stats->t_merge_ms;
            stats->peak_workspace_bytes = (int64_t)mem.peak;
            stats->bin_cols[7] = ntiles;  // merge tiles
        }
    });
}

int mcl_symbolic(const mcl_csc *A, const mcl_csc *B, int64_t *flops_per_col, int64_t *nnz_per_col,
                 const mcl_allocator *alloc, void *stream)
{
    return with_mem(alloc, stream, nullptr, [&](Mem &mem) {
        check_csc(A, "A");
        check_csc(B, "B");
        if (A->ncols != B->nrows) fail(MCL_EINVAL, "A.ncols != B.nrows");
        if (!flops_per_col) fail(MCL_EINVAL, "flops_per_col is NULL");
        mcl_params p;
        mcl_default_params(&p);
        p.estimator = MCL_EST_BOUND;
        Timer tm{mem.st};
        const int64_t n = B->ncols;
        const mcl::DevCSC dA = dev(*A), dB = dev(*B);
        ProductPlan pl;
        plan_product(mem, dA, dB, p, nullptr, pl, tm, nullptr, nullptr, nullptr);
        HIPC(hipMemcpyAsync(flops_per_col, pl.flops, n * sizeof(int64_t), hipMemcpyDeviceToDevice, mem.st));
        if (nnz_per_col) {
            mcl::NumericArgs a{};
            a.A = dA;
            a.B = dB;
            EngineOut eo;
            engine(mem, n, A->nrows, mcl::MODE_COUNT, a, pl, eo, tm);
            HIPC(hipMemcpyAsync(nnz_per_col, pl.cnt, n * sizeof(int64_t), hipMemcpyDeviceToDevice, mem.st));
        }
        HIPC(hipStreamSynchronize(mem.st));
    });
}

int mcl_estimate(const mcl_csc *A, const mcl_csc *B, const mcl_params *params, float *est,
                 float *features, const mcl_allocator *alloc, void *stream)
{
    mcl_params p;
    mcl_default_params(&p);
    if (params) p = *params;
    return with_mem(alloc, stream, nullptr, [&](Mem &mem) {
        check_csc(A, "A");
        check_csc(B, "B");
        check_params(p);
        if (A->ncols != B->nrows) fail(MCL_EINVAL, "A.ncols != B.nrows");
        if (!est) fail(MCL_EINVAL, "est is NULL");
        Timer tm{mem.st};
        const int64_t n = B->ncols;
        const mcl::DevCSC dA = dev(*A), dB = dev(*B);
        p.est_out = est;
        ProductPlan pl;
        plan_product(mem, dA, dB, p, nullptr, pl, tm, nullptr, nullptr, features);
        if (p.estimator == MCL_EST_BOUND) mcl::launch_bound_estimate(n, pl.flops, pl.lo, pl.hi, A->nrows, est, mem.st);
        HIPC(hipStreamSynchronize(mem.st));
    });
}

int mcl_components(const mcl_csc *A, int32_t *labels, int64_t *ncomp, const mcl_allocator *alloc,
                   void *stream)
{
    return with_mem(alloc, stream, nullptr, [&](Mem &mem) {
        check_csc(A, "A");
        if (A->nrows != A->ncols) fail(MCL_EINVAL, "mcl_components needs a square matrix");
        const int64_t n = A->ncols;
        if (n > 0 && !labels) fail(MCL_EINVAL, "labels is NULL");
        int64_t roots = 0;
        if (n > 0) {
            int32_t *parent = mem.ws<int32_t>(n);
            int64_t *cnt = mem.ws<int64_t>(1);
            mcl::launch_components(dev(*A), parent, labels, cnt, mem.st);
            HIPC(hipGetLastError());
            HIPC(hipMemcpyAsync(&roots, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, mem.st));
        }
        HIPC(hipStreamSynchronize(mem.st));
        if (ncomp) *ncomp = roots;
    });
}

int mcl_components_noalloc(const mcl_csc *A, int32_t *labels, int64_t *ncomp, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = guarded([&] {
        check_csc(A, "A");
        if (A->nrows != A->ncols) fail(MCL_EINVAL, "mcl_components_noalloc needs a square matrix");
        const int64_t n = A->ncols;
        if (n > (int64_t)MCL_NOALLOC_MAX_VERTICES)
            fail(MCL_EINVAL, "mcl_components_noalloc: " + std::to_string(n) +
                                 " vertices exceed the scratch limit of " +
                                 std::to_string((int64_t)MCL_NOALLOC_MAX_VERTICES));
        if (n > 0 && !labels) fail(MCL_EINVAL, "labels is NULL");
        if (n == 0) {
            if (ncomp) *ncomp = 0;
            return;
        }
        unsigned char *base = scratch_on_current_device();
        int64_t *cnt = (int64_t *)base;
        int32_t *parent = (int32_t *)(base + NOALLOC_HEADER_BYTES);
        mcl::launch_components(dev(*A), parent, labels, cnt, st);
        HIPC(hipGetLastError());
        if (ncomp) {
            int64_t roots = 0;
            HIPC(hipMemcpyAsync(&roots, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            *ncomp = roots;
        }
    });
    if (rc != MCL_OK) (void)hipStreamSynchronize(st);
    return rc;
}

size_t mcl_mlp_packed_bytes(void) { return mcl::mlp_packed_bytes(); }
size_t mcl_mlp_state_floats(void) { return mcl::mlp_state_floats(); }

int mcl_mlp_forward(const void *weights, const float *feat, int64_t rows, float *out, void *stream)
{
    return guarded([&] {
        if (!weights || (rows > 0 && (!feat || !out))) fail(MCL_EINVAL, "NULL argument");
        if (rows < 0) fail(MCL_EINVAL, "rows < 0");
        mcl::launch_mlp_forward(weights, feat, rows, out, (hipStream_t)stream);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize((hipStream_t)stream));
    });
}

int mcl_mlp_init(float *state, uint64_t seed, void *stream)
{
    return guarded([&] {
        if (!state) fail(MCL_EINVAL, "state is NULL");
        mcl::launch_mlp_init(state, seed, (hipStream_t)stream);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize((hipStream_t)stream));
    });
}

int mcl_mlp_train_step(float *state, void *packed, const float *feat, const float *target, int64_t rows,
                       float lr, float *loss, float *grad_out, void *stream)
{
    Mem mem{nullptr, (hipStream_t)stream};
    int rc = guarded([&] {
        if (!state || !packed || !feat || !target) fail(MCL_EINVAL, "NULL argument");
        if (rows <= 0) fail(MCL_EINVAL, "rows must be > 0");
        float *tmp = mem.ws<float>((int64_t)mcl::mlp_train_tmp_floats(rows));
        mcl::launch_mlp_train_step(state, packed, feat, target, rows, lr, tmp, grad_out, tmp + 1,
                                   mem.st);
        HIPC(hipGetLastError());
        if (loss) HIPC(hipMemcpyAsync(loss, tmp, sizeof(float), hipMemcpyDeviceToHost, mem.st));
        HIPC(hipStreamSynchronize(mem.st));
    });
    mem.free_work();
    if (rc != MCL_OK) (void)hipStreamSynchronize((hipStream_t)stream);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Host hash SpGEMM and the CPU/GPU dispatch (host matrices)
// ---------------------------------------------------------------------------
namespace {

mcl::host::CSC host_csc(const mcl_csc *m, const char *name)
{
    if (!m) fail(MCL_EINVAL, std::string(name) + " is NULL");
    if (m->nrows >= (int64_t)INT32_MAX || m->ncols >= (int64_t)INT32_MAX)
        fail(MCL_EINVAL, std::string(name) + ": dimensions must be < 2^31");
    mcl::host::CSC h{m->nrows, m->ncols, m->nnz, m->colptr, m->rowidx, m->val};
    const char *why = mcl::host::check(h);
    if (*why) fail(MCL_EINVAL, std::string(name) + ": " + why);
    return h;
}

void host_product(const mcl::host::CSC &a, const mcl::host::CSC &b, int32_t nthreads, mcl_csc *C,
                  mcl_stats *stats)
{
    mcl::host::Out o;
    mcl::host::spgemm(a, b, mcl::host::threads_for(nthreads), o);
    C->nrows = a.nrows;
    C->ncols = b.ncols;
    C->nnz = o.nnz;
    C->colptr = o.colptr;
    C->rowidx = o.rowidx;
    C->val = o.val;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->flops = o.flops;
        stats->nnz_product = o.nnz;
        stats->nnz_kept = o.nnz;
        stats->t_symbolic_ms = o.t_symbolic_ms;
        stats->t_numeric_ms = o.t_numeric_ms;
        stats->t_total_ms = o.t_symbolic_ms + o.t_numeric_ms;
    }
}

}  // namespace

extern "C" {

int mcl_expand_host(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, int32_t nthreads, mcl_stats *stats)
{
    int rc = guarded([&] {
        if (!C) fail(MCL_EINVAL, "C is NULL");
        zero_out(C);
        const mcl::host::CSC a = host_csc(A, "A"), b = host_csc(B, "B");
        if (a.ncols != b.nrows) fail(MCL_EINVAL, "A.ncols != B.nrows");
        host_product(a, b, nthreads, C, stats);
    });
    if (rc != MCL_OK && C) zero_out(C);
    return rc;
}

void mcl_host_free(mcl_csc *C)
{
    if (!C) return;
    std::free(C->colptr);
    std::free(C->rowidx);
    std::free(C->val);
    zero_out(C);
}

int mcl_expand_dispatch(const mcl_csc *A, const mcl_csc *B, mcl_csc *C, int64_t gpu_min_flops,
                        int32_t nthreads, const mcl_params *params, const mcl_allocator *alloc,
                        void *stream, mcl_stats *stats, int32_t *where)
{
    mcl_csc dC{};
    Mem mem{alloc, (hipStream_t)stream};
    int rc = guarded([&] {
        if (!C) fail(MCL_EINVAL, "C is NULL");
        zero_out(C);
        const mcl::host::CSC a = host_csc(A, "A"), b = host_csc(B, "B");
        if (a.ncols != b.nrows) fail(MCL_EINVAL, "A.ncols != B.nrows");
        const auto t0 = std::chrono::steady_clock::now();
        const int nt = mcl::host::threads_for(nthreads);
        const int64_t fl = mcl::host::flops(a, b, nt);
        const int64_t cut = gpu_min_flops > 0 ? gpu_min_flops : (int64_t)MCL_DISPATCH_GPU_MIN_FLOPS;
        if (where) *where = fl >= cut ? 1 : 0;
        if (fl < cut) {
            host_product(a, b, nthreads, C, stats);
            if (stats)
                stats->t_total_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            return;
        }
        // GPU: upload A and B, expand, download C
        mcl_csc dA{a.nrows, a.ncols, a.nnz, nullptr, nullptr, nullptr};
        mcl_csc dB{b.nrows, b.ncols, b.nnz, nullptr, nullptr, nullptr};
        for (auto pr : {std::make_pair(&dA, A), std::make_pair(&dB, B)}) {
            mcl_csc &d = *pr.first;
            d.colptr = mem.ws<int64_t>(d.ncols + 1);
            d.rowidx = mem.ws<int32_t>(d.nnz);
            d.val = mem.ws<double>(d.nnz);
            HIPC(hipMemcpyAsync(d.colptr, pr.second->colptr, sizeof(int64_t) * (d.ncols + 1),
                                hipMemcpyHostToDevice, mem.st));
            if (d.nnz > 0) {
                HIPC(hipMemcpyAsync(d.rowidx, pr.second->rowidx, sizeof(int32_t) * d.nnz,
                                    hipMemcpyHostToDevice, mem.st));
                HIPC(hipMemcpyAsync(d.val, pr.second->val, sizeof(double) * d.nnz, hipMemcpyHostToDevice,
                                    mem.st));
            }
        }
        const int e = mcl_expand(&dA, &dB, &dC, params, alloc, stream, stats);
        if (e != MCL_OK) fail(e, g_err);
        // the device C belongs to this call until it is copied out
        mem.work.push_back(dC.colptr);
        mem.work.push_back(dC.rowidx);
        mem.work.push_back(dC.val);
        mem.wsz.insert(mem.wsz.end(), 3, 0);
        const int64_t n = dC.ncols, nz = dC.nnz;
        dC = mcl_csc{};
        int64_t *hc = (int64_t *)std::malloc(sizeof(int64_t) * (size_t)(n + 1));
        int32_t *hr = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nz, 1));
        double *hv = (double *)std::malloc(sizeof(double) * (size_t)std::max<int64_t>(nz, 1));
        C->colptr = hc;
        C->rowidx = hr;
        C->val = hv;
        if (!hc || !hr || !hv) fail(MCL_ENOMEM, "host out of memory for C");
        HIPC(hipMemcpyAsync(hc, mem.work[mem.work.size() - 3], sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost,
                            mem.st));
        if (nz > 0) {
            HIPC(hipMemcpyAsync(hr, mem.work[mem.work.size() - 2], sizeof(int32_t) * nz, hipMemcpyDeviceToHost,
                                mem.st));
            HIPC(hipMemcpyAsync(hv, mem.work[mem.work.size() - 1], sizeof(double) * nz, hipMemcpyDeviceToHost,
                                mem.st));
        }
        HIPC(hipStreamSynchronize(mem.st));
        C->nrows = a.nrows;
        C->ncols = n;
        C->nnz = nz;
        if (stats)
            stats->t_total_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
    if (rc != MCL_OK) {
        (void)hipStreamSynchronize(mem.st);
        if (dC.colptr) {  // mcl_expand succeeded but the call failed before taking C
            mem.release(dC.colptr);
            mem.release(dC.rowidx);
            mem.release(dC.val);
        }
        if (C) mcl_host_free(C);
    }
    mem.free_work();
    (void)hipStreamSynchronize(mem.st);
    return rc;
}

}  // extern "C"
