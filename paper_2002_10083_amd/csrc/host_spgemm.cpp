// Multithreaded CPU hash SpGEMM (arXiv 2002.10083, Section 6 "Faster SpGEMM
// on CPU", after Nagasaka et al.): every worker thread owns one hash table
// for its whole lifetime, grown to the largest column it has met (each
// column probes only the power-of-two prefix it needs, at most half full,
// starting small and growing as its rows arrive).  A column's products are
// inserted and accumulated, then its table entries are sorted by row.
// Instead of the symbolic pass that sizes the output up front, each worker
// appends its finished columns to a buffer of its own; once every column is
// counted, the buffers are copied into place (one extra copy of the output
// instead of a second pass over all products).  Columns are dealt to the
// workers in small chunks from a shared counter (heavy columns are spread
// over the column range).
//
// Built by the host compiler with -ffp-contract=off: `acc + a * b` rounds the
// product before the addition, and the products of a column are added in
// ascending order of k, so the output is bit-identical to the GPU kernels.
#include "host_spgemm.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <new>
#include <thread>
#include <vector>

namespace mcl {
namespace host {
namespace {

constexpr int64_t CHUNK = 32;         // columns per scheduling unit
constexpr int64_t START_KEYS = 4096;  // initial key capacity of a column's table

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Runs body(worker, j) for every column j in [0, n) on `threads` workers;
// a worker takes CHUNK consecutive columns at a time.  An exception thrown
// by a worker stops the others and is rethrown here.
template <typename Body>
void parallel_columns(int64_t n, int threads, Body &&body)
{
    std::atomic<int64_t> next{0};
    std::atomic<bool> failed{false};
    std::exception_ptr err;
    std::atomic_flag err_lock = ATOMIC_FLAG_INIT;
    auto work = [&](int w) {
        try {
            for (;;) {
                if (failed.load(std::memory_order_relaxed)) return;
                const int64_t c0 = next.fetch_add(CHUNK, std::memory_order_relaxed);
                if (c0 >= n) return;
                const int64_t c1 = std::min(n, c0 + CHUNK);
                for (int64_t j = c0; j < c1; ++j) body(w, j);
            }
        } catch (...) {
            failed.store(true);
            while (err_lock.test_and_set()) {
            }
            if (!err) err = std::current_exception();
            err_lock.clear();
        }
    };
    if (threads <= 1 || n <= CHUNK) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(threads - 1);
        for (int w = 1; w < threads; ++w) pool.emplace_back(work, w);
        work(0);
        for (auto &t : pool) t.join();
    }
    if (err) std::rethrow_exception(err);
}

// One worker's hash table: keys (row, -1 = empty) and values, grown to the
// largest capacity any of its columns needed; `used` lists the occupied
// slots of the current column in insertion order (cleared per column).  A
// column uses only the power-of-two prefix of 2^lg slots it needs.
struct Table {
    std::vector<int32_t> key;
    std::vector<double> val;
    std::vector<int32_t> used;
    std::vector<uint64_t> order;

    // prepares a column expected to hold at most `keys` distinct rows
    // (load at most 1/2); returns log2 of its capacity
    int begin(int64_t keys, bool values)
    {
        const int64_t want = std::max<int64_t>(16, 2 * keys);
        int lg = 4;
        while (((int64_t)1 << lg) < want) ++lg;
        reserve(lg, values);
        used.clear();
        return lg;
    }
    void reserve(int lg, bool values)
    {
        const size_t cap = (size_t)1 << lg;
        if (key.size() < cap) key.assign(cap, -1);  // every slot is empty between columns
        if (values && val.size() < cap) val.resize(cap);
    }
    void end()
    {
        for (int32_t s : used) key[s] = -1;
    }
};

// home slot of row r in a table of 2^lg slots: top bits of a multiplicative hash
inline uint32_t home(int32_t r, int lg) { return ((uint32_t)r * 2654435761u) >> (32 - lg); }

}  // namespace

const char *check(const CSC &m)
{
    if (m.nrows < 0 || m.ncols < 0 || m.nnz < 0) return "negative dimension";
    if (!m.colptr) return "colptr is NULL";
    if (m.nnz > 0 && (!m.rowidx || !m.val)) return "rowidx/val NULL with nnz > 0";
    if (m.colptr[0] != 0) return "colptr[0] != 0";
    for (int64_t j = 0; j < m.ncols; ++j)
        if (m.colptr[j + 1] < m.colptr[j]) return "colptr is decreasing";
    if (m.colptr[m.ncols] != m.nnz) return "colptr[ncols] != nnz";
    for (int64_t p = 0; p < m.nnz; ++p)
        if (m.rowidx[p] < 0 || m.rowidx[p] >= m.nrows) return "row index out of range";
    return "";
}

int threads_for(int nthreads)
{
    if (nthreads > 0) return nthreads;
    if (const char *e = std::getenv("OMP_NUM_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0) return v;
    }
    const unsigned hc = std::thread::hardware_concurrency();
    return hc ? (int)hc : 1;
}

int64_t flops(const CSC &A, const CSC &B, int threads)
{
    std::vector<int64_t> part((size_t)std::max(threads, 1), 0);
    parallel_columns(B.ncols, threads, [&](int w, int64_t j) {
        int64_t f = 0;
        for (int64_t t = B.colptr[j]; t < B.colptr[j + 1]; ++t) {
            const int32_t k = B.rowidx[t];
            f += A.colptr[k + 1] - A.colptr[k];
        }
        part[w] += f;
    });
    int64_t s = 0;
    for (int64_t f : part) s += f;
    return s;
}

void release(Out &out)
{
    std::free(out.colptr);
    std::free(out.rowidx);
    std::free(out.val);
    out.colptr = nullptr;
    out.rowidx = nullptr;
    out.val = nullptr;
}

void spgemm(const CSC &A, const CSC &B, int threads, Out &out)
{
    const int64_t n = B.ncols;
    const int nw = std::max(threads, 1);
    out.threads = nw;
    const auto t0 = std::chrono::steady_clock::now();
    out.colptr = (int64_t *)std::malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!out.colptr) throw std::bad_alloc();
    std::vector<Table> tab((size_t)nw);
    // per worker: its columns' sorted entries back to back, and for every
    // column it took, (column, offset in its buffer)
    std::vector<std::vector<int32_t>> lrow((size_t)nw);
    std::vector<std::vector<double>> lval((size_t)nw);
    std::vector<std::vector<std::pair<int64_t, int64_t>>> lcol((size_t)nw);
    std::vector<int64_t> wflops((size_t)nw, 0);
    int64_t *cnt = out.colptr + 1;
    try {
        parallel_columns(n, nw, [&](int w, int64_t j) {
            int64_t f = 0;
            for (int64_t t = B.colptr[j]; t < B.colptr[j + 1]; ++t) {
                const int32_t k = B.rowidx[t];
                f += A.colptr[k + 1] - A.colptr[k];
            }
            wflops[w] += f;
            // the column's distinct rows are not known in advance: the table
            // starts for min(flops, nrows, START_KEYS) keys and grows 4x
            // (rehashing what it holds) whenever it passes half full
            Table &T = tab[w];
            int lg = T.begin(std::min<int64_t>(std::min(f, A.nrows), START_KEYS), true);
            uint32_t mask = ((uint32_t)1 << lg) - 1;
            size_t limit = (size_t)1 << (lg - 1);
            int32_t *key = T.key.data();
            double *val = T.val.data();
            for (int64_t t = B.colptr[j]; t < B.colptr[j + 1]; ++t) {
                const int32_t k = B.rowidx[t];
                const double b = B.val[t];
                for (int64_t p = A.colptr[k]; p < A.colptr[k + 1]; ++p) {
                    const int32_t r = A.rowidx[p];
                    const double prod = A.val[p] * b;
                    uint32_t h = home(r, lg);
                    while (key[h] != r && key[h] != -1) h = (h + 1) & mask;
                    if (key[h] != -1) {
                        val[h] = val[h] + prod;
                        continue;
                    }
                    key[h] = r;
                    val[h] = 0.0 + prod;
                    T.used.push_back((int32_t)h);
                    if (T.used.size() <= limit) continue;
                    std::vector<std::pair<int32_t, double>> held(T.used.size());
                    for (size_t q = 0; q < held.size(); ++q) held[q] = {key[T.used[q]], val[T.used[q]]};
                    T.end();
                    lg += 2;
                    T.reserve(lg, true);
                    key = T.key.data();
                    val = T.val.data();
                    mask = ((uint32_t)1 << lg) - 1;
                    limit = (size_t)1 << (lg - 1);
                    T.used.clear();
                    for (const auto &e : held) {
                        uint32_t g = home(e.first, lg);
                        while (key[g] != -1) g = (g + 1) & mask;
                        key[g] = e.first;
                        val[g] = e.second;
                        T.used.push_back((int32_t)g);
                    }
                }
            }
            // rows are non-negative: (row << 32 | slot) sorts by row
            const size_t m = T.used.size();
            T.order.resize(m);
            for (size_t q = 0; q < m; ++q)
                T.order[q] = ((uint64_t)(uint32_t)key[T.used[q]] << 32) | (uint32_t)T.used[q];
            std::sort(T.order.begin(), T.order.end());
            std::vector<int32_t> &R = lrow[w];
            std::vector<double> &V = lval[w];
            lcol[w].push_back({j, (int64_t)R.size()});
            for (uint64_t e : T.order) {
                R.push_back((int32_t)(e >> 32));
                V.push_back(val[(uint32_t)e]);
            }
            cnt[j] = (int64_t)m;
            T.end();
        });
    } catch (...) {
        release(out);
        throw;
    }
    out.flops = 0;
    for (int64_t f : wflops) out.flops += f;
    out.colptr[0] = 0;
    for (int64_t j = 0; j < n; ++j) out.colptr[j + 1] += out.colptr[j];
    out.nnz = out.colptr[n];
    out.t_symbolic_ms = 0.0;
    out.t_numeric_ms = ms_since(t0);

    // gather every worker's columns into place
    const auto t1 = std::chrono::steady_clock::now();
    const size_t mm = (size_t)std::max<int64_t>(out.nnz, 1);
    out.rowidx = (int32_t *)std::malloc(sizeof(int32_t) * mm);
    out.val = (double *)std::malloc(sizeof(double) * mm);
    if (!out.rowidx || !out.val) {
        release(out);
        throw std::bad_alloc();
    }
    auto gather = [&](int w) {
        const std::vector<std::pair<int64_t, int64_t>> &L = lcol[w];
        for (size_t q = 0; q < L.size(); ++q) {
            const int64_t j = L[q].first, o = L[q].second;
            const int64_t m = out.colptr[j + 1] - out.colptr[j];
            std::copy(lrow[w].begin() + o, lrow[w].begin() + o + m, out.rowidx + out.colptr[j]);
            std::copy(lval[w].begin() + o, lval[w].begin() + o + m, out.val + out.colptr[j]);
        }
        std::vector<int32_t>().swap(lrow[w]);
        std::vector<double>().swap(lval[w]);
    };
    if (nw == 1) {
        gather(0);
    } else {
        std::vector<std::thread> pool;
        for (int w = 1; w < nw; ++w) pool.emplace_back(gather, w);
        gather(0);
        for (auto &t : pool) t.join();
    }
    out.t_numeric_ms += ms_since(t1);
}

}  // namespace host
}  // namespace mcl
