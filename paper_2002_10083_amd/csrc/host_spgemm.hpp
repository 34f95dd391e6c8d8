// Multithreaded CPU hash SpGEMM (arXiv 2002.10083, Section 6 "Faster SpGEMM
// on CPU"): the host path of the expansion, used by the per-multiplication
// CPU/GPU dispatch (Section 3 "Pipelined Sparse SUMMA": too few flops to
// occupy the GPU -> CPU).  Plain C++ (no HIP), built with the host compiler
// and linked into libmcl.so.  Not installed.
#pragma once

#include <stdint.h>

namespace mcl {
namespace host {

struct CSC {
    int64_t nrows, ncols, nnz;
    const int64_t *colptr;
    const int32_t *rowidx;
    const double *val;
};

struct Out {
    int64_t *colptr = nullptr;  // malloc'd, ncols + 1
    int32_t *rowidx = nullptr;  // malloc'd, nnz (at least one element)
    double *val = nullptr;      // malloc'd, nnz (at least one element)
    int64_t nnz = 0;
    int64_t flops = 0;
    double t_symbolic_ms = 0, t_numeric_ms = 0;
    int threads = 0;            // worker threads used
};

// Structure checks a host CSC must pass before it is read: colptr[0] == 0,
// non-decreasing, colptr[ncols] == nnz, 0 <= row < nrows.  Returns an empty
// string when the matrix is well formed, else what is wrong.
const char *check(const CSC &m);

// Number of worker threads: nthreads > 0 as given, else OMP_NUM_THREADS when
// it is set to a positive count, else the host's hardware concurrency.
int threads_for(int nthreads);

// flops = sum_j sum_{k in B_*j} nnz(A_*k) on `threads` workers.
int64_t flops(const CSC &A, const CSC &B, int threads);

// C = A*B.  Per column j the products a_ik * b_kj are accumulated in
// ascending order of k, each product rounded before the addition (build
// without contraction), so the result is bit-identical to every other
// expansion of the library.  Throws std::bad_alloc when host memory runs
// out (nothing is leaked).
void spgemm(const CSC &A, const CSC &B, int threads, Out &out);

// Releases the arrays of an Out (or of an output handed to the caller).
void release(Out &out);

}  // namespace host
}  // namespace mcl
