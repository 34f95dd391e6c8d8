// Connected components of the pattern of a sparse matrix (arXiv 2002.10083,
// Alg. 1: the clusters MCL returns are the connected components of the
// converged matrix).  The graph is the undirected one with an edge i -- j for
// every stored entry a_ij (i != j), i.e. weak connectivity of the directed
// pattern; each vertex is labelled with the smallest vertex id of its
// component.
//
// Lock-free union-find on a parent array in HBM.  Every union links the
// larger of the two roots under the smaller one with a compare-and-swap on
// the larger root's parent slot, so parent ids only ever decrease, no cycle
// can form, and the root of every tree is the smallest id in it: once all
// edges are processed, find(v) is the component's smallest vertex id.  A
// failed compare-and-swap means another lane changed that root, so every
// retry follows a strictly smaller root and the loop ends.  Finds halve paths
// with atomicMin (a node may take any ancestor as its parent).
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace mcl {

// Parent reads bypass the non-coherent per-CU cache: a stale view would only
// cost a failed compare-and-swap, but fresh views keep retries short.
__device__ __forceinline__ int32_t parent_of(int32_t *parent, int32_t v)
{
    return __hip_atomic_load(parent + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t v)
{
    int32_t p = parent_of(parent, v);
    while (p != v) {
        const int32_t gp = parent_of(parent, p);
        if (gp != p) atomicMin(parent + v, gp);  // path halving: gp is an ancestor of v
        v = p;
        p = gp;
    }
    return v;
}

__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b)
{
    int32_t ra = find_root(parent, a), rb = find_root(parent, b);
    while (ra != rb) {
        const int32_t hi = max(ra, rb), lo = min(ra, rb);
        const int32_t old = atomicCAS(parent + hi, hi, lo);
        if (old == hi) return;          // hi now hangs under lo
        // hi stopped being a root: continue from the roots of both sides
        ra = find_root(parent, old);
        rb = find_root(parent, lo);
    }
}

// Every vertex starts as its own root; the root counter is cleared here (a
// kernel, not a memset, so the whole sequence can be recorded in a graph).
__global__ __launch_bounds__(256) void k_cc_init(int64_t n, int32_t *__restrict__ parent,
                                                 unsigned long long *__restrict__ nroots)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *nroots = 0ull;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = (int32_t)v;
}

// One wavefront per column j: every stored row i != j is united with j.
__global__ __launch_bounds__(256) void k_cc_hook(DevCSC A, int32_t *__restrict__ parent)
{
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t j = (int64_t)blockIdx.x * 4 + threadIdx.x / WAVE; j < A.ncols; j += nw) {
        const int64_t s = A.colptr[j], e = A.colptr[j + 1];
        for (int64_t p = s + lane(); p < e; p += WAVE) {
            const int32_t i = A.rowidx[p];
            if (i != (int32_t)j) unite(parent, i, (int32_t)j);
        }
    }
}

// Final labels: the root of every vertex (all unions have completed, so the
// trees no longer change); counts the roots.
__global__ __launch_bounds__(256) void k_cc_label(int64_t n, int32_t *__restrict__ parent,
                                                  int32_t *__restrict__ label,
                                                  unsigned long long *__restrict__ nroots)
{
    int64_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = find_root(parent, (int32_t)v);
        label[v] = r;
        c += (r == (int32_t)v) ? 1 : 0;
    }
    c = wave_sum_i64(c);
    if (lane() == 0 && c) atomicAdd(nroots, (unsigned long long)c);
}

void launch_components(const DevCSC &A, int32_t *parent, int32_t *label, int64_t *nroots, hipStream_t st)
{
    const int64_t n = A.nrows;
    if (n <= 0) return;
    const unsigned gv = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cc_init, dim3(gv), dim3(256), 0, st, n, parent, (unsigned long long *)nroots);
    if (A.ncols > 0) {
        const unsigned gc = (unsigned)std::min<int64_t>((A.ncols + 3) / 4, 65536);
        hipLaunchKernelGGL(k_cc_hook, dim3(gc), dim3(256), 0, st, A, parent);
    }
    hipLaunchKernelGGL(k_cc_label, dim3(gv), dim3(256), 0, st, n, parent, label,
                       (unsigned long long *)nroots);
}

}  // namespace mcl
