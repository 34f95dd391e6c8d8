// Device-side helpers shared by the gfx950 kernels: 64-lane wavefront
// collectives, fixed-shape (deterministic) reductions, workgroup scans and an
// exact radix select over FP64 bit patterns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcl {

constexpr int WAVE = 64;
constexpr int32_t EMPTY_KEY = -1;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l)
{
    int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
    int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    return __longlong_as_double(readlane_i64(__double_as_longlong(v), l));
}

// Load through a pointer known to address global memory.  Pointers that
// pass through readlane or a select lose their address space; without the
// cast the compiler emits flat loads, which also count against the LDS
// counter and serialise every LDS access behind outstanding gathers.
template <typename T>
__device__ __forceinline__ T ldg(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// Xor-butterfly sum over the 64 lanes.  Lane l and lane l^d always add the
// same two operands (in swapped order), so every lane ends with the same,
// schedule-independent value.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, WAVE));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, WAVE));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, WAVE));
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// Per-lane gathers from lane `src` (any lane index per lane).
__device__ __forceinline__ int shfl_i(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src)
{
    const int lo = shfl_i((int)(uint32_t)v, src), hi = shfl_i((int)(v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double shfl_d(double v, int src)
{
    return __longlong_as_double(shfl_i64(__double_as_longlong(v), src));
}

__device__ __forceinline__ int popc_below(uint64_t mask)
{
    return __popcll(mask & ((1ull << lane()) - 1ull));
}

// Inclusive prefix sum over lanes (Hillis-Steele on shuffles).
__device__ __forceinline__ int wave_incl_scan(int x)
{
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(x, d, WAVE);
        if (lane() >= d) x += y;
    }
    return x;
}

// Synchronisation of the NT threads that cooperate on one column: a
// workgroup barrier for a multi-wave group, a wavefront fence for a single
// wave (the LDS operations of one wavefront execute in order; the fence only
// keeps the compiler from reordering them).  NT-thread groups are aligned to
// wavefronts.
//
// GS (global scratch) selects what the barrier orders: false = LDS only --
// the fence is restricted to the local address space, so outstanding global
// loads (prefetched gathers) stay in flight across the barrier; true = LDS
// and global memory (a full workgroup fence, which on this architecture
// drains every outstanding vector memory operation).
template <int NT, bool GS = false>
__device__ __forceinline__ void group_sync()
{
    if constexpr (NT <= WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if constexpr (GS) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
}

// Group-wide exclusive scan of a[0..n) in place (LDS or global memory).
// `wsum` is LDS scratch of at least NT/64 ints owned by the group.  Returns
// the total to every thread.  Must be called by all NT threads of the group.
template <int NT, bool GS = false, typename T>
__device__ T block_exscan(T *a, int n, int *wsum)
{
    const int tid = threadIdx.x % NT;
    const int per = (n + NT - 1) / NT;
    const int st = min(n, tid * per), en = min(n, st + per);
    T s = 0;
    for (int i = st; i < en; ++i) s += a[i];
    int x = wave_incl_scan((int)s);
    if (lane() == WAVE - 1) wsum[tid / WAVE] = x;
    group_sync<NT, GS>();
    int off = 0, tot = 0;
    for (int w = 0; w < (NT + WAVE - 1) / WAVE; ++w) {
        int v = wsum[w];
        if (w < tid / WAVE) off += v;
        tot += v;
    }
    T run = (T)(off + x - (int)s);
    for (int i = st; i < en; ++i) { T t = a[i]; a[i] = run; run += t; }
    group_sync<NT, GS>();
    return (T)tot;
}

// Second and third level of the fixed reduction tree: lane l accumulates the
// block sums l, l+64, l+128, ... in order, then the lanes are combined by the
// butterfly.  Called by one whole wave.
__device__ __forceinline__ double fixed_tree_finish(const double *blk, int nblk)
{
    double acc = 0.0;
    for (int b = lane(); b < nblk; b += WAVE) acc += blk[b];
    return wave_sum(acc);
}

// Hash of a row index into a power-of-two table (Fibonacci hashing).
__device__ __forceinline__ uint32_t hash_slot(int32_t key, int logS)
{
    return ((uint32_t)key * 2654435761u) >> (32 - logS);
}

// Inflation power c^r; r == 2 is an exact square, r == 1 the identity.
__device__ __forceinline__ double inflate_pow(double c, double r)
{
    return (r == 2.0) ? c * c : (r == 1.0) ? c : pow(c, r);
}

}  // namespace mcl
