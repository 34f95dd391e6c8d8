// Learned output-size estimator: a 12 -> 64 -> 64 -> 1 ReLU MLP predicting
// log(1 + nnz) of a product column from 12 per-column features.  Weights are
// stored in BF16 (round-to-nearest-even from FP32 master weights); the layer
// inputs (features, hidden activations) are rounded to BF16 too, so every
// product is exact in FP32 and accumulation is FP32 in a fixed order
// (bias first, then inputs in index order).  Training: mean squared error on
// log(1 + nnz), analytic backward (the BF16 roundings are treated as the
// identity), Adam on the FP32 masters.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

namespace mcl {

// parameter layout (FP32 master and BF16 packed use the same order)
constexpr int OFF_W1 = 0;                          // [64][12]
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;    // [64]
constexpr int OFF_W2 = OFF_B1 + MLP_H;             // [64][64]
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;     // [64]
constexpr int OFF_W3 = OFF_B2 + MLP_H;             // [64]
constexpr int OFF_B3 = OFF_W3 + MLP_H;             // [1]
constexpr int NPARAM = OFF_B3 + 1;                 // 5057
constexpr int NPARAM_PAD = 5120;
// state: master[NPARAM_PAD], m[NPARAM_PAD], v[NPARAM_PAD], step[1] (+pad)
constexpr int ST_M = NPARAM_PAD, ST_V = 2 * NPARAM_PAD, ST_T = 3 * NPARAM_PAD;
constexpr int STATE_FLOATS = 3 * NPARAM_PAD + 64;

size_t mlp_packed_bytes() { return (size_t)NPARAM_PAD * 2; }
size_t mlp_state_floats() { return STATE_FLOATS; }

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16 round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float rbf(float f) { return bf16_to_f(f_to_bf16(f)); }

// Forward of one row with weights in LDS (as FP32 values of the BF16 weights).
// Returns the output; fills h1, h2 (BF16-rounded activations) and the
// pre-activation signs when requested.
struct Acts {
    float x[MLP_IN];
    float h1[MLP_H];
    float h2[MLP_H];
};

__device__ __forceinline__ float mlp_row(const float *__restrict__ w, const float *__restrict__ feat, Acts &a)
{
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a.x[i] = rbf(feat[i]);
#pragma unroll 4
    for (int o = 0; o < MLP_H; ++o) {
        float acc = w[OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(w[OFF_W1 + o * MLP_IN + i], a.x[i], acc);
        a.h1[o] = rbf(fmaxf(acc, 0.f));
    }
#pragma unroll 2
    for (int o = 0; o < MLP_H; ++o) {
        float acc = w[OFF_B2 + o];
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) acc = fmaf(w[OFF_W2 + o * MLP_H + k], a.h1[k], acc);
        a.h2[o] = rbf(fmaxf(acc, 0.f));
    }
    float out = w[OFF_B3];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) out = fmaf(w[OFF_W3 + k], a.h2[k], out);
    return out;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *__restrict__ packed,
                                                     const float *__restrict__ feat, int64_t rows,
                                                     float *__restrict__ out)
{
    __shared__ float w[NPARAM_PAD];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) w[i] = bf16_to_f(packed[i]);
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        Acts a;
        out[r] = mlp_row(w, feat + r * MLP_IN, a);
    }
}

void launch_mlp_forward(const void *packed, const float *feat, int64_t rows, float *out, hipStream_t st)
{
    if (rows <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((rows + 255) / 256, 2048);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, st, (const uint16_t *)packed, feat, rows,
                       out);
}

// est = max(expm1(est), 0): the learned model predicts log(1 + nnz).
__global__ void k_expm1(float *__restrict__ v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = fmaxf(expm1f(fminf(v[i], 40.f)), 0.f);
}

void launch_expm1_inplace(float *v, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_expm1, dim3(grid), dim3(256), 0, st, v, n);
}

// ---------------------------------------------------------------------------
// initialisation: He-uniform weights from SplitMix64, zero biases and moments
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_mlp_init(float *__restrict__ st, uint64_t seed)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < STATE_FLOATS; i += gridDim.x * blockDim.x) {
        float v = 0.f;
        if (i < NPARAM) {
            int fan_in = 0;
            if (i < OFF_B1) fan_in = MLP_IN;
            else if (i >= OFF_W2 && i < OFF_B2) fan_in = MLP_H;
            else if (i >= OFF_W3 && i < OFF_B3) fan_in = MLP_H;
            if (fan_in) {
                const uint64_t x = mix64(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
                const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);  // [0,1)
                const double lim = sqrt(6.0 / fan_in);
                v = (float)((2.0 * u - 1.0) * lim);
            }
        }
        st[i] = v;
    }
}

void launch_mlp_init(float *state, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3(64), dim3(256), 0, st, state, seed);
}

// ---------------------------------------------------------------------------
// training step
// ---------------------------------------------------------------------------
// Per-row intermediates (row-major, floats): x[12] h1[64] h2[64] dz1[64]
// dz2[64] dout[1]  -> 269 floats per row.
constexpr int ROWF = MLP_IN + 4 * MLP_H + 1;
constexpr int TILE_ROWS = 64;
constexpr int GRAD_BLOCKS = 128;

size_t mlp_train_tmp_floats(int64_t rows)
{
    // loss[1] | grad partials [GRAD_BLOCKS][NPARAM_PAD] | grad[NPARAM_PAD] | loss partials | rows
    return 64 + (size_t)GRAD_BLOCKS * NPARAM_PAD + NPARAM_PAD + 4096 + (size_t)rows * ROWF;
}

__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float *__restrict__ master,
                                                     const float *__restrict__ feat,
                                                     const float *__restrict__ target, int64_t rows,
                                                     float *__restrict__ inter, float *__restrict__ loss_part)
{
    __shared__ float w[NPARAM_PAD];
    __shared__ float red[256];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) w[i] = rbf(master[i]);
    __syncthreads();
    float lsum = 0.f;
    const float inv_n = 1.0f / (float)rows;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        Acts a;
        const float out = mlp_row(w, feat + r * MLP_IN, a);
        const float err = out - target[r];
        lsum += err * err;
        const float dout = 2.f * err * inv_n;
        float *q = inter + r * ROWF;
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) q[i] = a.x[i];
        float dz2[MLP_H];
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) {
            q[MLP_IN + k] = a.h1[k];
            q[MLP_IN + MLP_H + k] = a.h2[k];
            dz2[k] = (a.h2[k] > 0.f) ? dout * w[OFF_W3 + k] : 0.f;
            q[MLP_IN + 3 * MLP_H + k] = dz2[k];
        }
#pragma unroll 2
        for (int k = 0; k < MLP_H; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int o = 0; o < MLP_H; ++o) acc = fmaf(w[OFF_W2 + o * MLP_H + k], dz2[o], acc);
            q[MLP_IN + 2 * MLP_H + k] = (a.h1[k] > 0.f) ? acc : 0.f;
        }
        q[MLP_IN + 4 * MLP_H] = dout;
    }
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Gradient partials: block b sums rows [b*chunk, (b+1)*chunk) for every
// parameter, staged through LDS tiles of 64 rows.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ inter, int64_t rows,
                                                  float *__restrict__ part)
{
    __shared__ float tile[TILE_ROWS][ROWF + 1];
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = std::min<int64_t>(rows, r0 + chunk);
    float acc[(NPARAM + 255) / 256];
#pragma unroll
    for (int q = 0; q < (NPARAM + 255) / 256; ++q) acc[q] = 0.f;
    for (int64_t t0 = r0; t0 < r1; t0 += TILE_ROWS) {
        const int nr = (int)std::min<int64_t>(TILE_ROWS, r1 - t0);
        for (int e = threadIdx.x; e < nr * ROWF; e += blockDim.x) tile[e / ROWF][e % ROWF] = inter[t0 * ROWF + e];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (NPARAM + 255) / 256; ++q) {
            const int p = threadIdx.x + q * 256;
            if (p >= NPARAM) continue;
            int ga, gb;  // gradient = sum_r tile[r][ga] * (gb < 0 ? 1 : tile[r][gb])
            if (p < OFF_B1) { ga = MLP_IN + 2 * MLP_H + p / MLP_IN; gb = p % MLP_IN; }
            else if (p < OFF_W2) { ga = MLP_IN + 2 * MLP_H + (p - OFF_B1); gb = -1; }
            else if (p < OFF_B2) { ga = MLP_IN + 3 * MLP_H + (p - OFF_W2) / MLP_H; gb = MLP_IN + (p - OFF_W2) % MLP_H; }
            else if (p < OFF_W3) { ga = MLP_IN + 3 * MLP_H + (p - OFF_B2); gb = -1; }
            else if (p < OFF_B3) { ga = MLP_IN + 4 * MLP_H; gb = MLP_IN + MLP_H + (p - OFF_W3); }
            else { ga = MLP_IN + 4 * MLP_H; gb = -1; }
            float s = acc[q];
            for (int r = 0; r < nr; ++r) s = fmaf(tile[r][ga], (gb < 0) ? 1.f : tile[r][gb], s);
            acc[q] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < (NPARAM + 255) / 256; ++q) {
        const int p = threadIdx.x + q * 256;
        if (p < NPARAM) part[(int64_t)blockIdx.x * NPARAM_PAD + p] = acc[q];
    }
}

// Final gradient (blocks summed in order), loss, Adam update and BF16 pack.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ st, uint16_t *__restrict__ packed,
                                                  const float *__restrict__ part, int nparts,
                                                  const float *__restrict__ loss_part, int nloss,
                                                  int64_t rows, float lr, float *__restrict__ loss,
                                                  float *__restrict__ grad_out)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float t = st[ST_T] + 1.f;
    __syncthreads();
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPARAM; p += gridDim.x * blockDim.x) {
        float g = 0.f;
        for (int b = 0; b < nparts; ++b) g += part[(int64_t)b * NPARAM_PAD + p];
        if (grad_out) grad_out[p] = g;
        const float m = b1 * st[ST_M + p] + (1.f - b1) * g;
        const float v = b2 * st[ST_V + p] + (1.f - b2) * g * g;
        st[ST_M + p] = m;
        st[ST_V + p] = v;
        const float mh = m / (1.f - powf(b1, t));
        const float vh = v / (1.f - powf(b2, t));
        const float w = st[p] - lr * mh / (sqrtf(vh) + eps);
        st[p] = w;
        packed[p] = f_to_bf16(w);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.f;
        for (int b = 0; b < nloss; ++b) s += loss_part[b];
        *loss = s / (float)rows;
    }
}

__global__ void k_mlp_step_count(float *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st[ST_T] += 1.f;
}

void launch_mlp_train_step(float *state, void *packed, const float *feat, const float *target, int64_t rows,
                           float lr, float *tmp, float *grad_out, float *, hipStream_t st)
{
    float *loss = tmp;
    float *part = tmp + 64;
    float *loss_part = part + (size_t)GRAD_BLOCKS * NPARAM_PAD + NPARAM_PAD;
    float *inter = loss_part + 4096;
    const int fb = (int)std::min<int64_t>((rows + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(fb), dim3(256), 0, st, state, feat, target, rows, inter, loss_part);
    const int gb = (int)std::min<int64_t>(GRAD_BLOCKS, (rows + TILE_ROWS - 1) / TILE_ROWS);
    hipLaunchKernelGGL(k_mlp_grad, dim3(gb), dim3(256), 0, st, inter, rows, part);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, state, (uint16_t *)packed,
                       part, gb, loss_part, fb, rows, lr, loss, grad_out);
    hipLaunchKernelGGL(k_mlp_step_count, dim3(1), dim3(64), 0, st, state);
}

}  // namespace mcl
