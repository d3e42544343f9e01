// Surrogate network kernels (gfx950): forward, backward and Adam of the
// 6 -> 128 -> 128 -> 128 -> 1 GELU network declared in include/lbm_mlp.h.
//
// Work split.  A workgroup of four waves owns 16 samples.  The 128 x 128
// layers are 16 x 128 by 128 x 128 products: each wave computes two 16 x 16
// output tiles with v_mfma_f32_16x16x4f32 (32 steps of K = 4), reading the
// 16 x 128 activation block from LDS and the weights from global memory (L2
// resident, 64 KB per layer).  The 6-wide input layer and the 1-wide output
// layer are plain FMA loops.  The weight gradients sum over the batch: each
// 16 x 16 tile of dW = dZ^T A is one wave running MFMA steps over the samples
// four at a time, so the sums have a fixed order and no atomics.
//
// Workspace (floats): nine planes of Bp x 128 (Bp = B rounded up to 16):
// Z1 A1 Z2 A2 Z3 A3 D1 D2 D3 (pre-activations, activations, dL/dZ), then Bp/16
// loss partials.  Rows B..Bp-1 hold the network's values at x = 0 and zero
// deltas, so they add nothing to the gradients.
#include "lbm_ctx.h"
#include "lbm_mlp.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

// Fixed scratch of lbm_mlp_gradient_noalloc: the workspace of the largest
// batch it accepts (LBM_MLP_NOALLOC_MAX_BATCH is a multiple of 16 samples, so
// rows_padded(B) stays within it for every accepted B).  Each device that
// loads the library holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel: the address of the current
// device's copy comes from noalloc_scratch().
constexpr size_t kScratchFloats =
    9 * (size_t)LBM_MLP_NOALLOC_MAX_BATCH * LBM_MLP_HIDDEN + LBM_MLP_NOALLOC_MAX_BATCH / 16;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kIn = LBM_MLP_IN;
constexpr int kH = LBM_MLP_HIDDEN;
constexpr int kRows = 16;               // samples per workgroup
constexpr int kLd = kH + 4;             // LDS row stride (floats)
constexpr int kThreads = 256;

// Offsets of the parameter blocks in the flat vector.
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kH,
              kParams = oB4 + 1;
static_assert(kParams == LBM_MLP_PARAMS, "parameter layout");

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

size_t rows_padded(int B) { return ((size_t)B + kRows - 1) / kRows * kRows; }

// One 16 x 16 tile of C = A B^T where A is a 16 x 128 block in LDS (row
// stride kLd) and B^T's columns are rows n0..n0+15 of a 128-wide row-major
// matrix W in global memory (C[i][j] = sum_k A[i][k] W[n0 + j][k]).
// v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][k0 + l / 16] and
// W[n0 + l % 16][k0 + l / 16]; it receives C[4 (l / 16) + r][l % 16], r = 0..3.
__device__ __forceinline__ f4 tile_abt(const float* A, const float* __restrict__ W, int n0, int lane)
{
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int i = lane & 15, kq = lane >> 4;
    const float* wrow = W + (size_t)(n0 + i) * kH;
#pragma unroll 8
    for (int k0 = 0; k0 < kH; k0 += 4) {
        const float a = A[i * kLd + k0 + kq];
        const float b = wrow[k0 + kq];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Same with B = W itself (C[i][j] = sum_n A[i][n] W[n][j0 + j]): the delta
// propagation dA = dZ W.
__device__ __forceinline__ f4 tile_ab(const float* A, const float* __restrict__ W, int j0, int lane)
{
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int i = lane & 15, kq = lane >> 4;
#pragma unroll 8
    for (int k0 = 0; k0 < kH; k0 += 4) {
        const float a = A[i * kLd + k0 + kq];
        const float b = W[(size_t)(k0 + kq) * kH + j0 + i];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    return acc;
}

__global__ void __launch_bounds__(kThreads)
mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ X, int B, size_t Bp,
                   float* __restrict__ y, float* __restrict__ ws)
{
    __shared__ float buf[2][kRows * kLd];
    __shared__ float xin[kRows * kIn];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s0 = blockIdx.x * kRows;
    float* Z[3] = {ws + 0 * Bp * kH, ws + 2 * Bp * kH, ws + 4 * Bp * kH};
    float* A[3] = {ws + 1 * Bp * kH, ws + 3 * Bp * kH, ws + 5 * Bp * kH};

    if (tid < kRows * kIn) {
        const int s = s0 + tid / kIn;
        xin[tid] = s < B ? X[(size_t)s * kIn + tid % kIn] : 0.0f;
    }
    __syncthreads();
    // Layer 1 (K = 6): 16 x 128 outputs, 8 per thread.
    for (int o = tid; o < kRows * kH; o += kThreads) {
        const int i = o / kH, n = o % kH;
        float z = P[oB1 + n];
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            z = fmaf(P[oW1 + n * kIn + k], xin[i * kIn + k], z);
        const float a = gelu(z);
        Z[0][(size_t)(s0 + i) * kH + n] = z;
        A[0][(size_t)(s0 + i) * kH + n] = a;
        buf[0][i * kLd + n] = a;
    }
    __syncthreads();
    // Layers 2 and 3 on the matrix cores: wave w owns neurons 32 w .. 32 w + 31.
    for (int l = 1; l < 3; ++l) {
        const float* W = P + (l == 1 ? oW2 : oW3);
        const float* bias = P + (l == 1 ? oB2 : oB3);
        const float* in = buf[(l - 1) & 1];
        float* out = buf[l & 1];
        for (int t = 0; t < 2; ++t) {
            const int n0 = 32 * wave + 16 * t;
            const f4 acc = tile_abt(in, W, n0, lane);
            const int j = lane & 15, ib = 4 * (lane >> 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ib + r, n = n0 + j;
                const float z = acc[r] + bias[n];
                const float a = gelu(z);
                Z[l][(size_t)(s0 + i) * kH + n] = z;
                A[l][(size_t)(s0 + i) * kH + n] = a;
                out[i * kLd + n] = a;
            }
        }
        __syncthreads();
    }
    // Layer 4 (N = 1): wave w reduces samples 4 w .. 4 w + 3.
    const float* a3 = buf[0];  // layer 1 wrote buf[0], layer 2 buf[1], layer 3 buf[0]
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * wave + q;
        float v = P[oW4 + lane] * a3[i * kLd + lane] + P[oW4 + 64 + lane] * a3[i * kLd + 64 + lane];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o, 64);
        if (lane == 0 && s0 + i < B)
            y[s0 + i] = v + P[oB4];
    }
}

// dL/dZ of the three hidden layers for the block's 16 samples.
__global__ void __launch_bounds__(kThreads)
mlp_delta_kernel(const float* __restrict__ P, const float* __restrict__ y,
                 const float* __restrict__ t, int B, size_t Bp, float* __restrict__ ws)
{
    __shared__ float buf[2][kRows * kLd];
    __shared__ float dy[kRows];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s0 = blockIdx.x * kRows;
    const float* Z[3] = {ws + 0 * Bp * kH, ws + 2 * Bp * kH, ws + 4 * Bp * kH};
    float* D[3] = {ws + 6 * Bp * kH, ws + 7 * Bp * kH, ws + 8 * Bp * kH};
    float* partial = ws + 9 * Bp * kH;

    if (tid < kRows) {
        const int s = s0 + tid;
        const float e = s < B ? y[s] - t[s] : 0.0f;
        dy[tid] = 2.0f * e / (float)B;
        float sq = e * e;  // loss partial of the block, fixed summation order
#pragma unroll
        for (int o = 8; o > 0; o >>= 1)
            sq += __shfl_xor(sq, o, 16);
        if (tid == 0)
            partial[blockIdx.x] = sq;
    }
    __syncthreads();
    // Layer 3: dZ3 = dy W4 o GELU'(Z3).
    for (int o = tid; o < kRows * kH; o += kThreads) {
        const int i = o / kH, n = o % kH;
        const size_t g = (size_t)(s0 + i) * kH + n;
        const float d = dy[i] * P[oW4 + n] * gelu_grad(Z[2][g]);
        D[2][g] = d;
        buf[0][i * kLd + n] = d;
    }
    __syncthreads();
    // Layers 2 and 1: dZ_l = (dZ_{l+1} W_{l+1}) o GELU'(Z_l) on the matrix cores.
    for (int l = 1; l >= 0; --l) {
        const float* W = P + (l == 1 ? oW3 : oW2);
        // dZ3 is in buf[0]; dZ2 goes to buf[1]; dZ1 is not needed in LDS.
        const float* in = buf[1 - l];
        float* out = buf[1];
        for (int tt = 0; tt < 2; ++tt) {
            const int j0 = 32 * wave + 16 * tt;
            const f4 acc = tile_ab(in, W, j0, lane);
            const int j = lane & 15, ib = 4 * (lane >> 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ib + r, k = j0 + j;
                const size_t g = (size_t)(s0 + i) * kH + k;
                const float d = acc[r] * gelu_grad(Z[l][g]);
                D[l][g] = d;
                if (l == 1)
                    out[i * kLd + k] = d;
            }
        }
        __syncthreads();
    }
}

// Weight gradients of layers 2 and 3: tile (n0, k0) of dW_l = D_l^T A_{l-1},
// one 16 x 16 tile per wave, samples four at a time.
// v_mfma_f32_16x16x4f32 with A-operand D_l[s][n0 + l % 16] and B-operand
// A_{l-1}[s][k0 + l % 16], s = s0 + l / 16: lane receives
// dW[n0 + 4 (l / 16) + r][k0 + l % 16].
__global__ void __launch_bounds__(kThreads)
mlp_wgrad_kernel(size_t Bp, const float* __restrict__ ws, float* __restrict__ grad)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int task = blockIdx.x * 4 + (tid >> 6);  // 0..127: layer (task / 64), tile (task % 64)
    const int l = 1 + task / 64, tile = task % 64;
    const int n0 = 16 * (tile / 8), k0 = 16 * (tile % 8);
    const float* Dl = ws + (size_t)(6 + l) * Bp * kH;
    const float* Ap = ws + (size_t)(2 * l - 1) * Bp * kH;  // A1 for l = 1, A2 for l = 2
    const int c = lane & 15, sq = lane >> 4;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (size_t s = 0; s < Bp; s += 4) {
        const float a = Dl[(s + sq) * kH + n0 + c];
        const float b = Ap[(s + sq) * kH + k0 + c];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    float* gW = grad + (l == 1 ? oW2 : oW3);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        gW[(size_t)(n0 + 4 * sq + r) * kH + k0 + c] = acc[r];
}

// The remaining gradients (W1, all biases, W4, b4) and the loss: one thread
// per parameter, each summing over the samples in order.
__global__ void mlp_grad_small_kernel(const float* __restrict__ X, const float* __restrict__ y,
                                      const float* __restrict__ t, int B, size_t Bp,
                                      const float* __restrict__ ws, float* __restrict__ grad,
                                      float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const float* A3 = ws + 5 * Bp * kH;
    const float* D1 = ws + 6 * Bp * kH;
    const float* partial = ws + 9 * Bp * kH;
    float acc = 0.0f;
    if (p < kH * kIn) {  // W1[n][k] = sum_s D1[s][n] x[s][k]
        const int n = p / kIn, k = p % kIn;
        for (int s = 0; s < B; ++s)
            acc = fmaf(D1[(size_t)s * kH + n], X[(size_t)s * kIn + k], acc);
        grad[oW1 + p] = acc;
    } else if (p < kH * kIn + 3 * kH) {  // b1, b2, b3
        const int q = p - kH * kIn, l = q / kH, n = q % kH;
        const float* Dl = ws + (size_t)(6 + l) * Bp * kH;
        for (int s = 0; s < B; ++s)
            acc += Dl[(size_t)s * kH + n];
        grad[(l == 0 ? oB1 : (l == 1 ? oB2 : oB3)) + n] = acc;
    } else if (p < kH * kIn + 4 * kH) {  // W4[n] = sum_s dy[s] A3[s][n]
        const int n = p - kH * kIn - 3 * kH;
        for (int s = 0; s < B; ++s)
            acc = fmaf(2.0f * (y[s] - t[s]) / (float)B, A3[(size_t)s * kH + n], acc);
        grad[oW4 + n] = acc;
    } else if (p == kH * kIn + 4 * kH) {  // b4, loss
        float sq = 0.0f;
        for (int s = 0; s < B; ++s)
            acc += 2.0f * (y[s] - t[s]) / (float)B;
        grad[oB4] = acc;
        for (size_t b = 0; b < Bp / kRows; ++b)
            sq += partial[b];
        if (loss)
            loss[0] = sq / (float)B;
    }
}

__global__ void mlp_adam_kernel(float* __restrict__ P, const float* __restrict__ g,
                                float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams)
        return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

size_t ws_bytes_for(int B) { return sizeof(float) * (9 * rows_padded(B) * kH + rows_padded(B) / kRows); }

static_assert(LBM_MLP_NOALLOC_MAX_BATCH % kRows == 0, "scratch batch must be a multiple of 16");
static_assert(kScratchFloats == 9 * (size_t)LBM_MLP_NOALLOC_MAX_BATCH * kH +
                                    LBM_MLP_NOALLOC_MAX_BATCH / kRows,
              "scratch holds the workspace of the largest accepted batch");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device
// (with that device current) and kept.
lbm_status noalloc_scratch(float** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return lbm::fail(LBM_ERR_DEVICE, "lbm_mlp_gradient_noalloc: hipGetDevice: %s",
                         hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return lbm::fail(LBM_ERR_UNSUPPORTED, "lbm_mlp_gradient_noalloc: device %d beyond %d",
                         dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return lbm::fail(LBM_ERR_DEVICE,
                             "lbm_mlp_gradient_noalloc: hipGetSymbolAddress(scratch): %s",
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

// The four launches of one forward and backward pass over workspace ws.
hipError_t launch_forward_backward(const float* params, const float* X, const float* t, int B,
                                   float* y, float* grad, float* loss, float* ws,
                                   hipStream_t st)
{
    const size_t Bp = rows_padded(B);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)(Bp / kRows)), dim3(kThreads), 0, st,
                       params, X, B, Bp, y, ws);
    hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)(Bp / kRows)), dim3(kThreads), 0, st,
                       params, y, t, B, Bp, ws);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(32), dim3(kThreads), 0, st, Bp,
                       (const float*)ws, grad);
    const int small = kH * kIn + 4 * kH + 1;
    hipLaunchKernelGGL(mlp_grad_small_kernel, dim3((small + 255) / 256), dim3(256), 0, st, X, y,
                       t, B, Bp, (const float*)ws, grad, loss);
    return hipGetLastError();
}

}  // namespace

using lbm::fail;

extern "C" {

size_t lbm_mlp_workspace_bytes(int32_t max_batch)
{
    return max_batch < 1 ? 0 : ws_bytes_for(max_batch);
}

lbm_status lbm_mlp_forward(const float* params, const float* X, int32_t B, float* y, void* ws,
                           size_t ws_bytes, void* hip_stream)
{
    if (!params || !X || !y || !ws || B < 1)
        return fail(LBM_ERR_INVALID, "lbm_mlp_forward: null pointer or B < 1");
    if (ws_bytes < ws_bytes_for(B))
        return fail(LBM_ERR_OOM, "lbm_mlp_forward: workspace %zu < %zu bytes", ws_bytes,
                    ws_bytes_for(B));
    const size_t Bp = rows_padded(B);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)(Bp / kRows)), dim3(kThreads), 0,
                       (hipStream_t)hip_stream, params, X, (int)B, Bp, y, (float*)ws);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "lbm_mlp_forward: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_mlp_backward(const float* params, const float* X, const float* y,
                            const float* t, int32_t B, float* grad, float* loss, void* ws,
                            size_t ws_bytes, void* hip_stream)
{
    if (!params || !X || !y || !t || !grad || !ws || B < 1)
        return fail(LBM_ERR_INVALID, "lbm_mlp_backward: null pointer or B < 1");
    if (ws_bytes < ws_bytes_for(B))
        return fail(LBM_ERR_OOM, "lbm_mlp_backward: workspace %zu < %zu bytes", ws_bytes,
                    ws_bytes_for(B));
    const size_t Bp = rows_padded(B);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)(Bp / kRows)), dim3(kThreads), 0, st,
                       params, y, t, (int)B, Bp, (float*)ws);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(32), dim3(kThreads), 0, st, Bp,
                       (const float*)ws, grad);
    const int small = kH * kIn + 4 * kH + 1;
    hipLaunchKernelGGL(mlp_grad_small_kernel, dim3((small + 255) / 256), dim3(256), 0, st, X, y,
                       t, (int)B, Bp, (const float*)ws, grad, loss);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "lbm_mlp_backward: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_mlp_gradient_noalloc(const float* params, const float* X, const float* t,
                                    int32_t B, float* y, float* grad, float* loss,
                                    void* hip_stream)
{
    if (!params || !X || !t || !y || !grad || B < 1)
        return fail(LBM_ERR_INVALID, "lbm_mlp_gradient_noalloc: null pointer or B < 1");
    if (B > LBM_MLP_NOALLOC_MAX_BATCH)
        return fail(LBM_ERR_INVALID,
                    "lbm_mlp_gradient_noalloc: B = %d exceeds the fixed scratch of %d samples",
                    (int)B, LBM_MLP_NOALLOC_MAX_BATCH);
    float* ws = nullptr;
    const lbm_status st = noalloc_scratch(&ws);
    if (st != LBM_OK)
        return st;
    const hipError_t e = launch_forward_backward(params, X, t, (int)B, y, grad, loss, ws,
                                                 (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "lbm_mlp_gradient_noalloc: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t k,
                        float lr, float beta1, float beta2, float eps, void* hip_stream)
{
    if (!params || !grad || !m || !v || k < 1)
        return fail(LBM_ERR_INVALID, "lbm_mlp_adam: null pointer or k < 1");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)k));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)k));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                       (hipStream_t)hip_stream, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(LBM_ERR_DEVICE, "lbm_mlp_adam: %s", hipGetErrorString(e));
    return LBM_OK;
}

}  // extern "C"
