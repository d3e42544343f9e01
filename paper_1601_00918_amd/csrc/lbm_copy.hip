// Streaming device copy: the bandwidth ceiling the step kernels are measured
// against.  A step reads every population once and writes it once, in equal
// amounts, with nontemporal stores; this kernel moves bytes the same way and
// does nothing else.  Each lane moves 16-byte vectors, UNROLL of them in
// flight (all loads issued before the first store), over a grid-stride loop;
// a tail shorter than one vector per lane is copied 4 bytes at a time.
#include "lbm.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef uint32_t u4v __attribute__((ext_vector_type(4)));

template <int UNROLL>
__global__ void __launch_bounds__(256)
copy_kernel(const u4v* __restrict__ src, u4v* __restrict__ dst, int64_t n_vec)
{
    const int64_t lanes = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t i = tid;
    for (; i + (UNROLL - 1) * lanes < n_vec; i += UNROLL * lanes) {
        u4v v[UNROLL];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k)
            v[k] = __builtin_nontemporal_load(src + i + k * lanes);
#pragma unroll
        for (int k = 0; k < UNROLL; ++k)
            __builtin_nontemporal_store(v[k], dst + i + k * lanes);
    }
    for (; i < n_vec; i += lanes)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void copy_tail_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                 int64_t n_words)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_words)
        dst[i] = src[i];
}

}  // namespace

extern "C" lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes,
                                      int32_t blocks, void* hip_stream)
{
    if (!src || !dst || bytes % 4 || ((uintptr_t)src | (uintptr_t)dst) % 16 || blocks < 1)
        return LBM_ERR_INVALID;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t n_vec = (int64_t)(bytes / 16);
    if (n_vec > 0)
        copy_kernel<4><<<dim3(blocks), dim3(256), 0, st>>>(static_cast<const u4v*>(src),
                                                          static_cast<u4v*>(dst), n_vec);
    const int64_t tail = (int64_t)(bytes % 16) / 4;
    if (tail > 0)
        copy_tail_kernel<<<dim3(1), dim3(64), 0, st>>>(
            static_cast<const uint32_t*>(src) + 4 * n_vec, static_cast<uint32_t*>(dst) + 4 * n_vec,
            tail);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_DEVICE;
}
