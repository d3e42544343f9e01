// Device helpers shared by the D2Q9 and D3Q19 step kernels: the population
// storage formats (FP32 pairs and the 16-bit deviation formats), rounding
// helpers, the counter-based hash that drives stochastic rounding, the
// XCD-aware workgroup remap and an LDS-only barrier.  Device code only.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {
namespace dev {

struct F16Tag {};
struct BF16Tag {};

typedef float f2v __attribute__((ext_vector_type(2)));

template <typename T>
struct Store;

template <>
struct Store<float> {
    static constexpr uint32_t kBytes = 4;  // one species value
    static constexpr uint32_t kPair = 8;   // one (oil, water) pair
    static constexpr float kScale = 1.0f;
    static constexpr bool kRef = false;
    using Pair = f2v;
    __device__ static Pair load(const char* p) { return *reinterpret_cast<const f2v*>(p); }
    __device__ static void unpack(Pair v, float& a, float& b)
    {
        a = v.x;
        b = v.y;
    }
    __device__ static void put(char* p, float a, float b)
    {
        f2v v;
        v.x = a;
        v.y = b;
        __builtin_nontemporal_store(v, reinterpret_cast<f2v*>(p));
    }
};

__device__ __forceinline__ void put32(char* p, uint32_t b)
{
    __builtin_nontemporal_store(b, reinterpret_cast<uint32_t*>(p));
}

__device__ __forceinline__ float h2f(uint32_t b)
{
    return __half2float(__ushort_as_half((unsigned short)b));
}
__device__ __forceinline__ uint32_t f2h_rn(float v) { return __half_as_ushort(__float2half_rn(v)); }

template <>
struct Store<F16Tag> {
    static constexpr uint32_t kBytes = 2;
    static constexpr uint32_t kPair = 4;
    static constexpr float kScale = 36.0f;
    static constexpr bool kRef = true;
    using Pair = uint32_t;
    __device__ static Pair load(const char* p) { return *reinterpret_cast<const uint32_t*>(p); }
    __device__ static void unpack(Pair v, float& a, float& b)
    {
        a = h2f(v & 0xffffu);
        b = h2f(v >> 16);
    }
    __device__ static float val(uint32_t b) { return h2f(b); }
    __device__ static uint32_t rne(float v) { return f2h_rn(v); }
    // Stochastic rounding to binary16 with 16 uniform random bits r16: add
    // random bits below the target precision to the magnitude and truncate
    // (exact conversion after).  Where more than 16 bits lie below the last
    // place (deep subnormals) the random offset is r16 shifted up, so the
    // probability of rounding up is quantised to 2^-16.
    __device__ static uint32_t sr(float v, uint32_t r16)
    {
        const uint32_t u = __float_as_uint(v);
        const uint32_t sign = u & 0x80000000u;
        uint32_t a = u & 0x7fffffffu;
        const int e = (int)(a >> 23) - 127;
        if (e >= -14) {  // binary16 normal range: 13 bits below the last place
            a = (a + (r16 & 0x1fffu)) & ~0x1fffu;
        } else if (e >= -24) {  // subnormal: the last place is 2^-24, k bits below it
            const int k = -1 - e;
            const uint32_t m = (1u << (uint32_t)k) - 1u;
            const uint32_t rk = k > 16 ? (r16 << (uint32_t)(k - 16)) : (r16 & m);
            a = (a + rk) & ~m;
        } else {  // below 2^-24: 0 or 2^-24 with probability |v| / 2^-24
            a = (float)r16 * 0x1p-16f < __uint_as_float(a) * 0x1p24f ? 0x33800000u : 0u;
        }
        return f2h_rn(__uint_as_float(sign | a));
    }
};

template <>
struct Store<BF16Tag> {
    static constexpr uint32_t kBytes = 2;
    static constexpr uint32_t kPair = 4;
    static constexpr float kScale = 36.0f;
    static constexpr bool kRef = true;
    using Pair = uint32_t;
    __device__ static Pair load(const char* p) { return *reinterpret_cast<const uint32_t*>(p); }
    __device__ static void unpack(Pair v, float& a, float& b)
    {
        a = __uint_as_float(v << 16);
        b = __uint_as_float(v & 0xffff0000u);
    }
    __device__ static float val(uint32_t b) { return __uint_as_float(b << 16); }
    // Round to nearest even (the deviations are finite by construction).
    __device__ static uint32_t rne(float v)
    {
        const uint32_t u = __float_as_uint(v);
        return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    }
    // Stochastic rounding with 16 uniform random bits r16.
    __device__ static uint32_t sr(float v, uint32_t r16)
    {
        return (__float_as_uint(v) + (r16 & 0xffffu)) >> 16;
    }
};

// Integer hash (Wellons' "lowbias32", from his 2018 hash-prospector search):
// a bijection of 32-bit integers with low bias, used as a counter-based
// generator for the stochastic rounding bits.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Two independent 16-bit random values for the stochastic rounding of both
// species at one node: the halves of one hash of the node's key.
__device__ __forceinline__ void split_rnd(uint32_t h, uint32_t (&rnd)[2])
{
    rnd[0] = h & 0xffffu;
    rnd[1] = h >> 16;
}

// x / 36 and 1 / x to within about half a unit in the last place, in three
// operations each (a product or the hardware reciprocal, then one
// residual-correction step with FMA), for the 16-bit formats' collisions,
// which are bound by instruction issue.  Inputs are positive densities
// (normal numbers), so no scaling for denormals or overflow is needed.
__device__ __forceinline__ float div36_fast(float x)
{
    constexpr float r = 1.0f / 36.0f;
    const float q = x * r;
    return fmaf(fmaf(-36.0f, q, x), r, q);
}
__device__ __forceinline__ float rcp_fast(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}

__device__ __forceinline__ int wrapi(int a, int n)
{
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

__device__ __forceinline__ int remap_xcd(int b, int n)
{
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of items so neighbouring strips share one L2.
    const int q = n >> 3, rem = n & 7;
    const int xcd = b & 7, slot = b >> 3;
    const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return start + slot;
}

// Barrier that orders LDS only: global loads of the next row stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace dev
}  // namespace lbm
