// Device helpers shared by the kernels: Philox4x32-10 normals, MFMA tile
// wrappers for gfx950, and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "msrs_internal.h"

namespace msrs {

// ---------------------------------------------------------------- Philox
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round,
// two 32x32->64 products of counter words 0 and 2 with the multipliers
// below; the key advances by the two Weyl constants before every round
// after the first.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

// Uniform in (0, 1]: (k + 1/2) 2^-53 with k = (a >> 5) 2^26 + (b >> 6).
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    const uint64_t k = ((uint64_t)(a >> 5) << 26) + (uint64_t)(b >> 6);
    return ((double)k + 0.5) * 0x1p-53;
}

// One standard normal for (node, sample, patch) under key seed: Box-Muller
// with the cosine branch.
__device__ __forceinline__ double philox_normal(uint64_t seed, uint32_t node, uint32_t sample, uint32_t patch) {
    const U4 r = philox4x32_10(U4{node, sample, patch, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = uniform53(r.x, r.y);
    const double u2 = uniform53(r.z, r.w);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// ---------------------------------------------------------------- MFMA
// 16x16x4 tiles (one wave): A is 16x4 with lane l holding A[l%16][l/16] and B
// is 4x16 with lane l holding B[l/16][l%16] for both types.  The accumulator
// rows differ (measured on gfx950): element t of lane l holds D[row][l%16]
// with row = 4*(l/16) + t for f32 and row = 4*t + l/16 for f64.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int t) { return 4 * t + (lane >> 4); }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int t) { return 4 * (lane >> 4) + t; }
};

// ---------------------------------------------------------------- reductions
// Sum over the 256 threads of a workgroup; all threads receive the result.
// red must hold kThreads doubles.  Deterministic (fixed tree order).
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Workgroup barrier that orders LDS only: outstanding global loads (software
// prefetches) stay in flight across it.  Valid where no thread reads global
// memory that another thread of the workgroup wrote in the same kernel.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void raise_flag(int32_t* flags, int which) {
    // sticky flag: every writer stores the same value, so a plain store suffices
    ((volatile int32_t*)flags)[which] = 1;
}

}  // namespace msrs
