// Device helpers shared by the search kernels and the ranker kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spl_internal.h"

#pragma clang fp contract(off)

namespace spl {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Read-only tables (delays) are read through the constant address space so that
// wave-uniform indices become scalar loads.
typedef __attribute__((address_space(4))) const int32_t cint32;
__device__ __forceinline__ const cint32 *as_const(const int32_t *p) { return (const cint32 *)p; }
// Input blocks are read through the global address space (global_load, not flat_load).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const uint8_t gu8;
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
typedef __attribute__((address_space(1))) const uint32_t gu32;
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Correctly rounded (nearest-even) conversion of the unsigned 128-bit integer hi:lo.
__device__ inline double u128_to_f64(uint64_t hi, uint64_t lo) {
    if (hi == 0) return (double)lo;
    const int lz = __clzll((long long)hi);
    uint64_t m = lz ? ((hi << lz) | (lo >> (64 - lz))) : hi;
    const uint64_t rest = lz ? (lo << lz) : lo;
    m |= (rest != 0) ? 1ull : 0ull;   // sticky bit below the rounding position
    return ldexp((double)m, 64 - lz);
}

// mean and sigma of a segment from exact moments: V = n*S2 - S1^2 (128-bit),
// mu = S1/n, sigma = sqrt(V)/n, sigma = 0 for V = 0.
__device__ inline void mu_sigma(int64_t n, int64_t S1, int64_t S2, double &mu, double &sigma) {
    const uint64_t un = (uint64_t)n, u2 = (uint64_t)S2, u1 = (uint64_t)S1;
    const uint64_t a_lo = un * u2, a_hi = __umul64hi(un, u2);
    const uint64_t b_lo = u1 * u1, b_hi = __umul64hi(u1, u1);
    const uint64_t v_lo = a_lo - b_lo;
    const uint64_t v_hi = a_hi - b_hi - (a_lo < b_lo ? 1ull : 0ull);
    mu = (double)S1 / (double)n;
    sigma = (v_hi == 0 && v_lo == 0) ? 0.0 : sqrt(u128_to_f64(v_hi, v_lo)) / (double)n;
}

__device__ __forceinline__ double snr_of(int64_t B, int w, double mu, double sigma) {
    return ((double)B - (double)w * mu) / (sigma * sqrt((double)w));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Exclusive scan over the 256 threads of a workgroup; *total gets the sum.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *total, T *sh) {
    const int lane = lane_id(), wave = wave_id();
    T x = wave_inclusive_scan(v);
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        T s = sh[w];
        if (w < wave) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}


}  // namespace spl
