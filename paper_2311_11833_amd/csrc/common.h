// common.h -- device-side helpers and launch parameter blocks shared by the
// HIP kernels of libpsp (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace psp {

constexpr int kMaxK = 16;          // largest perturbation set per call

// Perturbation nodes and combination weights, passed by value.
struct EpsSet {
    int32_t K;
    double eps[kMaxK];
    double c[kMaxK];
};

// Reads eps[k] / c[k] with compile-time indices only: a run-time index into a
// by-value kernel argument would make the compiler copy it to scratch.
__device__ __forceinline__ double eps_at(const EpsSet& es, int k) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) v = (i == k) ? es.eps[i] : v;
    return v;
}
__device__ __forceinline__ double c_at(const EpsSet& es, int k) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) v = (i == k) ? es.c[i] : v;
    return v;
}

// The exact operation sequence matters (results are compared bit for bit
// with the CPU reference), so every multiply-add below is an explicit fma,
// the product eps*d is rounded before it is added, and division is IEEE
// division.  The library is built with -ffp-contract=off.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ bool bad_pivot(double p) { return p == 0.0 || !__builtin_isfinite(p); }

}  // namespace psp
