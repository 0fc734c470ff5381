// Shared device helpers of the Priori L+S library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace pls {

constexpr int kWave = 64;

// ---------------------------------------------------------------- complex float helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * (-i) and a * (+i)
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }

// 1 - w for a prior weight w = q / 255 (the threshold factor of the support-aware shrink),
// formed as (255 - q) / 255 so that a full weight gives exactly 0.  Written as 1 - q / 255,
// the compiler contracts it into fma(-q, 1/255, 1), whose unrounded product leaves -5.9e-8 at
// q = 255: a negative threshold and a negative term in the weighted l1 norm.
__device__ __forceinline__ float weight_complement(unsigned q) {
    return (float)(255u - q) * (1.0f / 255.0f);
}

// ---------------------------------------------------------------- compile-time trigonometry
// Taylor series after reduction to [-pi, pi]; used only in constant expressions, so the
// twiddle constants of the in-register DFTs are exact double values rounded to float.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_reduce(double x) {
    while (x > kPi) x -= 2 * kPi;
    while (x < -kPi) x += 2 * kPi;
    return x;
}
constexpr double cx_sin(double x) {
    x = cx_reduce(x);
    double term = x, sum = x;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double cx_cos(double x) {
    x = cx_reduce(x);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n - 1) * (2.0 * n));
        sum += term;
    }
    return sum;
}

// v * exp(-+ 2 pi i NUM / DEN): the forward DFT uses the minus sign, the inverse the plus.
template <int NUM, int DEN, bool INV>
__device__ __forceinline__ float2 ctw(float2 v) {
    constexpr int n = ((NUM % DEN) + DEN) % DEN;
    if constexpr (n == 0) {
        return v;
    } else if constexpr (2 * n == DEN) {
        return make_float2(-v.x, -v.y);
    } else if constexpr (4 * n == DEN) {
        return INV ? cmul_pi(v) : cmul_mi(v);
    } else if constexpr (4 * n == 3 * DEN) {
        return INV ? cmul_mi(v) : cmul_pi(v);
    } else {
        constexpr double ang = 2.0 * kPi * n / DEN;
        constexpr float c = (float)cx_cos(ang);
        constexpr float s = INV ? (float)cx_sin(ang) : (float)(-cx_sin(ang));
        return make_float2(fmaf(v.x, c, -v.y * s), fmaf(v.x, s, v.y * c));
    }
}

// ---------------------------------------------------------------- static for
template <int... Is, class F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F&& f) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(std::make_integer_sequence<int, N>{}, static_cast<F&&>(f));
}

// ---------------------------------------------------------------- deterministic block sums
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum of `v` over the block in a fixed order; result valid in every thread.
// `red` must hold >= (blockDim.x / 64) doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) s += red[i];
    return s;
}

}  // namespace pls
