// Storage element types of the device state and their conversions.
//
// The state is kept as deviations from rest (see moment_math.hpp), one
// contiguous array per field.  FP64 storage computes in FP64; FP32, FP16 and
// BF16 storage compute in FP32.  16-bit conversions round to nearest even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct bf16 {
    uint16_t bits;
};
using f16 = _Float16;

template <class S>
struct Store;

template <>
struct Store<double> {
    using real = double;
    __device__ __forceinline__ static double load(double v) { return v; }
    __device__ __forceinline__ static double make(double v) { return v; }
};

template <>
struct Store<float> {
    using real = float;
    __device__ __forceinline__ static float load(float v) { return v; }
    __device__ __forceinline__ static float make(float v) { return v; }
};

template <>
struct Store<f16> {
    using real = float;
    __device__ __forceinline__ static float load(f16 v) { return (float)v; }
    __device__ __forceinline__ static f16 make(float v) { return (f16)v; }
};

template <>
struct Store<bf16> {
    using real = float;
    __device__ __forceinline__ static float load(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
    // The hardware conversion of gfx950 (round to nearest even, NaN stays NaN).
    __device__ __forceinline__ static bf16 make(float v)
    {
        bf16 r;
        r.bits = __builtin_bit_cast(uint16_t, (__bf16)v);
        return r;
    }
};

} // namespace lbm
