// Storage types and conversions used by the PW advection kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pw {

// bfloat16 stored as its raw 16 bits; FP16 as the compiler's _Float16;
// 16- and 32-bit fixed point as signed integers (value = stored / scale).
struct bf16_t {
    uint16_t bits;
};
using f16_t = _Float16;
struct fx16_t {
    int16_t v;
};
struct fx32_t {
    int32_t v;
};

// Device memory seen through the global address space.  Loads and stores
// through such a pointer are global_* instructions, which count against
// vmcnt only.  Through a generic pointer that the compiler cannot prove
// global -- one read from device memory, as a batched record's fields are --
// they are flat_* instructions, which also count against lgkmcnt, so every
// wait for an LDS read would also wait for all memory loads in flight.
template <typename T> using global_ptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ global_ptr<T> as_global(T* p) { return (global_ptr<T>)p; }

// ---------------------------------------------------------------------------
// compute type of each storage type
// ---------------------------------------------------------------------------
// 32-bit fixed point computes in FP64: every int32 converts exactly, and FP32
// would drop the low 8 bits of the stored values.
template <typename ST> struct compute_of { using type = float; };
template <> struct compute_of<double> { using type = double; };
template <> struct compute_of<fx32_t> { using type = double; };

// Fixed-point storage: every stored value is a finite integer, and a zero of
// either sign rounds to the stored integer 0.
template <typename ST> inline constexpr bool is_fixed_point = false;
template <> inline constexpr bool is_fixed_point<fx16_t> = true;
template <> inline constexpr bool is_fixed_point<fx32_t> = true;

// ---------------------------------------------------------------------------
// storage -> compute
// ---------------------------------------------------------------------------
__device__ __forceinline__ double to_compute(double x) { return x; }
__device__ __forceinline__ float to_compute(float x) { return x; }
__device__ __forceinline__ float to_compute(f16_t x) { return static_cast<float>(x); }
__device__ __forceinline__ float to_compute(fx16_t x) { return static_cast<float>(x.v); }
__device__ __forceinline__ double to_compute(fx32_t x) { return static_cast<double>(x.v); }
__device__ __forceinline__ float to_compute(bf16_t x) {
    return __uint_as_float(static_cast<uint32_t>(x.bits) << 16);
}

// ---------------------------------------------------------------------------
// compute -> storage (round to nearest even)
// ---------------------------------------------------------------------------
template <typename ST> __device__ __forceinline__ ST from_compute(typename compute_of<ST>::type x);
template <> __device__ __forceinline__ double from_compute<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_compute<float>(float x) { return x; }
template <> __device__ __forceinline__ f16_t from_compute<f16_t>(float x) { return static_cast<f16_t>(x); }
// round to nearest even, saturate to the int16 range (NaN becomes -32768)
__device__ __forceinline__ int fx16_round(float x) {
    return static_cast<int>(__builtin_fminf(__builtin_fmaxf(__builtin_rintf(x), -32768.0f), 32767.0f));
}
template <> __device__ __forceinline__ fx16_t from_compute<fx16_t>(float x) {
    fx16_t y;
    y.v = static_cast<int16_t>(fx16_round(x));
    return y;
}
// round to nearest even, saturate to the int32 range (NaN becomes -2^31)
template <> __device__ __forceinline__ fx32_t from_compute<fx32_t>(double x) {
    const double r = __builtin_fmin(__builtin_fmax(__builtin_rint(x), -2147483648.0), 2147483647.0);
    fx32_t y;
    y.v = static_cast<int32_t>(r);
    return y;
}
template <> __device__ __forceinline__ bf16_t from_compute<bf16_t>(float x) {
    const __bf16 h = static_cast<__bf16>(x);   // v_cvt_pk_bf16_f32: round to nearest even
    bf16_t r;
    __builtin_memcpy(&r.bits, &h, 2);
    return r;
}

}  // namespace pw
