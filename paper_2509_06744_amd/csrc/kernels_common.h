// Device-side helpers shared by kernels: BF16 storage and element loads.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace chf {

// BF16 held as raw 16-bit patterns (the upper half of an IEEE binary32).
struct bf16_t {
    uint16_t bits;
};

// Round a binary32 value to BF16, nearest-even (finite inputs).
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_bits_to_f32(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

template <typename TO>
__device__ inline TO load_as(const double* p) { return (TO)(*p); }
template <typename TO>
__device__ inline TO load_as(const float* p) { return (TO)(*p); }
template <typename TO>
__device__ inline TO load_as(const bf16_t* p) { return (TO)bf16_bits_to_f32(p->bits); }

template <typename T>
__device__ inline void store_from_f64(T* p, double v);
template <>
__device__ inline void store_from_f64<double>(double* p, double v) { *p = v; }
template <>
__device__ inline void store_from_f64<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ inline void store_from_f64<bf16_t>(bf16_t* p, double v) {
    p->bits = f32_to_bf16_bits((float)v);
}

}  // namespace chf
