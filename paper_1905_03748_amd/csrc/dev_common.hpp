// Device helpers: 16/32-bit storage loads and stores, dtype dispatch, deterministic reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ct_internal.hpp"

namespace ct {

// bfloat16 storage (upper 16 bits of an IEEE binary32)
struct bf16s {
    uint16_t v;
};
using f16s = _Float16;

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(f16s x) { return (float)x; }
__device__ __forceinline__ float to_f(bf16s x) { return __uint_as_float(((uint32_t)x.v) << 16); }

template <typename T>
__device__ __forceinline__ T from_f(float f);
template <>
__device__ __forceinline__ float from_f<float>(float f) { return f; }
template <>
__device__ __forceinline__ f16s from_f<f16s>(float f) { return (f16s)f; }
template <>
__device__ __forceinline__ bf16s from_f<bf16s>(float f) {
    uint32_t u = __float_as_uint(f);
    bf16s r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.v = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);      // round to nearest, ties to even
        r.v = (uint16_t)(u >> 16);
    }
    return r;
}

template <typename T>
__device__ __forceinline__ float ldf(const T *p, int64_t i) {
    return to_f(p[i]);
}

// FP64 values (conversion and inner products only): widened exactly, narrowed to FP32 with one
// rounding and to the 16-bit types through FP32
__device__ __forceinline__ double to_d(double x) { return x; }
template <typename T>
__device__ __forceinline__ double to_d(T x) { return (double)to_f(x); }
template <typename TD>
__device__ __forceinline__ TD from_d(double x) {
    // the FP32 value is kept (the compiler would otherwise fold the two narrowings to FP16 into
    // one), so both 16-bit types are rounded from the FP32 rounding
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return from_f<TD>(f);
}
template <>
__device__ __forceinline__ float from_d<float>(double x) { return (float)x; }
template <>
__device__ __forceinline__ double from_d<double>(double x) { return x; }

// Buffer loads (CDNA raw buffer instructions with 32-bit byte offsets).  The hardware range check
// returns 0 for offsets at or beyond the resource size (negative offsets wrap to huge unsigned
// values), which the backprojectors use as the detector's zero padding; it also keeps addresses
// 32-bit.  Word 3 of the resource selects the 32-bit data format of the gfx9 family.
constexpr int BUF_WORD3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t proj_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, BUF_WORD3);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off, float *) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off, f16s *) {
    return (float)__builtin_bit_cast(f16s, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off, bf16s *) {
    return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)) << 16);
}

// Wave64 sum of a double, fixed butterfly order (bitwise repeatable).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum (blockDim.x multiple of 64, <= 1024); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) r += lds[i];
    __syncthreads();
    return r;
}

}  // namespace ct

// Dispatch a templated call on one storage type: DISPATCH1(dt, T, expr-using-T)
#define CT_DISPATCH1(dt, T, ...)                  \
    switch (dt) {                                 \
        case CT_F32: {                            \
            using T = float;                      \
            __VA_ARGS__;                          \
        } break;                                  \
        case CT_F16: {                            \
            using T = ::ct::f16s;                 \
            __VA_ARGS__;                          \
        } break;                                  \
        default: {                                \
            using T = ::ct::bf16s;                \
            __VA_ARGS__;                          \
        } break;                                  \
    }

#define CT_DISPATCH2(d1, T1, d2, T2, ...) CT_DISPATCH1(d1, T1, CT_DISPATCH1(d2, T2, __VA_ARGS__))

// The same over every type including FP64 (conversion and inner products)
#define CT_DISPATCH1_ANY(dt, T, ...)              \
    switch (dt) {                                 \
        case CT_F64: {                            \
            using T = double;                     \
            __VA_ARGS__;                          \
        } break;                                  \
        default:                                  \
            CT_DISPATCH1(dt, T, __VA_ARGS__);     \
            break;                                \
    }
