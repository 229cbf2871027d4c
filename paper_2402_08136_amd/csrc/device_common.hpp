// Small device helpers shared by the sweep kernels and the batched executor.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hhlsv {

template <typename R> struct V2;
template <> struct V2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct V2<float> { typedef float type __attribute__((ext_vector_type(2))); };

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// Fused multiply-add in the operands' own precision (__builtin_fma is the
// double one: on float operands it would widen every product to FP64).
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += m * v (complex), as four fused multiply-adds.
template <typename C>
__device__ __forceinline__ void cmac(C &acc, const C m, const C v)
{
    acc.x = fmadd(m.x, v.x, acc.x);
    acc.x = fmadd(-m.y, v.y, acc.x);
    acc.y = fmadd(m.x, v.y, acc.y);
    acc.y = fmadd(m.y, v.x, acc.y);
}

template <typename C>
__device__ __forceinline__ C cmul(const C m, const C v)
{
    C y;
    y.x = m.x * v.x - m.y * v.y;
    y.y = m.x * v.y + m.y * v.x;
    return y;
}

// Offset the (uniform) matrix pointer by a zero the optimiser cannot see
// through, so loads of the matrix are not hoisted out of a loop (which would
// pin the whole gate matrix in registers).  The pointer keeps its global
// address space and stays uniform, so the loads remain scalar.
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p)
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int p)
{
    const uint64_t lo = x & ((uint64_t(1) << p) - 1);
    return ((x >> p) << (p + 1)) | lo;
}

__device__ __forceinline__ uint32_t insert_zero32(uint32_t x, int p)
{
    const uint32_t lo = x & ((1u << p) - 1);
    return ((x >> p) << (p + 1)) | lo;
}

}  // namespace hhlsv
