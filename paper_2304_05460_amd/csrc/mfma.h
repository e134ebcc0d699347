// MFMA 16x16x4 (FP32 and FP64) on gfx950, wave64.  Operand layout (checked
// on the device): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element i of lane l is C[4 (l / 16) + i][l % 16] for FP32 and
// C[l / 16 + 4 i][l % 16] for FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace afn {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    using acc_t = floatx4;
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <>
struct Mfma<double> {
    using acc_t = doublex4;
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

}  // namespace afn
