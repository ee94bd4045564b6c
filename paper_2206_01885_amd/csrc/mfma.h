// 16x16x4 matrix-core step per value type (FP64 v_mfma_f64_16x16x4f64,
// FP32 v_mfma_f32_16x16x4f32), shared by the apply sweeps and the blocked
// compression of the interpolative decompositions.
//
// Operand layout (both types): lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Result register r of lane l holds row row(r, l/16) of
// column l%16: 4r + l/16 (FP64) or 4(l/16) + r (FP32).
#pragma once

#include <hip/hip_runtime.h>

namespace h2 {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double4_t V;
    __device__ static V step(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __host__ __device__ static constexpr int row(int r, int k4) { return 4 * r + k4; }
};
template <>
struct Mfma<float> {
    typedef float4_t V;
    __device__ static V step(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __host__ __device__ static constexpr int row(int r, int k4) { return 4 * k4 + r; }
};

}  // namespace h2
