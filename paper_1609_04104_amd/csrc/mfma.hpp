// Matrix-core (MFMA) helpers for gfx950.
#pragma once
#include <hip/hip_runtime.h>

namespace tsl {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16x16x4 FP32 step, D += A B with A 16x4 and B 4x16.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; element i of lane l of D is
// D[4 (l / 16) + i][l % 16].
__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One 32x32x2 FP32 step, D += A B with A 32x2 and B 2x32.  Lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; element v of lane l of D is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
__device__ __forceinline__ f32x16 mfma_32x32x2(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// One 16x16x4 FP64 step (products and sums in FP64).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] as in the FP32 step, but the output
// rows interleave differently: element i of lane l of D is D[4 i + l / 16][l % 16].
__device__ __forceinline__ f64x4 mfma_16x16x4_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of D held by element v of lane l in the 32x32 layout above.
__device__ __forceinline__ int mfma32_row(int v, int lane) { return 8 * (v / 4) + 4 * (lane / 32) + v % 4; }

}  // namespace tsl

namespace tsl {

// BF16 matrix-core steps with FP32 accumulation (gfx950).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// One 32x32x16 step: lane l supplies A[l % 32][8 (l / 32) + j] and
// B[8 (l / 32) + j][l % 32] for j < 8; D has the layout of the 32x32x2 FP32 step.
__device__ __forceinline__ f32x16 mfma_32x32x16_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// One 16x16x16 step: lane l supplies A[l % 16][4 (l / 16) + j] and
// B[4 (l / 16) + j][l % 16] for j < 4; D has the layout of the 16x16x4 FP32 step.
__device__ __forceinline__ f32x4 mfma_16x16x16_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c,
                                                     0, 0, 0);
}

// Synthesis precision (tsl_opts.synth_bf16): FP32 operands; BF16 operands
// (rounded to nearest even); or split BF16, x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (x - hi is exact in FP32), a product taken as
// hi_a hi_b + hi_a lo_b + lo_a hi_b (three BF16 steps, about 16 significant bits).
enum : int { SYN_FP32 = 0, SYN_BF16 = 1, SYN_BF16X3 = 2 };
struct BfPair {
    __bf16 hi, lo;
};
__device__ __forceinline__ BfPair split_bf16(float x) {
    const __bf16 hi = static_cast<__bf16>(x);
    return BfPair{hi, static_cast<__bf16>(x - static_cast<float>(hi))};
}

}  // namespace tsl
