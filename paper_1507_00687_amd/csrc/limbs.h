// bf16 / fp16 limbs of FP32 values and the MFMA products of limb fragments (gfx950), shared by
// the limb GEMM and the limb-plane formation.
#pragma once
#include <hip/hip_runtime.h>

namespace fastmm {
namespace {

typedef float g4v __attribute__((ext_vector_type(4)));
typedef float g16v __attribute__((ext_vector_type(16)));
typedef __bf16 gbf8 __attribute__((ext_vector_type(8)));
typedef _Float16 gh8 __attribute__((ext_vector_type(8)));
typedef short gs8 __attribute__((ext_vector_type(8)));

template <bool HALF>
struct LimbT;
template <>
struct LimbT<false> {
    __device__ static unsigned short split(float x, float &back) {
        const __bf16 h = (__bf16)x;  // round to nearest even
        back = (float)h;
        return __builtin_bit_cast(unsigned short, h);
    }
    // D(16x16) += A(16x32) B(32x16): lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
    // B[8(l/16) .. 8(l/16)+7][l%16]; accumulator element v of lane l is D[4(l/16)+v][l%16].
    __device__ static g4v mma(gs8 a, gs8 b, g4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(gbf8, a), __builtin_bit_cast(gbf8, b), c,
                                                       0, 0, 0);
    }
    // D(32x32) += A(32x16) B(16x32): lane l supplies A[l%32][8(l/32) .. 8(l/32)+7] and
    // B[8(l/32) .. 8(l/32)+7][l%32]; accumulator element v of lane l is
    // D[8(v/4) + 4(l/32) + v%4][l%32].
    __device__ static g16v mma32(gs8 a, gs8 b, g16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(gbf8, a), __builtin_bit_cast(gbf8, b), c,
                                                       0, 0, 0);
    }
};
template <>
struct LimbT<true> {
    __device__ static unsigned short split(float x, float &back) {
        const _Float16 h = (_Float16)x;
        back = (float)h;
        return __builtin_bit_cast(unsigned short, h);
    }
    __device__ static g4v mma(gs8 a, gs8 b, g4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(gh8, a), __builtin_bit_cast(gh8, b), c, 0, 0,
                                                      0);
    }
    __device__ static g16v mma32(gs8 a, gs8 b, g16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(gh8, a), __builtin_bit_cast(gh8, b), c, 0, 0,
                                                      0);
    }
};

}  // namespace
}  // namespace fastmm
