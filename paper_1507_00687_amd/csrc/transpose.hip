// Out-of-place transposition (FP32 / FP64), used by the backward pass for G^T and the results.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.h"

namespace fastmm {
namespace {

// out (C x R, row-major ldo) = in^T where in is R x C row-major (ldi); 32x32 tiles via LDS
// (a padded column so both the row reads and the column writes are conflict-free).
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *in, int64_t ldi, int64_t R, int64_t C, T *out,
                                                        int64_t ldo) {
    __shared__ T tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
        const int64_t r = r0 + ty + i, c = c0 + tx;
        if (r < R && c < C) tile[ty + i][tx] = in[r * ldi + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
        const int64_t c = c0 + ty + i, r = r0 + tx;
        if (r < R && c < C) out[c * ldo + r] = tile[tx][ty + i];
    }
}

template <typename T>
hipError_t transpose_go(const T *in, int64_t ldi, int64_t R, int64_t C, T *out, int64_t ldo, hipStream_t s) {
    if (R <= 0 || C <= 0) return hipSuccess;
    if ((C + 31) / 32 > 0x7fffffffLL || (R + 31) / 32 > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, in, ldi, R, C, out, ldo);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose(Elem e, const void *in, int64_t ldi, int64_t R, int64_t C, void *out, int64_t ldo,
                            hipStream_t s) {
    if (e == Elem::F32) return transpose_go((const float *)in, ldi, R, C, (float *)out, ldo, s);
    return transpose_go((const double *)in, ldi, R, C, (double *)out, ldo, s);
}

}  // namespace fastmm
