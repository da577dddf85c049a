// Per-block max-abs scaling and rounding to BF16/FP16 (row a4).
//
// s_b = max |P_b| (1 for an all-zero lattice); the stored lattice is
// RNE(P_b / s_b), so every stored magnitude is <= 1 and the low-precision
// decode multiplies by s_b in FP32.  One workgroup per block.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
    _Float16 h = (_Float16)x;  // v_cvt_f16_f32, round to nearest even
    uint16_t r;
    __builtin_memcpy(&r, &h, 2);
    return r;
}

__global__ __launch_bounds__(256) void quantize_kernel(fa_block *blocks, const float *ctrl,
                                                       int dtype, uint16_t *out) {
    __shared__ float red[256];
    fa_block &B = blocks[blockIdx.x];
    const int64_t cnt = (int64_t)B.ncp[0] * B.ncp[1] * B.ncp[2];
    const float *src = ctrl + B.ctrl_off;
    float m = 0.0f;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) m = fmaxf(m, fabsf(src[e]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const float s = red[0] > 0.0f ? red[0] : 1.0f;
    const float inv = 1.0f / s;
    uint16_t *dst = out + B.ctrl_off;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        // P / s: multiply by the correctly rounded reciprocal, then clamp the
        // rare 1 + ulp to 1 so |stored| <= 1 holds exactly
        float q = src[e] * inv;
        q = fminf(fmaxf(q, -1.0f), 1.0f);
        dst[e] = dtype == FA_BF16 ? f32_to_bf16_rne(q) : f32_to_f16_rne(q);
    }
    if (threadIdx.x == 0) B.scale = s;
}

}  // namespace

hipError_t launch_quantize(fa_block *blocks, int nblocks, const float *ctrl, int dtype,
                           void *out, hipStream_t s) {
    hipLaunchKernelGGL(quantize_kernel, dim3(nblocks), dim3(256), 0, s, blocks, ctrl, dtype,
                       static_cast<uint16_t *>(out));
    return hipGetLastError();
}

}  // namespace fa
