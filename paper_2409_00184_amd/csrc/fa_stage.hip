// Staging gather (Alg. 2, memory copy step): one workgroup per staged
// micro-model reads its cache slot straight from page-locked, mapped host
// memory over the host link and writes the packed device batch.  The
// table entry is read once per workgroup into LDS (host reads are not
// cached, so every lane reading it would be a separate transfer); the
// lattice moves as 16-byte vectors (slots and lattice destinations are
// 16-byte aligned).
#include "fa_internal.hpp"

namespace fa {
namespace {

__global__ __launch_bounds__(256) void stage_gather_kernel(const StageEntry *table, int n,
                                                           const float *slots,
                                                           fa_block *dev_blocks,
                                                           float *dev_knots, float *dev_ctrl) {
    __shared__ StageEntry e;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        if (threadIdx.x < (int)(sizeof(StageEntry) / 4))
            reinterpret_cast<uint32_t *>(&e)[threadIdx.x] =
                reinterpret_cast<const uint32_t *>(table + i)[threadIdx.x];
        __syncthreads();
        const float *src = slots + e.slot_off;
        for (int k = threadIdx.x; k < e.kl; k += blockDim.x) dev_knots[e.kdst + k] = src[k];
        const float4 *s4 = reinterpret_cast<const float4 *>(src + e.koff);
        float4 *d4 = reinterpret_cast<float4 *>(dev_ctrl + e.cdst);
        const int64_t n4 = e.cl / 4;
        for (int64_t k = threadIdx.x; k < n4; k += blockDim.x) d4[k] = s4[k];
        for (int64_t k = n4 * 4 + threadIdx.x; k < e.cl; k += blockDim.x)
            dev_ctrl[e.cdst + k] = src[e.koff + k];
        if (threadIdx.x == 0) dev_blocks[e.dst] = e.desc;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_stage_gather(const StageEntry *table, int n, const float *slots,
                               fa_block *dev_blocks, float *dev_knots, float *dev_ctrl,
                               hipStream_t s) {
    const int grid = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(stage_gather_kernel, dim3(grid), dim3(256), 0, s, table, n, slots,
                       dev_blocks, dev_knots, dev_ctrl);
    return hipGetLastError();
}

}  // namespace fa
