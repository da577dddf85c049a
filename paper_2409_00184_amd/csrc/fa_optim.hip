// One Adam step on the control points of a gradient-based fit (the
// least-squares fit of the lattice to the block's samples that the
// model(NCP, degree) step of Alg. 1, Sec. 4.2.1, solves; its gradient is
// fa_decode_backward of the scaled residual).  Adam (Kingma and Ba, 2015)
// with bias-corrected moments, in the form PyTorch's Adam uses:
//     m = m + (1 - b1) (g - m),  v = b2 v + (1 - b2) g^2,
//     p = p - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps),
// g = grad + weight_decay p.  The step count lives in device memory so that
// a captured graph advances it on every replay: a one-thread kernel moves t
// to t + 1 and stores the two bias corrections, then the update kernel
// streams the arrays once (16-byte accesses when every array is aligned).
// The fit's loss, the mean of the squared residuals, comes from the
// per-block FP64 sums of squares in one single-workgroup launch.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

// state[0] = t, state[1] = 1 - b1^t, state[2] = sqrt(1 - b2^t)
__global__ void adam_count_kernel(float *state, float beta1, float beta2) {
    const float t = state[0] + 1.0f;
    state[0] = t;
    state[1] = 1.0f - powf(beta1, t);
    state[2] = sqrtf(1.0f - powf(beta2, t));
}

struct AdamArgs {
    float *p;
    const float *g;
    float *m, *v;
    int64_t n;
    float lr, beta1, beta2, eps, wd;
    const float *state;
};

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, const AdamArgs &a,
                                         float step_size, float bc2s) {
    if (a.wd != 0.0f) g = fmaf(a.wd, p, g);
    m = fmaf(1.0f - a.beta1, g - m, m);
    v = fmaf(1.0f - a.beta2, g * g, a.beta2 * v);
    const float denom = sqrtf(v) / bc2s + a.eps;
    p = p - step_size * (m / denom);
}

template <bool VEC>
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const float step_size = a.lr / a.state[1];
    const float bc2s = a.state[2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VEC) {
        const int64_t n4 = a.n / 4;
        for (int64_t i = i0; i < n4; i += stride) {
            float4 p = reinterpret_cast<const float4 *>(a.p)[i];
            const float4 g = reinterpret_cast<const float4 *>(a.g)[i];
            float4 m = reinterpret_cast<const float4 *>(a.m)[i];
            float4 v = reinterpret_cast<const float4 *>(a.v)[i];
            adam_one(p.x, g.x, m.x, v.x, a, step_size, bc2s);
            adam_one(p.y, g.y, m.y, v.y, a, step_size, bc2s);
            adam_one(p.z, g.z, m.z, v.z, a, step_size, bc2s);
            adam_one(p.w, g.w, m.w, v.w, a, step_size, bc2s);
            reinterpret_cast<float4 *>(a.p)[i] = p;
            reinterpret_cast<float4 *>(a.m)[i] = m;
            reinterpret_cast<float4 *>(a.v)[i] = v;
        }
        for (int64_t i = 4 * n4 + i0; i < a.n; i += stride)
            adam_one(a.p[i], a.g[i], a.m[i], a.v[i], a, step_size, bc2s);
    } else {
        for (int64_t i = i0; i < a.n; i += stride)
            adam_one(a.p[i], a.g[i], a.m[i], a.v[i], a, step_size, bc2s);
    }
}

// loss[0] = (float)(sum_b sumsq[b] / count): thread t adds blocks t, t + 256,
// ... in order, then the threads' sums meet in a fixed binary tree, so the
// result does not depend on timing.
__global__ __launch_bounds__(256) void mse_loss_kernel(const double *sumsq, int n, double count,
                                                       float *loss) {
    __shared__ double part[256];
    double t = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) t += sumsq[b];
    part[threadIdx.x] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(part[0] / count);
}

}  // namespace

hipError_t launch_mse_loss(const double *sumsq, int nblocks, double count, float *loss,
                           hipStream_t s) {
    hipLaunchKernelGGL(mse_loss_kernel, dim3(1), dim3(256), 0, s, sumsq, nblocks, count, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *param, const float *grad, float *exp_avg, float *exp_avg_sq,
                       int64_t n, float lr, float beta1, float beta2, float eps, float wd,
                       float *state, hipStream_t s) {
    hipLaunchKernelGGL(adam_count_kernel, dim3(1), dim3(1), 0, s, state, beta1, beta2);
    if (n == 0) return hipGetLastError();
    const AdamArgs a{param, grad, exp_avg, exp_avg_sq, n, lr, beta1, beta2, eps, wd, state};
    const auto al = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    const bool vec = al(param) && al(grad) && al(exp_avg) && al(exp_avg_sq);
    const int64_t work = vec ? (n + 3) / 4 : n;
    const int grid = (int)std::min<int64_t>((work + 255) / 256, 2048);
    if (vec) hipLaunchKernelGGL(adam_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(adam_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fa
