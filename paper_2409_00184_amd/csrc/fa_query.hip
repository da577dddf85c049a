// Point query over a tiled domain on gfx950 (rows a1-a6 for ray samples).
//
// Alg. 4 evaluates valueMicroModel and gradientMicroModel at every ray
// sample.  One lane per sample, grid-stride over the samples (which arrive
// ray-major, so the lanes of a wave walk one ray and mostly share a block):
//   a1  block lookup in FP32 (one rounding per operation, see fa.h);
//   a2  span per axis: for knots flagged uniform, a guess p + floor(u(n-p))
//       corrected against the stored knots, else a binary search;
//   a3  FP32 basis and first derivative (triangular de Boor form);
//   a4  the (p+1)^3 control window, z-runs of p+1 consecutive points;
//   a5  separable contraction of the window: z, then y, then x;
//   a6  chain rule d/dx = r d/du and one 16-byte store per sample.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

template <int P>
__device__ __forceinline__ int axis_span(int n, const float *t, float u, bool uniform) {
    if (uniform) return span_from_guess(n, P, t, u, P + (int)(u * float(n - P)));
    return span_search(n, P, t, u);
}

template <int P>
__device__ __forceinline__ float4 query_block(const QueryLaunch &a, const fa_block &B,
                                              const float (&uu)[3]) {
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const uint32_t fl = B.flags;
    const float *tx = a.knots + B.knot_off;
    const float *ty = tx + nx + P + 1;
    const float *tz = ty + ny + P + 1;
    const int sx = axis_span<P>(nx, tx, uu[0], fl & FA_FLAG_UNIFORM_X);
    const int sy = axis_span<P>(ny, ty, uu[1], fl & FA_FLAG_UNIFORM_Y);
    const int sz = axis_span<P>(nz, tz, uu[2], fl & FA_FLAG_UNIFORM_Z);
    float xB[P + 1], xD[P + 1], yB[P + 1], yD[P + 1], zB[P + 1], zD[P + 1];
    basis_ders<P>(tx, sx, uu[0], xB, xD);
    basis_ders<P>(ty, sy, uu[1], yB, yD);
    basis_ders<P>(tz, sz, uu[2], zB, zD);
    const int64_t base = B.ctrl_off + ((int64_t)(sx - P) * ny + (sy - P)) * nz + (sz - P);
    const float scale = B.scale;
    float f = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        float uBB = 0.0f, uDB = 0.0f, uBD = 0.0f;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            const int64_t row = base + ((int64_t)i * ny + j) * nz;
            float c[P + 1];
            if (a.dtype == FA_F32) {
                const float *cp = static_cast<const float *>(a.ctrl) + row;
#pragma unroll
                for (int k = 0; k <= P; ++k) c[k] = cp[k];
            } else {
#pragma unroll
                for (int k = 0; k <= P; ++k) c[k] = load_ctrl(a.ctrl, a.dtype, row + k, scale);
            }
            float tB = 0.0f, tD = 0.0f;
#pragma unroll
            for (int k = 0; k <= P; ++k) {
                tB = fmaf(zB[k], c[k], tB);
                tD = fmaf(zD[k], c[k], tD);
            }
            uBB = fmaf(yB[j], tB, uBB);
            uDB = fmaf(yD[j], tB, uDB);
            uBD = fmaf(yB[j], tD, uBD);
        }
        f = fmaf(xB[i], uBB, f);
        fx = fmaf(xD[i], uBB, fx);
        fy = fmaf(xB[i], uDB, fy);
        fz = fmaf(xB[i], uBD, fz);
    }
    return make_float4(f, fx, fy, fz);
}

// Block lookup in FP32 with no fused operations: the block index is an
// integer decided by floating point and must come out as documented.
__device__ __forceinline__ int lookup_axis(float x, float origin, float r, int nb, float &u) {
#pragma clang fp contract(off)
    float g = (x - origin) * r;
    const float top = float(nb);
    if (!(g >= 0.0f)) g = 0.0f;  // also sends NaN to 0
    if (g > top) g = top;
    int b = (int)floorf(g);
    if (b > nb - 1) b = nb - 1;
    u = g - float(b);
    return b;
}

__global__ __launch_bounds__(256) void query_kernel(QueryLaunch a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.n; q += stride) {
        const float x = a.xyz[3 * q], y = a.xyz[3 * q + 1], z = a.xyz[3 * q + 2];
        float uu[3];
        const int bx = lookup_axis(x, a.origin[0], a.rscale[0], a.nb[0], uu[0]);
        const int by = lookup_axis(y, a.origin[1], a.rscale[1], a.nb[1], uu[1]);
        const int bz = lookup_axis(z, a.origin[2], a.rscale[2], a.nb[2], uu[2]);
        const int blk = a.block_of_cell[(bx * a.nb[1] + by) * a.nb[2] + bz];
        float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (blk >= 0 && blk < a.nblocks) {  // anything else is an empty cell
            const fa_block &B = a.blocks[blk];
            const int p = B.degree[0];
            if (p == 3) r = query_block<3>(a, B, uu);
            else if (p == 2) r = query_block<2>(a, B, uu);
            else r = query_block<1>(a, B, uu);
            r.y *= a.rscale[0];
            r.z *= a.rscale[1];
            r.w *= a.rscale[2];
        }
        if (!(a.mask & 1u)) r.x = 0.0f;
        if (!(a.mask & 2u)) r.y = 0.0f;
        if (!(a.mask & 4u)) r.z = 0.0f;
        if (!(a.mask & 8u)) r.w = 0.0f;
        const f32x4 rv = {r.x, r.y, r.z, r.w};
        __builtin_nontemporal_store(rv, reinterpret_cast<f32x4 *>(a.out) + q);
    }
}

}  // namespace

hipError_t launch_query(const QueryLaunch &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    int64_t waves = (a.n + 255) / 256;
    const int64_t cap = 256 * 64;  // grid-stride beyond 64 workgroups per CU
    const int grid = (int)(waves < cap ? waves : cap);
    hipLaunchKernelGGL(query_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fa
