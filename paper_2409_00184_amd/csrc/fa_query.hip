// Point query over a tiled domain on gfx950 (rows a1-a6 for ray samples).
//
// Alg. 4 evaluates valueMicroModel and gradientMicroModel at every ray
// sample.  One lane per sample, grid-stride over the samples (which arrive
// ray-major, so the 64 lanes of a wave walk one ray and mostly share a
// micro-model):
//   a1  block lookup in FP32 (one rounding per operation, see fa.h); when
//       every lane of the wave is in the same block the descriptor is read
//       once with scalar loads;
//   a2  span per axis: for knots flagged uniform, the guess p + floor(u(n-p))
//       is corrected by one comparison each way against the stored knots,
//       which arrive with the whole knot window in two vector loads; other
//       knot vectors take a binary search;
//   a3  FP32 basis and first derivative on the register knot window;
//   a4  the (p+1)^3 control window as (p+1)^2 vector loads of p+1
//       consecutive z points (served by L1/L2: neighbouring lanes overlap);
//   a5  separable contraction of the window: z, then y, then x;
//   a6  chain rule d/dx = r d/du and one 16-byte store per sample.
#include "fa_eval.hpp"

namespace fa {
namespace {

// One sample for every lane of the wave; `live` false makes the lane an
// empty sample that still takes part in the wave-wide votes.
template <int DT>
__device__ __forceinline__ void query_sample(const QueryLaunch &a, int64_t q, bool live) {
    float x = 0.0f, y = 0.0f, z = 0.0f;
    if (live) {
        // streamed once: non-temporal, so positions do not displace the
        // lattice lines neighbouring samples and rays reuse from L2
        const float *pp = a.xyz + 3 * q;
        x = __builtin_nontemporal_load(pp);
        y = __builtin_nontemporal_load(pp + 1);
        z = __builtin_nontemporal_load(pp + 2);
    }
    float4 r = eval_point<DT>(a, x, y, z, live);
    if (!live) return;
    if (!(a.mask & 1u)) r.x = 0.0f;
    if (!(a.mask & 2u)) r.y = 0.0f;
    if (!(a.mask & 4u)) r.z = 0.0f;
    if (!(a.mask & 8u)) r.w = 0.0f;
    const f32x4 rv = {r.x, r.y, r.z, r.w};
    __builtin_nontemporal_store(rv, reinterpret_cast<f32x4 *>(a.out) + q);
}

// Flat list: lanes take consecutive samples.
template <int DT>
__global__ __launch_bounds__(256) void query_kernel(QueryLaunch a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane runs the same trip count, so the wave-wide votes see all
    // 64 lanes (lanes past the end take part as empty samples)
    const int64_t n_round = (a.n + blockDim.x - 1) / blockDim.x * blockDim.x;
    const int wg = xcd_order(blockIdx.x, gridDim.x);
    for (int64_t q = (int64_t)wg * blockDim.x + threadIdx.x; q < n_round; q += stride)
        query_sample<DT>(a, q, q < a.n);
}

// Ray-structured: a workgroup of kTX x kTY waves (2 x 4 measured fastest of
// 2x2, 2x4, 4x2, 4x4, 8x2 on the 1920x1080x512 camera) owns a tile of adjacent
// rays; wave q walks one ray of the tile, 64 consecutive samples per step
// (coalesced positions and outputs), and the waves advance in lockstep so
// that, at each step, they gather from the same micro-models and knot spans
// and reuse each other's lattice lines in the CU's L1.
#ifndef FA_RAY_TX
#define FA_RAY_TX 2
#endif
#ifndef FA_RAY_TY
#define FA_RAY_TY 4
#endif
#ifndef FA_RAY_SYNC
#define FA_RAY_SYNC 1
#endif
constexpr int kTX = FA_RAY_TX, kTY = FA_RAY_TY, kSync = FA_RAY_SYNC;

template <int DT>
__global__ __launch_bounds__(64 * kTX * kTY) void query_rays_kernel(QueryLaunch a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tw = (a.rw + kTX - 1) / kTX, th = (a.rh + kTY - 1) / kTY;
    const int64_t tiles = (int64_t)tw * th;
    const int wg = xcd_order(blockIdx.x, gridDim.x);
    for (int64_t t = wg; t < tiles; t += gridDim.x) {
        const int px = (int)(t % tw) * kTX + (wave % kTX);
        const int py = (int)(t / tw) * kTY + (wave / kTX);
        const bool ray_ok = px < a.rw && py < a.rh;
        const int64_t ray = ray_ok ? (int64_t)py * a.rw + px : 0;
        for (int k0 = 0; k0 < a.rk; k0 += kWave) {
            const int k = k0 + lane;
            query_sample<DT>(a, ray * a.rk + k, ray_ok && k < a.rk);
            // keep the rays of the tile at the same depth; no data is exchanged,
            // so a bare barrier (outputs stay in flight)
            if ((k0 / kWave) % kSync == kSync - 1) __builtin_amdgcn_s_barrier();
        }
    }
}

}  // namespace

hipError_t launch_query(const QueryLaunch &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int64_t cap = 256 * 64;  // grid-stride beyond 64 workgroups per CU
    if (a.rk > 0) {
        const int64_t wgs = (int64_t)((a.rw + kTX - 1) / kTX) * ((a.rh + kTY - 1) / kTY);
        const int grid = (int)(wgs < cap ? wgs : cap);
        const dim3 blk(64 * kTX * kTY);
        if (a.dtype == FA_BF16) hipLaunchKernelGGL(query_rays_kernel<FA_BF16>, dim3(grid), blk, 0, s, a);
        else if (a.dtype == FA_F16) hipLaunchKernelGGL(query_rays_kernel<FA_F16>, dim3(grid), blk, 0, s, a);
        else hipLaunchKernelGGL(query_rays_kernel<FA_F32>, dim3(grid), blk, 0, s, a);
        return hipGetLastError();
    }
    const int64_t wgs = (a.n + 255) / 256;
    const int grid = (int)(wgs < cap ? wgs : cap);
    if (a.dtype == FA_BF16) hipLaunchKernelGGL(query_kernel<FA_BF16>, dim3(grid), dim3(256), 0, s, a);
    else if (a.dtype == FA_F16) hipLaunchKernelGGL(query_kernel<FA_F16>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(query_kernel<FA_F32>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fa
