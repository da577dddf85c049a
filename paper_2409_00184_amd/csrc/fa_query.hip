// Point query over a tiled domain on gfx950 (rows a1-a6 for ray samples).
//
// Alg. 4 evaluates valueMicroModel and gradientMicroModel at every ray
// sample.  One lane per sample:
//   a1  block lookup in FP32 (one rounding per operation, see fa.h);
//   a2  span per axis: for knots flagged uniform, the guess p + floor(u(n-p))
//       checked against the stored knots t[s] and t[s+1] of the window the
//       guess loads (a wave re-reads its windows only when some lane's guess
//       was off by one, which needs u within a few ulps of a knot); other
//       knot vectors take a binary search;
//   a3  FP32 basis and first derivative on the register knot window;
//   a4  the (p+1)^3 control window as (p+1)^2 rows of p+1 consecutive z
//       points;
//   a5  separable contraction of the window: z, then y, then x;
//   a6  chain rule d/dx = r d/du and one 16-byte store per sample.
// The flat list (fa_query_points) gathers knots and rows from global memory
// (vector L1); the ray-structured order (fa_query_rays) keeps the one or two
// micro-models a workgroup's step touches in LDS and gathers from there.
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

// Ray-structured order with the lattices in LDS.  A workgroup owns a tile of
// kLR x kLW adjacent rays (wave w takes row w of the tile, lane = ray * kLS +
// sample) and marches it kLS samples per ray per step, all waves at the same
// depth.  One step of the tile covers under half a micro-block along the rays
// and a few pixel footprints across them, so its samples fall in one or two
// micro-models: the step's first and last samples name them, and the
// workgroup keeps both in two LDS slots (knots and lattice, copied with
// coalesced 16-byte loads when a micro-model first appears, typically once
// per micro-model a ray tile crosses).  Every window gather of the
// evaluation then reads LDS instead of the vector L1; a wave with a sample
// outside both slots (a third micro-model, or one larger than a slot) takes
// the per-lane global form of eval_point for the step (FP32 lattices), or
// serves its other micro-models one at a time (2-byte lattices).  Positions and
// results stay coalesced: kLS consecutive samples of a ray are kLS * 12 and
// kLS * 16 contiguous bytes.
#ifndef FA_RAYS_WAVES
#define FA_RAYS_WAVES 16
#endif
#ifndef FA_SLOT_WORDS
#define FA_SLOT_WORDS 18432
#endif
constexpr int kLW = FA_RAYS_WAVES;       // waves per workgroup = rows of rays
constexpr int kLR = 16;                  // rays per wave (one row of pixels)
constexpr int kLS = kWave / kLR;         // samples per ray and step
constexpr int kSlotWords = FA_SLOT_WORDS;  // lattice words (4 bytes) per slot
constexpr int kSlotKnots = 3 * (FA_MAX_NCP + FA_MAX_DEGREE + 1);
static_assert(kSlotWords % 4 == 0, "slots are filled in 16-byte chunks");
static_assert(2 * kLW <= kWave, "one lane per published block id");

struct RaySmem {
    uint32_t lat[2][kSlotWords + 4];  // +4: 2-byte rows read whole dwords past the end
    float kn[2][kSlotKnots + 4];
    int hdr[2][8];                    // nx, ny, nz, p, flags, scale bits
    int pub[2][2 * kLW];              // per step parity: each wave's first and last block
};

// Knot windows and lattice rows of a micro-model held in an LDS slot.
struct LdsLoads {
    static constexpr bool kRowPointers = true;
    static constexpr bool kWaveKnots = false;
    const float *kn;
    const uint32_t *lat;
    __device__ __forceinline__ const float *row_base(uint32_t o0) const {
        return reinterpret_cast<const float *>(lat) + o0;
    }
    template <int N>
    __device__ __forceinline__ Vec<N> knots(uint32_t i, uint32_t u) const {
        return ldv<N>(kn + (i + u));
    }
    template <int N>
    __device__ __forceinline__ Vec<N> rowf(uint32_t i, uint32_t u) const {
        return ldv<N>(reinterpret_cast<const float *>(lat) + (i + u));
    }
    template <int N>
    __device__ __forceinline__ void pairs(uint32_t i, uint32_t u,
                                          uint32_t (&p)[(N + 1) / 2]) const {
        const uint32_t e = i + u;
        constexpr int W = (N + 2) / 2;
        uint32_t w[W];
#pragma unroll
        for (int m = 0; m < W; ++m) w[m] = lat[(e >> 1) + m];
        align_pairs<N>(w, (int)(e & 1u), p);
    }
};

template <int DT>
__device__ __forceinline__ float4 eval_slot(const RaySmem &sm, int sl, const float (&uu)[3]) {
    const int *h = sm.hdr[sl];
    BlockView V;
    V.nx = h[0];
    V.ny = h[1];
    V.nz = h[2];
    V.flags = (uint32_t)h[4];
    V.knot_off = 0;
    V.ctrl_off = 0;
    V.scale = __int_as_float(h[5]);
    const LdsLoads L{sm.kn[sl], sm.lat[sl]};
    const int p = h[3];
    if (p == 3) return eval_window<3, DT>(L, V, sm.kn[sl], uu);
    if (p == 2) return eval_window<2, DT>(L, V, sm.kn[sl], uu);
    return eval_window<1, DT>(L, V, sm.kn[sl], uu);
}

// 32-bit lattice words of block B (2-byte values rounded up to whole words)
template <int DT>
__device__ __forceinline__ int lattice_words(const fa_block &B) {
    const int n = B.ncp[0] * B.ncp[1] * B.ncp[2];
    return DT == FA_F32 ? n : (n + 1) / 2;
}

// Copy micro-model `blk` (uniform) into slot `sl`: the whole workgroup.
template <int DT>
__device__ __forceinline__ void stage_slot(const QueryLaunch &a, RaySmem &sm, int sl, int blk) {
    const fa_block &B = a.blocks[blk];
    const int nx = uni(B.ncp[0]), ny = uni(B.ncp[1]), nz = uni(B.ncp[2]), p = uni(B.degree[0]);
    const int nk = nx + ny + nz + 3 * (p + 1);
    const int nw = DT == FA_F32 ? nx * ny * nz : (nx * ny * nz + 1) / 2;
    const BlockView V = uniform_view_of(B);
    constexpr uint32_t esz = DT == FA_F32 ? 4u : 2u;
    const float *kp = a.knots + V.knot_off;
    for (int e = threadIdx.x; e < nk; e += blockDim.x) sm.kn[sl][e] = kp[e];
    const __amdgpu_buffer_rsrc_t r =
        make_rsrc(static_cast<const char *>(a.ctrl) + V.ctrl_off * esz, (uint32_t)nw * 4u);
    const int nc = (nw + 3) / 4;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const Vec<4> v = bload<4>(r, (uint32_t)c * 16u);
        uint32_t w[4];
        __builtin_memcpy(w, &v, 16);
        *reinterpret_cast<uint4 *>(&sm.lat[sl][4 * c]) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (threadIdx.x == 0) {
        sm.hdr[sl][0] = nx;
        sm.hdr[sl][1] = ny;
        sm.hdr[sl][2] = nz;
        sm.hdr[sl][3] = p;
        sm.hdr[sl][4] = (int)V.flags;
        sm.hdr[sl][5] = __float_as_int(V.scale);
    }
}

// Position of sample smp of a ray (zeros for a dead lane).
__device__ __forceinline__ float3 ray_position(const QueryLaunch &a, int64_t ray, int smp,
                                               bool live) {
    float3 v = make_float3(0.0f, 0.0f, 0.0f);
    if (live) {
        // streamed once: non-temporal, so positions do not displace lattice lines
        const float *pp = a.xyz + 3 * (ray * a.rk + smp);
        v.x = __builtin_nontemporal_load(pp);
        v.y = __builtin_nontemporal_load(pp + 1);
        v.z = __builtin_nontemporal_load(pp + 2);
    }
    return v;
}

// Block lookup of a position: block coordinates uu and the descriptor index
// (-1 for a dead lane or an empty cell).
__device__ __forceinline__ int ray_lookup(const QueryLaunch &a, float3 v, bool live,
                                          float (&uu)[3]) {
    const int bx = lookup_axis(v.x, a.origin[0], a.rscale[0], a.nb[0], uu[0]);
    const int by = lookup_axis(v.y, a.origin[1], a.rscale[1], a.nb[1], uu[1]);
    const int bz = lookup_axis(v.z, a.origin[2], a.rscale[2], a.nb[2], uu[2]);
    int blk = live ? a.block_of_cell[(bx * a.nb[1] + by) * a.nb[2] + bz] : -1;
    return blk >= a.nblocks ? -1 : blk;
}

template <int DT>
__global__ __launch_bounds__(64 * kLW) void query_rays_lds_kernel(QueryLaunch a) {
    extern __shared__ uint4 ray_lds[];
    RaySmem &sm = *reinterpret_cast<RaySmem *>(ray_lds);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rr = lane / kLS, k = lane % kLS;
    const int tw = (a.rw + kLR - 1) / kLR, th = (a.rh + kLW - 1) / kLW;
    const int64_t tiles = (int64_t)tw * th;
    const int wg = xcd_order(blockIdx.x, gridDim.x);
    // which micro-model each slot holds: every thread takes the same
    // decisions from the same published ids, so these stay uniform
    int held0 = -1, held1 = -1, recent = 1, parity = 0;
    for (int64_t t = wg; t < tiles; t += gridDim.x) {
        const int px = (int)(t % tw) * kLR + rr;
        const int py = (int)(t / tw) * kLW + wave;
        const bool ray_ok = px < a.rw && py < a.rh;
        const int64_t ray = ray_ok ? (int64_t)py * a.rw + px : 0;
        // software pipeline: positions two steps ahead and the block lookup
        // one step ahead are issued before the current step's evaluation, so
        // their memory latency hides behind it
        float uu[3];
        bool live = ray_ok && k < a.rk;
        int blk = ray_lookup(a, ray_position(a, ray, k, live), live, uu);
        float3 pos1 = ray_position(a, ray, kLS + k, ray_ok && kLS + k < a.rk);
        for (int k0 = 0; k0 < a.rk; k0 += kLS) {
            // publish this wave's first and last micro-model of the step
            const uint64_t mb = __ballot(blk >= 0);
            const int f = mb ? __builtin_amdgcn_readlane(blk, (int)__builtin_ctzll(mb)) : -1;
            const int l = mb ? __builtin_amdgcn_readlane(blk, 63 - (int)__builtin_clzll(mb)) : -1;
            if (lane == 0) {
                sm.pub[parity][2 * wave] = f;
                sm.pub[parity][2 * wave + 1] = l;
            }
            __syncthreads();
            // the step's first (A) and last (B) micro-model, in scalar registers
            const int v = lane < 2 * kLW ? sm.pub[parity][lane] : -1;
            const uint64_t mv = __ballot(v >= 0);
            const int A = mv ? __builtin_amdgcn_readlane(v, (int)__builtin_ctzll(mv)) : -1;
            int B = mv ? __builtin_amdgcn_readlane(v, 63 - (int)__builtin_clzll(mv)) : -1;
            if (B == A) B = -1;
            const bool fitA = A >= 0 && lattice_words<DT>(a.blocks[A]) <= kSlotWords;
            const bool fitB = B >= 0 && lattice_words<DT>(a.blocks[B]) <= kSlotWords;
            const int inA = A < 0 ? -1 : (A == held0 ? 0 : (A == held1 ? 1 : -1));
            const int inB = B < 0 ? -1 : (B == held0 ? 0 : (B == held1 ? 1 : -1));
            int stA = -1, stB = -1;
            if (fitA && inA < 0) stA = inB >= 0 ? 1 - inB : 1 - recent;
            if (fitB && inB < 0) {
                const int sa = stA >= 0 ? stA : inA;
                stB = sa >= 0 ? 1 - sa : 1 - recent;
            }
            if (stA >= 0) stage_slot<DT>(a, sm, stA, A);
            if (stB >= 0) stage_slot<DT>(a, sm, stB, B);
            if (stA >= 0 || stB >= 0) __syncthreads();
            if (stA == 0) held0 = A;
            if (stA == 1) held1 = A;
            if (stB == 0) held0 = B;
            if (stB == 1) held1 = B;
            if (A >= 0) recent = A == held0 ? 0 : (A == held1 ? 1 : recent);
            parity ^= 1;
            // next step's lookup and the positions after it
            const int smp = k0 + k;
            const bool cur_live = live;
            const int cur_blk = blk;
            const float cu[3] = {uu[0], uu[1], uu[2]};
            live = ray_ok && smp + kLS < a.rk;
            blk = ray_lookup(a, pos1, live, uu);
            pos1 = ray_position(a, ray, smp + 2 * kLS, ray_ok && smp + 2 * kLS < a.rk);
            // evaluate: from the slots when every sample of the wave is in one
            const int sl = cur_blk < 0 ? -1 : (cur_blk == held0 ? 0 : (cur_blk == held1 ? 1 : -1));
            float4 res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (__all(cur_blk < 0 || sl >= 0)) {
                if (sl >= 0) res = eval_slot<DT>(sm, sl, cu);
            } else if constexpr (DT == FA_F32) {
                if (cur_blk >= 0) {
                    const fa_block &Bd = a.blocks[cur_blk];
                    res = query_any<DT, false>(a, view_of(Bd), Bd.degree[0], cu);
                }
            } else {
                // 2-byte lattices: lanes whose micro-model is in a slot read
                // it there; the wave's other micro-models are served one
                // after the other through scalar descriptors, every lane
                // taking part (the span search exchanges knots across lanes)
                // and keeping the result of its own micro-model.  The
                // per-lane form would need more than the 128 registers a
                // 1024-thread workgroup allows.
                if (sl >= 0) res = eval_slot<DT>(sm, sl, cu);
                bool pend = cur_blk >= 0 && sl < 0;
                while (__any(pend)) {
                    const uint64_t pm = __ballot(pend);
                    const int b0 = __builtin_amdgcn_readlane(cur_blk, (int)__builtin_ctzll(pm));
                    const fa_block &B0 = a.blocks[b0];
                    const float4 r =
                        query_any<DT, true>(a, uniform_view_of(B0), uni(B0.degree[0]), cu);
                    if (pend && cur_blk == b0) {
                        res = r;
                        pend = false;
                    }
                }
            }
            if (!cur_live) continue;
            res.y *= a.rscale[0];
            res.z *= a.rscale[1];
            res.w *= a.rscale[2];
            if (!(a.mask & 1u)) res.x = 0.0f;
            if (!(a.mask & 2u)) res.y = 0.0f;
            if (!(a.mask & 4u)) res.z = 0.0f;
            if (!(a.mask & 8u)) res.w = 0.0f;
            const f32x4 rv = {res.x, res.y, res.z, res.w};
            __builtin_nontemporal_store(rv, reinterpret_cast<f32x4 *>(a.out) + (ray * a.rk + smp));
        }
    }
}

}  // namespace

hipError_t launch_query(const QueryLaunch &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int64_t cap = 256 * 64;  // grid-stride beyond 64 workgroups per CU
    if (a.rk > 0) {
        const int64_t wgs = (int64_t)((a.rw + kLR - 1) / kLR) * ((a.rh + kLW - 1) / kLW);
        const int grid = (int)(wgs < cap ? wgs : cap);
        const dim3 blk(64 * kLW);
        const size_t lds = sizeof(RaySmem);
        static const hipError_t attr =
            [] {
                hipError_t e = hipFuncSetAttribute(
                    reinterpret_cast<const void *>(&query_rays_lds_kernel<FA_F32>),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(RaySmem));
                if (e == hipSuccess)
                    e = hipFuncSetAttribute(
                        reinterpret_cast<const void *>(&query_rays_lds_kernel<FA_BF16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(RaySmem));
                if (e == hipSuccess)
                    e = hipFuncSetAttribute(
                        reinterpret_cast<const void *>(&query_rays_lds_kernel<FA_F16>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(RaySmem));
                return e;
            }();
        if (attr != hipSuccess) return attr;
        if (a.dtype == FA_BF16) hipLaunchKernelGGL(query_rays_lds_kernel<FA_BF16>, dim3(grid), blk, lds, s, a);
        else if (a.dtype == FA_F16) hipLaunchKernelGGL(query_rays_lds_kernel<FA_F16>, dim3(grid), blk, lds, s, a);
        else hipLaunchKernelGGL(query_rays_lds_kernel<FA_F32>, dim3(grid), blk, lds, s, a);
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
