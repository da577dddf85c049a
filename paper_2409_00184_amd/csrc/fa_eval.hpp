// Point evaluation shared by the query and render kernels (rows a1-a6).
//
// Block lookup in FP32 with one rounding per operation (fa.h documents the
// rule), span from a guess corrected against the stored knots (uniform
// knots) or a binary search, knot window and lattice rows fetched as vector
// loads, FP32 basis and derivatives, separable (p+1)^3 contraction.
#pragma once

#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {

template <int N>
struct Vec {
    float v[N];
};

// N consecutive floats from a 4-byte aligned address as one vector load
// (gfx950 accepts dword-aligned multi-dword global loads).
template <int N>
__device__ __forceinline__ Vec<N> ldv(const float *p) {
    Vec<N> r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// Span and register knot window tw[m] = t[s-P+1+m] of one axis.
template <int P>
__device__ __forceinline__ int axis_window(int n, const float *t, float u, bool uniform,
                                           float (&tw)[2 * P]) {
    if (uniform) {
        int s0 = P + (int)(u * float(n - P));
        s0 = s0 > n - 1 ? n - 1 : s0;
        // t[s0-P .. s0+P+1]: covers the windows of s0-1, s0, s0+1
        const Vec<2 * P + 2> w = ldv<2 * P + 2>(t + s0 - P);
        int d = 0;
        if (s0 > P && u < w.v[P]) d = -1;                   // u < t[s0]
        else if (s0 < n - 1 && u >= w.v[P + 1]) d = 1;      // u >= t[s0+1]
#pragma unroll
        for (int m = 0; m < 2 * P; ++m)
            tw[m] = d < 0 ? w.v[m] : (d > 0 ? w.v[m + 2] : w.v[m + 1]);
        return s0 + d;
    }
    const int s = span_search(n, P, t, u);
    const Vec<2 * P> w = ldv<2 * P>(t + s - P + 1);
#pragma unroll
    for (int m = 0; m < 2 * P; ++m) tw[m] = w.v[m];
    return s;
}

struct BlockView {
    int nx, ny, nz;
    uint32_t flags;
    int64_t knot_off, ctrl_off;
    float scale;
};

template <int P, int DT>
__device__ __forceinline__ float4 query_block(const QueryLaunch &a, const BlockView &B,
                                              const float (&uu)[3]) {
    const float *tx = a.knots + B.knot_off;
    const float *ty = tx + B.nx + P + 1;
    const float *tz = ty + B.ny + P + 1;
    float wx[2 * P], wy[2 * P], wz[2 * P];
    const int sx = axis_window<P>(B.nx, tx, uu[0], B.flags & FA_FLAG_UNIFORM_X, wx);
    const int sy = axis_window<P>(B.ny, ty, uu[1], B.flags & FA_FLAG_UNIFORM_Y, wy);
    const int sz = axis_window<P>(B.nz, tz, uu[2], B.flags & FA_FLAG_UNIFORM_Z, wz);
    float xB[P + 1], xD[P + 1], yB[P + 1], yD[P + 1], zB[P + 1], zD[P + 1];
    basis_ders_win<P>(wx, uu[0], xB, xD);
    basis_ders_win<P>(wy, uu[1], yB, yD);
    basis_ders_win<P>(wz, uu[2], zB, zD);
    const int64_t base = B.ctrl_off + ((int64_t)(sx - P) * B.ny + (sy - P)) * B.nz + (sz - P);
    float f = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        float uBB = 0.0f, uDB = 0.0f, uBD = 0.0f;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            const int64_t row = base + ((int64_t)i * B.ny + j) * B.nz;
            float c[P + 1];
            if (DT == FA_F32) {
                const Vec<P + 1> r = ldv<P + 1>(static_cast<const float *>(a.ctrl) + row);
#pragma unroll
                for (int k = 0; k <= P; ++k) c[k] = r.v[k];
            } else {
                const uint16_t *h = static_cast<const uint16_t *>(a.ctrl) + row;
#pragma unroll
                for (int k = 0; k <= P; ++k)
                    c[k] = (DT == FA_BF16 ? bf16_to_f32(h[k]) : f16_to_f32(h[k]));
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
    const float s = DT == FA_F32 ? 1.0f : B.scale;
    return make_float4(f * s, fx * s, fy * s, fz * s);
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

__device__ __forceinline__ BlockView view_of(const fa_block &B) {
    BlockView v;
    v.nx = B.ncp[0];
    v.ny = B.ncp[1];
    v.nz = B.ncp[2];
    v.flags = B.flags;
    v.knot_off = B.knot_off;
    v.ctrl_off = B.ctrl_off;
    v.scale = B.scale;
    return v;
}

template <int DT>
__device__ __forceinline__ float4 query_any(const QueryLaunch &a, const BlockView &V, int p,
                                            const float (&uu)[3]) {
    if (p == 3) return query_block<3, DT>(a, V, uu);
    if (p == 2) return query_block<2, DT>(a, V, uu);
    return query_block<1, DT>(a, V, uu);
}


// Value and domain-unit gradient at (x, y, z); zeros in an empty cell.
// Every lane of the wave must call it (wave-wide vote inside); `live`
// false makes the lane an empty sample.
template <int DT>
__device__ __forceinline__ float4 eval_point(const QueryLaunch &a, float x, float y, float z,
                                             bool live) {
    float uu[3];
    const int bx = lookup_axis(x, a.origin[0], a.rscale[0], a.nb[0], uu[0]);
    const int by = lookup_axis(y, a.origin[1], a.rscale[1], a.nb[1], uu[1]);
    const int bz = lookup_axis(z, a.origin[2], a.rscale[2], a.nb[2], uu[2]);
    int blk = live ? a.block_of_cell[(bx * a.nb[1] + by) * a.nb[2] + bz] : -1;
    if (blk >= a.nblocks) blk = -1;  // anything outside [0, nblocks) is an empty cell
    float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int blk0 = __builtin_amdgcn_readfirstlane(blk);
    if (__all(blk == blk0)) {
        // wave-uniform block: scalar descriptor loads, no divergence
        if (blk0 >= 0) {
            const fa_block &B = a.blocks[blk0];
            r = query_any<DT>(a, view_of(B), B.degree[0], uu);
        }
    } else if (blk >= 0) {
        const fa_block &B = a.blocks[blk];
        r = query_any<DT>(a, view_of(B), B.degree[0], uu);
    }
    r.y *= a.rscale[0];
    r.z *= a.rscale[1];
    r.w *= a.rscale[2];
    return r;
}

}  // namespace fa
