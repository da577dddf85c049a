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

// N consecutive 32-bit words at byte offset voff + soff of a buffer
// resource: the base sits in scalar registers, voff is one 32-bit VGPR (the
// lane's part) and soff a wave-uniform SGPR (added by the load itself, no
// vector instruction); offsets past the resource's size read as zero.
template <int N>
__device__ __forceinline__ Vec<N> bload(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                        uint32_t soff = 0) {
    Vec<N> v;
    if constexpr (N == 1) {
        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        __builtin_memcpy(&v, &x, 4);
    } else if constexpr (N == 2) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        __builtin_memcpy(&v, &x, 8);
    } else if constexpr (N == 3) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
        __builtin_memcpy(&v, &x, 12);
    } else if constexpr (N == 4) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        __builtin_memcpy(&v, &x, 16);
    } else {
        static_assert(N > 4 && N <= 8, "window of at most 8 words");
        const Vec<4> lo = bload<4>(r, voff, soff);
        const Vec<N - 4> hi = bload<N - 4>(r, voff + 16u, soff);
#pragma unroll
        for (int m = 0; m < 4; ++m) v.v[m] = lo.v[m];
#pragma unroll
        for (int m = 0; m < N - 4; ++m) v.v[4 + m] = hi.v[m];
    }
    return v;
}

// Pairs of 2-byte lattice values: p[j] holds values 2j (low half) and 2j+1
// (high half) of a window, from the dwords w[] around it when the window
// starts on the high half of w[0] (sh = 1) or on its low half (sh = 0):
// one byte-align per pair.
template <int N, int W>
__device__ __forceinline__ void align_pairs(const uint32_t (&w)[W], int sh,
                                            uint32_t (&p)[(N + 1) / 2]) {
#pragma unroll
    for (int j = 0; j < (N + 1) / 2; ++j)
        p[j] = __builtin_amdgcn_alignbyte(w[j + 1 < W ? j + 1 : W - 1], w[j], (uint32_t)sh * 2u);
}

// Knot windows and lattice rows of one block, either through buffer
// resources (the block is the same in every lane) or through plain 64-bit
// addresses (lanes in different blocks).
template <bool UNI>
struct BlockLoads;

template <>
struct BlockLoads<true> {
    static constexpr bool kRowPointers = false;
    static constexpr bool kWaveKnots = true;  // every lane in one micro-model
    __amdgpu_buffer_rsrc_t kr, cr;
    // the lattice resource ends on a dword boundary: with 2-byte values and
    // an odd count the last value shares its dword with the next two bytes,
    // and the hardware range check is per dword
    __device__ BlockLoads(const float *knots, uint32_t nknots, const void *ctrl, uint32_t cbytes)
        : kr(make_rsrc(knots, nknots * 4u)), cr(make_rsrc(ctrl, (cbytes + 3u) & ~3u)) {}
    // element offsets split into the lane's part i and a wave-uniform part u
    template <int N>
    __device__ __forceinline__ Vec<N> knots(uint32_t i, uint32_t u) const {
        return bload<N>(kr, i * 4u, u * 4u);
    }
    // Span and knot window of a non-uniform axis (knots from element k0):
    // every lane of the wave is in this micro-model, so the wave reads the
    // axis's knots once, lane j holding t[j] (and t[64 + j]), and each lane
    // runs its binary search and gathers its window with cross-lane reads
    // (ds_bpermute) instead of dependent memory loads.  Same span and
    // window values as span_search and a knot load.
    template <int P>
    __device__ __forceinline__ int span_window(uint32_t k0, int n, float u,
                                               float (&tw)[2 * P]) const {
        const int lane = (int)__lane_id(), nk = n + P + 1;
        const float ka = bload<1>(kr, (uint32_t)min(lane, nk - 1) * 4u, k0 * 4u).v[0];
        const bool two = nk > kWave;  // uniform
        const float kb =
            two ? bload<1>(kr, (uint32_t)min(kWave + lane, nk - 1) * 4u, k0 * 4u).v[0] : 0.0f;
        auto kn = [&](int j) {
            const float a = __shfl(ka, j & (kWave - 1));
            if (!two) return a;
            const float b = __shfl(kb, j & (kWave - 1));
            return j < kWave ? a : b;
        };
        // every lane takes part in every cross-lane read (no divergent
        // branch around them): largest s in [P, n-1] with t[s] <= u, by
        // bisection keeping t[lo] <= u < t[hi]; u >= t[n] gives n-1
        const bool top = u >= kn(n);
        int lo = P, hi = n;
        while (__any(hi - lo > 1)) {
            const int mid = (lo + hi) >> 1;
            const float tm = kn(mid);
            const bool act = hi - lo > 1, below = u < tm;
            hi = act && below ? mid : hi;
            lo = act && !below ? mid : lo;
        }
        const int s = top ? n - 1 : lo;
#pragma unroll
        for (int m = 0; m < 2 * P; ++m) tw[m] = kn(s - P + 1 + m);
        return s;
    }
    template <int N>
    __device__ __forceinline__ Vec<N> rowf(uint32_t i, uint32_t u) const {
        return bload<N>(cr, i * 4u, u * 4u);
    }
    // N two-byte lattice values from element i + u as pairs (align_pairs):
    // the dwords around them (reads past the lattice's end come back as zero)
    template <int N>
    __device__ __forceinline__ void pairs(uint32_t i, uint32_t u,
                                          uint32_t (&p)[(N + 1) / 2]) const {
        const uint32_t e = i + u;
        constexpr int W = (N + 2) / 2;
        const Vec<W> v = bload<W>(cr, (e * 2u) & ~3u);
        uint32_t w[W];
        __builtin_memcpy(w, &v, sizeof(w));
        align_pairs<N>(w, (int)(e & 1u), p);
    }
};

template <>
struct BlockLoads<false> {
    static constexpr bool kRowPointers = false;
    static constexpr bool kWaveKnots = false;
    const float *kp;
    const char *cp;
    __device__ BlockLoads(const float *knots, uint32_t, const void *ctrl, uint32_t)
        : kp(knots), cp(static_cast<const char *>(ctrl)) {}
    template <int N>
    __device__ __forceinline__ Vec<N> knots(uint32_t i, uint32_t u) const {
        return ldv<N>(kp + (i + u));
    }
    template <int N>
    __device__ __forceinline__ Vec<N> rowf(uint32_t i, uint32_t u) const {
        return ldv<N>(reinterpret_cast<const float *>(cp) + (i + u));
    }
    // as BlockLoads<true>::pairs; the dwords are read only as far as the
    // window reaches (a window starting on a high half needs one dword more
    // when N is even), which stays within two bytes of its last value
    template <int N>
    __device__ __forceinline__ void pairs(uint32_t i, uint32_t u,
                                          uint32_t (&p)[(N + 1) / 2]) const {
        const uint32_t e = i + u;
        const int sh = (int)(e & 1u);
        constexpr int B = (N + 1) / 2, W = (N + 2) / 2;
        const uint32_t *wp = reinterpret_cast<const uint32_t *>(cp) + (e >> 1);
        uint32_t w[W];
        const Vec<B> v = ldv<B>(reinterpret_cast<const float *>(wp));
        __builtin_memcpy(w, &v, sizeof(v));
        if constexpr (W > B) w[B] = sh ? wp[B] : 0u;
        align_pairs<N>(w, sh, p);
    }
};

// Span and register knot window tw[m] = t[s-P+1+m] of one axis (knots of
// the axis start at element k0 of the block's knots).  Uniform knots: the
// guess p + floor(u (n-p)) is off by at most one (and only within a few
// ulps of a knot); one load of the knots around it covers the windows of
// the guess and of both neighbours, and the comparisons with t[s0] and
// t[s0+1] pick one (selects, no branch).
template <int P, class LD>
__device__ __forceinline__ int axis_window(const LD &L, uint32_t k0, int n,
                                           const float *t, float u, bool uniform,
                                           float (&tw)[2 * P]) {
    if (uniform) {
        int s0 = P + (int)(u * float(n - P));
        s0 = s0 > n - 1 ? n - 1 : s0;
        // the window of the guess, t[s0-P+1 .. s0+P], holds t[s0] and t[s0+1]
        Vec<2 * P> w = L.template knots<2 * P>((uint32_t)(s0 - P + 1), k0);
        int d = 0;
        if (s0 > P && u < w.v[P - 1]) d = -1;           // u < t[s0]
        else if (s0 < n - 1 && u >= w.v[P]) d = 1;      // u >= t[s0+1]
        // a wrong guess needs u within a few ulps of a knot: when some lane of
        // the wave has one, the lanes re-read their windows at the corrected
        // span (the others read the same window again)
        if (__builtin_expect(__any(d != 0), 0))
            w = L.template knots<2 * P>((uint32_t)(s0 + d - P + 1), k0);
#pragma unroll
        for (int m = 0; m < 2 * P; ++m) tw[m] = w.v[m];
        return s0 + d;
    }
    if constexpr (LD::kWaveKnots) return L.template span_window<P>(k0, n, u, tw);
    const int s = span_search(n, P, t, u);
    const Vec<2 * P> w = L.template knots<2 * P>((uint32_t)(s - P + 1), k0);
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

// Value and d/du of one micro-model at block coordinates uu, with its knots
// (tx: the x, y and z vectors back to back) and lattice read through the
// loader L (buffer resources, per-lane addresses or a copy in LDS).
template <int P, int DT, class LD>
__device__ __forceinline__ float4 eval_window(const LD &L, const BlockView &B, const float *tx,
                                              const float (&uu)[3]) {
    const uint32_t kx = 0, ky = (uint32_t)B.nx + P + 1, kz = ky + (uint32_t)B.ny + P + 1;
    float wx[2 * P], wy[2 * P], wz[2 * P];
    const int sx = axis_window<P>(L, kx, B.nx, tx, uu[0], B.flags & FA_FLAG_UNIFORM_X, wx);
    const int sy = axis_window<P>(L, ky, B.ny, tx + ky, uu[1], B.flags & FA_FLAG_UNIFORM_Y, wy);
    const int sz = axis_window<P>(L, kz, B.nz, tx + kz, uu[2], B.flags & FA_FLAG_UNIFORM_Z, wz);
    float xB[P + 1], xD[P + 1], yB[P + 1], yD[P + 1], zB[P + 1], zD[P + 1];
    basis_ders_win<P>(wx, uu[0], xB, xD);
    basis_ders_win<P>(wy, uu[1], yB, yD);
    basis_ders_win<P>(wz, uu[2], zB, zD);
    // a block's lattice has at most 64^3 points: 32-bit offsets from its base
    const uint32_t plane = (uint32_t)B.ny * (uint32_t)B.nz;
    const uint32_t o0 = ((uint32_t)(sx - P) * (uint32_t)B.ny + (uint32_t)(sy - P)) *
                            (uint32_t)B.nz + (uint32_t)(sz - P);
    float f = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        float uBB = 0.0f, uDB = 0.0f, uBD = 0.0f;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            // the row's offset from o0 depends on the block only
            const uint32_t ru = (uint32_t)i * plane + (uint32_t)j * (uint32_t)B.nz;
            float c[P + 1];
            if constexpr (DT == FA_F32 && LD::kRowPointers) {
                // loaders with per-lane strides walk a row pointer (one add
                // per row, both halves of the row at immediate offsets)
                const Vec<P + 1> r = ldv<P + 1>(L.row_base(o0) + (i * plane + j * (uint32_t)B.nz));
#pragma unroll
                for (int k = 0; k <= P; ++k) c[k] = r.v[k];
            } else if constexpr (DT == FA_F32) {
                const Vec<P + 1> r = L.template rowf<P + 1>(o0, ru);
#pragma unroll
                for (int k = 0; k <= P; ++k) c[k] = r.v[k];
            } else {
                uint32_t pw[(P + 2) / 2];
                L.template pairs<P + 1>(o0, ru, pw);
#pragma unroll
                for (int k = 0; k <= P; ++k) {
                    const uint32_t v = pw[k >> 1];
                    if (DT == FA_BF16)
                        c[k] = __uint_as_float(k & 1 ? v & 0xffff0000u : v << 16);
                    else
                        c[k] = f16_to_f32((uint16_t)(k & 1 ? v >> 16 : v & 0xffffu));
                }
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

// UNI: the block is the same in every lane (its knots and lattice are read
// through buffer resources).
template <int P, int DT, bool UNI>
__device__ __forceinline__ float4 query_block(const QueryLaunch &a, const BlockView &B,
                                              const float (&uu)[3]) {
    const float *tx = a.knots + B.knot_off;
    const uint32_t nk = (uint32_t)B.nx + (uint32_t)B.ny + (uint32_t)B.nz + 3u * (P + 1);
    constexpr uint32_t esz = DT == FA_F32 ? 4u : 2u;
    const uint32_t nctrl = (uint32_t)B.nx * (uint32_t)B.ny * (uint32_t)B.nz;
    const BlockLoads<UNI> L(tx, nk, static_cast<const char *>(a.ctrl) + B.ctrl_off * esz,
                            nctrl * esz);
    return eval_window<P, DT>(L, B, tx, uu);
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

// The descriptor of a micro-model every active lane shares, as scalar
// values: each field is read once and marked wave-uniform, so offsets built
// from it stay in scalar registers (buffer-load soffset operands).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ BlockView uniform_view_of(const fa_block &B) {
    BlockView v;
    v.nx = uni(B.ncp[0]);
    v.ny = uni(B.ncp[1]);
    v.nz = uni(B.ncp[2]);
    v.flags = (uint32_t)uni((int)B.flags);
    const int64_t ko = B.knot_off, co = B.ctrl_off;
    v.knot_off = (int64_t)(((uint64_t)(uint32_t)uni((int)(ko >> 32)) << 32) |
                           (uint32_t)uni((int)ko));
    v.ctrl_off = (int64_t)(((uint64_t)(uint32_t)uni((int)(co >> 32)) << 32) |
                           (uint32_t)uni((int)co));
    v.scale = __int_as_float(uni(__float_as_int(B.scale)));
    return v;
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

template <int DT, bool UNI>
__device__ __forceinline__ float4 query_any(const QueryLaunch &a, const BlockView &V, int p,
                                            const float (&uu)[3]) {
    if (p == 3) return query_block<3, DT, UNI>(a, V, uu);
    if (p == 2) return query_block<2, DT, UNI>(a, V, uu);
    return query_block<1, DT, UNI>(a, V, uu);
}


// Value and domain-unit gradient at (x, y, z); zeros in an empty cell.
// Every lane of the wave must call it (wave-wide vote inside); `live`
// false makes the lane an empty sample.  When every lane of the wave is in
// one micro-model its descriptor is read once into scalar registers and its
// knots and lattice sit behind buffer resources; otherwise each lane reads
// its own (measured: serving the micro-models of a wave one after the other
// costs more than the per-lane form).
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
    // the micro-model of the first live lane; lanes that are not live take
    // part in its evaluation and their results are discarded by the caller
    const uint64_t lv = __ballot(live);
    const int blk0 = lv ? __builtin_amdgcn_readlane(blk, (int)__builtin_ctzll(lv)) : -1;
    if (__all(!live || blk == blk0)) {
        if (blk0 >= 0) {
            const fa_block &B = a.blocks[blk0];
            r = query_any<DT, true>(a, uniform_view_of(B), uni(B.degree[0]), uu);
        }
    } else if (blk >= 0) {
        const fa_block &B = a.blocks[blk];
        r = query_any<DT, false>(a, view_of(B), B.degree[0], uu);
    }
    r.y *= a.rscale[0];
    r.z *= a.rscale[1];
    r.w *= a.rscale[2];
    return r;
}

}  // namespace fa
