// Adjoint of the grid decode on gfx950 (row a7): G = B^T g.
//
// The fit of control points to samples (the least-squares model(NCP,
// degree) that Alg. 1 runs for each candidate NCP) has gradient
// (2/M) B^T r.  B^T is the transposed separable contraction:
//   HB[i][v][w] = sum_u Bx[u][i] g0 + Dx[u][i] g1,  H2, H3 = sum_u Bx[u][i] g2, g3
//   KB[i][j][w] = sum_v By[v][j] HB + Dy[v][j] H2,  K3 = sum_v By[v][j] H3
//   G[i][j][k]  = sum_w Bz[w][k] KB + Dz[w][k] K3
// One workgroup (16 waves) per micro-model streams its cotangent block once:
// lanes own z columns, wave q owns y rows q, q+16, ...; walking x, every
// lane keeps the p+1 newest partial x contractions of its columns in
// registers (the transpose of the forward decode's sliding window).  When
// control plane i leaves the window it is final: the workgroup writes
// HB/H2/H3 of that plane to LDS, contracts y over each j's contiguous v
// support, then z over each k's w support, and stores the plane of G once.
// Fixed summation order, no atomics: the result is deterministic.
//
// This form serves cotangents with derivative channels; a value-only
// cotangent (the fit's residual) goes to the matrix-core form of
// fa_adjoint_mfma.hip.  The kernel can also split a micro-model's control
// planes between segments: a segment owns planes [i0, i1), streams exactly
// the x positions whose basis touches them (neighbouring segments re-read
// the p-plane overlap) and stores only its own planes, so every plane is
// still written by one workgroup.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

constexpr int kAdjMaxYZ = 64;                      // res[1], res[2] limit
constexpr int kPlane = kAdjMaxYZ * kWave;          // one (v, w) plane

// waves per workgroup: 16 with derivative cotangents, 8 for value only
template <bool DER>
constexpr int adj_waves() { return DER ? 16 : 8; }

template <bool DER>
struct AdjSmem {
    float4 xB[kMaxRes], xD[kMaxRes];
    int xS[kMaxRes];
    float4 yB[kAdjMaxYZ], yD[kAdjMaxYZ];
    int yS[kAdjMaxYZ];
    float4 zB[kAdjMaxYZ], zD[kAdjMaxYZ];
    int zS[kAdjMaxYZ];
    int jva[FA_MAX_NCP], jvb[FA_MAX_NCP];  // v support of control row j
    int kwa[FA_MAX_NCP], kwb[FA_MAX_NCP];  // w support of control column k
    float kn[kMaxKnotsPerBlock + 4];
    float H[DER ? 3 : 1][kPlane];          // HB, H2, H3 of the plane being emitted
    float K[DER ? 2 : 1][FA_MAX_NCP * kWave];  // KB, K3
};

__device__ __forceinline__ float comp4(const float4 &v, int r) {
    return r == 0 ? v.x : (r == 1 ? v.y : (r == 2 ? v.z : v.w));
}

template <int P>
__device__ __forceinline__ void tab_axis(const float *t, int n, int R, int idx, float4 &b4,
                                         float4 &d4, int &s) {
    const float pos = grid_pos(idx, R);
    s = span_search(n, P, t, pos);
    float N[P + 1], D[P + 1];
    basis_ders<P>(t, s, pos, N, D);
    float nb[4] = {0, 0, 0, 0}, nd[4] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        nb[r] = N[r];
        nd[r] = D[r];
    }
    b4 = make_float4(nb[0], nb[1], nb[2], nb[3]);
    d4 = make_float4(nd[0], nd[1], nd[2], nd[3]);
}

// DER: cotangents of derivative channels present (H2, H3, K3 in use)
template <int P, bool DER>
__device__ void adj_block(const fa_block &B, const float *knots, int rx, int ry, int rz,
                          uint32_t mask, int nch, const float *g, float *G, int b, int seg,
                          int nseg, AdjSmem<DER> &sm) {
    constexpr int kAdjWaves = adj_waves<DER>();
    constexpr int kAdjRows = kAdjMaxYZ / kAdjWaves;  // y rows per wave
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const int nkn = nx + ny + nz + 3 * (P + 1);
    for (int e = tid; e < nkn; e += nthr) sm.kn[e] = knots[B.knot_off + e];
    for (int j = tid; j < FA_MAX_NCP; j += nthr) {
        sm.jva[j] = sm.kwa[j] = 0x7fffffff;
        sm.jvb[j] = sm.kwb[j] = -1;
    }
    lds_barrier();
    const float *tx = sm.kn, *ty = tx + nx + P + 1, *tz = ty + ny + P + 1;
    for (int u = tid; u < rx; u += nthr) tab_axis<P>(tx, nx, rx, u, sm.xB[u], sm.xD[u], sm.xS[u]);
    for (int v = tid; v < ry; v += nthr) {
        tab_axis<P>(ty, ny, ry, v, sm.yB[v], sm.yD[v], sm.yS[v]);
        for (int r = 0; r <= P; ++r) {
            atomicMin(&sm.jva[sm.yS[v] - P + r], v);
            atomicMax(&sm.jvb[sm.yS[v] - P + r], v);
        }
    }
    for (int w = tid; w < rz; w += nthr) {
        tab_axis<P>(tz, nz, rz, w, sm.zB[w], sm.zD[w], sm.zS[w]);
        for (int r = 0; r <= P; ++r) {
            atomicMin(&sm.kwa[sm.zS[w] - P + r], w);
            atomicMax(&sm.kwb[sm.zS[w] - P + r], w);
        }
    }
    lds_barrier();

    const int64_t vox = (int64_t)rx * ry * rz;
    const int64_t plane = (int64_t)ry * rz;
    const bool wok = lane < rz;
    const int w = wok ? lane : 0;
    const float *gb = g + (int64_t)b * nch * vox + w;
    int64_t choff[4];
    {
        int c = 0;
        for (int ch = 0; ch < 4; ++ch) {
            choff[ch] = (int64_t)c * vox;
            c += (mask >> ch) & 1u;
        }
    }
    float *Gb = G + B.ctrl_off;

    // sliding windows: planes top-P .. top, rows v = wave + 8 m
    float hB[kAdjRows][P + 1], h2[DER ? kAdjRows : 1][P + 1], h3[DER ? kAdjRows : 1][P + 1];
#pragma unroll
    for (int m = 0; m < kAdjRows; ++m)
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            hB[m][r] = 0.0f;
            if (DER) h2[m][r] = h3[m][r] = 0.0f;
        }
    int top = -1;

    // write plane i (window slot 0) of every column, contract y then z, store
    auto emit = [&](int i) {
#pragma unroll
        for (int m = 0; m < kAdjRows; ++m) {
            const int v = wave + kAdjWaves * m;
            if (v < ry) {
                sm.H[0][v * kWave + lane] = wok ? hB[m][0] : 0.0f;
                if (DER) {
                    sm.H[1][v * kWave + lane] = wok ? h2[m][0] : 0.0f;
                    sm.H[2][v * kWave + lane] = wok ? h3[m][0] : 0.0f;
                }
            }
        }
        lds_barrier();
        for (int e = tid; e < ny * kWave; e += nthr) {
            const int j = e >> 6, ww = e & 63;
            float kb = 0.0f, k3 = 0.0f;
            for (int v = sm.jva[j]; v <= sm.jvb[j]; ++v) {
                const int r = j - (sm.yS[v] - P);
                const float cb = comp4(sm.yB[v], r);
                kb = fmaf(cb, sm.H[0][v * kWave + ww], kb);
                if (DER) {
                    kb = fmaf(comp4(sm.yD[v], r), sm.H[1][v * kWave + ww], kb);
                    k3 = fmaf(cb, sm.H[2][v * kWave + ww], k3);
                }
            }
            sm.K[0][e] = kb;
            if (DER) sm.K[1][e] = k3;
        }
        lds_barrier();
        for (int e = tid; e < ny * nz; e += nthr) {
            const int j = e / nz, k = e - j * nz;
            float acc = 0.0f;
            for (int ww = sm.kwa[k]; ww <= sm.kwb[k]; ++ww) {
                const int r = k - (sm.zS[ww] - P);
                acc = fmaf(comp4(sm.zB[ww], r), sm.K[0][j * kWave + ww], acc);
                if (DER) acc = fmaf(comp4(sm.zD[ww], r), sm.K[1][j * kWave + ww], acc);
            }
            Gb[((int64_t)i * ny + j) * nz + k] = acc;
        }
        lds_barrier();
    };
    // the control planes this segment owns
    const int i0 = (int)((int64_t)seg * nx / nseg), i1 = (int)((int64_t)(seg + 1) * nx / nseg);
    auto advance = [&]() {  // plane top-P is final; shift the windows by one
        if (top - P >= i0 && top - P < i1) emit(top - P);
#pragma unroll
        for (int m = 0; m < kAdjRows; ++m) {
#pragma unroll
            for (int r = 0; r < P; ++r) {
                hB[m][r] = hB[m][r + 1];
                if (DER) {
                    h2[m][r] = h2[m][r + 1];
                    h3[m][r] = h3[m][r + 1];
                }
            }
            hB[m][P] = 0.0f;
            if (DER) h2[m][P] = h3[m][P] = 0.0f;
        }
        ++top;
    };

    // cotangent rows of x position u, loaded one step ahead of their use
    float g0[kAdjRows], g1[kAdjRows], g2[kAdjRows], g3[kAdjRows];
    float n0[kAdjRows], n1[kAdjRows], n2[kAdjRows], n3[kAdjRows];
    auto fetch = [&](int u, float(&f0)[kAdjRows], float(&f1)[kAdjRows], float(&f2)[kAdjRows],
                     float(&f3)[kAdjRows]) {
        const float *gu = gb + (int64_t)u * plane;
#pragma unroll
        for (int m = 0; m < kAdjRows; ++m) {
            const int v = wave + kAdjWaves * m;
            const bool ok = u < rx && wok && v < ry;
            const float *gp = gu + (int64_t)(ok ? v : 0) * rz;
            f0[m] = (ok && (mask & 1u)) ? gp[choff[0]] : 0.0f;
            f1[m] = (ok && DER && (mask & 2u)) ? gp[choff[1]] : 0.0f;
            f2[m] = (ok && DER && (mask & 4u)) ? gp[choff[2]] : 0.0f;
            f3[m] = (ok && DER && (mask & 8u)) ? gp[choff[3]] : 0.0f;
        }
    };
    // x positions whose basis touches [i0, i1): spans s(u) in [i0, i1 - 1 + P]
    // (s(u) is non-decreasing in u)
    int ulo = 0, uhi = rx - 1;
    while (ulo < rx && sm.xS[ulo] < i0) ++ulo;
    while (uhi >= ulo && sm.xS[uhi] - P > i1 - 1) --uhi;
    if (i0 < i1) {
        fetch(ulo, g0, g1, g2, g3);
        for (int u = ulo; u <= uhi; ++u) {
            if (u + 1 <= uhi) fetch(u + 1, n0, n1, n2, n3);
            const int s = sm.xS[u];
            while (top < s) advance();  // uniform over the workgroup
            const float4 bx = sm.xB[u], dx = sm.xD[u];
#pragma unroll
            for (int m = 0; m < kAdjRows; ++m) {
#pragma unroll
                for (int r = 0; r <= P; ++r) {
                    hB[m][r] = fmaf(comp4(bx, r), g0[m], hB[m][r]);
                    if (DER) {
                        hB[m][r] = fmaf(comp4(dx, r), g1[m], hB[m][r]);
                        h2[m][r] = fmaf(comp4(bx, r), g2[m], h2[m][r]);
                        h3[m][r] = fmaf(comp4(bx, r), g3[m], h3[m][r]);
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < kAdjRows; ++m) {
                g0[m] = n0[m];
                g1[m] = n1[m];
                g2[m] = n2[m];
                g3[m] = n3[m];
            }
        }
        // the owned planes not emitted yet (also those no x position touches)
        while (top - P < i1) advance();
    }
}

template <bool DER>
__global__ __launch_bounds__(64 * adj_waves<DER>()) void adjoint_kernel(
    const fa_block *blocks, int nblocks, int nseg, const float *knots, int rx, int ry, int rz,
    uint32_t mask, int nch, const float *g, float *G) {
    extern __shared__ float4 dyn_lds[];
    AdjSmem<DER> &sm = *reinterpret_cast<AdjSmem<DER> *>(dyn_lds);
    const int64_t items = (int64_t)nblocks * nseg;
    for (int64_t it = xcd_order(blockIdx.x, gridDim.x); it < items; it += gridDim.x) {
        const int b = (int)(it / nseg), seg = (int)(it - (int64_t)b * nseg);
        const fa_block &B = blocks[b];
        const int p = B.degree[0];
        if (p == 3) adj_block<3, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, seg, nseg, sm);
        else if (p == 2) adj_block<2, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, seg, nseg, sm);
        else adj_block<1, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, seg, nseg, sm);
        lds_barrier();
    }
}

}  // namespace

hipError_t launch_adjoint(const fa_block *blocks, int nblocks, const float *knots, int rx,
                          int ry, int rz, uint32_t mask, const float *g, float *G, int /*it*/,
                          hipStream_t s) {
    if ((mask & 15u) == 1u) {  // the value channel alone: the matrix-core form
        const hipError_t e = launch_adjoint_value(blocks, nblocks, knots, rx, ry, rz, g, G, s);
        if (e != hipErrorNotSupported) return e;  // else rows it cannot load as 16-byte vectors
    }
    const int nch = __builtin_popcount(mask & 15u);  // derivative channels present
    // raise the dynamic LDS limit once per process (before any graph capture)
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&adjoint_kernel<true>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(AdjSmem<true>));
    if (attr != hipSuccess) return attr;
    const int grid = nblocks < 65536 ? nblocks : 65536;
    hipLaunchKernelGGL((adjoint_kernel<true>), dim3(grid), dim3(64 * adj_waves<true>()),
                       sizeof(AdjSmem<true>), s, blocks, nblocks, 1, knots, rx, ry, rz, mask, nch,
                       g, G);
    return hipGetLastError();
}

}  // namespace fa
