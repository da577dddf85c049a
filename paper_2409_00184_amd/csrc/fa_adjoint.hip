// Adjoint of the grid decode on gfx950 (row a7): G = B^T g.
//
// The fit of control points to samples (the least-squares model(NCP,
// degree) that Alg. 1 runs for each candidate NCP) has gradient
// (2/M) B^T r.  B^T is the transposed separable contraction:
//   H[i][v][w]  = sum_u Bx[u][i] g0 + Dx[u][i] g1     (x: u -> i)
//   H2, H3      = sum_u Bx[u][i] g2, g3
//   J[i][j][w]  = sum_v By[v][j] H + Dy[v][j] H2,  J3 = sum_v By[v][j] H3
//   G[i][j][k]  = sum_w Bz[w][k] J + Dz[w][k] J3
// Owner computes, no atomics: a workgroup owns IT consecutive x control
// planes of one block and reads the u-planes of g in their support.  Lanes
// own z columns, the four waves interleave over y rows; the y reduction is
// done wave after wave into LDS so the summation order never changes, and
// the z reduction reads the LDS rows over each k's contiguous support.
// Workgroups of one block are mapped onto one XCD so re-read u-planes stay
// in that XCD's L2.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

constexpr int kAdjWaves = 4;
constexpr int kAdjMaxYZ = 64;                      // res[1], res[2] limit
constexpr int kAdjVPW = kAdjMaxYZ / kAdjWaves;     // y rows per wave
constexpr int kAdjJFloats = 2 * kAdjMaxYZ * kWave;  // IT * nchJ * ny(64) * 64 lanes

struct AdjSmem {
    float4 xB[kMaxRes], xD[kMaxRes];
    int xS[kMaxRes];
    float4 yB[kAdjMaxYZ], yD[kAdjMaxYZ];
    int yS[kAdjMaxYZ];
    float4 zB[kAdjMaxYZ], zD[kAdjMaxYZ];
    int zS[kAdjMaxYZ];
    int kwa[FA_MAX_NCP], kwb[FA_MAX_NCP];
    int ua, ub;
    float kn[kMaxKnotsPerBlock + 4];
    float J[kAdjJFloats];
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

// IT x-planes per workgroup; DER: cotangents of derivative channels present
template <int P, int IT, bool DER>
__device__ void adj_item(const fa_block &B, const float *knots, int rx, int ry, int rz,
                         uint32_t mask, int nch, const float *g, float *G, int b, int i0,
                         AdjSmem &sm) {
    constexpr int NJ = DER ? 2 : 1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const int nkn = nx + ny + nz + 3 * (P + 1);
    for (int e = tid; e < nkn; e += nthr) sm.kn[e] = knots[B.knot_off + e];
    if (tid == 0) {
        sm.ua = 0x7fffffff;
        sm.ub = -1;
    }
    for (int k = tid; k < nz; k += nthr) {
        sm.kwa[k] = 0x7fffffff;
        sm.kwb[k] = -1;
    }
    for (int e = tid; e < IT * NJ * ny * kWave; e += nthr) sm.J[e] = 0.0f;
    __syncthreads();
    const float *tx = sm.kn, *ty = tx + nx + P + 1, *tz = ty + ny + P + 1;
    for (int u = tid; u < rx; u += nthr) {
        tab_axis<P>(tx, nx, rx, u, sm.xB[u], sm.xD[u], sm.xS[u]);
        // u contributes to planes xS-P .. xS; keep it if that meets [i0, i0+IT)
        const int s = sm.xS[u];
        if (s - P <= i0 + IT - 1 && s >= i0) {
            atomicMin(&sm.ua, u);
            atomicMax(&sm.ub, u);
        }
    }
    for (int v = tid; v < ry; v += nthr) tab_axis<P>(ty, ny, ry, v, sm.yB[v], sm.yD[v], sm.yS[v]);
    for (int w = tid; w < rz; w += nthr) {
        tab_axis<P>(tz, nz, rz, w, sm.zB[w], sm.zD[w], sm.zS[w]);
        const int s = sm.zS[w];
        for (int r = 0; r <= P; ++r) {
            atomicMin(&sm.kwa[s - P + r], w);
            atomicMax(&sm.kwb[s - P + r], w);
        }
    }
    __syncthreads();

    // stage A: x contraction into registers, rows v = wave + 4 m
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
    float H[IT][kAdjVPW], H2[DER ? IT : 1][kAdjVPW], H3[DER ? IT : 1][kAdjVPW];
#pragma unroll
    for (int ii = 0; ii < IT; ++ii)
#pragma unroll
        for (int m = 0; m < kAdjVPW; ++m) {
            H[ii][m] = 0.0f;
            if (DER) H2[ii][m] = H3[ii][m] = 0.0f;
        }
    const int ua = sm.ua, ub = sm.ub;
    for (int u = ua; u <= ub; ++u) {
        const int s = sm.xS[u];
        const float4 bx = sm.xB[u], dx = sm.xD[u];
        float cb[IT], cd[IT];
#pragma unroll
        for (int ii = 0; ii < IT; ++ii) {
            const int r = i0 + ii - (s - P);
            const bool in = (r >= 0 && r <= P);
            cb[ii] = in ? comp4(bx, r) : 0.0f;
            cd[ii] = in ? comp4(dx, r) : 0.0f;
        }
        const float *gu = gb + (int64_t)u * plane;
#pragma unroll
        for (int m = 0; m < kAdjVPW; ++m) {
            const int v = wave + kAdjWaves * m;
            if (v < ry && wok) {
                const float *gp = gu + (int64_t)v * rz;
                const float g0 = (mask & 1u) ? gp[choff[0]] : 0.0f;
                const float g1 = (DER && (mask & 2u)) ? gp[choff[1]] : 0.0f;
                const float g2 = (DER && (mask & 4u)) ? gp[choff[2]] : 0.0f;
                const float g3 = (DER && (mask & 8u)) ? gp[choff[3]] : 0.0f;
#pragma unroll
                for (int ii = 0; ii < IT; ++ii) {
                    H[ii][m] = fmaf(cb[ii], g0, H[ii][m]);
                    if (DER) {
                        H[ii][m] = fmaf(cd[ii], g1, H[ii][m]);
                        H2[ii][m] = fmaf(cb[ii], g2, H2[ii][m]);
                        H3[ii][m] = fmaf(cb[ii], g3, H3[ii][m]);
                    }
                }
            }
        }
    }

    // stage B: y contraction into J[ch][ii][j][lane], one wave at a time
    for (int q = 0; q < kAdjWaves; ++q) {
        if (wave == q && wok) {
#pragma unroll
            for (int m = 0; m < kAdjVPW; ++m) {
                const int v = wave + kAdjWaves * m;
                if (v < ry) {
                    const int s = sm.yS[v];
                    const float4 by = sm.yB[v], dy = sm.yD[v];
#pragma unroll
                    for (int r = 0; r <= P; ++r) {
                        const int j = s - P + r;
                        const float cb = comp4(by, r), cd = comp4(dy, r);
#pragma unroll
                        for (int ii = 0; ii < IT; ++ii) {
                            float *jp = sm.J + ((0 * IT + ii) * ny + j) * kWave + lane;
                            float acc = *jp;
                            acc = fmaf(cb, H[ii][m], acc);
                            if (DER) acc = fmaf(cd, H2[ii][m], acc);
                            *jp = acc;
                            if (DER) {
                                float *j3 = sm.J + ((1 * IT + ii) * ny + j) * kWave + lane;
                                *j3 = fmaf(cb, H3[ii][m], *j3);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // stage C: z contraction over each k's support, one output per thread step
    const int nout = IT * ny * nz;
    for (int e = tid; e < nout; e += nthr) {
        const int ii = e / (ny * nz);
        const int rem = e - ii * ny * nz;
        const int j = rem / nz, k = rem - j * nz;
        if (i0 + ii >= nx) continue;
        const float *jr = sm.J + ((0 * IT + ii) * ny + j) * kWave;
        const float *j3 = sm.J + ((1 * IT + ii) * ny + j) * kWave;
        float acc = 0.0f;
        for (int ww = sm.kwa[k]; ww <= sm.kwb[k]; ++ww) {
            const int r = k - (sm.zS[ww] - P);
            acc = fmaf(comp4(sm.zB[ww], r), jr[ww], acc);
            if (DER) acc = fmaf(comp4(sm.zD[ww], r), j3[ww], acc);
        }
        G[B.ctrl_off + ((int64_t)(i0 + ii) * ny + j) * nz + k] = acc;
    }
}

template <int IT, bool DER>
__global__ __launch_bounds__(256) void adjoint_kernel(const fa_block *blocks, int nblocks,
                                                     const float *knots, int rx, int ry, int rz,
                                                     uint32_t mask, int nch, const float *g,
                                                     float *G, int tiles) {
    __shared__ AdjSmem sm;
    // XCD-aware order: workgroups are dealt round-robin over 8 XCDs, so give
    // consecutive logical items (tiles of one block) to one XCD.
    const int nwg = gridDim.x;
    const int per_xcd = nwg / 8;
    int id = blockIdx.x;
    if (per_xcd * 8 == nwg) id = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int b = id / tiles;
    const int i0 = (id - b * tiles) * IT;
    if (b >= nblocks) return;
    const fa_block &B = blocks[b];
    if (i0 >= B.ncp[0]) return;
    const int p = B.degree[0];
    if (p == 3) adj_item<3, IT, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, i0, sm);
    else if (p == 2) adj_item<2, IT, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, i0, sm);
    else adj_item<1, IT, DER>(B, knots, rx, ry, rz, mask, nch, g, G, b, i0, sm);
}

}  // namespace

hipError_t launch_adjoint(const fa_block *blocks, int nblocks, const float *knots, int rx,
                          int ry, int rz, uint32_t mask, const float *g, float *G, int it,
                          hipStream_t s) {
    const bool der = (mask & 14u) != 0;
    const int nch = __builtin_popcount(mask & 15u);
    if (der) it = 1;  // LDS holds two J channels of one plane
    else if (it != 1) it = 2;
    const int tiles = (FA_MAX_NCP + it - 1) / it;
    int64_t nwg = (int64_t)nblocks * tiles;
    nwg = (nwg + 7) / 8 * 8;
    if (der)
        hipLaunchKernelGGL((adjoint_kernel<1, true>), dim3(nwg), dim3(256), 0, s, blocks, nblocks,
                           knots, rx, ry, rz, mask, nch, g, G, tiles);
    else if (it == 1)
        hipLaunchKernelGGL((adjoint_kernel<1, false>), dim3(nwg), dim3(256), 0, s, blocks,
                           nblocks, knots, rx, ry, rz, mask, nch, g, G, tiles);
    else
        hipLaunchKernelGGL((adjoint_kernel<2, false>), dim3(nwg), dim3(256), 0, s, blocks,
                           nblocks, knots, rx, ry, rz, mask, nch, g, G, tiles);
    return hipGetLastError();
}

}  // namespace fa
