// Adjoint of the value channel on the FP32 matrix cores (row a7): G = B^T g
// for a cotangent of the decoded values only -- the least-squares fit's
// gradient (2/M) B^T r that the NCP search of Alg. 1 and the fit of control
// points need.
//
// The transposed tensor-product contraction is ordered per x slice u of the
// cotangent block:
//     Z_u[v][k] = sum_w g[u][v][w] Bz[w][k]        (z, dense product)
//     Y_u[j][k] = sum_v By[v][j] Z_u[v][k]         (y, dense product)
//     G[i][j][k] += Bx[u][i] Y_u[j][k]             (x, p+1 planes per slice)
// Both products run on v_mfma_f32_16x16x4f32 over 16 x 16 output tiles,
// each summing only over the K steps inside the basis band of its columns
// (the w support of its k, the v support of its j).  The x contraction is
// banded: every wave keeps its Y tiles' contributions to the p+1 planes the
// current slice touches in a register ring (plane i in slot i mod (p+1));
// when the span along x advances, the plane leaving the ring is complete
// and is stored once.  One workgroup (8 waves) per micro-model streams its
// cotangent block once, two x slices per step: a wave runs the same tile of
// both slices as two independent accumulation chains, which hides each
// other's latencies and halves the barriers per slice.  Slice pairs are
// double-buffered in LDS and the next pair is in flight in registers.  Fixed summation order, no floating-point
// atomics: the result is deterministic.
//
// Operand layout of v_mfma_f32_16x16x4f32 (checked on the device): lane l
// holds A[l%16][l/16] and B[l/16][l%16] and receives D[4(l/16)+r][l%16].
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

typedef float f32x4a __attribute__((ext_vector_type(4)));

constexpr int kAW = 8;           // waves per workgroup
constexpr int kAT = kAW * 64;    // threads per workgroup
constexpr int kAM = 64;          // res[1], res[2] and NCP_y, NCP_z limit
// LDS row strides (floats): operand reads of half a wave (16 rows x 2
// columns of a slice, 2 rows x 16 columns of Z and of the dense bases) hit
// distinct banks
constexpr int kSS = 66;
constexpr int kTS = 80;
constexpr int kPre = (kAM * kAM) / kAT;  // slice floats per thread and slice

struct AmSmem {
    float g[4][kAM * kSS];  // cotangent slices [v][w]: two pairs
    float Z[2][kAM * kTS];  // [v][k] of the pair's two slices
    float Bz[kAM * kTS];    // dense z basis [w][k]
    float By[kAM * kTS];    // dense y basis [v][j]
    float4 xB[kMaxRes];     // x basis of each slice in ring order
    int xS[kMaxRes];        // span along x of each slice
    int tw[2][kAM / 16];    // first and last w with a basis entry in each k tile
    int tv[2][kAM / 16];    // first and last v with a basis entry in each j tile
    float kn[kMaxKnotsPerBlock + 4];
};

__device__ __forceinline__ f32x4a mma4(float a, float b, const f32x4a &c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int P, int TW>
__device__ __forceinline__ void adj_value_block(const fa_block &B, const float *knots, int rx,
                                                int ry, int rz,
                                const float *g, float *G, int b, AmSmem &sm) {
    constexpr int R = P + 1;  // ring slots
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int gq = lane >> 4, l16 = lane & 15;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];

    // knots; dense y / z bases and the x table
    const int nkn = nx + ny + nz + 3 * R;
    for (int e = tid; e < nkn; e += kAT) sm.kn[e] = knots[B.knot_off + e];
    for (int e = tid; e < kAM * kTS; e += kAT) sm.Bz[e] = sm.By[e] = 0.0f;
    if (tid < kAM / 16) {
        sm.tw[0][tid] = sm.tv[0][tid] = 0x7fffffff;
        sm.tw[1][tid] = sm.tv[1][tid] = -1;
    }
    lds_barrier();
    const float *tx = sm.kn, *ty = tx + nx + R, *tz = ty + ny + R;
    for (int t = tid; t < ry + rz; t += kAT) {
        const bool isy = t < ry;
        const int pos = isy ? t : t - ry;
        const int n = isy ? ny : nz;
        const float *tk = isy ? ty : tz;
        const float x = grid_pos(pos, isy ? ry : rz);
        const int s = span_search(n, P, tk, x);
        float N[R], D[R];
        basis_ders<P>(tk, s, x, N, D);
        float *M = isy ? sm.By : sm.Bz;
#pragma unroll
        for (int r = 0; r < R; ++r) M[pos * kTS + s - P + r] = N[r];
        // the tiles of 16 lattice indices this position's window touches
        int(*T)[kAM / 16] = isy ? sm.tv : sm.tw;
        for (int tt = (s - P) >> 4; tt <= s >> 4; ++tt) {
            atomicMin(&T[0][tt], pos);
            atomicMax(&T[1][tt], pos);
        }
    }
    for (int u = tid; u < rx; u += kAT) {
        const float x = grid_pos(u, rx);
        const int s = span_search(nx, P, tx, x);
        float N[R], D[R];
        basis_ders<P>(tx, s, x, N, D);
        const int base = (s - P) % R;
        float c[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int r = (m - base + R) % R;
#pragma unroll
            for (int q = 0; q < R; ++q) c[m] = r == q ? N[q] : c[m];
        }
        sm.xB[u] = make_float4(c[0], c[1], c[2], c[3]);
        sm.xS[u] = s;
    }
    const int nvt = (ry + 15) >> 4, njt = (ny + 15) >> 4, nkt = (nz + 15) >> 4;

    // slice loader: thread element e = tid + kAT m of the ry x rz slice
    const int nslice = ry * rz;
    const int64_t vox = (int64_t)rx * ry * rz;
    const float *gb = g + (int64_t)b * vox;
    int loff[kPre];
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
        const int e = tid + kAT * m;
        loff[m] = e < nslice ? (e / rz) * kSS + e % rz : -1;
    }
    float pf[2][kPre];  // the next pair of slices, in flight during this one
    auto fetch = [&](int u, float(&f)[kPre]) {
#pragma unroll
        for (int m = 0; m < kPre; ++m) {
            const int e = tid + kAT * m;
            f[m] = (u < rx && e < nslice) ? gb[(int64_t)u * nslice + e] : 0.0f;
        }
    };
    auto put = [&](int buf, const float(&f)[kPre]) {
#pragma unroll
        for (int m = 0; m < kPre; ++m)
            if (loff[m] >= 0) sm.g[buf][loff[m]] = f[m];
    };
    fetch(0, pf[0]);
    fetch(1, pf[1]);
    put(0, pf[0]);
    put(1, pf[1]);
    fetch(2, pf[0]);
    fetch(3, pf[1]);

    // the Y tiles of this wave (at most TW) and their rings
    const int ntiles = njt * nkt;
    f32x4a ring[TW][R];
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
        for (int m = 0; m < R; ++m) ring[t][m] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
    float *Gb = G + B.ctrl_off;
    auto store_plane = [&](int i, int slot) {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const int tt = wave + kAW * t;
            if (tt >= ntiles) continue;
            const int mt = tt % njt, nt = tt / njt;
            const int k = 16 * nt + l16;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (m != slot) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = 16 * mt + 4 * gq + r;
                    if (j < ny && k < nz) Gb[((int64_t)i * ny + j) * nz + k] = ring[t][m][r];
                }
                ring[t][m] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
    };
    int top = -1;  // newest plane in the rings

    lds_barrier();  // first slice, tile ranges visible

    // x contraction of one slice's Y tiles: advance the rings to its span,
    // then add its contributions to the p+1 planes it touches
    auto accumulate = [&](int u, const f32x4a (&y)[TW]) {
        const int s = __builtin_amdgcn_readfirstlane(sm.xS[u]);
        while (top < s) {  // uniform: plane top+1 enters, plane top-P leaves
            ++top;
            if (top - R >= 0) store_plane(top - R, top % R);
        }
        const float4 cx = sm.xB[u];
        const float c[4] = {cx.x, cx.y, cx.z, cx.w};
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            if (wave + kAW * t >= ntiles) continue;
#pragma unroll
            for (int m = 0; m < R; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) ring[t][m][r] = fmaf(c[m], y[t][r], ring[t][m][r]);
        }
    };

    for (int u = 0; u < rx; u += 2) {
        const int b0 = 2 * ((u >> 1) & 1);  // buffers of slices u, u+1
        const bool two = u + 1 < rx;
        // z: Z tiles (16 v x 16 k) of both slices, two chains per wave
        for (int t = wave; t < nvt * nkt; t += kAW) {
            const int mt = t % nvt, nt = t / nvt;
            const int ao = (16 * mt + l16) * kSS + gq;
            const float *ga0 = sm.g[b0] + ao, *ga1 = sm.g[b0 + 1] + ao;
            const float *bz = sm.Bz + gq * kTS + 16 * nt + l16;
            // K steps of 4 positions covering the tile's band (none if empty),
            // even and odd steps in separate chains (four independent chains
            // per wave hide the matrix cores' latency), added at the end
            f32x4a z0 = {0.0f, 0.0f, 0.0f, 0.0f}, z1 = z0, z0o = z0, z1o = z0;
            const int s1 = sm.tw[1][nt] >> 2;
            int st = sm.tw[0][nt] >> 2;
            for (; st + 1 <= s1; st += 2) {
                const float bb = bz[4 * st * kTS], bo = bz[4 * (st + 1) * kTS];
                const float a0 = ga0[4 * st], a1 = ga1[4 * st];
                const float o0 = ga0[4 * (st + 1)], o1 = ga1[4 * (st + 1)];
                z0 = mma4(a0, bb, z0);
                z1 = mma4(a1, bb, z1);
                z0o = mma4(o0, bo, z0o);
                z1o = mma4(o1, bo, z1o);
            }
            if (st <= s1) {
                const float bb = bz[4 * st * kTS];
                z0 = mma4(ga0[4 * st], bb, z0);
                z1 = mma4(ga1[4 * st], bb, z1);
            }
            z0 += z0o;
            z1 += z1o;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int zo = (16 * mt + 4 * gq + r) * kTS + 16 * nt + l16;
                sm.Z[0][zo] = z0[r];
                sm.Z[1][zo] = z1[r];
            }
        }
        lds_barrier();
        // y: Y tiles (16 j x 16 k) of both slices, then x for slice u, u+1
        f32x4a y0[TW], y1[TW];
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            y0[t] = y1[t] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
            const int tt = wave + kAW * t;
            if (tt >= ntiles) continue;
            const int mt = tt % njt, nt = tt / njt;
            const float *by = sm.By + gq * kTS + 16 * mt + l16;
            const int zo = gq * kTS + 16 * nt + l16;
            f32x4a y0o = {0.0f, 0.0f, 0.0f, 0.0f}, y1o = y0o;
            const int s1 = sm.tv[1][mt] >> 2;
            int st = sm.tv[0][mt] >> 2;
            for (; st + 1 <= s1; st += 2) {
                const float aa = by[4 * st * kTS], ao = by[4 * (st + 1) * kTS];
                const float b0 = sm.Z[0][zo + 4 * st * kTS], b1 = sm.Z[1][zo + 4 * st * kTS];
                const float o0 = sm.Z[0][zo + 4 * (st + 1) * kTS];
                const float o1 = sm.Z[1][zo + 4 * (st + 1) * kTS];
                y0[t] = mma4(aa, b0, y0[t]);
                y1[t] = mma4(aa, b1, y1[t]);
                y0o = mma4(ao, o0, y0o);
                y1o = mma4(ao, o1, y1o);
            }
            if (st <= s1) {
                const float aa = by[4 * st * kTS];
                y0[t] = mma4(aa, sm.Z[0][zo + 4 * st * kTS], y0[t]);
                y1[t] = mma4(aa, sm.Z[1][zo + 4 * st * kTS], y1[t]);
            }
            y0[t] += y0o;
            y1[t] += y1o;
        }
        accumulate(u, y0);
        if (two) accumulate(u + 1, y1);
        // slices u+2, u+3 (loaded while this pair was contracted) into the
        // other pair of buffers, u+4, u+5 into flight; the registers are
        // written only by the loads, so waiting for them never waits for
        // the newer ones (a deeper ring of three pairs in registers was
        // measured slower: 0.152 against 0.130 ms on C4)
        put(b0 ^ 2, pf[0]);
        put((b0 ^ 2) + 1, pf[1]);
        fetch(u + 4, pf[0]);
        fetch(u + 5, pf[1]);
        lds_barrier();
    }
    // planes still in the rings, then planes no slice touches (zero)
    for (int i = max(0, top - P); i <= top; ++i) store_plane(i, i % R);
    for (int e = tid; e < (nx - 1 - top) * ny * nz; e += kAT)
        Gb[(int64_t)(top + 1) * ny * nz + e] = 0.0f;
}

// TW: Y tiles per wave.  Blocks with at most kAW tiles (NCP_y, NCP_z <= 32
// for the usual shapes) run in the TW = 1 kernel, the others in the TW = 2
// kernel; each kernel skips the other's blocks (one register budget per
// kernel: the second tile's rings would halve the first's headroom).
template <int TW>
__global__ __launch_bounds__(kAT) void adjoint_value_kernel(const fa_block *blocks, int nblocks,
                                                             const float *knots, int rx, int ry,
                                                             int rz, const float *g, float *G) {
    extern __shared__ float4 dyn_lds[];
    AmSmem &sm = *reinterpret_cast<AmSmem *>(dyn_lds);
    // slice rows and columns outside ry x rz are never loaded: zero them once
    for (int e = threadIdx.x; e < 4 * kAM * kSS; e += kAT) (&sm.g[0][0])[e] = 0.0f;
    for (int it = xcd_order(blockIdx.x, gridDim.x); it < nblocks; it += gridDim.x) {
        lds_barrier();  // the previous block is done with the LDS
        const fa_block &B = blocks[it];
        const int tiles = ((B.ncp[1] + 15) >> 4) * ((B.ncp[2] + 15) >> 4);
        if ((tiles > kAW) != (TW == 2)) continue;  // uniform: the other kernel's block
        const int p = B.degree[0];
        if (p == 3) adj_value_block<3, TW>(B, knots, rx, ry, rz, g, G, it, sm);
        else if (p == 2) adj_value_block<2, TW>(B, knots, rx, ry, rz, g, G, it, sm);
        else adj_value_block<1, TW>(B, knots, rx, ry, rz, g, G, it, sm);
    }
}

}  // namespace

hipError_t launch_adjoint_value(const fa_block *blocks, int nblocks, const float *knots, int rx,
                                int ry, int rz, const float *g, float *G, hipStream_t s) {
    if (ry > kAM || rz > kAM) return hipErrorNotSupported;
    static const hipError_t attr = [] {
        hipError_t e1 = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&adjoint_value_kernel<1>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(AmSmem));
        hipError_t e2 = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&adjoint_value_kernel<2>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(AmSmem));
        return e1 != hipSuccess ? e1 : e2;
    }();
    if (attr != hipSuccess) return attr;
    const int grid = nblocks < 65536 ? nblocks : 65536;
    hipLaunchKernelGGL(adjoint_value_kernel<1>, dim3(grid), dim3(kAT), sizeof(AmSmem), s,
                       blocks, nblocks, knots, rx, ry, rz, g, G);
    hipLaunchKernelGGL(adjoint_value_kernel<2>, dim3(grid), dim3(kAT), sizeof(AmSmem), s,
                       blocks, nblocks, knots, rx, ry, rz, g, G);
    return hipGetLastError();
}

}  // namespace fa
