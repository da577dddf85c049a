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
// Both products run on v_mfma_f32_16x16x4f32 and never leave the wave's
// registers: the z product of a 16-row band of the slice leaves its 16 x 16
// tile of Z_u in exactly the operand layout of four K steps of the y
// product, so a wave contracts its slices from HBM to Y_u without LDS or
// barriers.  A wave owns one 16-wide k tile and up to two 16-wide j tiles
// of the output and a chunk of consecutive x slices; it keeps the p+1
// control planes its current slice touches in a register ring (plane i in
// slot i mod (p+1)) and stores a plane once when the span along x moves
// past it.  The waves of one micro-model split its x slices into chunks
// whose plane ranges overlap only with their neighbours' (at most p+1
// planes per boundary): the chunk to the right of a boundary leaves its
// partial planes there in LDS, and the chunk to the left adds them to its
// own after the block's one barrier.  The z product's K steps cover the
// 16-column groups of w inside the basis band of the wave's k tile; the y
// product runs over all four row bands (its y basis operands are zero
// outside each j tile's band).  The slice body is straight-line code, one
// instance per (band width, one or two j tiles), so that the four z chains
// (one per row band), the loads of the next slice and the y chains of a
// slice are scheduled together.  Fixed summation order, no floating-point
// atomics: the result is deterministic.
//
// Operand layout of v_mfma_f32_16x16x4f32 (checked on the device): lane l
// holds A[l%16][l/16] and B[l/16][l%16] and receives D[4(l/16)+r][l%16].
// The z product sums w in the order w = 16 q + 4 (l/16) + j (step (q, j)),
// so each lane reads four consecutive w of its row with one 16-byte load;
// the y product sums v = 16 m + 4 (l/16) + r (step (m, r)), which is the
// row that lane's result register r of band m's Z tile holds.
#include "fa_device.hpp"
#include "fa_internal.hpp"

#include <type_traits>

namespace fa {
namespace {

typedef float f32x4a __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kAW = 8;           // waves per workgroup
constexpr int kAT = kAW * 64;    // threads per workgroup
constexpr int kAM = 64;          // res[1], res[2] and NCP_y, NCP_z limit
constexpr int kJT = 2;           // j tiles per wave
// partial planes of the chunk boundaries: at most (X - 1) (p + 1) NCP_y
// NCP_z floats, X <= kAW / (k tiles x j tile pairs), which is below
// (p + 1) * 4096 for every shape
constexpr int kLB = 4 * 4096;

struct AmSmem {
    float kn[kMaxKnotsPerBlock + 4];
    float4 xB[kMaxRes];  // x basis of each slice in ring order
    int xS[kMaxRes];     // span along x of each slice
    float4 yN[kAM];      // y basis of each v (entries beyond p zero)
    float4 zN[kAM];
    int ys[kAM];         // span along y of each v
    int zs[kAM];
    int tw[2][kAM / 16];  // first and last w with a basis entry in each k tile
    float lb[kLB];        // left partial planes of chunks 1..X-1
};

__device__ __forceinline__ f32x4a mma4(float a, float b, const f32x4a &c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float pick4(const float4 &v, int d) {
    return d == 0 ? v.x : (d == 1 ? v.y : (d == 2 ? v.z : v.w));
}

template <int P>
__device__ __forceinline__ void adj_value_block(const fa_block &B, const float *knots, int rx,
                                                int ry, int rz, const float *g, float *G, int b,
                                                AmSmem &sm) {
    constexpr int R = P + 1;  // ring slots
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int gq = lane >> 4, l16 = lane & 15;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];

    // knots; span and basis tables of the y and z positions and the x slices
    const int nkn = nx + ny + nz + 3 * R;
    for (int e = tid; e < nkn; e += kAT) sm.kn[e] = knots[B.knot_off + e];
    if (tid < kAM / 16) {
        sm.tw[0][tid] = 0x7fffffff;
        sm.tw[1][tid] = -1;
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
        float c[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < R; ++r) c[r] = N[r];
        (isy ? sm.yN : sm.zN)[pos] = make_float4(c[0], c[1], c[2], c[3]);
        (isy ? sm.ys : sm.zs)[pos] = s;
        // the k tiles of 16 lattice indices this w position's window touches
        if (!isy) {
            for (int tt = (s - P) >> 4; tt <= s >> 4; ++tt) {
                atomicMin(&sm.tw[0][tt], pos);
                atomicMax(&sm.tw[1][tt], pos);
            }
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
    lds_barrier();

    // waves: (chunk, j tile pair, k tile).  The x slices are split into X
    // chunks of consecutive slices; each chunk after the first starts at the
    // first change of the span along x at or after c rx / X, when there is
    // one (neighbouring chunks then share fewer control planes), and X is
    // as large as the waves allow with every chunk non-empty and no control
    // plane touched by three chunks.  (Values read from LDS that are the
    // same in every lane go through readfirstlane, so the control flow they
    // decide stays scalar.)
    const int njt = (ny + 15) >> 4, nkt = (nz + 15) >> 4;
    const int njp = (njt + 1) >> 1;
    const int W1 = nkt * njp;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int cw = wv / W1, wr = wv % W1;
    uint64_t first[4];  // bit u % 64 of word u / 64: slice u starts a span
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int u = 64 * w + lane;
        first[w] = __ballot(u < rx && u > 0 && sm.xS[u] != sm.xS[u - 1]);
    }
    auto next_start = [&](int u) -> int {  // the first span start >= u, else rx
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w < (u >> 6)) continue;
            uint64_t m = first[w];
            if (w == (u >> 6)) m &= ~0ull << (u & 63);
            if (m) return min(64 * w + __builtin_ctzll(m), rx);
        }
        return rx;
    };
    int X = min(kAW / W1, rx), ua = 0, ue = rx;  // this wave's chunk [ua, ue)
    for (;; --X) {
        bool ok = true;
        int prev = 0;
        ua = 0;
        ue = rx;
        for (int c = 1; c < X && ok; ++c) {
            const int u0 = max(c * rx / X, prev + 1);
            int u = next_start(u0);
            if (u >= rx) u = u0;
            ok = u < rx && (c < 2 || sm.xS[prev - 1] < sm.xS[u] - P);
            if (c == cw) ua = u;
            if (c == cw + 1) ue = u;
            prev = u;
        }
        if (ok || X == 1) break;
    }
    X = __builtin_amdgcn_readfirstlane(X);
    ua = __builtin_amdgcn_readfirstlane(ua);
    ue = __builtin_amdgcn_readfirstlane(ue);
    float *Gb = G + B.ctrl_off;
    const int plane = ny * nz;
    const int c = cw;
    const bool active = c < X;
    const int nt = wr % nkt, jp = wr / nkt;
    const int ub = ue - 1;
    const int Lc = __builtin_amdgcn_readfirstlane(sm.xS[active ? ua : 0] - P);
    // last plane of chunk c-1, first plane of chunk c+1
    const int Hprev = c > 0 && active ? __builtin_amdgcn_readfirstlane(sm.xS[ua - 1]) : -1;
    const int Lnext = c + 1 < X ? __builtin_amdgcn_readfirstlane(sm.xS[ue] - P) : nx;
    const int k = 16 * nt + l16;

    f32x4a ring[kJT][R];
#pragma unroll
    for (int jj = 0; jj < kJT; ++jj)
#pragma unroll
        for (int m = 0; m < R; ++m) ring[jj][m] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
    // plane i of the wave's tiles: into G, or (dst != null) into a partial
    // plane buffer; with add, the buffer's values are added first.  Element
    // (j, k) of a plane is lane_e + (16 jt + r) nz; G is written through a
    // buffer resource, the plane and row in the scalar offset.
    const __amdgpu_buffer_rsrc_t gs = make_rsrc(Gb, (uint32_t)((int64_t)nx * plane * 4));
    const int lane_e = 4 * gq * nz + k;
    auto put_plane = [&](int slot, float *dst, int i, const float *add) {
#pragma unroll
        for (int jj = 0; jj < kJT; ++jj) {
            const int jt = 2 * jp + jj;
            if (jt >= njt) continue;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (m != slot) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = (16 * jt + r) * nz;  // uniform
                    if (16 * jt + 4 * gq + r < ny && k < nz) {
                        float v = ring[jj][m][r];
                        if (add) v = add[lane_e + row] + v;
                        if (dst) dst[lane_e + row] = v;
                        else
                            __builtin_amdgcn_raw_buffer_store_b32(
                                __float_as_uint(v), gs, (uint32_t)lane_e * 4u,
                                (uint32_t)(i * plane + row) * 4u, 0);
                    }
                }
                ring[jj][m] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
    };
    // a completed plane of this chunk: shared with the chunk to the left
    // (its partial goes to LDS) or this chunk's alone (stored)
    auto flush = [&](int i) {
        if (i <= Hprev) put_plane(i % R, sm.lb + ((c - 1) * R + (i - Lc)) * plane, i, nullptr);
        else put_plane(i % R, nullptr, i, nullptr);
    };

    int top = Lc - 1;  // newest plane in the ring
    if (active) {
        // the k tile's z band: the 16-column groups q = q0 + q', q' < nq, in
        // which some w has a basis entry for one of the tile's k (a tile no
        // position touches takes one group of zero weights)
        const int qlo = __builtin_amdgcn_readfirstlane(sm.tw[0][nt] >> 4);
        const int qhi = __builtin_amdgcn_readfirstlane(sm.tw[1][nt] >> 4);
        const int nq = qhi >= qlo ? qhi - qlo + 1 : 1;
        const int q0 = qhi >= qlo ? qlo : 0;
        // operands held for the whole block: the z basis at the lane's w =
        // 16 (q0 + q') + 4 gq + j for its k, the y basis at its 16 v
        // positions for its j (zero outside each j tile's band, so the y
        // product runs over all four row bands)
        float bzs[4][4], by[4][4][kJT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int w = 16 * (q0 + q) + 4 * gq + j;
                float val = 0.0f;
                if (w < rz && k < nz) {
                    const int d = k - (sm.zs[w] - P);
                    if (d >= 0 && d <= P) val = pick4(sm.zN[w], d);
                }
                bzs[q][j] = val;
            }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jj = 0; jj < kJT; ++jj) {
                    const int v = 16 * mt + 4 * gq + r, j = 16 * (2 * jp + jj) + l16;
                    float val = 0.0f;
                    if (v < ry && j < ny) {
                        const int d = j - (sm.ys[v] - P);
                        if (d >= 0 && d <= P) val = pick4(sm.yN[v], d);
                    }
                    by[mt][r][jj] = val;
                }

        // slice loads: 16 bytes of row 16 m + l16 at w = 16 q + 4 gq, rows
        // and columns clamped into the slice (the bases are zero there, so
        // the values read have no weight; every lane issues the same loads):
        // a buffer resource over the block, the lane's row and column in
        // one 32-bit offset, the slice in the scalar offset
        const int64_t vox = (int64_t)rx * ry * rz;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(g + (int64_t)b * vox, (uint32_t)(vox * 4));
        uint32_t roff[4], coff[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            roff[t] = (uint32_t)(min(16 * t + l16, ry - 1) * rz * 4);
            coff[t] = (uint32_t)(min(16 * t + 4 * gq, rz - 4) * 4);
        }
        const uint32_t sbytes = (uint32_t)(ry * rz * 4);
        auto load = [&](int u, int mt, int q) -> float4 {
            const u32x4 x =
                __builtin_amdgcn_raw_buffer_load_b128(rs, roff[mt] + coff[q], (uint32_t)u * sbytes, 0);
            return make_float4(__uint_as_float(x[0]), __uint_as_float(x[1]), __uint_as_float(x[2]),
                               __uint_as_float(x[3]));
        };
        const int nj = min(2, njt - 2 * jp);
        // the slice loop, straight-line code for each (nq, one or two j tiles)
        auto slices = [&](auto NQc, auto NJc) {
            constexpr int NQ = decltype(NQc)::value, NJ = decltype(NJc)::value;
            auto loadq = [&](int u, int mt, int q) { return load(u, mt, min(q0 + q, 3)); };
            float4 ga[4][NQ];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int q = 0; q < NQ; ++q) ga[mt][q] = loadq(ua, mt, q);
            for (int u = ua; u <= ub; ++u) {
                const int un = u < ub ? u + 1 : u;  // the next slice (the last one again at the end)
                // z: four independent chains (one per 16-row band)
                f32x4a Z[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) Z[mt] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int mt = 0; mt < 4; ++mt) {
                            const float4 &a = ga[mt][q];
                            const float av = j == 0 ? a.x : (j == 1 ? a.y : (j == 2 ? a.z : a.w));
                            Z[mt] = mma4(av, bzs[q][j], Z[mt]);
                        }
                // the next slice, in flight during the rest of this one
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int q = 0; q < NQ; ++q) ga[mt][q] = loadq(un, mt, q);
                // y: the y basis is zero outside each j tile's band
                f32x4a Y[kJT], Yo[kJT];
#pragma unroll
                for (int jj = 0; jj < kJT; ++jj) Y[jj] = Yo[jj] = f32x4a{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj) {
                        Y[jj] = mma4(by[mt][0][jj], Z[mt][0], Y[jj]);
                        Yo[jj] = mma4(by[mt][1][jj], Z[mt][1], Yo[jj]);
                        Y[jj] = mma4(by[mt][2][jj], Z[mt][2], Y[jj]);
                        Yo[jj] = mma4(by[mt][3][jj], Z[mt][3], Yo[jj]);
                    }
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) Y[jj] += Yo[jj];
                // x contraction: advance the ring to this slice's span, then
                // add its contributions to the p+1 planes it touches
                const int s = __builtin_amdgcn_readfirstlane(sm.xS[u]);
                while (top < s) {  // uniform: plane top+1 enters, plane top-P leaves
                    ++top;
                    if (top - R >= Lc) flush(top - R);
                }
                const float4 cx = sm.xB[u];
                const float cf[4] = {cx.x, cx.y, cx.z, cx.w};
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj)
#pragma unroll
                    for (int m = 0; m < R; ++m)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            ring[jj][m][r] = fmaf(cf[m], Y[jj][r], ring[jj][m][r]);
            }
        };
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        if (nj == 2) {
            if (nq == 4) slices(I4{}, I2{});
            else if (nq == 3) slices(I3{}, I2{});
            else if (nq == 2) slices(I2{}, I2{});
            else slices(I1{}, I2{});
        } else {
            if (nq == 4) slices(I4{}, I1{});
            else if (nq == 3) slices(I3{}, I1{});
            else if (nq == 2) slices(I2{}, I1{});
            else slices(I1{}, I1{});
        }
        // planes between this chunk's last and the next chunk's first (no
        // slice touches them when the x span jumps by more than p+1 between
        // neighbouring slices) leave the ring as zeros
        while (c + 1 < X && top < Lnext - 1) {
            ++top;
            if (top - R >= Lc) flush(top - R);
        }
        // planes still in the ring that no chunk to the right shares
        for (int i = max(Lc, top - P); i <= top && i < Lnext; ++i) flush(i);
    }
    lds_barrier();  // left partial planes of every chunk in LDS
    if (active && c + 1 < X) {
        // planes shared with the chunk to the right: its partial + this one
        for (int i = Lnext; i <= top; ++i)
            put_plane(i % R, nullptr, i, sm.lb + (c * R + (i - Lnext)) * plane);
    }
    // planes no slice touches (zero)
    const int hl = __builtin_amdgcn_readfirstlane(sm.xS[rx - 1]);
    for (int e = tid; e < (nx - 1 - hl) * plane; e += kAT) Gb[(int64_t)(hl + 1) * plane + e] = 0.0f;
}

__global__ __launch_bounds__(kAT) void adjoint_value_kernel(const fa_block *blocks, int nblocks,
                                                             const float *knots, int rx, int ry,
                                                             int rz, const float *g, float *G) {
    extern __shared__ float4 dyn_lds[];
    AmSmem &sm = *reinterpret_cast<AmSmem *>(dyn_lds);
    // one workgroup per micro-model
    const int it = blockIdx.x;
    if (it >= nblocks) return;
    const fa_block &B = blocks[it];
    const int p = B.degree[0];
    if (p == 3) adj_value_block<3>(B, knots, rx, ry, rz, g, G, it, sm);
    else if (p == 2) adj_value_block<2>(B, knots, rx, ry, rz, g, G, it, sm);
    else adj_value_block<1>(B, knots, rx, ry, rz, g, G, it, sm);
}

}  // namespace

hipError_t launch_adjoint_value(const fa_block *blocks, int nblocks, const float *knots, int rx,
                                int ry, int rz, const float *g, float *G, hipStream_t s) {
    // 16-byte row loads: every row of the cotangent starts on a 16-byte
    // boundary
    if (ry > kAM || rz > kAM || rz % 4 != 0 || (reinterpret_cast<uintptr_t>(g) & 15) != 0)
        return hipErrorNotSupported;
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&adjoint_value_kernel),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(AmSmem));
    if (attr != hipSuccess) return attr;
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_value_kernel, dim3(nblocks), dim3(kAT), sizeof(AmSmem), s, blocks,
                       nblocks, knots, rx, ry, rz, g, G);
    return hipGetLastError();
}

}  // namespace fa
