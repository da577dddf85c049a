// Grid decode of BF16/FP16 micro-models with matrix cores (gfx950 MFMA).
//
// Pattern: for every control plane i (lattice index along x) the 2-D
// contraction of the plane with the y and z bases,
//     U_i[v][w] = sum_j sum_k By[v][j] P[i][j][k] Bz[w][k],
// is a pair of dense products, both on matrix cores with FP32 accumulation:
//     Q[j][w] = sum_k P[i][j][k] Bz[w][k]    v_mfma_f32_16x16x32 (K = NCP_z <= 32)
//     U[w][v] = sum_j Q[j][w] By[v][j]       v_mfma_f32_16x16x16 (K = 16 y-window rows)
// and, for the gradients, Q_D with Dz in place of Bz, U_DB = Dy Q, U_BD =
// By Q_D.  A lane receives Q[4(l/16)+r][l%16] from the first product and
// the second reads its A operand as A[l%16][4(l/16)+e], so Q moves from
// the accumulators to the next product in registers, rounded once to the
// input type (no LDS round trip).
// The x contraction is banded (p+1 non-zero basis functions per position)
// and runs on the VALU: each lane keeps U of the last p+1 planes for its
// four outputs in a ring indexed by plane mod (p+1) and walks u = 0..Rx-1,
//     value = sum Bx U_BB,  d/du = sum Dx U_BB,
//     d/dv  = sum Bx U_DB,  d/dw = sum Bx U_BD,
// with the x basis in FP32 from a per-item LDS table (the per-block scale
// folded in, coefficients stored in ring order).  A new plane is produced
// only when the span along x advances, so the matrix-core work per item is
// NCP_x planes x 5 products per wave.
//
// Rounded to the input type: the stored lattice (P / s_b), the z basis, Q
// and the y basis.  Knot spans and every basis value are computed in FP32.
//
// Work item = (block, 16 consecutive y rows, 64 z columns); wave q of the
// four owns columns col0+16q .. col0+16q+15 and lane (g, l16) computes the
// outputs (v = row0 + l16, w = col0 + 16q + 4g + r), r = 0..3.  Per x
// position the four waves pass their 16 x 16 tiles through an LDS tile of
// the item's 16 rows x 64 columns, so that every store instruction writes
// four whole 256-byte z rows (a quarter wave per row): quarter rows stored
// by different waves reach L2 at different times and were measured at 3.6
// against 5.7 TB/s for whole rows.  With interleaved output (one 16-byte
// record per voxel) the same LDS tile holds the item's 16 x 64 records
// instead, and each store instruction writes one whole z row (1 KB).
// Items the tile does not take (NCP_z > 32, or a y window of more than 16
// lattice rows) are decoded voxel by voxel by the same workgroup.
//
// Operand layouts (checked on the device):
//   v_mfma_f32_16x16x32: lane l holds A[l%16][8(l/16)+e], B[8(l/16)+e][l%16], e < 8
//   v_mfma_f32_16x16x16: lane l holds A[l%16][4(l/16)+e], B[4(l/16)+e][l%16], e < 4
//   both: lane l receives D[4(l/16)+r][l%16], r < 4.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kRows = kMfmaRows;  // y rows per item (N of the second product)
constexpr int kK = 32;     // K of the first product: NCP_z
constexpr int kJ = 16;     // K of the second product: y-window lattice rows
constexpr int kCpol = 0;  // ordinary stores (measured faster than non-temporal here)
constexpr int kStage = 32;   // control planes whose fragments LDS holds at once

// Two FP32 values as one dword of two 16-bit values (round to nearest even).
template <int DT>
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    uint32_t r;
    if constexpr (DT == FA_BF16) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        const bf16x2 v = {(__bf16)lo, (__bf16)hi};
        __builtin_memcpy(&r, &v, 4);
    } else {
        typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
        const f16x2 v = {(_Float16)lo, (_Float16)hi};
        __builtin_memcpy(&r, &v, 4);
    }
    return r;
}

template <int DT>
__device__ __forceinline__ f32x4v mma32(const u32x4 &a, const u32x4 &b) {
    const f32x4v z = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (DT == FA_BF16) {
        bf16x8 x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, z, 0, 0, 0);
    } else {
        f16x8 x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, z, 0, 0, 0);
    }
}

template <int DT>
__device__ __forceinline__ f32x4v mma16(const u32x2 &a, const u32x2 &b) {
    const f32x4v z = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (DT == FA_BF16) {
        i16x4 x, y;
        __builtin_memcpy(&x, &a, 8);
        __builtin_memcpy(&y, &b, 8);
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, z, 0, 0, 0);
    } else {
        f16x4 x, y;
        __builtin_memcpy(&x, &a, 8);
        __builtin_memcpy(&y, &b, 8);
        return __builtin_amdgcn_mfma_f32_16x16x16f16(x, y, z, 0, 0, 0);
    }
}

// Entries [k0, k0 + 2 NW) of the dense basis row of a position whose span
// is s (N[r] sits at lattice index s-P+r, zeros elsewhere), as NW dwords of
// two 16-bit values.
template <int DT, int P, int NW>
__device__ __forceinline__ void dense_frag(const float (&N)[P + 1], int s, int k0,
                                           uint32_t (&f)[NW]) {
#pragma unroll
    for (int m = 0; m < NW; ++m) {
        const int r0 = k0 + 2 * m - (s - P);
        float lo = 0.0f, hi = 0.0f;
#pragma unroll
        for (int r = 0; r <= P; ++r) {
            lo = (r0 == r) ? N[r] : lo;
            hi = (r0 + 1 == r) ? N[r] : hi;
        }
        f[m] = pack2<DT>(lo, hi);
    }
}

// Dynamic LDS of one workgroup: the first product's A fragments of up to
// kStage control planes (fragment of lane l of plane i at [i][l], 16 bytes),
// the per-x-position table and the knots.
struct MSmem {
    u32x4 *frag;
    f32x4v *tile;  // [channel][row 16][16 groups of 4 columns], group ^ row;
                   // interleaved: [row 16][64 column records], column ^ row
    float4 *xB;  // scale * Bx in ring order
    float4 *xD;  // scale * Dx in ring order
    int *xS;     // span along x
    float *kn;
};

__host__ __device__ inline size_t mfma_lds_bytes(int rx) {
    return size_t(kStage) * kWave * 16 + size_t(4 * kRows * 16) * 16 + sizeof(float4) * 2 * rx +
           sizeof(int) * ((rx + 3) & ~3) + sizeof(float) * (kMaxKnotsPerBlock + 4);
}

__device__ __forceinline__ MSmem mcarve(void *base, int rx) {
    MSmem s;
    char *p = static_cast<char *>(base);
    s.frag = reinterpret_cast<u32x4 *>(p);
    p += size_t(kStage) * kWave * 16;
    s.tile = reinterpret_cast<f32x4v *>(p);
    p += size_t(4 * kRows * 16) * 16;
    s.xB = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * rx;
    s.xD = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * rx;
    s.xS = reinterpret_cast<int *>(p);
    p += sizeof(int) * ((rx + 3) & ~3);
    s.kn = reinterpret_cast<float *>(p);
    return s;
}

// Voxel-by-voxel decode of one item (items the tile does not take).
template <int P, bool INTER>
__device__ void direct_item(const DecodeLaunch &a, const fa_block &B, int b, int row0, int nrows,
                            int col0) {
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const float *tx = a.knots + B.knot_off;
    const float *ty = tx + nx + P + 1;
    const float *tz = ty + ny + P + 1;
    const int ncol = min(kWave, a.rz - col0);
    const int64_t vox = (int64_t)a.rx * a.ry * a.rz;
    const int total = a.rx * nrows * ncol;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int w = col0 + e % ncol;
        const int v = row0 + (e / ncol) % nrows;
        const int u = e / (ncol * nrows);
        const float pu = grid_pos(u, a.rx), pv = grid_pos(v, a.ry), pw = grid_pos(w, a.rz);
        const int su = span_search(nx, P, tx, pu), sv = span_search(ny, P, ty, pv),
                  sw = span_search(nz, P, tz, pw);
        float xB[P + 1], xD[P + 1], yB[P + 1], yD[P + 1], zB[P + 1], zD[P + 1];
        basis_ders<P>(tx, su, pu, xB, xD);
        basis_ders<P>(ty, sv, pv, yB, yD);
        basis_ders<P>(tz, sw, pw, zB, zD);
        float r[4] = {0, 0, 0, 0};
        const int64_t base = B.ctrl_off + ((int64_t)(su - P) * ny + (sv - P)) * nz + (sw - P);
#pragma unroll 1
        for (int i = 0; i <= P; ++i) {
#pragma unroll 1
            for (int j = 0; j <= P; ++j) {
                const int64_t row = base + ((int64_t)i * ny + j) * nz;
                float tB = 0.0f, tD = 0.0f;
#pragma unroll
                for (int k = 0; k <= P; ++k) {
                    const float c = load_ctrl(a.ctrl, a.dtype, row + k, B.scale);
                    tB = fmaf(zB[k], c, tB);
                    tD = fmaf(zD[k], c, tD);
                }
                r[0] = fmaf(xB[i] * yB[j], tB, r[0]);
                r[1] = fmaf(xD[i] * yB[j], tB, r[1]);
                r[2] = fmaf(xB[i] * yD[j], tB, r[2]);
                r[3] = fmaf(xB[i] * yB[j], tD, r[3]);
            }
        }
        const int64_t vi = ((int64_t)u * a.ry + v) * a.rz + w;
        if constexpr (INTER) {
            const f32x4v rec = {r[0], r[1], r[2], r[3]};
            reinterpret_cast<f32x4v *>(a.out)[(int64_t)b * vox + vi] = rec;
            continue;
        }
        float *o = a.out + (int64_t)b * a.nch * vox + vi;
        int c = 0;
        for (int ch = 0; ch < 4; ++ch)
            if ((a.mask >> ch) & 1u) o[(int64_t)(c++) * vox] = r[ch];
    }
}

template <int DT, int P, bool INTER>
__device__ void mfma_item(const DecodeLaunch &a, const fa_block &B, int b, int row0, int nrows,
                          int col0, const MSmem &sm) {
    const int tid = threadIdx.x, q = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];

    lds_barrier();  // the previous item is done with the LDS table
    const int nkn = nx + ny + nz + 3 * (P + 1);
    for (int e = tid; e < nkn; e += blockDim.x) sm.kn[e] = a.knots[B.knot_off + e];
    lds_barrier();
    const float *tx = sm.kn, *ty = tx + nx + P + 1, *tz = ty + ny + P + 1;

    const int jlo = span_search(ny, P, ty, grid_pos(row0, a.ry)) - P;
    const int jhi = span_search(ny, P, ty, grid_pos(row0 + nrows - 1, a.ry));
    if (nz > kK || jhi - jlo + 1 > kJ) {
        direct_item<P, INTER>(a, B, b, row0, nrows, col0);
        return;
    }

    // x table: span and scale * basis, the coefficient of plane s-P+r in
    // ring slot (s-P+r) mod (P+1)
    const float scale = B.scale;
    for (int u = tid; u < a.rx; u += blockDim.x) {
        const float pu = grid_pos(u, a.rx);
        const int s = span_search(nx, P, tx, pu);
        float N[P + 1], D[P + 1];
        basis_ders<P>(tx, s, pu, N, D);
        const int base = (s - P) % (P + 1);
        float cb[4] = {0.0f, 0.0f, 0.0f, 0.0f}, cd[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            const int r = (m - base + P + 1) % (P + 1);
#pragma unroll
            for (int t = 0; t <= P; ++t) {
                cb[m] = r == t ? N[t] * scale : cb[m];
                cd[m] = r == t ? D[t] * scale : cd[m];
            }
        }
        sm.xB[u] = make_float4(cb[0], cb[1], cb[2], cb[3]);
        sm.xD[u] = make_float4(cd[0], cd[1], cd[2], cd[3]);
        sm.xS[u] = s;
    }

    // B operand of the second product: By / Dy of row v = row0 + l16 at
    // lattice rows jlo + 4g .. jlo + 4g + 3
    uint32_t fBy[2], fDy[2];
    {
        const float pv = grid_pos(row0 + min(l16, nrows - 1), a.ry);
        const int sv = span_search(ny, P, ty, pv);
        float N[P + 1], D[P + 1];
        basis_ders<P>(ty, sv, pv, N, D);
        dense_frag<DT, P, 2>(N, sv, jlo + 4 * g, fBy);
        dense_frag<DT, P, 2>(D, sv, jlo + 4 * g, fDy);
    }
    // B operand of the first product: Bz / Dz of column col0 + 16q + l16 at
    // lattice indices 8g .. 8g + 7
    uint32_t fBz[4], fDz[4];
    {
        const float pw = grid_pos(min(col0 + 16 * q + l16, a.rz - 1), a.rz);
        const int sw = span_search(nz, P, tz, pw);
        float N[P + 1], D[P + 1];
        basis_ders<P>(tz, sw, pw, N, D);
        dense_frag<DT, P, 4>(N, sw, 8 * g, fBz);
        dense_frag<DT, P, 4>(D, sw, 8 * g, fDz);
    }
    const u32x4 bz = {fBz[0], fBz[1], fBz[2], fBz[3]};
    const u32x4 dz = {fDz[0], fDz[1], fDz[2], fDz[3]};
    const u32x2 by = {fBy[0], fBy[1]};
    const u32x2 dy = {fDy[0], fDy[1]};

    // A operand of the first product: P[i][jlo + l16][8g .. 8g + 7] through a
    // buffer resource over this block's lattice, rounded up to whole dwords
    // (the hardware range check is per dword; reads past the end return
    // zero).  Entries k >= NCP_z and rows j >= NCP_y hold other lattice
    // values or the bytes after the lattice: they are masked to zero, so
    // only this block's values reach the product.  With NCP_z odd a row may
    // start on a half dword: five dwords are read and realigned.
    const __amdgpu_buffer_rsrc_t pr =
        make_rsrc(static_cast<const uint16_t *>(a.ctrl) + B.ctrl_off,
                  ((uint32_t)nx * (uint32_t)ny * (uint32_t)nz * 2u + 3u) & ~3u);
    const uint32_t plane_el = (uint32_t)ny * (uint32_t)nz;
    const uint32_t row_el = (uint32_t)(jlo + l16) * (uint32_t)nz + 8u * (uint32_t)g;
    const bool odd = (nz & 1) != 0;
    uint32_t keep[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int k0 = 8 * g + 2 * m;
        keep[m] = (jlo + l16 >= ny || k0 >= nz) ? 0u : (k0 + 1 >= nz ? 0xffffu : 0xffffffffu);
    }
    auto load_frag = [&](int i) -> u32x4 {
        const uint32_t el = (uint32_t)i * plane_el + row_el;
        u32x4 r;
        if (!odd) {
            r = __builtin_amdgcn_raw_buffer_load_b128(pr, el * 2u, 0, 0);
        } else {
            const uint32_t w0 = (el * 2u) & ~3u;
            const uint32_t sh = (el & 1u) * 2u;
            const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(pr, w0, 0, 0);
            const uint32_t t4 = __builtin_amdgcn_raw_buffer_load_b32(pr, w0 + 16u, 0, 0);
            r[0] = __builtin_amdgcn_alignbyte(t[1], t[0], sh);
            r[1] = __builtin_amdgcn_alignbyte(t[2], t[1], sh);
            r[2] = __builtin_amdgcn_alignbyte(t[3], t[2], sh);
            r[3] = __builtin_amdgcn_alignbyte(t4, t[3], sh);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) r[m] &= keep[m];
        return r;
    };

    // LDS tile slots: this lane writes row l16, group 4q + g; it stores row
    // 4q + g, group l16 (columns col0 + 4 l16 .. + 3) through a buffer
    // resource over this block's output
    const int wslot = l16 * 16 + ((4 * q + g) ^ l16);
    const int srow = 4 * q + g;
    const int rslot = srow * 16 + (l16 ^ srow);
    const int ws = col0 + 4 * l16;
    const bool vok = srow < nrows;
    const bool vec = (a.rz & 3) == 0;  // 16-byte aligned groups of 4 columns
    const uint32_t vox = (uint32_t)a.rx * (uint32_t)a.ry * (uint32_t)a.rz;
    const __amdgpu_buffer_rsrc_t orc =
        make_rsrc(a.out + (int64_t)b * a.nch * vox, (uint32_t)a.nch * vox * 4u);
    const uint32_t plane_b = (uint32_t)a.ry * (uint32_t)a.rz * 4u;
    uint32_t vo = ((uint32_t)(row0 + srow) * (uint32_t)a.rz + (uint32_t)ws) * 4u;
    // interleaved: this lane writes records (l16, 16q + 4g + r) at column
    // slot col ^ l16 (the 16 lanes of a row group hit 16 bank groups), and
    // wave q stores rows 4q .. 4q+3, lane = column, 16 bytes each
    const __amdgpu_buffer_rsrc_t irc =
        make_rsrc(reinterpret_cast<f32x4v *>(a.out) + (int64_t)b * vox, vox * 16u);
    const bool iok = col0 + lane < a.rz;
    uint32_t io = ((uint32_t)row0 * (uint32_t)a.rz + (uint32_t)(col0 + lane)) * 16u;
    const uint32_t irow_b = (uint32_t)a.rz * 16u, iplane_b = (uint32_t)a.ry * irow_b;
    uint32_t choff[4];
    {
        uint32_t c = 0;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            choff[ch] = c * vox * 4u;
            c += (a.mask >> ch) & 1u;
        }
    }

    f32x4v W[3][P + 1];
#pragma unroll
    for (int m = 0; m <= P; ++m) W[0][m] = W[1][m] = W[2][m] = f32x4v{0.0f, 0.0f, 0.0f, 0.0f};
    // fragments of planes [clo, clo + kStage) in LDS: every wave loads a
    // quarter of the planes, every wave reads all of them; the x walk then
    // touches no global memory but its stores (a global load in the walk
    // would make each new plane wait for every store issued before it)
    int clo = 0;
    auto stage = [&](int c0) {
        const int c1 = min(nx, c0 + kStage);
        for (int i = c0 + q; i < c1; i += 4) sm.frag[(i - c0) * kWave + lane] = load_frag(i);
    };
    stage(0);
    int top = -1;
    lds_barrier();  // x table and fragments visible

    for (int u = 0; u < a.rx; ++u) {
        const int s = __builtin_amdgcn_readfirstlane(sm.xS[u]);
        while (top < s) {  // uniform: the next control plane enters the ring
            ++top;
            if (top >= clo + kStage) {  // uniform over the workgroup
                lds_barrier();
                clo += kStage;
                stage(clo);
                lds_barrier();
            }
            const u32x4 cur = sm.frag[(top - clo) * kWave + lane];
            const f32x4v qb = mma32<DT>(cur, bz);
            const f32x4v qd = mma32<DT>(cur, dz);
            const u32x2 ab = {pack2<DT>(qb[0], qb[1]), pack2<DT>(qb[2], qb[3])};
            const u32x2 ad = {pack2<DT>(qd[0], qd[1]), pack2<DT>(qd[2], qd[3])};
            const f32x4v ubb = mma16<DT>(ab, by);
            const f32x4v udb = mma16<DT>(ab, dy);
            const f32x4v ubd = mma16<DT>(ad, by);
            const int slot = top % (P + 1);
#pragma unroll
            for (int m = 0; m <= P; ++m) {
                if (slot == m) {
                    W[0][m] = ubb;
                    W[1][m] = udb;
                    W[2][m] = ubd;
                }
            }
        }
        const float4 cb4 = sm.xB[u], cd4 = sm.xD[u];
        const float cb[4] = {cb4.x, cb4.y, cb4.z, cb4.w};
        const float cd[4] = {cd4.x, cd4.y, cd4.z, cd4.w};
        f32x4v o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float val = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
            for (int m = 0; m <= P; ++m) {
                val = fmaf(cb[m], W[0][m][r], val);
                gx = fmaf(cd[m], W[0][m][r], gx);
                gy = fmaf(cb[m], W[1][m][r], gy);
                gz = fmaf(cb[m], W[2][m][r], gz);
            }
            o[0][r] = val;
            o[1][r] = gx;
            o[2][r] = gy;
            o[3][r] = gz;
        }
        lds_barrier();  // every wave is done reading the previous tile
        if constexpr (INTER) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const f32x4v rec = {o[0][r], o[1][r], o[2][r], o[3][r]};
                sm.tile[l16 * 64 + ((16 * q + 4 * g + r) ^ l16)] = rec;
            }
            lds_barrier();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int row = 4 * q + k;
                const f32x4v t = sm.tile[row * 64 + (lane ^ row)];
                if (row < nrows && iok) {
                    uint32_t d[4];
                    __builtin_memcpy(d, &t, 16);
                    const u32x4 dv = {d[0], d[1], d[2], d[3]};
                    __builtin_amdgcn_raw_buffer_store_b128(dv, irc, io + (uint32_t)row * irow_b,
                                                           0, kCpol);
                }
            }
            io += iplane_b;
            continue;
        }
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
            if ((a.mask >> ch) & 1u) sm.tile[ch * 256 + wslot] = o[ch];
        lds_barrier();
        if (vok) {
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (!((a.mask >> ch) & 1u)) continue;
                const f32x4v t = sm.tile[ch * 256 + rslot];
                uint32_t d[4];
                __builtin_memcpy(d, &t, 16);
                if (vec) {
                    if (ws < a.rz) {
                        const u32x4 dv = {d[0], d[1], d[2], d[3]};
                        __builtin_amdgcn_raw_buffer_store_b128(dv, orc, vo, choff[ch], kCpol);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (ws + r < a.rz)
                            __builtin_amdgcn_raw_buffer_store_b32(d[r], orc, vo + 4u * r,
                                                                  choff[ch], kCpol);
                }
            }
        }
        vo += plane_b;
    }
}

template <int DT, bool INTER>
__global__ __launch_bounds__(256) void decode_mfma_kernel(DecodeLaunch a) {
    extern __shared__ float4 dyn_lds[];
    const MSmem sm = mcarve(dyn_lds, a.rx);
    const int wg = xcd_order(blockIdx.x, gridDim.x);
    int64_t beg, end, step;
    if (a.work) {
        beg = a.wg_off[wg];
        end = a.wg_off[wg + 1];
        step = 1;
    } else {
        beg = wg;
        end = a.nitems;
        step = gridDim.x;
    }
    const int64_t per = (int64_t)a.nrowt * a.ncolt;
    for (int64_t it = beg; it < end; it += step) {
        int b, row0, nrows, col0;
        if (a.work) {
            const fa_work wk = a.work[it];
            b = wk.block;
            row0 = wk.row0;
            nrows = wk.nrows;
            col0 = wk.col0;
        } else {
            b = (int)(it / per);
            const int r = (int)(it - (int64_t)b * per);
            row0 = (r / a.ncolt) * a.rows;
            nrows = min(a.rows, a.ry - row0);
            col0 = (r % a.ncolt) * kWave;
        }
        const fa_block &B = a.blocks[b];
        const int p = B.degree[0];
        if (p == 3) mfma_item<DT, 3, INTER>(a, B, b, row0, nrows, col0, sm);
        else if (p == 2) mfma_item<DT, 2, INTER>(a, B, b, row0, nrows, col0, sm);
        else mfma_item<DT, 1, INTER>(a, B, b, row0, nrows, col0, sm);
    }
}

}  // namespace

hipError_t launch_decode_mfma(const DecodeLaunch &d, int waves, int grid, hipStream_t s) {
    if ((d.dtype != FA_BF16 && d.dtype != FA_F16) || d.rows != kRows || waves != 4)
        return hipErrorNotSupported;
    const size_t lds = mfma_lds_bytes(d.rx);
    if (d.dtype == FA_BF16) {
        if (d.interleave)
            hipLaunchKernelGGL((decode_mfma_kernel<FA_BF16, true>), dim3(grid), dim3(256), lds, s, d);
        else
            hipLaunchKernelGGL((decode_mfma_kernel<FA_BF16, false>), dim3(grid), dim3(256), lds, s, d);
    } else {
        if (d.interleave)
            hipLaunchKernelGGL((decode_mfma_kernel<FA_F16, true>), dim3(grid), dim3(256), lds, s, d);
        else
            hipLaunchKernelGGL((decode_mfma_kernel<FA_F16, false>), dim3(grid), dim3(256), lds, s, d);
    }
    return hipGetLastError();
}

}  // namespace fa
