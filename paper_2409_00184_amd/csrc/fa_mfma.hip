// Grid decode of BF16/FP16 micro-models with matrix cores (gfx950 MFMA).
//
// Pattern: the per-axis contractions of the tensor-product decode are dense
// products with the basis matrices B_a (R x NCP_a, p+1 non-zeros per row),
// so two of the three stages run as v_mfma_f32_16x16x32_{bf16,f16} with FP32
// accumulation (K = 32 covers NCP <= 32 in one instruction; smaller NCP are
// zero padded):
//   x stage (MFMA):  R1_B[u][(j,k)] = sum_i Bx[u][i] P[i][j][k]   (and Dx -> R1_D)
//   y stage (VALU):  R2_BB = sum_j By R1_B, R2_DB = sum_j By R1_D,
//                    R2_BD = sum_j Dy R1_B        (banded, FP32, rounded once)
//   z stage (MFMA):  value = sum_k Bz[w][k] R2_BB,  d/dw = sum_k Dz R2_BB,
//                    d/du = sum_k Bz R2_DB,        d/dv = sum_k Bz R2_BD
// Knot spans and basis values are computed in FP32 and rounded to the
// input type only as MFMA operands; the stored lattice holds P / s_b and
// the outputs are multiplied by the per-block scale s_b in FP32.
//
// A work item is (block, 4 consecutive y rows, up to 64 z columns); its
// lattice slab P[:, jlo..jhi, :] is staged once in LDS transposed to
// [(j,k)][i] so an MFMA B fragment is one 16-byte LDS read.  The x axis is
// walked in chunks of 16 voxels; in each chunk the four waves share the x
// stage, then the y stage, then each wave runs the z stage for 4 x voxels x
// 4 rows and stores straight from the accumulators (16 lanes write 64
// contiguous bytes per row, the 4 column tiles of a wave complete 256 B).
// Items the tile does not fit (NCP > 32, or a y window wider than the LDS
// budget) are decoded voxel by voxel by the same workgroup.
//
// Operand layouts of v_mfma_f32_16x16x32 (checked on the device): lane l
// holds A[l%16][8(l/16) .. 8(l/16)+7], B[8(l/16) .. +7][l%16], and receives
// D[4(l/16) + r][l%16], r = 0..3.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kRows = 4;     // y rows per item
constexpr int kUC = 16;      // x voxels per chunk
constexpr int kK = 32;       // MFMA K (NCP padded)
constexpr int kPtStride = 40;  // halfs per (j,k) row of the transposed slab
constexpr int kR2Stride = 40;  // halfs per (u,v) row of R2
constexpr int kStageStride = 68;  // floats per staged output row (64 + 4: no bank conflicts)

// FP32 -> BF16 / FP16 bits, round to nearest even (the hardware conversions
// v_cvt_pk_bf16_f32 / v_cvt_f16_f32).
__device__ __forceinline__ uint16_t to_bits(float x, bool bf) {
    uint16_t r;
    if (bf) {
        __bf16 h = (__bf16)x;
        __builtin_memcpy(&r, &h, 2);
    } else {
        _Float16 h = (_Float16)x;
        __builtin_memcpy(&r, &h, 2);
    }
    return r;
}

__device__ __forceinline__ f32x4v mfma(const u16x8 &a, const u16x8 &b, const f32x4v &c, bool bf) {
    if (bf) {
        bf16x8 x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
    f16x8 x, y;
    __builtin_memcpy(&x, &a, 16);
    __builtin_memcpy(&y, &b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
}

struct MfmaArgs {
    DecodeLaunch d;
    int ncmax;  // slab columns (j,k) the LDS holds
};

__host__ __device__ inline size_t mfma_lds_bytes(int ncmax) {
    return size_t(ncmax) * kPtStride * 2        // transposed slab
           + size_t(kUC) * (ncmax + 4) * 4 * 2  // R1_B, R1_D (FP32)
           + size_t(kUC * kRows) * kR2Stride * 2 * 3  // R2 (16-bit)
           + sizeof(float) * (kMaxKnotsPerBlock + 4)   // knots
           + sizeof(float) * 9 * kRows;                 // y basis rows
}

// Basis row of one position (span s, degree p) as the 8 consecutive 16-bit
// K entries [8g, 8g+8) of a dense row.
__device__ __forceinline__ u16x8 basis_frag(const float (&N)[4], int s, int p, int g, bool bf) {
    u16x8 f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int r = 8 * g + e - (s - p);
        float v = 0.0f;
#pragma unroll
        for (int q = 0; q <= 3; ++q) v = (r == q) ? N[q] : v;
        f[e] = to_bits(v, bf);
    }
    return f;
}

// Voxel-by-voxel decode of one item (items the tile does not fit).
template <int P>
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
        float *o = a.out + (int64_t)b * a.nch * vox + ((int64_t)u * a.ry + v) * a.rz + w;
        int c = 0;
        for (int ch = 0; ch < 4; ++ch)
            if ((a.mask >> ch) & 1u) o[(int64_t)(c++) * vox] = r[ch];
    }
}

__device__ void mfma_item(const MfmaArgs &A, const fa_block &B, int b, int row0, int nrows,
                          int col0, char *lds) {
    const DecodeLaunch &a = A.d;
    const bool bf = a.dtype == FA_BF16;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];

    uint16_t *Pt = reinterpret_cast<uint16_t *>(lds);
    float *R1B = reinterpret_cast<float *>(lds + size_t(A.ncmax) * kPtStride * 2);
    const int r1s = A.ncmax + 4;
    float *R1D = R1B + kUC * r1s;
    uint16_t *R2 = reinterpret_cast<uint16_t *>(R1D + kUC * r1s);
    float *kn = reinterpret_cast<float *>(R2 + kUC * kRows * kR2Stride * 3);
    float *ytab = kn + kMaxKnotsPerBlock + 4;  // per row: By[4], Dy[4], window start
    const int P = B.degree[0];

    lds_barrier();  // previous item done with LDS
    const int nkn = nx + ny + nz + 3 * (P + 1);
    for (int e = tid; e < nkn; e += blockDim.x) kn[e] = a.knots[B.knot_off + e];
    lds_barrier();
    const float *tx = kn, *ty = tx + nx + P + 1, *tz = ty + ny + P + 1;

    const int jlo = span_search(ny, P, ty, grid_pos(row0, a.ry)) - P;
    const int jhi = span_search(ny, P, ty, grid_pos(row0 + nrows - 1, a.ry));
    const int jn = jhi - jlo + 1;
    const int ncols = jn * nz;
    const int nct = (ncols + 15) >> 4;
    if (nx > kK || ny > kK || nz > kK || nct * 16 > A.ncmax || nrows > kRows) {
        if (P == 3) direct_item<3>(a, B, b, row0, nrows, col0);
        else if (P == 2) direct_item<2>(a, B, b, row0, nrows, col0);
        else direct_item<1>(a, B, b, row0, nrows, col0);
        return;
    }

    // transposed slab Pt[(j,k)][i], zero padded to 16 columns x 32 K entries;
    // one column per thread (consecutive threads read consecutive z points),
    // written to LDS 8 K entries (16 bytes) at a time
    const uint16_t *P16 = static_cast<const uint16_t *>(a.ctrl) + B.ctrl_off;
    const int64_t pstride = (int64_t)ny * nz;
    for (int c = tid; c < nct * 16; c += blockDim.x) {
        const bool cv = c < ncols;
        const int jj = cv ? c / nz : 0;
        const uint16_t *src = P16 + (int64_t)(jlo + jj) * nz + (c - jj * nz);
#pragma unroll
        for (int i8 = 0; i8 < kK; i8 += 8) {
            u16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (cv && i8 + e < nx) ? src[(i8 + e) * pstride] : 0;
            *reinterpret_cast<u16x8 *>(Pt + c * kPtStride + i8) = v;
        }
    }
    // R2 K padding (k >= nz) stays zero for the whole item
    for (int e = tid; e < kUC * kRows * 3 * (kK - nz); e += blockDim.x) {
        const int row = e / (kK - nz), k = nz + e % (kK - nz);
        R2[row * kR2Stride + k] = 0;
    }

    // z fragments of this lane: columns w = col0 + 16 nt + l16, K entries 8g..8g+7
    u16x8 fBz[4], fDz[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int w = min(col0 + 16 * nt + l16, a.rz - 1);
        const float pw = grid_pos(w, a.rz);
        const int sw = span_search(nz, P, tz, pw);
        float N[4], D[4];
        basis_ders_rt(tz, sw, pw, P, N, D);
        fBz[nt] = basis_frag(N, sw, P, g, bf);
        fDz[nt] = basis_frag(D, sw, P, g, bf);
    }
    // y basis of the item's rows (FP32, for the VALU y stage) into LDS
    if (tid < kRows) {
        const int v = row0 + min(tid, nrows - 1);
        const float pv = grid_pos(v, a.ry);
        const int sv = span_search(ny, P, ty, pv);
        float N[4], D[4];
        basis_ders_rt(ty, sv, pv, P, N, D);
        for (int q = 0; q < 4; ++q) {
            ytab[tid * 9 + q] = N[q];
            ytab[tid * 9 + 4 + q] = D[q];
        }
        ytab[tid * 9 + 8] = __int_as_float((sv - P - jlo) * nz);
    }

    const int64_t vox = (int64_t)a.rx * a.ry * a.rz;
    const int64_t plane = (int64_t)a.ry * a.rz;
    int64_t choff[4];
    {
        int c = 0;
        for (int ch = 0; ch < 4; ++ch) {
            choff[ch] = (int64_t)c * vox;
            c += (a.mask >> ch) & 1u;
        }
    }
    float *ob = a.out + (int64_t)b * a.nch * vox;
    const float scale = B.scale;
    lds_barrier();  // slab and padding visible

    for (int u0 = 0; u0 < a.rx; u0 += kUC) {
        // x stage: A = x basis rows u0..u0+15, B = slab columns
        {
            const int u = min(u0 + l16, a.rx - 1);
            const float pu = grid_pos(u, a.rx);
            const int su = span_search(nx, P, tx, pu);
            float N[4], D[4];
            basis_ders_rt(tx, su, pu, P, N, D);
            const u16x8 fBx = basis_frag(N, su, P, g, bf);
            const u16x8 fDx = basis_frag(D, su, P, g, bf);
            for (int ct = wave; ct < nct; ct += 4) {
                const u16x8 pf = *reinterpret_cast<const u16x8 *>(Pt + (16 * ct + l16) * kPtStride + 8 * g);
                const f32x4v z = {0.0f, 0.0f, 0.0f, 0.0f};
                const f32x4v dB = mfma(fBx, pf, z, bf);
                const f32x4v dD = mfma(fDx, pf, z, bf);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    R1B[(4 * g + r) * r1s + 16 * ct + l16] = dB[r];
                    R1D[(4 * g + r) * r1s + 16 * ct + l16] = dD[r];
                }
            }
        }
        lds_barrier();
        // y stage: (u, k) pairs over the workgroup, all rows, three channels
        for (int e = tid; e < kUC * kK; e += blockDim.x) {
            const int ul = e >> 5, k = e & (kK - 1);
            if (k >= nz) continue;
            const float *rb = R1B + ul * r1s + k;
            const float *rd = R1D + ul * r1s + k;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                float bb = 0.0f, db = 0.0f, bd = 0.0f;
                const float *yt = ytab + r * 9;
                const int c0 = __float_as_int(yt[8]);
#pragma unroll
                for (int q = 0; q <= 3; ++q) {
                    if (q > P) break;
                    const float xb = rb[c0 + q * nz], xd = rd[c0 + q * nz];
                    bb = fmaf(yt[q], xb, bb);
                    db = fmaf(yt[q], xd, db);
                    bd = fmaf(yt[4 + q], xb, bd);
                }
                const int row = ul * kRows + r;
                R2[(0 * kUC * kRows + row) * kR2Stride + k] = to_bits(bb, bf);
                R2[(1 * kUC * kRows + row) * kR2Stride + k] = to_bits(db, bf);
                R2[(2 * kUC * kRows + row) * kR2Stride + k] = to_bits(bd, bf);
            }
        }
        lds_barrier();
        // z stage: wave q owns R2 rows 16q..16q+15 = x voxels u0+4q..u0+4q+3,
        // 4 rows.  Each channel's 4 x 4 x 64 tile goes through this wave's
        // LDS region (the R1 buffer, dead until the next chunk) so every
        // global store writes one whole 256-byte z row.
        {
            const int row = 16 * wave + l16;
            const u16x8 aBB = *reinterpret_cast<const u16x8 *>(R2 + (0 * kUC * kRows + row) * kR2Stride + 8 * g);
            const u16x8 aDB = *reinterpret_cast<const u16x8 *>(R2 + (1 * kUC * kRows + row) * kR2Stride + 8 * g);
            const u16x8 aBD = *reinterpret_cast<const u16x8 *>(R2 + (2 * kUC * kRows + row) * kR2Stride + 8 * g);
            float *stage = R1B + wave * (16 * kStageStride);
            const int w = col0 + lane;
            // whole 64-column tile, rows of a multiple of 4 floats: every
            // 4-voxel group is a 16-byte aligned store
            const bool vec_store = col0 + kWave <= a.rz && (a.rz & 3) == 0;
            for (int ch = 0; ch < 4; ++ch) {
                if (!((a.mask >> ch) & 1u)) continue;
                const u16x8 &aa = ch == 1 ? aDB : (ch == 2 ? aBD : aBB);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const f32x4v z = {0.0f, 0.0f, 0.0f, 0.0f};
                    const f32x4v d = mfma(aa, ch == 3 ? fDz[nt] : fBz[nt], z, bf);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        stage[(4 * g + r) * kStageStride + 16 * nt + l16] = d[r] * scale;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int ub = u0 + 4 * wave;
                if (vec_store) {
                    // 16-byte non-temporal stores: a quarter-wave writes one
                    // whole 256-byte z row
                    float *oc = ob + choff[ch] + (int64_t)ub * plane + (int64_t)row0 * a.rz +
                                col0 + 4 * l16;
#pragma unroll
                    for (int it = 0; it < 4; ++it) {
                        const int rr = 4 * it + g;
                        const f32x4 val =
                            *reinterpret_cast<const f32x4 *>(stage + rr * kStageStride + 4 * l16);
                        if (ub + it < a.rx && g < nrows)
                            __builtin_nontemporal_store(
                                val, reinterpret_cast<f32x4 *>(oc + it * plane + g * a.rz));
                    }
                } else {
                    float *oc = ob + choff[ch] + (int64_t)ub * plane + (int64_t)row0 * a.rz + w;
                    const bool wok = w < a.rz;
#pragma unroll
                    for (int rr = 0; rr < 16; ++rr) {
                        const float val = stage[rr * kStageStride + lane];
                        if (wok && ub + (rr >> 2) < a.rx && (rr & 3) < nrows)
                            oc[(rr >> 2) * plane + (rr & 3) * a.rz] = val;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        lds_barrier();  // R1/R2 reused by the next chunk
    }
}

__global__ __launch_bounds__(256, 2) void decode_mfma_kernel(MfmaArgs A) {
    extern __shared__ float4 dyn_lds[];
    char *lds = reinterpret_cast<char *>(dyn_lds);
    const DecodeLaunch &a = A.d;
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
        mfma_item(A, a.blocks[b], b, row0, nrows, col0, lds);
    }
}

}  // namespace

// The x-stage slab holds jn * NCP_z <= ncmax columns; jn of 4 consecutive
// rows of a uniform 32-point axis is at most ceil(3*29/(R-1)) + 4.
int mfma_ncmax(int ry) {
    int jn = (3 * 29 + (ry - 2)) / (ry - 1) + 4;
    jn = jn < 12 ? jn : 12;
    return ((jn * kK + 15) / 16) * 16;
}

hipError_t launch_decode_mfma(const DecodeLaunch &d, int waves, int grid, hipStream_t s) {
    if ((d.dtype != FA_BF16 && d.dtype != FA_F16) || d.rows != kRows || waves != 4 ||
        d.rz > kWave)
        return hipErrorNotSupported;
    MfmaArgs A{d, mfma_ncmax(d.ry)};
    const size_t lds = mfma_lds_bytes(A.ncmax);
    // raise the dynamic LDS limit once per process to the largest tile
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&decode_mfma_kernel),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)mfma_lds_bytes(mfma_ncmax(2)));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(decode_mfma_kernel, dim3(grid), dim3(256), lds, s, A);
    return hipGetLastError();
}

}  // namespace fa
