// Grid decode of batched micro-models on gfx950 (FP32 VALU forms).
//
// decode_sep: the batched, persistent, separable form (rows a0-a6).
//   The tensor-product sum over the (p+1)^3 window factorises per axis, so
//   one column (v, w) of a work item is decoded as
//     T_B[j] = sum_k Bz[w][k] P[i][j][k],   T_D[j] = sum_k Dz[w][k] P[i][j][k]
//     U_BB[i] = sum_j By[v][j] T_B[j],  U_DB[i] = sum_j Dy[v][j] T_B[j],
//     U_BD[i] = sum_j By[v][j] T_D[j]
//     value = sum_i Bx[u][i] U_BB[i], d/du = sum_i Dx[u][i] U_BB[i],
//     d/dv  = sum_i Bx[u][i] U_DB[i], d/dw = sum_i Bx[u][i] U_BD[i]
//   with every sum banded to the p+1 non-zero basis functions.  A lane owns
//   one (v, w) column (lanes along z, so every store is a contiguous 256 B
//   row) and walks u = 0..Rx-1 keeping the p+1 newest U values in
//   registers; U[i] is built on the fly from a lattice slab staged once per
//   work item in LDS.  The x-axis basis (span + p+1 values + p+1
//   derivatives per u) is tabulated in LDS once per item and read as
//   broadcasts.  Work items are (block, y-row range, 64-wide z chunk); a
//   workgroup runs the items a host plan assigned to it, or a grid-stride
//   share of the default order.
//
// The residual form (MODE 1) decodes the value channel only and, instead of
//   the value f, stores gscale * (f - samples) for a fit's loss, summing
//   (f - samples)^2 in FP64 per lane (x order), per wave (fixed shuffle
//   tree) and per work item (waves in order) into one partial per item; a
//   second kernel adds each block's partials in item order.  The samples
//   are read one x position ahead through a buffer resource, and dead lanes
//   load and store at an offset outside every resource (no branch), so the
//   x walk issues a fixed number of memory operations per step.
// The error form (MODE 2) reads the samples the same way and stores nothing per
//   voxel: each item leaves max |f - samples| and the FP64 sum of squares,
//   and a second kernel turns them into each block's (max, rms) error, the
//   error-map entry of the adaptive NCP search, without the decode ever
//   reaching memory.
//
// decode_plain: the baseline -- one thread per voxel, one launch per block,
//   each thread doing its own span searches, basis evaluation and (p+1)^3
//   window sum straight from global memory.
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

// Dynamic LDS of the separable decode: x table (rx rows), knots, slab.
struct SepSmem {
    float4 *xB;
    float4 *xD;
    int *xS;
    float *kn;
    float *slab;
    int slab_floats;
};

__device__ __forceinline__ SepSmem carve(void *base, int rx, int slab) {
    SepSmem s;
    char *p = static_cast<char *>(base);
    s.xB = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * rx;
    s.xD = reinterpret_cast<float4 *>(p);
    p += sizeof(float4) * rx;
    s.kn = reinterpret_cast<float *>(p);
    p += sizeof(float) * (kMaxKnotsPerBlock + 4);
    s.xS = reinterpret_cast<int *>(p);
    p += sizeof(int) * ((rx + 3) & ~3);
    s.slab = reinterpret_cast<float *>(p);
    s.slab_floats = slab;
    return s;
}

__host__ __device__ size_t sep_lds_bytes(int rx, int slab) {
    return sizeof(float4) * 2 * rx + sizeof(float) * (kMaxKnotsPerBlock + 4) +
           sizeof(int) * ((rx + 3) & ~3) + sizeof(float) * slab;
}

template <int P>
__device__ __forceinline__ float4 pack4(const float (&v)[P + 1]) {
    float4 r;
    r.x = v[0];
    r.y = P >= 1 ? v[P >= 1 ? 1 : 0] : 0.0f;
    r.z = P >= 2 ? v[P >= 2 ? 2 : 0] : 0.0f;
    r.w = P >= 3 ? v[P >= 3 ? 3 : 0] : 0.0f;
    return r;
}

__device__ __forceinline__ float comp(const float4 &v, int r) {
    return r == 0 ? v.x : (r == 1 ? v.y : (r == 2 ? v.z : v.w));
}

// MODE 0: decode, 1: residual form, 2: error form, 3: decode of all four
// channels stored interleaved (one 16-byte record per voxel)
template <int P, bool NT, int MODE>
__device__ void sep_item(const DecodeLaunch &a, int b, int row0, int nrows, int col0, int64_t item,
                         SepSmem &sm) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nthr >> 6;
    const fa_block &B = a.blocks[b];
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const int64_t koff = B.knot_off, coff = B.ctrl_off;
    const float scale = B.scale;
    const int nkn = nx + ny + nz + 3 * (P + 1);
    constexpr bool RESID = MODE == 1 || MODE == 2;  // reads the samples
    constexpr bool GRAD = MODE == 1;   // stores the scaled residual

    lds_barrier();  // the previous item is done with the shared buffers
    for (int e = tid; e < nkn; e += nthr) sm.kn[e] = a.knots[koff + e];
    lds_barrier();
    const float *tx = sm.kn;
    const float *ty = tx + nx + P + 1;
    const float *tz = ty + ny + P + 1;

    // x table: span and basis of every grid position along x
    for (int u = tid; u < a.rx; u += nthr) {
        const float uu = grid_pos(u, a.rx);
        const int s = span_search(nx, P, tx, uu);
        float N[P + 1], D[P + 1];
        basis_ders<P>(tx, s, uu, N, D);
        sm.xB[u] = pack4<P>(N);
        sm.xD[u] = pack4<P>(D);
        sm.xS[u] = s;
    }

    // lattice rows j in [jlo, jhi] cover the y windows of every row of the item
    const int jlo = span_search(ny, P, ty, grid_pos(row0, a.ry)) - P;
    const int jhi = span_search(ny, P, ty, grid_pos(row0 + nrows - 1, a.ry));
    const int plane = (jhi - jlo + 1) * nz;  // slab floats per x plane
    const int ic = min(nx, sm.slab_floats / plane);
    const bool single = (ic == nx);

    // z basis of this lane's column
    const bool wok = (col0 + lane) < a.rz;
    const int w = wok ? col0 + lane : a.rz - 1;
    const float zw = grid_pos(w, a.rz);
    const int sz = span_search(nz, P, tz, zw);
    float zB[P + 1], zD[P + 1];
    basis_ders<P>(tz, sz, zw, zB, zD);
    const int kz0 = sz - P;

    // Slab element e = ii * plane + r is value r of control plane c0 + ii's
    // rows jlo..jhi, which lie back to back in the lattice.  A thread walks
    // its elements (stride nthr) with (ii, r) kept incrementally, and issues
    // four loads before their four LDS writes.
    const int nynz = ny * nz;
    const int dii = nthr / plane, dr = nthr - dii * plane;
    const int ii0 = tid / plane, r0 = tid - ii0 * plane;
    auto stage = [&](int c0, int c1) {
        const int cnt = (c1 - c0) * plane;
        const int64_t base = coff + (int64_t)(c0 * ny + jlo) * nz;
        int ii = ii0, r = r0;
        for (int e0 = tid; e0 < cnt; e0 += 4 * nthr) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q] = e0 + q * nthr < cnt
                           ? load_ctrl(a.ctrl, a.dtype, base + (ii * nynz + r), scale)
                           : 0.0f;
                r += dr;
                ii += dii;
                if (r >= plane) {
                    r -= plane;
                    ++ii;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (e0 + q * nthr < cnt) sm.slab[e0 + q * nthr] = v[q];
        }
    };

    lds_barrier();  // x table visible
    if (single) {
        stage(0, nx);
        lds_barrier();
    }

    const int64_t vox = (int64_t)a.rx * a.ry * a.rz;
    const int64_t plane_out = (int64_t)a.ry * a.rz;
    int64_t choff[4];
    {
        int c = 0;
        for (int ch = 0; ch < 4; ++ch) {
            choff[ch] = (int64_t)c * vox;
            c += (a.mask >> ch) & 1u;
        }
    }

    // residual form: samples and cotangent of this block through buffer
    // resources (value channel only, so both have the layout [u][v][w])
    constexpr uint32_t kDead = 0xfffffff0u;  // beyond every resource
    double acc = 0.0;
    float amax = 0.0f;
    const __amdgpu_buffer_rsrc_t yr =
        make_rsrc(RESID ? a.samples + (int64_t)b * vox : a.out, RESID ? (uint32_t)vox * 4u : 0u);
    const __amdgpu_buffer_rsrc_t gr =
        make_rsrc(GRAD ? a.out + (int64_t)b * vox : a.samples, GRAD ? (uint32_t)vox * 4u : 0u);

    for (int rb = 0; rb < nrows; rb += nwaves) {
        const int rr = rb + wave;
        const bool rok = rr < nrows;
        const int v = row0 + (rok ? rr : nrows - 1);
        const float yv = grid_pos(v, a.ry);
        const int sy = span_search(ny, P, ty, yv);
        float yB[P + 1], yD[P + 1];
        basis_ders<P>(ty, sy, yv, yB, yD);
        const int jrow = sy - P - jlo;

        float *ob = a.out + (int64_t)b * a.nch * vox + (int64_t)v * a.rz + w;
        const bool live = rok && wok;
        const uint32_t col_off = ((uint32_t)v * (uint32_t)a.rz + (uint32_t)w) * 4u;
        const uint32_t pstep = (uint32_t)plane_out * 4u;

      // the x walk, specialised on whether the slab holds every control
      // plane (then it stages nothing inside the walk)
      auto walk = [&](auto single_c) {
        constexpr bool SINGLE = decltype(single_c)::value;
        int clo = 0, chi = SINGLE ? nx : ic;
        if (!SINGLE) {
            lds_barrier();
            stage(0, ic);
            lds_barrier();
        }

        float wBB[P + 1], wDB[P + 1], wBD[P + 1];
#pragma unroll
        for (int r = 0; r <= P; ++r) wBB[r] = wDB[r] = wBD[r] = 0.0f;
        int top = -1;
        // residual form: the sample of x position u, loaded four positions
        // ahead into one of four registers used in turn (no register copy
        // waits for a load in flight)
        auto yload = [&](int u) {
            return RESID ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                         yr, (live && u < a.rx)
                                                                 ? col_off + (uint32_t)u * pstep
                                                                 : kDead,
                                                         0, 0))
                         : 0.0f;
        };
        // issue order load, store, load, store as in every step, so the
        // counter wait at a step is the same on entry as in the loop (the
        // stores go beyond the resource and are dropped)
        auto ydummy = [&]() {
            if (GRAD) __builtin_amdgcn_raw_buffer_store_b32(0u, gr, kDead, 0, 0);
        };
        float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f, y3 = 0.0f;
        if constexpr (RESID) {
            y0 = yload(0);
            ydummy();
            y1 = yload(1);
            ydummy();
            y2 = yload(2);
            ydummy();
            y3 = yload(3);
            ydummy();
        }

        auto step = [&](int u, float &ycur) {
            const int s = sm.xS[u];
            while (top < s) {  // uniform over the workgroup
                ++top;
                if (!SINGLE && top >= chi) {
                    lds_barrier();
                    clo = chi;
                    chi = min(clo + ic, nx);
                    stage(clo, chi);
                    lds_barrier();
                }
                const float *sl = sm.slab + (top - clo) * plane + jrow * nz + kz0;
                float tB[P + 1], tD[P + 1];
#pragma unroll
                for (int jj = 0; jj <= P; ++jj) {
                    float x = 0.0f, y = 0.0f;
#pragma unroll
                    for (int kk = 0; kk <= P; ++kk) {
                        const float c = sl[jj * nz + kk];
                        x = fmaf(zB[kk], c, x);
                        y = fmaf(zD[kk], c, y);
                    }
                    tB[jj] = x;
                    tD[jj] = y;
                }
                float uBB = 0.0f, uDB = 0.0f, uBD = 0.0f;
#pragma unroll
                for (int jj = 0; jj <= P; ++jj) {
                    uBB = fmaf(yB[jj], tB[jj], uBB);
                    uDB = fmaf(yD[jj], tB[jj], uDB);
                    uBD = fmaf(yB[jj], tD[jj], uBD);
                }
#pragma unroll
                for (int r = 0; r < P; ++r) {
                    wBB[r] = wBB[r + 1];
                    wDB[r] = wDB[r + 1];
                    wBD[r] = wBD[r + 1];
                }
                wBB[P] = uBB;
                wDB[P] = uDB;
                wBD[P] = uBD;
            }
            const float4 bx = sm.xB[u];
            const float4 dx = sm.xD[u];
            float val = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
                const float cb = comp(bx, r), cd = comp(dx, r);
                val = fmaf(cb, wBB[r], val);
                gx = fmaf(cd, wBB[r], gx);
                gy = fmaf(cb, wDB[r], gy);
                gz = fmaf(cb, wBD[r], gz);
            }
            if (RESID) {
                // use the sample before the register is reloaded, so the
                // old and new values never live at once (no copy)
                const float r = val - ycur;
                const uint32_t off = col_off + (uint32_t)u * pstep;
                ycur = yload(u + 4);
                const double rd = live ? (double)r : 0.0;
                acc = fma(rd, rd, acc);
                if (GRAD)
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, r * a.gscale),
                                                          gr, live ? off : kDead, 0, NT ? 2 : 0);
                else
                    amax = fmaxf(amax, live ? fabsf(r) : 0.0f);
            } else if (MODE == 3) {
                if (live) {
                    const f32x4 rec = {val, gx, gy, gz};
                    f32x4 *o = reinterpret_cast<f32x4 *>(a.out) +
                               ((int64_t)b * vox + (int64_t)u * plane_out + (int64_t)v * a.rz + w);
                    if (NT) __builtin_nontemporal_store(rec, o);
                    else *o = rec;
                }
            } else if (live) {
                float *o = ob + (int64_t)u * plane_out;
                if (NT) {
                    if (a.mask & 1u) __builtin_nontemporal_store(val, o + choff[0]);
                    if (a.mask & 2u) __builtin_nontemporal_store(gx, o + choff[1]);
                    if (a.mask & 4u) __builtin_nontemporal_store(gy, o + choff[2]);
                    if (a.mask & 8u) __builtin_nontemporal_store(gz, o + choff[3]);
                } else {
                    if (a.mask & 1u) o[choff[0]] = val;
                    if (a.mask & 2u) o[choff[1]] = gx;
                    if (a.mask & 4u) o[choff[2]] = gy;
                    if (a.mask & 8u) o[choff[3]] = gz;
                }
            }
        };
        int u = 0;
        if constexpr (RESID) {
            for (; u + 3 < a.rx; u += 4) {
                step(u, y0);
                step(u + 1, y1);
                step(u + 2, y2);
                step(u + 3, y3);
            }
            if (u < a.rx) step(u, y0);
            if (u + 1 < a.rx) step(u + 1, y1);
            if (u + 2 < a.rx) step(u + 2, y2);
        } else {  // no samples: two steps per iteration keep the code small
            for (; u + 1 < a.rx; u += 2) {
                step(u, y0);
                step(u + 1, y1);
            }
            if (u < a.rx) step(u, y0);
        }
      };
        if (single) walk(std::true_type{});
        else walk(std::false_type{});
    }

    if (RESID) {
        // fixed-order sum of the item: lanes by a shuffle tree (lane 0's
        // result), then waves in order
        __shared__ double wsum[8];
        __shared__ float wmax[8];
        for (int off = 32; off >= 1; off >>= 1) {
            acc += __shfl_xor(acc, off);
            if (!GRAD) amax = fmaxf(amax, __shfl_xor(amax, off));
        }
        if (lane == 0) {
            wsum[wave] = acc;
            wmax[wave] = amax;
        }
        lds_barrier();
        if (tid == 0) {
            double t = 0.0;
            float m = 0.0f;
            for (int q = 0; q < nwaves; ++q) {
                t += wsum[q];
                m = fmaxf(m, wmax[q]);
            }
            if (GRAD) {
                a.partials[item] = t;
            } else {
                a.partials[2 * item] = (double)m;
                a.partials[2 * item + 1] = t;
            }
        }
    }
}

template <int WAVES, bool NT, int MODE>
__global__ __launch_bounds__(WAVES * 64) void decode_sep_kernel(DecodeLaunch a) {
    extern __shared__ float4 dyn_lds[];
    SepSmem sm = carve(dyn_lds, a.rx, a.slab);
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
        // the item's index in the default order, whatever order runs it
        const int64_t item = (int64_t)b * per + (row0 / a.rows) * a.ncolt + col0 / kWave;
        const int p = a.blocks[b].degree[0];
        if (p == 3) sep_item<3, NT, MODE>(a, b, row0, nrows, col0, item, sm);
        else if (p == 2) sep_item<2, NT, MODE>(a, b, row0, nrows, col0, item, sm);
        else sep_item<1, NT, MODE>(a, b, row0, nrows, col0, item, sm);
    }
}

// ------------------------------------------------------------------ plain

template <int P>
__device__ __forceinline__ void plain_voxel(const fa_block &B, const float *knots,
                                            const float *ctrl, int u, int v, int w, int rx,
                                            int ry, int rz, float (&res)[4]) {
    const int nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
    const float *tx = knots + B.knot_off;
    const float *ty = tx + nx + P + 1;
    const float *tz = ty + ny + P + 1;
    const float pu = grid_pos(u, rx), pv = grid_pos(v, ry), pw = grid_pos(w, rz);
    const int su = span_search(nx, P, tx, pu);
    const int sv = span_search(ny, P, ty, pv);
    const int sw = span_search(nz, P, tz, pw);
    float xB[P + 1], xD[P + 1], yB[P + 1], yD[P + 1], zB[P + 1], zD[P + 1];
    basis_ders<P>(tx, su, pu, xB, xD);
    basis_ders<P>(ty, sv, pv, yB, yD);
    basis_ders<P>(tz, sw, pw, zB, zD);
    float f = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
    const float *base = ctrl + B.ctrl_off;
    for (int i = 0; i <= P; ++i) {
        for (int j = 0; j <= P; ++j) {
            for (int k = 0; k <= P; ++k) {
                const float c = base[((int64_t)(su - P + i) * ny + (sv - P + j)) * nz + (sw - P + k)];
                f += xB[i] * yB[j] * zB[k] * c;
                fx += xD[i] * yB[j] * zB[k] * c;
                fy += xB[i] * yD[j] * zB[k] * c;
                fz += xB[i] * yB[j] * zD[k] * c;
            }
        }
    }
    res[0] = f;
    res[1] = fx;
    res[2] = fy;
    res[3] = fz;
}

__global__ __launch_bounds__(256) void decode_plain_kernel(const fa_block *blocks, int b,
                                                           const float *knots,
                                                           const float *ctrl, int rx, int ry,
                                                           int rz, uint32_t mask, int nch,
                                                           float *out) {
    const int64_t vox = (int64_t)rx * ry * rz;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= vox) return;
    const int w = (int)(idx % rz);
    const int v = (int)((idx / rz) % ry);
    const int u = (int)(idx / ((int64_t)ry * rz));
    const fa_block &B = blocks[b];
    float res[4];
    const int p = B.degree[0];
    if (p == 3) plain_voxel<3>(B, knots, ctrl, u, v, w, rx, ry, rz, res);
    else if (p == 2) plain_voxel<2>(B, knots, ctrl, u, v, w, rx, ry, rz, res);
    else plain_voxel<1>(B, knots, ctrl, u, v, w, rx, ry, rz, res);
    float *o = out + (int64_t)b * nch * vox + idx;
    int c = 0;
    for (int ch = 0; ch < 4; ++ch) {
        if ((mask >> ch) & 1u) {
            o[(int64_t)c * vox] = res[ch];
            ++c;
        }
    }
}

// sumsq[b] = sum of block b's per-item partials, in item order
__global__ void residual_combine_kernel(const double *partials, int nblocks, int per,
                                        double *sumsq) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    double t = 0.0;
    for (int k = 0; k < per; ++k) t += partials[(int64_t)b * per + k];
    sumsq[b] = t;
}

// errs[b * stride + {0, 1}] = (max, sqrt(sum / vox)) of block b's per-item
// (max, sum of squares) partials, in item order
__global__ void errors_combine_kernel(const double *partials, int nblocks, int per, int64_t vox,
                                      float *errs, int64_t stride) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    double m = 0.0, t = 0.0;
    for (int k = 0; k < per; ++k) {
        m = fmax(m, partials[2 * ((int64_t)b * per + k)]);
        t += partials[2 * ((int64_t)b * per + k) + 1];
    }
    errs[(int64_t)b * stride] = (float)m;
    errs[(int64_t)b * stride + 1] = (float)sqrt(t / (double)vox);
}

}  // namespace

template <bool NT, int MODE>
hipError_t launch_sep(const DecodeLaunch &a, int waves, int grid, hipStream_t s) {
    const size_t lds = sep_lds_bytes(a.rx, a.slab);
    // raise the dynamic LDS limit once per process to the largest layout
    static const hipError_t attr = [] {
        const int most = (int)sep_lds_bytes(kMaxRes, kSlabMax);
        hipError_t r = hipSuccess, e;
        const void *ks[4] = {reinterpret_cast<const void *>(&decode_sep_kernel<1, NT, MODE>),
                             reinterpret_cast<const void *>(&decode_sep_kernel<2, NT, MODE>),
                             reinterpret_cast<const void *>(&decode_sep_kernel<4, NT, MODE>),
                             reinterpret_cast<const void *>(&decode_sep_kernel<8, NT, MODE>)};
        for (const void *k : ks)
            if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, most)) !=
                hipSuccess)
                r = e;
        return r;
    }();
    if (attr != hipSuccess) return attr;
    switch (waves) {
    case 2: hipLaunchKernelGGL((decode_sep_kernel<2, NT, MODE>), dim3(grid), dim3(128), lds, s, a); break;
    case 4: hipLaunchKernelGGL((decode_sep_kernel<4, NT, MODE>), dim3(grid), dim3(256), lds, s, a); break;
    case 8: hipLaunchKernelGGL((decode_sep_kernel<8, NT, MODE>), dim3(grid), dim3(512), lds, s, a); break;
    default: hipLaunchKernelGGL((decode_sep_kernel<1, NT, MODE>), dim3(grid), dim3(64), lds, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_decode_sep(const DecodeLaunch &a, int waves, int grid, hipStream_t s) {
    if (a.samples && a.errs) return launch_sep<false, 2>(a, waves, grid, s);
    if (a.interleave)
        return a.nt_store ? launch_sep<true, 3>(a, waves, grid, s)
                          : launch_sep<false, 3>(a, waves, grid, s);
    if (a.samples)
        return a.nt_store ? launch_sep<true, 1>(a, waves, grid, s)
                          : launch_sep<false, 1>(a, waves, grid, s);
    return a.nt_store ? launch_sep<true, 0>(a, waves, grid, s)
                      : launch_sep<false, 0>(a, waves, grid, s);
}

hipError_t launch_residual_combine(const double *partials, int nblocks, int per, double *sumsq,
                                   hipStream_t s) {
    hipLaunchKernelGGL(residual_combine_kernel, dim3((nblocks + 255) / 256), dim3(256), 0, s,
                       partials, nblocks, per, sumsq);
    return hipGetLastError();
}

hipError_t launch_errors_combine(const double *partials, int nblocks, int per, int64_t vox,
                                 float *errs, int64_t stride, hipStream_t s) {
    hipLaunchKernelGGL(errors_combine_kernel, dim3((nblocks + 255) / 256), dim3(256), 0, s,
                       partials, nblocks, per, vox, errs, stride);
    return hipGetLastError();
}

hipError_t launch_decode_plain(const fa_block *blocks, int nblocks, const float *knots,
                               const float *ctrl, int rx, int ry, int rz, uint32_t mask,
                               float *out, hipStream_t s) {
    const int64_t vox = (int64_t)rx * ry * rz;
    const int nch = __builtin_popcount(mask & 15u);
    const int grid = (int)((vox + 255) / 256);
    for (int b = 0; b < nblocks; ++b) {
        hipLaunchKernelGGL(decode_plain_kernel, dim3(grid), dim3(256), 0, s, blocks, b, knots,
                           ctrl, rx, ry, rz, mask, nch, out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fa
