// Least-squares fit of micro-models to grid samples and its error map
// (the model(NCP, degree) step of the adaptive encoding, Sec. 4.2.1 and
// Alg. 1; Error(NCP) of Eq. 4).
//
// The design matrix of a block is the Kronecker product of the per-axis
// collocation matrices B_a[i][j] = N_j(u_i) on the decode grid, so the
// least-squares lattice is P = y x_1 B_x^+ x_2 B_y^+ x_3 B_z^+ with
// B_a^+ = (B_a^T B_a)^{-1} B_a^T.  The B^T part is exactly the decode
// adjoint (fa_adjoint.hip, value channel); what remains is a solve with the
// Gram matrix G_a = B_a^T B_a along every axis.  G_a is symmetric positive
// definite (full column rank when res >= ncp on the uniform grid) and
// banded with half-bandwidth p (two degree-p B-splines overlap only when
// their indices differ by at most p), so a band Cholesky factor of at most
// 64 x 4 entries, built per block in FP64 from the same FP32 basis values
// the decode uses, serves every line of the axis.
//
// solve kernel: one workgroup per block; per axis, the factor is built in
// LDS, then the lattice lines along that axis are solved in chunks of 256
// lines staged in LDS in FP64 (one rounding to FP32 per axis pass).
// residual kernel: one workgroup per block reduces y - f to (max |r|,
// sqrt(mean r^2)) in a fixed order (deterministic).
#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

constexpr int kFitThreads = 256;
constexpr int kFitLines = 256;  // lattice lines per LDS chunk
constexpr int kFitMaxN = FA_MAX_NCP;

struct FitSmem {
    double x[kFitMaxN][kFitLines];  // x[j][line]: chunk of lines along the axis
    double L[kFitMaxN][4];          // band Cholesky factor: L[j][d] = L(j, j - d)
    double G[kFitMaxN][4];          // band Gram matrix: G[j][d] = G(j, j + d)
    float N[kMaxRes][4];            // basis at the grid points of the axis
    int span[kMaxRes];
};

__global__ __launch_bounds__(kFitThreads) void fit_solve_kernel(const fa_block *blocks,
                                                                 int nblocks, const float *knots,
                                                                 int r0, int r1, int r2,
                                                                 float *ctrl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    FitSmem &sm = *reinterpret_cast<FitSmem *>(smem_raw);
    const int tid = threadIdx.x;
    for (int bi = blockIdx.x; bi < nblocks; bi += gridDim.x) {
        const fa_block b = blocks[bi];
        const int n[3] = {b.ncp[0], b.ncp[1], b.ncp[2]};
        const int R[3] = {r0, r1, r2};
        const float *tb = knots + b.knot_off;
        float *P = ctrl + b.ctrl_off;
        for (int a = 0; a < 3; ++a) {
            const int na = n[a], p = b.degree[a], Ra = R[a];
            const float *t = tb + (a >= 1 ? n[0] + b.degree[0] + 1 : 0) +
                             (a >= 2 ? n[1] + b.degree[1] + 1 : 0);
            // basis of the axis at the decode grid (the decode's FP32 values)
            for (int i = tid; i < Ra; i += kFitThreads) {
                const float u = grid_pos(i, Ra);
                const int s = span_search(na, p, t, u);
                float Nv[4], Dv[4];
                basis_ders_rt(t, s, u, p, Nv, Dv);
                sm.span[i] = s;
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.N[i][r] = Nv[r];
            }
            __syncthreads();
            // band Gram matrix G(j, j+d) = sum_i N_j(u_i) N_{j+d}(u_i), FP64
            for (int e = tid; e < na * 4; e += kFitThreads) {
                const int j = e >> 2, d = e & 3;
                double g = 0.0;
                if (d <= p) {
                    for (int i = 0; i < Ra; ++i) {
                        const int s0 = sm.span[i] - p;  // first non-zero function at u_i
                        const int r = j - s0;
                        if (r >= 0 && r + d <= p) g += (double)sm.N[i][r] * (double)sm.N[i][r + d];
                    }
                }
                sm.G[j][d] = g;
            }
            __syncthreads();
            // band Cholesky G = L L^T (sequential, at most 64 x 4 entries)
            if (tid == 0) {
                for (int j = 0; j < na; ++j) {
                    for (int d = p; d >= 1; --d) {  // L(j, j-d)
                        const int k = j - d;
                        if (k < 0) {
                            sm.L[j][d] = 0.0;
                            continue;
                        }
                        double v = sm.G[k][d];  // G(k, j) = G(j, k)
                        for (int m = d + 1; m <= p; ++m)  // sum_c L(j, c) L(k, c), c = j - m
                            if (j - m >= 0) v -= sm.L[j][m] * sm.L[k][m - d];
                        sm.L[j][d] = v / sm.L[k][0];
                    }
                    double v = sm.G[j][0];
                    for (int d = 1; d <= p; ++d) v -= sm.L[j][d] * sm.L[j][d];
                    sm.L[j][0] = sqrt(v);
                }
            }
            __syncthreads();
            // lines along axis a: element j of line l sits at base(l) + j * stride
            const int64_t nyz = (int64_t)n[1] * n[2];
            const int64_t nlines = (int64_t)n[0] * n[1] * n[2] / na;
            const int64_t stride = a == 0 ? nyz : (a == 1 ? n[2] : 1);
            auto base = [&](int64_t l) -> int64_t {
                if (a == 0) return l;
                if (a == 1) return (l / n[2]) * nyz + (l % n[2]);
                return l * n[2];
            };
            for (int64_t l0 = 0; l0 < nlines; l0 += kFitLines) {
                const int cl = (int)(nlines - l0 < kFitLines ? nlines - l0 : kFitLines);
                // load (global addresses contiguous across threads)
                for (int e = tid; e < cl * na; e += kFitThreads) {
                    int li, j;
                    if (a == 2) {
                        li = e / na;
                        j = e - li * na;
                    } else {
                        j = e / cl;
                        li = e - j * cl;
                    }
                    sm.x[j][li] = (double)P[base(l0 + li) + j * stride];
                }
                __syncthreads();
                if (tid < cl) {
                    // forward: L z = rhs
                    for (int j = 0; j < na; ++j) {
                        double v = sm.x[j][tid];
                        for (int d = 1; d <= p; ++d)
                            if (j - d >= 0) v -= sm.L[j][d] * sm.x[j - d][tid];
                        sm.x[j][tid] = v / sm.L[j][0];
                    }
                    // backward: L^T x = z
                    for (int j = na - 1; j >= 0; --j) {
                        double v = sm.x[j][tid];
                        for (int d = 1; d <= p; ++d)
                            if (j + d < na) v -= sm.L[j + d][d] * sm.x[j + d][tid];
                        sm.x[j][tid] = v / sm.L[j][0];
                    }
                }
                __syncthreads();
                for (int e = tid; e < cl * na; e += kFitThreads) {
                    int li, j;
                    if (a == 2) {
                        li = e / na;
                        j = e - li * na;
                    } else {
                        j = e / cl;
                        li = e - j * cl;
                    }
                    P[base(l0 + li) + j * stride] = (float)sm.x[j][li];
                }
                __syncthreads();
            }
        }
    }
}

// errs[b * stride + 0] = max |y - f|, errs[b * stride + 1] = sqrt(mean (y-f)^2)
__global__ __launch_bounds__(kFitThreads) void residual_kernel(const float *y, const float *f,
                                                                int64_t vox, int nblocks,
                                                                float *errs, int64_t stride) {
    __shared__ float smax[kFitThreads];
    __shared__ double ssum[kFitThreads];
    const int tid = threadIdx.x;
    for (int bi = blockIdx.x; bi < nblocks; bi += gridDim.x) {
        const float *yb = y + (int64_t)bi * vox;
        const float *fb = f + (int64_t)bi * vox;
        float m = 0.0f;
        double s = 0.0;
        if ((vox & 3) == 0) {
            const float4 *y4 = reinterpret_cast<const float4 *>(yb);
            const float4 *f4 = reinterpret_cast<const float4 *>(fb);
            for (int64_t i = tid; i < vox / 4; i += kFitThreads) {
                const float4 a = y4[i], c = f4[i];
                const float r0 = a.x - c.x, r1 = a.y - c.y, r2 = a.z - c.z, r3 = a.w - c.w;
                m = fmaxf(m, fmaxf(fmaxf(fabsf(r0), fabsf(r1)), fmaxf(fabsf(r2), fabsf(r3))));
                s += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2 + (double)r3 * r3;
            }
        } else {
            for (int64_t i = tid; i < vox; i += kFitThreads) {
                const float r = yb[i] - fb[i];
                m = fmaxf(m, fabsf(r));
                s += (double)r * r;
            }
        }
        smax[tid] = m;
        ssum[tid] = s;
        __syncthreads();
        for (int w = kFitThreads / 2; w > 0; w >>= 1) {
            if (tid < w) {
                smax[tid] = fmaxf(smax[tid], smax[tid + w]);
                ssum[tid] += ssum[tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            errs[(int64_t)bi * stride] = smax[0];
            errs[(int64_t)bi * stride + 1] = (float)sqrt(ssum[0] / (double)vox);
        }
        __syncthreads();
    }
}

// Descriptors and shared knots of one candidate NCP (same n and p on every
// axis, clamped uniform knots t_{p+j} = j / (n - p)); lattices at `cstride`.
__global__ void candidate_kernel(fa_block *desc, float *knots, int nblocks, int n, int p,
                                 int64_t cstride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nk = n + p + 1;
    if (i < 3 * nk) {
        const int j = i % nk;
        float v;
        if (j <= p) v = 0.0f;
        else if (j >= n) v = 1.0f;
        else v = (float)(j - p) / (float)(n - p);
        knots[i] = v;
    }
    if (i < nblocks) {
        fa_block d{};
        d.ncp[0] = d.ncp[1] = d.ncp[2] = n;
        d.degree[0] = d.degree[1] = d.degree[2] = p;
        d.knot_off = 0;
        d.ctrl_off = (int64_t)i * cstride;
        d.scale = 1.0f;
        d.flags = FA_FLAG_UNIFORM_X | FA_FLAG_UNIFORM_Y | FA_FLAG_UNIFORM_Z;
        desc[i] = d;
    }
}

}  // namespace

hipError_t launch_fit_solve(const fa_block *blocks, int nblocks, const float *knots, int rx,
                            int ry, int rz, float *ctrl, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fit_solve_kernel),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(FitSmem));
    if (attr != hipSuccess) return attr;
    const int grid = nblocks < 65536 ? nblocks : 65536;
    hipLaunchKernelGGL(fit_solve_kernel, dim3(grid), dim3(kFitThreads), sizeof(FitSmem), s,
                       blocks, nblocks, knots, rx, ry, rz, ctrl);
    return hipGetLastError();
}

hipError_t launch_residual(const float *y, const float *f, int64_t vox, int nblocks, float *errs,
                           int64_t stride, hipStream_t s) {
    const int grid = nblocks < 65536 ? nblocks : 65536;
    hipLaunchKernelGGL(residual_kernel, dim3(grid), dim3(kFitThreads), 0, s, y, f, vox, nblocks,
                       errs, stride);
    return hipGetLastError();
}

hipError_t launch_candidate(fa_block *desc, float *knots, int nblocks, int n, int p,
                            int64_t cstride, hipStream_t s) {
    const int cnt = nblocks > 3 * (n + p + 1) ? nblocks : 3 * (n + p + 1);
    hipLaunchKernelGGL(candidate_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, desc, knots,
                       nblocks, n, p, cstride);
    return hipGetLastError();
}

}  // namespace fa
