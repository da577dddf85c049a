// Least-squares fit of micro-models to grid samples and its error map
// (the model(NCP, degree) step of the adaptive encoding, Sec. 4.2.1 and
// Alg. 1; Error(NCP) of Eq. 4).
//
// The design matrix of a block is the Kronecker product of the per-axis
// collocation matrices B_a[i][j] = N_j(u_i) on the decode grid, so the
// least-squares lattice is P = y x_1 X_x x_2 X_y x_3 X_z with the
// pseudo-inverses X_a = B_a^+ = (B_a^T B_a)^{-1} B_a^T (n_a x R_a).  Each X_a
// is built in FP64 inside the workgroup that needs it: the basis at the
// grid points in FP64 (same spans as the decode), the band Gram matrix
// B_a^T B_a (half-bandwidth p), its band Cholesky factor, and one
// forward/backward solve per grid point.  Forming X_a first and applying it
// as a dense contraction keeps the error proportional to the condition
// number of B_a, where solving the normal equations on B^T y would square
// it (the collocation matrix of NCP close to R on the uniform grid is
// badly conditioned).  Three kernels, FP64 throughout:
//   fit_pinv: X_a of every (block, axis), one workgroup each, into the
//           caller's workspace,
//   fit_z:  T[b][k][x][y] = sum_z X_z[k][z] y[b][x][y][z]   (chunks of 128
//           (x, y) lines staged in LDS, T in the workspace),
//   fit_xy: for each k, P[:, :, k] = X_x T[b][k] X_y^T        (one workgroup
//           per (block, group of k), the slice in LDS, X_x T in registers),
// the dense products of fit_z and fit_xy on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), and the lattice rounded to FP32 once.
// residual kernel: one workgroup per block reduces y - f to (max |r|,
// sqrt(mean r^2)) in a fixed order (deterministic).
#include <algorithm>

#include "fa_device.hpp"
#include "fa_internal.hpp"

namespace fa {
namespace {

constexpr int kFitThreads = 256;
constexpr int kFitR = 64;  // grid points per axis a fit supports
constexpr int kFitN = FA_MAX_NCP;

// FP64 basis of degree p <= 3 on span s: N[r] = N_{s-p+r,p}(u), triangular
// form of the de Boor recursion.
__device__ __forceinline__ void basis64(const float *t, int s, double u, int p, double (&N)[4]) {
    double left[4] = {0, 0, 0, 0}, right[4] = {0, 0, 0, 0};
    N[0] = 1.0;
    N[1] = N[2] = N[3] = 0.0;
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (k > p) break;
        left[k] = u - (double)t[s + 1 - k];
        right[k] = (double)t[s + k] - u;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < k; ++r) {
            const double q = N[r] / (right[r + 1] + left[k - r]);
            N[r] = saved + right[r + 1] * q;
            saved = left[k - r] * q;
        }
        N[k] = saved;
    }
}

struct PinvScratch {
    double N[kFitR][4];
    int span[kFitR];
    double G[kFitN][4];  // G[j][d] = G(j, j + d)
    double L[kFitN][4];  // L[j][d] = L(j, j - d)
};

// X = B^+ of one axis (n functions of degree p, knots t, R grid points),
// written as X[j * sj + i * si] for j < n, i < R.  All threads of the
// workgroup take part; ends with a barrier.
__device__ void build_pinv(PinvScratch &w, const float *t, int n, int p, int R, double *X,
                           int sj, int si) {
    const int tid = threadIdx.x;
    for (int i = tid; i < R; i += kFitThreads) {
        const float uf = grid_pos(i, R);
        const int s = span_search(n, p, t, uf);
        double Nv[4];
        basis64(t, s, (double)uf, p, Nv);
        w.span[i] = s;
#pragma unroll
        for (int r = 0; r < 4; ++r) w.N[i][r] = Nv[r];
    }
    __syncthreads();
    for (int e = tid; e < n * 4; e += kFitThreads) {
        const int j = e >> 2, d = e & 3;
        double g = 0.0;
        if (d <= p)
            for (int i = 0; i < R; ++i) {
                const int r = j - (w.span[i] - p);
                if (r >= 0 && r + d <= p) g += w.N[i][r] * w.N[i][r + d];
            }
        w.G[j][d] = g;
    }
    __syncthreads();
    if (tid == 0) {  // band Cholesky G = L L^T
        for (int j = 0; j < n; ++j) {
            for (int d = p; d >= 1; --d) {
                const int k = j - d;
                if (k < 0) {
                    w.L[j][d] = 0.0;
                    continue;
                }
                double v = w.G[k][d];
                for (int m = d + 1; m <= p; ++m)
                    if (j - m >= 0) v -= w.L[j][m] * w.L[k][m - d];
                w.L[j][d] = v / w.L[k][0];
            }
            double v = w.G[j][0];
            for (int d = 1; d <= p; ++d) v -= w.L[j][d] * w.L[j][d];
            w.L[j][0] = sqrt(v);
        }
    }
    __syncthreads();
    // column i of X solves G x = B[i, :]^T (non-zero at s_i - p .. s_i)
    for (int i = tid; i < R; i += kFitThreads) {
        const int j0 = w.span[i] - p;
        for (int j = 0; j < n; ++j) {  // forward: L z = rhs
            double v = (j >= j0 && j <= j0 + p) ? w.N[i][j - j0] : 0.0;
            if (j > j0)
                for (int d = 1; d <= p; ++d)
                    if (j - d >= j0) v -= w.L[j][d] * X[(j - d) * sj + i * si];
            X[j * sj + i * si] = j >= j0 ? v / w.L[j][0] : 0.0;
        }
        for (int j = n - 1; j >= 0; --j) {  // backward: L^T x = z
            double v = X[j * sj + i * si];
            for (int d = 1; d <= p; ++d)
                if (j + d < n) v -= w.L[j + d][d] * X[(j + d) * sj + i * si];
            X[j * sj + i * si] = v / w.L[j][0];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ const float *axis_knots(const float *knots, const fa_block &b, int a) {
    const float *t = knots + b.knot_off;
    if (a >= 1) t += b.ncp[0] + b.degree[0] + 1;
    if (a >= 2) t += b.ncp[1] + b.degree[1] + 1;
    return t;
}

constexpr int64_t kPinvStride = (int64_t)kFitN * kFitR;  // doubles per (block, axis)

struct PinvSmem {
    double X[kFitN][kFitR];
    PinvScratch w;
};

// Xg[(b * 3 + a) * kPinvStride + j * kFitR + i] = X_a[j][i]
__global__ __launch_bounds__(kFitThreads) void fit_pinv_kernel(const fa_block *blocks,
                                                               int nblocks, const float *knots,
                                                               int r0, int r1, int r2,
                                                               double *Xg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    PinvSmem &sm = *reinterpret_cast<PinvSmem *>(smem_raw);
    for (int64_t item = blockIdx.x; item < (int64_t)nblocks * 3; item += gridDim.x) {
        const int bi = (int)(item / 3), a = (int)(item - (int64_t)bi * 3);
        const fa_block b = blocks[bi];
        const int n = a == 0 ? b.ncp[0] : (a == 1 ? b.ncp[1] : b.ncp[2]);
        const int p = a == 0 ? b.degree[0] : (a == 1 ? b.degree[1] : b.degree[2]);
        const int Ra = a == 0 ? r0 : (a == 1 ? r1 : r2);
        build_pinv(sm.w, axis_knots(knots, b, a), n, p, Ra, &sm.X[0][0], kFitR, 1);
        double *dst = Xg + item * kPinvStride;
        for (int e = threadIdx.x; e < n * kFitR; e += kFitThreads) dst[e] = (&sm.X[0][0])[e];
        __syncthreads();
    }
}

// knot j of a clamped uniform vector: t_j = 0 (j <= p), 1 (j >= n), else
// fl32((j - p) / (n - p))
__device__ __forceinline__ float candidate_knot(int j, int n, int p) {
    if (j <= p) return 0.0f;
    if (j >= n) return 1.0f;
    return (float)(j - p) / (float)(n - p);
}

// The search's candidates share one knot vector per NCP (every block, every
// axis), so their pseudo-inverses are built once per (candidate, axis), all
// candidates in one launch: knots of candidate c (n = ncp_lo + c) at
// kall + c * kstride (x, y, z vectors back to back), X_a at
// xall + (c * 3 + a) * kPinvStride.
__global__ __launch_bounds__(kFitThreads) void pinv_candidates_kernel(float *kall, int ncp_lo,
                                                                      int ncand, int p,
                                                                      int kstride, int r0, int r1,
                                                                      int r2, double *xall) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    PinvSmem &sm = *reinterpret_cast<PinvSmem *>(smem_raw);
    for (int item = blockIdx.x; item < ncand * 3; item += gridDim.x) {
        const int c = item / 3, a = item - 3 * c, n = ncp_lo + c, nk = n + p + 1;
        float *t = kall + (int64_t)c * kstride + a * nk;
        for (int j = threadIdx.x; j < nk; j += kFitThreads) t[j] = candidate_knot(j, n, p);
        __syncthreads();
        const int Ra = a == 0 ? r0 : (a == 1 ? r1 : r2);
        build_pinv(sm.w, t, n, p, Ra, &sm.X[0][0], kFitR, 1);
        double *dst = xall + (int64_t)item * kPinvStride;
        for (int e = threadIdx.x; e < n * kFitR; e += kFitThreads) dst[e] = (&sm.X[0][0])[e];
        __syncthreads();
    }
}

// FP64 matrix-core contraction tiles: v_mfma_f64_16x16x4f64 takes
// A[l%16][l/16] and B[l/16][l%16] from lane l and returns D[4r + l/16][l%16]
// in component r (layout checked on the device).
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kXS = kFitR + 1;  // padded row of an LDS matrix (doubles)

constexpr int kZLines = 128;  // (x, y) lines per fit_z chunk: two workgroups per CU

struct FitZSmem {
    double X[kFitN][kXS];                 // X_z[k][z]
    float ys[kZLines][kFitR + 1];         // staged lines (padded)
};

// T[b][k][l] = sum_z X_z[k][z] y[b][l][z], l = x * R1 + y: per chunk of 128
// lines, a (n_z x R2) x (R2 x 128) product on the FP64 matrix cores.  A
// workgroup takes `cgroup` consecutive chunks of one block: X_z is staged
// once, and the next chunk's samples are loaded into registers while the
// products of the current one run.
constexpr int kZRegs = kZLines * kFitR / kFitThreads;  // chunk floats per thread

__global__ __launch_bounds__(kFitThreads) void fit_z_kernel(const fa_block *blocks, int nblocks,
                                                            const float *knots, int r0, int r1,
                                                            int r2, int max_n, int cgroup,
                                                            const float *y, const double *Xg,
                                                            int64_t xstride, double *T) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    FitZSmem &sm = *reinterpret_cast<FitZSmem *>(smem_raw);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t lines = (int64_t)r0 * r1;
    const int chunks = (int)((lines + kZLines - 1) / kZLines);
    const int groups = (chunks + cgroup - 1) / cgroup;
    for (int64_t item = blockIdx.x; item < (int64_t)nblocks * groups; item += gridDim.x) {
        const int bi = (int)(item / groups);
        const int c0 = (int)(item - (int64_t)bi * groups) * cgroup;
        const int c1 = min(chunks, c0 + cgroup);
        const fa_block b = blocks[bi];
        const int nz = b.ncp[2];
        if (nz > max_n) continue;  // the workspace has no room; the lattice is left as is
        __syncthreads();  // the previous item is done with the LDS
        const double *Xz = Xg + (int64_t)bi * xstride + 2 * kPinvStride;
        for (int e = tid; e < nz * kFitR; e += kFitThreads) {
            const int k = e / kFitR;
            sm.X[k][e - k * kFitR] = Xz[e];
        }
        // chunk c in registers: element e = tid + kFitThreads m of its cl x r2 samples
        float yv[kZRegs];
        auto fetch = [&](int c) {
            const int64_t l0 = (int64_t)c * kZLines;
            const int cl = (int)(lines - l0 < kZLines ? lines - l0 : kZLines);
            const float *yb = y + ((int64_t)bi * lines + l0) * r2;
#pragma unroll
            for (int m = 0; m < kZRegs; ++m) {
                const int e = tid + kFitThreads * m;
                yv[m] = (c < c1 && e < cl * r2) ? yb[e] : 0.0f;
            }
        };
        fetch(c0);
        const int mt = (nz + 15) >> 4, ksteps = (r2 + 3) >> 2;
        for (int c = c0; c < c1; ++c) {
            const int64_t l0 = (int64_t)c * kZLines;
            const int cl = (int)(lines - l0 < kZLines ? lines - l0 : kZLines);
            if (c > c0) __syncthreads();  // the previous chunk's products are done
#pragma unroll
            for (int m = 0; m < kZRegs; ++m) {
                const int e = tid + kFitThreads * m;
                if (e < cl * r2) {
                    const int li = e / r2;
                    sm.ys[li][e - li * r2] = yv[m];
                }
            }
            __syncthreads();
            fetch(c + 1);  // in flight during this chunk's products
            const int nt = (cl + 15) >> 4;
            const int nst = (nt + 3) >> 2;  // strips of 4 line tiles sharing the A operand
            double *Tb = T + (int64_t)bi * max_n * lines + l0;
            for (int unit = wave; unit < mt * nst; unit += kFitThreads / 64) {
                const int ti = unit / nst, tj0 = 4 * (unit - ti * nst);
                const int k = 16 * ti + lr;
                f64x4 acc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
                for (int ks = 0; ks < ksteps; ++ks) {
                    const int z = 4 * ks + lk;
                    const bool zok = z < r2;
                    const double av = (k < nz && zok) ? sm.X[k][z] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int li = 16 * (tj0 + q) + lr;
                        const double bv = (li < cl && zok) ? (double)sm.ys[li][z] : 0.0;
                        acc[q] = mfma64(av, bv, acc[q]);  // four independent chains
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int kk = 16 * ti + 4 * r + lk, ll = 16 * (tj0 + q) + lr;
                        if (kk < nz && ll < cl) Tb[(int64_t)kk * lines + ll] = acc[q][r];
                    }
            }
        }
    }
}

struct FitXYSmem {
    double Xy[kFitN][kXS];  // X_y[j][y]
    double S[kFitR][kXS];   // slice T[b][k] as [x][y]
};

// For each k: P[:, :, k] = X_x T[b][k] X_y^T, two products on the FP64
// matrix cores, one workgroup per (b, group of k), wave w owning rows
// 16w..16w+15 of P.  The first product is formed transposed, U^T = S^T X_x^T:
// its accumulator layout (row 4r + l/16, column l%16 in component r of lane
// l) is then exactly the A operand of the second product U X_y^T for the K
// steps 4t + r (t = the U^T tile), so U never leaves registers; the wave's
// X_x rows are held in registers as the B operand of the first product for
// every k of the group.  LDS holds X_y and the slice only (two workgroups
// per CU); the next k's slice is loaded into registers while the products
// of this one run, and the second product runs over the block's j tiles
// only (one straight-line instance per tile count).
constexpr int kSliceRegs = kFitR * kFitR / kFitThreads;  // slice doubles per thread

template <int NQ>
__device__ __forceinline__ void fit_xy_slice(const FitXYSmem &sm, int wave, int lr, int lk,
                                             int r0, int r1, int nx, int ny, int nz, int k,
                                             const double (&xb)[kFitR / 4], float *Pb) {
    constexpr int kKS = kFitR / 4;  // K steps of a 64-long contraction
    // U^T[yy][i] for the yy tiles t: A = S^T[yy][x] = S[x][yy]
    f64x4 u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    // every K step and tile runs (entries outside the slice are selected to
    // zero: no scalar conditions in the unrolled chains)
#pragma unroll
    for (int ks = 0; ks < kKS; ++ks) {
        const int x = 4 * ks + lk;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int yy = 16 * t + lr;
            const double sv = sm.S[x][yy];
            u[t] = mfma64((yy < r1 && x < r0) ? sv : 0.0, xb[ks], u[t]);
        }
    }
    // P[i][j] = sum_yy U[i][yy] X_y[j][yy]: A for K step 4t + r is component
    // r of u[t] (U[16 wave + l%16][4(4t + r) + l/16]), over the NQ j tiles
    f64x4 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int yy = 4 * (4 * t + r) + lk;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int j = 16 * q + lr;
                const double xv = sm.Xy[j][yy];
                acc[q] = mfma64(u[t][r], (j < ny && yy < r1) ? xv : 0.0, acc[q]);
            }
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = 16 * wave + 4 * r + lk, jj = 16 * q + lr;
            if (ii < nx && jj < ny) Pb[((int64_t)ii * ny + jj) * nz + k] = (float)acc[q][r];
        }
}

__global__ __launch_bounds__(kFitThreads) void fit_xy_kernel(const fa_block *blocks, int nblocks,
                                                             const float *knots, int r0, int r1,
                                                             int max_n, int kgroup,
                                                             const double *Xg, int64_t xstride,
                                                             const double *T, float *ctrl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    FitXYSmem &sm = *reinterpret_cast<FitXYSmem *>(smem_raw);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int kKS = kFitR / 4;  // K steps of a 64-long contraction
    const int lines = r0 * r1;
    const int groups = (max_n + kgroup - 1) / kgroup;
    for (int64_t item = blockIdx.x; item < (int64_t)nblocks * groups; item += gridDim.x) {
        const int bi = (int)(item / groups);
        const int k0 = (int)(item - (int64_t)bi * groups) * kgroup;
        const fa_block b = blocks[bi];
        const int nx = b.ncp[0], ny = b.ncp[1], nz = b.ncp[2];
        if (k0 >= nz || nz > max_n) continue;
        const double *Xx = Xg + (int64_t)bi * xstride;
        const double *Xy = Xx + kPinvStride;
        for (int e = tid; e < ny * kFitR; e += kFitThreads) {
            const int j = e / kFitR;
            sm.Xy[j][e - j * kFitR] = Xy[e];
        }
        // B operand of U^T = S^T X_x^T: X_x[i][x], i = 16 wave + l%16, x = 4 ks + l/16
        const int i = 16 * wave + lr;
        const bool rows = 16 * wave < nx;  // the wave has rows of P
        double xb[kKS];
#pragma unroll
        for (int ks = 0; ks < kKS; ++ks) {
            const int x = 4 * ks + lk;
            xb[ks] = (i < nx && x < r0) ? Xx[(int64_t)i * kFitR + x] : 0.0;
        }
        float *Pb = ctrl + b.ctrl_off;
        const int k1 = min(nz, k0 + kgroup);
        const int nq = (ny + 15) >> 4;
        // slice k in registers: element e = tid + kFitThreads m of the r0 x r1 slice
        double sv[kSliceRegs];
        auto fetch = [&](int k) {
            const double *Tk = T + ((int64_t)bi * max_n + k) * lines;
#pragma unroll
            for (int m = 0; m < kSliceRegs; ++m) {
                const int e = tid + kFitThreads * m;
                sv[m] = (k < k1 && e < lines) ? Tk[e] : 0.0;
            }
        };
        fetch(k0);
        for (int k = k0; k < k1; ++k) {
#pragma unroll
            for (int m = 0; m < kSliceRegs; ++m) {
                const int e = tid + kFitThreads * m;
                if (e < lines) {
                    const int x = e / r1;
                    sm.S[x][e - x * r1] = sv[m];
                }
            }
            __syncthreads();
            fetch(k + 1);  // in flight during this slice's products
            if (rows) {
                if (nq >= 4) fit_xy_slice<4>(sm, wave, lr, lk, r0, r1, nx, ny, nz, k, xb, Pb);
                else if (nq == 3) fit_xy_slice<3>(sm, wave, lr, lk, r0, r1, nx, ny, nz, k, xb, Pb);
                else if (nq == 2) fit_xy_slice<2>(sm, wave, lr, lk, r0, r1, nx, ny, nz, k, xb, Pb);
                else fit_xy_slice<1>(sm, wave, lr, lk, r0, r1, nx, ny, nz, k, xb, Pb);
            }
            __syncthreads();
        }
    }
}

// errs[b * stride + 0] = max |y - f|, errs[b * stride + 1] = sqrt(mean (y-f)^2).
// With chunks > 1 a block's voxels are split into `chunks` equal ranges,
// each reduced by its own workgroup into part[(b * chunks + c) * 2 + {0,1}]
// (max, sum of squares), and combine_kernel finishes the block in a fixed
// order (deterministic either way).
__global__ __launch_bounds__(kFitThreads) void residual_kernel(const float *y, const float *f,
                                                                int64_t vox, int nblocks,
                                                                int chunks, double *part,
                                                                float *errs, int64_t stride) {
    __shared__ float smax[kFitThreads];
    __shared__ double ssum[kFitThreads];
    const int tid = threadIdx.x;
    const int64_t cv = (vox / chunks + 3) / 4 * 4;  // voxels per chunk, a multiple of 4
    for (int64_t item = blockIdx.x; item < (int64_t)nblocks * chunks; item += gridDim.x) {
        const int bi = (int)(item / chunks), c = (int)(item - (int64_t)bi * chunks);
        const int64_t v0 = (int64_t)c * cv;
        const int64_t v1 = c == chunks - 1 ? vox : (v0 + cv < vox ? v0 + cv : vox);
        const float *yb = y + (int64_t)bi * vox;
        const float *fb = f + (int64_t)bi * vox;
        float m = 0.0f;
        double s = 0.0;
        if ((vox & 3) == 0) {
            const float4 *y4 = reinterpret_cast<const float4 *>(yb);
            const float4 *f4 = reinterpret_cast<const float4 *>(fb);
            for (int64_t i = v0 / 4 + tid; i < v1 / 4; i += kFitThreads) {
                const float4 a = y4[i], cc = f4[i];
                const float r0 = a.x - cc.x, r1 = a.y - cc.y, r2 = a.z - cc.z, r3 = a.w - cc.w;
                m = fmaxf(m, fmaxf(fmaxf(fabsf(r0), fabsf(r1)), fmaxf(fabsf(r2), fabsf(r3))));
                s += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2 + (double)r3 * r3;
            }
        } else {
            for (int64_t i = v0 + tid; i < v1; i += kFitThreads) {
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
            if (chunks == 1) {
                errs[(int64_t)bi * stride] = smax[0];
                errs[(int64_t)bi * stride + 1] = (float)sqrt(ssum[0] / (double)vox);
            } else {
                part[item * 2] = (double)smax[0];
                part[item * 2 + 1] = ssum[0];
            }
        }
        __syncthreads();
    }
}

__global__ void combine_kernel(const double *part, int chunks, int64_t vox, int nblocks,
                               float *errs, int64_t stride) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= nblocks) return;
    double m = 0.0, s = 0.0;
    for (int c = 0; c < chunks; ++c) {
        m = fmax(m, part[((int64_t)bi * chunks + c) * 2]);
        s += part[((int64_t)bi * chunks + c) * 2 + 1];
    }
    errs[(int64_t)bi * stride] = (float)m;
    errs[(int64_t)bi * stride + 1] = (float)sqrt(s / (double)vox);
}

// Least-squares loss of a fit and its cotangent in one pass (the residual
// step between the forward decode and the adjoint): per block b,
//   grad[b][v] = scale * (f[b][v] - y[b][v]),  sumsq[b] = sum_v (f - y)^2
// (FP64 sum, fixed order).
__global__ __launch_bounds__(kFitThreads) void mse_grad_kernel(const float *f, const float *y,
                                                                int64_t vox, int nblocks,
                                                                float scale, float *grad,
                                                                double *sumsq) {
    __shared__ double ssum[kFitThreads];
    const int tid = threadIdx.x;
    for (int bi = blockIdx.x; bi < nblocks; bi += gridDim.x) {
        const int64_t o = (int64_t)bi * vox;
        double acc = 0.0;
        if ((vox & 3) == 0) {
            const f32x4 *f4 = reinterpret_cast<const f32x4 *>(f + o);
            const f32x4 *y4 = reinterpret_cast<const f32x4 *>(y + o);
            f32x4 *g4 = reinterpret_cast<f32x4 *>(grad + o);
            for (int64_t i = tid; i < vox / 4; i += kFitThreads) {
                const f32x4 a = __builtin_nontemporal_load(f4 + i);
                const f32x4 c = __builtin_nontemporal_load(y4 + i);
                const f32x4 r = a - c;
                acc += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z +
                       (double)r.w * r.w;
                g4[i] = r * scale;
            }
        } else {
            for (int64_t i = tid; i < vox; i += kFitThreads) {
                const float r = f[o + i] - y[o + i];
                acc += (double)r * r;
                grad[o + i] = r * scale;
            }
        }
        ssum[tid] = acc;
        __syncthreads();
        for (int w = kFitThreads / 2; w > 0; w >>= 1) {
            if (tid < w) ssum[tid] += ssum[tid + w];
            __syncthreads();
        }
        if (tid == 0) sumsq[bi] = ssum[0];
        __syncthreads();
    }
}

// Descriptors and shared knots of one candidate NCP (same n and p on every
// axis, clamped uniform knots t_{p+j} = j / (n - p)); lattices at `cstride`.
__global__ void candidate_kernel(fa_block *desc, float *knots, int nblocks, int n, int p,
                                 int64_t cstride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nk = n + p + 1;
    if (i < 3 * nk) knots[i] = candidate_knot(i % nk, n, p);
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

int64_t fit_workspace_bytes(int nblocks, int rx, int ry, int max_n) {
    return ((int64_t)nblocks * max_n * rx * ry + (int64_t)nblocks * 3 * kPinvStride) *
           (int64_t)sizeof(double);
}

namespace {
// raise the dynamic LDS limits of the fit kernels once per process
hipError_t fit_attributes() {
    static const hipError_t attr = [] {
        const void *ks[4] = {reinterpret_cast<const void *>(&fit_z_kernel),
                             reinterpret_cast<const void *>(&fit_xy_kernel),
                             reinterpret_cast<const void *>(&fit_pinv_kernel),
                             reinterpret_cast<const void *>(&pinv_candidates_kernel)};
        const int bytes[4] = {(int)sizeof(FitZSmem), (int)sizeof(FitXYSmem),
                              (int)sizeof(PinvSmem), (int)sizeof(PinvSmem)};
        hipError_t r = hipSuccess;
        for (int i = 0; i < 4; ++i) {
            const hipError_t e =
                hipFuncSetAttribute(ks[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[i]);
            if (e != hipSuccess) r = e;
        }
        return r;
    }();
    return attr;
}

// the two products of a fit given the pseudo-inverses: block b's X_a at
// X + b * xstride + a * kPinvStride
hipError_t launch_fit_products(const fa_block *blocks, int nblocks, const float *knots, int rx,
                               int ry, int rz, int max_n, const float *samples, double *T,
                               const double *X, int64_t xstride, float *ctrl, hipStream_t s) {
    const int64_t chunks = ((int64_t)rx * ry + kZLines - 1) / kZLines;
    // chunks per workgroup: as many as leave about 512 workgroups (two per CU)
    const int cgroup =
        (int)std::max<int64_t>(1, std::min<int64_t>(chunks, (int64_t)nblocks * chunks / 512));
    const int64_t zitems = (int64_t)nblocks * ((chunks + cgroup - 1) / cgroup);
    const int gz = (int)std::min<int64_t>(zitems, 65536);
    hipLaunchKernelGGL(fit_z_kernel, dim3(gz), dim3(kFitThreads), sizeof(FitZSmem), s, blocks,
                       nblocks, knots, rx, ry, rz, max_n, cgroup, samples, X, xstride, T);
    // k values per workgroup: as many as keep about 2048 workgroups busy
    const int kgroup = (int)std::max<int64_t>(1, std::min<int64_t>(max_n, (int64_t)nblocks * max_n / 2048));
    const int64_t groups = (max_n + kgroup - 1) / kgroup;
    const int gxy = (int)std::min<int64_t>((int64_t)nblocks * groups, 65536);
    hipLaunchKernelGGL(fit_xy_kernel, dim3(gxy), dim3(kFitThreads), sizeof(FitXYSmem), s, blocks,
                       nblocks, knots, rx, ry, max_n, kgroup, X, xstride, T, ctrl);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fit(const fa_block *blocks, int nblocks, const float *knots, int rx, int ry,
                      int rz, int max_n, const float *samples, double *T, float *ctrl,
                      hipStream_t s) {
    const hipError_t attr = fit_attributes();
    if (attr != hipSuccess) return attr;
    double *Xg = T + (int64_t)nblocks * max_n * rx * ry;
    const int gp = (int)std::min<int64_t>((int64_t)nblocks * 3, 65536);
    hipLaunchKernelGGL(fit_pinv_kernel, dim3(gp), dim3(kFitThreads), sizeof(PinvSmem), s, blocks,
                       nblocks, knots, rx, ry, rz, Xg);
    return launch_fit_products(blocks, nblocks, knots, rx, ry, rz, max_n, samples, T, Xg,
                               3 * kPinvStride, ctrl, s);
}

int64_t pinv_doubles() { return kPinvStride; }

hipError_t launch_pinv_candidates(float *kall, int ncp_lo, int ncand, int p, int kstride, int rx,
                                  int ry, int rz, double *xall, hipStream_t s) {
    const hipError_t attr = fit_attributes();
    if (attr != hipSuccess) return attr;
    const int grid = std::min(ncand * 3, 65536);
    hipLaunchKernelGGL(pinv_candidates_kernel, dim3(grid), dim3(kFitThreads), sizeof(PinvSmem), s,
                       kall, ncp_lo, ncand, p, kstride, rx, ry, rz, xall);
    return hipGetLastError();
}

hipError_t launch_fit_shared(const fa_block *blocks, int nblocks, const float *knots, int rx,
                             int ry, int rz, int max_n, const float *samples, double *T,
                             const double *X, float *ctrl, hipStream_t s) {
    const hipError_t attr = fit_attributes();
    if (attr != hipSuccess) return attr;
    return launch_fit_products(blocks, nblocks, knots, rx, ry, rz, max_n, samples, T, X, 0, ctrl,
                               s);
}

hipError_t launch_residual(const float *y, const float *f, int64_t vox, int nblocks, float *errs,
                           int64_t stride, hipStream_t s, int chunks, double *part) {
    if (chunks < 1 || !part) chunks = 1;
    const int64_t items = (int64_t)nblocks * chunks;
    const int grid = (int)(items < 65536 ? items : 65536);
    hipLaunchKernelGGL(residual_kernel, dim3(grid), dim3(kFitThreads), 0, s, y, f, vox, nblocks,
                       chunks, part, errs, stride);
    if (chunks > 1)
        hipLaunchKernelGGL(combine_kernel, dim3((nblocks + 255) / 256), dim3(256), 0, s, part,
                           chunks, vox, nblocks, errs, stride);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float *f, const float *y, int64_t vox, int nblocks, float scale,
                           float *grad, double *sumsq, hipStream_t s) {
    const int grid = nblocks < 65536 ? nblocks : 65536;
    hipLaunchKernelGGL(mse_grad_kernel, dim3(grid), dim3(kFitThreads), 0, s, f, y, vox, nblocks,
                       scale, grad, sumsq);
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
