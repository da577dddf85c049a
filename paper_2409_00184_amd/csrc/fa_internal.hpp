// Launchers shared between the C ABI (fa_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fa.h"

namespace fa {

constexpr int kWaveLanes = 64;
constexpr int kSlabDefault = 8192;  // LDS lattice slab of the separable decode (floats)
constexpr int kSlabMin = 4096;      // >= NCP_y * NCP_z of any block: one x plane fits
constexpr int kSlabMax = 16384;
constexpr int kMaxRes = FA_MAX_RES;
constexpr int kMfmaRows = 16;      // y rows per work item of the matrix-core decode

struct DecodeLaunch {
    const fa_block *blocks;
    const float *knots;
    const void *ctrl;
    int dtype;
    int rx, ry, rz;
    uint32_t mask;
    int nch;
    const fa_work *work;     // may be null: default order
    const int32_t *wg_off;
    int rows;                // rows per item in default order
    int nrowt, ncolt;        // tiles per block (default order)
    int64_t nitems;          // items in default order
    int slab;                // LDS slab floats
    int nt_store;            // 1: non-temporal stores
    float *out;
    // residual form (value channel only, FP32): out = gscale * (f - samples),
    // per-item FP64 sums of (f - samples)^2 into partials[item]
    const float *samples;    // null: plain decode
    float gscale;
    double *partials;
    // error form (samples set, errs set, nothing stored per voxel): per-item
    // max |f - samples| and FP64 sum of squares into partials[2 item + {0,1}]
    float *errs;
    int64_t errs_stride;
    // decode form: all four channels stored as one 16-byte record per voxel,
    // out = [block][u][v][w][4]
    int interleave;
};

hipError_t launch_decode_sep(const DecodeLaunch &a, int waves, int grid, hipStream_t s);
hipError_t launch_decode_mfma(const DecodeLaunch &a, int waves, int grid, hipStream_t s);
// per-block sums of the per-item partials of the residual decode
hipError_t launch_residual_combine(const double *partials, int nblocks, int per, double *sumsq,
                                   hipStream_t s);
// errs[b * stride + {0, 1}] = (max, rms) of block b from the error form's
// per-item partials, items in order
hipError_t launch_errors_combine(const double *partials, int nblocks, int per, int64_t vox,
                                 float *errs, int64_t stride, hipStream_t s);
hipError_t launch_decode_plain(const fa_block *blocks, int nblocks, const float *knots,
                               const float *ctrl, int rx, int ry, int rz, uint32_t mask,
                               float *out, hipStream_t s);

struct QueryLaunch {
    const fa_block *blocks;
    int nblocks;
    const int32_t *block_of_cell;
    int nb[3];
    float origin[3];
    float rscale[3];  // (float)nb / extent
    const float *knots;
    const void *ctrl;
    int dtype;
    const float *xyz;
    int64_t n;
    uint32_t mask;
    float *out;
    // ray-structured order (0 = flat list): positions are [rh][rw][rk]
    int rw, rh, rk;
};

hipError_t launch_query(const QueryLaunch &a, hipStream_t s);

hipError_t launch_render(const QueryLaunch &q, const fa_ray *rays, int width, int height,
                         const fa_render_params &p, const float *tf, float *image,
                         hipStream_t s);

hipError_t launch_visible(const fa_ray *rays, int64_t nrays, int samples, const int nb[3],
                          const float origin[3], const float rscale[3], int32_t *flags,
                          hipStream_t s);

hipError_t launch_adjoint(const fa_block *blocks, int nblocks, const float *knots, int rx,
                          int ry, int rz, uint32_t mask, const float *g, float *G, int it,
                          hipStream_t s);
// value-channel cotangent only (mask 1), on the FP32 matrix cores
hipError_t launch_adjoint_value(const fa_block *blocks, int nblocks, const float *knots, int rx,
                                int ry, int rz, const float *g, float *G, hipStream_t s);

int64_t fit_workspace_bytes(int nblocks, int rx, int ry, int max_n);
hipError_t launch_fit(const fa_block *blocks, int nblocks, const float *knots, int rx, int ry,
                      int rz, int max_n, const float *samples, double *T, float *ctrl,
                      hipStream_t s);
hipError_t launch_residual(const float *y, const float *f, int64_t vox, int nblocks, float *errs,
                           int64_t stride, hipStream_t s, int chunks = 1, double *part = nullptr);
hipError_t launch_mse_grad(const float *f, const float *y, int64_t vox, int nblocks, float scale,
                           float *grad, double *sumsq, hipStream_t s);
hipError_t launch_candidate(fa_block *desc, float *knots, int nblocks, int n, int p,
                            int64_t cstride, hipStream_t s);
// doubles of one (block or candidate, axis) pseudo-inverse
int64_t pinv_doubles();
// knots and per-axis pseudo-inverses of every candidate NCP ncp_lo + c,
// c < ncand, of a search (clamped uniform knots shared by all blocks):
// knots at kall + c * kstride, X_a at xall + (3 c + a) * pinv_doubles()
hipError_t launch_pinv_candidates(float *kall, int ncp_lo, int ncand, int p, int kstride, int rx,
                                  int ry, int rz, double *xall, hipStream_t s);
// launch_fit with one set of pseudo-inverses X (3 axes) shared by every block
hipError_t launch_fit_shared(const fa_block *blocks, int nblocks, const float *knots, int rx,
                             int ry, int rz, int max_n, const float *samples, double *T,
                             const double *X, float *ctrl, hipStream_t s);

// One block of a staging gather: its slot in the mapped host cache, where
// its knots and lattice go in the device batch, and its descriptor.
struct StageEntry {
    int64_t slot_off;  // floats from the start of the slots
    int64_t kdst;      // knot destination (floats)
    int64_t cdst;      // lattice destination (floats, multiple of 64)
    int64_t cl;        // lattice floats
    int32_t kl;        // knot floats
    int32_t koff;      // lattice offset inside the slot (floats, multiple of 4)
    int32_t dst;       // descriptor index in the batch
    int32_t pad;
    fa_block desc;
};

hipError_t launch_stage_gather(const StageEntry *table, int n, const float *slots,
                               fa_block *dev_blocks, float *dev_knots, float *dev_ctrl,
                               hipStream_t s);

hipError_t launch_quantize(fa_block *blocks, int nblocks, const float *ctrl, int dtype,
                           void *out, hipStream_t s);

// loss[0] = (float)(sum of sumsq[0..nblocks) / count), fixed order
hipError_t launch_mse_loss(const double *sumsq, int nblocks, double count, float *loss,
                           hipStream_t s);

// one Adam step (state: device float[3] = {t, 1 - b1^t, sqrt(1 - b2^t)}, advanced first)
hipError_t launch_adam(float *param, const float *grad, float *exp_avg, float *exp_avg_sq,
                       int64_t n, float lr, float beta1, float beta2, float eps, float wd,
                       float *state, hipStream_t s);

}  // namespace fa
