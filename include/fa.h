/*
 * fa.h -- C ABI of the MI355X (gfx950) micro-model decode/query library.
 *
 * A micro-model (paper Sec. 4.2, Eq. 2 and the micro-model layout figure)
 * is a clamped tensor-product B-spline over one micro-block: three knot
 * vectors plus an NCP_x x NCP_y x NCP_z lattice of control points.  The
 * renderer of Alg. 4 queries it through valueMicroModel(x,y,z) and
 * gradientMicroModel(x,y,z); this library evaluates both, for whole
 * batches of micro-models of uneven NCP* (Sec. 4.2.1, Eq. 4), either on a
 * voxel grid per block (fa_decode_blocks) or at arbitrary sample positions
 * of a tiled domain (fa_query_points), and provides the adjoint of the grid
 * decode (fa_decode_backward), i.e. the gradient of a least-squares fit of
 * the control points (the fit that Alg. 1 runs for every candidate NCP).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Parameter domain of a block: [0,1]^3.  Knots are clamped: the first
 *    p+1 knots of an axis are 0, the last p+1 are 1, interior knots are
 *    non-decreasing, and every knot span used has positive length.
 *  - Span rule: the span of u is the largest s in [p, n-1] with t_s <= u;
 *    u = 1 belongs to the last span (n-1).
 *  - Lattice layout: C order [x][y][z] (z fastest); element (i,j,k) of
 *    block b is ctrl[ctrl_off + (i*ncp_y + j)*ncp_z + k].
 *  - Knot layout: knots[knot_off ...] holds the x knots (ncp_x+p+1 values),
 *    then the y knots, then the z knots, FP32.
 *  - Decode grid: voxel i of an axis of resolution R sits at the FP32
 *    value (float)i / (float)(R-1) (end points included, so neighbouring
 *    blocks that share a boundary sample -- Sec. 4.2 -- decode it twice).
 *  - Channel mask: bit 0 value, bit 1 d/du (x), bit 2 d/dv (y), bit 3
 *    d/dw (z).  Outputs hold only the selected channels, in that order.
 *  - Pointers documented "device" must be device memory of the current
 *    HIP device; "host" pointers are read synchronously and may be freed
 *    on return.  The caller owns every buffer; no hot call allocates.
 *  - `stream` is a hipStream_t (0 = the null stream).  Hot calls are
 *    asynchronous on it, never synchronise, and may be captured into a
 *    HIP graph.  Argument errors are returned before anything is launched
 *    and leave every output untouched.
 */
#ifndef FA_H
#define FA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fa_status {
    FA_OK = 0,
    FA_ERR_INVALID_ARG = 1, /* null pointer, bad size, malformed descriptor */
    FA_ERR_UNSUPPORTED = 2, /* valid B-spline outside what the kernels take */
    FA_ERR_DEVICE = 3       /* a HIP call or launch failed */
} fa_status;

typedef enum fa_dtype {
    FA_F32 = 0,  /* control points stored as float                         */
    FA_BF16 = 1, /* bfloat16 holding P / scale (per-block max-abs scaling) */
    FA_F16 = 2   /* IEEE half holding P / scale                             */
} fa_dtype;
/* 2-byte lattices are read in whole dwords: a block whose lattice has an odd
 * number of values is read up to two bytes past its last value (values
 * outside the block never enter a result), so the allocation must extend
 * to the next 4-byte boundary (any hipMalloc allocation does). */

/* Maximum degree and control points per axis taken by the kernels. */
#define FA_MAX_DEGREE 3
#define FA_MAX_NCP 64
#define FA_MAX_RES 256

/* Decode output layout flag (OR-ed into fa_decode_blocks' mask with all
 * four channels): one 16-byte record (value, d/du, d/dv, d/dw) per voxel. */
#define FA_OUT_INTERLEAVED 0x100u

/* Descriptor flag bits written by fa_validate_blocks. */
#define FA_FLAG_UNIFORM_X 1u /* x knots are exactly (float)(j-p)/(float)(n-p) */
#define FA_FLAG_UNIFORM_Y 2u
#define FA_FLAG_UNIFORM_Z 4u

/* One micro-model (64 bytes).  ncp[a] >= degree[a]+1 and <= FA_MAX_NCP;
 * the three degrees must be equal (a micro-model has one degree, Eq. 2)
 * and lie in [1, FA_MAX_DEGREE].  scale multiplies every stored control
 * point of a BF16/FP16 lattice; FP32 lattices ignore it. */
typedef struct fa_block {
    int32_t ncp[3];
    int32_t degree[3];
    int64_t knot_off; /* element offset into the knot array          */
    int64_t ctrl_off; /* element offset into the lattice array; a
                         multiple of 4 elements                       */
    float scale;
    uint32_t flags;   /* FA_FLAG_* (set by fa_validate_blocks)        */
    int32_t reserved[4];
} fa_block;

/* One unit of work of the batched decode: rows [row0, row0+nrows) of the
 * y axis, z lanes [col0, col0+64), all x, of block `block`. */
typedef struct fa_work {
    int32_t block;
    int16_t row0;
    int16_t nrows;
    int16_t col0;
    int16_t pad;
} fa_work;

/* Tunables of the batched decode (a0: batch plan and persistent schedule).
 * Zero fields take defaults. */
typedef struct fa_tune {
    int32_t rows_per_item; /* y rows per work item, 1..64 (default 8)           */
    int32_t waves;         /* waves (64 lanes) per workgroup: 1, 2, 4, 8        */
    int32_t grid;          /* persistent workgroups (capped at the item count)  */
    int32_t kernel;        /* 0 = separable VALU, 1 = MFMA (BF16/FP16 lattices;
                              16 rows x 64 columns per item and 4 waves: pass
                              rows_per_item 0 or 16 and waves 0 or 4)       */
    int32_t slab_floats;   /* LDS lattice slab, 4096..16384 floats (default 8192);
                              larger lattices are staged in x chunks            */
    int32_t store;         /* 0 = non-temporal stores, 1 = ordinary stores
                              (separable VALU kernel; the MFMA kernel writes
                              partial lines and always stores ordinarily)    */
} fa_tune;

const char *fa_status_string(fa_status s);

/* Version of this ABI (major*10000 + minor*100 + patch). */
int32_t fa_version(void);

/*
 * Check host copies of the descriptors and knots (Sec. 4.2 micro-model
 * content) once, before any hot call, and set each descriptor's `flags`.
 *   blocks  host, nblocks entries, read and written (flags only)
 *   knots   host, nknots floats
 *   nctrl   number of lattice elements the caller will pass
 * Returns FA_ERR_INVALID_ARG for: null pointers, nblocks <= 0, ncp <
 * degree+1, unequal degrees, offsets or lengths outside the arrays, knots
 * that are not clamped on [0,1] or decrease; FA_ERR_UNSUPPORTED for degree
 * > FA_MAX_DEGREE or ncp > FA_MAX_NCP.  Nothing is written on error.
 */
fa_status fa_validate_blocks(fa_block *blocks, int32_t nblocks, const float *knots,
                             int64_t nknots, int64_t nctrl);

/*
 * Batch plan (row a0): split every block into work items and assign them
 * to `grid` persistent workgroups by longest-processing-time-first on a
 * per-item cost model (work of uneven NCP* and degree differs).
 *   blocks  host descriptors (validated)
 *   res     host, 3 ints in [2, FA_MAX_RES]
 *   tune    host, may be NULL
 *   work    host, capacity entries; receives the items grouped by
 *           workgroup
 *   wg_off  host, capacity+1 entries; workgroup g runs
 *           work[wg_off[g] .. wg_off[g+1])
 *   nwork, ngroups  receive the item and workgroup counts
 * The item count is nblocks * ceil(res[1]/rows) * ceil(res[2]/64); a
 * capacity below it returns FA_ERR_INVALID_ARG.
 */
fa_status fa_plan_decode(const fa_block *blocks, int32_t nblocks, const int32_t res[3],
                         const fa_tune *tune, fa_work *work, int32_t *wg_off,
                         int64_t capacity, int64_t *nwork, int32_t *ngroups);

/*
 * Decode every block on its res[0] x res[1] x res[2] grid: value and/or
 * gradient with respect to the block parameters (Alg. 4, valueMicroModel
 * and gradientMicroModel at every voxel) -- the batched, persistent form.
 *   blocks  device, nblocks descriptors (validated on the host first)
 *   knots   device FP32
 *   ctrl    device lattice of `dtype` (FA_BF16/FA_F16 hold P/scale)
 *   work, wg_off  device copies of a plan from fa_plan_decode made with
 *           the same tune and res, or both NULL for the default order
 *   ngroups workgroups in the plan (ignored when work is NULL)
 *   out     device FP32 [nblocks][popcount(mask)][res0][res1][res2], or
 *           with mask = 15 | FA_OUT_INTERLEAVED [nblocks][res0][res1][res2][4]
 *           (the same values, one 16-byte record per voxel)
 * FA_ERR_UNSUPPORTED if tune->kernel selects the MFMA kernel with an FP32
 * lattice or with a tile other than 16 rows and 4 waves; FA_ERR_INVALID_ARG
 * for FA_OUT_INTERLEAVED without all four channels.
 */
fa_status fa_decode_blocks(const fa_block *blocks, int32_t nblocks, const float *knots,
                           const void *ctrl, fa_dtype dtype, const int32_t res[3],
                           uint32_t mask, const fa_tune *tune, const fa_work *work,
                           const int32_t *wg_off, int32_t ngroups, float *out,
                           void *stream);

/*
 * The plain form of the same decode: one launch per block, one thread per
 * voxel, each thread doing its own span search, basis evaluation and
 * (p+1)^3 window sum.  Same arguments and output as fa_decode_blocks
 * (FP32 lattices only).  It exists as the baseline the batched form is
 * measured against.
 */
fa_status fa_decode_blocks_plain(const fa_block *blocks, int32_t nblocks,
                                 const float *knots, const float *ctrl,
                                 const int32_t res[3], uint32_t mask, float *out,
                                 void *stream);

/*
 * Point query over a domain tiled by nb[0] x nb[1] x nb[2] cells (Alg. 4:
 * getSampleLocation, then valueMicroModel and gradientMicroModel).
 *   blocks, knots, ctrl, dtype   as for fa_decode_blocks
 *   block_of_cell  device int32 [nb0][nb1][nb2]: descriptor index of each
 *           cell; -1 (or any index outside [0, nblocks)) marks an empty
 *           cell, whose samples return zeros
 *   nb, origin, extent  host, 3 each; extent > 0
 *   xyz     device FP32 [n][3]
 *   out     device FP32 [n][4] = value, d/dx, d/dy, d/dz in domain units
 *           (channels not in mask are written as 0)
 * Block lookup in FP32, one rounding per operation:
 *   r = (float)nb/extent;  q = clamp((x - origin)*r, 0, nb);
 *   b = min(floor(q), nb-1);  u = q - b  (exact);  d/dx = r * d/du.
 * Positions outside the domain are clamped onto it.
 */
fa_status fa_query_points(const fa_block *blocks, int32_t nblocks,
                          const int32_t *block_of_cell, const int32_t nb[3],
                          const float origin[3], const float extent[3], const float *knots,
                          const void *ctrl, fa_dtype dtype, const float *xyz, int64_t n,
                          uint32_t mask, float *out, void *stream);

/*
 * Ray-structured point query: the same evaluation as fa_query_points for
 * positions laid out as Alg. 4's pixel loop produces them, xyz =
 * [height][width][samples][3] (ray-major, row-major pixels), out =
 * [height][width][samples][4].  Results are identical to fa_query_points
 * on the flattened arrays; only the order in which the GPU visits the
 * samples differs: a workgroup marches a 16 x 16 tile of adjacent rays in
 * lockstep (a wave: one row of 16 rays, 4 consecutive samples of each per
 * step), and copies the one or two micro-models its rays are in at each
 * step into LDS, where the evaluation reads them.
 * Errors: FA_ERR_INVALID_ARG for width, height or samples <= 0, and as
 * fa_query_points.
 */
fa_status fa_query_rays(const fa_block *blocks, int32_t nblocks, const int32_t *block_of_cell,
                        const int32_t nb[3], const float origin[3], const float extent[3],
                        const float *knots, const void *ctrl, fa_dtype dtype, const float *xyz,
                        int32_t width, int32_t height, int32_t samples, uint32_t mask,
                        float *out, void *stream);

/* One image ray: origin, unit direction, and the parameter interval
 * [t0, t1] over which it is sampled (t1 <= t0: the ray misses). 32 bytes. */
typedef struct fa_ray {
    float origin[3];
    float dir[3];
    float t0, t1;
} fa_ray;

/* Ray-marching parameters of fa_render_rays (Alg. 4). */
typedef struct fa_render_params {
    int32_t samples;       /* samples per ray (>= 1)                           */
    float opacity_max;     /* stop a ray once accumulated opacity exceeds it   */
    float tf_lo, tf_hi;    /* value range covered by the transfer function     */
    int32_t tf_size;       /* RGBA entries of the transfer function (>= 2)     */
    float light[3];        /* unit direction towards the light                 */
    float ka, kd, ks;      /* ambient, diffuse, specular coefficients          */
    float shininess;       /* Blinn-Phong exponent                             */
    float grad_min;        /* shade only where |gradient| > grad_min (>= 0)    */
} fa_render_params;

/*
 * Direct volume rendering by front-to-back ray casting over the micro-models
 * of a tiled domain (Alg. 4; Sec. 4.3.3): for every pixel, for samples
 * s = 0..S-1 at getSampleLocation(s), valueMicroModel -> transfer function,
 * gradientMicroModel -> shading, compositing, early termination once the
 * accumulated opacity exceeds opacity_max.
 *   blocks .. dtype  the micro-models, as for fa_query_points
 *   rays     device fa_ray [height][width]
 *   params   host; tf device FP32 [tf_size][4] (RGBA, A = opacity per sample)
 *   image    device FP32 [height][width][4] = composited RGB, accumulated A
 * Sample position, in FP32 with one rounding per operation:
 *   dt = (t1 - t0) / S;  t = t0 + ((float)s + 0.5f) * dt;  x = o + t * d.
 * Transfer function: q = clamp((v - tf_lo) / (tf_hi - tf_lo) * (n - 1), 0,
 * n - 1), linear interpolation between entries floor(q) and floor(q) + 1.
 * Shading (two-sided Blinn-Phong, V = -d, H = (L + V)/|L + V|, N = g/|g|):
 *   rgb *= ka + kd |N.L| + ks |N.H|^shininess   (ka alone where |g| <=
 *   grad_min: the normal of a flat region is undefined).
 * Compositing: C += (1 - A) a rgb;  A += (1 - A) a.
 * Errors: FA_ERR_INVALID_ARG for null pointers, width/height/samples <= 0,
 * tf_size < 2, tf_hi <= tf_lo, grad_min < 0, and as fa_query_points.
 */
fa_status fa_render_rays(const fa_block *blocks, int32_t nblocks, const int32_t *block_of_cell,
                         const int32_t nb[3], const float origin[3], const float extent[3],
                         const float *knots, const void *ctrl, fa_dtype dtype,
                         const fa_ray *rays, int32_t width, int32_t height,
                         const fa_render_params *params, const float *tf, float *image,
                         void *stream);

/*
 * Adjoint of the grid decode: grad_ctrl = B^T grad_out, where B is the
 * linear map ctrl -> decode output of fa_decode_blocks for the same blocks,
 * res and mask.  With grad_out the residual 2(f - y)/M of a least-squares
 * fit of the lattice to samples y on the block's grid, this is the fit's
 * gradient: the step model(NCP, degree) of Alg. 1 (Sec. 4.2.1) solves that
 * fit for every candidate NCP.  Deterministic (fixed summation order, no
 * floating-point atomics).  A value-only cotangent (mask 1) whose rows start
 * on 16-byte boundaries (res[2] a multiple of 4, grad_out 16-byte aligned)
 * runs on the FP32 matrix cores; other cotangents run on the VALU.
 *   grad_out   device FP32 [nblocks][popcount(mask)][res0][res1][res2]
 *   grad_ctrl  device FP32 lattice layout (same offsets as ctrl); the
 *              lattices of the blocks are overwritten, other elements are
 *              left untouched
 * res[1] and res[2] (the y and z resolutions) must be at most 64: one
 * workgroup streams each block's cotangent one x slice at a time, the
 * matrix-core form holding a slice's y and z extent as four 16-row bands of
 * four 16-column groups in registers, the VALU form holding the slice, its
 * z-contracted form and the dense y and z basis matrices in LDS
 * (FA_ERR_UNSUPPORTED above 64; res[0] takes up to FA_MAX_RES).
 */
fa_status fa_decode_backward(const fa_block *blocks, int32_t nblocks, const float *knots,
                             const int32_t res[3], uint32_t mask, const float *grad_out,
                             float *grad_ctrl, void *stream);

/*
 * One Adam step (Kingma and Ba, 2015) on the control points of a
 * gradient-based fit: the least-squares fit of a lattice to its block's
 * samples that Alg. 1's model(NCP, degree) step (Sec. 4.2.1) solves, whose
 * gradient fa_decode_backward gives.  In place, over n FP32 values, in the
 * form PyTorch's Adam uses (no amsgrad):
 *   g = grad + weight_decay * param
 *   exp_avg    = exp_avg + (1 - beta1) (g - exp_avg)
 *   exp_avg_sq = beta2 exp_avg_sq + (1 - beta2) g^2
 *   param     -= lr / (1 - beta1^t) * exp_avg / (sqrt(exp_avg_sq) / sqrt(1 - beta2^t) + eps)
 *   param, exp_avg, exp_avg_sq  device FP32 [n], updated in place
 *   grad                        device FP32 [n]
 *   state      device FP32 [3], caller-owned, zero before the first step:
 *              {t, 1 - beta1^t, sqrt(1 - beta2^t)}; every call first
 *              advances t by one on the device, so a captured graph steps
 *              correctly on every replay
 * With n = 0 only the step count advances (the arrays may be null).
 * Errors: FA_ERR_INVALID_ARG for a null state, null arrays with n > 0,
 * n < 0, beta1 or beta2 outside [0, 1), eps <= 0 and non-finite lr, eps or
 * weight_decay.
 */
fa_status fa_adam_step(float *param, const float *grad, float *exp_avg, float *exp_avg_sq,
                       int64_t n, float lr, float beta1, float beta2, float eps,
                       float weight_decay, float *state, void *stream);

/*
 * Per-block max-abs scaling and rounding to BF16/FP16 (row a4): for each
 * block, s_b = max |P_b| (1 when the lattice is all zeros), blocks[b].scale
 * = s_b, and ctrl_lp = round-to-nearest-even(P_b / s_b).
 *   blocks   device descriptors; `scale` is written
 *   ctrl_f32 device FP32 lattices
 *   ctrl_lp  device, 2-byte elements, same offsets
 */
fa_status fa_quantize_blocks(fa_block *blocks, int32_t nblocks, const float *ctrl_f32,
                             fa_dtype dtype, void *ctrl_lp, void *stream);

/* ------------------------------------------------------------------ */
/* Adaptive encoding (Sec. 4.2): fit, error map, NCP selection         */
/* ------------------------------------------------------------------ */

/*
 * Least-squares fit of every micro-model's lattice to samples on its decode
 * grid: the model(NCP, degree) step of Alg. 1 (Sec. 4.2.1).  With B the
 * value map of fa_decode_blocks at `res` (grid u_i = fl32(i / (res - 1))),
 * ctrl = argmin_P |y - B P|_2 = y x_1 B_x^+ x_2 B_y^+ x_3 B_z^+, with each
 * per-axis pseudo-inverse B_a^+ = (B_a^T B_a)^{-1} B_a^T formed in FP64 (FP64
 * basis at the FP32 grid positions, band Cholesky of the Gram matrix) and
 * applied as FP64 contractions; the lattice is rounded to FP32 once.
 *   blocks, knots  device descriptors/knots (FP32 lattices); ncp[a] <= res[a]
 *                  is the caller's to guarantee (a larger ncp makes the Gram
 *                  matrix singular and the lattice non-finite)
 *   samples        device FP32 [nblocks][res0][res1][res2]
 *   ctrl           device FP32, lattice layout; the blocks' lattices are
 *                  overwritten, other elements are left untouched
 *   max_ncp        >= ncp[2] of every block (blocks above it are skipped)
 *   workspace      device, >= fa_fit_workspace(nblocks, res, max_ncp) bytes,
 *                  256-B aligned (FP64 intermediate; the call allocates
 *                  nothing)
 * Errors: FA_ERR_INVALID_ARG for null pointers, nblocks <= 0, res < 2,
 * max_ncp < 2, a small or misaligned workspace; FA_ERR_UNSUPPORTED for
 * res > 64 on any axis or max_ncp > FA_MAX_NCP.
 */
int64_t fa_fit_workspace(int32_t nblocks, const int32_t res[3], int32_t max_ncp);
fa_status fa_fit_blocks(const fa_block *blocks, int32_t nblocks, const float *knots,
                        const int32_t res[3], const float *samples, float *ctrl, int32_t max_ncp,
                        void *workspace, int64_t workspace_bytes, void *stream);

/*
 * Error of every micro-model against samples on its decode grid (Error(NCP)
 * of Eq. 4): with f the value decode at `res`,
 *   errs[b * errs_stride + 0] = max |y - f|,
 *   errs[b * errs_stride + 1] = sqrt(mean (y - f)^2)   (FP64 sum of squares).
 *   decoded  device FP32 [nblocks][res0][res1][res2], filled with f
 *            (caller-owned workspace: the call allocates nothing)
 *   errs     device FP32, errs_stride >= 2
 * Deterministic.  Errors as fa_decode_blocks, and FA_ERR_INVALID_ARG for a
 * null samples/decoded/errs or errs_stride < 2.
 */
fa_status fa_model_errors(const fa_block *blocks, int32_t nblocks, const float *knots,
                          const void *ctrl, fa_dtype dtype, const int32_t res[3],
                          const float *samples, float *decoded, float *errs,
                          int64_t errs_stride, void *stream);

/*
 * Mean-squared-error step of a fit (the loss whose gradient the adjoint
 * carries back to the control points, Alg. 1's model fit): for every block
 * b and voxel v of its value decode,
 *   grad[b][v] = grad_scale * (decoded - samples),
 *   sumsq[b]   = sum_v (decoded - samples)^2   (FP64, fixed order).
 * With grad_scale = 2 / M (M = all voxels) grad is dLoss/ddecoded of
 * Loss = sum_b sumsq[b] / M.  grad may alias decoded.  All device pointers:
 * decoded, samples, grad FP32 [nblocks][vox]; sumsq FP64 [nblocks].
 * Deterministic.  FA_ERR_INVALID_ARG for null pointers, nblocks or vox <= 0,
 * a non-finite grad_scale.
 */
fa_status fa_mse_grad(const float *decoded, const float *samples, int32_t nblocks, int64_t vox,
                      float grad_scale, float *grad, double *sumsq, void *stream);

/*
 * The loss of a fit from the per-block sums of squares of fa_mse_grad or
 * fa_decode_residual (Alg. 1's model fit minimises it):
 *   loss[0] = (float)(sum_b sumsq[b] / count),
 * with count the number of residuals (all voxels of all blocks).  The FP64
 * sum runs in a fixed order (each of 256 threads adds every 256th block in
 * order, then a binary tree over the threads), one launch.
 *   sumsq  device FP64 [nblocks];  loss  device FP32 [1]
 * FA_ERR_INVALID_ARG for null pointers, nblocks <= 0 or count not positive
 * and finite.
 */
fa_status fa_mse_loss(const double *sumsq, int32_t nblocks, double count, float *loss,
                      void *stream);

/*
 * The value decode of fa_decode_blocks fused with fa_mse_grad: for every
 * block b and voxel v, with f the value decode (mask 1) of the FP32 lattice,
 *   grad[b][v] = grad_scale * (f[b][v] - samples[b][v]),
 *   sumsq[b]   = sum_v (f - samples)^2   (FP64, fixed order),
 * in one pass that reads the samples and writes grad (f itself is never
 * stored).  grad equals fa_decode_blocks + fa_mse_grad bit for bit; sumsq
 * differs only in the order of its FP64 sum.  Runs the separable VALU
 * kernel (tune->kernel must be 0); tune, work, wg_off, ngroups as in
 * fa_decode_blocks, except that waves left at 0 (or a null tune) mean 8
 * here (one y row per wave at the default 8 rows per item).
 *   samples, grad  device FP32 [nblocks][res0][res1][res2]
 *   sumsq          device FP64 [nblocks]
 *   workspace      device, fa_decode_residual_workspace(...) bytes (one
 *                  FP64 partial sum per work item)
 * FA_ERR_INVALID_ARG as fa_decode_blocks, for a non-finite grad_scale or a
 * small workspace; FA_ERR_UNSUPPORTED for the MFMA kernel.
 */
int64_t fa_decode_residual_workspace(int32_t nblocks, const int32_t res[3], const fa_tune *tune);
fa_status fa_decode_residual(const fa_block *blocks, int32_t nblocks, const float *knots,
                             const float *ctrl, const int32_t res[3], const fa_tune *tune,
                             const fa_work *work, const int32_t *wg_off, int32_t ngroups,
                             const float *samples, float grad_scale, float *grad,
                             double *sumsq, void *workspace, int64_t workspace_bytes,
                             void *stream);

/*
 * fa_decode_residual for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results (bit for bit), with
 * the per-item FP64 partial sums kept in a fixed device array of the
 * library, FA_NOALLOC_SCRATCH_BYTES long, instead of a caller workspace.
 * The call allocates nothing (no hipMalloc, no allocating library call);
 * the caller still passes the outputs.  The first call on a device looks up
 * that device's array (hipGetSymbolAddress); make it outside a graph
 * capture.  Every call on one GPU shares that GPU's array and leaves the
 * last call's partial sums in it (each call writes every partial it reads,
 * so nothing needs clearing): calls that overlap on one GPU, on different
 * streams or from different threads, race and must be serialised by the
 * caller.  FA_ERR_UNSUPPORTED when fa_decode_residual_workspace(nblocks,
 * res, tune) exceeds FA_NOALLOC_SCRATCH_BYTES (more than 131072 work items,
 * e.g. more than 16384 blocks at 64^3 with 8 y rows per item); otherwise
 * errors as fa_decode_residual, FA_ERR_DEVICE if the array's address cannot
 * be resolved.
 */
#define FA_NOALLOC_SCRATCH_BYTES (1 << 20)
fa_status fa_decode_residual_noalloc(const fa_block *blocks, int32_t nblocks,
                                     const float *knots, const float *ctrl,
                                     const int32_t res[3], const fa_tune *tune,
                                     const fa_work *work, const int32_t *wg_off,
                                     int32_t ngroups, const float *samples, float grad_scale,
                                     float *grad, double *sumsq, void *stream);

/* Bytes of device workspace fa_ncp_search needs (-1 for invalid sizes). */
int64_t fa_ncp_search_workspace(int32_t nblocks, const int32_t res[3], int32_t degree,
                                int32_t ncp_hi);

/*
 * In-level exhaustive search of Sec. 4.2.1 (the inner loop of Alg. 1): for
 * every NCP n from ncp_hi down to ncp_lo, every block is fitted with n
 * control points per axis (clamped uniform knots t_{p+j} = j / (n - p),
 * degree `degree` on every axis) and its error map entry is written:
 *   errs[(b * ncand + (n - ncp_lo)) * 2 + {0, 1}] = (max, rms) as
 *   fa_model_errors, ncand = ncp_hi - ncp_lo + 1.
 * Each candidate's value decode is reduced to its error-map entry as it is
 * computed (never stored): max |f - y| exact, the sum of squares in FP64 in
 * a fixed order, so the map is deterministic.
 *   samples    device FP32 [nblocks][res0][res1][res2]
 *   workspace  device, >= fa_ncp_search_workspace(...) bytes, 256-B aligned
 * Requires degree + 1 <= ncp_lo <= ncp_hi <= min(res) (FA_ERR_INVALID_ARG
 * otherwise); degree > 3, ncp_hi > FA_MAX_NCP or res > 64 on any axis give
 * FA_ERR_UNSUPPORTED.  Asynchronous on `stream`; no allocation.
 */
fa_status fa_ncp_search(const float *samples, int32_t nblocks, const int32_t res[3],
                        int32_t degree, int32_t ncp_lo, int32_t ncp_hi, float *errs,
                        void *workspace, int64_t workspace_bytes, void *stream);

/*
 * NCP* of Eq. 4 from host error maps laid out as fa_ncp_search writes them:
 * ncp_star[b] = the smallest n whose error (metric 0: max, 1: rms) is below
 * `bound`, or the largest candidate when none is; complex_[b] (may be null)
 * = 1 when some candidate's error exceeds `bound` (the complex-set test of
 * Alg. 1), else 0.  Host only.
 */
fa_status fa_ncp_select(const float *errs, int32_t nblocks, int32_t ncand, int32_t ncp_lo,
                        int32_t metric, float bound, int32_t *ncp_star, int32_t *complex_);

/*
 * The cross-level step of Alg. 1 (Sec. 4.2.2), host only.  Level k of the
 * pyramid tiles the domain with (2^k)^3 micro-blocks, block (bx, by, bz) at
 * index (bx * 2^k + by) * 2^k + bz; its parent is the level k-1 block (bx/2,
 * by/2, bz/2).  fa_search_set names the blocks of level `level` the in-level
 * search runs on: every block of level 0, and a block of a finer level
 * exactly when its parent is in the complex set of level k-1 (the blocks
 * "covered by ComplexSet"):
 *   parent_complex  host, (2^(k-1))^3 flags of level k-1 (ignored at k = 0)
 *   searched        host, (2^k)^3 entries: 1 if searched, else 0
 *   search_ids      host, may be null; receives the searched indices in
 *                   increasing order
 *   nsearched       receives their count
 * fa_level_select then sets the level's outcome from the error maps of the
 * searched blocks (laid out as fa_ncp_search writes them, one row per entry
 * of search_ids): NCP* and the complex flag of a searched block by the rule
 * of fa_ncp_select; every other block takes NCP* = degree + 1 and is not
 * complex.  ncp_star and complex_ are host arrays of nblocks entries.
 * Errors: FA_ERR_INVALID_ARG for null pointers, level outside [0, 10],
 * search_ids not increasing or outside [0, nblocks), ncp_lo < degree + 1,
 * an unknown metric or a non-finite bound.
 */
fa_status fa_search_set(int32_t level, const int32_t *parent_complex, int32_t *searched,
                        int32_t *search_ids, int32_t *nsearched);
fa_status fa_level_select(int32_t nblocks, const int32_t *search_ids, int32_t nsearched,
                          const float *errs, int32_t ncand, int32_t ncp_lo, int32_t degree,
                          int32_t metric, float bound, int32_t *ncp_star, int32_t *complex_);

/*
 * Host layout of a batch of micro-models with clamped uniform knots: for
 * per-block ncp[b][3] and degree[b][3] (equal on the axes), fills the
 * descriptors (may be null), the knots (may be null; t_{p+j} = fl32(j /
 * (n - p))) and returns the knot and lattice element counts; lattices start
 * at multiples of 64 elements (256 B in FP32).  FA_ERR_INVALID_ARG for
 * ncp < degree + 1, degree < 1, unequal degrees or too small a capacity.
 */
fa_status fa_uniform_layout(int32_t nblocks, const int32_t *ncp, const int32_t *degree,
                            fa_block *blocks, float *knots, int64_t knot_capacity,
                            int64_t *nknots, int64_t *nctrl);

/* ------------------------------------------------------------------ */
/* Storage, host cache and staging of micro-models (Eq. 2; Alg. 2)     */
/* ------------------------------------------------------------------ */

/*
 * Visible micro-models of a view, the first step of Alg. 2: flags[cell] = 1
 * for every cell of the nb[0] x nb[1] x nb[2] tiling that some sample of
 * fa_render_rays (same rays, same `samples`, same sample positions and
 * block lookup) falls in, else 0.  The cells a rendering of this view
 * queries are exactly the flagged ones.
 *   rays   device fa_ray [height][width]; flags device int32 [ncells]
 *          (overwritten in full; no memset is used, graph-capturable)
 * Errors: FA_ERR_INVALID_ARG for null pointers, width/height/samples <= 0,
 * non-positive or non-finite extent, non-finite origin.
 */
fa_status fa_visible_cells(const fa_ray *rays, int32_t width, int32_t height, int32_t samples,
                           const int32_t nb[3], const float origin[3], const float extent[3],
                           int32_t *flags, void *stream);

/*
 * Micro-model file (Eq. 2).  Header: "FAM1", int32 version (1), int32
 * nblocks, int32 0; index: int64 offset, int64 size per block; records:
 * one byte (degree p), for x, y, z the clamped knot vector without its last
 * knot (NCP + p FP32 values; the last knot of a clamped vector on [0, 1] is
 * 1), then the NCP^3 FP32 control points [x][y][z].  A record therefore
 * takes exactly 1 + ((NCP + p) * 3 + NCP^3) * 4 bytes, and NCP is recovered
 * from its size.  One NCP and one degree per block (as Eq. 2 counts them):
 * blocks with unequal NCP or degree per axis are FA_ERR_INVALID_ARG, and so
 * are knot vectors that are not clamped on [0, 1] and non-decreasing;
 * degree > FA_MAX_DEGREE or NCP > FA_MAX_NCP is FA_ERR_UNSUPPORTED.
 *   blocks, knots, ctrl  host arrays (FP32 lattices)
 * FA_ERR_DEVICE on an I/O error.
 */
fa_status fa_store_write(const char *path, int32_t nblocks, const fa_block *blocks,
                         const float *knots, const float *ctrl);

typedef struct fa_store fa_store;  /* opaque: an open file plus its host cache */

#define FA_STORE_PINNED 1u  /* page-locked cache slots (required by fa_store_stage) */

typedef struct fa_store_stats {
    int64_t hits, misses, evictions;  /* cache lookups since fa_store_open   */
    int64_t bytes_read;               /* record bytes read from the file     */
    int64_t bytes_h2d;                /* bytes copied to the device (stage)  */
} fa_store_stats;

/*
 * Open a micro-model file with a host cache of `cache_blocks` slots (each
 * large enough for the file's largest record).  With FA_STORE_PINNED the
 * slots are page-locked (hipHostMalloc) so staging copies are DMA
 * transfers.  Allocates; not for hot loops.  FA_ERR_INVALID_ARG for a
 * missing or malformed file (bad header, a record outside the file or of a
 * size no NCP gives); FA_ERR_UNSUPPORTED for a record of degree >
 * FA_MAX_DEGREE.
 */
fa_status fa_store_open(const char *path, int32_t cache_blocks, uint32_t flags, fa_store **out);
fa_status fa_store_close(fa_store *s);

/* Block count and per-block NCP and degree (arrays of nblocks, may be null). */
fa_status fa_store_info(const fa_store *s, int32_t *nblocks, int32_t *ncp, int32_t *degree);

/*
 * The caching step of Alg. 2 on the host: for ids[0..n) in order, a cached
 * block is a hit (and becomes the most recently used), a missing one is
 * read from the file into a free slot or, with the cache full, into the
 * slot of the least recently used block.  slots[i] (may be null) receives
 * the slot holding ids[i] at the time it was looked up (a later lookup in
 * the same call can evict it when n exceeds the cache).  stats (may be null)
 * receives the running counters.  Waits first for the copies of a previous
 * fa_store_stage on this store (they read slots a refill would overwrite).
 * A record is read and checked before the cache changes: FA_ERR_DEVICE for
 * a read error, FA_ERR_INVALID_ARG for knots that are not clamped and
 * non-decreasing; the blocks before it in ids stay cached and the cache is
 * otherwise unchanged.
 */
fa_status fa_store_fetch(fa_store *s, const int32_t *ids, int32_t n, int32_t *slots,
                         fa_store_stats *stats);

/* Host view of a cache slot: block id, its 3 full knot vectors (x, y, z
 * back to back, last knot included) and its lattice. */
fa_status fa_store_slot(const fa_store *s, int32_t slot, int32_t *block, const float **knots,
                        const float **ctrl);

/*
 * Caching plus memory copy of Alg. 2: blocks ids[0..n) are fetched as by
 * fa_store_fetch and copied, as they are fetched, into a packed device batch
 * on `stream`: descriptor i = block ids[i] with knots at dev_knots[knot_off]
 * and its lattice at dev_ctrl[ctrl_off] (64-element aligned), uniform-knot
 * flags set as fa_validate_blocks would.  Asynchronous; the cache keeps a
 * slot from being refilled while a copy from it may still run.  Requires a
 * store opened with FA_STORE_PINNED.  FA_ERR_INVALID_ARG for bad ids, n >
 * nblocks of the file, or capacities below the batch's knot/lattice counts.
 */
fa_status fa_store_stage(fa_store *s, const int32_t *ids, int32_t n, fa_block *dev_blocks,
                         float *dev_knots, int64_t knot_capacity, float *dev_ctrl,
                         int64_t ctrl_capacity, fa_store_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FA_H */
