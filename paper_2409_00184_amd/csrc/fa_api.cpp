// C ABI of the micro-model decode/query library: argument checking,
// descriptor validation, the batch planner (row a0) and the launches.
// Every entry point is declared and documented in include/fa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <queue>
#include <vector>

#include "../../include/fa.h"
#include "fa_internal.hpp"

using namespace fa;

// Scratch of fa_decode_residual_noalloc (see scratch_address below).
static __device__ __align__(256) double scratch[FA_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kDefaultWaves = 4;
constexpr int kDefaultRows = 8;
constexpr int kDefaultGrid = 768;  // 256 CUs x 3 resident workgroups (LDS bound)
// residual and error forms: one y row per wave by default (a wave that walks
// several rows restages a large lattice's slab for each; at NCP 64 one row
// per wave runs 2.5x faster)
constexpr int kReduceWaves = 8;

struct Tune {
    int rows, waves, grid, kernel, slab, store;
};

Tune resolve(const fa_tune *t) {
    Tune r{kDefaultRows, kDefaultWaves, 0, 0, kSlabDefault, 0};
    if (t && t->kernel == 1) r.rows = kMfmaRows;
    if (t) {
        if (t->rows_per_item > 0) r.rows = t->rows_per_item;
        if (t->waves > 0) r.waves = t->waves;
        if (t->grid > 0) r.grid = t->grid;
        r.kernel = t->kernel;
        if (t->slab_floats > 0) r.slab = t->slab_floats;
        r.store = t->store;
    }
    return r;
}

// Default workgroup count: the separable VALU kernel runs persistently on
// kDefaultGrid workgroups; the matrix-core kernel (two resident per CU, items
// of very uneven length) runs one workgroup per item, which avoids the tail
// of a persistent grid that does not divide the resident slots.
int64_t default_grid(const Tune &t, int64_t items) {
    if (t.grid > 0) return t.grid;
    return t.kernel == 1 ? items : kDefaultGrid;
}

int popcount4(uint32_t m) { return __builtin_popcount(m & 15u); }

bool waves_ok(int w) { return w == 1 || w == 2 || w == 4 || w == 8; }

bool res_ok(const int32_t *res) {
    if (!res) return false;
    for (int a = 0; a < 3; ++a)
        if (res[a] < 2) return false;
    return true;
}

bool res_supported(const int32_t *res) {
    for (int a = 0; a < 3; ++a)
        if (res[a] > FA_MAX_RES) return false;
    return true;
}

bool tune_ok(const Tune &t) {
    return waves_ok(t.waves) && t.rows >= 1 && t.rows <= 64 && t.slab >= kSlabMin &&
           t.slab <= kSlabMax && (t.store == 0 || t.store == 1) &&
           (t.kernel == 0 || t.kernel == 1);
}

// launch arguments of a grid decode (default item order unless work is set)
DecodeLaunch grid_args(const fa_block *blocks, int32_t nblocks, const float *knots,
                       const void *ctrl, fa_dtype dtype, const int32_t res[3], uint32_t mask,
                       const Tune &t, const fa_work *work, const int32_t *wg_off, float *out) {
    DecodeLaunch a{};
    a.blocks = blocks;
    a.knots = knots;
    a.ctrl = ctrl;
    a.dtype = dtype;
    a.rx = res[0];
    a.ry = res[1];
    a.rz = res[2];
    a.mask = mask;
    a.nch = popcount4(mask);
    a.work = work;
    a.wg_off = wg_off;
    a.rows = t.rows;
    a.nrowt = (res[1] + t.rows - 1) / t.rows;
    a.ncolt = (res[2] + kWaveLanes - 1) / kWaveLanes;
    a.nitems = (int64_t)nblocks * a.nrowt * a.ncolt;
    a.slab = t.slab;
    a.nt_store = t.store == 0;
    a.out = out;
    return a;
}

// work items per block of a grid decode in the default order
int64_t items_per_block(const int32_t res[3], const Tune &t) {
    return (int64_t)((res[1] + t.rows - 1) / t.rows) * ((res[2] + kWaveLanes - 1) / kWaveLanes);
}


// `scratch` holds the per-item FP64 partial sums of
// fa_decode_residual_noalloc in a device array of fixed size (each GPU the
// library runs on holds its own copy until the process ends).  Host code
// never passes `scratch` itself to a kernel (in host code the name stands
// for a host-side placeholder, not the device array); it uses the device
// address that hipGetSymbolAddress returns, resolved once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_of[kMaxDevices] = {};

// Device address of the current device's scratch array.
hipError_t scratch_address(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_of[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_of[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_of[dev];
    return hipSuccess;
}

// fa_decode_residual with its per-item partial sums in `partials`
// (partials_bytes long), or, with partials null, in the current device's
// scratch array (fa_decode_residual_noalloc).  Every argument check comes
// before the scratch lookup and any launch.
fa_status decode_residual_impl(const fa_block *blocks, int32_t nblocks, const float *knots,
                               const float *ctrl, const int32_t res[3], const fa_tune *tune,
                               const fa_work *work, const int32_t *wg_off, int32_t ngroups,
                               const float *samples, float grad_scale, float *grad,
                               double *sumsq, int64_t partials_bytes, double *partials,
                               void *stream) {
    if (!blocks || !knots || !ctrl || !samples || !grad || !sumsq || nblocks <= 0 ||
        !res_ok(res) || !std::isfinite(grad_scale))
        return FA_ERR_INVALID_ARG;
    if ((work == nullptr) != (wg_off == nullptr)) return FA_ERR_INVALID_ARG;
    if (work && ngroups <= 0) return FA_ERR_INVALID_ARG;
    if (!res_supported(res)) return FA_ERR_UNSUPPORTED;
    Tune t = resolve(tune);
    if (!tune || tune->waves <= 0) t.waves = kReduceWaves;
    if (!tune_ok(t)) return FA_ERR_INVALID_ARG;
    if (t.kernel != 0) return FA_ERR_UNSUPPORTED;
    const int64_t need = (int64_t)nblocks * items_per_block(res, t) * (int64_t)sizeof(double);
    if (partials) {
        if (partials_bytes < need) return FA_ERR_INVALID_ARG;
    } else {
        if (need > FA_NOALLOC_SCRATCH_BYTES) return FA_ERR_UNSUPPORTED;
        if (scratch_address(&partials) != hipSuccess) return FA_ERR_DEVICE;
    }
    DecodeLaunch a = grid_args(blocks, nblocks, knots, ctrl, FA_F32, res, 1u, t, work, wg_off,
                               grad);
    a.samples = samples;
    a.gscale = grad_scale;
    a.partials = partials;
    const int grid = work ? ngroups : (int)std::min<int64_t>(a.nitems, default_grid(t, a.nitems));
    hipError_t e = launch_decode_sep(a, t.waves, grid, (hipStream_t)stream);
    if (e == hipSuccess)
        e = launch_residual_combine(a.partials, nblocks, a.nrowt * a.ncolt, sumsq,
                                    (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

}  // namespace

extern "C" {

const char *fa_status_string(fa_status s) {
    switch (s) {
    case FA_OK: return "ok";
    case FA_ERR_INVALID_ARG: return "invalid argument";
    case FA_ERR_UNSUPPORTED: return "unsupported";
    case FA_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

int32_t fa_version(void) { return 10000; }

fa_status fa_validate_blocks(fa_block *blocks, int32_t nblocks, const float *knots,
                             int64_t nknots, int64_t nctrl) {
    if (!blocks || !knots || nblocks <= 0 || nknots <= 0 || nctrl <= 0)
        return FA_ERR_INVALID_ARG;
    std::vector<uint32_t> flags(nblocks, 0u);
    fa_status worst = FA_OK;
    for (int32_t b = 0; b < nblocks; ++b) {
        const fa_block &B = blocks[b];
        const int p = B.degree[0];
        if (B.degree[1] != p || B.degree[2] != p || p < 1) return FA_ERR_INVALID_ARG;
        if (p > FA_MAX_DEGREE) worst = FA_ERR_UNSUPPORTED;
        int64_t klen = 0, clen = 1;
        for (int a = 0; a < 3; ++a) {
            if (B.ncp[a] < p + 1) return FA_ERR_INVALID_ARG;
            if (B.ncp[a] > FA_MAX_NCP) worst = FA_ERR_UNSUPPORTED;
            klen += B.ncp[a] + p + 1;
            clen *= B.ncp[a];
        }
        if (B.knot_off < 0 || B.knot_off + klen > nknots) return FA_ERR_INVALID_ARG;
        if (B.ctrl_off < 0 || B.ctrl_off % 4 != 0 || B.ctrl_off + clen > nctrl)
            return FA_ERR_INVALID_ARG;
        if (worst != FA_OK) continue;
        const float *t = knots + B.knot_off;
        for (int a = 0; a < 3; ++a) {
            const int n = B.ncp[a];
            for (int j = 0; j <= p; ++j)
                if (t[j] != 0.0f || t[n + j] != 1.0f) return FA_ERR_INVALID_ARG;
            for (int j = 1; j < n + p + 1; ++j)
                if (!(t[j] >= t[j - 1])) return FA_ERR_INVALID_ARG;
            bool uni = true;
            for (int j = 0; j <= n - p && uni; ++j)
                uni = t[p + j] == (float)j / (float)(n - p);
            if (uni) flags[b] |= (1u << a);
            t += n + p + 1;
        }
    }
    if (worst != FA_OK) return worst;
    for (int32_t b = 0; b < nblocks; ++b) blocks[b].flags = flags[b];
    return FA_OK;
}

fa_status fa_plan_decode(const fa_block *blocks, int32_t nblocks, const int32_t res[3],
                         const fa_tune *tune, fa_work *work, int32_t *wg_off,
                         int64_t capacity, int64_t *nwork, int32_t *ngroups) {
    if (!blocks || nblocks <= 0 || !res_ok(res) || !work || !wg_off || !nwork || !ngroups)
        return FA_ERR_INVALID_ARG;
    if (!res_supported(res)) return FA_ERR_UNSUPPORTED;
    const Tune t = resolve(tune);
    if (!tune_ok(t)) return FA_ERR_INVALID_ARG;
    if (t.kernel == 1 && (t.rows != kMfmaRows || t.waves != 4)) return FA_ERR_UNSUPPORTED;
    const int nrowt = (res[1] + t.rows - 1) / t.rows;
    const int ncolt = (res[2] + kWaveLanes - 1) / kWaveLanes;
    const int64_t n = (int64_t)nblocks * nrowt * ncolt;
    if (capacity < n) return FA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < nblocks; ++b) {
        const int p = blocks[b].degree[0];
        if (p < 1 || p > FA_MAX_DEGREE) return FA_ERR_INVALID_ARG;
        for (int a = 0; a < 3; ++a)
            if (blocks[b].ncp[a] < p + 1 || blocks[b].ncp[a] > FA_MAX_NCP)
                return FA_ERR_INVALID_ARG;
    }
    // items and their cost: stores + banded x stage per voxel, the on-the-fly
    // (z, y) contraction per column and x plane, the per-item set-up
    std::vector<fa_work> items(n);
    std::vector<double> cost(n);
    int64_t q = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        const fa_block &B = blocks[b];
        const int p = B.degree[0], nx = B.ncp[0], ny = B.ncp[1], nz = B.ncp[2];
        const double per_vox = 4.0 + 4.0 * (p + 1);
        const double per_col_plane = 2.0 * (p + 1) * (p + 1) + 3.0 * (p + 1);
        for (int rt = 0; rt < nrowt; ++rt) {
            const int row0 = rt * t.rows;
            const int nrows = std::min(t.rows, res[1] - row0);
            const double jn = std::min<double>(ny, (double)(nrows - 1) * (ny - p) / (res[1] - 1) + p + 2);
            for (int ct = 0; ct < ncolt; ++ct) {
                const int col0 = ct * kWaveLanes;
                const int ncols = std::min(kWaveLanes, res[2] - col0);
                items[q] = fa_work{b, (int16_t)row0, (int16_t)nrows, (int16_t)col0, 0};
                cost[q] = (double)res[0] * nrows * ncols * per_vox +
                          (double)nrows * ncols * nx * per_col_plane + 40.0 * res[0] +
                          2.0 * nx * jn * nz;
                ++q;
            }
        }
    }
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n, default_grid(t, n)));
    // longest processing time first onto the least loaded workgroup
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    using Slot = std::pair<double, int>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int g = 0; g < grid; ++g) heap.push({0.0, g});
    std::vector<int> owner(n);
    std::vector<int32_t> count(grid, 0);
    for (int64_t k = 0; k < n; ++k) {
        Slot s = heap.top();
        heap.pop();
        owner[order[k]] = s.second;
        count[s.second]++;
        heap.push({s.first + cost[order[k]], s.second});
    }
    wg_off[0] = 0;
    for (int g = 0; g < grid; ++g) wg_off[g + 1] = wg_off[g] + count[g];
    std::vector<int32_t> fill(wg_off, wg_off + grid);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t it = order[k];
        work[fill[owner[it]]++] = items[it];
    }
    *nwork = n;
    *ngroups = grid;
    return FA_OK;
}

fa_status fa_decode_blocks(const fa_block *blocks, int32_t nblocks, const float *knots,
                           const void *ctrl, fa_dtype dtype, const int32_t res[3],
                           uint32_t mask, const fa_tune *tune, const fa_work *work,
                           const int32_t *wg_off, int32_t ngroups, float *out,
                           void *stream) {
    const bool inter = (mask & FA_OUT_INTERLEAVED) != 0;
    const uint32_t ch = mask & 15u;
    if (!blocks || !knots || !ctrl || !out || nblocks <= 0 || !res_ok(res) || ch == 0 ||
        (mask & ~(15u | FA_OUT_INTERLEAVED)) != 0 || (inter && ch != 15u))
        return FA_ERR_INVALID_ARG;
    if (dtype != FA_F32 && dtype != FA_BF16 && dtype != FA_F16) return FA_ERR_INVALID_ARG;
    if ((work == nullptr) != (wg_off == nullptr)) return FA_ERR_INVALID_ARG;
    if (work && ngroups <= 0) return FA_ERR_INVALID_ARG;
    if (!res_supported(res)) return FA_ERR_UNSUPPORTED;
    const Tune t = resolve(tune);
    if (!tune_ok(t)) return FA_ERR_INVALID_ARG;
    DecodeLaunch a = grid_args(blocks, nblocks, knots, ctrl, dtype, res, ch, t, work, wg_off,
                               out);
    a.interleave = inter ? 1 : 0;
    int grid = work ? ngroups : (int)std::min<int64_t>(a.nitems, default_grid(t, a.nitems));
    hipError_t e;
    if (t.kernel == 1) e = launch_decode_mfma(a, t.waves, grid, (hipStream_t)stream);
    else e = launch_decode_sep(a, t.waves, grid, (hipStream_t)stream);
    if (e == hipErrorNotSupported) return FA_ERR_UNSUPPORTED;
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

int64_t fa_decode_residual_workspace(int32_t nblocks, const int32_t res[3], const fa_tune *tune) {
    if (nblocks <= 0 || !res_ok(res) || !res_supported(res)) return -1;
    const Tune t = resolve(tune);
    if (!tune_ok(t)) return -1;
    return (int64_t)nblocks * items_per_block(res, t) * (int64_t)sizeof(double);
}

fa_status fa_decode_residual(const fa_block *blocks, int32_t nblocks, const float *knots,
                             const float *ctrl, const int32_t res[3], const fa_tune *tune,
                             const fa_work *work, const int32_t *wg_off, int32_t ngroups,
                             const float *samples, float grad_scale, float *grad,
                             double *sumsq, void *workspace, int64_t workspace_bytes,
                             void *stream) {
    if (!workspace) return FA_ERR_INVALID_ARG;
    return decode_residual_impl(blocks, nblocks, knots, ctrl, res, tune, work, wg_off, ngroups,
                                samples, grad_scale, grad, sumsq, workspace_bytes,
                                static_cast<double *>(workspace), stream);
}

fa_status fa_decode_residual_noalloc(const fa_block *blocks, int32_t nblocks,
                                     const float *knots, const float *ctrl,
                                     const int32_t res[3], const fa_tune *tune,
                                     const fa_work *work, const int32_t *wg_off,
                                     int32_t ngroups, const float *samples, float grad_scale,
                                     float *grad, double *sumsq, void *stream) {
    return decode_residual_impl(blocks, nblocks, knots, ctrl, res, tune, work, wg_off, ngroups,
                                samples, grad_scale, grad, sumsq, 0, nullptr, stream);
}

fa_status fa_decode_blocks_plain(const fa_block *blocks, int32_t nblocks, const float *knots,
                                 const float *ctrl, const int32_t res[3], uint32_t mask,
                                 float *out, void *stream) {
    if (!blocks || !knots || !ctrl || !out || nblocks <= 0 || !res_ok(res) ||
        (mask & 15u) == 0 || (mask & ~15u) != 0)
        return FA_ERR_INVALID_ARG;
    if (!res_supported(res)) return FA_ERR_UNSUPPORTED;
    hipError_t e = launch_decode_plain(blocks, nblocks, knots, ctrl, res[0], res[1], res[2],
                                       mask, out, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

}  // extern "C"

namespace {
fa_status query_common(const fa_block *blocks, int32_t nblocks, const int32_t *block_of_cell,
                       const int32_t nb[3], const float origin[3], const float extent[3],
                       const float *knots, const void *ctrl, fa_dtype dtype, const float *xyz,
                       int64_t n, uint32_t mask, float *out, int rw, int rh, int rk,
                       void *stream) {
    if (!blocks || nblocks <= 0 || !block_of_cell || !nb || !origin || !extent || !knots ||
        !ctrl || n < 0 || (n > 0 && (!xyz || !out)) || (mask & 15u) == 0 ||
        (mask & ~15u) != 0)
        return FA_ERR_INVALID_ARG;
    if (dtype != FA_F32 && dtype != FA_BF16 && dtype != FA_F16) return FA_ERR_INVALID_ARG;
    QueryLaunch a{};
    for (int k = 0; k < 3; ++k) {
        if (nb[k] <= 0 || !(extent[k] > 0.0f) || !std::isfinite(origin[k]) ||
            !std::isfinite(extent[k]))
            return FA_ERR_INVALID_ARG;
        a.nb[k] = nb[k];
        a.origin[k] = origin[k];
        a.rscale[k] = (float)nb[k] / extent[k];
    }
    if ((int64_t)nb[0] * nb[1] * nb[2] > (int64_t)1 << 30) return FA_ERR_UNSUPPORTED;
    a.blocks = blocks;
    a.nblocks = nblocks;
    a.block_of_cell = block_of_cell;
    a.knots = knots;
    a.ctrl = ctrl;
    a.dtype = dtype;
    a.xyz = xyz;
    a.n = n;
    a.mask = mask;
    a.out = out;
    a.rw = rw;
    a.rh = rh;
    a.rk = rk;
    hipError_t e = launch_query(a, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}
}  // namespace

extern "C" {

fa_status fa_query_points(const fa_block *blocks, int32_t nblocks,
                          const int32_t *block_of_cell, const int32_t nb[3],
                          const float origin[3], const float extent[3], const float *knots,
                          const void *ctrl, fa_dtype dtype, const float *xyz, int64_t n,
                          uint32_t mask, float *out, void *stream) {
    return query_common(blocks, nblocks, block_of_cell, nb, origin, extent, knots, ctrl, dtype,
                        xyz, n, mask, out, 0, 0, 0, stream);
}

fa_status fa_query_rays(const fa_block *blocks, int32_t nblocks, const int32_t *block_of_cell,
                        const int32_t nb[3], const float origin[3], const float extent[3],
                        const float *knots, const void *ctrl, fa_dtype dtype, const float *xyz,
                        int32_t width, int32_t height, int32_t samples, uint32_t mask,
                        float *out, void *stream) {
    if (width <= 0 || height <= 0 || samples <= 0) return FA_ERR_INVALID_ARG;
    return query_common(blocks, nblocks, block_of_cell, nb, origin, extent, knots, ctrl, dtype,
                        xyz, (int64_t)width * height * samples, mask, out, width, height,
                        samples, stream);
}

fa_status fa_render_rays(const fa_block *blocks, int32_t nblocks, const int32_t *block_of_cell,
                         const int32_t nb[3], const float origin[3], const float extent[3],
                         const float *knots, const void *ctrl, fa_dtype dtype,
                         const fa_ray *rays, int32_t width, int32_t height,
                         const fa_render_params *params, const float *tf, float *image,
                         void *stream) {
    if (!blocks || nblocks <= 0 || !block_of_cell || !nb || !origin || !extent || !knots ||
        !ctrl || !rays || !params || !tf || !image || width <= 0 || height <= 0)
        return FA_ERR_INVALID_ARG;
    if (dtype != FA_F32 && dtype != FA_BF16 && dtype != FA_F16) return FA_ERR_INVALID_ARG;
    const fa_render_params &p = *params;
    if (p.samples <= 0 || p.tf_size < 2 || !(p.tf_hi > p.tf_lo) || !std::isfinite(p.tf_lo) ||
        !std::isfinite(p.tf_hi) || !(p.grad_min >= 0.0f))
        return FA_ERR_INVALID_ARG;
    QueryLaunch a{};
    for (int k = 0; k < 3; ++k) {
        if (nb[k] <= 0 || !(extent[k] > 0.0f) || !std::isfinite(origin[k]) ||
            !std::isfinite(extent[k]))
            return FA_ERR_INVALID_ARG;
        a.nb[k] = nb[k];
        a.origin[k] = origin[k];
        a.rscale[k] = (float)nb[k] / extent[k];
    }
    if ((int64_t)nb[0] * nb[1] * nb[2] > (int64_t)1 << 30) return FA_ERR_UNSUPPORTED;
    a.blocks = blocks;
    a.nblocks = nblocks;
    a.block_of_cell = block_of_cell;
    a.knots = knots;
    a.ctrl = ctrl;
    a.dtype = dtype;
    a.mask = 15u;
    hipError_t e = launch_render(a, rays, width, height, p, tf, image, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_visible_cells(const fa_ray *rays, int32_t width, int32_t height, int32_t samples,
                           const int32_t nb[3], const float origin[3], const float extent[3],
                           int32_t *flags, void *stream) {
    if (!rays || width <= 0 || height <= 0 || samples <= 0 || !nb || !origin || !extent ||
        !flags)
        return FA_ERR_INVALID_ARG;
    int n[3];
    float o[3], r[3];
    for (int k = 0; k < 3; ++k) {
        if (nb[k] <= 0 || !(extent[k] > 0.0f) || !std::isfinite(origin[k]) ||
            !std::isfinite(extent[k]))
            return FA_ERR_INVALID_ARG;
        n[k] = nb[k];
        o[k] = origin[k];
        r[k] = (float)nb[k] / extent[k];
    }
    if ((int64_t)nb[0] * nb[1] * nb[2] > (int64_t)1 << 30) return FA_ERR_UNSUPPORTED;
    hipError_t e = launch_visible(rays, (int64_t)width * height, samples, n, o, r, flags,
                                  (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_decode_backward(const fa_block *blocks, int32_t nblocks, const float *knots,
                             const int32_t res[3], uint32_t mask, const float *grad_out,
                             float *grad_ctrl, void *stream) {
    if (!blocks || nblocks <= 0 || !knots || !res_ok(res) || !grad_out || !grad_ctrl ||
        (mask & 15u) == 0 || (mask & ~15u) != 0)
        return FA_ERR_INVALID_ARG;
    if (!res_supported(res) || res[1] > 64 || res[2] > 64) return FA_ERR_UNSUPPORTED;
    hipError_t e = launch_adjoint(blocks, nblocks, knots, res[0], res[1], res[2], mask,
                                  grad_out, grad_ctrl, 0, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_adam_step(float *param, const float *grad, float *exp_avg, float *exp_avg_sq,
                       int64_t n, float lr, float beta1, float beta2, float eps,
                       float weight_decay, float *state, void *stream) {
    if ((n > 0 && (!param || !grad || !exp_avg || !exp_avg_sq)) || !state || n < 0 ||
        !std::isfinite(lr) ||
        !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f) || !std::isfinite(eps) || !std::isfinite(weight_decay))
        return FA_ERR_INVALID_ARG;
    hipError_t e = launch_adam(param, grad, exp_avg, exp_avg_sq, n, lr, beta1, beta2, eps,
                               weight_decay, state, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_mse_loss(const double *sumsq, int32_t nblocks, double count, float *loss,
                      void *stream) {
    if (!sumsq || !loss || nblocks <= 0 || !(count > 0.0) || !std::isfinite(count))
        return FA_ERR_INVALID_ARG;
    hipError_t e = launch_mse_loss(sumsq, nblocks, count, loss, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_quantize_blocks(fa_block *blocks, int32_t nblocks, const float *ctrl_f32,
                             fa_dtype dtype, void *ctrl_lp, void *stream) {
    if (!blocks || nblocks <= 0 || !ctrl_f32 || !ctrl_lp) return FA_ERR_INVALID_ARG;
    if (dtype != FA_BF16 && dtype != FA_F16) return FA_ERR_INVALID_ARG;
    hipError_t e = launch_quantize(blocks, nblocks, ctrl_f32, dtype, ctrl_lp,
                                   (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}


fa_status fa_mse_grad(const float *decoded, const float *samples, int32_t nblocks, int64_t vox,
                      float grad_scale, float *grad, double *sumsq, void *stream) {
    if (!decoded || !samples || !grad || !sumsq || nblocks <= 0 || vox <= 0 ||
        !std::isfinite(grad_scale))
        return FA_ERR_INVALID_ARG;
    hipError_t e = launch_mse_grad(decoded, samples, vox, nblocks, grad_scale, grad, sumsq,
                                   (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

int64_t fa_fit_workspace(int32_t nblocks, const int32_t res[3], int32_t max_ncp) {
    if (nblocks <= 0 || !res_ok(res) || max_ncp < 2) return -1;
    return fit_workspace_bytes(nblocks, res[0], res[1], max_ncp);
}

fa_status fa_fit_blocks(const fa_block *blocks, int32_t nblocks, const float *knots,
                        const int32_t res[3], const float *samples, float *ctrl, int32_t max_ncp,
                        void *workspace, int64_t workspace_bytes, void *stream) {
    if (!blocks || nblocks <= 0 || !knots || !res_ok(res) || !samples || !ctrl || !workspace ||
        max_ncp < 2)
        return FA_ERR_INVALID_ARG;
    if (res[0] > 64 || res[1] > 64 || res[2] > 64 || max_ncp > FA_MAX_NCP)
        return FA_ERR_UNSUPPORTED;
    if (workspace_bytes < fit_workspace_bytes(nblocks, res[0], res[1], max_ncp) ||
        (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return FA_ERR_INVALID_ARG;
    hipError_t e = launch_fit(blocks, nblocks, knots, res[0], res[1], res[2], max_ncp, samples,
                              static_cast<double *>(workspace), ctrl, (hipStream_t)stream);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

fa_status fa_model_errors(const fa_block *blocks, int32_t nblocks, const float *knots,
                          const void *ctrl, fa_dtype dtype, const int32_t res[3],
                          const float *samples, float *decoded, float *errs,
                          int64_t errs_stride, void *stream) {
    if (!blocks || nblocks <= 0 || !knots || !ctrl || !res_ok(res) || !samples || !decoded ||
        !errs || errs_stride < 2)
        return FA_ERR_INVALID_ARG;
    if (dtype != FA_F32 && dtype != FA_BF16 && dtype != FA_F16) return FA_ERR_INVALID_ARG;
    if (!res_supported(res)) return FA_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const fa_status st = fa_decode_blocks(blocks, nblocks, knots, ctrl, dtype, res, 1u, nullptr,
                                          nullptr, nullptr, 0, decoded, stream);
    if (st != FA_OK) return st;
    const int64_t vox = (int64_t)res[0] * res[1] * res[2];
    hipError_t e = launch_residual(samples, decoded, vox, nblocks, errs, errs_stride, s);
    return e == hipSuccess ? FA_OK : FA_ERR_DEVICE;
}

namespace {
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct SearchLayout {
    int64_t desc, knots, ctrl, fitws, pinv, part, total, cstride, kstride;
};

SearchLayout search_layout(int32_t nblocks, const int32_t res[3], int32_t degree,
                           int32_t ncp_hi) {
    SearchLayout L{};
    const int64_t ncand = ncp_hi - (degree + 1) + 1;  // room for every ncp_lo
    L.cstride = align_up((int64_t)ncp_hi * ncp_hi * ncp_hi, 64);
    L.kstride = 3 * (int64_t)(ncp_hi + degree + 1);
    L.desc = 0;
    L.knots = align_up(L.desc + (int64_t)nblocks * (int64_t)sizeof(fa_block), 256);
    L.ctrl = align_up(L.knots + ncand * L.kstride * 4, 256);
    L.fitws = align_up(L.ctrl + (int64_t)nblocks * L.cstride * 4, 256);
    // per-candidate pseudo-inverses (3 axes each)
    L.pinv = align_up(L.fitws + fit_workspace_bytes(nblocks, res[0], res[1], ncp_hi), 256);
    L.part = align_up(L.pinv + ncand * 3 * pinv_doubles() * 8, 256);
    // (max, sum of squares) per decode item
    L.total = align_up(L.part + (int64_t)nblocks * items_per_block(res, resolve(nullptr)) * 16,
                       256);
    return L;
}

bool search_args_ok(int32_t nblocks, const int32_t res[3], int32_t degree, int32_t ncp_lo,
                    int32_t ncp_hi) {
    if (nblocks <= 0 || !res_ok(res) || degree < 1 || ncp_lo < degree + 1 || ncp_hi < ncp_lo)
        return false;
    for (int a = 0; a < 3; ++a)
        if (ncp_hi > res[a]) return false;  // full column rank needs ncp <= res
    return true;
}

bool search_supported(const int32_t res[3], int32_t degree, int32_t ncp_hi) {
    return degree <= FA_MAX_DEGREE && ncp_hi <= FA_MAX_NCP && res[0] <= 64 && res[1] <= 64 &&
           res[2] <= 64;
}
}  // namespace

int64_t fa_ncp_search_workspace(int32_t nblocks, const int32_t res[3], int32_t degree,
                                int32_t ncp_hi) {
    if (nblocks <= 0 || !res_ok(res) || degree < 1 || ncp_hi < degree + 1) return -1;
    return search_layout(nblocks, res, degree, ncp_hi).total;
}

fa_status fa_ncp_search(const float *samples, int32_t nblocks, const int32_t res[3],
                        int32_t degree, int32_t ncp_lo, int32_t ncp_hi, float *errs,
                        void *workspace, int64_t workspace_bytes, void *stream) {
    if (!samples || !errs || !workspace || !search_args_ok(nblocks, res, degree, ncp_lo, ncp_hi))
        return FA_ERR_INVALID_ARG;
    if (!search_supported(res, degree, ncp_hi)) return FA_ERR_UNSUPPORTED;
    const SearchLayout L = search_layout(nblocks, res, degree, ncp_hi);
    if (workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return FA_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(workspace);
    fa_block *desc = reinterpret_cast<fa_block *>(w + L.desc);
    float *knots = reinterpret_cast<float *>(w + L.knots);
    float *ctrl = reinterpret_cast<float *>(w + L.ctrl);
    const int ncand = ncp_hi - ncp_lo + 1;
    Tune t = resolve(nullptr);
    t.waves = kReduceWaves;
    const int64_t vox = (int64_t)res[0] * res[1] * res[2];
    double *xall = reinterpret_cast<double *>(w + L.pinv);
    // every candidate's knots and pseudo-inverses depend on (n, p, res) only:
    // built once for all candidates, in one launch
    hipError_t e = launch_pinv_candidates(knots, ncp_lo, ncand, degree, (int)L.kstride, res[0],
                                          res[1], res[2], xall, s);
    if (e != hipSuccess) return FA_ERR_DEVICE;
    // from the largest NCP down, as the in-level search runs (Sec. 4.2.1)
    for (int n = ncp_hi; n >= ncp_lo; --n) {
        float *kn = knots + (int64_t)(n - ncp_lo) * L.kstride;
        e = launch_candidate(desc, kn, nblocks, n, degree, L.cstride, s);
        if (e != hipSuccess) return FA_ERR_DEVICE;
        e = launch_fit_shared(desc, nblocks, kn, res[0], res[1], res[2], n, samples,
                              reinterpret_cast<double *>(w + L.fitws), xall + (int64_t)(n - ncp_lo) * 3 * pinv_doubles(),
                              ctrl, s);
        if (e != hipSuccess) return FA_ERR_DEVICE;
        // the candidate's value decode reduced straight to its error-map
        // entry (the decode itself is never stored)
        DecodeLaunch a = grid_args(desc, nblocks, kn, ctrl, FA_F32, res, 1u, t, nullptr,
                                   nullptr, nullptr);
        a.samples = samples;
        a.partials = reinterpret_cast<double *>(w + L.part);
        a.errs = errs + 2 * (n - ncp_lo);
        a.errs_stride = 2 * (int64_t)ncand;
        e = launch_decode_sep(a, t.waves, (int)std::min<int64_t>(a.nitems, default_grid(t, a.nitems)),
                              s);
        if (e == hipSuccess)
            e = launch_errors_combine(a.partials, nblocks, a.nrowt * a.ncolt, vox, a.errs,
                                      a.errs_stride, s);
        if (e != hipSuccess) return FA_ERR_DEVICE;
    }
    return FA_OK;
}

fa_status fa_ncp_select(const float *errs, int32_t nblocks, int32_t ncand, int32_t ncp_lo,
                        int32_t metric, float bound, int32_t *ncp_star, int32_t *complex_) {
    if (!errs || nblocks <= 0 || ncand <= 0 || (metric != 0 && metric != 1) || !ncp_star ||
        !std::isfinite(bound))
        return FA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < nblocks; ++b) {
        const float *eb = errs + (int64_t)b * ncand * 2 + metric;
        int best = -1;
        bool over = false;
        for (int c = 0; c < ncand; ++c) {
            const float v = eb[2 * c];
            if (best < 0 && v < bound) best = c;
            if (v > bound) over = true;
        }
        ncp_star[b] = ncp_lo + (best >= 0 ? best : ncand - 1);
        if (complex_) complex_[b] = over ? 1 : 0;
    }
    return FA_OK;
}

fa_status fa_search_set(int32_t level, const int32_t *parent_complex, int32_t *searched,
                        int32_t *search_ids, int32_t *nsearched) {
    if (level < 0 || level > 10 || !searched || !nsearched || (level > 0 && !parent_complex))
        return FA_ERR_INVALID_ARG;
    const int m = 1 << level, h = m >> 1;
    const int64_t nb = (int64_t)m * m * m;
    int32_t count = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int32_t on = 1;
        if (level > 0) {
            const int bx = (int)(b / ((int64_t)m * m)), by = (int)((b / m) % m), bz = (int)(b % m);
            const int64_t parent = ((int64_t)(bx / 2) * h + by / 2) * h + bz / 2;
            on = parent_complex[parent] != 0;
        }
        searched[b] = on;
        if (on) {
            if (search_ids) search_ids[count] = (int32_t)b;
            ++count;
        }
    }
    *nsearched = count;
    return FA_OK;
}

fa_status fa_level_select(int32_t nblocks, const int32_t *search_ids, int32_t nsearched,
                          const float *errs, int32_t ncand, int32_t ncp_lo, int32_t degree,
                          int32_t metric, float bound, int32_t *ncp_star, int32_t *complex_) {
    if (nblocks <= 0 || nsearched < 0 || nsearched > nblocks || (nsearched > 0 && !search_ids) ||
        (nsearched > 0 && !errs) || ncand <= 0 || degree < 1 || ncp_lo < degree + 1 ||
        !ncp_star || !complex_ || (metric != 0 && metric != 1) || !std::isfinite(bound))
        return FA_ERR_INVALID_ARG;
    for (int32_t i = 0; i < nsearched; ++i)
        if (search_ids[i] < 0 || search_ids[i] >= nblocks || (i > 0 && search_ids[i] <= search_ids[i - 1]))
            return FA_ERR_INVALID_ARG;
    // searched blocks first into scratch of the caller's outputs: the
    // selection rule of fa_ncp_select, then scattered to their indices
    std::vector<int32_t> ns(nsearched), cx(nsearched);
    if (nsearched > 0) {
        const fa_status st = fa_ncp_select(errs, nsearched, ncand, ncp_lo, metric, bound,
                                           ns.data(), cx.data());
        if (st != FA_OK) return st;
    }
    for (int32_t b = 0; b < nblocks; ++b) {
        ncp_star[b] = degree + 1;
        complex_[b] = 0;
    }
    for (int32_t i = 0; i < nsearched; ++i) {
        ncp_star[search_ids[i]] = ns[i];
        complex_[search_ids[i]] = cx[i];
    }
    return FA_OK;
}

fa_status fa_uniform_layout(int32_t nblocks, const int32_t *ncp, const int32_t *degree,
                            fa_block *blocks, float *knots, int64_t knot_capacity,
                            int64_t *nknots, int64_t *nctrl) {
    if (nblocks <= 0 || !ncp || !degree || !nknots || !nctrl) return FA_ERR_INVALID_ARG;
    int64_t ko = 0, co = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        const int p = degree[3 * b];
        if (p < 1 || degree[3 * b + 1] != p || degree[3 * b + 2] != p) return FA_ERR_INVALID_ARG;
        int64_t clen = 1;
        for (int a = 0; a < 3; ++a) {
            const int n = ncp[3 * b + a];
            if (n < p + 1) return FA_ERR_INVALID_ARG;
            clen *= n;
        }
        co = align_up(co, 64);
        if (blocks) {
            fa_block d{};
            for (int a = 0; a < 3; ++a) {
                d.ncp[a] = ncp[3 * b + a];
                d.degree[a] = p;
            }
            d.knot_off = ko;
            d.ctrl_off = co;
            d.scale = 1.0f;
            d.flags = FA_FLAG_UNIFORM_X | FA_FLAG_UNIFORM_Y | FA_FLAG_UNIFORM_Z;
            blocks[b] = d;
        }
        for (int a = 0; a < 3; ++a) {
            const int n = ncp[3 * b + a];
            if (knots) {
                if (ko + n + p + 1 > knot_capacity) return FA_ERR_INVALID_ARG;
                for (int j = 0; j < n + p + 1; ++j)
                    knots[ko + j] = j <= p ? 0.0f
                                           : (j >= n ? 1.0f : (float)(j - p) / (float)(n - p));
            }
            ko += n + p + 1;
        }
        co += clen;
    }
    *nknots = ko;
    *nctrl = align_up(co, 64);
    return FA_OK;
}
}  // extern "C"
