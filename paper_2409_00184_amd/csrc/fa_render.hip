// Direct volume rendering over micro-models (Alg. 4, Sec. 4.3.3).
//
// Front-to-back ray casting: for each pixel, samples along its ray are
// evaluated (value and gradient, the same code as the point query), mapped
// through an RGBA transfer function, shaded (two-sided Blinn-Phong from the
// gradient) and composited, until the accumulated opacity exceeds the
// threshold.  A wave marches an 8 x 8 tile of pixels in lockstep: at one
// sample index its 64 rays lie within a pixel footprint of each other, so
// they mostly share a micro-model and knot spans and their lattice gathers
// hit the same cache lines.  A wave stops when all of its rays have.
#include <algorithm>

#include "fa_eval.hpp"

namespace fa {
namespace {

struct RenderLaunch {
    QueryLaunch q;  // micro-models and lookup (xyz/out unused)
    const fa_ray *rays;
    int width, height;
    fa_render_params p;
    const float *tf;
    float *image;
};

template <int DT>
__global__ __launch_bounds__(256) void render_kernel(RenderLaunch a) {
#pragma clang fp contract(off)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tw = (a.width + 7) / 8, th = (a.height + 7) / 8;
    const int64_t tiles = (int64_t)tw * th;
    const int64_t wstride = (int64_t)gridDim.x * 4;
    for (int64_t t = (int64_t)xcd_order(blockIdx.x, gridDim.x) * 4 + wave; t < tiles; t += wstride) {
        const int px = (int)(t % tw) * 8 + (lane & 7);
        const int py = (int)(t / tw) * 8 + (lane >> 3);
        const bool pix = px < a.width && py < a.height;
        fa_ray r{};
        if (pix) r = a.rays[(int64_t)py * a.width + px];
        const float dt = (r.t1 - r.t0) / (float)a.p.samples;
        bool active = pix && r.t1 > r.t0;
        // half vector of this ray (V = -d)
        float hx = a.p.light[0] - r.dir[0], hy = a.p.light[1] - r.dir[1],
              hz = a.p.light[2] - r.dir[2];
        const float hn = sqrtf(hx * hx + hy * hy + hz * hz);
        if (hn > 0.0f) {
            hx /= hn;
            hy /= hn;
            hz /= hn;
        }
        float cr = 0.0f, cg = 0.0f, cb = 0.0f, ca = 0.0f;
        const float tscale = (float)(a.p.tf_size - 1) / (a.p.tf_hi - a.p.tf_lo);
        for (int s = 0; s < a.p.samples; ++s) {
            if (!__any(active)) break;
            const float ts = ((float)s + 0.5f) * dt;
            const float tt = r.t0 + ts;
            const float x = r.origin[0] + tt * r.dir[0];
            const float y = r.origin[1] + tt * r.dir[1];
            const float z = r.origin[2] + tt * r.dir[2];
            const float4 e = eval_point<DT>(a.q, x, y, z, active);
            if (!active) continue;
            // transfer function (linear interpolation of RGBA entries)
            float q = (e.x - a.p.tf_lo) * tscale;
            q = fminf(fmaxf(q, 0.0f), (float)(a.p.tf_size - 1));
            int i = (int)q;
            if (i > a.p.tf_size - 2) i = a.p.tf_size - 2;
            const float f = q - (float)i;
            const float4 t0 = reinterpret_cast<const float4 *>(a.tf)[i];
            const float4 t1 = reinterpret_cast<const float4 *>(a.tf)[i + 1];
            const float al = t0.w + f * (t1.w - t0.w);
            if (al > 0.0f) {
                float shade = a.p.ka;
                const float gl = sqrtf(e.y * e.y + e.z * e.z + e.w * e.w);
                if (gl > a.p.grad_min) {
                    const float nx = e.y / gl, ny = e.z / gl, nz = e.w / gl;
                    const float dl = fabsf(nx * a.p.light[0] + ny * a.p.light[1] + nz * a.p.light[2]);
                    const float dh = fabsf(nx * hx + ny * hy + nz * hz);
                    shade = a.p.ka + a.p.kd * dl + a.p.ks * powf(dh, a.p.shininess);
                }
                const float w = (1.0f - ca) * al;
                cr += w * (t0.x + f * (t1.x - t0.x)) * shade;
                cg += w * (t0.y + f * (t1.y - t0.y)) * shade;
                cb += w * (t0.z + f * (t1.z - t0.z)) * shade;
                ca += w;
                if (ca > a.p.opacity_max) active = false;  // early termination (Alg. 4)
            }
        }
        if (pix) {
            const f32x4 o = {cr, cg, cb, ca};
            reinterpret_cast<f32x4 *>(a.image)[(int64_t)py * a.width + px] = o;
        }
    }
}

// Visible micro-models of a view (Alg. 2): flags[cell] = 1 for every cell
// that a sample of fa_render_rays would look up (same sample positions,
// same lookup), 0 for the others.  One thread per (ray, chunk of samples);
// a thread stores only when its cell changes along the ray.
__global__ __launch_bounds__(256) void visible_kernel(const fa_ray *rays, int64_t nrays,
                                                      int samples, int chunk, int nb0, int nb1,
                                                      int nb2, float o0, float o1, float o2,
                                                      float r0, float r1, float r2,
                                                      int32_t *flags) {
#pragma clang fp contract(off)
    const int nch = (samples + chunk - 1) / chunk;
    const int64_t total = nrays * nch;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ri = w / nch;
        const int c = (int)(w - ri * nch);
        const fa_ray r = rays[ri];
        if (!(r.t1 > r.t0)) continue;
        const float dt = (r.t1 - r.t0) / (float)samples;
        int last = -1;
        const int s1 = (c + 1) * chunk < samples ? (c + 1) * chunk : samples;
        for (int s = c * chunk; s < s1; ++s) {
            const float ts = ((float)s + 0.5f) * dt;
            const float tt = r.t0 + ts;
            const float x = r.origin[0] + tt * r.dir[0];
            const float y = r.origin[1] + tt * r.dir[1];
            const float z = r.origin[2] + tt * r.dir[2];
            float u;
            const int bx = lookup_axis(x, o0, r0, nb0, u);
            const int by = lookup_axis(y, o1, r1, nb1, u);
            const int bz = lookup_axis(z, o2, r2, nb2, u);
            const int cell = (bx * nb1 + by) * nb2 + bz;
            if (cell != last) {
                flags[cell] = 1;
                last = cell;
            }
        }
    }
}

__global__ void fill_kernel(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

hipError_t launch_visible(const fa_ray *rays, int64_t nrays, int samples, const int nb[3],
                          const float origin[3], const float rscale[3], int32_t *flags,
                          hipStream_t s) {
    const int64_t ncells = (int64_t)nb[0] * nb[1] * nb[2];
    const int fgrid = (int)std::min<int64_t>((ncells + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(fgrid), dim3(256), 0, s, flags, ncells);
    const int chunk = 64;
    const int64_t work = nrays * ((samples + chunk - 1) / chunk);
    const int grid = (int)std::min<int64_t>((work + 255) / 256, 65536);
    hipLaunchKernelGGL(visible_kernel, dim3(grid), dim3(256), 0, s, rays, nrays, samples, chunk,
                       nb[0], nb[1], nb[2], origin[0], origin[1], origin[2], rscale[0],
                       rscale[1], rscale[2], flags);
    return hipGetLastError();
}

hipError_t launch_render(const QueryLaunch &q, const fa_ray *rays, int width, int height,
                         const fa_render_params &p, const float *tf, float *image,
                         hipStream_t s) {
    RenderLaunch a{};
    a.q = q;
    a.rays = rays;
    a.width = width;
    a.height = height;
    a.p = p;
    a.tf = tf;
    a.image = image;
    const int64_t tiles = (int64_t)((width + 7) / 8) * ((height + 7) / 8);
    int64_t wgs = (tiles + 3) / 4;
    const int grid = (int)(wgs < 65536 ? wgs : 65536);
    if (q.dtype == FA_BF16) hipLaunchKernelGGL(render_kernel<FA_BF16>, dim3(grid), dim3(256), 0, s, a);
    else if (q.dtype == FA_F16) hipLaunchKernelGGL(render_kernel<FA_F16>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(render_kernel<FA_F32>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fa
