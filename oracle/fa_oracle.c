/*
 * FP64 CPU oracle for micro-model decode and query (test infrastructure).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the
 * HIP path; it is the plain definition of a clamped tensor-product B-spline
 * and its partial derivatives, evaluated point by point in double precision.
 *
 * What is evaluated (paper: Sec. 4.2 states that each micro-model is an MFA
 * tensor-product B-spline giving value and derivative anywhere in its block;
 * Alg. 4 calls valueMicroModel / gradientMicroModel per ray sample; Eq. 2 and
 * the micro-model layout figure fix the content of a micro-model: knot
 * vectors plus a lattice of control points):
 *
 *   f(u,v,w) = sum_i sum_j sum_k N_{i,px}(u) N_{j,py}(v) N_{k,pz}(w) P[i][j][k]
 *
 * with N_{i,p} the B-spline basis of de Boor's recursion (the spline basis
 * the paper cites in Sec. 1):
 *   N_{i,0}(u) = 1 if t_i <= u < t_{i+1}, else 0   (u = t_n belongs to the
 *                last non-empty interval)
 *   N_{i,k}(u) = (u - t_i)/(t_{i+k} - t_i) N_{i,k-1}(u)
 *              + (t_{i+k+1} - u)/(t_{i+k+1} - t_{i+1}) N_{i+1,k-1}(u)
 *   with any term whose denominator is zero taken as 0, and
 *   N'_{i,p}(u) = p N_{i,p-1}(u)/(t_{i+p} - t_i)
 *               - p N_{i+1,p-1}(u)/(t_{i+p+1} - t_{i+1}).
 *
 * Layout conventions (the interface shared with the GPU path, not code):
 *   lattice of a block: C order [x][y][z], element (i,j,k) at
 *     ctrl_off + (i*ny + j)*nz + k;
 *   knots of a block: knot_off -> x knots (nx+px+1), then y knots, then z;
 *   decode grid: position i on an axis of resolution R is the FP32 value
 *     (float)i / (float)(R-1), so both sides take the span decision on the
 *     same number;
 *   decode output: [block][channel][Rx][Ry][Rz], channels (value, d/du,
 *     d/dv, d/dw) restricted to the bits of the channel mask, in that order.
 *
 * Parity of this file is pinned by the CPU tests (partition of unity,
 * Bernstein closed form, cardinal cubic values, linear and quadratic
 * reproduction, endpoint interpolation and derivative, finite differences,
 * brute force over all basis functions on tiny lattices, adjoint dot-product
 * identity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXP 7

/* ------------------------------------------------------------------ */
/* one axis                                                            */
/* ------------------------------------------------------------------ */

/* Knot span: the largest s in [p, n-1] with t[s] <= u.  u at or beyond the
 * right end t[n] maps to the last span n-1.  Plain linear scan. */
int orc_find_span(int n, int p, const double *t, double u)
{
    if (u >= t[n])
        return n - 1;
    int s = p;
    while (s + 1 <= n - 1 && t[s + 1] <= u)
        s++;
    return s;
}

/* The p+1 basis functions that are non-zero on span s, N_{s-p+r,p}(u) for
 * r = 0..p, and their first derivatives, straight from the recursion above.
 * tab[k][r] holds N_{s-k+r,k}(u). */
void orc_basis(int p, const double *t, int s, double u, double *N, double *dN)
{
    double tab[ORC_MAXP + 1][ORC_MAXP + 1];
    memset(tab, 0, sizeof tab);
    tab[0][0] = 1.0; /* N_{s,0} = 1: u lies in span s by construction */
    for (int k = 1; k <= p; k++) {
        for (int r = 0; r <= k; r++) {
            int i = s - k + r;
            /* N_{i,k-1} sits at row k-1, column r-1; N_{i+1,k-1} at column r */
            double a = (r >= 1) ? tab[k - 1][r - 1] : 0.0;
            double b = (r <= k - 1) ? tab[k - 1][r] : 0.0;
            double d1 = t[i + k] - t[i];
            double d2 = t[i + k + 1] - t[i + 1];
            double v = 0.0;
            if (d1 != 0.0)
                v += (u - t[i]) / d1 * a;
            if (d2 != 0.0)
                v += (t[i + k + 1] - u) / d2 * b;
            tab[k][r] = v;
        }
    }
    for (int r = 0; r <= p; r++) {
        int i = s - p + r;
        N[r] = tab[p][r];
        double d = 0.0;
        if (p >= 1) {
            double a = (r >= 1) ? tab[p - 1][r - 1] : 0.0; /* N_{i,p-1}   */
            double b = (r <= p - 1) ? tab[p - 1][r] : 0.0;  /* N_{i+1,p-1} */
            double d1 = t[i + p] - t[i];
            double d2 = t[i + p + 1] - t[i + 1];
            if (d1 != 0.0)
                d += p * a / d1;
            if (d2 != 0.0)
                d -= p * b / d2;
        }
        dN[r] = d;
    }
}

/* ------------------------------------------------------------------ */
/* one point of one block                                              */
/* ------------------------------------------------------------------ */

/* Value and the three partials with respect to the block parameters
 * (u,v,w) in [0,1]^3 (clamped).  abs_out (may be NULL) receives, per
 * channel, sum |basis product| * |P|, the scale of the rounding error of
 * any evaluation order. */
void orc_eval_point(const int32_t ncp[3], const int32_t deg[3],
                    const double *knots /* x then y then z */,
                    const double *P, const double uvw[3],
                    double out[4], double abs_out[4])
{
    const double *t[3];
    t[0] = knots;
    t[1] = t[0] + ncp[0] + deg[0] + 1;
    t[2] = t[1] + ncp[1] + deg[1] + 1;
    int s[3];
    double N[3][ORC_MAXP + 1], D[3][ORC_MAXP + 1];
    for (int a = 0; a < 3; a++) {
        double u = uvw[a];
        if (u < 0.0) u = 0.0;
        if (u > 1.0) u = 1.0;
        s[a] = orc_find_span(ncp[a], deg[a], t[a], u);
        orc_basis(deg[a], t[a], s[a], u, N[a], D[a]);
    }
    double f = 0, fx = 0, fy = 0, fz = 0;
    double af = 0, afx = 0, afy = 0, afz = 0;
    for (int ri = 0; ri <= deg[0]; ri++) {
        int i = s[0] - deg[0] + ri;
        for (int rj = 0; rj <= deg[1]; rj++) {
            int j = s[1] - deg[1] + rj;
            for (int rk = 0; rk <= deg[2]; rk++) {
                int k = s[2] - deg[2] + rk;
                double c = P[((int64_t)i * ncp[1] + j) * ncp[2] + k];
                double bv = N[0][ri] * N[1][rj] * N[2][rk];
                double bx = D[0][ri] * N[1][rj] * N[2][rk];
                double by = N[0][ri] * D[1][rj] * N[2][rk];
                double bz = N[0][ri] * N[1][rj] * D[2][rk];
                f += bv * c;
                fx += bx * c;
                fy += by * c;
                fz += bz * c;
                af += fabs(bv * c);
                afx += fabs(bx * c);
                afy += fabs(by * c);
                afz += fabs(bz * c);
            }
        }
    }
    out[0] = f; out[1] = fx; out[2] = fy; out[3] = fz;
    if (abs_out) {
        abs_out[0] = af; abs_out[1] = afx; abs_out[2] = afy; abs_out[3] = afz;
    }
}

/* ------------------------------------------------------------------ */
/* decode grids                                                        */
/* ------------------------------------------------------------------ */

static double grid_pos(int i, int R)
{
    /* the FP32 grid position, widened exactly */
    float q = (float)i / (float)(R - 1);
    return (double)q;
}

static int popcount4(uint32_t m)
{
    int c = 0;
    for (int b = 0; b < 4; b++)
        c += (m >> b) & 1u;
    return c;
}

/* Decode every block on its full Rx x Ry x Rz grid.
 * out: [nblocks][nch][Rx][Ry][Rz], nch = popcount(mask & 15). */
void orc_decode_blocks(int32_t nblocks, const int32_t *ncp /* [nb][3] */,
                       const int32_t *deg /* [nb][3] */,
                       const int64_t *knot_off, const int64_t *ctrl_off,
                       const double *knots, const double *ctrl,
                       const int32_t res[3], uint32_t mask, double *out,
                       int nthreads)
{
    const int Rx = res[0], Ry = res[1], Rz = res[2];
    const int nch = popcount4(mask & 15u);
    const int64_t vox = (int64_t)Rx * Ry * Rz;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int b = 0; b < nblocks; b++) {
        for (int x = 0; x < Rx; x++) {
            for (int y = 0; y < Ry; y++) {
                for (int z = 0; z < Rz; z++) {
                    double uvw[3] = {grid_pos(x, Rx), grid_pos(y, Ry), grid_pos(z, Rz)};
                    double r[4];
                    orc_eval_point(ncp + 3 * b, deg + 3 * b, knots + knot_off[b],
                                   ctrl + ctrl_off[b], uvw, r, NULL);
                    int c = 0;
                    for (int ch = 0; ch < 4; ch++) {
                        if (!((mask >> ch) & 1u))
                            continue;
                        int64_t o = ((int64_t)b * nch + c) * vox +
                                    ((int64_t)x * Ry + y) * Rz + z;
                        out[o] = r[ch];
                        c++;
                    }
                }
            }
        }
    }
}

/* Decode selected voxels: sample m is (block, x, y, z) = idx[4m..4m+3].
 * out: [m][4] (all four channels), abs_out: [m][4] or NULL. */
void orc_decode_samples(int64_t m, const int32_t *idx, const int32_t *ncp,
                        const int32_t *deg, const int64_t *knot_off,
                        const int64_t *ctrl_off, const double *knots,
                        const double *ctrl, const int32_t res[3], double *out,
                        double *abs_out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; q++) {
        int b = idx[4 * q];
        double uvw[3] = {grid_pos(idx[4 * q + 1], res[0]),
                         grid_pos(idx[4 * q + 2], res[1]),
                         grid_pos(idx[4 * q + 3], res[2])};
        orc_eval_point(ncp + 3 * b, deg + 3 * b, knots + knot_off[b],
                       ctrl + ctrl_off[b], uvw, out + 4 * q,
                       abs_out ? abs_out + 4 * q : NULL);
    }
}

/* Evaluate arbitrary block-parameter positions: sample m is block blk[m] at
 * uvw[3m..3m+2] (double).  out: [m][4]. */
void orc_eval_params(int64_t m, const int32_t *blk, const double *uvw,
                     const int32_t *ncp, const int32_t *deg,
                     const int64_t *knot_off, const int64_t *ctrl_off,
                     const double *knots, const double *ctrl, double *out,
                     double *abs_out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; q++) {
        int b = blk[q];
        orc_eval_point(ncp + 3 * b, deg + 3 * b, knots + knot_off[b],
                       ctrl + ctrl_off[b], uvw + 3 * q, out + 4 * q,
                       abs_out ? abs_out + 4 * q : NULL);
    }
}

/* ------------------------------------------------------------------ */
/* point query over a tiled domain                                     */
/* ------------------------------------------------------------------ */

/* Block lookup, taken in FP32 exactly as the query kernel takes it (an
 * integer decided by floating point is decided in the same precision on
 * both sides).  This translation unit is compiled without FP contraction,
 * so every line below is one correctly rounded FP32 operation:
 *   r   = (float)nb / extent            (host side, once per axis)
 *   q   = (x - origin) * r, clamped to [0, nb]
 *   b   = min(floor(q), nb - 1)
 *   u   = q - b                          (exact)
 * The gradient is taken with respect to x: d/dx = r * d/du. */
/* One point: FP32 lookup, FP64 evaluation, chain rule.  Returns 0 for an
 * empty cell (outputs zero). */
static int query_one(const float p[3], const int32_t nb[3], const float origin[3],
                     const float r[3], const int32_t *block_of_cell, int32_t nblocks,
                     const int32_t *ncp, const int32_t *deg, const int64_t *knot_off,
                     const int64_t *ctrl_off, const double *knots, const double *ctrl,
                     double o[4], double ao[4])
{
    int bidx[3];
    double uvw[3];
    for (int a = 0; a < 3; a++) {
        float d = p[a] - origin[a];
        float g = d * r[a];
        float top = (float)nb[a];
        if (!(g >= 0.0f)) g = 0.0f; /* also maps NaN to 0 */
        if (g > top) g = top;
        int b = (int)floorf(g);
        if (b > nb[a] - 1) b = nb[a] - 1;
        float u = g - (float)b;
        bidx[a] = b;
        uvw[a] = (double)u;
    }
    int cell = (bidx[0] * nb[1] + bidx[1]) * nb[2] + bidx[2];
    int blk = block_of_cell[cell];
    if (blk < 0 || blk >= nblocks) {
        o[0] = o[1] = o[2] = o[3] = 0.0;
        if (ao)
            ao[0] = ao[1] = ao[2] = ao[3] = 0.0;
        return 0;
    }
    double loc[4], aloc[4];
    orc_eval_point(ncp + 3 * blk, deg + 3 * blk, knots + knot_off[blk], ctrl + ctrl_off[blk],
                   uvw, loc, aloc);
    o[0] = loc[0];
    for (int a = 0; a < 3; a++)
        o[1 + a] = loc[1 + a] * (double)r[a];
    if (ao) {
        ao[0] = aloc[0];
        for (int a = 0; a < 3; a++)
            ao[1 + a] = aloc[1 + a] * (double)r[a];
    }
    return 1;
}

/* Block lookup, taken in FP32 exactly as the query kernel takes it (an
 * integer decided by floating point is decided in the same precision on
 * both sides).  This translation unit is compiled without FP contraction,
 * so every line of the lookup is one correctly rounded FP32 operation:
 *   r   = (float)nb / extent            (host side, once per axis)
 *   q   = (x - origin) * r, clamped to [0, nb]
 *   b   = min(floor(q), nb - 1)
 *   u   = q - b                          (exact)
 * The gradient is taken with respect to x: d/dx = r * d/du.  A cell whose
 * block index is negative (or not below nblocks) is empty. */
void orc_query_points(int64_t n, const float *xyz /* [n][3] */,
                      const int32_t nb[3], const float origin[3],
                      const float extent[3], const int32_t *block_of_cell, int32_t nblocks,
                      const int32_t *ncp, const int32_t *deg,
                      const int64_t *knot_off, const int64_t *ctrl_off,
                      const double *knots, const double *ctrl,
                      double *out /* [n][4] */, double *abs_out, int nthreads)
{
    float r[3];
    for (int a = 0; a < 3; a++)
        r[a] = (float)nb[a] / extent[a];
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++)
        query_one(xyz + 3 * q, nb, origin, r, block_of_cell, nblocks, ncp, deg, knot_off,
                  ctrl_off, knots, ctrl, out + 4 * q, abs_out ? abs_out + 4 * q : NULL);
}

/* ------------------------------------------------------------------ */
/* direct volume rendering (ray casting)                               */
/* ------------------------------------------------------------------ */

/* Front-to-back ray casting of Alg. 4 (Sec. 4.3.3), per pixel:
 *   sample s at t = t0 + (s + 1/2) (t1 - t0) / S, positions in FP32 with one
 *   rounding per operation (the same numbers the GPU forms);
 *   value and gradient by query_one (FP32 lookup, FP64 evaluation);
 *   RGBA transfer function, linear between entries over [tf_lo, tf_hi];
 *   two-sided Blinn-Phong: rgb *= ka + kd |N.L| + ks |N.H|^shininess with
 *   N = g/|g|, V = -d, H = (L + V)/|L + V| (ka alone where |g| <= grad_min);
 *   C += (1 - A) a rgb, A += (1 - A) a; stop once A > opacity_max.
 * rays: [npix][8] = origin xyz, dir xyz, t0, t1 (FP32); tf: [tf_size][4];
 * image: [npix][4] = (C, A) in FP64. */
void orc_render(int64_t npix, const float *rays, int samples, float opacity_max,
                float tf_lo, float tf_hi, int tf_size, const float light[3], float ka,
                float kd, float ks, float shininess, float grad_min, const float *tf,
                const int32_t nb[3], const float origin[3], const float extent[3],
                const int32_t *block_of_cell, int32_t nblocks, const int32_t *ncp,
                const int32_t *deg, const int64_t *knot_off, const int64_t *ctrl_off,
                const double *knots, const double *ctrl, double *image, int nthreads)
{
    float r[3];
    for (int a = 0; a < 3; a++)
        r[a] = (float)nb[a] / extent[a];
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < npix; q++) {
        const float *ray = rays + 8 * q;
        double C[3] = {0, 0, 0}, A = 0.0;
        double *img = image + 4 * q;
        if (!(ray[7] > ray[6])) {
            img[0] = img[1] = img[2] = img[3] = 0.0;
            continue;
        }
        float dt = (ray[7] - ray[6]) / (float)samples;
        double H[3], hn = 0.0;
        for (int a = 0; a < 3; a++) {
            H[a] = (double)light[a] - (double)ray[3 + a];
            hn += H[a] * H[a];
        }
        hn = sqrt(hn);
        for (int a = 0; a < 3 && hn > 0.0; a++)
            H[a] /= hn;
        for (int s = 0; s < samples; s++) {
            float ts = ((float)s + 0.5f) * dt;
            float tt = ray[6] + ts;
            float p[3];
            for (int a = 0; a < 3; a++) {
                float step = tt * ray[3 + a];
                p[a] = ray[a] + step;
            }
            double e[4];
            query_one(p, nb, origin, r, block_of_cell, nblocks, ncp, deg, knot_off, ctrl_off,
                      knots, ctrl, e, NULL);
            double x = (e[0] - tf_lo) / ((double)tf_hi - tf_lo) * (tf_size - 1);
            if (x < 0.0) x = 0.0;
            if (x > tf_size - 1) x = tf_size - 1;
            int i = (int)floor(x);
            if (i > tf_size - 2) i = tf_size - 2;
            double f = x - i;
            double rgba[4];
            for (int c = 0; c < 4; c++)
                rgba[c] = (1.0 - f) * tf[4 * i + c] + f * tf[4 * (i + 1) + c];
            if (!(rgba[3] > 0.0))
                continue;
            double gl = sqrt(e[1] * e[1] + e[2] * e[2] + e[3] * e[3]);
            double shade = ka;
            if (gl > grad_min) {
                double dl = 0.0, dh = 0.0;
                for (int a = 0; a < 3; a++) {
                    dl += e[1 + a] / gl * light[a];
                    dh += e[1 + a] / gl * H[a];
                }
                shade = ka + kd * fabs(dl) + ks * pow(fabs(dh), shininess);
            }
            double w = (1.0 - A) * rgba[3];
            for (int c = 0; c < 3; c++)
                C[c] += w * rgba[c] * shade;
            A += w;
            if (A > opacity_max)
                break;
        }
        img[0] = C[0]; img[1] = C[1]; img[2] = C[2]; img[3] = A;
    }
}

/* ------------------------------------------------------------------ */
/* adjoint of the grid decode                                          */
/* ------------------------------------------------------------------ */

/* G = B^T g: for every voxel of every block, scatter the cotangents of the
 * selected channels onto the control points of its (p+1)^3 window, weighted
 * by the same basis products the forward decode uses.  g has the decode
 * output layout for `mask`; G has the lattice layout and is overwritten.
 * Blocks are distributed over threads (each block's lattice is written by
 * one thread only). */
void orc_decode_adjoint(int32_t nblocks, const int32_t *ncp, const int32_t *deg,
                        const int64_t *knot_off, const int64_t *ctrl_off,
                        const double *knots, const int32_t res[3], uint32_t mask,
                        const double *g, double *G, int nthreads)
{
    const int Rx = res[0], Ry = res[1], Rz = res[2];
    const int nch = popcount4(mask & 15u);
    const int64_t vox = (int64_t)Rx * Ry * Rz;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nblocks; b++) {
        const int32_t *n = ncp + 3 * b, *p = deg + 3 * b;
        double *Gb = G + ctrl_off[b];
        int64_t cnt = (int64_t)n[0] * n[1] * n[2];
        for (int64_t e = 0; e < cnt; e++)
            Gb[e] = 0.0;
        const double *t[3];
        t[0] = knots + knot_off[b];
        t[1] = t[0] + n[0] + p[0] + 1;
        t[2] = t[1] + n[1] + p[1] + 1;
        for (int x = 0; x < Rx; x++) {
            for (int y = 0; y < Ry; y++) {
                for (int z = 0; z < Rz; z++) {
                    double uvw[3] = {grid_pos(x, Rx), grid_pos(y, Ry), grid_pos(z, Rz)};
                    int s[3];
                    double N[3][ORC_MAXP + 1], D[3][ORC_MAXP + 1];
                    for (int a = 0; a < 3; a++) {
                        s[a] = orc_find_span(n[a], p[a], t[a], uvw[a]);
                        orc_basis(p[a], t[a], s[a], uvw[a], N[a], D[a]);
                    }
                    double gc[4] = {0, 0, 0, 0};
                    int c = 0;
                    for (int ch = 0; ch < 4; ch++) {
                        if (!((mask >> ch) & 1u))
                            continue;
                        gc[ch] = g[((int64_t)b * nch + c) * vox +
                                   ((int64_t)x * Ry + y) * Rz + z];
                        c++;
                    }
                    for (int ri = 0; ri <= p[0]; ri++) {
                        int i = s[0] - p[0] + ri;
                        for (int rj = 0; rj <= p[1]; rj++) {
                            int j = s[1] - p[1] + rj;
                            for (int rk = 0; rk <= p[2]; rk++) {
                                int k = s[2] - p[2] + rk;
                                double w = N[0][ri] * N[1][rj] * N[2][rk] * gc[0] +
                                           D[0][ri] * N[1][rj] * N[2][rk] * gc[1] +
                                           N[0][ri] * D[1][rj] * N[2][rk] * gc[2] +
                                           N[0][ri] * N[1][rj] * D[2][rk] * gc[3];
                                Gb[((int64_t)i * n[1] + j) * n[2] + k] += w;
                            }
                        }
                    }
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* one-axis helpers exported for the pin tests                         */
/* ------------------------------------------------------------------ */

/* For m parameters u[m] on one axis: span s[m], values N[m][p+1] and
 * derivatives dN[m][p+1]. */
void orc_axis_basis(int n, int p, const double *t, int64_t m, const double *u,
                    int32_t *s, double *N, double *dN)
{
    for (int64_t q = 0; q < m; q++) {
        double x = u[q];
        if (x < 0.0) x = 0.0;
        if (x > 1.0) x = 1.0;
        int sp = orc_find_span(n, p, t, x);
        s[q] = sp;
        orc_basis(p, t, sp, x, N + q * (p + 1), dN + q * (p + 1));
    }
}

int orc_max_degree(void) { return ORC_MAXP; }
