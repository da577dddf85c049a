"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no decode arithmetic: it only draws lattices, knot
vectors, ray samples and fields.  Both the HIP path and the FP64 oracle
consume what it returns; neither is imported here.

Recipes (all seeded with numpy.random.Generator(PCG64(seed))):

* knots: clamped uniform, t_0..t_p = 0, t_{p+j} = j/(n-p), t_n..t_{n+p} = 1,
  stored FP32 (micro-models store 4-byte values, Eq. 2).
* sinusoid field: f(x) = sum_{m=1..8} sin(2 pi <k_m, x> + phi_m), unit
  amplitudes, k_m ~ U[-3, 3]^3 cycles per block, phi_m ~ U[0, 2 pi).
* control points of a sinusoid block: f at the Greville abscissae of the
  block's knots (xi_i = mean of t_{i+1..i+p}), plus optional N(0, sigma^2).
* turbulence field: random-phase Fourier modes on a periodic m^3 grid with
  shell energy E(k) ~ k^(-5/3), i.e. mode amplitude ~ |k|^(-11/6), 1 <= |k|
  up to Nyquist, normalised to zero mean and unit variance, FP32.
* Marschner-Lobb field (Eq. 5) with f_M = 6, alpha = 0.05 on [0, 7]^3, and
  its analytic gradient (the ground truth of the quality workload).
* pyramids of micro-blocks: level k tiles the domain with (2^k)^3 blocks
  sharing their boundary samples, each sampled on its own R^3 grid.
"""
import math
from dataclasses import dataclass, field

import numpy as np

CTRL_ALIGN = 64  # lattice offsets are multiples of 64 elements (256 B in FP32)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def clamped_uniform_knots(n, p):
    """n + p + 1 clamped uniform knots on [0, 1] as FP32."""
    if n < p + 1:
        raise ValueError("need n >= p + 1")
    t = np.zeros(n + p + 1, np.float64)
    t[n:] = 1.0
    for j in range(1, n - p):
        t[p + j] = j / (n - p)
    return t.astype(np.float32)


def greville(t, n, p):
    """Greville abscissae xi_i = (t_{i+1} + ... + t_{i+p}) / p, i = 0..n-1."""
    t = np.asarray(t, np.float64)
    if p == 0:
        return 0.5 * (t[:n] + t[1:n + 1])
    return np.array([t[i + 1:i + p + 1].mean() for i in range(n)])


@dataclass
class Batch:
    """A packed batch of micro-models.

    ncp, deg: int32 [nb, 3]; knot_off, ctrl_off: int64 [nb];
    knots: float32 flat (per block: x, y, z knot vectors back to back);
    ctrl: float32 flat (per block: [x][y][z] lattice at ctrl_off);
    ctrl64: float64 source lattice when the recipe has one (else None).
    """
    ncp: np.ndarray
    deg: np.ndarray
    knot_off: np.ndarray
    ctrl_off: np.ndarray
    knots: np.ndarray
    ctrl: np.ndarray
    ctrl64: np.ndarray = None
    meta: dict = field(default_factory=dict)

    @property
    def nblocks(self):
        return int(self.ncp.shape[0])

    def lattice(self, b, src="ctrl"):
        n = self.ncp[b]
        a = getattr(self, src)
        o = int(self.ctrl_off[b])
        return a[o:o + int(n.prod())].reshape(int(n[0]), int(n[1]), int(n[2]))

    def block_knots(self, b):
        n, p = self.ncp[b], self.deg[b]
        o = int(self.knot_off[b])
        out = []
        for a in range(3):
            L = int(n[a] + p[a] + 1)
            out.append(self.knots[o:o + L])
            o += L
        return out


def pack(ncp, deg, knot_list, lattices, lattices64=None, align=CTRL_ALIGN):
    """Pack per-block knots ([kx, ky, kz]) and lattices into a Batch."""
    nb = len(ncp)
    ncp = np.asarray(ncp, np.int32).reshape(nb, 3)
    deg = np.asarray(deg, np.int32).reshape(nb, 3)
    knot_off = np.zeros(nb, np.int64)
    ctrl_off = np.zeros(nb, np.int64)
    ko = co = 0
    for b in range(nb):
        knot_off[b] = ko
        ko += sum(len(k) for k in knot_list[b])
        co = (co + align - 1) // align * align
        ctrl_off[b] = co
        co += int(np.prod(ncp[b]))
    total = (co + align - 1) // align * align
    knots = np.concatenate([np.concatenate([np.asarray(k, np.float32) for k in kl])
                            for kl in knot_list]).astype(np.float32)
    ctrl = np.zeros(total, np.float32)
    ctrl64 = np.zeros(total, np.float64) if lattices64 is not None else None
    for b in range(nb):
        o = int(ctrl_off[b])
        m = int(np.prod(ncp[b]))
        ctrl[o:o + m] = np.asarray(lattices[b], np.float32).reshape(-1)
        if ctrl64 is not None:
            ctrl64[o:o + m] = np.asarray(lattices64[b], np.float64).reshape(-1)
    return Batch(ncp, deg, knot_off, ctrl_off, knots, ctrl, ctrl64)


# ------------------------------------------------------------------ fields

def sinusoid_params(g, nterms=8, kmax=3.0):
    k = g.uniform(-kmax, kmax, size=(nterms, 3))
    phi = g.uniform(0.0, 2.0 * math.pi, size=nterms)
    return k, phi


def sinusoid_field(k, phi, x, y, z):
    """sum_m sin(2 pi (k_m . (x, y, z)) + phi_m), broadcasting x, y, z."""
    f = 0.0
    for m in range(k.shape[0]):
        f = f + np.sin(2.0 * math.pi * (k[m, 0] * x + k[m, 1] * y + k[m, 2] * z) + phi[m])
    return f


def sinusoid_lattice(k, phi, tx, ty, tz, n, p, offset=(0.0, 0.0, 0.0), scale=1.0):
    """Control points = field at the Greville abscissae (block-local -> field
    coordinates: offset + scale * xi)."""
    gx = offset[0] + scale * greville(tx, n[0], p[0])
    gy = offset[1] + scale * greville(ty, n[1], p[1])
    gz = offset[2] + scale * greville(tz, n[2], p[2])
    return sinusoid_field(k, phi, gx[:, None, None], gy[None, :, None], gz[None, None, :])


def turbulence_cube(g, m, nblocks=1):
    """[nblocks, m, m, m] float32 fields with E(k) ~ k^-5/3 (see module doc)."""
    kx = np.fft.fftfreq(m) * m
    kz = np.fft.rfftfreq(m) * m
    K = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(K)
    nz = K >= 1.0
    amp[nz] = K[nz] ** (-11.0 / 6.0)
    amp[K > m / 2] = 0.0
    out = np.empty((nblocks, m, m, m), np.float32)
    for b in range(nblocks):
        phase = g.uniform(0.0, 2.0 * math.pi, size=K.shape)
        spec = amp * np.exp(1j * phase)
        f = np.fft.irfftn(spec, s=(m, m, m), axes=(0, 1, 2))
        f = f - f.mean()
        sd = f.std()
        out[b] = (f / sd if sd > 0 else f).astype(np.float32)
    return out


# ----------------------------------------------------------------- configs

NCP_CHOICES_C2 = (8, 12, 16, 24, 32)


def config_c1(seed=1, n=16, p=3, sigma=0.01):
    """One block, degree p, n^3 control points = sinusoid field at the
    Greville abscissae + N(0, sigma^2), FP64 source (FP32 stored)."""
    g = rng(seed)
    k, phi = sinusoid_params(g)
    t = clamped_uniform_knots(n, p)
    P = sinusoid_lattice(k, phi, t, t, t, (n, n, n), (p, p, p))
    P = P + g.normal(0.0, sigma, size=P.shape)
    b = pack([(n, n, n)], [(p, p, p)], [[t, t, t]], [P], [P])
    b.meta.update(config="C1", res=(64, 64, 64))
    return b


def config_c2(seed=2, nblocks=512, ncp_choices=NCP_CHOICES_C2, deg_choices=(2, 3)):
    """Uneven NCP* per axis and degree per block; sinusoid field with a
    per-block offset o_b ~ U[0, 16)^3."""
    g = rng(seed)
    k, phi = sinusoid_params(g)
    ncp = g.choice(np.asarray(ncp_choices), size=(nblocks, 3))
    p = g.choice(np.asarray(deg_choices), size=nblocks)
    off = g.uniform(0.0, 16.0, size=(nblocks, 3))
    kl, lat = [], []
    for b in range(nblocks):
        n = tuple(int(v) for v in ncp[b])
        pp = int(p[b])
        ts = [clamped_uniform_knots(n[a], pp) for a in range(3)]
        kl.append(ts)
        lat.append(sinusoid_lattice(k, phi, ts[0], ts[1], ts[2], n, (pp, pp, pp), off[b]))
    out = pack(ncp, np.repeat(p[:, None], 3, axis=1), kl, lat)
    out.meta.update(config="C2", res=(64, 64, 64))
    return out


def jittered_knots(g, n, p, amount=0.3):
    """Clamped knots on [0, 1] whose interior knots are the uniform ones
    moved by up to amount/2 of a knot spacing each way (non-uniform, strictly
    increasing), FP32."""
    t = clamped_uniform_knots(n, p).astype(np.float64)
    h = 1.0 / (n - p)
    m = n - p - 1
    if m > 0:
        t[p + 1:n] += g.uniform(-0.5 * amount * h, 0.5 * amount * h, m)
    return t.astype(np.float32)


def config_c3_blocks(seed=3, nb=16, ncp_lo=8, ncp_hi=32, p=3, nonuniform=False):
    """nb^3 blocks tiling [0,1]^3; n_a ~ U{ncp_lo..ncp_hi}; one global
    sinusoid field (k in cycles per block) so neighbours agree at faces.
    nonuniform: every interior knot jittered (jittered_knots), drawn from a
    stream of its own so the NCP draws and the field stay those of the
    uniform configuration."""
    g = rng(seed)
    k, phi = sinusoid_params(g)
    ncp = g.integers(ncp_lo, ncp_hi + 1, size=(nb ** 3, 3))
    gk = rng(seed + 1000)
    kl, lat = [], []
    for bx in range(nb):
        for by in range(nb):
            for bz in range(nb):
                b = (bx * nb + by) * nb + bz
                n = tuple(int(v) for v in ncp[b])
                ts = [jittered_knots(gk, n[a], p) if nonuniform else
                      clamped_uniform_knots(n[a], p) for a in range(3)]
                kl.append(ts)
                # block-local xi in [0,1] -> field coordinate (b + xi) in blocks
                lat.append(sinusoid_lattice(k, phi, ts[0], ts[1], ts[2], n, (p, p, p),
                                            offset=(bx, by, bz)))
    out = pack(ncp, np.full((nb ** 3, 3), p, np.int32), kl, lat)
    out.meta.update(config="C3", nb=(nb, nb, nb), origin=(0.0, 0.0, 0.0),
                    extent=(1.0, 1.0, 1.0))
    return out


def identity_cells(nb):
    """block_of_cell for a batch laid out cell-major (bx, by, bz)."""
    return np.arange(int(np.prod(nb)), dtype=np.int32)


def camera_rays(seed, width, height, fov_v_deg=13.9, dist=2.0):
    """Seeded camera at distance `dist` from the centre of [0,1]^3, looking
    at it.  Returns (origins [R,3], dirs [R,3], t_in [R], t_out [R],
    jitter [R]) in float64, R = width * height, row-major pixels.  With the
    default field of view every ray meets the inscribed sphere, hence the
    cube."""
    g = rng(seed)
    c = np.array([0.5, 0.5, 0.5])
    v = g.normal(size=3)
    v /= np.linalg.norm(v)
    eye = c + dist * v
    fwd = (c - eye) / np.linalg.norm(c - eye)
    up0 = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up0)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_v_deg) / 2.0)
    aspect = width / height
    px = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    X, Y = np.meshgrid(px * th * aspect, py * th)
    d = fwd[None, :] + X.reshape(-1, 1) * right[None, :] + Y.reshape(-1, 1) * up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape).copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (0.0 - o) * inv
        t1 = (1.0 - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    jit = g.uniform(0.0, 1.0, size=d.shape[0])
    return o, d, tmin, tmax, jit


def render_rays(seed, width, height, fov_v_deg=13.9, dist=2.0):
    """Image rays of camera_rays as FP32 [width*height, 8] = (origin, unit
    direction, t_in, t_out); with a wide field of view some rays miss the
    cube and get t_out <= t_in."""
    o, d, t0, t1, _ = camera_rays(seed, width, height, fov_v_deg, dist)
    miss = ~(t1 > t0)
    t0 = np.where(miss, 0.0, t0)
    t1 = np.where(miss, -1.0, t1)
    return np.concatenate([o, d, t0[:, None], t1[:, None]], axis=1).astype(np.float32)


def transfer_function(seed, n=256, bumps=5, alpha_max=0.08):
    """Seeded RGBA transfer function table [n, 4] float32: colours in [0, 1]
    from a few Gaussian bumps per channel, opacity per sample in
    [0, alpha_max] with a transparent band around the middle of the range."""
    g = rng(seed)
    x = np.linspace(0.0, 1.0, n)
    tf = np.zeros((n, 4))
    for c in range(4):
        mu = g.uniform(0.0, 1.0, size=bumps)
        sd = g.uniform(0.04, 0.2, size=bumps)
        h = g.uniform(0.2, 1.0, size=bumps)
        f = (h[None, :] * np.exp(-0.5 * ((x[:, None] - mu[None, :]) / sd[None, :]) ** 2)).sum(1)
        tf[:, c] = f / f.max()
    tf[:, 3] *= alpha_max * (np.abs(x - 0.5) > 0.08)
    return tf.astype(np.float32)


def ray_samples_np(seed, width, height, nsamples):
    """Ray-major FP32 sample positions [width*height*nsamples, 3] (numpy).
    Sample s of a ray sits at t_in + (s + j)/nsamples * (t_out - t_in)."""
    o, d, t0, t1, j = camera_rays(seed, width, height)
    s = np.arange(nsamples, dtype=np.float64)
    t = t0[:, None] + (s[None, :] + j[:, None]) / nsamples * (t1 - t0)[:, None]
    xyz = o[:, None, :] + d[:, None, :] * t[:, :, None]
    return xyz.reshape(-1, 3).astype(np.float32)


def config_c4(seed=4, nblocks=256, res=64, ncp_choices=(16, 24, 32), p=3):
    """Fit targets: k^-5/3 samples on res^3 per block; n_a ~ {16,24,32};
    lattices start at zero."""
    g = rng(seed)
    ncp = g.choice(np.asarray(ncp_choices), size=(nblocks, 3))
    y = turbulence_cube(g, res, nblocks)
    kl, lat = [], []
    for b in range(nblocks):
        n = tuple(int(v) for v in ncp[b])
        kl.append([clamped_uniform_knots(n[a], p) for a in range(3)])
        lat.append(np.zeros(n, np.float32))
    out = pack(ncp, np.full((nblocks, 3), p, np.int32), kl, lat)
    out.meta.update(config="C4", res=(res, res, res))
    return out, y


def config_c5(seed=5, nblocks=4096, n=32, p=3):
    """nblocks lattices of n^3 control points, each a k^-5/3 field."""
    g = rng(seed)
    P = turbulence_cube(g, n, nblocks)
    t = clamped_uniform_knots(n, p)
    out = pack(np.full((nblocks, 3), n, np.int32), np.full((nblocks, 3), p, np.int32),
               [[t, t, t]] * nblocks, list(P))
    out.meta.update(config="C5", res=(64, 64, 64))
    return out


def voxel_subset(nblocks, res, frac=0.01, seed=55):
    """A seeded uniform sample, without replacement, of floor(frac * N) of the
    N = nblocks * res0 * res1 * res2 (block, voxel) pairs of a grid decode,
    as int32 [k, 4] rows (block, x, y, z) in increasing flat order.  At C5
    (4096 blocks of 64^3) the 1% sample holds 10,737,418 pairs."""
    res = tuple(int(r) for r in res)
    vox = res[0] * res[1] * res[2]
    total = int(nblocks) * vox
    flat = np.sort(rng(seed).choice(total, size=int(total * frac), replace=False))
    out = np.empty((flat.size, 4), np.int32)
    out[:, 0] = flat // vox
    r = flat % vox
    out[:, 1] = r // (res[1] * res[2])
    out[:, 2] = (r // res[2]) % res[1]
    out[:, 3] = r % res[2]
    return out


# ----------------------------------------------------------- Marschner-Lobb

ML_FM, ML_ALPHA, ML_EXTENT = 6.0, 0.05, 7.0


def ml_value(x, y, z, fm=ML_FM, alpha=ML_ALPHA, xp=np):
    """F = (1 - sin(pi z / 2) + alpha (1 + rho(sqrt(x^2 + y^2)))) / (2 (1 + alpha)),
    rho(r) = cos(2 pi f_M cos(pi r / 2))  (Eq. 5).  xp: numpy or torch."""
    r = xp.sqrt(x * x + y * y)
    rho = xp.cos(2.0 * math.pi * fm * xp.cos(math.pi * r / 2.0))
    return (1.0 - xp.sin(math.pi * z / 2.0) + alpha * (1.0 + rho)) / (2.0 * (1.0 + alpha))


def ml_gradient(x, y, z, fm=ML_FM, alpha=ML_ALPHA, xp=np):
    """(dF/dx, dF/dy, dF/dz) of ml_value, differentiated by hand:
    drho/dr = pi^2 f_M sin(pi r / 2) sin(2 pi f_M cos(pi r / 2)), and
    dr/dx = x / r (the x, y derivatives vanish at r = 0)."""
    c = 1.0 / (2.0 * (1.0 + alpha))
    r = xp.sqrt(x * x + y * y)
    drho = math.pi ** 2 * fm * xp.sin(math.pi * r / 2.0) * xp.sin(
        2.0 * math.pi * fm * xp.cos(math.pi * r / 2.0))
    safe = xp.where(r > 0, r, xp.ones_like(r))
    k = xp.where(r > 0, c * alpha * drho / safe, xp.zeros_like(r))
    gz = -c * (math.pi / 2.0) * xp.cos(math.pi * z / 2.0)
    return k * x, k * y, gz + 0.0 * x


def block_grid(level, b, R, extent=ML_EXTENT, lo=0.0):
    """Sample coordinates (x [R], y [R], z [R], float64) of block b of level
    `level` (block (bx, by, bz) at index (bx * m + by) * m + bz, m = 2^level),
    neighbours sharing boundary samples: x_i = lo + extent (bx + i/(R-1)) / m."""
    m = 1 << level
    bx, by, bz = b // (m * m), (b // m) % m, b % m
    u = np.arange(R, dtype=np.float64) / (R - 1)
    h = extent / m
    return lo + h * (bx + u), lo + h * (by + u), lo + h * (bz + u)


def ml_blocks(level, R, blocks=None, extent=ML_EXTENT):
    """FP32 samples [nb, R, R, R] of the Marschner-Lobb field on the blocks
    of one pyramid level (all blocks, or the listed ones)."""
    m = 1 << level
    ids = range(m ** 3) if blocks is None else blocks
    out = []
    for b in ids:
        x, y, z = block_grid(level, b, R, extent)
        out.append(ml_value(x[:, None, None], y[None, :, None], z[None, None, :]))
    return np.asarray(out, np.float32)

