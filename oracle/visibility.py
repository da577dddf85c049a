"""Visible micro-models of a view -- TEST INFRASTRUCTURE (oracle side).

Only tests/ may import this module.  For the ray caster of Alg. 4, the
micro-models a view needs (the first step of Alg. 2) are the cells its
samples fall in.  Sample positions and the block lookup are formed in FP32
with one rounding per operation, exactly as the ray caster states them:
  dt = (t1 - t0) / S;  t = t0 + ((float)s + 0.5f) * dt;  x = o + t * d;
  g = (x - origin) * (nb / extent), clamped to [0, nb], b = min(floor(g), nb - 1).
The decision is an integer taken in the kernel's precision (FP32) on both
sides, so the sets must be equal.
"""
import numpy as np


def visible_cells(rays, samples, nb, origin, extent):
    """int32 flags [nb0 * nb1 * nb2] for FP32 rays [n, 8]."""
    f32 = np.float32
    rays = np.asarray(rays, f32).reshape(-1, 8)
    nb = [int(v) for v in nb]
    o = np.asarray(origin, f32)
    r = np.asarray(nb, f32) / np.asarray(extent, f32)
    flags = np.zeros(nb[0] * nb[1] * nb[2], np.int32)
    hit = rays[:, 7] > rays[:, 6]
    R = rays[hit]
    dt = (R[:, 7] - R[:, 6]) / f32(samples)
    s = np.arange(samples, dtype=f32)
    ts = (s[None, :] + f32(0.5)) * dt[:, None]
    tt = R[:, 6][:, None] + ts
    cell = np.zeros(tt.shape, np.int64)
    for a in range(3):
        x = R[:, a][:, None] + tt * R[:, 3 + a][:, None]
        g = (x - o[a]) * r[a]
        g = np.where(g >= f32(0), g, f32(0))  # also NaN -> 0
        g = np.minimum(g, f32(nb[a]))
        b = np.minimum(np.floor(g).astype(np.int64), nb[a] - 1)
        cell = cell * nb[a] + b
    flags[np.unique(cell)] = 1
    return flags
