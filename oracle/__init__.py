"""FP64 CPU oracle for micro-model decode and query -- TEST INFRASTRUCTURE.

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import this package.  The product path (paper_2409_00184_amd)
never imports it and shares no code with it.

Functions take plain numpy arrays describing a batch of micro-models:
  ncp      int32 [nb, 3]   control points per axis (x, y, z)
  deg      int32 [nb, 3]   degree per axis
  knot_off int64 [nb]      offset of the block's x knots in `knots`
                           (y and z knots follow)
  ctrl_off int64 [nb]      offset of the block's [x][y][z] lattice in `ctrl`
  knots    float64 [*]     (exact copies of the stored FP32 knots)
  ctrl     float64 [*]

Every routine follows the plain definition of a clamped tensor-product
B-spline (fa_oracle.c states it); `brute` holds a second, structurally
different implementation for tiny lattices.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_find_span.restype = ctypes.c_int
    lib.orc_find_span.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_double]
    lib.orc_axis_basis.restype = None
    lib.orc_axis_basis.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, ctypes.c_int64,
                                   _f64p, _i32p, _f64p, _f64p]
    lib.orc_eval_point.restype = None
    lib.orc_eval_point.argtypes = [_i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_decode_blocks.restype = None
    lib.orc_decode_blocks.argtypes = [ctypes.c_int32, _i32p, _i32p, _i64p, _i64p,
                                      _f64p, _f64p, _i32p, ctypes.c_uint32, _f64p,
                                      ctypes.c_int]
    lib.orc_decode_samples.restype = None
    lib.orc_decode_samples.argtypes = [ctypes.c_int64, _i32p, _i32p, _i32p, _i64p, _i64p,
                                       _f64p, _f64p, _i32p, _f64p, ctypes.c_void_p,
                                       ctypes.c_int]
    lib.orc_eval_params.restype = None
    lib.orc_eval_params.argtypes = [ctypes.c_int64, _i32p, _f64p, _i32p, _i32p, _i64p,
                                    _i64p, _f64p, _f64p, _f64p, ctypes.c_void_p,
                                    ctypes.c_int]
    lib.orc_query_points.restype = None
    lib.orc_query_points.argtypes = [ctypes.c_int64, _f32p, _i32p, _f32p, _f32p, _i32p,
                                     ctypes.c_int32, _i32p, _i32p, _i64p, _i64p, _f64p, _f64p,
                                     _f64p, ctypes.c_void_p, ctypes.c_int]
    lib.orc_render.restype = None
    lib.orc_render.argtypes = [ctypes.c_int64, _f32p, ctypes.c_int, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_int, _f32p,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, _f32p, _i32p, _f32p, _f32p, _i32p,
                               ctypes.c_int32, _i32p, _i32p,
                               _i64p, _i64p, _f64p, _f64p, _f64p, ctypes.c_int]
    lib.orc_decode_adjoint.restype = None
    lib.orc_decode_adjoint.argtypes = [ctypes.c_int32, _i32p, _i32p, _i64p, _i64p, _f64p,
                                       _i32p, ctypes.c_uint32, _f64p, _f64p, ctypes.c_int]
    _lib = lib
    return lib


class using:
    """Context manager: route every call of this module through the oracle
    library at `path` (used by the tests that plant mistakes in a copy of
    the oracle and check that the pins catch them)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib, _LIB_PATH
        self._saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        return _load()

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self._saved
        return False


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def nthreads_default():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# ---------------------------------------------------------------- one axis

def find_span(n, p, t, u):
    """Largest s in [p, n-1] with t[s] <= u (u >= t[n] -> n-1)."""
    return _load().orc_find_span(int(n), int(p), _c(t, np.float64), float(u))


def axis_basis(n, p, t, u):
    """Spans [m], basis values [m, p+1] and derivatives [m, p+1] on one axis."""
    u = _c(np.atleast_1d(u), np.float64)
    m = u.shape[0]
    s = np.empty(m, np.int32)
    N = np.empty((m, p + 1), np.float64)
    dN = np.empty((m, p + 1), np.float64)
    _load().orc_axis_basis(int(n), int(p), _c(t, np.float64), m, u, s, N, dN)
    return s, N, dN


# ------------------------------------------------------------------ blocks

class Blocks:
    """FP64 view of a batch of micro-models (see module docstring)."""

    def __init__(self, ncp, deg, knot_off, ctrl_off, knots, ctrl):
        self.ncp = _c(ncp, np.int32).reshape(-1, 3)
        self.deg = _c(deg, np.int32).reshape(-1, 3)
        self.knot_off = _c(knot_off, np.int64).reshape(-1)
        self.ctrl_off = _c(ctrl_off, np.int64).reshape(-1)
        self.knots = _c(knots, np.float64).reshape(-1)
        self.ctrl = _c(ctrl, np.float64).reshape(-1)

    @property
    def nblocks(self):
        return self.ncp.shape[0]

    def with_ctrl(self, ctrl):
        return Blocks(self.ncp, self.deg, self.knot_off, self.ctrl_off, self.knots, ctrl)


def eval_point(ncp, deg, knots, P, uvw, with_abs=False):
    """One point of one block: (value, d/du, d/dv, d/dw) [and abs sums]."""
    out = np.empty(4, np.float64)
    ab = np.empty(4, np.float64)
    _load().orc_eval_point(_c(ncp, np.int32), _c(deg, np.int32), _c(knots, np.float64),
                           _c(P, np.float64).reshape(-1), _c(uvw, np.float64), out, ab)
    return (out, ab) if with_abs else out


def _nch(mask):
    return bin(int(mask) & 15).count("1")


def decode_blocks(b: Blocks, res, mask=15, nthreads=None):
    """Full grid decode: [nb, nch, Rx, Ry, Rz] float64."""
    res = _c(res, np.int32)
    out = np.empty((b.nblocks, _nch(mask), int(res[0]), int(res[1]), int(res[2])), np.float64)
    _load().orc_decode_blocks(b.nblocks, b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots,
                              b.ctrl, res, int(mask), out.reshape(-1),
                              nthreads or nthreads_default())
    return out


def decode_samples(b: Blocks, res, idx, with_abs=False, nthreads=None):
    """Selected voxels idx [m, 4] = (block, x, y, z) -> [m, 4] (all channels)."""
    idx = _c(idx, np.int32).reshape(-1, 4)
    m = idx.shape[0]
    out = np.empty((m, 4), np.float64)
    ab = np.empty((m, 4), np.float64) if with_abs else None
    _load().orc_decode_samples(m, idx.reshape(-1), b.ncp, b.deg, b.knot_off, b.ctrl_off,
                               b.knots, b.ctrl, _c(res, np.int32), out.reshape(-1),
                               ab.ctypes.data if with_abs else None,
                               nthreads or nthreads_default())
    return (out, ab) if with_abs else out


def eval_params(b: Blocks, blk, uvw, with_abs=False, nthreads=None):
    """Arbitrary parameters: block blk[m] at uvw[m, 3] -> [m, 4]."""
    blk = _c(blk, np.int32).reshape(-1)
    uvw = _c(uvw, np.float64).reshape(-1, 3)
    m = blk.shape[0]
    out = np.empty((m, 4), np.float64)
    ab = np.empty((m, 4), np.float64) if with_abs else None
    _load().orc_eval_params(m, blk, uvw.reshape(-1), b.ncp, b.deg, b.knot_off, b.ctrl_off,
                            b.knots, b.ctrl, out.reshape(-1),
                            ab.ctypes.data if with_abs else None,
                            nthreads or nthreads_default())
    return (out, ab) if with_abs else out


def query_points(b: Blocks, xyz, nb, origin, extent, block_of_cell, with_abs=False,
                 nthreads=None):
    """Point query over a domain tiled by nb[0] x nb[1] x nb[2] cells.

    xyz float32 [n, 3]; block_of_cell int32 [nb0*nb1*nb2] (-1 = empty cell).
    Returns [n, 4] float64 = (value, d/dx, d/dy, d/dz) in domain coordinates.
    """
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    n = xyz.shape[0]
    out = np.empty((n, 4), np.float64)
    ab = np.empty((n, 4), np.float64) if with_abs else None
    _load().orc_query_points(n, xyz.reshape(-1), _c(nb, np.int32), _c(origin, np.float32),
                             _c(extent, np.float32), _c(block_of_cell, np.int32).reshape(-1),
                             b.nblocks, b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots, b.ctrl,
                             out.reshape(-1), ab.ctypes.data if with_abs else None,
                             nthreads or nthreads_default())
    return (out, ab) if with_abs else out


def decode_adjoint(b: Blocks, res, g, mask=1, nthreads=None):
    """G = B^T g.  g: [nb, nch, Rx, Ry, Rz]; returns G in the lattice layout."""
    g = _c(g, np.float64).reshape(-1)
    G = np.zeros_like(b.ctrl)
    _load().orc_decode_adjoint(b.nblocks, b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots,
                               _c(res, np.int32), int(mask), g, G,
                               nthreads or nthreads_default())
    return G


def render(b: Blocks, rays, samples, opacity_max, tf_lo, tf_hi, tf, light, ka, kd, ks,
           shininess, nb, origin, extent, block_of_cell, grad_min=1e-6, nthreads=None):
    """Front-to-back ray casting (see orc_render).  rays: float32 [npix, 8]
    (origin, dir, t0, t1); tf: float32 [n, 4]; returns float64 [npix, 4]."""
    rays = _c(rays, np.float32).reshape(-1, 8)
    tf = _c(tf, np.float32).reshape(-1, 4)
    img = np.empty((rays.shape[0], 4), np.float64)
    _load().orc_render(rays.shape[0], rays.reshape(-1), int(samples), float(opacity_max),
                       float(tf_lo), float(tf_hi), tf.shape[0], _c(light, np.float32),
                       float(ka), float(kd), float(ks), float(shininess), float(grad_min),
                       tf.reshape(-1),
                       _c(nb, np.int32), _c(origin, np.float32), _c(extent, np.float32),
                       _c(block_of_cell, np.int32).reshape(-1), b.nblocks, b.ncp, b.deg,
                       b.knot_off, b.ctrl_off, b.knots, b.ctrl, img.reshape(-1),
                       nthreads or nthreads_default())
    return img
