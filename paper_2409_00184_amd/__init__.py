"""MI355X (gfx950) micro-model decode and query: thin Python binding.

Every computation runs in the HIP kernels of libfa.so (include/fa.h); this
module only marshals arguments: torch tensors provide device memory and the
current stream.  There is no CPU fallback: if libfa.so is missing, importing
the binding raises.

Entry points (same names as the C ABI):
  fa_validate_blocks, fa_plan_decode, fa_decode_blocks,
  fa_decode_blocks_plain, fa_query_points, fa_query_rays, fa_decode_backward,
  fa_quantize_blocks, fa_adam_step, fa_mse_loss
and the conveniences MicroModels, Plan, decode, decode_plain, query, query_rays,
decode_backward, FADecode (torch.autograd.Function), Adam, capture.
"""
import ctypes
import os

import numpy as np
import torch

__all__ = ["FA_F32", "FA_BF16", "FA_F16", "BLOCK_DTYPE", "WORK_DTYPE", "FAError", "lib",
           "MicroModels", "Plan", "decode", "decode_plain", "query", "query_rays",
           "decode_backward", "mse_loss",
           "FADecode", "capture", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# FA_LIBRARY selects another build of the same library (e.g. a tuning variant)
_LIB_PATH = os.environ.get("FA_LIBRARY") or os.path.join(_HERE, "libfa.so")

FA_OK, FA_ERR_INVALID_ARG, FA_ERR_UNSUPPORTED, FA_ERR_DEVICE = 0, 1, 2, 3
FA_F32, FA_BF16, FA_F16 = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 1 << 20  # FA_NOALLOC_SCRATCH_BYTES
DTYPES = {"f32": FA_F32, "bf16": FA_BF16, "f16": FA_F16}

BLOCK_DTYPE = np.dtype([("ncp", "<i4", (3,)), ("degree", "<i4", (3,)), ("knot_off", "<i8"),
                        ("ctrl_off", "<i8"), ("scale", "<f4"), ("flags", "<u4"),
                        ("reserved", "<i4", (4,))], align=True)
assert BLOCK_DTYPE.itemsize == 64
WORK_DTYPE = np.dtype([("block", "<i4"), ("row0", "<i2"), ("nrows", "<i2"), ("col0", "<i2"),
                       ("pad", "<i2")])
assert WORK_DTYPE.itemsize == 12


class FATune(ctypes.Structure):
    _fields_ = [("rows_per_item", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("slab_floats", ctypes.c_int32), ("store", ctypes.c_int32)]


class FARenderParams(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32), ("opacity_max", ctypes.c_float),
                ("tf_lo", ctypes.c_float), ("tf_hi", ctypes.c_float),
                ("tf_size", ctypes.c_int32), ("light", ctypes.c_float * 3),
                ("ka", ctypes.c_float), ("kd", ctypes.c_float), ("ks", ctypes.c_float),
                ("shininess", ctypes.c_float), ("grad_min", ctypes.c_float)]


class FAStoreStats(ctypes.Structure):
    _fields_ = [("hits", ctypes.c_int64), ("misses", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("bytes_read", ctypes.c_int64),
                ("bytes_h2d", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class FAError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        super().__init__(f"{call}: {lib.fa_status_string(status).decode()} (status {status})")


def library_path():
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()'); there is no CPU fallback")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.fa_status_string.restype = ctypes.c_char_p
    L.fa_status_string.argtypes = [ctypes.c_int]
    L.fa_version.restype = i32
    L.fa_validate_blocks.restype = ctypes.c_int
    L.fa_validate_blocks.argtypes = [vp, i32, vp, i64, i64]
    L.fa_plan_decode.restype = ctypes.c_int
    L.fa_plan_decode.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp, vp]
    L.fa_decode_blocks.restype = ctypes.c_int
    L.fa_decode_blocks.argtypes = [vp, i32, vp, vp, ctypes.c_int, vp, u32, vp, vp, vp, i32, vp,
                                   vp]
    L.fa_decode_blocks_plain.restype = ctypes.c_int
    L.fa_decode_blocks_plain.argtypes = [vp, i32, vp, vp, vp, u32, vp, vp]
    L.fa_query_points.restype = ctypes.c_int
    L.fa_query_points.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, i64, u32,
                                  vp, vp]
    L.fa_query_rays.restype = ctypes.c_int
    L.fa_query_rays.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, i32, i32, i32,
                                u32, vp, vp]
    L.fa_render_rays.restype = ctypes.c_int
    L.fa_render_rays.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, i32, i32,
                                 vp, vp, vp, vp]
    L.fa_adam_step.restype = ctypes.c_int
    L.fa_adam_step.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp]
    L.fa_mse_loss.restype = ctypes.c_int
    L.fa_mse_loss.argtypes = [vp, i32, ctypes.c_double, vp, vp]
    L.fa_mse_grad.restype = ctypes.c_int
    L.fa_mse_grad.argtypes = [vp, vp, i32, i64, ctypes.c_float, vp, vp, vp]
    L.fa_decode_residual_workspace.restype = i64
    L.fa_decode_residual_workspace.argtypes = [i32, vp, vp]
    L.fa_decode_residual.restype = ctypes.c_int
    L.fa_decode_residual.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp, ctypes.c_float,
                                     vp, vp, vp, i64, vp]
    L.fa_decode_residual_noalloc.restype = ctypes.c_int
    L.fa_decode_residual_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp,
                                             ctypes.c_float, vp, vp, vp]
    L.fa_fit_workspace.restype = i64
    L.fa_fit_workspace.argtypes = [i32, vp, i32]
    L.fa_fit_blocks.restype = ctypes.c_int
    L.fa_fit_blocks.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, i64, vp]
    L.fa_model_errors.restype = ctypes.c_int
    L.fa_model_errors.argtypes = [vp, i32, vp, vp, ctypes.c_int, vp, vp, vp, vp, i64, vp]
    L.fa_ncp_search_workspace.restype = i64
    L.fa_ncp_search_workspace.argtypes = [i32, vp, i32, i32]
    L.fa_ncp_search.restype = ctypes.c_int
    L.fa_ncp_search.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp, i64, vp]
    L.fa_ncp_select.restype = ctypes.c_int
    L.fa_ncp_select.argtypes = [vp, i32, i32, i32, i32, ctypes.c_float, vp, vp]
    L.fa_uniform_layout.restype = ctypes.c_int
    L.fa_uniform_layout.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp]
    L.fa_visible_cells.restype = ctypes.c_int
    L.fa_visible_cells.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.fa_store_write.restype = ctypes.c_int
    L.fa_store_write.argtypes = [ctypes.c_char_p, i32, vp, vp, vp]
    L.fa_store_open.restype = ctypes.c_int
    L.fa_store_open.argtypes = [ctypes.c_char_p, i32, u32, ctypes.POINTER(vp)]
    L.fa_store_close.restype = ctypes.c_int
    L.fa_store_close.argtypes = [vp]
    L.fa_store_info.restype = ctypes.c_int
    L.fa_store_info.argtypes = [vp, vp, vp, vp]
    L.fa_store_fetch.restype = ctypes.c_int
    L.fa_store_fetch.argtypes = [vp, vp, i32, vp, vp]
    L.fa_store_slot.restype = ctypes.c_int
    L.fa_store_slot.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_float)),
                                ctypes.POINTER(ctypes.POINTER(ctypes.c_float))]
    L.fa_store_stage.restype = ctypes.c_int
    L.fa_store_stage.argtypes = [vp, vp, i32, vp, vp, i64, vp, i64, vp, vp]
    L.fa_decode_backward.restype = ctypes.c_int
    L.fa_decode_backward.argtypes = [vp, i32, vp, vp, u32, vp, vp, vp]
    L.fa_search_set.restype = ctypes.c_int
    L.fa_search_set.argtypes = [i32, vp, vp, vp, vp]
    L.fa_level_select.restype = ctypes.c_int
    L.fa_level_select.argtypes = [i32, vp, i32, vp, i32, i32, i32, i32, ctypes.c_float, vp, vp]
    L.fa_quantize_blocks.restype = ctypes.c_int
    L.fa_quantize_blocks.argtypes = [vp, i32, vp, ctypes.c_int, vp, vp]
    return L


lib = _load()


def _check(call, st):
    if st != FA_OK:
        raise FAError(call, st)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _i32x3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def _f32x3(v):
    return (ctypes.c_float * 3)(*[float(x) for x in v])


def nch(mask):
    return bin(int(mask) & 15).count("1")


def host_descriptors(ncp, deg, knot_off, ctrl_off):
    d = np.zeros(len(ncp), BLOCK_DTYPE)
    d["ncp"] = np.asarray(ncp, np.int32).reshape(-1, 3)
    d["degree"] = np.asarray(deg, np.int32).reshape(-1, 3)
    d["knot_off"] = np.asarray(knot_off, np.int64)
    d["ctrl_off"] = np.asarray(ctrl_off, np.int64)
    d["scale"] = 1.0
    return d


def fa_validate_blocks(desc, knots, nctrl):
    """Host validation; sets desc['flags'] in place (C ABI fa_validate_blocks)."""
    knots = np.ascontiguousarray(knots, np.float32)
    st = lib.fa_validate_blocks(desc.ctypes.data, len(desc), knots.ctypes.data, knots.size,
                                int(nctrl))
    _check("fa_validate_blocks", st)
    return desc


class MicroModels:
    """A batch of micro-models resident on the GPU.

    Built from host arrays (ncp, degree, knot_off, ctrl_off, knots, ctrl);
    validated by fa_validate_blocks, then copied to the device.  Low-precision
    lattices are made on the device by fa_quantize_blocks (per-block max-abs
    scale written into the device descriptors `desc_lp`).
    """

    def __init__(self, ncp, deg, knot_off, ctrl_off, knots, ctrl, device="cuda"):
        ctrl = torch.as_tensor(ctrl, dtype=torch.float32)
        self.host_desc = fa_validate_blocks(host_descriptors(ncp, deg, knot_off, ctrl_off),
                                            knots, ctrl.numel())
        self.nblocks = len(self.host_desc)
        self.device = torch.device(device)
        self.desc = torch.from_numpy(self.host_desc.view(np.uint8).copy()).to(self.device)
        self.knots = torch.as_tensor(np.ascontiguousarray(knots, np.float32)).to(self.device)
        self.ctrl = ctrl.to(self.device).contiguous()
        self.ctrl_lp = {}
        self.desc_lp = {}

    @classmethod
    def from_batch(cls, b, device="cuda"):
        return cls(b.ncp, b.deg, b.knot_off, b.ctrl_off, b.knots, b.ctrl, device)

    def set_ctrl(self, ctrl):
        """Replace the FP32 lattice (same layout); drops low-precision copies."""
        assert ctrl.shape == self.ctrl.shape and ctrl.dtype == torch.float32
        self.ctrl = ctrl.contiguous()
        self.ctrl_lp.clear()
        self.desc_lp.clear()

    def lattice(self, dtype="f32", stream=None):
        """(device descriptors, lattice) for a storage dtype."""
        if dtype == "f32":
            return self.desc, self.ctrl
        if dtype not in self.ctrl_lp:
            desc = self.desc.clone()
            lp = torch.zeros(self.ctrl.numel(), dtype=torch.int16, device=self.device)
            st = lib.fa_quantize_blocks(_ptr(desc), self.nblocks, _ptr(self.ctrl), DTYPES[dtype],
                                        _ptr(lp), _stream(stream))
            _check("fa_quantize_blocks", st)
            self.desc_lp[dtype], self.ctrl_lp[dtype] = desc, lp
        return self.desc_lp[dtype], self.ctrl_lp[dtype]


class Plan:
    """Host batch plan (fa_plan_decode) copied to the device."""

    def __init__(self, models, res, rows=0, waves=0, grid=0, kernel=0, slab=0, store=0):
        self.tune = FATune(int(rows), int(waves), int(grid), int(kernel), int(slab), int(store))
        cap = models.nblocks * ((int(res[1]) + 0) * ((int(res[2]) + 63) // 64))
        work = np.zeros(cap, WORK_DTYPE)
        off = np.zeros(cap + 1, np.int32)
        nwork = ctypes.c_int64(0)
        ngroups = ctypes.c_int32(0)
        st = lib.fa_plan_decode(models.host_desc.ctypes.data, models.nblocks, _i32x3(res),
                                ctypes.byref(self.tune), work.ctypes.data, off.ctypes.data,
                                cap, ctypes.byref(nwork), ctypes.byref(ngroups))
        _check("fa_plan_decode", st)
        self.nwork, self.ngroups = nwork.value, ngroups.value
        self.host_work = work[:self.nwork].copy()
        self.host_off = off[:self.ngroups + 1].copy()
        self.work = torch.from_numpy(self.host_work.view(np.uint8).copy()).to(models.device)
        self.wg_off = torch.from_numpy(self.host_off).to(models.device)
        self.res = tuple(int(r) for r in res)


OUT_INTERLEAVED = 0x100  # FA_OUT_INTERLEAVED: one (value, d/du, d/dv, d/dw) record per voxel


def decode(models, res, mask=15, dtype="f32", plan=None, tune=None, out=None, stream=None):
    """Batched grid decode (fa_decode_blocks) -> [nb, nch, R0, R1, R2] float32,
    or [nb, R0, R1, R2, 4] with mask = 15 | OUT_INTERLEAVED."""
    desc, ctrl = models.lattice(dtype, stream)
    if out is None:
        r = tuple(int(v) for v in res)
        shape = ((models.nblocks,) + r + (4,) if mask & OUT_INTERLEAVED
                 else (models.nblocks, nch(mask)) + r)
        out = torch.empty(shape, dtype=torch.float32, device=models.device)
    if plan is not None:
        assert plan.res == tuple(int(r) for r in res)
        t, work, off, ng = plan.tune, _ptr(plan.work), _ptr(plan.wg_off), plan.ngroups
    else:
        t = tune if tune is not None else FATune(0, 0, 0, 0, 0, 0)
        work, off, ng = None, None, 0
    st = lib.fa_decode_blocks(_ptr(desc), models.nblocks, _ptr(models.knots), _ptr(ctrl),
                              DTYPES[dtype], _i32x3(res), int(mask), ctypes.byref(t), work, off,
                              ng, _ptr(out), _stream(stream))
    _check("fa_decode_blocks", st)
    return out


def decode_plain(models, res, mask=15, out=None, stream=None):
    """Plain per-voxel decode, one launch per block (fa_decode_blocks_plain)."""
    if out is None:
        out = torch.empty((models.nblocks, nch(mask)) + tuple(int(r) for r in res),
                          dtype=torch.float32, device=models.device)
    st = lib.fa_decode_blocks_plain(_ptr(models.desc), models.nblocks, _ptr(models.knots),
                                    _ptr(models.ctrl), _i32x3(res), int(mask), _ptr(out),
                                    _stream(stream))
    _check("fa_decode_blocks_plain", st)
    return out


def query(models, xyz, nb, origin, extent, block_of_cell, mask=15, dtype="f32", out=None,
          stream=None):
    """Point query (fa_query_points): xyz [n, 3] float32 -> [n, 4] float32."""
    desc, ctrl = models.lattice(dtype, stream)
    assert xyz.dtype == torch.float32 and xyz.is_contiguous() and xyz.shape[-1] == 3
    n = xyz.numel() // 3
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=models.device)
    st = lib.fa_query_points(_ptr(desc), models.nblocks, _ptr(block_of_cell), _i32x3(nb),
                             _f32x3(origin), _f32x3(extent), _ptr(models.knots), _ptr(ctrl),
                             DTYPES[dtype], _ptr(xyz), n, int(mask), _ptr(out),
                             _stream(stream))
    _check("fa_query_points", st)
    return out


def query_rays(models, xyz, width, height, samples, nb, origin, extent, block_of_cell,
               mask=15, dtype="f32", out=None, stream=None):
    """Ray-structured query (fa_query_rays): xyz [height*width*samples, 3]
    ray-major -> [height*width*samples, 4]; same values as query()."""
    desc, ctrl = models.lattice(dtype, stream)
    n = int(width) * int(height) * int(samples)
    assert xyz.dtype == torch.float32 and xyz.is_contiguous() and xyz.numel() == 3 * n
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=models.device)
    st = lib.fa_query_rays(_ptr(desc), models.nblocks, _ptr(block_of_cell), _i32x3(nb),
                           _f32x3(origin), _f32x3(extent), _ptr(models.knots), _ptr(ctrl),
                           DTYPES[dtype], _ptr(xyz), int(width), int(height), int(samples),
                           int(mask), _ptr(out), _stream(stream))
    _check("fa_query_rays", st)
    return out


def render(models, rays, width, height, tf, nb, origin, extent, block_of_cell, samples,
           opacity_max=0.98, tf_range=(0.0, 1.0), light=(0.0, 0.0, 1.0), ka=0.3, kd=0.6,
           ks=0.3, shininess=32.0, grad_min=1e-6, dtype="f32", out=None, stream=None):
    """Direct volume rendering (fa_render_rays): rays [height*width, 8] float32
    (origin, direction, t0, t1), tf [n, 4] float32 RGBA -> image
    [height, width, 4] float32 (composited RGB, accumulated opacity)."""
    desc, ctrl = models.lattice(dtype, stream)
    n = int(width) * int(height)
    assert rays.dtype == torch.float32 and rays.is_contiguous() and rays.numel() == 8 * n
    assert tf.dtype == torch.float32 and tf.is_contiguous() and tf.shape[-1] == 4
    if out is None:
        out = torch.empty((int(height), int(width), 4), dtype=torch.float32,
                          device=models.device)
    p = FARenderParams(int(samples), float(opacity_max), float(tf_range[0]), float(tf_range[1]),
                       int(tf.shape[0]), (ctypes.c_float * 3)(*[float(v) for v in light]),
                       float(ka), float(kd), float(ks), float(shininess), float(grad_min))
    st = lib.fa_render_rays(_ptr(desc), models.nblocks, _ptr(block_of_cell), _i32x3(nb),
                            _f32x3(origin), _f32x3(extent), _ptr(models.knots), _ptr(ctrl),
                            DTYPES[dtype], _ptr(rays), int(width), int(height),
                            ctypes.byref(p), _ptr(tf), _ptr(out), _stream(stream))
    _check("fa_render_rays", st)
    return out


def decode_backward(models, res, grad_out, mask=1, grad_ctrl=None, stream=None):
    """Adjoint B^T g (fa_decode_backward) -> lattice-layout float32."""
    assert grad_out.dtype == torch.float32 and grad_out.is_contiguous()
    if grad_ctrl is None:
        grad_ctrl = torch.zeros_like(models.ctrl)
    st = lib.fa_decode_backward(_ptr(models.desc), models.nblocks, _ptr(models.knots),
                                _i32x3(res), int(mask), _ptr(grad_out), _ptr(grad_ctrl),
                                _stream(stream))
    _check("fa_decode_backward", st)
    return grad_ctrl


class Adam(torch.optim.Optimizer):
    """Adam on FP32 CUDA parameters, one fa_adam_step per parameter tensor
    (two HIP launches: the device step counter, then the update).  Same
    update as torch.optim.Adam (no amsgrad, weight decay added to the
    gradient); the step count is kept on the device, so the step can be
    captured into a HIP graph (capture_fit_step) once one eager step has
    created the state."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0):
        super().__init__(params, dict(lr=lr, betas=betas, eps=eps, weight_decay=weight_decay))

    @torch.no_grad()
    def step(self, closure=None):
        loss = None
        if closure is not None:
            with torch.enable_grad():
                loss = closure()
        for group in self.param_groups:
            b1, b2 = group["betas"]
            for p in group["params"]:
                if p.grad is None:
                    continue
                assert p.dtype == torch.float32 and p.is_cuda and p.is_contiguous()
                g = p.grad if p.grad.is_contiguous() else p.grad.contiguous()
                st = self.state[p]
                if not st:
                    st["exp_avg"] = torch.zeros_like(p)
                    st["exp_avg_sq"] = torch.zeros_like(p)
                    st["state"] = torch.zeros(3, dtype=torch.float32, device=p.device)
                _check("fa_adam_step", lib.fa_adam_step(
                    _ptr(p), _ptr(g), _ptr(st["exp_avg"]), _ptr(st["exp_avg_sq"]), p.numel(),
                    float(group["lr"]), float(b1), float(b2), float(group["eps"]),
                    float(group["weight_decay"]), _ptr(st["state"]), _stream()))
        return loss


# ------------------------------------------------------- adaptive encoding

def uniform_models(ncp, degree, device="cuda"):
    """MicroModels with clamped uniform knots for per-block ncp [nb, 3] and
    degree [nb] or [nb, 3] (fa_uniform_layout); lattices zero."""
    ncp = np.ascontiguousarray(np.asarray(ncp, np.int32).reshape(-1, 3))
    nb = ncp.shape[0]
    deg = np.asarray(degree, np.int32)
    deg = np.ascontiguousarray(np.broadcast_to(deg.reshape(-1, 1) if deg.ndim == 1 else deg,
                                               (nb, 3)), np.int32)
    desc = np.zeros(nb, BLOCK_DTYPE)
    nk, nc = ctypes.c_int64(0), ctypes.c_int64(0)
    _check("fa_uniform_layout", lib.fa_uniform_layout(nb, ncp.ctypes.data, deg.ctypes.data,
                                                      None, None, 0, ctypes.byref(nk),
                                                      ctypes.byref(nc)))
    knots = np.zeros(nk.value, np.float32)
    _check("fa_uniform_layout", lib.fa_uniform_layout(nb, ncp.ctypes.data, deg.ctypes.data,
                                                      desc.ctypes.data, knots.ctypes.data,
                                                      knots.size, ctypes.byref(nk),
                                                      ctypes.byref(nc)))
    return MicroModels(desc["ncp"], desc["degree"], desc["knot_off"], desc["ctrl_off"], knots,
                       np.zeros(nc.value, np.float32), device)


def fit(models, res, samples, workspace=None, stream=None):
    """Least-squares lattices (fa_fit_blocks) of samples [nb, *res] float32;
    overwrites models.ctrl (and drops low-precision copies)."""
    assert samples.dtype == torch.float32 and samples.is_contiguous()
    assert samples.numel() == models.nblocks * int(np.prod(res))
    max_n = int(models.host_desc["ncp"][:, 2].max())
    need = lib.fa_fit_workspace(models.nblocks, _i32x3(res), max_n)
    if need < 0:
        raise FAError("fa_fit_workspace", FA_ERR_INVALID_ARG)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=models.device)
    st = lib.fa_fit_blocks(_ptr(models.desc), models.nblocks, _ptr(models.knots), _i32x3(res),
                           _ptr(samples), _ptr(models.ctrl), max_n, _ptr(workspace),
                           workspace.numel(), _stream(stream))
    _check("fa_fit_blocks", st)
    models.set_ctrl(models.ctrl)
    return models


def model_errors(models, res, samples, dtype="f32", decoded=None, stream=None):
    """Per-block (max |y - f|, rms(y - f)) of the decoded models (fa_model_errors)."""
    desc, ctrl = models.lattice(dtype, stream)
    assert samples.dtype == torch.float32 and samples.is_contiguous()
    if decoded is None:
        decoded = torch.empty_like(samples)
    errs = torch.empty((models.nblocks, 2), dtype=torch.float32, device=models.device)
    st = lib.fa_model_errors(_ptr(desc), models.nblocks, _ptr(models.knots), _ptr(ctrl),
                             DTYPES[dtype], _i32x3(res), _ptr(samples), _ptr(decoded),
                             _ptr(errs), 2, _stream(stream))
    _check("fa_model_errors", st)
    return errs


def ncp_search(samples, degree, ncp_lo=None, ncp_hi=None, workspace=None, stream=None):
    """Error maps [nb, ncand, 2] (max, rms) of model(n, degree) for n =
    ncp_lo..ncp_hi (fa_ncp_search); samples [nb, R0, R1, R2] float32."""
    assert samples.dtype == torch.float32 and samples.is_contiguous() and samples.dim() == 4
    nb, res = samples.shape[0], tuple(int(r) for r in samples.shape[1:])
    lo = degree + 2 if ncp_lo is None else int(ncp_lo)
    hi = min(res) if ncp_hi is None else int(ncp_hi)
    need = lib.fa_ncp_search_workspace(nb, _i32x3(res), int(degree), hi)
    if need < 0:
        raise FAError("fa_ncp_search_workspace", FA_ERR_INVALID_ARG)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=samples.device)
    errs = torch.empty((nb, hi - lo + 1, 2), dtype=torch.float32, device=samples.device)
    st = lib.fa_ncp_search(_ptr(samples), nb, _i32x3(res), int(degree), lo, hi, _ptr(errs),
                           _ptr(workspace), workspace.numel(), _stream(stream))
    _check("fa_ncp_search", st)
    return errs


METRIC_MAX, METRIC_RMS = 0, 1


def ncp_select(errs, ncp_lo, bound, metric=METRIC_RMS):
    """(NCP* [nb], complex [nb]) of Eq. 4 from error maps (fa_ncp_select)."""
    e = np.ascontiguousarray(errs.cpu().numpy() if torch.is_tensor(errs) else errs, np.float32)
    nb, ncand = e.shape[0], e.shape[1]
    nstar = np.zeros(nb, np.int32)
    cplx = np.zeros(nb, np.int32)
    st = lib.fa_ncp_select(e.ctypes.data, nb, ncand, int(ncp_lo), int(metric), float(bound),
                           nstar.ctypes.data, cplx.ctypes.data)
    _check("fa_ncp_select", st)
    return nstar, cplx.astype(bool)


def search_set(level, parent_complex=None):
    """(searched [(2^k)^3] bool, search_ids) of Alg. 1's cross-level step
    (fa_search_set): every block of level 0, and at a finer level the blocks
    whose parent is complex."""
    nb = 1 << (3 * int(level))
    pc = (None if parent_complex is None else
          np.ascontiguousarray(np.asarray(parent_complex).astype(np.int32)))
    searched = np.zeros(nb, np.int32)
    ids = np.zeros(nb, np.int32)
    n = ctypes.c_int32(0)
    st = lib.fa_search_set(int(level), None if pc is None else pc.ctypes.data,
                           searched.ctypes.data, ids.ctypes.data, ctypes.byref(n))
    _check("fa_search_set", st)
    return searched.astype(bool), ids[:n.value].copy()


def level_select(nblocks, search_ids, errs, ncp_lo, degree, bound, metric=METRIC_RMS):
    """(NCP* [nb], complex [nb]) of one pyramid level (fa_level_select) from
    the error maps of its searched blocks."""
    ids = np.ascontiguousarray(np.asarray(search_ids, np.int32))
    e = (None if errs is None else
         np.ascontiguousarray(errs.cpu().numpy() if torch.is_tensor(errs) else errs, np.float32))
    ncand = int(e.shape[1]) if e is not None and e.size else 1
    nstar = np.zeros(int(nblocks), np.int32)
    cplx = np.zeros(int(nblocks), np.int32)
    st = lib.fa_level_select(int(nblocks), ids.ctypes.data if ids.size else None, int(ids.size),
                             e.ctypes.data if e is not None and e.size else None, ncand,
                             int(ncp_lo), int(degree), int(metric), float(bound),
                             nstar.ctypes.data, cplx.ctypes.data)
    _check("fa_level_select", st)
    return nstar, cplx.astype(bool)


def adaptive_encode(levels, degree, bound, metric=METRIC_RMS, ncp_lo=None, ncp_hi=None):
    """Cross-level adaptive encoding (Alg. 1) over a pyramid of micro-blocks.

    levels[k]: samples [(2^k)^3, R, R, R] float32 on the GPU, level 0 the
    coarsest, block (bx, by, bz) of level k at (bx * 2^k + by) * 2^k + bz.
    Per level: fa_search_set names the blocks to search, fa_ncp_search
    builds their error maps, fa_level_select sets NCP* and the complex set,
    and every block is fitted at its NCP* (fa_fit_blocks).  Returns, per
    level, a dict with ncp_star, complex, searched (numpy) and the fitted
    MicroModels."""
    out = []
    prev = None
    for k, Y in enumerate(levels):
        nb, R = Y.shape[0], int(Y.shape[1])
        lo = degree + 2 if ncp_lo is None else int(ncp_lo)
        hi = R if ncp_hi is None else int(ncp_hi)
        searched, ids = search_set(k, prev)
        assert searched.size == nb, "level k holds (2^k)^3 blocks"
        errs = None
        if ids.size:
            sub = Y[torch.as_tensor(ids, device=Y.device).long()].contiguous()
            errs = ncp_search(sub, degree, lo, hi)
        nstar, cplx = level_select(nb, ids, errs, lo, degree, bound, metric)
        models = uniform_models(np.repeat(nstar[:, None], 3, 1), np.full(nb, degree))
        fit(models, Y.shape[1:], Y.contiguous())
        out.append(dict(ncp_star=nstar, complex=cplx, searched=searched, models=models))
        prev = cplx
    return out


# ------------------------------------------------- storage, cache, staging

FA_STORE_PINNED = 1


def visible_cells(rays, width, height, samples, nb, origin, extent, out=None, stream=None):
    """int32 flags [ncells]: cells some sample of render() looks up (fa_visible_cells)."""
    assert rays.dtype == torch.float32 and rays.is_contiguous()
    assert rays.numel() == 8 * int(width) * int(height)
    if out is None:
        out = torch.empty(int(np.prod(nb)), dtype=torch.int32, device=rays.device)
    st = lib.fa_visible_cells(_ptr(rays), int(width), int(height), int(samples), _i32x3(nb),
                              _f32x3(origin), _f32x3(extent), _ptr(out), _stream(stream))
    _check("fa_visible_cells", st)
    return out


def store_write(path, host_desc, knots, ctrl):
    """Write micro-models (host descriptors, FP32 knots and lattices) to a
    file in the Eq. 2 record format (fa_store_write)."""
    knots = np.ascontiguousarray(knots, np.float32)
    ctrl = np.ascontiguousarray(ctrl, np.float32)
    desc = np.ascontiguousarray(host_desc)
    st = lib.fa_store_write(os.fsencode(path), len(desc), desc.ctypes.data, knots.ctypes.data,
                            ctrl.ctypes.data)
    _check("fa_store_write", st)


class StagedModels:
    """A device batch filled by Store.stage(): the same interface as
    MicroModels for decode/query/render (FP32 lattices)."""

    def __init__(self, desc, knots, ctrl, nblocks, device):
        self.desc, self.knots, self.ctrl = desc, knots, ctrl
        self.nblocks, self.device = nblocks, device

    def lattice(self, dtype="f32", stream=None):
        if dtype != "f32":
            raise ValueError("staged micro-models are FP32")
        return self.desc, self.ctrl


class Store:
    """An open micro-model file with a host LRU cache (fa_store_*)."""

    def __init__(self, path, cache_blocks=200, pinned=True, max_stage=None, device="cuda"):
        h = ctypes.c_void_p()
        st = lib.fa_store_open(os.fsencode(path), int(cache_blocks),
                               FA_STORE_PINNED if pinned else 0, ctypes.byref(h))
        _check("fa_store_open", st)
        self.h = h
        n = ctypes.c_int32(0)
        _check("fa_store_info", lib.fa_store_info(h, ctypes.byref(n), None, None))
        self.nblocks = n.value
        self.ncp = np.zeros(self.nblocks, np.int32)
        self.degree = np.zeros(self.nblocks, np.int32)
        _check("fa_store_info", lib.fa_store_info(h, None, self.ncp.ctypes.data,
                                                  self.degree.ctypes.data))
        self.device = torch.device(device)
        self.max_stage = self.nblocks if max_stage is None else int(max_stage)
        self._arena = None

    def close(self):
        if self.h:
            _check("fa_store_close", lib.fa_store_close(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fetch(self, ids):
        """Caching step on the host: (slots [n], stats dict)."""
        ids = np.ascontiguousarray(ids, np.int32)
        slots = np.zeros(ids.size, np.int32)
        stats = FAStoreStats()
        st = lib.fa_store_fetch(self.h, ids.ctypes.data, ids.size, slots.ctypes.data,
                                ctypes.byref(stats))
        _check("fa_store_fetch", st)
        return slots, stats.as_dict()

    def slot(self, slot):
        """(block, knots [3 vectors], lattice [n, n, n]) copies of one slot."""
        b = ctypes.c_int32(0)
        kp = ctypes.POINTER(ctypes.c_float)()
        cp = ctypes.POINTER(ctypes.c_float)()
        _check("fa_store_slot", lib.fa_store_slot(self.h, int(slot), ctypes.byref(b),
                                                  ctypes.byref(kp), ctypes.byref(cp)))
        n, p = int(self.ncp[b.value]), int(self.degree[b.value])
        kn = np.ctypeslib.as_array(kp, shape=(3 * (n + p + 1),)).copy()
        P = np.ctypeslib.as_array(cp, shape=(n * n * n,)).copy().reshape(n, n, n)
        return b.value, kn.reshape(3, n + p + 1), P

    def _arena_for(self):
        if self._arena is None:
            order = np.sort(self.ncp.astype(np.int64) ** 3)[::-1][:self.max_stage]
            kcap = int(np.sort(3 * (self.ncp + self.degree + 1))[::-1][:self.max_stage].sum())
            ccap = int(((order + 63) // 64 * 64).sum())
            self._arena = (
                torch.zeros(self.max_stage * BLOCK_DTYPE.itemsize, dtype=torch.uint8,
                            device=self.device),
                torch.zeros(max(kcap, 1), dtype=torch.float32, device=self.device),
                torch.zeros(max(ccap, 64), dtype=torch.float32, device=self.device))
        return self._arena

    def stage(self, ids, stream=None):
        """Caching + copy to the GPU (fa_store_stage) -> (StagedModels, stats)."""
        ids = np.ascontiguousarray(ids, np.int32)
        assert 0 < ids.size <= self.max_stage
        d, k, c = self._arena_for()
        stats = FAStoreStats()
        st = lib.fa_store_stage(self.h, ids.ctypes.data, ids.size, _ptr(d), _ptr(k), k.numel(),
                                _ptr(c), c.numel(), ctypes.byref(stats), _stream(stream))
        _check("fa_store_stage", st)
        return StagedModels(d, k, c, int(ids.size), self.device), stats.as_dict()


class FADecode(torch.autograd.Function):
    """value (and gradient channels) = B(ctrl); backward = B^T (HIP adjoint)."""

    @staticmethod
    def forward(ctx, ctrl, models, res, mask, plan):
        models.set_ctrl(ctrl.detach())
        out = decode(models, res, mask, plan=plan)
        ctx.models, ctx.res, ctx.mask = models, res, mask
        return out

    @staticmethod
    def backward(ctx, g):
        gc = decode_backward(ctx.models, ctx.res, g.contiguous(), ctx.mask)
        return gc, None, None, None, None


def decode_residual(models, res, samples, grad_scale, plan=None, tune=None, grad=None,
                    sumsq=None, workspace=None, stream=None):
    """Value decode fused with the fit's residual (fa_decode_residual):
    returns (grad, sumsq) with grad = grad_scale (f - samples) [nb, *res]
    and sumsq[b] = sum (f - samples)^2 (FP64), f never stored."""
    res3 = _i32x3(res)
    if plan is not None:
        assert plan.res == tuple(int(r) for r in res)
        t, work, off, ng = plan.tune, _ptr(plan.work), _ptr(plan.wg_off), plan.ngroups
    else:
        t = tune if tune is not None else FATune(0, 0, 0, 0, 0, 0)
        work, off, ng = None, None, 0
    need = lib.fa_decode_residual_workspace(models.nblocks, res3, ctypes.byref(t))
    if need < 0:
        raise FAError("fa_decode_residual_workspace", 1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(int(need), 8), dtype=torch.uint8, device=models.device)
    if grad is None:
        grad = torch.empty((models.nblocks,) + tuple(int(r) for r in res), dtype=torch.float32,
                           device=models.device)
    if sumsq is None:
        sumsq = torch.empty(models.nblocks, dtype=torch.float64, device=models.device)
    assert samples.dtype == torch.float32 and samples.is_contiguous()
    st = lib.fa_decode_residual(_ptr(models.desc), models.nblocks, _ptr(models.knots),
                                _ptr(models.ctrl), res3, ctypes.byref(t), work, off, ng,
                                _ptr(samples), float(grad_scale), _ptr(grad), _ptr(sumsq),
                                _ptr(workspace), int(workspace.numel()), _stream(stream))
    _check("fa_decode_residual", st)
    return grad, sumsq


def decode_residual_noalloc(models, res, samples, grad_scale, plan=None, tune=None, grad=None,
                            sumsq=None, stream=None):
    """decode_residual through fa_decode_residual_noalloc: the partial sums
    live in the library's fixed device array, so the call itself allocates
    nothing (pass grad and sumsq to keep this wrapper from allocating them).
    Calls that overlap on one GPU race on that array."""
    res3 = _i32x3(res)
    if plan is not None:
        assert plan.res == tuple(int(r) for r in res)
        t, work, off, ng = plan.tune, _ptr(plan.work), _ptr(plan.wg_off), plan.ngroups
    else:
        t = tune if tune is not None else FATune(0, 0, 0, 0, 0, 0)
        work, off, ng = None, None, 0
    if grad is None:
        grad = torch.empty((models.nblocks,) + tuple(int(r) for r in res), dtype=torch.float32,
                           device=models.device)
    if sumsq is None:
        sumsq = torch.empty(models.nblocks, dtype=torch.float64, device=models.device)
    assert samples.dtype == torch.float32 and samples.is_contiguous()
    st = lib.fa_decode_residual_noalloc(_ptr(models.desc), models.nblocks, _ptr(models.knots),
                                        _ptr(models.ctrl), res3, ctypes.byref(t), work, off, ng,
                                        _ptr(samples), float(grad_scale), _ptr(grad),
                                        _ptr(sumsq), _stream(stream))
    _check("fa_decode_residual_noalloc", st)
    return grad, sumsq


def mse_loss(sumsq, count, loss=None, stream=None):
    """(float32 scalar) sum(sumsq) / count in one launch (fa_mse_loss)."""
    assert sumsq.dtype == torch.float64 and sumsq.is_contiguous()
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=sumsq.device)
    _check("fa_mse_loss", lib.fa_mse_loss(_ptr(sumsq), sumsq.numel(), float(count), _ptr(loss),
                                          _stream(stream)))
    return loss


class FAFitMSE(torch.autograd.Function):
    """Loss = mean over all voxels of (B(ctrl) - y)^2 in two HIP passes: the
    value decode fused with the residual, loss and cotangent
    (fa_decode_residual; the decoded values are never stored) and the loss
    from its per-block sums (fa_mse_loss), and in backward the adjoint B^T of
    the cotangent.  y: [nblocks, *res] float32.  The adjoint writes into a
    buffer kept on `models` (zeroed once: the padding between blocks'
    lattices, which the adjoint leaves alone, stays zero); the gradient
    returned is a new tensor, its product with the incoming gradient, so
    only backward passes on one `models` that overlap on different streams
    would share the buffer (run them on one stream)."""

    @staticmethod
    def forward(ctx, ctrl, models, res, y, plan):
        models.set_ctrl(ctrl.detach())
        nvox = int(np.prod(res))
        m_all = models.nblocks * nvox
        g, sumsq = decode_residual(models, res, y, 2.0 / m_all, plan=plan)
        ctx.models, ctx.res = models, res
        ctx.save_for_backward(g)  # the cotangent 2 (f - y) / M
        return mse_loss(sumsq, m_all)

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        m = ctx.models
        buf = getattr(m, "_adjoint_buf", None)
        if buf is None or buf.numel() != m.ctrl.numel() or buf.device != m.ctrl.device:
            buf = torch.zeros_like(m.ctrl)
            m._adjoint_buf = buf
        gc = decode_backward(m, ctx.res, g, 1, grad_ctrl=buf)
        return gc * gl, None, None, None, None


def capture_fit_step(ctrl, opt, models, res, y, plan=None, warmup=3):
    """One fit iteration -- FAFitMSE forward (value decode and fused
    residual/loss/cotangent), the adjoint in backward, opt.step() --
    captured into a HIP graph, so that a fit loop is one graph launch per
    iteration.  The gradient is set by the adjoint (it writes every control
    point), not accumulated into a zeroed buffer: inside the capture it is a
    tensor of the graph's pool that every replay rewrites.  `opt` must be
    capturable (e.g. Adam(..., capturable=True), or fused=True for one
    update kernel); `warmup` eager iterations run first on a side stream
    (they are real steps of the fit).  Returns (graph, loss): every replay
    performs one more iteration and overwrites the static `loss` tensor."""
    def step():
        opt.zero_grad(set_to_none=True)
        loss = FAFitMSE.apply(ctrl, models, res, y, plan)
        loss.backward()
        opt.step()
        return loss

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(1, warmup)):
            step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        loss = step()
    return g, loss


def capture(fn, warmup=1):
    """Capture fn() (HIP calls on the current stream) into a graph; returns
    (graph, result of the captured call)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warmup):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = fn()
    return g, res
