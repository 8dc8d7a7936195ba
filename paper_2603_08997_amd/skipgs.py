"""Python binding of libskipgs.so (the C ABI in include/skipgs.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library. torch is used for device memory and the current
stream. Importing this module loads the library and raises if it is missing
or was not built for this package; there is no fallback.

The functions keep the C names without the ``sgs_`` prefix.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libskipgs.so")

SGS_OK = 0
STATUS_PAIR_OVERFLOW = 0x1
STATUS_NONFINITE_LOSS = 0x2
STATUS_BAD_VIEW = 0x4
MAX_VIEWS = 16
MAX_PLANES = 59


class SkipGSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"skipgs status {status}: {msg}")
        self.status = status


class GaussiansC(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("data", C.c_void_p), ("n", C.c_int64), ("stride", C.c_int64),
                ("sh_degree", C.c_int32)]


class CameraC(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class RasterParamsC(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("super_tile", C.c_int32), ("lds_batch", C.c_int32),
                ("split_prefix", C.c_int32), ("bg", C.c_float * 3),
                ("near_z", C.c_float), ("dilation", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("jac_clamp", C.c_float)]


class WorkspaceLayoutC(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in ("records", "tiles", "depth", "sup_key", "sup_entry",
                                            "sup_ranges", "tile_entry", "tile_ranges",
                                            "t_final", "n_last", "accum", "counters")] + \
               [(k, C.c_int64) for k in ("entries", "total_tiles", "total_pixels",
                                         "total_supers")] + \
               [("key_bits", C.c_int32), ("rect_bits", C.c_int32), ("batch", C.c_int32),
                ("super_tile", C.c_int32)]


class GateParamsC(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("beta", C.c_double), ("eps", C.c_double), ("delta", C.c_double),
                ("rho_lo", C.c_double), ("warmup", C.c_int32), ("window", C.c_int32),
                ("calibrate", C.c_int32), ("budget", C.c_int32), ("n_views", C.c_int32)]


class GateSnapshotC(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("t", "b", "t_w", "b_w", "warm_hits", "warm_count")] + \
               [(k, C.c_double) for k in ("rho_min", "last_s", "last_rho")] + \
               [(k, C.c_int32) for k in ("calibrated", "flags", "last_g", "last_proposed",
                                         "last_forced", "last_view")]


class DensifyParamsC(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("grad_threshold", C.c_float),
                ("percent_dense", C.c_float), ("scene_extent", C.c_float),
                ("min_opacity", C.c_float), ("split_scale", C.c_float)]


class AdamParamsC(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("lr", C.c_float * MAX_PLANES), ("visible_only", C.c_int32)]


EXPORTS = [
    "sgs_last_error", "sgs_version", "sgs_default_raster_params", "sgs_forward_workspace_size",
    "sgs_render_forward", "sgs_read_status", "sgs_clear_status", "sgs_render_backward",
    "sgs_project", "sgs_load_records", "sgs_bin", "sgs_rasterize", "sgs_rasterize_backward",
    "sgs_project_backward", "sgs_get_workspace_layout", "sgs_loss_workspace_size",
    "sgs_photometric_loss", "sgs_photometric_loss_backward", "sgs_photometric_loss_static",
    "sgs_gate_state_size",
    "sgs_gate_init", "sgs_gate_update", "sgs_gate_read", "sgs_adam_step",
    "sgs_project_backward_adam", "sgs_render_backward_adam", "sgs_camera_table_size",
    "sgs_camera_table_init", "sgs_view_sequence_next", "sgs_train_iteration",
    "sgs_default_densify_params", "sgs_densify_stats", "sgs_densify_workspace_size",
    "sgs_densify",
]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2603_08997_amd.build`")
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    sig = {
        "sgs_last_error": (C.c_char_p, []),
        "sgs_version": (i32, []),
        "sgs_default_raster_params": (None, [P(RasterParamsC)]),
        "sgs_forward_workspace_size": (i32, [P(RasterParamsC), i64, P(CameraC), i32, i64, P(sz)]),
        "sgs_render_forward": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp, sz, i64,
                                     vp, vp]),
        "sgs_read_status": (i32, [vp, P(C.c_uint32), P(i64), P(i64), vp]),
        "sgs_clear_status": (i32, [vp, vp]),
        "sgs_render_backward": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp, sz, i64,
                                      vp, vp, vp, vp]),
        "sgs_project": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp, sz, i64, vp]),
        "sgs_load_records": (i32, [P(CameraC), i32, i64, P(RasterParamsC), vp, sz, i64, vp, vp, vp,
                                   vp, vp, vp, vp, vp]),
        "sgs_bin": (i32, [P(CameraC), i32, i64, P(RasterParamsC), vp, sz, i64, vp]),
        "sgs_rasterize": (i32, [P(CameraC), i32, i64, P(RasterParamsC), vp, sz, i64, vp, vp]),
        "sgs_rasterize_backward": (i32, [P(CameraC), i32, i64, P(RasterParamsC), vp, sz, i64, vp, vp,
                                         vp]),
        "sgs_project_backward": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp, sz, i64,
                                       vp, vp, vp]),
        "sgs_get_workspace_layout": (i32, [P(RasterParamsC), i64, P(CameraC), i32, i64,
                                           P(WorkspaceLayoutC)]),
        "sgs_loss_workspace_size": (i32, [i32, i32, P(sz)]),
        "sgs_photometric_loss": (i32, [vp, vp, i32, i32, f32, vp, sz, vp, vp]),
        "sgs_photometric_loss_static": (i32, [vp, vp, i32, i32, f32, vp, vp]),
        "sgs_photometric_loss_backward": (i32, [vp, vp, i32, i32, f32, vp, sz, vp, vp, vp]),
        "sgs_gate_state_size": (i32, [P(GateParamsC), P(sz)]),
        "sgs_gate_init": (i32, [P(GateParamsC), vp, vp]),
        "sgs_gate_update": (i32, [P(GateParamsC), vp, vp, vp, vp, vp]),
        "sgs_gate_read": (i32, [P(GateParamsC), vp, P(GateSnapshotC), vp, vp, vp]),
        "sgs_adam_step": (i32, [P(AdamParamsC), vp, vp, vp, vp, i64, i64, i32, vp, vp, vp]),
        "sgs_project_backward_adam": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp,
                                            sz, i64, P(AdamParamsC), vp, vp, vp, vp, vp]),
        "sgs_render_backward_adam": (i32, [P(GaussiansC), P(CameraC), i32, P(RasterParamsC), vp,
                                           sz, i64, vp, P(AdamParamsC), vp, vp, vp, vp, vp]),
        "sgs_camera_table_size": (i32, [i32, P(sz)]),
        "sgs_camera_table_init": (i32, [P(CameraC), i32, P(RasterParamsC), vp, sz, vp]),
        "sgs_view_sequence_next": (i32, [vp, i64, vp, vp, vp]),
        "sgs_train_iteration": (i32, [P(GaussiansC), P(CameraC), vp, i32, vp, P(RasterParamsC),
                                      vp, sz, i64, vp, f32, vp, sz, vp, vp, vp, P(GateParamsC),
                                      vp, vp, P(AdamParamsC), vp, vp, vp, vp]),
        "sgs_default_densify_params": (None, [P(DensifyParamsC)]),
        "sgs_densify_stats": (i32, [P(CameraC), i32, i64, P(RasterParamsC), vp, sz, i64, vp, vp,
                                    vp, vp]),
        "sgs_densify_workspace_size": (i32, [i64, P(sz)]),
        "sgs_densify": (i32, [P(DensifyParamsC), P(GaussiansC), vp, vp, vp, vp, vp, vp, vp, vp,
                              i64, vp, sz, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def _check(status: int):
    if status != SGS_OK:
        raise SkipGSError(status, LIB.sgs_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ---------------------------------------------------------------------------
# Marshalling helpers
# ---------------------------------------------------------------------------
@dataclass
class RasterParams:
    tile_w: int = 16
    tile_h: int = 16
    super_tile: int = 8
    lds_batch: int = 64
    split_prefix: int = 8192
    bg: tuple = (0.0, 0.0, 0.0)
    near_z: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    jac_clamp: float = 1.3

    def c(self) -> RasterParamsC:
        r = RasterParamsC()
        r.struct_size = C.sizeof(RasterParamsC)
        r.tile_w, r.tile_h = self.tile_w, self.tile_h
        r.super_tile, r.lds_batch = self.super_tile, self.lds_batch
        r.split_prefix = self.split_prefix
        for k in range(3):
            r.bg[k] = self.bg[k]
        r.near_z, r.dilation = self.near_z, self.dilation
        r.alpha_min, r.alpha_max, r.t_min, r.jac_clamp = (self.alpha_min, self.alpha_max,
                                                          self.t_min, self.jac_clamp)
        return r


def camera_c(cam) -> CameraC:
    c = CameraC()
    R = np.asarray(cam.R, dtype=np.float32).reshape(9)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def cameras_c(cams):
    arr = (CameraC * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_c(cam)
    return arr


def gaussians_c(planes: torch.Tensor, n: int, sh_degree: int) -> GaussiansC:
    if planes.dtype != torch.float32 or planes.dim() != 2:
        raise ValueError("planes must be a 2-D float32 tensor [F][stride]")
    g = GaussiansC()
    g.struct_size = C.sizeof(GaussiansC)
    g.data = _ptr(planes)
    g.n = int(n)
    g.stride = int(planes.shape[1])
    g.sh_degree = int(sh_degree)
    return g


def alloc_bytes(nbytes: int, device="cuda") -> torch.Tensor:
    """Device buffer of at least nbytes, 256-byte aligned (torch allocations are)."""
    return torch.empty(max(256, (int(nbytes) + 255) // 256 * 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# C entry points (same names without the sgs_ prefix)
# ---------------------------------------------------------------------------
def version() -> int:
    return LIB.sgs_version()


def forward_workspace_size(rp: RasterParams, n: int, cams, pair_capacity: int) -> int:
    out = C.c_size_t()
    cc = cameras_c(cams)
    _check(LIB.sgs_forward_workspace_size(C.byref(rp.c()), n, cc, len(cams), pair_capacity,
                                          C.byref(out)))
    return out.value


def get_workspace_layout(rp: RasterParams, n: int, cams, pair_capacity: int) -> WorkspaceLayoutC:
    out = WorkspaceLayoutC()
    _check(LIB.sgs_get_workspace_layout(C.byref(rp.c()), n, cameras_c(cams), len(cams),
                                        pair_capacity, C.byref(out)))
    return out


def render_forward(planes, n, sh_degree, cams, rp: RasterParams, workspace, pair_capacity, out_rgb,
                   stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_render_forward(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                                  _ptr(workspace), workspace.numel(), pair_capacity, _ptr(out_rgb),
                                  _stream(stream)))


def render_backward(planes, n, sh_degree, cams, rp: RasterParams, workspace, pair_capacity, dl_drgb,
                    d_gate, grads, stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_render_backward(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                                   _ptr(workspace), workspace.numel(), pair_capacity, _ptr(dl_drgb),
                                   _ptr(d_gate), _ptr(grads), _stream(stream)))


def project(planes, n, sh_degree, cams, rp, workspace, pair_capacity, stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_project(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                           _ptr(workspace), workspace.numel(), pair_capacity, _stream(stream)))


def load_records(cams, n, rp, workspace, pair_capacity, u, v, depth, extent, conic, opacity, rgb,
                 stream=None):
    _check(LIB.sgs_load_records(cameras_c(cams), len(cams), n, C.byref(rp.c()), _ptr(workspace),
                                workspace.numel(), pair_capacity, _ptr(u), _ptr(v), _ptr(depth),
                                _ptr(extent), _ptr(conic), _ptr(opacity), _ptr(rgb),
                                _stream(stream)))


def bin(cams, n, rp, workspace, pair_capacity, stream=None):  # noqa: A001 (C name)
    _check(LIB.sgs_bin(cameras_c(cams), len(cams), n, C.byref(rp.c()), _ptr(workspace),
                       workspace.numel(), pair_capacity, _stream(stream)))


def rasterize(cams, n, rp, workspace, pair_capacity, out_rgb, stream=None):
    _check(LIB.sgs_rasterize(cameras_c(cams), len(cams), n, C.byref(rp.c()), _ptr(workspace),
                             workspace.numel(), pair_capacity, _ptr(out_rgb), _stream(stream)))


def rasterize_backward(cams, n, rp, workspace, pair_capacity, dl_drgb, d_gate=None, stream=None):
    _check(LIB.sgs_rasterize_backward(cameras_c(cams), len(cams), n, C.byref(rp.c()),
                                      _ptr(workspace), workspace.numel(), pair_capacity,
                                      _ptr(dl_drgb), _ptr(d_gate), _stream(stream)))


def project_backward(planes, n, sh_degree, cams, rp, workspace, pair_capacity, d_gate, grads,
                     stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_project_backward(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                                    _ptr(workspace), workspace.numel(), pair_capacity,
                                    _ptr(d_gate), _ptr(grads), _stream(stream)))


def read_status(workspace, stream=None):
    flags = C.c_uint32()
    vis = C.c_int64()
    pairs = C.c_int64()
    _check(LIB.sgs_read_status(_ptr(workspace), C.byref(flags), C.byref(vis), C.byref(pairs),
                               _stream(stream)))
    return flags.value, vis.value, pairs.value


def read_counters(workspace, stream=None) -> dict:
    """Synchronises and reads the workspace counters (offset 0): status bits,
    visible entries, super-tile pairs (needed, written, kept), tile-list
    entries (of the prefix split; up to each tile's last blend; of the
    completing split), list segments, whether a tile needed more than its
    list prefix, and the blended / examined (pixel, Gaussian) pairs of the
    last bin + rasterize."""
    s = torch.cuda.current_stream() if stream is None else stream
    s.synchronize()
    w = workspace[:64].cpu().numpy().view(np.uint32)
    u64 = lambda i: int(w[i]) | (int(w[i + 1]) << 32)
    return {"status": int(w[0]), "visible": int(w[1]), "pairs": int(w[2]),
            "pairs_written": int(w[3]), "blended": u64(4), "evaluated": u64(6),
            "pairs_kept": int(w[8]), "items": int(w[9]), "segments": int(w[10]),
            "used": int(w[11]), "items_rest": int(w[12]), "redo": int(w[13])}


def clear_status(workspace, stream=None):
    _check(LIB.sgs_clear_status(_ptr(workspace), _stream(stream)))


def loss_workspace_size(width: int, height: int) -> int:
    out = C.c_size_t()
    _check(LIB.sgs_loss_workspace_size(width, height, C.byref(out)))
    return out.value


def photometric_loss(rgb, target, width, height, lam, workspace, d_loss, stream=None):
    _check(LIB.sgs_photometric_loss(_ptr(rgb), _ptr(target), width, height, float(lam),
                                    _ptr(workspace), workspace.numel(), _ptr(d_loss),
                                    _stream(stream)))


def photometric_loss_static(rgb, target, width, height, lam, d_loss, stream=None):
    """sgs_photometric_loss without a workspace (the library's static scratch)."""
    _check(LIB.sgs_photometric_loss_static(_ptr(rgb), _ptr(target), width, height, float(lam),
                                           _ptr(d_loss), _stream(stream)))


def photometric_loss_backward(rgb, target, width, height, lam, workspace, d_gate, dl_drgb,
                              stream=None):
    _check(LIB.sgs_photometric_loss_backward(_ptr(rgb), _ptr(target), width, height, float(lam),
                                             _ptr(workspace), workspace.numel(), _ptr(d_gate),
                                             _ptr(dl_drgb), _stream(stream)))


@dataclass
class GateParams:
    n_views: int
    beta: float = 0.95
    eps: float = 1e-8
    delta: float = 0.0
    rho_lo: float = 0.5
    warmup: int = 500
    window: int = 0
    calibrate: bool = True
    budget: bool = True

    def c(self) -> GateParamsC:
        return GateParamsC(C.sizeof(GateParamsC), self.beta, self.eps, self.delta, self.rho_lo, self.warmup, self.window,
                           int(self.calibrate), int(self.budget), self.n_views)


def paper_gate(n_views: int) -> GateParams:
    """Sec. 5.1 hyper-parameters: W = 500, beta = 0.95, eps = 1e-8, rho_lo = 0.5."""
    return GateParams(n_views=n_views)


def windowed_gate(n_views: int) -> GateParams:
    """EMA decay 0.9, skip within 2% of the EMA, >= 50% backward per 100 iterations."""
    return GateParams(n_views=n_views, beta=0.9, delta=0.02, warmup=0, window=100,
                      calibrate=False, budget=True)


def gate_state_size(p: GateParams) -> int:
    out = C.c_size_t()
    _check(LIB.sgs_gate_state_size(C.byref(p.c()), C.byref(out)))
    return out.value


def gate_init(p: GateParams, d_state, stream=None):
    _check(LIB.sgs_gate_init(C.byref(p.c()), _ptr(d_state), _stream(stream)))


def gate_update(p: GateParams, d_state, d_view, d_loss, d_gate, stream=None):
    """d_view: device int32 tensor holding the view index of the iteration."""
    _check(LIB.sgs_gate_update(C.byref(p.c()), _ptr(d_state), _ptr(d_view), _ptr(d_loss),
                               _ptr(d_gate), _stream(stream)))


def gate_read(p: GateParams, d_state, stream=None):
    snap = GateSnapshotC()
    ema = np.zeros(p.n_views, dtype=np.float64)
    has = np.zeros(p.n_views, dtype=np.uint8)
    _check(LIB.sgs_gate_read(C.byref(p.c()), _ptr(d_state), C.byref(snap),
                             ema.ctypes.data_as(C.c_void_p), has.ctypes.data_as(C.c_void_p),
                             _stream(stream)))
    d = {k: getattr(snap, k) for k, _ in GateSnapshotC._fields_}
    d["ema"] = ema
    d["has_ema"] = has
    return d


@dataclass
class AdamParams:
    lr: tuple
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    visible_only: bool = False

    def c(self) -> AdamParamsC:
        a = AdamParamsC()
        a.struct_size = C.sizeof(AdamParamsC)
        a.beta1, a.beta2, a.eps = self.beta1, self.beta2, self.eps
        a.visible_only = int(self.visible_only)
        for k, v in enumerate(self.lr):
            a.lr[k] = float(v)
        return a


@dataclass
class DensifyParams:
    grad_threshold: float = 2e-4
    percent_dense: float = 0.01
    scene_extent: float = 1.0
    min_opacity: float = 0.005
    split_scale: float = 1.6

    def c(self) -> DensifyParamsC:
        d = DensifyParamsC()
        d.struct_size = C.sizeof(DensifyParamsC)
        d.grad_threshold, d.percent_dense = self.grad_threshold, self.percent_dense
        d.scene_extent, d.min_opacity, d.split_scale = (self.scene_extent, self.min_opacity,
                                                        self.split_scale)
        return d


def densify_stats(cams, n, rp, workspace, pair_capacity, grad_sum, count, d_gate=None,
                  stream=None):
    _check(LIB.sgs_densify_stats(cameras_c(cams), len(cams), int(n), C.byref(rp.c()),
                                 _ptr(workspace), workspace.numel(), pair_capacity, _ptr(d_gate),
                                 _ptr(grad_sum), _ptr(count), _stream(stream)))


def densify_workspace_size(n: int) -> int:
    out = C.c_size_t()
    _check(LIB.sgs_densify_workspace_size(int(n), C.byref(out)))
    return out.value


def densify(p: DensifyParams, planes, n, sh_degree, m, v, grad_sum, count, normals, out_params,
            out_m, out_v, workspace, d_n_out, stream=None):
    """One clone / split / prune step into the output planes ([F][out_stride]);
    the new set's size goes to d_n_out (device int64[1])."""
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_densify(C.byref(p.c()), C.byref(g), _ptr(m), _ptr(v), _ptr(grad_sum),
                           _ptr(count), _ptr(normals), _ptr(out_params), _ptr(out_m), _ptr(out_v),
                           int(out_params.shape[1]), _ptr(workspace), workspace.numel(),
                           _ptr(d_n_out), _stream(stream)))


def default_lrs(sh_degree: int, means_lr: float = 1.6e-4) -> tuple:
    """Per-plane learning rates: means, log-scales, quaternion, opacity logit,
    SH DC, SH rest."""
    k = (sh_degree + 1) ** 2
    return tuple([means_lr] * 3 + [5e-3] * 3 + [1e-3] * 4 + [2.5e-2] + [2.5e-3] * 3
                 + [1.25e-4] * (3 * (k - 1)))


def project_backward_adam(planes, n, sh_degree, cams, rp, workspace, pair_capacity,
                          adam: AdamParams, m, v, d_step, d_gate=None, stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_project_backward_adam(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                                         _ptr(workspace), workspace.numel(), pair_capacity,
                                         C.byref(adam.c()), _ptr(m), _ptr(v), _ptr(d_step),
                                         _ptr(d_gate), _stream(stream)))


def render_backward_adam(planes, n, sh_degree, cams, rp, workspace, pair_capacity, dl_drgb,
                         adam: AdamParams, m, v, d_step, d_gate=None, stream=None):
    g = gaussians_c(planes, n, sh_degree)
    _check(LIB.sgs_render_backward_adam(C.byref(g), cameras_c(cams), len(cams), C.byref(rp.c()),
                                        _ptr(workspace), workspace.numel(), pair_capacity,
                                        _ptr(dl_drgb), C.byref(adam.c()), _ptr(m), _ptr(v),
                                        _ptr(d_step), _ptr(d_gate), _stream(stream)))


def adam_step(p: AdamParams, params, grads, m, v, n, d_step, d_gate=None, stream=None):
    _check(LIB.sgs_adam_step(C.byref(p.c()), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), int(n),
                             int(params.shape[1]), int(params.shape[0]), _ptr(d_step),
                             _ptr(d_gate), _stream(stream)))


class Prepared:
    """Pre-marshalled arguments for repeated calls on the same views and
    parameters (hot loops): C structs are built once, pointers are cached."""

    def __init__(self, planes, n, sh_degree, cams, rp: RasterParams, workspace, pair_capacity):
        self.g = gaussians_c(planes, n, sh_degree)
        self.cams = [cameras_c([c]) for c in cams]
        self.rp = rp.c()
        self.n = int(n)
        self.ws = _ptr(workspace)
        self.ws_bytes = workspace.numel()
        self.cap = int(pair_capacity)
        self._keep = (planes, workspace)

    def project(self, view, stream):
        _check(LIB.sgs_project(C.byref(self.g), self.cams[view], 1, C.byref(self.rp), self.ws,
                               self.ws_bytes, self.cap, stream))

    def bin(self, view, stream):
        _check(LIB.sgs_bin(self.cams[view], 1, self.n, C.byref(self.rp), self.ws, self.ws_bytes,
                           self.cap, stream))

    def rasterize(self, view, out_ptr, stream):
        _check(LIB.sgs_rasterize(self.cams[view], 1, self.n, C.byref(self.rp), self.ws,
                                 self.ws_bytes, self.cap, out_ptr, stream))

    def render_forward(self, view, out_ptr, stream):
        _check(LIB.sgs_render_forward(C.byref(self.g), self.cams[view], 1, C.byref(self.rp),
                                      self.ws, self.ws_bytes, self.cap, out_ptr, stream))

    def rasterize_backward(self, view, dl_ptr, gate_ptr, stream):
        _check(LIB.sgs_rasterize_backward(self.cams[view], 1, self.n, C.byref(self.rp), self.ws,
                                          self.ws_bytes, self.cap, dl_ptr, gate_ptr, stream))

    def project_backward_adam(self, view, adam_c, m_ptr, v_ptr, step_ptr, gate_ptr, stream):
        _check(LIB.sgs_project_backward_adam(C.byref(self.g), self.cams[view], 1, C.byref(self.rp),
                                             self.ws, self.ws_bytes, self.cap, C.byref(adam_c),
                                             m_ptr, v_ptr, step_ptr, gate_ptr, stream))

    def project_backward(self, view, gate_ptr, grads_ptr, stream):
        _check(LIB.sgs_project_backward(C.byref(self.g), self.cams[view], 1, C.byref(self.rp),
                                        self.ws, self.ws_bytes, self.cap, gate_ptr, grads_ptr,
                                        stream))


# ---------------------------------------------------------------------------
# Device-side view selection and the training iteration
# ---------------------------------------------------------------------------
def camera_table(cams, rp: RasterParams, device="cuda") -> torch.Tensor:
    """Device camera table of cameras of one resolution (synchronises)."""
    n = C.c_size_t()
    _check(LIB.sgs_camera_table_size(len(cams), C.byref(n)))
    t = alloc_bytes(n.value, device)
    _check(LIB.sgs_camera_table_init(cameras_c(cams), len(cams), C.byref(rp.c()), _ptr(t),
                                     t.numel(), _stream(None)))
    return t


def view_sequence_next(d_sequence, d_iter, d_view, stream=None):
    _check(LIB.sgs_view_sequence_next(_ptr(d_sequence), int(d_sequence.numel()), _ptr(d_iter),
                                      _ptr(d_view), _stream(stream)))


class TrainStep:
    """Pre-marshalled arguments of sgs_train_iteration (one call per
    iteration; the view index is read on the device)."""

    def __init__(self, planes, n, sh_degree, cams, table, d_view, rp: RasterParams, workspace,
                 pair_capacity, targets, lam, loss_ws, rgb, dl, d_loss, gate: "GateParams | None",
                 gate_state, d_gate, adam: "AdamParams", m, v, d_step):
        self.g = gaussians_c(planes, n, sh_degree)
        self.cams = cameras_c(cams)
        self.rp = rp.c()
        self.gp = gate.c() if gate is not None else None
        self.adam = adam.c()
        self.args = (_ptr(table), len(cams), _ptr(d_view), workspace.numel(), int(pair_capacity),
                     _ptr(targets), float(lam), _ptr(loss_ws), loss_ws.numel(), _ptr(rgb),
                     _ptr(dl), _ptr(d_loss), _ptr(gate_state) if gate is not None else None,
                     _ptr(d_gate), _ptr(m), _ptr(v), _ptr(d_step))
        self.ws = _ptr(workspace)
        self._keep = (planes, table, d_view, workspace, targets, loss_ws, rgb, dl, d_loss,
                      gate_state, d_gate, m, v, d_step)

    def __call__(self, stream):
        (tab, ncam, dview, wsb, cap, tgt, lam, lws, lwsb, rgb, dl, dloss, gst, dgate, m, v,
         step) = self.args
        gp = C.byref(self.gp) if self.gp is not None else None
        _check(LIB.sgs_train_iteration(C.byref(self.g), self.cams, tab, ncam, dview,
                                       C.byref(self.rp), self.ws, wsb, cap, tgt, lam, lws, lwsb,
                                       rgb, dl, dloss, gp, gst, dgate, C.byref(self.adam), m, v,
                                       step, stream))
