"""Python binding of ``libairgs_gs.so`` (the C ABI in ``include/airgs_gs.h``).

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory and streams.  The
library is loaded on first use and a missing library raises -- there is no
fallback path.

Structures mirror the header one to one; the functions keep the C names.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libairgs_gs.so")

GS_OK = 0
GS_ERR_INVALID_ARG = 1
GS_ERR_CAPACITY = 2
GS_ERR_OOM = 3
GS_ERR_HIP = 4
TILE = 16
GS_MAX_INSTANCES = (1 << 30) - 1
GS_NOALLOC_MAX_TILES = 1 << 18
SPLAT_FLOATS = 16
GS_PROJECT_TIGHT_RECT = 1
GS_PROJECT_TILE_SPANS = 2
GRAD2D_FLOATS = 12
STAGE_COUNT = 18
WORK_COUNTERS = 8  # GS_WORK_COUNTERS
WORK_COUNTER_NAMES = ("fwd_staged", "fwd_visits", "fwd_slots", "fwd_used", "bwd_staged",
                      "bwd_visits", "bwd_slots", "bwd_used")

c_int32, c_int64, c_void_p, c_double, c_float = (ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                                 ctypes.c_double, ctypes.c_float)


class GsGaussians(ctypes.Structure):
    _fields_ = [("n", c_int32), ("sh_degree", c_int32), ("ld", c_int32), ("reserved", c_int32),
                ("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p),
                ("opacity", c_void_p), ("sh", c_void_p)]


class GsCamera(ctypes.Structure):
    _fields_ = [("R", c_double * 9), ("t", c_double * 3), ("fx", c_double), ("fy", c_double),
                ("cx", c_double), ("cy", c_double), ("width", c_int32), ("height", c_int32),
                ("reserved", c_int32 * 2)]


class GsOpts(ctypes.Structure):
    _fields_ = [("bg", c_float * 3), ("reserved", c_float), ("usage", c_void_p),
                ("grad2d_norm", c_void_p), ("visible_views", c_void_p)]


class GsProjected(ctypes.Structure):
    _fields_ = [("n_views", c_int32), ("n", c_int32), ("ld", c_int32), ("options", c_int32),
                ("splat", c_void_p), ("rect", c_void_p), ("tiles_touched", c_void_p),
                ("depth_bits", c_void_p), ("flags", c_void_p)]


class GsTileLists(ctypes.Structure):
    _fields_ = [("capacity", c_int64), ("count", c_int64), ("n_segments", c_int64),
                ("keys", c_void_p), ("vals", c_void_p), ("ranges", c_void_p),
                ("gv_capacity", c_int64), ("gv_base", c_void_p)]


class GsFrameUpdate(ctypes.Structure):
    _fields_ = [("anchor_quat", c_void_p), ("ld", c_int32), ("gw", c_int32), ("gh", c_int32),
                ("temporal_weight", c_float), ("mask", c_void_p), ("delta", c_void_p),
                ("temporal_loss", c_void_p)]


assert ctypes.sizeof(GsCamera) == 144


class GsSequence(ctypes.Structure):
    _fields_ = [("anchor", GsGaussians), ("deltas", c_void_p), ("masks", c_void_p),
                ("n_frames", c_int32), ("gw", c_int32), ("gh", c_int32), ("reserved", c_int32)]


class GsRequest(ctypes.Structure):
    _fields_ = [("cam", GsCamera), ("frame", c_int32), ("reserved", c_int32),
                ("arrival_s", c_double)]


class GsServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", c_int32), ("n_workers", c_int32), ("options", c_int32),
                ("inline_singletons", c_int32), ("budget_bytes", c_int64),
                ("bg", c_float * 3), ("reserved", c_float)]


class GsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gs error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.gs_version.restype = ctypes.c_int
    lib.gs_create.argtypes = [P(c_void_p), ctypes.c_int]
    lib.gs_destroy.argtypes = [c_void_p]
    lib.gs_last_error.argtypes = [c_void_p]
    lib.gs_last_error.restype = ctypes.c_char_p
    lib.gs_num_segments.argtypes = [P(GsCamera), ctypes.c_int]
    lib.gs_num_segments.restype = c_int64
    lib.gs_bin_sort_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, c_int64, c_int64]
    lib.gs_bin_sort_workspace_size.restype = ctypes.c_size_t
    lib.gs_render_bwd_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, c_int64]
    lib.gs_render_bwd_workspace_size.restype = ctypes.c_size_t
    lib.gs_apply_frame_update.argtypes = [c_void_p, P(GsGaussians), c_void_p, c_void_p,
                                          ctypes.c_int, ctypes.c_int, P(GsGaussians), c_void_p]
    lib.gs_project.argtypes = [c_void_p, P(GsGaussians), P(GsCamera), c_void_p, ctypes.c_int,
                               P(GsProjected), c_void_p]
    lib.gs_bin_sort.argtypes = [c_void_p, P(GsProjected), P(GsCamera), c_void_p, ctypes.c_int,
                                P(GsTileLists), c_void_p, ctypes.c_size_t, c_void_p]
    lib.gs_render_fwd.argtypes = [c_void_p, P(GsProjected), P(GsTileLists), P(GsCamera),
                                  c_void_p, ctypes.c_int, P(GsOpts), c_void_p, c_void_p,
                                  c_void_p, c_void_p]
    lib.gs_render_fwd_l1_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gs_render_fwd_l1_workspace_size.restype = ctypes.c_size_t
    lib.gs_render_fwd_l1.argtypes = [c_void_p, P(GsProjected), P(GsTileLists), P(GsCamera),
                                     c_void_p, ctypes.c_int, P(GsOpts), c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                     ctypes.c_size_t, c_void_p]
    lib.gs_render_fwd_l1.restype = c_int32
    lib.gs_render_fwd_l1_noalloc.argtypes = [c_void_p, P(GsProjected), P(GsTileLists),
                                             P(GsCamera), c_void_p, ctypes.c_int, P(GsOpts),
                                             c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                             c_void_p, c_void_p]
    lib.gs_render_fwd_l1_noalloc.restype = c_int32
    lib.gs_render_bwd.argtypes = [c_void_p, P(GsGaussians), P(GsProjected), P(GsTileLists),
                                  P(GsCamera), c_void_p, ctypes.c_int, P(GsOpts), c_void_p,
                                  c_void_p, c_void_p, P(GsGaussians), P(GsFrameUpdate), c_void_p,
                                  c_void_p, ctypes.c_size_t, c_void_p]
    lib.gs_l1_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                    c_void_p]
    lib.gs_keyframe_temporal_l1.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int,
                                            ctypes.c_int, c_int64, c_float, c_void_p, c_void_p,
                                            c_void_p]
    lib.gs_cull_workspace_size.argtypes = [ctypes.c_int]
    lib.gs_cull_workspace_size.restype = ctypes.c_size_t
    lib.gs_cull_low_opacity.argtypes = [c_void_p, c_void_p, ctypes.c_int, c_float, c_void_p,
                                        P(c_int32), c_void_p, ctypes.c_size_t, c_void_p]
    lib.gs_gather_planes.argtypes = [c_void_p, c_void_p, c_int64, ctypes.c_int, c_void_p,
                                     ctypes.c_int, c_void_p, c_int64, c_void_p]
    lib.gs_residual_delta.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, c_void_p, c_void_p, c_void_p]
    lib.gs_quantize_delta.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p]
    lib.gs_apply_quantized_update.argtypes = [c_void_p, P(GsGaussians), c_void_p, ctypes.c_int,
                                              c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
                                              P(GsGaussians), c_void_p]
    for f in ("gs_keyframe_temporal_l1", "gs_cull_low_opacity", "gs_gather_planes",
              "gs_residual_delta", "gs_quantize_delta", "gs_apply_quantized_update"):
        getattr(lib, f).restype = c_int32
    lib.gs_l1_dssim_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gs_l1_dssim_workspace_size.restype = ctypes.c_size_t
    lib.gs_l1_dssim_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, c_float, c_void_p, c_void_p, c_void_p,
                                          ctypes.c_size_t, c_void_p]
    lib.gs_l1_dssim_loss_grad.restype = c_int32
    lib.gs_sq_error.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
    lib.gs_sq_error.restype = c_int32
    lib.gs_adam_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                 ctypes.c_int, c_float, c_float, c_float, c_float, c_void_p]
    lib.gs_render_batched_workspace_size.argtypes = [ctypes.c_int]
    lib.gs_render_batched_workspace_size.restype = ctypes.c_size_t
    lib.gs_render_fwd_batched.argtypes = [c_void_p, P(GsProjected), P(GsTileLists), P(GsCamera),
                                          c_void_p, ctypes.c_int, P(GsOpts), c_void_p, c_void_p,
                                          ctypes.c_size_t, c_void_p]
    lib.gs_render_fwd_batched.restype = c_int32
    lib.gs_set_timing.argtypes = [c_void_p, ctypes.c_int]
    lib.gs_set_timing_mask.argtypes = [c_void_p, ctypes.c_uint32]
    lib.gs_set_timing_mask.restype = c_int32
    lib.gs_set_work_counters.argtypes = [c_void_p, c_void_p]
    lib.gs_set_work_counters.restype = c_int32
    lib.gs_server_create.argtypes = [P(c_void_p), ctypes.c_int, P(GsSequence),
                                     P(GsServerConfig)]
    lib.gs_server_create.restype = c_int32
    lib.gs_server_destroy.argtypes = [c_void_p]
    lib.gs_server_last_error.argtypes = [c_void_p]
    lib.gs_server_last_error.restype = ctypes.c_char_p
    lib.gs_server_run.argtypes = [c_void_p, P(GsRequest), ctypes.c_int, ctypes.c_int,
                                  P(c_double), P(c_double), P(c_void_p)]
    lib.gs_server_run.restype = c_int32
    lib.gs_server_stats.argtypes = [c_void_p, P(c_int64)]
    lib.gs_server_stats.restype = c_int32
    lib.gs_peak_min_bytes.argtypes = [ctypes.c_int]
    lib.gs_peak_min_bytes.restype = ctypes.c_size_t
    lib.gs_peak_run.argtypes = [c_void_p, ctypes.c_int, c_void_p, ctypes.c_size_t, ctypes.c_int,
                                P(c_double), P(c_double), c_void_p]
    lib.gs_peak_run.restype = c_int32
    lib.gs_collect_timing.argtypes = [c_void_p, P(c_double), P(c_int64)]
    lib.gs_stage_name.argtypes = [ctypes.c_int]
    lib.gs_stage_name.restype = ctypes.c_char_p
    for f in ("gs_set_timing", "gs_collect_timing"):
        getattr(lib, f).restype = c_int32
    for f in ("gs_create", "gs_apply_frame_update", "gs_project", "gs_bin_sort", "gs_render_fwd",
              "gs_render_bwd", "gs_l1_loss_grad", "gs_adam_step"):
        getattr(lib, f).restype = c_int32
    _lib = lib
    return lib


def exported_symbols():
    return ["gs_version", "gs_create", "gs_destroy", "gs_last_error", "gs_num_segments",
            "gs_bin_sort_workspace_size", "gs_render_bwd_workspace_size",
            "gs_apply_frame_update", "gs_project", "gs_bin_sort", "gs_render_fwd",
            "gs_render_bwd", "gs_l1_loss_grad", "gs_adam_step", "gs_set_timing",
            "gs_collect_timing", "gs_stage_name", "gs_render_batched_workspace_size",
            "gs_render_fwd_batched", "gs_sq_error", "gs_l1_dssim_workspace_size",
            "gs_l1_dssim_loss_grad", "gs_keyframe_temporal_l1", "gs_cull_workspace_size",
            "gs_cull_low_opacity", "gs_gather_planes", "gs_residual_delta",
            "gs_quantize_delta", "gs_apply_quantized_update", "gs_render_fwd_l1_workspace_size",
            "gs_render_fwd_l1", "gs_render_fwd_l1_noalloc", "gs_set_work_counters",
            "gs_peak_min_bytes", "gs_peak_run", "gs_server_create", "gs_server_destroy",
            "gs_server_last_error", "gs_server_run", "gs_server_stats", "gs_set_timing_mask"]


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """Owns a gs_ctx bound to one device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = c_void_p()
        st = self.lib.gs_create(ctypes.byref(h), int(device))
        if st != GS_OK:
            raise GsError(st, self.lib.gs_last_error(None).decode())
        self.handle = h
        self.device = device

    def check(self, st: int):
        if st != GS_OK:
            raise GsError(st, self.lib.gs_last_error(self.handle).decode())

    def set_timing(self, on: bool):
        self.check(self.lib.gs_set_timing(self.handle, 1 if on else 0))

    def set_timing_stages(self, names):
        """Time only the named stages (an empty list switches timing off)."""
        mask = 0
        for nm in names:
            k = [self.lib.gs_stage_name(i).decode() for i in range(STAGE_COUNT)].index(nm)
            mask |= 1 << k
        self.check(self.lib.gs_set_timing_mask(self.handle, mask))

    def set_work_counters(self, counters):
        """counters: a zeroed int64 device tensor of WORK_COUNTERS values that
        the render calls of this context add their work tallies to, or None
        to switch counting off."""
        if counters is not None:
            assert counters.dtype == torch.int64 and counters.numel() >= WORK_COUNTERS
        self.check(self.lib.gs_set_work_counters(self.handle, _ptr(counters)))

    def collect_timing(self) -> dict:
        """{stage name: (total ms, launches)} since the last collection."""
        ms = (c_double * STAGE_COUNT)()
        n = (c_int64 * STAGE_COUNT)()
        self.check(self.lib.gs_collect_timing(self.handle, ms, n))
        return {self.lib.gs_stage_name(k).decode(): (ms[k], n[k]) for k in range(STAGE_COUNT)}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


_default_ctx: Context | None = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(torch.cuda.current_device())
    return _default_ctx


# ---------------------------------------------------------------------------
# argument holders
# ---------------------------------------------------------------------------

@dataclass
class Gaussians:
    """FP32 planar Gaussian set on the device (stride ld)."""
    n: int
    deg: int
    ld: int
    mean: torch.Tensor       # (3, ld)
    log_scale: torch.Tensor  # (3, ld)
    quat: torch.Tensor       # (4, ld)
    opacity: torch.Tensor    # (ld,)
    sh: torch.Tensor         # (K, 3, ld)

    def c(self) -> GsGaussians:
        return GsGaussians(self.n, self.deg, self.ld, 0, _ptr(self.mean), _ptr(self.log_scale),
                           _ptr(self.quat), _ptr(self.opacity), _ptr(self.sh))

    @staticmethod
    def from_scene(scene: dict, device="cuda") -> "Gaussians":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=device)  # noqa: E731
        return Gaussians(scene["n"], scene["deg"], scene["ld"], t(scene["mean"]),
                         t(scene["log_scale"]), t(scene["quat"]), t(scene["opacity"]),
                         t(scene["sh"]))

    @staticmethod
    def zeros_like(g: "Gaussians") -> "Gaussians":
        z = torch.zeros_like
        return Gaussians(g.n, g.deg, g.ld, z(g.mean), z(g.log_scale), z(g.quat), z(g.opacity),
                         z(g.sh))

    def planes(self):
        return [self.mean, self.log_scale, self.quat, self.opacity, self.sh]


class Cameras:
    """Host ctypes array plus its device copy."""

    def __init__(self, cams: dict, device="cuda"):
        R = np.asarray(cams["R"], np.float64).reshape(-1, 9)
        t = np.asarray(cams["t"], np.float64).reshape(-1, 3)
        f = np.asarray(cams["f"], np.float64).reshape(-1, 4)
        wh = np.asarray(cams["wh"]).reshape(-1, 2)
        V = R.shape[0]
        self.V = V
        self.host = (GsCamera * V)()
        for v in range(V):
            c = self.host[v]
            c.R[:] = R[v].tolist()
            c.t[:] = t[v].tolist()
            c.fx, c.fy, c.cx, c.cy = (float(x) for x in f[v])
            c.width, c.height = int(wh[v, 0]), int(wh[v, 1])
        raw = np.frombuffer(bytes(self.host), dtype=np.uint8).copy()
        self.dev = torch.from_numpy(raw).to(device)
        self.wh = [(int(wh[v, 0]), int(wh[v, 1])) for v in range(V)]

    def n_segments(self) -> int:
        return int(load().gs_num_segments(self.host, self.V))

    def slice(self, start: int, count: int) -> "Cameras":
        """Views start .. start+count-1, sharing this object's memory."""
        out = Cameras.__new__(Cameras)
        out.V = count
        out.host = (GsCamera * count).from_address(ctypes.addressof(self.host[start]))
        out._owner = self
        nb = ctypes.sizeof(GsCamera)
        out.dev = self.dev[start * nb:(start + count) * nb]
        out.wh = self.wh[start:start + count]
        return out

    @staticmethod
    def from_list(items, device="cuda", stream=None) -> "Cameras":
        """Cameras from (R, t, f, (W, H)) tuples."""
        R = np.stack([np.asarray(it[0], np.float64) for it in items])
        t = np.stack([np.asarray(it[1], np.float64) for it in items])
        f = np.stack([np.asarray(it[2], np.float64) for it in items])
        wh = np.array([it[3] for it in items], np.int32)
        return Cameras(dict(R=R, t=t, f=f, wh=wh), device)


@dataclass
class Projected:
    V: int
    n: int
    ld: int
    splat: torch.Tensor          # (V, ld, 16) f32
    rect: torch.Tensor           # (V, ld, 4) i32
    tiles_touched: torch.Tensor  # (V, ld) i32
    depth_bits: torch.Tensor     # (V, ld) i32 (uint32 bits)
    flags: torch.Tensor          # (V, ld) u8
    options: int = 0             # GS_PROJECT_TIGHT_RECT | GS_PROJECT_TILE_SPANS

    @staticmethod
    def empty(V: int, n: int, ld: int, device="cuda") -> "Projected":
        return Projected(V, n, ld, torch.empty(V, ld, SPLAT_FLOATS, device=device),
                         torch.empty(V, ld, 4, dtype=torch.int32, device=device),
                         torch.empty(V, ld, dtype=torch.int32, device=device),
                         torch.empty(V, ld, dtype=torch.int32, device=device),
                         torch.empty(V, ld, dtype=torch.uint8, device=device))

    def slice(self, start: int, count: int) -> "Projected":
        return Projected(count, self.n, self.ld, self.splat[start:start + count],
                         self.rect[start:start + count], self.tiles_touched[start:start + count],
                         self.depth_bits[start:start + count], self.flags[start:start + count],
                         self.options)

    def c(self) -> GsProjected:
        return GsProjected(self.V, self.n, self.ld, self.options, _ptr(self.splat),
                           _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_bits),
                           _ptr(self.flags))


class TileLists:
    """Sorted tile lists; ``gv`` > 0 also allocates the optional copy of the
    per-(view, Gaussian) emission bases (at least n_views * ld entries)."""

    def __init__(self, capacity: int, n_segments: int, with_keys: bool = False, device="cuda",
                 gv: int = 0):
        self.capacity = int(capacity)
        self.n_segments = int(n_segments)
        self.count = 0
        self.vals = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.keys = (torch.empty(max(self.capacity, 1), dtype=torch.int64, device=device)
                     if with_keys else None)
        self.ranges = torch.empty(max(self.n_segments, 1), 2, dtype=torch.int32, device=device)
        self.gv = int(gv)
        self.gv_base = (torch.empty(self.gv, dtype=torch.int32, device=device)
                        if self.gv > 0 else None)
        self._c = GsTileLists(self.capacity, 0, self.n_segments, _ptr(self.keys), _ptr(self.vals),
                              _ptr(self.ranges), self.gv, _ptr(self.gv_base))

    def c(self) -> GsTileLists:
        return self._c


# ---------------------------------------------------------------------------
# C ABI calls, same names
# ---------------------------------------------------------------------------

def gs_apply_frame_update(ctx: Context, anchor: Gaussians, delta: torch.Tensor,
                          mask: torch.Tensor, gw: int, gh: int, frame: Gaussians, stream=None):
    a, f = anchor.c(), frame.c()
    ctx.check(ctx.lib.gs_apply_frame_update(ctx.handle, ctypes.byref(a), _ptr(delta), _ptr(mask),
                                            gw, gh, ctypes.byref(f), _stream(stream)))


def gs_project(ctx: Context, g: Gaussians, cams: Cameras, out: Projected, stream=None):
    gc, oc = g.c(), out.c()
    ctx.check(ctx.lib.gs_project(ctx.handle, ctypes.byref(gc), cams.host, _ptr(cams.dev), cams.V,
                                 ctypes.byref(oc), _stream(stream)))


def gs_bin_sort(ctx: Context, proj: Projected, cams: Cameras, lists: TileLists,
                workspace: torch.Tensor, stream=None) -> int:
    """Returns the instance count; raises GsError(GS_ERR_CAPACITY) with
    ``lists.count`` set when the capacity is too small."""
    pc = proj.c()
    lc = lists.c()
    st = ctx.lib.gs_bin_sort(ctx.handle, ctypes.byref(pc), cams.host, _ptr(cams.dev), cams.V,
                             ctypes.byref(lc), _ptr(workspace), workspace.numel(),
                             _stream(stream))
    lists.count = int(lc.count)
    ctx.check(st)
    return lists.count


def gs_render_fwd(ctx: Context, proj: Projected, lists: TileLists, cams: Cameras, bg,
                  image: torch.Tensor, final_T: torch.Tensor, n_contrib: torch.Tensor,
                  stream=None, usage: torch.Tensor | None = None):
    """``usage`` (int32 tensor of n, nullable) accumulates composited-pixel
    counts per Gaussian."""
    pc = proj.c()
    opts = GsOpts((c_float * 3)(*[float(x) for x in bg]), 0.0, _ptr(usage), None, None)
    ctx.check(ctx.lib.gs_render_fwd(ctx.handle, ctypes.byref(pc), ctypes.byref(lists.c()),
                                    cams.host, _ptr(cams.dev), cams.V, ctypes.byref(opts),
                                    _ptr(image), _ptr(final_T), _ptr(n_contrib),
                                    _stream(stream)))


def render_fwd_l1_workspace_size(V: int, width: int, height: int) -> int:
    return int(load().gs_render_fwd_l1_workspace_size(V, width, height))


def gs_render_fwd_l1(ctx: Context, proj: Projected, lists: TileLists, cams: Cameras, bg,
                     target: torch.Tensor, image: torch.Tensor | None, final_T: torch.Tensor,
                     n_contrib: torch.Tensor, dL_dimage: torch.Tensor, loss_dev: torch.Tensor,
                     workspace: torch.Tensor, stream=None):
    """Forward fused with the L1 term: dL/dimage written, mean |image -
    target| accumulated into ``loss_dev``; ``image`` may be None."""
    pc = proj.c()
    opts = GsOpts((c_float * 3)(*[float(x) for x in bg]), 0.0, None, None, None)
    ctx.check(ctx.lib.gs_render_fwd_l1(ctx.handle, ctypes.byref(pc), ctypes.byref(lists.c()),
                                       cams.host, _ptr(cams.dev), cams.V, ctypes.byref(opts),
                                       _ptr(target), _ptr(image), _ptr(final_T),
                                       _ptr(n_contrib), _ptr(dL_dimage), _ptr(loss_dev),
                                       _ptr(workspace), workspace.numel(), _stream(stream)))


def gs_render_fwd_l1_noalloc(ctx: Context, proj: Projected, lists: TileLists, cams: Cameras,
                             bg, target: torch.Tensor, image: torch.Tensor | None,
                             final_T: torch.Tensor, n_contrib: torch.Tensor,
                             dL_dimage: torch.Tensor, loss_dev: torch.Tensor, stream=None):
    """gs_render_fwd_l1 with its per-tile partials in the library's fixed
    device array instead of a workspace (the call allocates nothing)."""
    pc = proj.c()
    opts = GsOpts((c_float * 3)(*[float(x) for x in bg]), 0.0, None, None, None)
    ctx.check(ctx.lib.gs_render_fwd_l1_noalloc(
        ctx.handle, ctypes.byref(pc), ctypes.byref(lists.c()), cams.host, _ptr(cams.dev),
        cams.V, ctypes.byref(opts), _ptr(target), _ptr(image), _ptr(final_T), _ptr(n_contrib),
        _ptr(dL_dimage), _ptr(loss_dev), _stream(stream)))


def gs_render_fwd_batched(ctx: Context, proj: Projected, lists: TileLists, cams: Cameras, bg,
                          images: torch.Tensor, workspace: torch.Tensor, stream=None):
    pc = proj.c()
    opts = GsOpts((c_float * 3)(*[float(x) for x in bg]), 0.0, None, None, None)
    ctx.check(ctx.lib.gs_render_fwd_batched(ctx.handle, ctypes.byref(pc), ctypes.byref(lists.c()),
                                            cams.host, _ptr(cams.dev), cams.V, ctypes.byref(opts),
                                            _ptr(images), _ptr(workspace), workspace.numel(),
                                            _stream(stream)))


def render_batched_workspace_size(V: int) -> int:
    return int(load().gs_render_batched_workspace_size(V))


def gs_render_bwd(ctx: Context, frame: Gaussians, proj: Projected, lists: TileLists,
                  cams: Cameras, bg, final_T, n_contrib, dL_dimage, grad: Gaussians,
                  workspace: torch.Tensor, upd=None, dL_ddelta=None, stream=None,
                  densify=None, temporal=None):
    """``upd`` = (anchor_quat tensor, mask tensor, gw, gh) or None;
    ``densify`` = (grad2d_norm float tensor, visible_views int32 tensor) or
    None; ``temporal`` = (weight, delta tensor, loss float64 tensor or None)
    or None, used with ``upd``."""
    fc, pc, gc = frame.c(), proj.c(), grad.c()
    dn, dv = densify if densify is not None else (None, None)
    opts = GsOpts((c_float * 3)(*[float(x) for x in bg]), 0.0, None, _ptr(dn), _ptr(dv))
    uc = None
    if upd is not None:
        aq, mask, gw, gh = upd
        tw, td, tl = temporal if temporal is not None else (0.0, None, None)
        uc = ctypes.byref(GsFrameUpdate(_ptr(aq), frame.ld, gw, gh, float(tw), _ptr(mask),
                                        _ptr(td), _ptr(tl)))
    ctx.check(ctx.lib.gs_render_bwd(ctx.handle, ctypes.byref(fc), ctypes.byref(pc),
                                    ctypes.byref(lists.c()), cams.host, _ptr(cams.dev), cams.V,
                                    ctypes.byref(opts), _ptr(final_T), _ptr(n_contrib),
                                    _ptr(dL_dimage), ctypes.byref(gc), uc, _ptr(dL_ddelta),
                                    _ptr(workspace), workspace.numel(), _stream(stream)))


PEAK_KINDS = {"copy": 0, "read": 1, "lds": 2, "fma": 3, "exp": 4, "atomic_spread": 5,
              "atomic_same": 6}


def peak_min_bytes(kind: str) -> int:
    return int(load().gs_peak_min_bytes(PEAK_KINDS[kind]))


def gs_peak_run(ctx: Context, kind: str, buf: torch.Tensor, iters: int = 1, stream=None):
    """One timed launch of a peak-rate probe: (milliseconds, work)."""
    ms, work = c_double(), c_double()
    ctx.check(ctx.lib.gs_peak_run(ctx.handle, PEAK_KINDS[kind], _ptr(buf),
                                  buf.numel() * buf.element_size(), int(iters),
                                  ctypes.byref(ms), ctypes.byref(work), _stream(stream)))
    return ms.value, work.value


def gs_l1_loss_grad(ctx: Context, image, target, grad, loss_dev, stream=None):
    ctx.check(ctx.lib.gs_l1_loss_grad(ctx.handle, _ptr(image), _ptr(target), image.numel(),
                                      _ptr(grad), _ptr(loss_dev), _stream(stream)))


def gs_l1_dssim_loss_grad(ctx: Context, image, target, grad, loss_dev, workspace, lam=0.2,
                          stream=None):
    """Eq. (1) loss over (V, 3, H, W) images; grad written, loss accumulated."""
    H, W = image.shape[-2], image.shape[-1]
    planes = image.numel() // (H * W)
    ctx.check(ctx.lib.gs_l1_dssim_loss_grad(ctx.handle, _ptr(image), _ptr(target), planes, H, W,
                                            float(lam), _ptr(grad), _ptr(loss_dev),
                                            _ptr(workspace), workspace.numel(), _stream(stream)))


def l1_dssim_workspace_size(planes: int, H: int, W: int) -> int:
    return int(load().gs_l1_dssim_workspace_size(planes, H, W))


def gs_sq_error(ctx: Context, a, b, sum_dev, stream=None):
    ctx.check(ctx.lib.gs_sq_error(ctx.handle, _ptr(a), _ptr(b), a.numel(), _ptr(sum_dev),
                                  _stream(stream)))


def gs_adam_step(ctx: Context, param, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, stream=None):
    ctx.check(ctx.lib.gs_adam_step(ctx.handle, _ptr(param), _ptr(grad), _ptr(m), _ptr(v),
                                   param.numel(), int(step), float(lr), float(beta1),
                                   float(beta2), float(eps), _stream(stream)))


def bin_sort_workspace_size(V: int, ld: int, capacity: int, n_segments: int) -> int:
    return int(load().gs_bin_sort_workspace_size(V, ld, capacity, n_segments))


def render_bwd_workspace_size(V: int, ld: int, instances: int) -> int:
    return int(load().gs_render_bwd_workspace_size(V, ld, instances))


# ---- keyframe reconstruction ---------------------------------------------

def gs_keyframe_temporal_l1(ctx: Context, x, x_prev, bound: int, weight: float, grad,
                            loss_dev=None, stream=None):
    """Eq. (9): grad += weight * sign(x - x_prev) over the first ``bound``
    columns of the (rows, ld) planes; loss accumulated when given."""
    rows, ld = x.shape[0], x.shape[-1]
    ctx.check(ctx.lib.gs_keyframe_temporal_l1(ctx.handle, _ptr(x), _ptr(x_prev), rows, bound, ld,
                                              float(weight), _ptr(grad), _ptr(loss_dev),
                                              _stream(stream)))


def gs_cull_low_opacity(ctx: Context, opacity_logit, n: int, min_opacity: float, kept_index,
                        workspace=None, stream=None) -> int:
    """Indices of the Gaussians kept by low-opacity culling (written to
    ``kept_index``); returns their number (blocking)."""
    if workspace is None:
        workspace = torch.empty(max(cull_workspace_size(n), 1), dtype=torch.uint8,
                                device=opacity_logit.device)
    out = c_int32(0)
    ctx.check(ctx.lib.gs_cull_low_opacity(ctx.handle, _ptr(opacity_logit), n, float(min_opacity),
                                          _ptr(kept_index), ctypes.byref(out), _ptr(workspace),
                                          workspace.numel(), _stream(stream)))
    return int(out.value)


def cull_workspace_size(n: int) -> int:
    return int(load().gs_cull_workspace_size(n))


def gs_gather_planes(ctx: Context, src, index, m: int, dst, stream=None):
    """dst[p, j] = src[p, index[j]] for the (planes, ld) views src and dst."""
    planes = src.shape[0] if src.dim() > 1 else 1
    ctx.check(ctx.lib.gs_gather_planes(ctx.handle, _ptr(src), src.shape[-1], planes, _ptr(index),
                                       m, _ptr(dst), dst.shape[-1], _stream(stream)))


# ---- sent updates --------------------------------------------------------

def gs_residual_delta(ctx: Context, D_t, Dp_prev, mask, n: int, gw: int, gh: int, d_out, absmax,
                      stream=None):
    ctx.check(ctx.lib.gs_residual_delta(ctx.handle, _ptr(D_t), _ptr(Dp_prev), _ptr(mask), n, gw,
                                        gh, _ptr(d_out), _ptr(absmax), _stream(stream)))


def gs_quantize_delta(ctx: Context, d, absmax, bits: int, n: int, gw: int, gh: int, q_out,
                      scale_out, Dp=None, stream=None):
    ctx.check(ctx.lib.gs_quantize_delta(ctx.handle, _ptr(d), _ptr(absmax), bits, n, gw, gh,
                                        _ptr(q_out), _ptr(scale_out), _ptr(Dp), _stream(stream)))


def gs_apply_quantized_update(ctx: Context, anchor: Gaussians, q, bits: int, scale, Dp, gw: int,
                              gh: int, frame: Gaussians, stream=None):
    a, f = anchor.c(), frame.c()
    ctx.check(ctx.lib.gs_apply_quantized_update(ctx.handle, ctypes.byref(a), _ptr(q), bits,
                                                _ptr(scale), _ptr(Dp), gw, gh, ctypes.byref(f),
                                                _stream(stream)))
