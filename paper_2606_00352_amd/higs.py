"""Thin ctypes binding of libhigs (include/higs.h).

Argument marshalling only: every step of the frame path runs in the HIP
kernels of libhigs.so.  Torch supplies device memory (tensor.data_ptr()) and
streams (torch.cuda.current_stream().cuda_stream, a hipStream_t on ROCm).
There is no fallback: if the library is not built this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhigs.so")

OK, E_INVALID, E_NOMEM, E_CAPACITY, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
OVF_PAIRS, OVF_BATCHES = 1, 2
DBG_PROJ, DBG_RECORDS, DBG_PAIRS, DBG_SORTED, DBG_MT_OFFSETS, DBG_BATCHES, DBG_ACTIVE, DBG_PARTIALS = range(1, 9)
DEBUG_KEEP_PAIRS, DEBUG_COUNT_EVALS, DEBUG_PROJ_FIELDS, DEBUG_TWO_WORD_PAIRS = 1, 2, 4, 8
SORT_SEGMENTED, SORT_ONESWEEP = 0, 1
RASTER_FP32, RASTER_FP16 = 0, 1
SH_FLOAT32, SH_PACKED32 = 0, 1
TIMER_NAMES = ("project", "scan", "fill", "sort", "batch", "raster", "merge")

# every symbol include/higs.h declares
EXPORTS = ("higs_default_params", "higs_ctx_create", "higs_ctx_destroy", "higs_project",
           "higs_bin_sort", "higs_batch", "higs_raster", "higs_render", "higs_get_counts",
           "higs_set_debug", "higs_debug_copy", "higs_set_timing", "higs_get_timers",
           "higs_error_string", "higs_raster_backward", "higs_ctx_footprint",
           "higs_server_create", "higs_server_destroy", "higs_server_add_scene", "higs_server_submit",
           "higs_server_poll", "higs_server_get_stats", "higs_render_noalloc", "higs_sh_packed_bytes",
           "higs_sh_compress", "higs_render_views", "higs_server_tune", "higs_server_set_class")


class HigsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {error_string(code)} ({code})")


class Params(ctypes.Structure):
    _fields_ = [("tile_px", ctypes.c_int32), ("mt_tiles_x", ctypes.c_int32),
                ("mt_tiles_y", ctypes.c_int32), ("batch_cap", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("alpha_max", ctypes.c_float),
                ("t_eps", ctypes.c_float), ("near_z", ctypes.c_float),
                ("dilation", ctypes.c_float), ("sort_mode", ctypes.c_int32),
                ("raster_precision", ctypes.c_int32), ("sh_format", ctypes.c_int32),
                ("max_views", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("raster_chain", ctypes.c_int32), ("fuse_merge", ctypes.c_int32)]


class CameraC(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12), ("background", ctypes.c_float * 3)]


class Counts(ctypes.Structure):
    _fields_ = [("n_gaussians", ctypes.c_int64), ("n_visible", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("overflow", ctypes.c_uint32), ("sort_passes", ctypes.c_int32),
                ("n_evaluations", ctypes.c_int64), ("sort_pair_bytes", ctypes.c_int32),
                ("graphs", ctypes.c_int32)]


MAX_CLASSES = 4
MAX_VIEWS = 64


class ViewC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("camera", CameraC), ("image", ctypes.c_void_p), ("T_out", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("width", ctypes.c_int32 * MAX_CLASSES),
                ("height", ctypes.c_int32 * MAX_CLASSES), ("max_pairs", ctypes.c_int64 * MAX_CLASSES),
                ("max_gaussians", ctypes.c_int64), ("hbm_budget", ctypes.c_int64),
                ("max_in_flight", ctypes.c_int32), ("views_per_frame", ctypes.c_int32 * MAX_CLASSES),
                ("use_graphs", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_int64), ("gpu_ms", ctypes.c_float),
                ("overflow", ctypes.c_uint32), ("cls", ctypes.c_int32), ("views", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("in_flight", ctypes.c_int32), ("contexts", ctypes.c_int32),
                ("bytes", ctypes.c_int64), ("completed", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("frames", ctypes.c_int64), ("views_per_frame", ctypes.c_int32 * MAX_CLASSES),
                ("batch_cap", ctypes.c_int32 * MAX_CLASSES)]


TUNE_MAX_TRIALS = 16


class TuneReport(ctypes.Structure):
    _fields_ = [("views_per_frame", ctypes.c_int32), ("batch_cap", ctypes.c_int32),
                ("n_trials", ctypes.c_int32), ("trial_views", ctypes.c_int32 * TUNE_MAX_TRIALS),
                ("trial_batch_cap", ctypes.c_int32 * TUNE_MAX_TRIALS),
                ("trial_fps", ctypes.c_float * TUNE_MAX_TRIALS)]


_lib = None


def lib():
    """Loads libhigs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhigs is not built ({LIB_PATH} missing): run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "higs_default_params": (None, [P]),
            "higs_ctx_create": (ctypes.c_int, [ctypes.c_int, P, i64, i64, i64, i32, i32, P]),
            "higs_ctx_destroy": (ctypes.c_int, [P]),
            "higs_project": (ctypes.c_int, [P, i64, P, P, P, P, P, P, P]),
            "higs_bin_sort": (ctypes.c_int, [P, P]),
            "higs_batch": (ctypes.c_int, [P, P]),
            "higs_raster": (ctypes.c_int, [P, P, P, P]),
            "higs_render": (ctypes.c_int, [P, i64, P, P, P, P, P, P, P, P, P]),
            "higs_get_counts": (ctypes.c_int, [P, P]),
            "higs_set_debug": (ctypes.c_int, [P, ctypes.c_int]),
            "higs_debug_copy": (ctypes.c_int, [P, ctypes.c_int, P, ctypes.c_size_t]),
            "higs_set_timing": (ctypes.c_int, [P, ctypes.c_int]),
            "higs_get_timers": (ctypes.c_int, [P, P]),
            "higs_error_string": (ctypes.c_char_p, [ctypes.c_int]),
            "higs_raster_backward": (ctypes.c_int, [P, P, P, P, P, P, P, P, P]),
            "higs_ctx_footprint": (i64, [P, i64, i64, i64, i32, i32]),
            "higs_server_create": (ctypes.c_int, [ctypes.c_int, P, P, P]),
            "higs_server_destroy": (ctypes.c_int, [P]),
            "higs_server_add_scene": (ctypes.c_int, [P, i32, i64, P, P, P, P, P, P]),
            "higs_server_submit": (ctypes.c_int, [P, i64, i32, i32, P, P, P]),
            "higs_server_tune": (ctypes.c_int, [P, i32, i32, i32, P, i32, i32, P]),
            "higs_server_set_class": (ctypes.c_int, [P, i32, i32, i32]),
            "higs_server_poll": (ctypes.c_int, [P, P, i32]),
            "higs_server_get_stats": (ctypes.c_int, [P, P]),
            "higs_render_noalloc": (ctypes.c_int, [i64, P, P, P, P, P, P, P, P, P]),
            "higs_sh_packed_bytes": (i64, [i64]),
            "higs_sh_compress": (ctypes.c_int, [i64, P, P, P, P]),
            "higs_render_views": (ctypes.c_int, [P, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().higs_error_string(int(code)).decode()


def _check(code: int, what: str):
    if code != OK:
        raise HigsError(code, what)


def default_params(**overrides) -> Params:
    p = Params()
    lib().higs_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def camera_c(cam) -> CameraC:
    """From any object with width, height, fx, fy, cx, cy, world_to_cam [3,4], background."""
    c = CameraC()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w = np.asarray(cam.world_to_cam, dtype=np.float32).reshape(-1)
    for k in range(12):
        c.world_to_cam[k] = float(w[k])
    bg = getattr(cam, "background", (0.0, 0.0, 0.0))
    for k in range(3):
        c.background[k] = float(bg[k])
    return c


def _ptr(t) -> int:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or t.dtype.itemsize != 4:
        raise ValueError("expected a contiguous 4-byte CUDA/HIP tensor")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


_dep_stream = _stream


class CapacityError(HigsError):
    """A frame needed more pairs or batches than its context holds (the
    library stops such a frame on the device: NaN image, no gradients)."""

    def __init__(self, counts):
        self.counts = counts
        super().__init__(E_CAPACITY, f"frame overflow (bits {counts.overflow:#x}: {counts.n_pairs} pairs, "
                                     f"{counts.n_batches} batches)")


class Context:
    """A libhigs context: device workspace sized for the given capacities."""

    def __init__(self, max_gaussians: int, max_width: int, max_height: int, max_pairs: int = None,
                 max_batches: int = None, device: int = 0, **params):
        self.params = default_params(**params)
        if max_pairs is None:
            max_pairs = max(4 * max_gaussians, 1 << 16)
        if max_batches is None:
            max_batches = self._batches_for(max_pairs, max_width, max_height)
        self.max_gaussians, self.max_pairs, self.max_batches = int(max_gaussians), int(max_pairs), int(max_batches)
        self.max_width, self.max_height = int(max_width), int(max_height)
        self.device = device
        self._h = None
        self._create()
        self.n = 0
        self.n_mt = 0
        self.frame_id = 0  # advances with every projected frame
        self.debug_flags = 0
        self.grown = 0  # times render_checked grew the context

    def _batches_for(self, max_pairs, max_width, max_height):
        n_mt = ((max_width + 63) // 64) * ((max_height + 31) // 32) * max(1, self.params.max_views)
        return max_pairs // max(1, self.params.batch_cap) + n_mt + 16

    def _create(self):
        h = ctypes.c_void_p()
        _check(lib().higs_ctx_create(self.device, ctypes.byref(self.params), self.max_gaussians, self.max_pairs,
                                     self.max_batches, self.max_width, self.max_height, ctypes.byref(h)),
               "higs_ctx_create")
        self._h = h

    def grow(self, max_pairs: int = None, max_batches: int = None):
        """Re-creates the device workspace with larger pair / batch
        capacities (same gaussians, image size and parameters); the last
        frame's intermediates are lost."""
        mp = max(self.max_pairs, int(max_pairs or 0))
        mb = max(self.max_batches, int(max_batches or 0), self._batches_for(mp, self.max_width, self.max_height))
        self.close()
        self.max_pairs, self.max_batches = mp, mb
        self._create()
        if self.debug_flags:
            self.set_debug(self.debug_flags)
        self.grown += 1

    def close(self):
        if getattr(self, "_h", None):
            lib().higs_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stages ----------------------------------------------------------------
    def project(self, means, scales, quats, opacities, sh, cam, stream=None):
        n = int(means.shape[0])
        self.frame_id += 1
        self._cam = camera_c(cam)
        self.n = n
        self.n_mt = ((cam.width + 63) // 64) * ((cam.height + 31) // 32)
        _check(lib().higs_project(self._h, n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacities),
                                  _ptr(sh), ctypes.byref(self._cam), _stream(stream)), "higs_project")

    def bin_sort(self, stream=None):
        _check(lib().higs_bin_sort(self._h, _stream(stream)), "higs_bin_sort")

    def batch(self, stream=None):
        _check(lib().higs_batch(self._h, _stream(stream)), "higs_batch")

    def raster(self, image, T=None, stream=None):
        _check(lib().higs_raster(self._h, _ptr(image), _ptr(T), _stream(stream)), "higs_raster")

    def render(self, means, scales, quats, opacities, sh, cam, image, T=None, stream=None):
        n = int(means.shape[0])
        self.frame_id += 1
        self._cam = camera_c(cam)
        self.n = n
        self.n_mt = ((cam.width + 63) // 64) * ((cam.height + 31) // 32)
        _check(lib().higs_render(self._h, n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacities),
                                 _ptr(sh), ctypes.byref(self._cam), _ptr(image), _ptr(T), _stream(stream)),
               "higs_render")

    def render_checked(self, means, scales, quats, opacities, sh, cam, image, T=None, stream=None,
                       grow: bool = True, tries: int = 4) -> "Counts":
        """render() followed by a read of the frame's counts (synchronises).
        On a capacity overflow the context grows to the sizes the frame asked
        for (with 25% headroom) and renders again (grow=True), or raises
        CapacityError (grow=False)."""
        for _ in range(tries):
            self.render(means, scales, quats, opacities, sh, cam, image, T, stream)
            c = self.counts()
            if not c.overflow:
                return c
            if not grow or c.overflow & ~(OVF_PAIRS | OVF_BATCHES):
                raise CapacityError(c)
            want_p = int(c.n_pairs * 1.25) + 1024 if c.overflow & OVF_PAIRS else self.max_pairs
            want_b = int(c.n_batches * 1.25) + 64 if c.overflow & OVF_BATCHES else 0
            self.grow(want_p, want_b)
        raise CapacityError(c)

    def render_views(self, views, stream=None):
        """higs_render_views: views = [(tensors (means, scales, quats, opacities,
        sh), camera, image [H,W,3], T [H,W] or None), ...], all cameras of one
        size; one launch per kernel for all of them."""
        arr = (ViewC * len(views))()
        for k, (tens, cam, image, T) in enumerate(views):
            means, scales, quats, opac, sh = tens
            v = arr[k]
            v.n = int(means.shape[0])
            v.means, v.scales, v.quats = _ptr(means), _ptr(scales), _ptr(quats)
            v.opacities, v.sh = _ptr(opac), _ptr(sh)
            v.camera = camera_c(cam)
            v.image, v.T_out = _ptr(image), _ptr(T)
        if views:
            self.frame_id += 1
            cam0 = views[0][1]
            self.n = int(views[0][0][0].shape[0])
            self.n_mt = ((cam0.width + 63) // 64) * ((cam0.height + 31) // 32) * len(views)
        _check(lib().higs_render_views(self._h, len(views), arr, _stream(stream)), "higs_render_views")

    def raster_backward(self, d_image, d_T, d_means, d_scales, d_quats, d_opacities, d_sh, stream=None):
        """Adjoint of the last frame (higs_raster_backward): writes the gradient
        tensors d_means [n,3], d_scales [n,3], d_quats [n,4], d_opacities [n],
        d_sh [n,(deg+1)^2,3] from d_image [H,W,3] and d_T [H,W] (or None)."""
        _check(lib().higs_raster_backward(self._h, _ptr(d_image), _ptr(d_T), _ptr(d_means), _ptr(d_scales),
                                          _ptr(d_quats), _ptr(d_opacities), _ptr(d_sh), _stream(stream)),
               "higs_raster_backward")

    # ---- host read-back ----------------------------------------------------------
    def counts(self) -> Counts:
        c = Counts()
        _check(lib().higs_get_counts(self._h, ctypes.byref(c)), "higs_get_counts")
        return c

    def set_debug(self, flags: int):
        _check(lib().higs_set_debug(self._h, flags), "higs_set_debug")
        self.debug_flags = int(flags)

    def set_timing(self, n_frames: int):
        """Keep per-kernel HIP-event times of the last n_frames frames (0: off)."""
        _check(lib().higs_set_timing(self._h, int(n_frames)), "higs_set_timing")

    def timers(self) -> dict:
        """Mean per-kernel milliseconds over the recorded frames (synchronises)."""
        ms = (ctypes.c_float * len(TIMER_NAMES))()
        _check(lib().higs_get_timers(self._h, ms), "higs_get_timers")
        return dict(zip(TIMER_NAMES, list(ms)))

    def _copy(self, which: int, arr: np.ndarray) -> np.ndarray:
        if arr.nbytes:
            _check(lib().higs_debug_copy(self._h, which, arr.ctypes.data_as(ctypes.c_void_p), arr.nbytes),
                   "higs_debug_copy")
        return arr

    def proj_fields(self) -> dict:
        raw = self._copy(DBG_PROJ, np.zeros((8, self.n), np.float32))
        names = ("mx", "my", "a", "b", "c", "tau")
        out = {k: raw[i] for i, k in enumerate(names)}
        out["key"] = raw[6].view(np.uint32)
        out["count"] = raw[7].view(np.uint32)
        return out

    def records(self) -> np.ndarray:
        return self._copy(DBG_RECORDS, np.zeros((self.n, 12), np.float32))

    def _pairs(self, which):
        c = self.counts()
        np_ = min(int(c.n_pairs), self.max_pairs)
        raw = self._copy(which, np.zeros(np_ * 12, np.uint8))
        keys = raw[:np_ * 8].view(np.uint64)
        vals = raw[np_ * 8:].view(np.uint32)
        return keys, vals

    def pairs(self):
        return self._pairs(DBG_PAIRS)

    def sorted_pairs(self):
        return self._pairs(DBG_SORTED)

    def mt_offsets(self) -> np.ndarray:
        return self._copy(DBG_MT_OFFSETS, np.zeros(self.n_mt + 1, np.uint32))

    def batches(self) -> np.ndarray:
        c = self.counts()
        nb = min(int(c.n_batches), self.max_batches)
        return self._copy(DBG_BATCHES, np.zeros((nb, 3), np.uint32))

    def active(self) -> np.ndarray:
        c = self.counts()
        nb = min(int(c.n_batches), self.max_batches)
        return self._copy(DBG_ACTIVE, np.zeros(nb, np.uint32))

    def partials(self, first: int = 0, count: int = None) -> np.ndarray:
        c = self.counts()
        nb = min(int(c.n_batches), self.max_batches)
        count = nb if count is None else min(count, nb)
        if first != 0:
            raise ValueError("partials are read from the first batch")
        return self._copy(DBG_PARTIALS, np.zeros((count, 32, 64, 4), np.float32))


def ctx_footprint(max_gaussians: int, max_pairs: int, max_batches: int, max_width: int, max_height: int,
                  **params) -> int:
    """Device bytes a context with these capacities allocates (host-only)."""
    p = default_params(**params)
    return int(lib().higs_ctx_footprint(ctypes.byref(p), int(max_gaussians), int(max_pairs), int(max_batches),
                                        int(max_width), int(max_height)))


class Server:
    """higs_server: resident scenes, continuous batching of frame requests over
    contexts (one stream each) within an HBM budget.  classes: [(W, H,
    max_pairs), ...]."""

    def __init__(self, classes, max_gaussians: int, hbm_budget: int, max_in_flight: int = 16, device: int = 0,
                 views_per_frame=None, use_graphs: bool = False, **params):
        cfg = ServerConfig()
        cfg.n_classes = len(classes)
        for k, (w, h, mp) in enumerate(classes):
            cfg.width[k], cfg.height[k], cfg.max_pairs[k] = int(w), int(h), int(mp)
            cfg.views_per_frame[k] = int(views_per_frame[k]) if views_per_frame else 1
        cfg.max_gaussians = int(max_gaussians)
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_in_flight = int(max_in_flight)
        cfg.use_graphs = 1 if use_graphs else 0
        self.params = default_params(**params)
        h = ctypes.c_void_p()
        _check(lib().higs_server_create(device, ctypes.byref(self.params), ctypes.byref(cfg), ctypes.byref(h)),
               "higs_server_create")
        self._h = h
        self._keep = []          # scene tensors stay referenced while the server lives
        self._done = (Completion * 256)()

    def close(self):
        if getattr(self, "_h", None):
            lib().higs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_scene(self, scene_id: int, tensors, stream=None):
        """Registers a resident scene; frames of it wait for the work enqueued
        so far on `stream` (default: torch's current stream)."""
        means, scales, quats, opac, sh = tensors
        self._keep.append(tensors)
        _check(lib().higs_server_add_scene(self._h, int(scene_id), int(means.shape[0]), _ptr(means), _ptr(scales),
                                           _ptr(quats), _ptr(opac), _ptr(sh), _dep_stream(stream)),
               "higs_server_add_scene")

    def submit(self, request_id: int, scene_id: int, cls: int, cam, image, stream=None):
        """Queues a request; its frame waits for the work enqueued so far on
        `stream` (default: torch's current stream), e.g. what last used image."""
        c = camera_c(cam)
        _check(lib().higs_server_submit(self._h, int(request_id), int(scene_id), int(cls), ctypes.byref(c),
                                        _ptr(image), _dep_stream(stream)), "higs_server_submit")

    def poll(self):
        """Retires finished frames and admits queued ones; returns a list of
        (request_id, gpu_ms, overflow, cls)."""
        n = lib().higs_server_poll(self._h, self._done, len(self._done))
        if n < 0:
            raise HigsError(n, "higs_server_poll")
        return [(d.request_id, d.gpu_ms, d.overflow, d.cls) for d in self._done[:n]]

    def tune(self, cls: int, scene_id: int, cams, frames: int = 64, allow_batch_cap: bool = False) -> TuneReport:
        """higs_server_tune: measures views per frame (and B_r) for class cls
        and keeps the fastest."""
        arr = (CameraC * len(cams))(*[camera_c(c) for c in cams])
        rep = TuneReport()
        _check(lib().higs_server_tune(self._h, int(cls), int(scene_id), len(cams), arr, int(frames),
                                      1 if allow_batch_cap else 0, ctypes.byref(rep)), "higs_server_tune")
        return rep

    def set_class(self, cls: int, views_per_frame: int, batch_cap: int = 1024):
        _check(lib().higs_server_set_class(self._h, int(cls), int(views_per_frame), int(batch_cap)),
               "higs_server_set_class")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().higs_server_get_stats(self._h, ctypes.byref(st)), "higs_server_get_stats")
        return st


def scene_tensors(scene, device="cuda"):
    """Scene arrays (numpy float32) as contiguous device tensors."""
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in scene.arrays())


def render(ctx: Context, tensors, cam, with_T: bool = True, stream=None, check: bool = True,
           grow: bool = True):
    """Renders one frame; returns (image [H,W,3], T [H,W] or None) device tensors.
    check=True reads the frame's counts (a synchronisation) and, on a capacity
    overflow, grows the context and renders again (grow=True) or raises
    CapacityError (grow=False); check=False only enqueues the frame (an
    overflowed frame then leaves a NaN image)."""
    import torch
    dev = tensors[0].device
    image = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=dev)
    T = torch.empty((cam.height, cam.width), dtype=torch.float32, device=dev) if with_T else None
    if check:
        ctx.render_checked(*tensors, cam, image, T, stream, grow=grow)
    else:
        ctx.render(*tensors, cam, image, T, stream)
    return image, T


def sh_compress(sh, opacities, stream=None):
    """The 32-byte packed SH of sh [n, 16, 3] (higs_sh_compress): an int32
    device tensor of higs_sh_packed_bytes(n) bytes (a header of 48 float32
    scales, then 8 words per gaussian); pass it as the scene's SH to a
    context with sh_format=SH_PACKED32."""
    import torch
    n = int(sh.shape[0])
    nbytes = int(lib().higs_sh_packed_bytes(n))
    out = torch.empty(nbytes // 4, dtype=torch.int32, device=sh.device)
    _check(lib().higs_sh_compress(n, _ptr(sh.contiguous()), _ptr(opacities.contiguous()), out.data_ptr(),
                                  _stream(stream)), "higs_sh_compress")
    return out


def render_noalloc(tensors, cam, image, T=None, stream=None):
    """higs_render_noalloc: one frame with the library's static scratch array
    (no device allocation); the image (and T) are written on `stream`."""
    means, scales, quats, opac, sh = tensors
    c = camera_c(cam)
    _check(lib().higs_render_noalloc(int(means.shape[0]), _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac),
                                     _ptr(sh), ctypes.byref(c), _ptr(image), _ptr(T), _stream(stream)),
           "higs_render_noalloc")


def _render_function():
    import torch

    class RenderFunction(torch.autograd.Function):
        """Differentiable frame: forward = higs_render, backward =
        higs_raster_backward.  The context must not render another frame
        between the two (checked)."""

        @staticmethod
        def forward(fctx, means, scales, quats, opacities, sh, hctx, cam):
            tens = tuple(t.contiguous() for t in (means, scales, quats, opacities, sh))
            # checked: a frame that overflowed its context is rendered again
            # in a grown one, so the backward never sees a stopped frame
            image, T = render(hctx, tens, cam, check=True)
            fctx.hctx = hctx
            fctx.frame_id = hctx.frame_id
            fctx.save_for_backward(*tens)
            return image, T

        @staticmethod
        def backward(fctx, d_image, d_T):
            hctx = fctx.hctx
            if hctx.frame_id != fctx.frame_id:
                raise RuntimeError("the context rendered another frame after this one: "
                                   "its backward needs the frame's intermediates")
            tens = fctx.saved_tensors
            outs = [torch.empty_like(t) for t in tens]
            if d_image is None:
                cam = hctx._cam
                d_image = torch.zeros((cam.height, cam.width, 3), device=tens[0].device)
            d_image = d_image.contiguous().float()
            d_T = None if d_T is None else d_T.contiguous().float()
            hctx.raster_backward(d_image, d_T, *outs)
            return (*outs, None, None)

    return RenderFunction


_RENDER_FN = None


def render_differentiable(hctx: Context, means, scales, quats, opacities, sh, cam):
    """(image [H,W,3], T [H,W]) with gradients to every scene tensor (scales
    linear, opacities in [0, 1], as higs_project takes them).  A context made
    with fuse_merge=0 keeps the partials the adjoint reads; with the default
    the adjoint first rasterises the frame again."""
    global _RENDER_FN
    if _RENDER_FN is None:
        _RENDER_FN = _render_function()
    return _RENDER_FN.apply(means, scales, quats, opacities, sh, hctx, cam)


def render_trainable(hctx: Context, means, log_scales, quats, opacity_logits, sh, cam):
    """The training parameterisation: scales = exp(log_scales), opacities =
    sigmoid(opacity_logits), applied in torch; gradients reach the raw
    parameters through torch's own chain rule."""
    import torch
    return render_differentiable(hctx, means, torch.exp(log_scales), quats, torch.sigmoid(opacity_logits),
                                 sh, cam)
