"""Python front of the plain FP64 CPU oracle (higs_oracle.c, and its adjoint
in higs_oracle_grad.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke entry point and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  The
oracle and the GPU path share no code; only the seeded input generators
(paper_2606_00352_amd.scenes) serve both.

`frame(scene, cam)` runs the whole forward path the paper describes
(projection, macro-tile binning, depth sort, batch split, rasterisation and
the post-blend merge of Eq. 1) and returns every intermediate.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("higs_oracle.c", "higs_oracle_grad.c", "higs_oracle.h")]
# HIGS_ORACLE_SANITIZE=1: a separate build under AddressSanitizer and
# UndefinedBehaviorSanitizer (for a process that preloads their runtimes)
_SANITIZE = os.environ.get("HIGS_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")

TILE = 8
MT_W, MT_H = 64, 32
MT_TILES = 32
AMB_ALPHA, AMB_T = 1, 2

# columns of the per-gaussian double record
G_TZ, G_MX, G_MY, G_A, G_B, G_C, G_TAU, G_L0, G_L1, G_L2, G_OP, G_R, G_G, G_BL = range(14)
G_NCOL = 14
# columns of the per-gaussian gradient with respect to the raster record
D_MX, D_MY, D_L0, D_L1, D_L2, D_OP, D_R, D_G, D_BL = range(9)
D_NCOL = 9


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (double precision, no contraction)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        san = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"] if _SANITIZE else ["-O2"])
        cmd = ["gcc"] + san + ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp] + [s for s in _SRCS if s.endswith(".c")] + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12), ("background", ctypes.c_float * 3)]


class _Params(ctypes.Structure):
    _fields_ = [("near_z", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_eps", ctypes.c_double),
                ("dilation", ctypes.c_double), ("batch_cap", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32)]


@dataclasses.dataclass
class Params:
    near_z: float = 0.2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_eps: float = 1e-4
    dilation: float = 0.3
    batch_cap: int = 1024
    sh_degree: int = 3

    def c(self) -> _Params:
        # near_z, alpha_max, t_eps and dilation cross the library interface as
        # float32, as the camera does: the oracle takes the same float values
        f = lambda v: float(np.float32(v))
        return _Params(f(self.near_z), self.alpha_min, f(self.alpha_max), f(self.t_eps), f(self.dilation),
                       self.batch_cap, self.sh_degree)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        sig = {
            "oc_project": (i64, [i64, P, P, P, P, P, P, P, P, P]),
            "oc_mt_list": (i32, [P, i32, i32, P, i32]),
            "oc_bin_count": (i64, [i64, P, P, i32, i32, P]),
            "oc_bin_fill": (None, [i64, P, P, i32, i32, P, P, P, P]),
            "oc_sort_pairs": (None, [i64, P, P, P]),
            "oc_batches": (i64, [i64, P, i32, i32, P, P, i64]),
            "oc_render_untiled": (None, [i64, P, P, P, P, P, i64, P, P, P]),
            "oc_render_tiled": (None, [P, P, P, P, i64, P, P, P, i64, P, P, P]),
            "oc_batch_partials": (None, [P, P, P, P, P, P, P]),
            "oc_sh_basis": (None, [P, ctypes.c_int, P]),
            "oc_depth_key": (ctypes.c_uint32, [ctypes.c_double]),
            "oc_num_threads": (ctypes.c_int, []),
            "oc_sh_basis_grad": (None, [P, ctypes.c_int, P]),
            "oc_project_grad": (None, [i64, P, P, P, P, P, P, P, P, P, P, P, P, P]),
            "oc_render_tiled_grad": (None, [P, P, P, i64, P, P, P, P, P]),
            "oc_render_tiled_signature": (ctypes.c_uint64, [P, P, P, i64, P, P]),
            "oc_render_tiled_ambiguous": (i64, [i64, P, P, P, i64, P, P, P]),
            "oc_alpha_flag_band": (None, [i64, P, P, P, P, P, P, P]),
            "oc_count_evals": (None, [P, P, P, i64, P, P, P]),
            "oc_set_threads": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cam(cam) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w = np.asarray(cam.world_to_cam, dtype=np.float32).reshape(-1)
    for k in range(12):
        c.world_to_cam[k] = float(w[k])
    for k in range(3):
        c.background[k] = float(cam.background[k])
    return c


def num_threads() -> int:
    return int(lib().oc_num_threads())


def set_threads(n: int):
    """Threads of the oracle's parallel loops from now on."""
    lib().oc_set_threads(int(n))


def n_macro_tiles(width: int, height: int):
    return (width + MT_W - 1) // MT_W, (height + MT_H - 1) // MT_H


def project(scene, cam, params: Params = None):
    """Returns (valid int8 [N], geo float64 [N, 14])."""
    params = params or Params()
    means, scales, quats, opac, sh = (np.ascontiguousarray(a, dtype=np.float32) for a in scene.arrays())
    n = means.shape[0]
    ncoef = (params.sh_degree + 1) ** 2
    sh = np.ascontiguousarray(sh[:, :ncoef, :])
    valid = np.zeros(n, dtype=np.int8)
    geo = np.zeros((n, G_NCOL), dtype=np.float64)
    c, p = _cam(cam), params.c()
    lib().oc_project(n, _p(means), _p(scales), _p(quats), _p(opac), _p(sh),
                     ctypes.byref(c), ctypes.byref(p), _p(valid), _p(geo))
    return valid, geo


def stored_fields(geo: np.ndarray) -> np.ndarray:
    """float32 [N, 6] = (mx, my, a, b, c, tau) rounded to nearest float."""
    return np.ascontiguousarray(geo[:, [G_MX, G_MY, G_A, G_B, G_C, G_TAU]].astype(np.float32))


def mt_list(fields6, width: int, height: int) -> np.ndarray:
    f = np.ascontiguousarray(np.asarray(fields6, dtype=np.float32).reshape(6))
    n = lib().oc_mt_list(_p(f), width, height, None, 0)
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib().oc_mt_list(_p(f), width, height, _p(out), n)
    return out[:n]


def depth_key(tz: float) -> int:
    return int(lib().oc_depth_key(float(tz)))


def sh_basis(direction, degree: int = 3) -> np.ndarray:
    d = np.ascontiguousarray(np.asarray(direction, dtype=np.float64).reshape(3))
    out = np.zeros(16, dtype=np.float64)
    lib().oc_sh_basis(_p(d), degree, _p(out))
    return out


def bin_pairs(valid, geo, width: int, height: int):
    """Pairs in emission order: gaussian id ascending, macro-tile ascending
    within a gaussian.  Returns (counts, mt, key, gid)."""
    n = valid.shape[0]
    counts = np.zeros(n, dtype=np.int32)
    total = lib().oc_bin_count(n, _p(valid), _p(geo), width, height, _p(counts))
    offsets = np.zeros(n, dtype=np.int64)
    if n > 1:
        np.cumsum(counts[:-1], out=offsets[1:])
    mt = np.zeros(max(total, 1), dtype=np.int32)
    key = np.zeros(max(total, 1), dtype=np.uint32)
    gid = np.zeros(max(total, 1), dtype=np.int32)
    lib().oc_bin_fill(n, _p(valid), _p(geo), width, height, _p(offsets), _p(mt), _p(key), _p(gid))
    return counts, mt[:total], key[:total], gid[:total]


def sort_pairs(mt, key, gid):
    mt, key, gid = (np.array(a, copy=True) for a in (mt, key, gid))
    lib().oc_sort_pairs(mt.shape[0], _p(mt), _p(key), _p(gid))
    return mt, key, gid


def batches(sorted_mt, n_mt: int, cap: int = 1024):
    """Returns (mt_off int64 [n_mt + 1], batch table int32 [nb, 3])."""
    sorted_mt = np.ascontiguousarray(sorted_mt, dtype=np.int32)
    mt_off = np.zeros(n_mt + 1, dtype=np.int64)
    nb = lib().oc_batches(sorted_mt.shape[0], _p(sorted_mt), n_mt, cap, _p(mt_off), None, 0)
    tab = np.zeros((max(nb, 1), 3), dtype=np.int32)
    lib().oc_batches(sorted_mt.shape[0], _p(sorted_mt), n_mt, cap, _p(mt_off), _p(tab), nb)
    return mt_off, tab[:nb]


def alpha_flag_band(geo, gid, px, py):
    """For evaluations k of gaussian gid[k] at pixel centre (px[k], py[k]):
    (q, band, bound) -- the double q, the half-width of the band around tau
    inside which the alpha decision is flagged ambiguous, and the float32
    bound (oc_f32_q_bound) the band is built from."""
    gid = np.ascontiguousarray(gid, dtype=np.int64)
    px = np.ascontiguousarray(px, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    n = gid.shape[0]
    q, band, bound = (np.zeros(n, dtype=np.float64) for _ in range(3))
    lib().oc_alpha_flag_band(n, _p(np.ascontiguousarray(geo)), _p(gid), _p(px), _p(py), _p(q), _p(band),
                             _p(bound))
    return q, band, bound


def count_evals(geo, sorted_gid, tab, cam, params: Params = None):
    """(all, read): pixel-gaussian evaluations of the batched form -- over
    every (unit, tile), and over the (unit, tile) pairs whose partial the
    merge reads (oc_count_evals)."""
    params = params or Params()
    out = np.zeros(2, dtype=np.int64)
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    lib().oc_count_evals(_p(np.ascontiguousarray(geo)), _p(sorted_gid), _p(tab), tab.shape[0], ctypes.byref(c),
                         ctypes.byref(p), _p(out))
    return int(out[0]), int(out[1])


def _pix(pixels):
    if pixels is None:
        return None, 0
    px = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32).reshape(-1, 2))
    return px, px.shape[0]


def render_untiled(valid, geo, cam, params: Params = None, pixels=None):
    """Per-pixel brute force.  Whole image -> (image [H,W,3], T [H,W], amb [H,W]);
    with `pixels` ([K,2] of (x, y)) -> ([K,3], [K], [K])."""
    params = params or Params()
    px, npix = _pix(pixels)
    total = npix if px is not None else cam.width * cam.height
    img = np.zeros((total, 3), dtype=np.float64)
    T = np.zeros(total, dtype=np.float64)
    amb = np.zeros(total, dtype=np.uint8)
    c, p = _cam(cam), params.c()
    lib().oc_render_untiled(valid.shape[0], _p(valid), _p(geo), ctypes.byref(c), ctypes.byref(p),
                            _p(px) if px is not None else None, npix, _p(img), _p(T), _p(amb))
    if px is None:
        return img.reshape(cam.height, cam.width, 3), T.reshape(cam.height, cam.width), amb.reshape(cam.height, cam.width)
    return img, T, amb


def render_tiled(geo, sorted_gid, mt_off, tab, cam, params: Params = None, pixels=None):
    params = params or Params()
    px, npix = _pix(pixels)
    total = npix if px is not None else cam.width * cam.height
    img = np.zeros((total, 3), dtype=np.float64)
    T = np.zeros(total, dtype=np.float64)
    amb = np.zeros(total, dtype=np.uint8)
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    lib().oc_render_tiled(_p(geo), _p(sorted_gid), _p(mt_off), _p(tab), tab.shape[0],
                          ctypes.byref(c), ctypes.byref(p),
                          _p(px) if px is not None else None, npix, _p(img), _p(T), _p(amb))
    if px is None:
        return img.reshape(cam.height, cam.width, 3), T.reshape(cam.height, cam.width), amb.reshape(cam.height, cam.width)
    return img, T, amb


def batch_partials(geo, sorted_gid, batch_row, cam, params: Params = None, with_amb: bool = False):
    """[32 tiles, 64 px, 4] partial (R, G, B, T) of one batch from (0, 1);
    with_amb: also the [32, 64] ambiguity flags of those evaluations."""
    params = params or Params()
    out = np.zeros((MT_TILES, 64, 4), dtype=np.float64)
    amb = np.zeros((MT_TILES, 64), dtype=np.uint8)
    row = np.ascontiguousarray(np.asarray(batch_row, dtype=np.int32).reshape(3))
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    lib().oc_batch_partials(_p(geo), _p(sorted_gid), _p(row), ctypes.byref(c), ctypes.byref(p), _p(out),
                            _p(amb))
    return (out, amb) if with_amb else out


@dataclasses.dataclass
class Frame:
    valid: np.ndarray
    geo: np.ndarray
    counts: np.ndarray
    pairs_mt: np.ndarray       # emission order
    pairs_key: np.ndarray
    pairs_gid: np.ndarray
    sorted_mt: np.ndarray
    sorted_key: np.ndarray
    sorted_gid: np.ndarray
    mt_off: np.ndarray
    batch_tab: np.ndarray
    image: np.ndarray = None   # tiled result, when rendered
    T: np.ndarray = None
    amb: np.ndarray = None


def frame(scene, cam, params: Params = None, render: bool = True, pixels=None) -> Frame:
    """Runs every stage of the forward path; `render` also composites the
    image with the batched (tiled) form."""
    params = params or Params()
    valid, geo = project(scene, cam, params)
    counts, mt, key, gid = bin_pairs(valid, geo, cam.width, cam.height)
    smt, skey, sgid = sort_pairs(mt, key, gid)
    nmx, nmy = n_macro_tiles(cam.width, cam.height)
    mt_off, tab = batches(smt, nmx * nmy, params.batch_cap)
    fr = Frame(valid, geo, counts, mt, key, gid, smt, skey, sgid, mt_off, tab)
    if render:
        fr.image, fr.T, fr.amb = render_tiled(geo, sgid, mt_off, tab, cam, params, pixels)
    return fr


# ------------------------------------------------------------------ adjoint --
def sh_basis_grad(direction, degree: int = 3) -> np.ndarray:
    """[16, 3]: d Y_k / d(x, y, z), components taken as independent."""
    d = np.ascontiguousarray(np.asarray(direction, dtype=np.float64).reshape(3))
    out = np.zeros((16, 3), dtype=np.float64)
    lib().oc_sh_basis_grad(_p(d), degree, _p(out))
    return out


def render_grad(geo, sorted_gid, tab, cam, dimg, dT=None, params: Params = None) -> np.ndarray:
    """dL/d(raster record) [N, 9] (columns D_*) of the batched render, from
    dL/dimage [H, W, 3] and dL/dT [H, W] (None: zero)."""
    params = params or Params()
    dgeo = np.zeros((geo.shape[0], D_NCOL), dtype=np.float64)
    dimg = np.ascontiguousarray(dimg, dtype=np.float64).reshape(cam.height, cam.width, 3)
    dT_ = None if dT is None else np.ascontiguousarray(dT, dtype=np.float64).reshape(cam.height, cam.width)
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    lib().oc_render_tiled_grad(_p(geo), _p(sorted_gid), _p(tab), tab.shape[0], ctypes.byref(c),
                               ctypes.byref(p), _p(dimg), None if dT_ is None else _p(dT_), _p(dgeo))
    return dgeo


def render_signature(geo, sorted_gid, tab, cam, params: Params = None) -> int:
    """Digest of every discrete decision of the batched render."""
    params = params or Params()
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    return int(lib().oc_render_tiled_signature(_p(geo), _p(sorted_gid), _p(tab), tab.shape[0],
                                               ctypes.byref(c), ctypes.byref(p)))


def ambiguous_gaussians(geo, sorted_gid, tab, cam, params: Params = None) -> np.ndarray:
    """uint8 [N]: 1 for gaussians with an evaluation whose alpha decision
    (against 1/255 or the alpha_max clamp) float32 may take the other way."""
    params = params or Params()
    gmask = np.zeros(geo.shape[0], dtype=np.uint8)
    c, p = _cam(cam), params.c()
    sorted_gid = np.ascontiguousarray(sorted_gid, dtype=np.int32)
    tab = np.ascontiguousarray(tab, dtype=np.int32)
    lib().oc_render_tiled_ambiguous(geo.shape[0], _p(geo), _p(sorted_gid), _p(tab), tab.shape[0],
                                    ctypes.byref(c), ctypes.byref(p), _p(gmask))
    return gmask


def project_grad(scene, cam, valid, dgeo, params: Params = None) -> dict:
    """Gradients of the scene inputs from dL/d(raster record)."""
    params = params or Params()
    means, scales, quats, opac, sh = (np.ascontiguousarray(a, dtype=np.float32) for a in scene.arrays())
    n = means.shape[0]
    ncoef = (params.sh_degree + 1) ** 2
    sh = np.ascontiguousarray(sh[:, :ncoef, :])
    out = {"means": np.zeros((n, 3)), "scales": np.zeros((n, 3)), "quats": np.zeros((n, 4)),
           "opacities": np.zeros(n), "sh": np.zeros((n, ncoef, 3))}
    c, p = _cam(cam), params.c()
    dgeo = np.ascontiguousarray(dgeo, dtype=np.float64)
    lib().oc_project_grad(n, _p(means), _p(scales), _p(quats), _p(sh), ctypes.byref(c), ctypes.byref(p),
                          _p(valid), _p(dgeo), _p(out["means"]), _p(out["scales"]), _p(out["quats"]),
                          _p(out["opacities"]), _p(out["sh"]))
    return out


def frame_grad(scene, cam, dimg, dT=None, params: Params = None, fr: Frame = None):
    """The adjoint of the whole forward path: returns (frame, dgeo, grads)."""
    params = params or Params()
    fr = fr or frame(scene, cam, params)
    dgeo = render_grad(fr.geo, fr.sorted_gid, fr.batch_tab, cam, dimg, dT, params)
    return fr, dgeo, project_grad(scene, cam, fr.valid, dgeo, params)
