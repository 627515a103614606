"""ctypes binding of the C rasterizer oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class _Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("pad_", C.c_int32),
                ("means", C.c_void_p), ("quats", C.c_void_p), ("log_scales", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("dmu", C.c_void_p),
                ("dq", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float),
                ("w2c", C.c_float * 12), ("cam_pos", C.c_float * 3), ("bg", C.c_float * 3)]


class _Grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("d_means", "d_quats", "d_log_scales", "d_opacity_logits",
                                          "d_sh", "d_dmu", "d_dq", "d_uv", "d_conic", "d_opacity",
                                          "d_rgb")]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        _lib.orc_spec_exp.restype = C.c_float
        _lib.orc_spec_exp.argtypes = [C.c_float]
        _lib.orc_sorted_pairs.restype = C.c_int64
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Pinned:
    """Keeps the float32 copies alive while the C call runs."""

    def __init__(self, g, dmu, dq):
        f = lambda a: None if a is None else np.ascontiguousarray(a, np.float32)
        self.arrs = [f(g.means), f(g.quats), f(g.log_scales), f(g.opacity_logits), f(g.sh), f(dmu), f(dq)]
        self.s = _Gaussians(g.n, g.sh_degree, 0, *[_ptr(a) for a in self.arrs])


def _cam(cam):
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy, c.near_z = cam.fx, cam.fy, cam.cx, cam.cy, cam.near
    for k, v in enumerate(np.asarray(cam.world_to_cam, np.float32).reshape(-1)):
        c.w2c[k] = float(v)
    for k in range(3):
        c.cam_pos[k] = float(cam.cam_pos[k])
        c.bg[k] = float(cam.bg[k])
    return c


def preprocess(g, cam, dmu=None, dq=None, tile: int = 16) -> dict:
    n = g.n
    out = dict(visible=np.zeros(n, np.uint8), key=np.zeros(n, np.uint32), box=np.zeros((n, 4), np.int32),
               rect=np.zeros((n, 4), np.int32), ntiles=np.zeros(n, np.int64), uv=np.zeros((n, 2)),
               conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)), depth=np.zeros(n))
    p = _Pinned(g, dmu, dq)
    c = _cam(cam)
    rc = lib().orc_preprocess(C.byref(p.s), C.byref(c), C.c_int(tile),
                              *[C.c_void_p(_ptr(out[k])) for k in ("visible", "key", "box", "rect", "ntiles",
                                                                   "uv", "conic", "opacity", "rgb", "depth")])
    assert rc == 0, rc
    return out


def pair_count(g, cam, dmu=None, dq=None, tile: int = 16) -> int:
    """Number of (tile, Gaussian) pairs, without building the list."""
    p = _Pinned(g, dmu, dq)
    c = _cam(cam)
    K = lib().orc_sorted_pairs(C.byref(p.s), C.byref(c), C.c_int(tile), None, None, C.c_int64(0), None)
    assert K >= 0, K
    return int(K)


def sorted_pairs(g, cam, dmu=None, dq=None, tile: int = 16):
    """(keys u64, vals u32, ranges (tiles, 2) u32) in (tile, depth bits, id) order."""
    p = _Pinned(g, dmu, dq)
    c = _cam(cam)
    tiles = ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    ranges = np.zeros((tiles, 2), np.uint32)
    K = lib().orc_sorted_pairs(C.byref(p.s), C.byref(c), C.c_int(tile), None, None, C.c_int64(0), None)
    assert K >= 0, K
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    K2 = lib().orc_sorted_pairs(C.byref(p.s), C.byref(c), C.c_int(tile), C.c_void_p(_ptr(keys)),
                                C.c_void_p(_ptr(vals)), C.c_int64(K), C.c_void_p(_ptr(ranges)))
    assert K2 == K
    return keys[:K], vals[:K], ranges


def render(g, cam, dmu=None, dq=None) -> dict:
    """Eq. 4 per pixel.  `ambiguous` bits: 1 the 0.99 clamp of alpha, 2 the
    transmittance cut-off, 4 a second cut-off decision, within single-
    precision reach of going the other way.  `image_alt` / `T_alt` are the
    pixel with the other outcome of the cut-off decision where bit 2 is set,
    and equal `image` / `T_final` elsewhere."""
    H, W = cam.height, cam.width
    out = dict(image=np.zeros((3, H, W)), T_final=np.zeros((H, W)), n_contrib=np.zeros((H, W), np.int32),
               ambiguous=np.zeros((H, W), np.uint8), image_alt=np.zeros((3, H, W)), T_alt=np.zeros((H, W)))
    p = _Pinned(g, dmu, dq)
    c = _cam(cam)
    rc = lib().orc_render(C.byref(p.s), C.byref(c), C.c_void_p(_ptr(out["image"])),
                          C.c_void_p(_ptr(out["T_final"])), C.c_void_p(_ptr(out["n_contrib"])),
                          C.c_void_p(_ptr(out["ambiguous"])), C.c_void_p(_ptr(out["image_alt"])),
                          C.c_void_p(_ptr(out["T_alt"])))
    assert rc == 0, rc
    return out


def image_error(img, ref: dict, T=None):
    """Distance of a rendered image (3 x H x W) and, if given, its final
    transmittance (H x W) from the oracle's render `ref`, per pixel, taking
    for each pixel whichever of the two outcomes of the cut-off decision
    (primary or alternative) fits both quantities better.  Returns
    (image error = max over channels (H x W), transmittance error (H x W) or
    None, mask of pixels that took the alternative, mask of pixels whose
    outcomes the two values do not cover)."""
    img = np.asarray(img, np.float64)
    d0 = np.abs(img - ref["image"]).max(axis=0)
    d1 = np.abs(img - ref["image_alt"]).max(axis=0)
    s0, s1 = d0, d1
    if T is not None:
        T = np.asarray(T, np.float64)
        t0, t1 = np.abs(T - ref["T_final"]), np.abs(T - ref["T_alt"])
        s0, s1 = np.maximum(d0, t0), np.maximum(d1, t1)
    use_alt = s1 < s0
    terr = None if T is None else np.where(use_alt, t1, t0)
    return np.where(use_alt, d1, d0), terr, use_alt, (ref["ambiguous"] & 4) != 0


def render_backward(g, cam, dl_dimg, dmu=None, dq=None) -> dict:
    """Gradients (float64) of <dl_dimg, image> with respect to every input."""
    n, K = g.n, (g.sh_degree + 1) ** 2
    shapes = dict(d_means=(n, 3), d_quats=(n, 4), d_log_scales=(n, 3), d_opacity_logits=(n,),
                  d_sh=(n, K, 3), d_dmu=(n, 3), d_dq=(n, 4), d_uv=(n, 2), d_conic=(n, 3),
                  d_opacity=(n,), d_rgb=(n, 3))
    out = {k: np.zeros(s) for k, s in shapes.items()}
    if dmu is None:
        out["d_dmu"] = None
    if dq is None:
        out["d_dq"] = None
    gr = _Grads(*[_ptr(out[k]) for k, _ in _Grads._fields_])
    touched = np.zeros(n, np.uint8)
    p = _Pinned(g, dmu, dq)
    c = _cam(cam)
    dl = np.ascontiguousarray(dl_dimg, np.float64)
    rc = lib().orc_render_backward(C.byref(p.s), C.byref(c), C.c_void_p(_ptr(dl)), C.byref(gr),
                                   C.c_void_p(_ptr(touched)))
    assert rc == 0, rc
    out["touched_ambiguous"] = touched.astype(bool)
    return out


def quat_mul(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    p = np.zeros(4)
    lib().orc_quat_mul(C.c_void_p(_ptr(a)), C.c_void_p(_ptr(b)), C.c_void_p(_ptr(p)))
    return p


def quat_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().orc_quat_rot(C.c_void_p(_ptr(q)), C.c_void_p(_ptr(R)))
    return R.reshape(3, 3)


def sh_basis(deg: int, d):
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().orc_sh_basis(C.c_int(deg), C.c_void_p(_ptr(d)), C.c_void_p(_ptr(Y)), C.c_void_p(_ptr(dY)))
    return Y, dY.reshape(16, 3)


def spec_exp(x: float) -> float:
    return float(lib().orc_spec_exp(C.c_float(x)))


def num_threads() -> int:
    return int(lib().orc_num_threads())
