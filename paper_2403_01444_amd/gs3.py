"""ctypes binding of libgs3.so (include/gs3.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; PyTorch only
provides device memory (contiguous float32 tensors on the GPU) and the
stream.  The module-level functions carry the C names; `Context` wraps them.
Importing this module never falls back to anything: when libgs3.so is not
built, or the GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs3.so")

GS3_OK, GS3_EINVAL, GS3_ENOMEM, GS3_EHIP, GS3_ECAPACITY, GS3_ENONFINITE, GS3_ESTATE = 0, -1, -2, -3, -4, -5, -6
GS3_F32, GS3_F16, GS3_BF16 = 0, 1, 2
GS3_SORT_DEPTH_FIRST, GS3_SORT_RADIX64 = 0, 1
PRECISIONS = {"f32": GS3_F32, "f16": GS3_F16, "bf16": GS3_BF16}
SORT_MODES = {"depth_first": GS3_SORT_DEPTH_FIRST, "radix64": GS3_SORT_RADIX64}
_STATUS = {0: "GS3_OK", -1: "GS3_EINVAL", -2: "GS3_ENOMEM", -3: "GS3_EHIP", -4: "GS3_ECAPACITY",
           -5: "GS3_ENONFINITE", -6: "GS3_ESTATE"}


class GS3Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class NtcConfigC(C.Structure):
    _fields_ = [("levels", C.c_int32), ("feats", C.c_int32), ("log2_T", C.c_int32), ("hidden", C.c_int32),
                ("precision", C.c_int32), ("res", C.c_int32 * 16), ("aabb_min", C.c_float * 3),
                ("inv_extent", C.c_float * 3)]


class ConfigC(C.Structure):
    _fields_ = [("max_gaussians", C.c_int64), ("max_pairs", C.c_int64), ("max_width", C.c_int32),
                ("max_height", C.c_int32), ("num_slots", C.c_int32), ("sort_mode", C.c_int32),
                ("enable_ntc", C.c_int32), ("grad_record_log2", C.c_int32), ("ntc", NtcConfigC)]


class GaussiansC(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32), ("means", C.c_void_p),
                ("quats", C.c_void_p), ("log_scales", C.c_void_p), ("opacity_logits", C.c_void_p),
                ("sh", C.c_void_p)]


class CameraC(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float), ("world_to_cam", C.c_float * 12),
                ("cam_pos", C.c_float * 3), ("bg", C.c_float * 3)]


GRAD_FIELDS = ("d_means", "d_quats", "d_log_scales", "d_opacity_logits", "d_sh", "d_dmu", "d_dq", "d_uv",
               "d_conic", "d_opacity", "d_rgb", "vspace_grad", "vspace_count")
GS3_SPAWN, GS3_SPLIT = 0, 1


class GradsC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in GRAD_FIELDS]


EXPORTED = ("gs3_create", "gs3_destroy", "gs3_last_error", "gs3_set_stream", "gs3_morton_order",
            "gs3_gather_rows", "gs3_ntc_num_params",
            "gs3_ntc_load", "gs3_ntc_save", "gs3_ntc_init", "gs3_ntc_state_bytes", "gs3_ntc_save_state",
            "gs3_ntc_load_state", "gs3_ntc_forward", "gs3_ntc_backward", "gs3_ntc_prepare", "gs3_ntc_step",
            "gs3_ntc_grads", "gs3_ntc_zero_grads", "gs3_warmup_loss", "gs3_render", "gs3_render_backward", "gs3_transform_bake", "gs3_select", "gs3_spawn",
            "gs3_loss", "gs3_loss_noalloc", "gs3_adam", "gs3_zero", "gs3_debug_counts", "gs3_debug_pairs", "gs3_debug_ranges",
            "gs3_debug_gaussians", "gs3_debug_pixels", "gs3_check_flags", "gs3_workspace_bytes", "gs3_profile_enable",
            "gs3_profile_only", "gs3_profile_reset", "gs3_profile_query")

_lib = None


def lib():
    """Load libgs3.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2403_01444_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    sig = {
        "gs3_create": [C.POINTER(ConfigC), C.POINTER(vp)],
        "gs3_destroy": [vp],
        "gs3_last_error": [vp],
        "gs3_set_stream": [vp, vp],
        "gs3_morton_order": [vp, vp, i64, C.POINTER(f32), C.POINTER(f32), vp],
        "gs3_gather_rows": [vp, vp, vp, i64, i32, vp],
        "gs3_ntc_num_params": [vp, C.POINTER(i64)],
        "gs3_ntc_load": [vp, vp, i64],
        "gs3_ntc_save": [vp, vp, i64],
        "gs3_ntc_init": [vp, C.c_uint64],
        "gs3_ntc_state_bytes": [vp, C.POINTER(C.c_size_t)],
        "gs3_ntc_save_state": [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)],
        "gs3_ntc_load_state": [vp, vp, C.c_size_t],
        "gs3_ntc_forward": [vp, vp, i64, C.c_uint64, vp, vp],
        "gs3_ntc_backward": [vp, vp, i64, C.c_uint64, vp, vp],
        "gs3_ntc_prepare": [vp, vp, i64, C.POINTER(C.c_uint64)],
        "gs3_ntc_step": [vp, f32, f32, f32, f32],
        "gs3_ntc_grads": [vp, vp, i64],
        "gs3_ntc_zero_grads": [vp],
        "gs3_warmup_loss": [vp, vp, vp, i64, vp, vp, vp],
        "gs3_render": [vp, i32, C.POINTER(GaussiansC), vp, vp, C.POINTER(CameraC), vp],
        "gs3_render_backward": [vp, i32, vp, C.POINTER(GradsC)],
        "gs3_transform_bake": [vp, C.POINTER(GaussiansC), vp, vp, vp, vp, vp],
        "gs3_select": [vp, vp, vp, i64, C.c_float, vp, C.POINTER(C.c_int64)],
        "gs3_spawn": [vp, C.POINTER(GaussiansC), vp, i64, vp, i32, vp, vp, vp, vp, vp],
        "gs3_loss": [vp, vp, vp, i32, i32, f32, vp, vp],
        "gs3_loss_noalloc": [vp, vp, i32, i32, f32, vp, vp, vp],
        "gs3_adam": [vp, vp, vp, vp, vp, i64, i32, f32, f32, f32, f32],
        "gs3_zero": [vp, vp, i64],
        "gs3_debug_counts": [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)],
        "gs3_debug_pairs": [vp, i32, vp, vp, i64],
        "gs3_debug_ranges": [vp, i32, vp],
        "gs3_debug_gaussians": [vp, i32, vp, vp, vp],
        "gs3_debug_pixels": [vp, i32, vp, vp],
        "gs3_check_flags": [vp],
        "gs3_workspace_bytes": [vp, C.POINTER(i64)],
        "gs3_profile_enable": [vp, i32],
        "gs3_profile_only": [vp, C.c_char_p],
        "gs3_profile_reset": [vp],
        "gs3_profile_query": [vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(i64)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.gs3_destroy.restype = None
    L.gs3_last_error.restype = C.c_char_p
    _lib = L
    return L


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def camera_struct(cam) -> CameraC:
    c = CameraC()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy, c.near_z = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), float(cam.near)
    for k, v in enumerate(np.asarray(cam.world_to_cam, np.float32).reshape(-1)):
        c.world_to_cam[k] = float(v)
    for k in range(3):
        c.cam_pos[k] = float(cam.cam_pos[k])
        c.bg[k] = float(cam.bg[k])
    return c


@dataclass
class GaussiansGPU:
    """Frozen Gaussians resident on the GPU (float32, contiguous)."""
    means: "object"
    quats: "object"
    log_scales: "object"
    opacity_logits: "object"
    sh: "object"
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @staticmethod
    def from_host(g, device="cuda"):
        import torch
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussiansGPU(t(g.means), t(g.quats), t(g.log_scales), t(g.opacity_logits), t(g.sh), g.sh_degree)

    def struct(self) -> GaussiansC:
        n = self.n
        k = (self.sh_degree + 1) ** 2
        return GaussiansC(n, self.sh_degree, 0, _ptr(self.means, numel=3 * n, name="means"),
                          _ptr(self.quats, numel=4 * n, name="quats"),
                          _ptr(self.log_scales, numel=3 * n, name="log_scales"),
                          _ptr(self.opacity_logits, numel=n, name="opacity_logits"),
                          _ptr(self.sh, numel=3 * k * n, name="sh"))


def _check(ctx_handle, status: int):
    if status != GS3_OK:
        msg = lib().gs3_last_error(ctx_handle)
        raise GS3Error(status, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# module-level functions with the C names (ctx = opaque handle)
# ---------------------------------------------------------------------------

def gs3_create(cfg: ConfigC):
    h = C.c_void_p()
    s = lib().gs3_create(C.byref(cfg), C.byref(h))
    if s != GS3_OK:
        raise GS3Error(s, "gs3_create failed")
    return h


def gs3_destroy(h):
    lib().gs3_destroy(h)


def gs3_last_error(h) -> str:
    msg = lib().gs3_last_error(h)
    return msg.decode() if msg else ""


def gs3_set_stream(h, stream_ptr: int):
    _check(h, lib().gs3_set_stream(h, C.c_void_p(stream_ptr)))


def gs3_morton_order(h, means, aabb_min, inv_extent, perm):
    n = means.shape[0]
    lo = (C.c_float * 3)(*[float(v) for v in aabb_min])
    inv = (C.c_float * 3)(*[float(v) for v in inv_extent])
    _check(h, lib().gs3_morton_order(h, _ptr(means, numel=3 * n), n, lo, inv, _ptr(perm, numel=n)))


def gs3_gather_rows(h, src, perm, n, row_floats, dst):
    """dst[i] = src[perm[i]] for n rows; src may hold more rows than dst."""
    if src.numel() % max(row_floats, 1) or src.numel() < n * row_floats:
        raise ValueError("src must hold whole rows of row_floats floats")
    _check(h, lib().gs3_gather_rows(h, _ptr(src, name="src"), _ptr(perm, numel=n), n, row_floats,
                                    _ptr(dst, numel=n * row_floats)))


def gs3_ntc_num_params(h) -> int:
    n = C.c_int64()
    _check(h, lib().gs3_ntc_num_params(h, C.byref(n)))
    return n.value


def gs3_ntc_load(h, params: np.ndarray):
    p = np.ascontiguousarray(params, np.float32)
    _check(h, lib().gs3_ntc_load(h, C.c_void_p(p.ctypes.data), p.size))


def gs3_ntc_save(h, n: int) -> np.ndarray:
    out = np.zeros(n, np.float32)
    _check(h, lib().gs3_ntc_save(h, C.c_void_p(out.ctypes.data), n))
    return out


def gs3_ntc_init(h, seed: int):
    _check(h, lib().gs3_ntc_init(h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF)))


def gs3_ntc_state_bytes(h) -> int:
    b = C.c_size_t(0)
    _check(h, lib().gs3_ntc_state_bytes(h, C.byref(b)))
    return int(b.value)


def gs3_ntc_save_state(h) -> bytes:
    n = gs3_ntc_state_bytes(h)
    buf = C.create_string_buffer(n)
    used = C.c_size_t(0)
    _check(h, lib().gs3_ntc_save_state(h, C.cast(buf, C.c_void_p), n, C.byref(used)))
    return buf.raw[:used.value]


def gs3_ntc_load_state(h, blob: bytes):
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _check(h, lib().gs3_ntc_load_state(h, C.cast(buf, C.c_void_p), len(blob)))


def gs3_ntc_forward(h, means, dmu, dq, token: int = 0):
    n = means.shape[0]
    _check(h, lib().gs3_ntc_forward(h, _ptr(means, numel=3 * n), n, C.c_uint64(token), _ptr(dmu, numel=3 * n),
                                    _ptr(dq, numel=4 * n)))


def gs3_ntc_backward(h, means, d_dmu, d_dq, token: int = 0):
    n = means.shape[0]
    _check(h, lib().gs3_ntc_backward(h, _ptr(means, numel=3 * n), n, C.c_uint64(token), _ptr(d_dmu, numel=3 * n),
                                     _ptr(d_dq, numel=4 * n)))


def gs3_ntc_prepare(h, means) -> int:
    n = means.shape[0]
    tok = C.c_uint64(0)
    _check(h, lib().gs3_ntc_prepare(h, _ptr(means, numel=3 * n), n, C.byref(tok)))
    return int(tok.value)


def gs3_ntc_step(h, lr, beta1, beta2, eps):
    _check(h, lib().gs3_ntc_step(h, lr, beta1, beta2, eps))


def gs3_ntc_grads(h, out):
    _check(h, lib().gs3_ntc_grads(h, _ptr(out), out.numel()))


def gs3_ntc_zero_grads(h):
    _check(h, lib().gs3_ntc_zero_grads(h))


def gs3_warmup_loss(h, dmu, dq, loss, d_dmu, d_dq):
    n = dmu.shape[0]
    _check(h, lib().gs3_warmup_loss(h, _ptr(dmu, numel=3 * n), _ptr(dq, numel=4 * n), n, _ptr(loss),
                                    _ptr(d_dmu, numel=3 * n), _ptr(d_dq, numel=4 * n)))


def gs3_render(h, slot, gs: GaussiansGPU, dmu, dq, cam, image):
    n = gs.n
    gsc = gs.struct()
    camc = camera_struct(cam)
    _check(h, lib().gs3_render(h, slot, C.byref(gsc), _ptr(dmu, numel=3 * n, name="dmu"),
                               _ptr(dq, numel=4 * n, name="dq"), C.byref(camc),
                               _ptr(image, numel=3 * cam.width * cam.height, name="image")))


def gs3_render_backward(h, slot, d_image, grads: dict):
    gr = GradsC(*[_ptr(grads.get(k), name=k) for k in GRAD_FIELDS])
    _check(h, lib().gs3_render_backward(h, slot, _ptr(d_image, name="d_image"), C.byref(gr)))


def gs3_transform_bake(h, gs: GaussiansGPU, dmu, dq, means_out, quats_out, sh_out):
    n = gs.n
    gsc = gs.struct()
    _check(h, lib().gs3_transform_bake(h, C.byref(gsc), _ptr(dmu, numel=3 * n, name="dmu"),
                                       _ptr(dq, numel=4 * n, name="dq"), _ptr(means_out, numel=3 * n),
                                       _ptr(quats_out, numel=4 * n), _ptr(sh_out, numel=gs.sh.numel())))


def gs3_workspace_bytes(h) -> int:
    b = C.c_int64(0)
    _check(h, lib().gs3_workspace_bytes(h, C.byref(b)))
    return int(b.value)


def gs3_select(h, num, den, n, threshold, idx) -> int:
    count = C.c_int64(0)
    _check(h, lib().gs3_select(h, _ptr(num, numel=n, name="num"), _ptr(den, numel=n, name="den"), n,
                               float(threshold), _ptr(idx, name="idx"), C.byref(count)))
    return int(count.value)


def gs3_spawn(h, src: GaussiansGPU, idx, m, z, mode, means, quats, log_scales, logits, sh):
    sc = src.struct()
    _check(h, lib().gs3_spawn(h, C.byref(sc), _ptr(idx, name="idx"), m, _ptr(z, numel=3 * m, name="z"), mode,
                              _ptr(means, numel=3 * m), _ptr(quats, numel=4 * m), _ptr(log_scales, numel=3 * m),
                              _ptr(logits, numel=m), _ptr(sh, numel=m * 3 * (src.sh_degree + 1) ** 2)))


def gs3_loss(h, image, target, height, width, lam, loss, d_image):
    N = 3 * height * width
    _check(h, lib().gs3_loss(h, _ptr(image, numel=N), _ptr(target, numel=N), height, width, lam, _ptr(loss),
                             _ptr(d_image, numel=N)))


def gs3_loss_noalloc(image, target, height, width, lam, loss, d_image, stream_ptr: int = 0):
    """gs3_loss without a context: scratch in the library's per-GPU static
    array (no device allocation); launches on the given HIP stream."""
    N = 3 * height * width
    st = lib().gs3_loss_noalloc(_ptr(image, numel=N), _ptr(target, numel=N), height, width, lam, _ptr(loss),
                                _ptr(d_image, numel=N), C.c_void_p(stream_ptr) if stream_ptr else None)
    if st != GS3_OK:
        raise GS3Error(st, "gs3_loss_noalloc failed")


def gs3_adam(h, param, grad, m, v, step, lr, beta1, beta2, eps):
    n = param.numel()
    _check(h, lib().gs3_adam(h, _ptr(param), _ptr(grad, numel=n), _ptr(m, numel=n), _ptr(v, numel=n), n, step,
                             lr, beta1, beta2, eps))


def gs3_zero(h, t):
    _check(h, lib().gs3_zero(h, _ptr(t, name="zero target"), t.numel()))


def gs3_debug_counts(h, slot):
    """(pairs K, overflow flag, sum over pixels of n_contrib, sum over tiles
    of the longest walk); the sums are -1 when the slot holds no render."""
    k, ov, sc, wk = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
    s = lib().gs3_debug_counts(h, slot, C.byref(k), C.byref(sc), C.byref(wk), C.byref(ov))
    if s not in (GS3_OK, GS3_ECAPACITY):
        _check(h, s)
    return k.value, ov.value, sc.value, wk.value


def gs3_debug_pairs(h, slot, keys, vals):
    _check(h, lib().gs3_debug_pairs(h, slot, _ptr(keys), _ptr(vals), keys.numel()))


def gs3_debug_ranges(h, slot, ranges):
    _check(h, lib().gs3_debug_ranges(h, slot, _ptr(ranges)))


def gs3_debug_gaussians(h, slot, key, box, rec):
    _check(h, lib().gs3_debug_gaussians(h, slot, _ptr(key), _ptr(box), _ptr(rec)))


def gs3_debug_pixels(h, slot, T_final, last):
    _check(h, lib().gs3_debug_pixels(h, slot, _ptr(T_final), _ptr(last)))


def gs3_check_flags(h):
    _check(h, lib().gs3_check_flags(h))


def gs3_profile_enable(h, on: bool):
    _check(h, lib().gs3_profile_enable(h, 1 if on else 0))


def gs3_profile_only(h, kernel):
    _check(h, lib().gs3_profile_only(h, None if not kernel else kernel.encode()))


def gs3_profile_reset(h):
    _check(h, lib().gs3_profile_reset(h))


def gs3_profile_query(h, kernel: str):
    ms, n = C.c_double(), C.c_int64()
    _check(h, lib().gs3_profile_query(h, kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

def torch_empty_like(t):
    import torch
    return torch.empty_like(t)


def make_config(max_gaussians: int, max_pairs: int, max_width: int, max_height: int, num_slots: int = 1,
                sort_mode: str = "depth_first", ntc=None, precision: str = "f32", grad_record_log2: int = 0) -> ConfigC:
    cfg = ConfigC()
    cfg.max_gaussians = int(max_gaussians)
    cfg.max_pairs = int(max_pairs)
    cfg.max_width, cfg.max_height = int(max_width), int(max_height)
    cfg.num_slots = int(num_slots)
    cfg.sort_mode = SORT_MODES[sort_mode]
    cfg.enable_ntc = 1 if ntc is not None else 0
    cfg.grad_record_log2 = int(grad_record_log2)
    if ntc is not None:
        cfg.ntc.levels, cfg.ntc.feats, cfg.ntc.log2_T, cfg.ntc.hidden = ntc.levels, ntc.feats, ntc.log2_T, ntc.hidden
        cfg.ntc.precision = PRECISIONS[precision]
        for l, r in enumerate(ntc.resolutions()):
            cfg.ntc.res[l] = r
        inv = ntc.inv_extent()
        for k in range(3):
            cfg.ntc.aabb_min[k] = float(np.float32(ntc.aabb_min[k]))
            cfg.ntc.inv_extent[k] = float(inv[k])
    return cfg


class Context:
    """Owns one gs3 context; launches on torch's current stream by default."""

    def __init__(self, max_gaussians, max_pairs, max_width, max_height, num_slots=1, sort_mode="depth_first",
                 ntc=None, precision="f32", device=None, grad_record_log2=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("gs3 needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device or "cuda")
        self.ntc_cfg = ntc
        self.precision = precision
        self._held = {}   # per slot: the buffers the last render read
        with torch.cuda.device(self.device):
            self.h = gs3_create(make_config(max_gaussians, max_pairs, max_width, max_height, num_slots, sort_mode,
                                            ntc, precision, grad_record_log2))
        self.use_current_stream()
        self.n_params = gs3_ntc_num_params(self.h) if ntc is not None else 0

    def use_current_stream(self):
        import torch
        gs3_set_stream(self.h, torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            gs3_destroy(self.h)
            self.h = None
        self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- allocation helpers (torch memory only)
    def empty(self, *shape, dtype=None):
        import torch
        return torch.empty(*shape, dtype=dtype or torch.float32, device=self.device)

    def zeros(self, *shape, dtype=None):
        import torch
        return torch.zeros(*shape, dtype=dtype or torch.float32, device=self.device)

    # -- per-frame setup
    def morton_order(self, means, aabb_min, inv_extent):
        import torch
        perm = torch.empty(means.shape[0], dtype=torch.int32, device=self.device)
        gs3_morton_order(self.h, means, aabb_min, inv_extent, perm)
        return perm

    def gather_rows(self, src, perm):
        n = perm.shape[0]
        dst = torch_empty_like(src)
        gs3_gather_rows(self.h, src, perm, n, src.numel() // max(n, 1), dst)
        return dst

    def take_rows(self, src, idx):
        """src[idx] along the first axis (idx: int tensor on the device)."""
        import torch
        m = int(idx.numel())
        rows = src.shape[0]
        dst = torch.empty((m,) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device)
        if m:
            gs3_gather_rows(self.h, src, idx.to(torch.int32).contiguous(), m, src.numel() // max(rows, 1), dst)
        return dst

    def reorder(self, gs: "GaussiansGPU", aabb_min, inv_extent):
        """Morton-ordered copy of a Gaussian set and the permutation used."""
        perm = self.morton_order(gs.means, aabb_min, inv_extent)
        return GaussiansGPU(self.gather_rows(gs.means, perm), self.gather_rows(gs.quats, perm),
                            self.gather_rows(gs.log_scales, perm), self.gather_rows(gs.opacity_logits, perm),
                            self.gather_rows(gs.sh, perm), gs.sh_degree), perm

    # -- NTC
    def ntc_load(self, params):
        gs3_ntc_load(self.h, params)

    def ntc_save(self):
        return gs3_ntc_save(self.h, self.n_params)

    def ntc_init(self, seed: int):
        gs3_ntc_init(self.h, seed)

    def ntc_save_state(self) -> bytes:
        return gs3_ntc_save_state(self.h)

    def ntc_load_state(self, blob: bytes):
        gs3_ntc_load_state(self.h, blob)

    def ntc_forward(self, means, dmu=None, dq=None, token: int = 0):
        n = means.shape[0]
        dmu = self.empty(n, 3) if dmu is None else dmu
        dq = self.empty(n, 4) if dq is None else dq
        gs3_ntc_forward(self.h, means, dmu, dq, token)
        return dmu, dq

    def ntc_backward(self, means, d_dmu, d_dq, token: int = 0):
        gs3_ntc_backward(self.h, means, d_dmu, d_dq, token)

    def ntc_prepare(self, means) -> int:
        """Per-frame contribution lists of frozen means; returns the token
        that forward and backward calls on these means pass."""
        return gs3_ntc_prepare(self.h, means)

    def ntc_step(self, lr=0.002, beta1=0.9, beta2=0.99, eps=1e-15):
        gs3_ntc_step(self.h, lr, beta1, beta2, eps)

    def ntc_grads(self):
        out = self.empty(self.n_params)
        gs3_ntc_grads(self.h, out)
        return out

    def ntc_zero_grads(self):
        gs3_ntc_zero_grads(self.h)

    def warmup_loss(self, dmu, dq):
        n = dmu.shape[0]
        loss = self.empty(1)
        g_mu, g_q = self.empty(n, 3), self.empty(n, 4)
        gs3_warmup_loss(self.h, dmu, dq, loss, g_mu, g_q)
        return loss, g_mu, g_q

    # -- render
    def render(self, gs: GaussiansGPU, cam, dmu=None, dq=None, slot=0, image=None):
        image = self.empty(3, cam.height, cam.width) if image is None else image
        gs3_render(self.h, slot, gs, dmu, dq, cam, image)
        # the slot's backward reads these buffers again: keep them alive
        self._held[slot] = (gs, dmu, dq)
        return image

    def render_backward(self, d_image, grads: dict, slot=0):
        gs3_render_backward(self.h, slot, d_image, grads)
        return grads

    def workspace_bytes(self) -> int:
        return gs3_workspace_bytes(self.h)

    def select(self, num, den=None, threshold=0.0):
        """Ascending indices passing the threshold (int64 tensor on the device)."""
        import torch
        n = num.numel()
        idx = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        m = gs3_select(self.h, num, den, n, threshold, idx)
        return idx[:m].long()

    def spawn(self, src: GaussiansGPU, idx, z, mode=GS3_SPAWN) -> GaussiansGPU:
        """Additional Gaussians around src[idx] (positions from z ~ N(0, I))."""
        import torch
        m = int(idx.numel())
        idx32 = idx.to(torch.int32).contiguous()
        K = (src.sh_degree + 1) ** 2
        out = GaussiansGPU(self.empty(m, 3), self.empty(m, 4), self.empty(m, 3), self.empty(m),
                           self.empty(m, K, 3), src.sh_degree)
        gs3_spawn(self.h, src, idx32, m, z, mode, out.means, out.quats, out.log_scales, out.opacity_logits, out.sh)
        return out

    def transform_bake(self, gs: GaussiansGPU, dmu=None, dq=None) -> GaussiansGPU:
        """The transformed Gaussians (frame carry-over)."""
        import torch
        out = GaussiansGPU(torch.empty_like(gs.means), torch.empty_like(gs.quats), gs.log_scales,
                           gs.opacity_logits, torch.empty_like(gs.sh), gs.sh_degree)
        gs3_transform_bake(self.h, gs, dmu, dq, out.means, out.quats, out.sh)
        return out

    def loss(self, image, target, lam=0.2, loss=None, d_image=None):
        _, H, W = image.shape
        loss = self.empty(1) if loss is None else loss
        d_image = self.empty(3, H, W) if d_image is None else d_image
        gs3_loss(self.h, image, target, H, W, lam, loss, d_image)
        return loss, d_image

    def adam(self, param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
        gs3_adam(self.h, param, grad, m, v, step, lr, beta1, beta2, eps)

    def zero(self, *tensors):
        for t in tensors:
            gs3_zero(self.h, t)

    # -- inspection
    def debug_counts(self, slot=0):
        """(pairs K, overflow flag)."""
        return gs3_debug_counts(self.h, slot)[:2]

    def debug_sums(self, slot=0):
        """(sum over pixels of n_contrib, sum over tiles of the longest walk)."""
        return gs3_debug_counts(self.h, slot)[2:]

    def debug_pairs(self, slot=0):
        import torch
        K, ov = gs3_debug_counts(self.h, slot)[:2]
        keys = torch.empty(max(K, 1), dtype=torch.int64, device=self.device)
        vals = torch.empty(max(K, 1), dtype=torch.int32, device=self.device)
        gs3_debug_pairs(self.h, slot, keys, vals)
        return keys[:K], vals[:K]

    def debug_ranges(self, cam, slot=0):
        import torch
        tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
        r = torch.empty(tiles, 2, dtype=torch.int32, device=self.device)
        gs3_debug_ranges(self.h, slot, r)
        return r

    def debug_gaussians(self, n, slot=0):
        import torch
        key = torch.empty(n, dtype=torch.int32, device=self.device)
        box = torch.empty(n, 4, dtype=torch.int32, device=self.device)
        rec = torch.empty(n, 9, dtype=torch.float32, device=self.device)
        gs3_debug_gaussians(self.h, slot, key, box, rec)
        return key, box, rec

    def debug_pixels(self, cam, slot=0):
        import torch
        T = torch.empty(cam.height, cam.width, dtype=torch.float32, device=self.device)
        last = torch.empty(cam.height, cam.width, dtype=torch.int32, device=self.device)
        gs3_debug_pixels(self.h, slot, T, last)
        return T, last

    def check_flags(self):
        gs3_check_flags(self.h)

    def profile(self, on=True):
        gs3_profile_enable(self.h, on)

    def profile_only(self, kernel=None):
        gs3_profile_only(self.h, kernel)

    def profile_reset(self):
        gs3_profile_reset(self.h)

    def profile_query(self, kernel):
        return gs3_profile_query(self.h, kernel)
