"""Seeded synthetic inputs shaped like the paper's multi-view captures.

This module only draws inputs: Gaussians, pinhole cameras, a motion field
that moves the Gaussians to make the next frame's scene, NTC initial
parameters and the integer table of hash-grid resolutions.  It holds none of
the method's arithmetic (no projection, compositing, encoding or MLP), so
both the HIP path and the CPU oracle take their inputs from here.

Scene recipe (stands in for the N3DV / Meet Room captures of Sec. 5.1, which
are not available): means U[-1,1]^3, log-scales N(-3, 0.3) per axis, unit
quaternions normalize(N(0, I4)) stored (w, x, y, z), opacity logits N(0, 1),
SH degree-0 term chosen so the DC colour is U[0,1]^3, higher bands
N(0, 0.05^2).  Cameras: pinhole, square pixels, principal point at the image
centre ((W-1)/2, (H-1)/2), looking at the origin from distance 3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Value of the degree-0 real spherical harmonic, used only to make the drawn
# DC colour uniform on [0, 1] (colour = sh0 * Y00 + 0.5).
_Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


@dataclass
class Gaussians:
    means: np.ndarray           # (n, 3) float32
    quats: np.ndarray           # (n, 4) float32, (w, x, y, z)
    log_scales: np.ndarray      # (n, 3) float32
    opacity_logits: np.ndarray  # (n,)   float32
    sh: np.ndarray              # (n, (deg+1)^2, 3) float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.means[idx].copy(), self.quats[idx].copy(),
                         self.log_scales[idx].copy(),
                         self.opacity_logits[idx].copy(), self.sh[idx].copy(),
                         self.sh_degree)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    near: float
    world_to_cam: np.ndarray    # (3, 4) float32, rows = camera x (right), y (down), z (forward)
    cam_pos: np.ndarray         # (3,) float32
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))


def make_gaussians(n: int, sh_degree: int, seed: int) -> Gaussians:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = rng.normal(-3.0, 0.3, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=(n,))
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    sh[:, 0, :] = (rng.uniform(0.0, 1.0, size=(n, 3)) - 0.5) / _Y00
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.05, size=(n, k - 1, 3))
    f = np.float32
    return Gaussians(means.astype(f), q.astype(f), log_scales.astype(f),
                     logits.astype(f), sh.astype(f), sh_degree)


def look_at_camera(width: int, height: int, fov_x_deg: float = 60.0,
                   azimuth_deg: float = 0.0, elevation_deg: float = 0.0,
                   distance: float = 3.0, near: float = 0.2,
                   bg=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at `distance` from the origin looking at it.

    Azimuth turns about the world +y axis; azimuth 0 sits on the -z axis.
    fx = fy = (W/2) / tan(fov_x/2); principal point ((W-1)/2, (H-1)/2).
    """
    th = math.radians(azimuth_deg)
    ph = math.radians(elevation_deg)
    eye = distance * np.array([math.sin(th) * math.cos(ph), math.sin(ph),
                               -math.cos(th) * math.cos(ph)])
    zc = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 1.0, 0.0])
    xc = np.cross(zc, up)
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    rot = np.stack([xc, yc, zc])
    t = -rot @ eye
    w2c = np.concatenate([rot, t[:, None]], axis=1)
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(width, height, float(np.float32(fx)), float(np.float32(fx)),
                  (width - 1) / 2.0, (height - 1) / 2.0, near,
                  w2c.astype(np.float32), eye.astype(np.float32),
                  np.asarray(bg, np.float32))


def ring_cameras(count: int, width: int, height: int, **kw) -> list[Camera]:
    """`count` cameras on a horizontal ring (azimuth 0, 360/count, ...)."""
    return [look_at_camera(width, height, azimuth_deg=360.0 * i / count, **kw)
            for i in range(count)]


def arc_cameras(count: int, width: int, height: int, half_angle: float = 30.0,
                **kw) -> list[Camera]:
    """`count` forward-facing cameras, azimuth evenly spaced in [-a, +a]."""
    if count == 1:
        return [look_at_camera(width, height, **kw)]
    return [look_at_camera(width, height,
                           azimuth_deg=-half_angle + 2 * half_angle * i / (count - 1),
                           **kw) for i in range(count)]


# --- motion fields: draw the next frame's scene -----------------------------

def _hamilton(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def smooth_displacement(g: Gaussians, seed: int, max_disp: float = 0.05) -> Gaussians:
    """Means shifted by a seeded smooth field with |d| <= max_disp."""
    rng = np.random.default_rng(seed)
    x = g.means.astype(np.float64)
    d = np.zeros_like(x)
    amp = max_disp / math.sqrt(3.0)
    for c in range(3):
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        phase = rng.uniform(0, 2 * math.pi)
        d[:, c] = amp * np.sin(math.pi * (x @ k) + phase)
    out = g.subset(slice(None))
    out.means = (x + d).astype(np.float32)
    return out


def rigid_sinusoid_motion(g: Gaussians, seed: int, angle_deg: float = 1.0,
                          translation: float = 0.01, wave: float = 0.01) -> Gaussians:
    """Rigid rotation about a random axis + translation + sinusoid.

    The rotation also turns every Gaussian: q_next = q_rot (x) q.
    """
    rng = np.random.default_rng(seed)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    half = math.radians(angle_deg) / 2.0
    q_rot = np.concatenate([[math.cos(half)], math.sin(half) * axis])
    w, (ax, ay, az) = q_rot[0], q_rot[1:]
    rot = np.array([[1 - 2 * (ay * ay + az * az), 2 * (ax * ay - w * az), 2 * (ax * az + w * ay)],
                    [2 * (ax * ay + w * az), 1 - 2 * (ax * ax + az * az), 2 * (ay * az - w * ax)],
                    [2 * (ax * az - w * ay), 2 * (ay * az + w * ax), 1 - 2 * (ax * ax + ay * ay)]])
    tdir = rng.normal(size=3)
    tdir /= np.linalg.norm(tdir)
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    phase = rng.uniform(0, 2 * math.pi, size=3)
    x = g.means.astype(np.float64)
    s = np.sin(2 * math.pi * (x @ k)[:, None] + phase[None, :]) * (wave / math.sqrt(3.0))
    moved = x @ rot.T + translation * tdir + s
    out = g.subset(slice(None))
    out.means = moved.astype(np.float32)
    qn = _hamilton(np.broadcast_to(q_rot, g.quats.shape), g.quats.astype(np.float64))
    out.quats = qn.astype(np.float32)
    return out


# --- a capture-like scene: textured surfaces, moving objects -------------------

def _quat_from_frame(t1: np.ndarray, t2: np.ndarray, nrm: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z) of rotations with columns (t1, t2, nrm)."""
    R = np.stack([t1, t2, nrm], axis=2)            # (n, 3, 3), columns
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    q = np.zeros((R.shape[0], 4))
    # Shepperd's method, branch on the largest of (tr, R00, R11, R22)
    cand = np.stack([tr, R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]], axis=1)
    k = np.argmax(cand, axis=1)
    for b in range(4):
        m = k == b
        if not m.any():
            continue
        r = R[m]
        if b == 0:
            s = np.sqrt(1.0 + tr[m]) * 2
            q[m] = np.stack([0.25 * s, (r[:, 2, 1] - r[:, 1, 2]) / s, (r[:, 0, 2] - r[:, 2, 0]) / s,
                             (r[:, 1, 0] - r[:, 0, 1]) / s], 1)
        elif b == 1:
            s = np.sqrt(1.0 + r[:, 0, 0] - r[:, 1, 1] - r[:, 2, 2]) * 2
            q[m] = np.stack([(r[:, 2, 1] - r[:, 1, 2]) / s, 0.25 * s, (r[:, 0, 1] + r[:, 1, 0]) / s,
                             (r[:, 0, 2] + r[:, 2, 0]) / s], 1)
        elif b == 2:
            s = np.sqrt(1.0 + r[:, 1, 1] - r[:, 0, 0] - r[:, 2, 2]) * 2
            q[m] = np.stack([(r[:, 0, 2] - r[:, 2, 0]) / s, (r[:, 0, 1] + r[:, 1, 0]) / s, 0.25 * s,
                             (r[:, 1, 2] + r[:, 2, 1]) / s], 1)
        else:
            s = np.sqrt(1.0 + r[:, 2, 2] - r[:, 0, 0] - r[:, 1, 1]) * 2
            q[m] = np.stack([(r[:, 1, 0] - r[:, 0, 1]) / s, (r[:, 0, 2] + r[:, 2, 0]) / s,
                             (r[:, 1, 2] + r[:, 2, 1]) / s, 0.25 * s], 1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


@dataclass
class SurfaceScene:
    gaussians: Gaussians
    labels: np.ndarray          # 0 = static background, k >= 1 = object k
    centres: np.ndarray         # (objects + 1, 3); row 0 unused


def surface_scene(n: int, sh_degree: int, seed: int, objects: int = 6) -> SurfaceScene:
    """Gaussians on textured surfaces, the structure of a reconstructed
    capture: a back wall (z = 0.9) and a floor (y = -0.9) of the [-1, 1]^3 box,
    and `objects` spheres in front of them.  Each Gaussian is a flat disk in
    its surface (tangent scales ~1.2x the sample spacing, normal scale 0.2x),
    nearly opaque, coloured by a smooth multi-frequency texture."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(0.15, 0.3, size=objects)
    centres = np.stack([rng.uniform(-0.6, 0.6, objects),
                        rng.uniform(-0.9 + radii, 0.4),
                        rng.uniform(-0.5, 0.5, objects)], axis=1)
    areas = np.concatenate([[4.0, 3.8], 4 * math.pi * radii ** 2])
    counts = np.floor(n * areas / areas.sum()).astype(np.int64)
    counts[0] += n - counts.sum()
    P, N, T1, L = [], [], [], []
    # back wall: x, y in [-1, 1], z = 0.9, normal towards the cameras (-z)
    c = counts[0]
    P.append(np.stack([rng.uniform(-1, 1, c), rng.uniform(-1, 1, c), np.full(c, 0.9)], 1))
    N.append(np.tile([0.0, 0.0, -1.0], (c, 1)))
    L.append(np.zeros(c, np.int64))
    # floor: x in [-1, 1], z in [-1, 0.9], y = -0.9, normal +y
    c = counts[1]
    P.append(np.stack([rng.uniform(-1, 1, c), np.full(c, -0.9), rng.uniform(-1, 0.9, c)], 1))
    N.append(np.tile([0.0, 1.0, 0.0], (c, 1)))
    L.append(np.zeros(c, np.int64))
    for k in range(objects):
        c = counts[2 + k]
        d = rng.normal(size=(c, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        P.append(centres[k] + radii[k] * d)
        N.append(d)
        L.append(np.full(c, k + 1, np.int64))
    P, N, L = np.concatenate(P), np.concatenate(N), np.concatenate(L)
    # random tangent frame about each normal
    a = rng.normal(size=(n, 3))
    t1 = a - (a * N).sum(1, keepdims=True) * N
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(N, t1)
    q = _quat_from_frame(t1, t2, N)
    spacing = math.sqrt(areas.sum() / n)
    log_scales = np.stack([np.log(1.2 * spacing) + rng.normal(0, 0.15, n),
                           np.log(1.2 * spacing) + rng.normal(0, 0.15, n),
                           np.log(0.2 * spacing) + rng.normal(0, 0.15, n)], 1)
    logits = rng.normal(2.5, 0.5, n)
    # texture: three octaves of random plane waves per channel, plus an object tint
    col = np.full((n, 3), 0.5)
    for amp, freq in ((0.2, 1.0), (0.12, 3.0), (0.08, 8.0)):
        for ch in range(3):
            f = rng.normal(size=3)
            f *= freq / np.linalg.norm(f)
            col[:, ch] += amp * np.sin(2 * math.pi * (P @ f) + rng.uniform(0, 2 * math.pi))
    tint = rng.uniform(-0.15, 0.15, size=(objects + 1, 3))
    tint[0] = 0
    col = np.clip(col + tint[L], 0.02, 0.98)
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    sh[:, 0, :] = (col - 0.5) / _Y00
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.02, size=(n, k - 1, 3))
    f32 = np.float32
    g = Gaussians(P.astype(f32), q.astype(f32), log_scales.astype(f32), logits.astype(f32),
                  sh.astype(f32), sh_degree)
    return SurfaceScene(g, L, np.concatenate([np.zeros((1, 3)), centres]))


def object_motion(scene: SurfaceScene, seed: int, angle_deg: float = 1.5, translation: float = 0.006,
                  wave: float = 0.002) -> Gaussians:
    """Next frame of a surface scene: the background stays, each object turns
    by `angle_deg` about a random axis through its centre, moves by
    `translation` in a random direction and bends by a sinusoid of amplitude
    `wave`; its Gaussians turn with it (q_next = q_rot (x) q)."""
    rng = np.random.default_rng(seed)
    g = scene.gaussians
    out = g.subset(slice(None))
    x = g.means.astype(np.float64)
    moved = x.copy()
    qn = g.quats.astype(np.float64).copy()
    for k in range(1, scene.centres.shape[0]):
        m = scene.labels == k
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        half = math.radians(angle_deg) / 2.0
        q_rot = np.concatenate([[math.cos(half)], math.sin(half) * axis])
        w, (ax, ay, az) = q_rot[0], q_rot[1:]
        rot = np.array([[1 - 2 * (ay * ay + az * az), 2 * (ax * ay - w * az), 2 * (ax * az + w * ay)],
                        [2 * (ax * ay + w * az), 1 - 2 * (ax * ax + az * az), 2 * (ay * az - w * ax)],
                        [2 * (ax * az - w * ay), 2 * (ay * az + w * ax), 1 - 2 * (ax * ax + ay * ay)]])
        tdir = rng.normal(size=3)
        tdir /= np.linalg.norm(tdir)
        kv = rng.normal(size=3)
        kv *= 3.0 / np.linalg.norm(kv)
        ph = rng.uniform(0, 2 * math.pi, size=3)
        c = scene.centres[k]
        s = np.sin(2 * math.pi * (x[m] @ kv)[:, None] + ph[None, :]) * (wave / math.sqrt(3.0))
        moved[m] = (x[m] - c) @ rot.T + c + translation * tdir + s
        qn[m] = _hamilton(np.broadcast_to(q_rot, (int(m.sum()), 4)), qn[m])
    out.means = moved.astype(np.float32)
    out.quats = qn.astype(np.float32)
    return out


def emerging_object(g: Gaussians, seed: int, n_obj: int = 2000, centre=(0.25, 0.05, -0.3),
                    radius: float = 0.12) -> Gaussians:
    """`g` plus a new textured sphere of `n_obj` flat, nearly opaque
    Gaussians (an object that was not in the previous frame: something only
    Stage 2 can add)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_obj, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = np.asarray(centre) + radius * d
    a = rng.normal(size=(n_obj, 3))
    t1 = a - (a * d).sum(1, keepdims=True) * d
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    q = _quat_from_frame(t1, np.cross(d, t1), d)
    spacing = math.sqrt(4 * math.pi * radius * radius / n_obj)
    ls = np.stack([np.log(1.2 * spacing) + rng.normal(0, 0.15, n_obj),
                   np.log(1.2 * spacing) + rng.normal(0, 0.15, n_obj),
                   np.log(0.2 * spacing) + rng.normal(0, 0.15, n_obj)], 1)
    col = np.tile(rng.uniform(0.2, 0.8, size=3), (n_obj, 1))
    for amp, freq in ((0.15, 4.0), (0.1, 12.0)):
        for ch in range(3):
            f = rng.normal(size=3)
            f *= freq / np.linalg.norm(f)
            col[:, ch] += amp * np.sin(2 * math.pi * (pts @ f) + rng.uniform(0, 2 * math.pi))
    col = np.clip(col, 0.02, 0.98)
    K = (g.sh_degree + 1) ** 2
    sh = np.zeros((n_obj, K, 3))
    sh[:, 0, :] = (col - 0.5) / _Y00
    f32 = np.float32
    return Gaussians(np.concatenate([g.means, pts.astype(f32)]), np.concatenate([g.quats, q.astype(f32)]),
                     np.concatenate([g.log_scales, ls.astype(f32)]),
                     np.concatenate([g.opacity_logits, rng.normal(2.5, 0.5, n_obj).astype(f32)]),
                     np.concatenate([g.sh, sh.astype(f32)]), g.sh_degree)


# --- NTC configuration and initial parameters --------------------------------

@dataclass
class NTCConfig:
    levels: int = 16
    feats: int = 2
    log2_T: int = 15
    base_res: int = 16
    max_res: int = 1024
    hidden: int = 64
    out_dim: int = 7
    aabb_min: tuple = (-1.2, -1.2, -1.2)
    aabb_max: tuple = (1.2, 1.2, 1.2)

    def resolutions(self) -> list[int]:
        """Integer grid resolution per level: floor(base * b^l), b^(L-1) = max/base.

        Evaluated in float64 with a 1e-9 guard so that exact powers (64, 256,
        1024 for base 16 and max 1024) do not round down.
        """
        if self.levels == 1:
            return [self.base_res]
        b = math.exp(math.log(self.max_res / self.base_res) / (self.levels - 1))
        return [int(math.floor(self.base_res * b ** l + 1e-9)) for l in range(self.levels)]

    def level_sizes(self) -> list[int]:
        T = 1 << self.log2_T
        return [min((r + 1) ** 3, T) for r in self.resolutions()]

    def num_table_params(self) -> int:
        return sum(self.level_sizes()) * self.feats

    def num_mlp_params(self) -> int:
        h, i = self.hidden, self.levels * self.feats
        return h * i + h * h + self.out_dim * h

    def num_params(self) -> int:
        return self.num_table_params() + self.num_mlp_params()

    def inv_extent(self) -> np.ndarray:
        ext = np.asarray(self.aabb_max, np.float64) - np.asarray(self.aabb_min, np.float64)
        return (1.0 / ext).astype(np.float32)


def ntc_init_params(cfg: NTCConfig, seed: int) -> np.ndarray:
    """Flat float32 vector [table | W1 | W2 | W3].

    Table U(-1e-4, 1e-4); each weight matrix (row-major [out][in])
    Kaiming-uniform U(-sqrt(6/fan_in), +sqrt(6/fan_in)).
    """
    rng = np.random.default_rng(seed)
    table = rng.uniform(-1e-4, 1e-4, size=cfg.num_table_params())
    h, i, o = cfg.hidden, cfg.levels * cfg.feats, cfg.out_dim
    ws = []
    for (fo, fi) in ((h, i), (h, h), (o, h)):
        bound = math.sqrt(6.0 / fi)
        ws.append(rng.uniform(-bound, bound, size=fo * fi))
    return np.concatenate([table] + ws).astype(np.float32)


def view_schedule(count: int, iters: int, seed: int) -> list[int]:
    """Training views of `iters` iterations: a fresh seeded permutation of
    the `count` views per epoch (reading C10).  The training loops draw their
    views in exactly this order, so the list can be handed to another
    implementation of the same loop."""
    rng = np.random.default_rng(seed)
    out: list[int] = []
    while len(out) < iters:
        out.extend(int(v) for v in rng.permutation(count))
    return out[:iters]


def warmup_points(means: np.ndarray, cfg: NTCConfig, seed: int, rel_sigma: float = 0.01) -> np.ndarray:
    """Noise-augmented means for the NTC warm-up: mu + N(0, (rel_sigma * extent)^2)."""
    rng = np.random.default_rng(seed)
    ext = np.asarray(cfg.aabb_max) - np.asarray(cfg.aabb_min)
    return (means + rng.normal(size=means.shape) * (rel_sigma * ext)).astype(np.float32)


# --- the benchmark workloads --------------------------------------------------

def workload(name: str, seed: int = 0):
    """Scene, cameras and motion for one named workload.

    small-2k-64px   : 2,000 Gaussians, SH0, one 64x64 camera.
    ring-50k-256px  : 50K Gaussians, SH1, four 256x256 cameras on a ring.
    arc-300k-1352px : 300K Gaussians, SH3, 20 training cameras at 1352x1014 on a
                      forward arc (azimuth in [-30, 30] deg) + one held-out
                      camera at azimuth 1.5 deg.
    grad-200-32px   : 200 Gaussians, SH3, one 32x32 camera.
    surfaces-300k-1352px-new : the same, and in the next frame a new object
                      (a textured sphere of about 2K Gaussians) appears.
    surfaces-50k-256px : 50K Gaussians (SH1) of the same kind of scene, 12 arc
                      cameras at 256x256, held-out camera at azimuth 0 (midway
                      between two training views).
    surfaces-300k-1352px : the arc cameras of arc-300k-1352px on a capture-like
                      scene of 300K Gaussians (SH3): textured wall, floor and six
                      spheres; the spheres move, the background stays.
    """
    if name == "small-2k-64px":
        g = make_gaussians(2000, 0, seed)
        cams = [look_at_camera(64, 64)]
        nxt = smooth_displacement(g, seed + 1000)
        return g, cams, [], nxt
    if name == "ring-50k-256px":
        g = make_gaussians(50_000, 1, seed)
        cams = ring_cameras(4, 256, 256)
        nxt = rigid_sinusoid_motion(g, seed + 1000)
        return g, cams, [look_at_camera(256, 256, azimuth_deg=45.0)], nxt
    if name == "arc-300k-1352px":
        g = make_gaussians(300_000, 3, seed)
        cams = arc_cameras(20, 1352, 1014)
        nxt = rigid_sinusoid_motion(g, seed + 1000)
        return g, cams, [look_at_camera(1352, 1014, azimuth_deg=1.5)], nxt
    if name == "surfaces-50k-256px":
        sc = surface_scene(50_000, 1, seed)
        cams = arc_cameras(12, 256, 256)
        nxt = object_motion(sc, seed + 1000)
        return sc.gaussians, cams, [look_at_camera(256, 256, azimuth_deg=0.0)], nxt
    if name == "surfaces-300k-1352px-new":
        sc = surface_scene(300_000, 3, seed)
        cams = arc_cameras(20, 1352, 1014)
        nxt = emerging_object(object_motion(sc, seed + 1000), seed + 2000)
        return sc.gaussians, cams, [look_at_camera(1352, 1014, azimuth_deg=1.5)], nxt
    if name == "surfaces-300k-1352px":
        sc = surface_scene(300_000, 3, seed)
        cams = arc_cameras(20, 1352, 1014)
        nxt = object_motion(sc, seed + 1000)
        return sc.gaussians, cams, [look_at_camera(1352, 1014, azimuth_deg=1.5)], nxt
    if name == "grad-200-32px":
        g = make_gaussians(200, 3, seed)
        return g, [look_at_camera(32, 32)], [], smooth_displacement(g, seed + 1000)
    raise KeyError(name)
