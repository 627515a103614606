"""Stage 2 (adaptive 3DG addition, Sec. 4.2) in float64 numpy: test
infrastructure only.

* view-space positional gradient: the norm of the loss gradient with respect
  to a Gaussian's projected mean in normalised device coordinates; a pixel
  coordinate u maps to ndc = (2u + 1)/W - 1, so dL/d ndc = dL/du * W/2
  (the 3DG-S convention the paper's threshold tau_grad = 0.00015 refers to);
  averaged over the views in which the Gaussian was visible;
* selection of Gaussians whose average exceeds tau_grad;
* spawning: X ~ N(mu, 2 Sigma) with Sigma = R S S^T R^T, i.e.
  X = mu + sqrt(2) R S z for z ~ N(0, I) (z is an input); the new Gaussian
  keeps the SH and scale of its source, identity rotation, opacity 0.1
  (mode "spawn"), or, in the quantity-control split, keeps the rotation, SH
  and opacity and takes 80% of the scale (mode "split");
* pruning: additional Gaussians with opacity below tau_alpha = 0.01 are
  discarded.
"""
from __future__ import annotations

import math

import numpy as np

from . import raster as orc

TAU_GRAD = 0.00015
TAU_ALPHA = 0.01
SPAWN_OPACITY = 0.1
SPLIT_SCALE = 0.8


def vspace_grad(d_uv: np.ndarray, width: int, height: int) -> np.ndarray:
    """Per Gaussian: |(dL/du W/2, dL/dv H/2)| (one view)."""
    d = np.asarray(d_uv, np.float64)
    return np.sqrt((d[:, 0] * (width / 2.0)) ** 2 + (d[:, 1] * (height / 2.0)) ** 2)


def select(total: np.ndarray, count: np.ndarray, tau: float = TAU_GRAD) -> np.ndarray:
    """Indices (ascending) of Gaussians seen at least once whose average
    view-space gradient exceeds tau."""
    total = np.asarray(total, np.float64)
    count = np.asarray(count, np.float64)
    avg = np.where(count > 0, total / np.maximum(count, 1), 0.0)
    return np.nonzero((count > 0) & (avg > tau))[0]


def spawn(g, idx: np.ndarray, z: np.ndarray, mode: str = "spawn"):
    """New Gaussians from the selected ones: (means, quats, log_scales,
    opacity_logits, sh), float64."""
    idx = np.asarray(idx, np.int64)
    m = idx.size
    K = (g.sh_degree + 1) ** 2
    means = np.zeros((m, 3))
    quats = np.zeros((m, 4))
    log_scales = np.asarray(g.log_scales, np.float64)[idx].copy()
    logits = np.asarray(g.opacity_logits, np.float64)[idx].copy()
    sh = np.asarray(g.sh, np.float64)[idx].reshape(m, K, 3).copy()
    for k, i in enumerate(idx):
        q = np.asarray(g.quats[i], np.float64)
        qn = np.linalg.norm(q)
        q = q / qn if qn > 0 else np.array([1.0, 0.0, 0.0, 0.0])
        R = orc.quat_rot(q)
        s = np.exp(np.asarray(g.log_scales[i], np.float64))
        means[k] = np.asarray(g.means[i], np.float64) + math.sqrt(2.0) * (R @ (s * np.asarray(z[k], np.float64)))
        if mode == "spawn":
            quats[k] = [1.0, 0.0, 0.0, 0.0]
        else:
            quats[k] = np.asarray(g.quats[i], np.float64)
    if mode == "spawn":
        logits[:] = math.log(SPAWN_OPACITY / (1.0 - SPAWN_OPACITY))
    elif mode == "split":
        log_scales += math.log(SPLIT_SCALE)
    else:
        raise ValueError(mode)
    return means, quats, log_scales, logits, sh


def keep_opaque(logits: np.ndarray, tau: float = TAU_ALPHA) -> np.ndarray:
    """Indices (ascending) of Gaussians whose opacity sigmoid(logit) >= tau."""
    l = np.asarray(logits, np.float64)
    return np.nonzero(1.0 / (1.0 + np.exp(-l)) >= tau)[0]
