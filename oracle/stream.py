"""One frame of the streaming loop on the oracle (test infrastructure only).

Sec. 4 and Fig. 2: Stage 1 trains the NTC from the stored warm-up parameters
on the frame's training views (Sec. 4.1, Eq. 5-6), tracking the view-space
positional gradient over its final epoch (readings S1, S2); the learned
transform is baked into the Gaussians carried to the next frame (reading
F2, Suppl. Sec. B); Stage 2 (Sec. 4.2) spawns additional Gaussians around
those above tau_grad, optimises only them with the per-attribute learning
rates of Suppl. Sec. A (reading S4) and applies quantity control at the end
of each epoch (split above tau_grad, readings S3; prune below tau_alpha,
reading S5).  All arithmetic float64; parameters are stored as float32
between steps, as the GPU keeps them.  The random numbers the method draws
(view orders, spawn and split positions) are inputs: view lists and a numpy
generator the caller seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import loss as oloss
from . import ntc as ontc
from . import optim as oopt
from . import raster as orc
from . import shrot
from . import stage1
from . import stage2

ATTRS = ("means", "quats", "log_scales", "opacity_logits", "sh")
LR = {"means": 0.0024, "sh": 0.0375, "opacity_logits": 0.75, "log_scales": 0.075, "quats": 0.015}


@dataclass
class Gaussians:
    means: np.ndarray
    quats: np.ndarray
    log_scales: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


def _f32(a):
    return np.asarray(a, np.float32)


def _cat(a: Gaussians, b: Gaussians) -> Gaussians:
    return Gaussians(*(np.concatenate([_f32(getattr(a, k)), _f32(getattr(b, k))]) for k in ATTRS), a.sh_degree)


def _rows(g: Gaussians, idx) -> Gaussians:
    return Gaussians(*(_f32(getattr(g, k))[idx] for k in ATTRS), g.sh_degree)


def _vspace(g, cam, d_uv):
    """Per-view view-space gradient norm and visibility (readings S2)."""
    vis = orc.preprocess(g, cam)["visible"].astype(bool)
    return np.where(vis, stage2.vspace_grad(d_uv, cam.width, cam.height), 0.0), vis.astype(np.float64)


def stage1_tracked(spec, params0, g, cams, targets, views, lam=0.2, lr=0.002, betas=(0.9, 0.99), eps=1e-15,
                   perturb=None):
    """Stage 1 (as stage1.ntc_stage1, including its `perturb`) with the
    view-space gradient summed over the final min(iterations, views)
    iterations.  Returns the final float32 parameters, the per-iteration
    (parameters, gradient), and (total, count)."""
    pert = stage1._perturber(perturb)
    p = np.asarray(params0, np.float32).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    vg, vc = np.zeros(g.n), np.zeros(g.n)
    last = min(len(views), len(cams))
    kept = []
    for t, view in enumerate(views, start=1):
        dmu, dq, cache = ontc.forward(spec, p, g.means)
        dmu32, dq32 = dmu.astype(np.float32), dq.astype(np.float32)
        cam = cams[view]
        img = pert(orc.render(g, cam, dmu32, dq32)["image"])
        L, dL = oloss.stage1_loss(img, np.asarray(targets[view], np.float64), lam)
        gr = orc.render_backward(g, cam, dL, dmu32, dq32)
        if t > len(views) - last:
            a, b = _vspace_transformed(g, cam, gr["d_uv"], dmu32, dq32)
            vg += a
            vc += b
        grad = pert(ontc.backward(spec, p, cache, gr["d_dmu"], gr["d_dq"]))
        p, m, v = oopt.adam(p, grad, m, v, t, lr, betas[0], betas[1], eps)
        p = p.astype(np.float32).astype(np.float64)
        kept.append((p.astype(np.float32), grad))
    return p.astype(np.float32), kept, (vg, vc)


def _vspace_transformed(g, cam, d_uv, dmu, dq):
    vis = orc.preprocess(g, cam, dmu, dq)["visible"].astype(bool)
    return np.where(vis, stage2.vspace_grad(d_uv, cam.width, cam.height), 0.0), vis.astype(np.float64)


def stage2_run(base: Gaussians, cams, targets, vg, vc, iters, views, rng, lam=0.2, tau_grad=stage2.TAU_GRAD,
               tau_alpha=stage2.TAU_ALPHA, max_add=None, betas=(0.9, 0.999), eps=1e-15):
    """Stage 2 on the baked Gaussians `base`: spawn, `iters` iterations on the
    additional Gaussians only, quantity control after every epoch.  The
    float32 threshold comparisons follow the decisions the method takes
    (average gradient above tau_grad; logit at or above float32(logit
    tau_alpha)).  Returns the additional Gaussians and (spawned count, the
    indices selected at each decision)."""
    logit_alpha = float(np.float32(math.log(tau_alpha / (1.0 - tau_alpha))))

    def choose(total, count, current):
        idx = stage2.select(total, count, tau_grad)
        if max_add is not None and idx.size + current > max_add:
            idx = idx[:max(max_add - current, 0)]
        return idx

    idx = choose(vg, vc, 0)
    z = rng.normal(size=(idx.size, 3)).astype(np.float32)
    add = Gaussians(*(_f32(a) for a in stage2.spawn(base, idx, z, "spawn")), base.sh_degree)
    decisions = [idx]
    spawned = int(idx.size)
    state = {k: (np.zeros(getattr(add, k).shape), np.zeros(getattr(add, k).shape)) for k in ATTRS}
    tv, tc = np.zeros(add.n), np.zeros(add.n)
    t = 0
    nb = base.n
    for it, view in enumerate(views[:iters], start=1):
        cam = cams[view]
        allg = _cat(base, add)
        img = orc.render(allg, cam)["image"]
        L, dL = oloss.stage1_loss(img, np.asarray(targets[view], np.float64), lam)
        if add.n:
            gr = orc.render_backward(allg, cam, dL)
            a, b = _vspace(allg, cam, gr["d_uv"])
            tv += a[nb:]
            tc += b[nb:]
            t += 1
            keys = {"means": "d_means", "quats": "d_quats", "log_scales": "d_log_scales",
                    "opacity_logits": "d_opacity_logits", "sh": "d_sh"}
            new = {}
            for k in ATTRS:
                g_k = gr[keys[k]][nb:].reshape(getattr(add, k).shape)
                m_, v_ = state[k]
                p_, m_, v_ = oopt.adam(getattr(add, k), g_k, m_, v_, t, LR[k], betas[0], betas[1], eps)
                new[k] = _f32(p_)
                state[k] = (m_, v_)
            add = Gaussians(*(new[k] for k in ATTRS), add.sh_degree)
        if it % len(cams) == 0 and add.n:
            sidx = choose(tv, tc, add.n)
            decisions.append(sidx)
            z = rng.normal(size=(sidx.size, 3)).astype(np.float32)
            extra = Gaussians(*(_f32(a) for a in stage2.spawn(add, sidx, z, "split")), add.sh_degree)
            merged = _cat(add, extra)
            state = {k: tuple(np.concatenate([s, np.zeros(getattr(extra, k).shape)]) for s in state[k]) for k in ATTRS}
            keep = np.nonzero(merged.opacity_logits.astype(np.float32) >= np.float32(logit_alpha))[0]
            decisions.append(keep)
            add = _rows(merged, keep)
            state = {k: tuple(s[keep] for s in state[k]) for k in ATTRS}
            tv, tc = np.zeros(add.n), np.zeros(add.n)
    return add, spawned, decisions


def frame(spec, warm_params, g: Gaussians, cams, targets, views1, views2, rng, s2_iters, perturb=None, **kw):
    """Stage 1, bake, Stage 2 of one frame.  Returns a dict with the Stage-1
    parameters (per iteration), the baked Gaussians carried to the next frame,
    the additional Gaussians and the Stage-2 decisions.  `perturb` perturbs
    Stage 1 as in stage1.ntc_stage1."""
    p, kept, (vg, vc) = stage1_tracked(spec, warm_params, g, cams, targets, views1, perturb=perturb)
    dmu, dq, _ = ontc.forward(spec, p.astype(np.float64), g.means)
    mu, q, sh = shrot.bake(g, dmu.astype(np.float32), dq.astype(np.float32))
    baked = Gaussians(_f32(mu), _f32(q), _f32(g.log_scales), _f32(g.opacity_logits), _f32(sh), g.sh_degree)
    add, spawned, decisions = stage2_run(baked, cams, targets, vg, vc, s2_iters, views2, rng, **kw)
    return {"params": kept, "vspace": (vg, vc), "baked": baked, "added": add, "spawned": spawned,
            "decisions": decisions, "all": _cat(baked, add)}


def psnr(img, target) -> float:
    return stage1.psnr(img, target)
