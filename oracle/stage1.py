"""Stage-1 training loops on the oracle (test infrastructure only).

Sec. 4.1: each iteration queries the NTC at every frozen mean (Eq. 5),
transforms the Gaussians, renders one training view (Eq. 1-4), takes the
loss of Eq. 6 against that view's target, back-propagates through the
renderer and the NTC, and steps Adam on the NTC parameters (lr 0.002,
Suppl. Sec. A; betas and epsilon of reading B7).  All arithmetic is
float64; the parameters are rounded to float32 after every step, since the
GPU keeps float32 master parameters.  The training views come as a list
(reading C10: the same schedule is handed to the GPU loop).

psnr() is reading C12: 10 log10(1 / MSE) on images clamped to [0, 1].

`perturb` = (seed, rel) multiplies every element of the rendered image and
of the parameter gradient of every iteration by (1 + rel z), z standard
normal, drawn afresh for every element.  This is not a step of the method:
a float32 implementation of the same loop carries relative errors of at
least that size, and copies of the loop perturbed this way show how far
such errors alone move its trajectory.  (Adam's normalised steps move a
parameter by about the learning rate whatever the size of its gradient, so
small differences grow once the loop oscillates near its optimum.)
"""
from __future__ import annotations

import numpy as np

from . import loss as oloss
from . import ntc as ontc
from . import optim as oopt
from . import raster as orc


def psnr(img, target) -> float:
    d = np.clip(np.asarray(img, np.float64), 0, 1) - np.clip(np.asarray(target, np.float64), 0, 1)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def _perturber(perturb):
    """The relative perturbation of `perturb` (identity for None)."""
    if perturb is None:
        return lambda a: a
    seed, rel = perturb
    rng = np.random.default_rng(seed)

    def apply(a):
        a = np.asarray(a, np.float64)
        return a * (1.0 + rel * rng.standard_normal(a.shape))
    return apply


def ntc_stage1(spec, params0, g, cams, targets, views, lam=0.2, lr=0.002, betas=(0.9, 0.99), eps=1e-15,
               held_cam=None, held_target=None, log_every=10, keep_params=0, perturb=None):
    """Run len(views) iterations from the float32 parameters params0.

    Returns a dict: loss per iteration; (iteration, held-out PSNR) every
    `log_every` iterations and at 0 when a held-out view is given; the
    float32 parameters after, the Adam moments (m, v) after, and the
    gradients of, each of the first `keep_params` iterations.
    """
    pert = _perturber(perturb)
    p = np.asarray(params0, np.float32).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    losses, log, kept, grads, moms = [], [], [], [], []

    def held_psnr():
        dmu, dq, _ = ontc.forward(spec, p, g.means)
        img = orc.render(g, held_cam, dmu.astype(np.float32), dq.astype(np.float32))["image"]
        return psnr(img, held_target)

    if held_cam is not None:
        log.append((0, held_psnr()))
    for t, view in enumerate(views, start=1):
        dmu, dq, cache = ontc.forward(spec, p, g.means)
        dmu32, dq32 = dmu.astype(np.float32), dq.astype(np.float32)     # the GPU hands float32 to the renderer
        cam = cams[view]
        img = pert(orc.render(g, cam, dmu32, dq32)["image"])
        L, dL = oloss.stage1_loss(img, np.asarray(targets[view], np.float64), lam)
        gr = orc.render_backward(g, cam, dL, dmu32, dq32)
        grad = pert(ontc.backward(spec, p, cache, gr["d_dmu"], gr["d_dq"]))
        p, m, v = oopt.adam(p, grad, m, v, t, lr, betas[0], betas[1], eps)
        p = p.astype(np.float32).astype(np.float64)
        losses.append(L)
        if t <= keep_params:
            kept.append(p.astype(np.float32))
            grads.append(grad)
            moms.append((m.copy(), v.copy()))
        if held_cam is not None and t % log_every == 0:
            log.append((t, held_psnr()))
    return {"loss": losses, "psnr": log, "params": kept, "grads": grads, "moments": moms}


def direct_stage1(g, cams, targets, views, lam=0.0, lr_mu=0.0024, lr_q=0.015, betas=(0.9, 0.999), eps=1e-15,
                  eval_cam=None, eval_target=None, log_every=10, keep_params=0, perturb=None):
    """The direct-optimisation comparator (Sec. 5.4, "Direct Opt."): per-
    Gaussian (dmu, dq) from (0, identity) trained with Adam (learning rates
    and betas of reading B7) on the same render and loss, float64, the
    parameters rounded to float32 after every step.  Returns the losses, the
    PSNR of eval_cam against eval_target every `log_every` iterations, and
    the parameters after, Adam moments ((m, v) of dmu, then of dq) after and
    gradients of the first `keep_params` iterations."""
    pert = _perturber(perturb)
    n = g.n
    dmu = np.zeros((n, 3))
    dq = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    m1, v1, m2, v2 = (np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 4)))
    losses, log, kept, grads, moms = [], [], [], [], []
    for t, view in enumerate(views, start=1):
        cam = cams[view]
        img = pert(orc.render(g, cam, dmu.astype(np.float32), dq.astype(np.float32))["image"])
        L, dL = oloss.stage1_loss(img, np.asarray(targets[view], np.float64), lam)
        gr = orc.render_backward(g, cam, dL, dmu.astype(np.float32), dq.astype(np.float32))
        g_mu, g_q = pert(gr["d_dmu"]), pert(gr["d_dq"])
        dmu, m1, v1 = oopt.adam(dmu, g_mu, m1, v1, t, lr_mu, betas[0], betas[1], eps)
        dq, m2, v2 = oopt.adam(dq, g_q, m2, v2, t, lr_q, betas[0], betas[1], eps)
        dmu, dq = dmu.astype(np.float32).astype(np.float64), dq.astype(np.float32).astype(np.float64)
        losses.append(L)
        if t <= keep_params:
            kept.append((dmu.astype(np.float32), dq.astype(np.float32)))
            grads.append((gr["d_dmu"], gr["d_dq"]))
            moms.append(((m1.copy(), v1.copy()), (m2.copy(), v2.copy())))
        if eval_cam is not None and t % log_every == 0:
            img = orc.render(g, eval_cam, dmu.astype(np.float32), dq.astype(np.float32))["image"]
            log.append((t, psnr(img, eval_target)))
    return {"loss": losses, "psnr": log, "params": kept, "grads": grads, "moments": moms}
