"""Stage-1 loops on the gs3 C ABI (Sec. 4.1).

Stage1NTC     one iteration = NTC query at every frozen mean (Eq. 5), transform
              and render one training view, loss of Eq. 6, backward through
              the renderer and the NTC, Adam on the NTC parameters.
Stage1Direct  the comparator of Sec. 5.4 ("Direct Opt."): per-Gaussian
              (dmu, dq) trained directly with the same renderer and loss.
warmup        the NTC warm-up of Eq. 7 on noise-augmented means.

Every step runs in libgs3.so; torch tensors only hold the buffers.  The
training views are visited in a seeded permutation per epoch.
"""
from __future__ import annotations

import math

import numpy as np

from . import gs3


class _Views:
    def __init__(self, count: int, seed: int):
        self.count = count
        self.rng = np.random.default_rng(seed)
        self.order: list[int] = []

    def next(self) -> int:
        if not self.order:
            self.order = list(self.rng.permutation(self.count))
        return int(self.order.pop(0))


class Stage1NTC:
    def __init__(self, ctx: gs3.Context, gauss: gs3.GaussiansGPU, cams, targets, lam: float = 0.2,
                 lr: float = 0.002, betas=(0.9, 0.99), eps: float = 1e-15, seed: int = 0):
        self.ctx, self.g, self.cams, self.targets = ctx, gauss, cams, targets
        self.lam, self.lr, self.betas, self.eps = lam, lr, betas, eps
        n = gauss.n
        self.dmu, self.dq = ctx.empty(n, 3), ctx.empty(n, 4)
        self.d_dmu, self.d_dq = ctx.zeros(n, 3), ctx.zeros(n, 4)
        H = max(c.height for c in cams)
        W = max(c.width for c in cams)
        self.img, self.dimg = ctx.empty(3 * H * W), ctx.empty(3 * H * W)
        self.loss = ctx.empty(1)
        self.views = _Views(len(cams), seed)
        # per-frame setup: the means stay frozen for the whole of Stage 1
        ctx.ntc_prepare(gauss.means)

    def step(self) -> int:
        ctx, cam = self.ctx, None
        v = self.views.next()
        cam = self.cams[v]
        P = 3 * cam.height * cam.width
        img, dimg = self.img[:P].view(3, cam.height, cam.width), self.dimg[:P].view(3, cam.height, cam.width)
        ctx.ntc_forward(self.g.means, self.dmu, self.dq)
        ctx.render(self.g, cam, self.dmu, self.dq, image=img)
        ctx.loss(img, self.targets[v], self.lam, loss=self.loss, d_image=dimg)
        ctx.zero(self.d_dmu, self.d_dq)
        ctx.render_backward(dimg, {"d_dmu": self.d_dmu, "d_dq": self.d_dq})
        ctx.ntc_backward(self.g.means, self.d_dmu, self.d_dq)
        ctx.ntc_step(self.lr, self.betas[0], self.betas[1], self.eps)
        return v

    def transform(self):
        self.ctx.ntc_forward(self.g.means, self.dmu, self.dq)
        return self.dmu, self.dq


class Stage1Direct:
    """Per-Gaussian translation and rotation optimised directly (float32)."""

    def __init__(self, ctx: gs3.Context, gauss: gs3.GaussiansGPU, cams, targets, lam: float = 0.2,
                 lr_mu: float = 0.0024, lr_q: float = 0.015, betas=(0.9, 0.999), eps: float = 1e-15, seed: int = 0):
        import torch
        self.ctx, self.g, self.cams, self.targets = ctx, gauss, cams, targets
        self.lam, self.lr_mu, self.lr_q, self.betas, self.eps = lam, lr_mu, lr_q, betas, eps
        n = gauss.n
        self.dmu = ctx.zeros(n, 3)
        self.dq = torch.tensor([1.0, 0.0, 0.0, 0.0], device=ctx.device).repeat(n, 1).contiguous()
        self.d_dmu, self.d_dq = ctx.zeros(n, 3), ctx.zeros(n, 4)
        self.m_mu, self.v_mu = ctx.zeros(n, 3), ctx.zeros(n, 3)
        self.m_q, self.v_q = ctx.zeros(n, 4), ctx.zeros(n, 4)
        H = max(c.height for c in cams)
        W = max(c.width for c in cams)
        self.img, self.dimg = ctx.empty(3 * H * W), ctx.empty(3 * H * W)
        self.loss = ctx.empty(1)
        self.views = _Views(len(cams), seed)
        self.t = 0

    def step(self) -> int:
        ctx = self.ctx
        v = self.views.next()
        cam = self.cams[v]
        P = 3 * cam.height * cam.width
        img, dimg = self.img[:P].view(3, cam.height, cam.width), self.dimg[:P].view(3, cam.height, cam.width)
        ctx.render(self.g, cam, self.dmu, self.dq, image=img)
        ctx.loss(img, self.targets[v], self.lam, loss=self.loss, d_image=dimg)
        ctx.zero(self.d_dmu, self.d_dq)
        ctx.render_backward(dimg, {"d_dmu": self.d_dmu, "d_dq": self.d_dq})
        self.t += 1
        ctx.adam(self.dmu, self.d_dmu, self.m_mu, self.v_mu, self.t, self.lr_mu, self.betas[0], self.betas[1], self.eps)
        ctx.adam(self.dq, self.d_dq, self.m_q, self.v_q, self.t, self.lr_q, self.betas[0], self.betas[1], self.eps)
        return v

    def transform(self):
        return self.dmu, self.dq


def warmup(ctx: gs3.Context, points, iters: int = 3000, lr: float = 0.002, betas=(0.9, 0.99), eps: float = 1e-15):
    """Eq. 7: drive the NTC towards the identity transform on `points`."""
    n = points.shape[0]
    dmu, dq = ctx.empty(n, 3), ctx.empty(n, 4)
    loss = ctx.empty(1)
    gmu, gq = ctx.empty(n, 3), ctx.empty(n, 4)
    ctx.ntc_prepare(points)          # the warm-up points stay fixed
    for _ in range(iters):
        ctx.ntc_forward(points, dmu, dq)
        gs3.gs3_warmup_loss(ctx.h, dmu, dq, loss, gmu, gq)
        ctx.ntc_backward(points, gmu, gq)
        ctx.ntc_step(lr, betas[0], betas[1], eps)
    return loss


def psnr(img, target) -> float:
    """10 log10(1 / MSE) on images clamped to [0, 1]."""
    d = (img.clamp(0, 1) - target.clamp(0, 1)).double()
    mse = float((d * d).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def logged_run(step, evaluate, iters: int, every: int = 10):
    """Run `step` iters times; every `every` iterations record (iterations,
    training seconds so far, evaluate()).  Training time is measured over
    synchronised blocks of `every` steps and excludes the evaluations."""
    import time

    import torch
    log = []
    t_train = 0.0
    done = 0
    while done < iters:
        k = min(every, iters - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            step()
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        done += k
        log.append((done, t_train, evaluate()))
    return log


def equal_psnr(ntc_log, direct_log, ntc_iters: int = 150, slack_db: float = 0.1):
    """Two equal-PSNR comparisons of logs of (iterations, training seconds,
    held-out PSNR).  (a) NTC at `ntc_iters` iterations reaches P*; the direct
    optimiser's time to reach P* - slack (None if it never does).  (b) The
    level both reach, min(best NTC, best direct) - slack, and each method's
    time to its first logged point at or above it."""
    at = [r for r in ntc_log if r[0] == ntc_iters]
    if not at:
        raise ValueError("the NTC log has no point at the requested iteration")
    _, t_ntc, p_star = at[0]
    hit = [r for r in direct_log if r[2] >= p_star - slack_db]
    d_same = [r for r in direct_log if r[0] == ntc_iters]
    common = min(max(r[2] for r in ntc_log), max(r[2] for r in direct_log)) - slack_db
    first = lambda log: next(r for r in log if r[2] >= common)
    fn, fd = first(ntc_log), first(direct_log)
    return {
        "ntc_iters": ntc_iters, "ntc_psnr_at_iters": p_star, "ntc_seconds": t_ntc,
        "direct_iters_to_match": hit[0][0] if hit else None,
        "direct_seconds_to_match": hit[0][1] if hit else None,
        "direct_psnr_at_same_iters": d_same[0][2] if d_same else None,
        "direct_seconds_at_same_iters": d_same[0][1] if d_same else None,
        "ntc_best_psnr": max(r[2] for r in ntc_log),
        "direct_best_psnr": max(r[2] for r in direct_log),
        "common_psnr": common,
        "ntc_iters_to_common": fn[0], "ntc_seconds_to_common": fn[1],
        "direct_iters_to_common": fd[0], "direct_seconds_to_common": fd[1],
    }
