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
                 lr: float = 0.002, betas=(0.9, 0.99), eps: float = 1e-15, seed: int = 0,
                 views_per_step: int = 1):
        if not 1 <= views_per_step <= len(cams):
            raise ValueError(f"views_per_step must be in [1, {len(cams)}]")
        self.ctx, self.g, self.cams, self.targets = ctx, gauss, cams, targets
        self.lam, self.lr, self.betas, self.eps = lam, lr, betas, eps
        self.views_per_step = views_per_step
        n = gauss.n
        self.dmu, self.dq = ctx.empty(n, 3), ctx.empty(n, 4)
        self.d_dmu, self.d_dq = ctx.zeros(n, 3), ctx.zeros(n, 4)
        H = max(c.height for c in cams)
        W = max(c.width for c in cams)
        self.img, self.dimg = ctx.empty(3 * H * W), ctx.empty(3 * H * W)
        self.loss = ctx.empty(views_per_step)   # per view of the last step
        self.views = _Views(len(cams), seed)
        # per-frame setup: the means stay frozen for the whole of Stage 1
        self.token = ctx.ntc_prepare(gauss.means)

    def accumulate(self, views, track=None):
        """NTC gradient of the summed loss over `views`: one NTC query, then
        per view render, loss and renderer backward, the (dmu, dq) gradients
        of all views summed, and one NTC backward.  With one view this is the
        paper's iteration; with several it is the multi-view batch, which
        queries and back-propagates the NTC once per batch.  (Adam's update is
        unchanged by a constant gradient scale apart from eps, so the sum and
        the mean over the views step alike.)"""
        ctx = self.ctx
        ctx.ntc_forward(self.g.means, self.dmu, self.dq, self.token)
        ctx.zero(self.d_dmu, self.d_dq)
        grads = {"d_dmu": self.d_dmu, "d_dq": self.d_dq}
        if track is not None:
            grads["vspace_grad"], grads["vspace_count"] = track
        for k, v in enumerate(views):
            cam = self.cams[v]
            P = 3 * cam.height * cam.width
            img, dimg = self.img[:P].view(3, cam.height, cam.width), self.dimg[:P].view(3, cam.height, cam.width)
            ctx.render(self.g, cam, self.dmu, self.dq, image=img)
            ctx.loss(img, self.targets[v], self.lam, loss=self.loss[k:k + 1], d_image=dimg)
            ctx.render_backward(dimg, grads)
        ctx.ntc_backward(self.g.means, self.d_dmu, self.d_dq, self.token)

    def step(self, track=None):
        """One iteration over `views_per_step` views of the epoch's
        permutation (returns the view, or the list of views).  `track` =
        (vspace_grad, vspace_count) accumulates the view-space gradient
        statistics Stage 2 selects from."""
        vs = [self.views.next() for _ in range(self.views_per_step)]
        self.accumulate(vs, track)
        self.ctx.ntc_step(self.lr, self.betas[0], self.betas[1], self.eps)
        return vs[0] if self.views_per_step == 1 else vs

    def run(self, iters: int):
        """`iters` iterations; the view-space gradient statistics of the last
        epoch (the iterations that cover the last len(views) views) are
        returned for Stage 2.  Raises GS3Error (GS3_ECAPACITY /
        GS3_ENONFINITE) when a render of the run overflowed its pair list or a
        loss was not finite: the run's results are then not the method's."""
        n = self.g.n
        vg, vc = self.ctx.zeros(n), self.ctx.zeros(n)
        last = min(iters, -(-len(self.cams) // self.views_per_step))
        for it in range(iters):
            self.step((vg, vc) if it >= iters - last else None)
        self.ctx.check_flags()
        return vg, vc

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

    def run(self, iters: int):
        """`iters` iterations, then the device flags are checked (GS3Error on
        a pair-list overflow or a non-finite loss)."""
        for _ in range(iters):
            self.step()
        self.ctx.check_flags()


class Stage2:
    """Adaptive 3DG addition (Sec. 4.2).  Additional Gaussians are spawned
    around the frame's (transformed, baked) Gaussians whose average view-space
    gradient over the last Stage-1 epoch exceeds tau_grad, at positions drawn
    from N(mu, 2 Sigma), with the source's SH and scale, identity rotation and
    opacity 0.1.  Only the additional Gaussians are optimised, with the same
    loss as Stage 1 and 3DG-S's per-attribute learning rates (Suppl. A).  At
    the end of each epoch, additional Gaussians above tau_grad are split
    (rotation, SH, opacity kept, 80% scale) and those below opacity tau_alpha
    are discarded.  The additional Gaussians belong to this frame only."""

    LR = {"means": 0.0024, "sh": 0.0375, "opacity_logits": 0.75, "log_scales": 0.075, "quats": 0.015}
    ATTRS = ("means", "quats", "log_scales", "opacity_logits", "sh")

    def __init__(self, ctx: gs3.Context, base: gs3.GaussiansGPU, cams, targets, vgrad, vcount, lam: float = 0.2,
                 tau_grad: float = 0.00015, tau_alpha: float = 0.01, max_add: int | None = None, seed: int = 0,
                 betas=(0.9, 0.999), eps: float = 1e-15):
        import torch
        self.ctx, self.base, self.cams, self.targets = ctx, base, cams, targets
        self.lam, self.tau_grad, self.betas, self.eps = lam, tau_grad, betas, eps
        self.logit_alpha = float(np.float32(math.log(tau_alpha / (1.0 - tau_alpha))))
        self.rng = np.random.default_rng(seed)
        self.max_add = max_add
        self.views = _Views(len(cams), seed + 1)
        idx = ctx.select(vgrad, vcount, tau_grad)
        idx = self._cap(idx, 0)
        z = torch.from_numpy(self.rng.normal(size=(int(idx.numel()), 3)).astype(np.float32)).to(ctx.device)
        add = ctx.spawn(base, idx, z, gs3.GS3_SPAWN)
        self.spawned = int(idx.numel())
        self._set(add, None)
        H = max(c.height for c in cams)
        W = max(c.width for c in cams)
        self.img, self.dimg = ctx.empty(3 * H * W), ctx.empty(3 * H * W)
        self.loss = ctx.empty(1)
        self.t = 0
        self.it = 0

    def _cap(self, idx, current):
        if self.max_add is not None and idx.numel() + current > self.max_add:
            idx = idx[: max(self.max_add - current, 0)]
        return idx

    def _set(self, add: gs3.GaussiansGPU, state):
        """Union [base | add] with its Adam state (state: previous m, v rows
        of `add`, or None for zeros) and fresh view-space statistics."""
        import torch
        ctx, b = self.ctx, self.base
        self.n_base, self.m = b.n, add.n
        self.all = gs3.GaussiansGPU(*(torch.cat([getattr(b, a), getattr(add, a)]).contiguous() for a in self.ATTRS),
                                    b.sh_degree)
        self.grad = {a: torch.zeros_like(getattr(self.all, a)) for a in self.ATTRS}
        if state is None:
            state = {a: (torch.zeros_like(getattr(add, a)), torch.zeros_like(getattr(add, a))) for a in self.ATTRS}
        self.state = state
        self.vg, self.vc = ctx.zeros(self.n_base + self.m), ctx.zeros(self.n_base + self.m)

    def added(self) -> gs3.GaussiansGPU:
        return gs3.GaussiansGPU(*(getattr(self.all, a)[self.n_base:] for a in self.ATTRS), self.all.sh_degree)

    def step(self) -> int:
        ctx = self.ctx
        v = self.views.next()
        cam = self.cams[v]
        P = 3 * cam.height * cam.width
        img, dimg = self.img[:P].view(3, cam.height, cam.width), self.dimg[:P].view(3, cam.height, cam.width)
        ctx.render(self.all, cam, image=img)
        ctx.loss(img, self.targets[v], self.lam, loss=self.loss, d_image=dimg)
        if self.m:
            ctx.zero(*self.grad.values())
            g = {"d_means": self.grad["means"], "d_quats": self.grad["quats"],
                 "d_log_scales": self.grad["log_scales"], "d_opacity_logits": self.grad["opacity_logits"],
                 "d_sh": self.grad["sh"], "vspace_grad": self.vg, "vspace_count": self.vc}
            ctx.render_backward(dimg, g)
            self.t += 1
            nb = self.n_base
            for a in self.ATTRS:
                p = getattr(self.all, a)[nb:]
                m_, v_ = self.state[a]
                ctx.adam(p, self.grad[a][nb:], m_, v_, self.t, self.LR[a], self.betas[0], self.betas[1], self.eps)
        self.it += 1
        if self.it % len(self.cams) == 0:
            self.control()
        return v

    def run(self, iters: int):
        """`iters` iterations, then the device flags are checked (GS3Error on
        a pair-list overflow, which Stage 2's growth can cause, or a
        non-finite loss)."""
        for _ in range(iters):
            self.step()
        self.ctx.check_flags()

    def control(self):
        """Quantity control at the end of an epoch: split the additional
        Gaussians above tau_grad, then drop those below opacity tau_alpha."""
        import torch
        if self.m == 0:
            return
        ctx, nb = self.ctx, self.n_base
        add = self.added()
        idx = ctx.select(self.vg[nb:].contiguous(), self.vc[nb:].contiguous(), self.tau_grad)
        idx = self._cap(idx, self.m)
        z = torch.from_numpy(self.rng.normal(size=(int(idx.numel()), 3)).astype(np.float32)).to(ctx.device)
        new = ctx.spawn(add, idx, z, gs3.GS3_SPLIT)
        merged = gs3.GaussiansGPU(*(torch.cat([getattr(add, a), getattr(new, a)]).contiguous() for a in self.ATTRS),
                                  add.sh_degree)
        state = {a: tuple(torch.cat([s, torch.zeros_like(getattr(new, a))]).contiguous() for s in self.state[a])
                 for a in self.ATTRS}
        keep = ctx.select(merged.opacity_logits, None, self.logit_alpha)
        kept = gs3.GaussiansGPU(*(ctx.take_rows(getattr(merged, a), keep) for a in self.ATTRS), add.sh_degree)
        state = {a: tuple(ctx.take_rows(s, keep) for s in state[a]) for a in self.ATTRS}
        self._set(kept, state)


def warmup(ctx: gs3.Context, points, iters: int = 3000, lr: float = 0.002, betas=(0.9, 0.99), eps: float = 1e-15):
    """Eq. 7: drive the NTC towards the identity transform on `points`."""
    n = points.shape[0]
    dmu, dq = ctx.empty(n, 3), ctx.empty(n, 4)
    loss = ctx.empty(1)
    gmu, gq = ctx.empty(n, 3), ctx.empty(n, 4)
    tok = ctx.ntc_prepare(points)    # the warm-up points stay fixed
    for _ in range(iters):
        ctx.ntc_forward(points, dmu, dq, tok)
        gs3.gs3_warmup_loss(ctx.h, dmu, dq, loss, gmu, gq)
        ctx.ntc_backward(points, gmu, gq, tok)
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
