"""Free-viewpoint video streaming loop (Sec. 4, Fig. 2) on the gs3 C ABI.

Per frame: Stage 1 trains the NTC on the frame's training views (the NTC
starts from the warm-up parameters, which the paper stores once and uses to
initialise every following timestep; Sec. 4.1), the learned transform is
baked into the Gaussians carried to the next frame (means, rotations and SH,
`gs3_transform_bake`), Stage 2 adds frame-specific Gaussians (Sec. 4.2) that
are used for this frame's views only, and the novel views are rendered.

`synthetic_sequence` yields the ground-truth scene of each frame for the
seeded capture-like scene: the objects move a little every frame and new
objects appear at given frames.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import gs3, synth, train


def synthetic_sequence(scene: synth.SurfaceScene, frames: int, seed: int, new_objects=(100, 200),
                       n_obj: int = 2000):
    """Ground truth of frames 1..frames (frame 0 is `scene` itself)."""
    cur = synth.SurfaceScene(scene.gaussians, scene.labels, scene.centres)
    centres = [(-0.35, 0.0, -0.35), (0.3, 0.25, -0.4), (0.0, -0.3, -0.5), (-0.2, 0.35, -0.3)]
    added = 0
    for f in range(1, frames + 1):
        g = synth.object_motion(cur, seed + f)
        labels = cur.labels
        if f in new_objects:
            g = synth.emerging_object(g, seed + 10_000 + f, n_obj=n_obj, centre=centres[added % len(centres)])
            labels = np.concatenate([labels, np.zeros(n_obj, np.int64)])   # new objects stay put
            added += 1
        cur = synth.SurfaceScene(g, labels, cur.centres)
        yield f, g


@dataclass
class FrameResult:
    frame: int
    stage1_s: float
    stage2_s: float
    spawned: int
    additional: int
    psnr_stage1: float      # novel views, carried Gaussians only
    psnr_stage2: float      # novel views, with the additional Gaussians
    render_fps: float       # novel views of the frame's full set


class StreamTrainer:
    def __init__(self, ctx: gs3.Context, g0: gs3.GaussiansGPU, train_cams, novel_cams, cfg: synth.NTCConfig,
                 warmup_iters: int = 3000, stage1_iters: int = 150, stage2_iters: int = 100,
                 max_add: int = 100_000, seed: int = 0):
        import torch
        self.ctx, self.g, self.cams, self.novel = ctx, g0, train_cams, novel_cams
        self.s1, self.s2, self.max_add, self.seed = stage1_iters, stage2_iters, max_add, seed
        ctx.ntc_load(synth.ntc_init_params(cfg, seed))
        pts = torch.from_numpy(synth.warmup_points(g0.means.cpu().numpy(), cfg, seed + 1)).to(ctx.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        train.warmup(ctx, pts, warmup_iters)
        torch.cuda.synchronize()
        self.warmup_s = time.perf_counter() - t0
        self.warm = ctx.ntc_save()

    def frame(self, f: int, targets, novel_targets) -> FrameResult:
        import torch
        ctx = self.ctx
        ctx.ntc_load(self.warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st1 = train.Stage1NTC(ctx, self.g, self.cams, targets, seed=self.seed + f)
        vg, vc = st1.run(self.s1)
        baked = ctx.transform_bake(self.g, *st1.transform())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2 = train.Stage2(ctx, baked, self.cams, targets, vg, vc, max_add=self.max_add, seed=self.seed + f)
        st2.run(self.s2)
        self.last_stage2 = st2
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p1 = float(np.mean([train.psnr(ctx.render(baked, c), t) for c, t in zip(self.novel, novel_targets)]))
        p2 = float(np.mean([train.psnr(ctx.render(st2.all, c), t) for c, t in zip(self.novel, novel_targets)]))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            for c in self.novel:
                ctx.render(st2.all, c)
        torch.cuda.synchronize()
        fps = reps * len(self.novel) / (time.perf_counter() - t3)
        res = FrameResult(f, t1 - t0, t2 - t1, st2.spawned, st2.m, p1, p2, fps)
        self.g = baked          # the additional Gaussians belong to this frame only
        return res


def novel_cameras(width: int, height: int):
    """Four novel views between the training arc's cameras."""
    return [synth.look_at_camera(width, height, azimuth_deg=a, elevation_deg=e)
            for a, e in ((-20.0, 4.0), (-6.0, -3.0), (8.0, 3.0), (21.0, -4.0))]
