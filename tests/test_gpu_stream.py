"""Streaming loop over frames: Stage 1, bake, Stage 2, novel views."""
import numpy as np
import pytest

from paper_2403_01444_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_three_frame_stream_with_an_appearing_object():
    """100K capture-like Gaussians, 8 training views at 640x480, 4 novel
    views; a new object appears at frame 2.  The carried set keeps its size
    (additional Gaussians are frame-specific), Stage 2 recovers the new
    object at that frame, and the baked carry-over keeps the novel views
    close to the ground truth across frames."""
    from paper_2403_01444_amd import gs3, stream
    cfg = synth.NTCConfig()
    sc = synth.surface_scene(100_000, 3, 5)
    cams = synth.arc_cameras(8, 640, 480)
    novel = stream.novel_cameras(640, 480)
    cap = 50_000
    ctx = gs3.Context(sc.gaussians.n + cap + 4000, 1 << 25, 640, 480, ntc=cfg, precision="f16")
    g0 = gs3.GaussiansGPU.from_host(sc.gaussians)
    tr = stream.StreamTrainer(ctx, g0, cams, novel, cfg, warmup_iters=1000, max_add=cap)
    res = []
    for f, gt in stream.synthetic_sequence(sc, 3, 7, new_objects=(2,)):
        gtg = gs3.GaussiansGPU.from_host(gt)
        targets = [ctx.render(gtg, c).clone() for c in cams]
        novel_t = [ctx.render(gtg, c).clone() for c in novel]
        res.append(tr.frame(f, targets, novel_t))
        assert tr.g.n == sc.gaussians.n
    assert [r.frame for r in res] == [1, 2, 3]
    r2 = res[1]
    assert r2.spawned > 0 and r2.psnr_stage2 > r2.psnr_stage1 + 0.3, r2
    assert all(r.psnr_stage1 > 28.0 for r in res), res
    assert all(r.render_fps > 0 for r in res)
    ctx.close()


def test_two_frames_track_the_oracle_stream():
    """Two frames of the streaming loop (Stage 1 with view-space tracking,
    bake, Stage 2 with spawn, Adam and quantity control, novel views) on the
    GPU beside the oracle's own loop (oracle/stream.py), 3,000 capture-like
    Gaussians (SH degree 1), four 64 x 64 arc views, a new 300-Gaussian
    object at frame 2, float32 NTC from seeded parameters, 4 Stage-1 and 8
    Stage-2 iterations (two epochs, two quantity-control steps) per frame.
    Each side carries its own baked Gaussians into the next frame, and so do
    four copies of the oracle's stream whose Stage 1 is perturbed by
    float32-sized relative noise (1e-6 on the image and gradient of every
    iteration): their distance from the oracle is how far rounding alone
    moves the stream, and widens each bar below.

    * Stage 1 of the first frame, which both sides start from the same
      Gaussians: NTC parameters after the frame's iterations within 1e-3 of
      lr where the oracle's gradient stood clear of rounding noise (>= 1e-3
      of its tensor's largest) in every iteration and the perturbed copies
      agree with the oracle to 1e-4 of lr.  (Later frames start from each
      side's own carried Gaussians; the outcomes below bound them.)
    * Spawned counts equal up to the Gaussians whose oracle view-space
      average lies within 1e-3 of tau_grad (single precision may decide
      those either way); the additional set after quantity control within
      that many plus 2%.  Both also widened by the perturbed copies'
      largest distance from the oracle's count: from the second frame on,
      each stream starts from its own carried Gaussians, and rounding alone
      moves the oracle's added count there by tens (1020-1101 against 1047
      over eight copies of this configuration).
    * The carried (baked) Gaussians: means within 1e-5, quaternions within
      1e-4, SH within 1e-4 of the largest coefficient, each plus the
      perturbed copies' largest distance from the oracle.
    * Novel-view PSNR, carried Gaussians alone and with the frame's
      additional ones, within 0.1 dB of the oracle's plus the copies'
      spread."""
    from oracle import ntc as ontc
    from oracle import raster as orc
    from oracle import stream as ostream
    from paper_2403_01444_amd import gs3, stream, train
    cfg = synth.NTCConfig()
    spec = ontc.NTCSpec(cfg)
    sc = synth.surface_scene(3000, 1, 5)
    cams = synth.arc_cameras(4, 64, 64)
    novel = [synth.look_at_camera(64, 64, azimuth_deg=a, elevation_deg=e) for a, e in ((-12.0, 3.0), (9.0, -2.0))]
    seed, s1, s2, cap, n_members = 3, 4, 8, 2000, 4
    ctx = gs3.Context(sc.gaussians.n + cap + 600, 1 << 22, 64, 64, ntc=cfg, precision="f32")
    tr = stream.StreamTrainer(ctx, gs3.GaussiansGPU.from_host(sc.gaussians), cams, novel, cfg, warmup_iters=0,
                              stage1_iters=s1, stage2_iters=s2, max_add=cap, seed=seed)
    warm = synth.ntc_init_params(cfg, seed)
    g0 = sc.gaussians
    og = ostream.Gaussians(g0.means, g0.quats, g0.log_scales, g0.opacity_logits, g0.sh, g0.sh_degree)
    ogs = [og] * n_members
    lr = 0.002
    novel_psnr = lambda gs, nt: np.mean([ostream.psnr(orc.render(gs, c)["image"], t) for c, t in zip(novel, nt)])
    for f, gt in stream.synthetic_sequence(sc, 2, 7, new_objects=(2,), n_obj=300):
        targets = [orc.render(gt, c)["image"].astype(np.float32) for c in cams]
        ntargets = [orc.render(gt, c)["image"].astype(np.float32) for c in novel]
        print(f"[stream] frame {f}", flush=True)
        res = tr.frame(f, [torch.from_numpy(t).cuda() for t in targets],
                       [torch.from_numpy(t).cuda() for t in ntargets])
        run = lambda start, perturb=None: ostream.frame(
            spec, warm, start, cams, targets, synth.view_schedule(len(cams), s1, seed + f),
            synth.view_schedule(len(cams), s2, seed + f + 1), np.random.default_rng(seed + f), s2, max_add=cap,
            perturb=perturb)
        fo = run(og)
        fm = [run(ogs[k], (10 * f + k + 1, 1e-6)) for k in range(n_members)]
        # Stage 1
        meas = np.ones(warm.size, bool)
        t = spec.n_table
        for _, gr in fo["params"]:
            for a, b in ((0, t), (t, warm.size)):
                meas[a:b] &= np.abs(gr[a:b]) >= 1e-3 * np.abs(gr[a:b]).max()
        ref_p = fo["params"][-1][0].astype(np.float64)
        for m in fm:
            meas &= np.abs(m["params"][-1][0] - ref_p) <= 1e-4 * lr
        got = ctx.ntc_save()
        err = np.abs(got.astype(np.float64) - ref_p)[meas].max() / lr
        print(f"[stream] frame {f}: Stage-1 parameter error {err:.2e} x lr over {meas.mean():.4f}", flush=True)
        if f == 1:
            assert err <= 1e-3
        # Stage-2 decisions: the oracle's averages clear of the threshold
        vg, vc = fo["vspace"]
        avg = np.where(vc > 0, vg / np.maximum(vc, 1), 0.0)
        near = int((np.abs(avg[vc > 0] / 0.00015 - 1) < 1e-3).sum())
        st2 = tr.last_stage2
        print(f"[stream] frame {f}: spawned {res.spawned} (oracle {fo['spawned']}), additional {st2.m} "
              f"(oracle {fo['added'].n}), {near} averages within 1e-3 of the threshold", flush=True)
        sp_spread = max(abs(m["spawned"] - fo["spawned"]) for m in fm)
        add_spread = max(abs(m["added"].n - fo["added"].n) for m in fm)
        print(f"[stream] frame {f}: copies' spread spawned {sp_spread}, added {add_spread}", flush=True)
        assert abs(res.spawned - fo["spawned"]) <= near + sp_spread
        assert abs(st2.m - fo["added"].n) <= near + 0.02 * fo["added"].n + add_spread
        # the carried Gaussians
        b = tr.g
        shmax = np.abs(fo["baked"].sh).max()
        for name, base in (("means", 1e-5), ("quats", 1e-4), ("sh", 1e-4 * shmax)):
            ref = getattr(fo["baked"], name)
            spread = max(float(np.abs(getattr(m["baked"], name) - ref).max()) for m in fm)
            e = float(np.abs(getattr(b, name).cpu().numpy() - ref).max())
            print(f"[stream] frame {f}: carried {name} error {e:.2e}, bar {base:.1e} + copies' spread {spread:.2e}",
                  flush=True)
            assert e <= base + spread, (name, e, spread)
        # novel views
        p1 = np.mean([train.psnr(ctx.render(b, c), torch.from_numpy(t).cuda()) for c, t in zip(novel, ntargets)])
        p2 = np.mean([train.psnr(ctx.render(st2.all, c), torch.from_numpy(t).cuda())
                      for c, t in zip(novel, ntargets)])
        r1, r2 = novel_psnr(fo["baked"], ntargets), novel_psnr(fo["all"], ntargets)
        m1 = [novel_psnr(m["baked"], ntargets) for m in fm]
        m2 = [novel_psnr(m["all"], ntargets) for m in fm]
        bar1 = 0.1 + max(m1 + [r1]) - min(m1 + [r1])
        bar2 = 0.1 + max(m2 + [r2]) - min(m2 + [r2])
        print(f"[stream] frame {f}: novel PSNR carried {p1:.3f} / {r1:.3f} (bar {bar1:.3f}), with additional "
              f"{p2:.3f} / {r2:.3f} (bar {bar2:.3f})", flush=True)
        assert abs(p1 - r1) <= bar1 and abs(p2 - r2) <= bar2
        og = fo["baked"]
        ogs = [m["baked"] for m in fm]
    ctx.close()
