"""GPU tests of the boundary calls around the hot path, through the C ABI:
device NTC initialisation, checkpoints of the NTC training state, the
render counters, the preparation token, overflow reporting in the training
loops, and the autograd.Function wrappers."""
import math

import numpy as np
import pytest

from oracle import ntc as ontc
from oracle import raster as orc
from paper_2403_01444_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M64 = (1 << 64) - 1


def splitmix64_at(seed, i):
    """Output i of SplitMix64 seeded with `seed` (Steele, Lea and Flood
    2014): the mixing function applied to seed + (i + 1) * golden gamma."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ntc_ctx(n, precision="f32", cfg=None, **kw):
    from paper_2403_01444_amd import gs3
    return gs3.Context(n, 1 << 20, 64, 64, ntc=cfg or synth.NTCConfig(), precision=precision, **kw)


def test_splitmix64_reference_values():
    """The test's own SplitMix64 against the published first outputs of the
    generator seeded with 0 (its reference implementation's stream)."""
    assert splitmix64_at(0, 0) == 0xE220A8397B1DCDAF
    assert splitmix64_at(0, 1) == 0x6E789E6AA1B965F4
    assert splitmix64_at(0, 2) == 0x06C45D188009454F


def test_ntc_init_on_device():
    cfg = synth.NTCConfig()
    seed = 1234567
    ctx = ntc_ctx(10, "f16", cfg)
    ctx.ntc_init(seed)
    p = ctx.ntc_save()
    n_tab = cfg.num_table_params()
    n1, n2 = 64 * 32, 64 * 64
    segs = [(0, n_tab, 1e-4), (n_tab, n_tab + n1, math.sqrt(6 / 32)),
            (n_tab + n1, n_tab + n1 + n2, math.sqrt(6 / 64)), (n_tab + n1 + n2, p.size, math.sqrt(6 / 64))]
    assert segs[-1][1] == cfg.num_params()
    rng = np.random.default_rng(0)
    for a, b, bound in segs:
        # bit for bit against the generator's definition at sampled indices
        b32 = np.float32(bound)
        for i in np.concatenate([[a, b - 1], rng.integers(a, b, size=300)]):
            u = np.float32(splitmix64_at(seed, int(i)) >> 40) * np.float32(2.0 ** -24)
            want = np.float32(b32 * (np.float32(2) * u - np.float32(1)))
            assert p[i] == want, (i, p[i], want)
        # and the distribution U(-bound, bound): range, mean, variance, KS distance
        x = p[a:b].astype(np.float64) / bound
        assert np.all(np.abs(x) <= 1.0)
        m = x.size
        assert abs(x.mean()) < 5 / math.sqrt(3 * m) + 1e-12
        assert abs(x.var() - 1 / 3) < 5 * math.sqrt(4 / 45 / m)
        xs = np.sort(x)
        ks = np.max(np.abs(np.arange(1, m + 1) / m - (xs + 1) / 2))
        assert ks < 1.63 / math.sqrt(m) + 1.0 / m, ks          # 1% level
    # another seed gives another draw; the state is reset like ntc_load
    ctx.ntc_init(seed + 1)
    assert np.abs(ctx.ntc_save() - p).max() > 0
    assert float(ctx.ntc_grads().abs().max()) == 0.0
    ctx.close()


def _fixed_steps(ctx, means, tok, gm, gq, steps):
    for _ in range(steps):
        ctx.ntc_forward(means, token=tok)
        ctx.ntc_backward(means, gm, gq, tok)
        ctx.ntc_step(0.002, 0.9, 0.99, 1e-15)


def test_ntc_state_checkpoint_round_trip():
    """Three steps, save the state, load it into a fresh context: the loaded
    context saves back the identical blob (parameters, Adam moments, step).
    One more step on both with the same input gradient: the table part
    agrees bit for bit (its gradient has a fixed summation order; a lost step
    counter would change Adam's bias correction), the MLP part to float32
    rounding (its weight gradients are summed with atomics)."""
    from paper_2403_01444_amd import gs3
    n = 4000
    rng = np.random.default_rng(5)
    means = cuda(rng.uniform(-1.1, 1.1, size=(n, 3)).astype(np.float32))
    gm = cuda(rng.normal(size=(n, 3)).astype(np.float32) * 1e-3)
    gq = cuda(rng.normal(size=(n, 4)).astype(np.float32) * 1e-3)
    cfg = synth.NTCConfig()
    a = ntc_ctx(n, "f16", cfg)
    a.ntc_init(7)
    tok_a = a.ntc_prepare(means)
    _fixed_steps(a, means, tok_a, gm, gq, 3)
    blob = a.ntc_save_state()
    assert len(blob) == gs3.gs3_ntc_state_bytes(a.h) == 136 + 3 * 4 * cfg.num_params()
    b = ntc_ctx(n, "f16", cfg)
    b.ntc_load_state(blob)
    assert b.ntc_save_state() == blob
    tok_b = b.ntc_prepare(means)
    _fixed_steps(a, means, tok_a, gm, gq, 1)
    _fixed_steps(b, means, tok_b, gm, gq, 1)
    pa, pb = a.ntc_save(), b.ntc_save()
    t = cfg.num_table_params()
    assert np.array_equal(pa[:t], pb[:t])
    np.testing.assert_allclose(pb[t:], pa[t:], rtol=1e-5, atol=1e-7)
    # a checkpoint of another shape is refused
    small = synth.NTCConfig(log2_T=14)
    d = ntc_ctx(n, "f16", small)
    with pytest.raises(gs3.GS3Error) as e:
        d.ntc_load_state(blob[:gs3.gs3_ntc_state_bytes(d.h)])
    assert e.value.status == gs3.GS3_EINVAL
    for x in (a, b, d):
        x.close()


def test_preparation_token():
    from paper_2403_01444_amd import gs3
    n = 1000
    rng = np.random.default_rng(6)
    means = cuda(rng.uniform(-1, 1, size=(n, 3)).astype(np.float32))
    other = means.clone()
    ctx = ntc_ctx(n)
    ctx.ntc_init(1)
    t1 = ctx.ntc_prepare(means)
    assert t1 != 0
    ctx.ntc_forward(means, token=t1)
    with pytest.raises(gs3.GS3Error) as e:                 # other means under the token
        ctx.ntc_forward(other, token=t1)
    assert e.value.status == gs3.GS3_EINVAL
    t2 = ctx.ntc_prepare(other)
    assert t2 != t1
    g = ctx.zeros(n, 3), ctx.zeros(n, 4)
    with pytest.raises(gs3.GS3Error) as e:                 # a stale token
        ctx.ntc_backward(means, *g, t1)
    assert e.value.status == gs3.GS3_ESTATE
    ctx.ntc_backward(other, *g, t2)
    ctx.ntc_backward(means, *g, 0)                          # no token: the atomic scatter
    ctx.close()


def test_render_counters_match_the_pixel_state():
    """gs3_debug_counts' sums equal the per-pixel state summed on the host:
    sum over pixels of n_contrib (entries walked up to the last contributor)
    and, per 16 x 16 tile, the longest walk."""
    from paper_2403_01444_amd import gs3
    g, cams, _, _ = synth.workload("ring-50k-256px", seed=2)
    cam = synth.look_at_camera(250, 201)                   # ragged tiles
    ctx = gs3.Context(g.n, 1 << 24, 256, 256)
    gg = gs3.GaussiansGPU.from_host(g)
    assert ctx.debug_sums() == (-1, -1)                     # no render yet
    ctx.render(gg, cam)
    sc, walked = ctx.debug_sums()
    T, last = ctx.debug_pixels(cam)
    lastn = last.cpu().numpy().astype(np.int64)
    assert sc == int(lastn.sum()) and sc > 0
    th, tw = -(-cam.height // 16), -(-cam.width // 16)
    pad = np.zeros((th * 16, tw * 16), np.int64)
    pad[:cam.height, :cam.width] = lastn
    assert walked == int(pad.reshape(th, 16, tw, 16).max(axis=(1, 3)).sum())
    K, ov = ctx.debug_counts()
    assert K == orc.pair_count(g, cam) and ov == 0
    ctx.close()


def test_stage1_loop_reports_pair_overflow():
    """A Stage-1 run whose renders overflow the pair list (depth-first
    binning) raises GS3_ECAPACITY at the end of the run."""
    from paper_2403_01444_amd import gs3, train
    g, cams, _, nxt = synth.workload("small-2k-64px", seed=3)
    cam = cams[0]
    K = orc.pair_count(g, cam)
    cfg = synth.NTCConfig()
    ctx = gs3.Context(g.n, K // 3, 64, 64, ntc=cfg, precision="f32")
    ctx.ntc_init(0)
    gg = gs3.GaussiansGPU.from_host(g)
    target = torch.zeros(3, 64, 64, device="cuda")
    st = train.Stage1NTC(ctx, gg, [cam], [target])
    with pytest.raises(gs3.GS3Error) as e:
        st.run(2)
    assert e.value.status == gs3.GS3_ECAPACITY
    ctx.check_flags()                                        # the check cleared the flags
    ctx.close()


def test_autograd_wrappers_give_the_explicit_calls_gradient():
    """NTCQuery -> Render -> Loss with loss.backward() accumulates the same
    NTC gradient as the explicit calls and the same loss.  The table gradient
    is bit for bit the same (deterministic gradient records in the renderer,
    per-entry sums over the prepared contribution lists); the MLP weight
    gradient sums per-workgroup partials with float atomics, whose order
    varies, so it agrees to float32 summation order (1e-6 of its largest)."""
    from paper_2403_01444_amd import autograd as ag
    from paper_2403_01444_amd import gs3
    g, cams, _, nxt = synth.workload("small-2k-64px", seed=4)
    cam = cams[0]
    cfg = synth.NTCConfig()
    ctx = gs3.Context(g.n, 1 << 20, 64, 64, ntc=cfg, precision="f32", grad_record_log2=20)
    ctx.ntc_init(3)
    gg, gn = gs3.GaussiansGPU.from_host(g), gs3.GaussiansGPU.from_host(nxt)
    target = ctx.render(gn, cam).clone()
    tok = ctx.ntc_prepare(gg.means)
    # explicit calls
    dmu, dq = ctx.ntc_forward(gg.means, token=tok)
    img = ctx.render(gg, cam, dmu, dq)
    loss_e, d_img = ctx.loss(img, target, 0.2)
    grads = {"d_dmu": ctx.zeros(g.n, 3), "d_dq": ctx.zeros(g.n, 4)}
    ctx.render_backward(d_img, grads)
    ctx.ntc_backward(gg.means, grads["d_dmu"], grads["d_dq"], tok)
    ref = ctx.ntc_grads().cpu().numpy()
    ref_loss = loss_e.item()
    ctx.ntc_zero_grads()
    # the same through autograd
    anchor = ag.ntc_anchor()
    dmu2, dq2 = ag.NTCQuery.apply(anchor, ctx, gg.means, tok)
    img2 = ag.Render.apply(dmu2, dq2, ctx, gg, cam, 0)
    loss = ag.Loss.apply(img2, target, ctx, 0.2)
    loss.backward()
    got = ctx.ntc_grads().cpu().numpy()
    assert loss.item() == ref_loss
    t = ontc.NTCSpec(cfg).n_table
    assert np.array_equal(got[:t], ref[:t])
    assert np.abs(got[t:] - ref[t:]).max() <= 1e-6 * np.abs(ref[t:]).max()
    assert np.abs(ref[:t]).max() > 0 and np.abs(ref[t:]).max() > 0
    ctx.close()
