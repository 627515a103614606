"""Pins of the Stage-2 oracle (CPU only)."""
import math

import numpy as np

from oracle import stage2
from oracle import raster as orc
from paper_2403_01444_amd import synth


def test_vspace_gradient_uses_half_image_size_per_axis():
    # a unit pixel-space gradient along u is W/2 per NDC unit, along v H/2
    d = np.array([[1.0, 0.0], [0.0, 1.0], [3.0, 4.0]])
    v = stage2.vspace_grad(d, 100, 80)
    assert np.allclose(v, [50.0, 40.0, math.hypot(150.0, 160.0)])


def test_select_is_a_strict_threshold_on_the_visible_average():
    total = np.array([0.0, 3e-4, 2e-4, 1.5e-4, 9.0])
    count = np.array([0, 2, 1, 1, 0])
    # averages 1.5e-4 (not above), 2e-4, 1.5e-4 (not above); unseen ones excluded
    assert stage2.select(total, count, 1.5e-4).tolist() == [2]
    rng = np.random.default_rng(0)
    t, c = rng.uniform(0, 1e-3, 1000), rng.integers(0, 4, 1000)
    brute = [i for i in range(1000) if c[i] > 0 and t[i] / c[i] > 2e-4]
    assert stage2.select(t, c, 2e-4).tolist() == brute


def test_spawn_closed_form_for_identity_rotation_and_unit_scale():
    g = synth.make_gaussians(4, 1, seed=0)
    g.quats[:] = [2.0, 0.0, 0.0, 0.0]          # identity after normalisation
    g.log_scales[:] = 0.0
    z = np.arange(12, dtype=np.float64).reshape(4, 3) / 10
    m, q, ls, lo, sh = stage2.spawn(g, np.arange(4), z, "spawn")
    assert np.allclose(m, g.means + math.sqrt(2.0) * z)
    assert np.array_equal(q, np.tile([1.0, 0, 0, 0], (4, 1)))
    assert np.allclose(1 / (1 + np.exp(-lo)), 0.1)
    assert np.array_equal(sh, g.sh.astype(np.float64))


def test_spawn_samples_have_covariance_two_sigma():
    g = synth.make_gaussians(1, 0, seed=3)
    n = 200_000
    rng = np.random.default_rng(4)
    z = rng.normal(size=(n, 3))
    gi = g.subset(np.zeros(n, np.int64))
    m, *_ = stage2.spawn(gi, np.arange(n), z, "spawn")
    R = orc.quat_rot(g.quats[0] / np.linalg.norm(g.quats[0]))
    S = np.diag(np.exp(g.log_scales[0].astype(np.float64)))
    sigma = R @ S @ S.T @ R.T
    cov = np.cov((m - g.means[0]).T)
    assert np.abs(cov - 2 * sigma).max() < 0.02 * np.abs(2 * sigma).max()
    assert np.abs((m - g.means[0]).mean(0)).max() < 0.01 * math.sqrt(np.abs(sigma).max())


def test_split_keeps_rotation_and_opacity_and_shrinks_scale():
    g = synth.make_gaussians(5, 2, seed=5)
    z = np.zeros((5, 3))
    m, q, ls, lo, sh = stage2.spawn(g, np.arange(5), z, "split")
    assert np.allclose(m, g.means)
    assert np.array_equal(q, g.quats.astype(np.float64))
    assert np.allclose(np.exp(ls), 0.8 * np.exp(g.log_scales.astype(np.float64)))
    assert np.array_equal(lo, g.opacity_logits.astype(np.float64))


def test_keep_opaque_threshold():
    tau = 0.01
    l = np.array([math.log(tau / (1 - tau)) - 1e-9, math.log(tau / (1 - tau)) + 1e-9, 5.0, -10.0])
    assert stage2.keep_opaque(l, tau).tolist() == [1, 2]
