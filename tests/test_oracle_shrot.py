"""Pins of the SH-rotation / transform-bake oracle (CPU only)."""
import numpy as np

from oracle import raster as orc
from oracle import shrot
from paper_2403_01444_amd import synth


def rand_rot(rng):
    q = rng.normal(size=4)
    return orc.quat_rot(q / np.linalg.norm(q))


def sh_eval(c, d, l):
    Y, _ = orc.sh_basis(3, d)
    return Y[l * l:(l + 1) * (l + 1)] @ c


def test_rotated_coefficients_equal_rotated_direction():
    """f_{M c}(d) = f_c(R^T d) for every band: the rotation invariance of the
    band-l function space (Suppl. Sec. B, M P(N) = P(R N))."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        R = rand_rot(rng)
        for l in range(4):
            M = shrot.band_matrix(l, R)
            c = rng.normal(size=2 * l + 1)
            for _ in range(5):
                d = rng.normal(size=3)
                d /= np.linalg.norm(d)
                assert abs(sh_eval(M @ c, d, l) - sh_eval(c, R.T @ d, l)) < 1e-11


def test_band_matrices_orthogonal_and_multiplicative():
    rng = np.random.default_rng(1)
    for _ in range(10):
        R1, R2 = rand_rot(rng), rand_rot(rng)
        for l in range(1, 4):
            M1, M2, M12 = shrot.band_matrix(l, R1), shrot.band_matrix(l, R2), shrot.band_matrix(l, R1 @ R2)
            np.testing.assert_allclose(M1 @ M1.T, np.eye(2 * l + 1), atol=1e-11)
            np.testing.assert_allclose(M12, M1 @ M2, atol=1e-11)
    assert np.array_equal(shrot.band_matrix(0, rand_rot(rng)), np.ones((1, 1)))
    np.testing.assert_allclose(shrot.band_matrix(2, np.eye(3)), np.eye(5), atol=1e-12)


def test_bake_then_render_equals_transformed_render():
    """Rendering the baked Gaussians without a transform reproduces the render
    of the originals with (dmu, dq)."""
    g, _, _, _ = synth.workload("grad-200-32px", seed=3)
    cam = synth.look_at_camera(32, 32)
    rng = np.random.default_rng(4)
    dmu = (rng.normal(size=(g.n, 3)) * 0.02).astype(np.float32)
    dq = (np.array([1, 0, 0, 0]) + rng.normal(size=(g.n, 4)) * 0.3).astype(np.float32)
    mu, q, sh = shrot.bake(g, dmu, dq)
    baked = g.subset(slice(None))
    baked.means, baked.quats, baked.sh = mu.astype(np.float32), q.astype(np.float32), sh.astype(np.float32)
    a = orc.render(g, cam, dmu, dq)
    b = orc.render(baked, cam)
    ok = ~(a["ambiguous"].astype(bool) | b["ambiguous"].astype(bool))
    assert np.abs(a["image"] - b["image"])[:, ok].max() < 2e-5
