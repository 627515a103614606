"""Pins of the oracle's analytic adjoint (CPU only):
  * float64 central finite differences of the oracle's own forward pass;
  * an independent naive renderer written here in PyTorch float64 whose
    gradient comes from autograd, on a handful of Gaussians."""
import math

import numpy as np
import pytest
import torch

from oracle import raster as orc
from paper_2403_01444_amd import synth

GRAD_KEYS = ("means", "quats", "log_scales", "opacity_logits", "sh", "dmu", "dq")


def fd_scene(n=24, size=32, seed=0, sh_degree=3):
    """Small scene that avoids kinks: opacity < 0.99, colours away from 0, no J clamp."""
    rng = np.random.default_rng(seed)
    g = synth.make_gaussians(n, sh_degree, seed)
    g.means[:] = rng.uniform(-0.6, 0.6, size=(n, 3)).astype(np.float32)
    g.log_scales[:] = rng.normal(-2.2, 0.2, size=(n, 3)).astype(np.float32)
    g.opacity_logits[:] = rng.uniform(-1.0, 1.5, size=n).astype(np.float32)
    dc = rng.uniform(0.25, 0.75, size=(n, 3))
    g.sh[:, 0, :] = ((dc - 0.5) / (0.5 / math.sqrt(math.pi))).astype(np.float32)
    cam = synth.look_at_camera(size, size, bg=(0.1, 0.2, 0.3))
    dmu = (rng.normal(size=(n, 3)) * 0.02).astype(np.float32)
    dq = (np.array([1, 0, 0, 0]) + rng.normal(size=(n, 4)) * 0.2).astype(np.float32)
    return g, cam, dmu, dq


def _arrays(g, dmu, dq):
    return dict(means=g.means, quats=g.quats, log_scales=g.log_scales, opacity_logits=g.opacity_logits,
                sh=g.sh, dmu=dmu, dq=dq)


def _signature(g, cam, dmu, dq):
    pre = orc.preprocess(g, cam, dmu, dq)
    r = orc.render(g, cam, dmu, dq)
    return pre["visible"].tobytes() + pre["box"].tobytes() + r["n_contrib"].tobytes(), r


def clamp_scene(n=24, size=32, seed=0, sh_degree=3, frac=0.5):
    """Scene whose first frac * n Gaussians sit beyond 1.3 x the half-FOV
    tangent in x or y (camera space), where the EWA Jacobian takes the
    clamped coordinate (reading C4), and are large enough that their pixel
    boxes still reach into the image."""
    rng = np.random.default_rng(seed)
    g = synth.make_gaussians(n, sh_degree, seed)
    cam = synth.look_at_camera(size, size, bg=(0.1, 0.2, 0.3))
    W = np.asarray(cam.world_to_cam, np.float64)
    R, t = W[:, :3], W[:, 3]
    lim = 0.5 * size / cam.fx
    z = rng.uniform(2.6, 3.4, size=n)
    xy = rng.uniform(-0.5, 0.5, size=(n, 2)) * lim * z[:, None]
    k = int(round(frac * n))
    ax = np.arange(k) % 2                        # every (axis, side) case appears
    sg = np.where((np.arange(k) // 2) % 2, 1.0, -1.0)
    off = rng.uniform(1.35, 1.6, size=k) * lim
    for i in range(k):
        xy[i, ax[i]] = sg[i] * off[i] * z[i]
    tc = np.concatenate([xy, z[:, None]], 1)
    g.means[:] = ((tc - t) @ R).astype(np.float32)
    ls = rng.normal(-2.2, 0.2, size=(n, 3))
    ls[:k] = rng.normal(-1.0, 0.15, size=(k, 3))
    g.log_scales[:] = ls.astype(np.float32)
    g.opacity_logits[:] = rng.uniform(-1.0, 1.5, size=n).astype(np.float32)
    dc = rng.uniform(0.25, 0.75, size=(n, 3))
    g.sh[:, 0, :] = ((dc - 0.5) / (0.5 / math.sqrt(math.pi))).astype(np.float32)
    dmu = (rng.normal(size=(n, 3)) * 0.02).astype(np.float32)
    dq = (np.array([1, 0, 0, 0]) + rng.normal(size=(n, 4)) * 0.2).astype(np.float32)
    return g, cam, dmu, dq


def clamped_mask(g, cam, dmu):
    """Gaussians whose camera-space x/z or y/z lies beyond 1.3 x the half-FOV
    tangent and that are visible (their box reaches the image)."""
    W = np.asarray(cam.world_to_cam, np.float64)
    tc = (g.means.astype(np.float64) + dmu) @ W[:, :3].T + W[:, 3]
    clx = np.abs(tc[:, 0] / tc[:, 2]) > 1.3 * 0.5 * cam.width / cam.fx
    cly = np.abs(tc[:, 1] / tc[:, 2]) > 1.3 * 0.5 * cam.height / cam.fy
    return (clx | cly) & orc.preprocess(g, cam, dmu, None)["visible"].astype(bool)


def _check_central_differences(g, cam, dmu, dq, seed, per_key=60, min_checked=300, only=None):
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(3, cam.height, cam.width))
    grads = orc.render_backward(g, cam, w, dmu, dq)
    sig0, _ = _signature(g, cam, dmu, dq)
    h = 1e-4
    checked = 0
    for key in GRAD_KEYS:
        arr = _arrays(g, dmu, dq)[key]
        flat = arr.reshape(-1)
        gflat = grads["d_" + key].reshape(-1)
        scale = np.abs(gflat).max() + 1e-30
        rows = np.arange(flat.size) // (flat.size // g.n)
        pool = np.arange(flat.size) if only is None else np.nonzero(only[rows])[0]
        for j in rng.choice(pool, size=min(pool.size, per_key), replace=False):
            x0 = flat[j]
            flat[j] = np.float32(x0 + h)
            sp, rp = _signature(g, cam, dmu, dq)
            xp = float(flat[j])
            flat[j] = np.float32(x0 - h)
            sm, rm = _signature(g, cam, dmu, dq)
            xm = float(flat[j])
            flat[j] = x0
            if sp != sig0 or sm != sig0:
                continue   # a discrete decision moved: no derivative there
            fd = float(np.sum(w * (rp["image"] - rm["image"]))) / (xp - xm)
            err = abs(fd - gflat[j]) / scale
            assert err < 1e-5, (key, j, fd, gflat[j])
            checked += 1
    assert checked > min_checked, checked


def test_adjoint_matches_central_differences():
    g, cam, dmu, dq = fd_scene()
    _check_central_differences(g, cam, dmu, dq, 1)


def test_adjoint_matches_central_differences_with_clamped_jacobian():
    """Half the Gaussians beyond the J clamp (reading C4): the forward takes
    the clamped coordinate and the adjoint has no term through it.  The
    components checked belong to the clamped Gaussians only."""
    g, cam, dmu, dq = clamp_scene(seed=3)
    cl = clamped_mask(g, cam, dmu)
    assert cl.sum() >= g.n // 3, cl.sum()
    _check_central_differences(g, cam, dmu, dq, 4, only=cl, min_checked=250)


# ---------------------------------------------------------------------------
# independent naive renderer (PyTorch float64 + autograd)
# ---------------------------------------------------------------------------

def _hamilton(a, b):
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


def _rotation(q):
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _sh_basis(d):
    x, y, z = d.unbind(-1)
    pi = math.pi
    c1 = math.sqrt(3 / (4 * pi))
    a, b, e = 0.5 * math.sqrt(15 / pi), 0.25 * math.sqrt(5 / pi), 0.25 * math.sqrt(15 / pi)
    f, h = 0.25 * math.sqrt(35 / (2 * pi)), 0.5 * math.sqrt(105 / pi)
    s, t, u = 0.25 * math.sqrt(21 / (2 * pi)), 0.25 * math.sqrt(7 / pi), 0.25 * math.sqrt(105 / pi)
    return torch.stack([torch.full_like(x, 0.5 / math.sqrt(pi)),
                        -c1 * y, c1 * z, -c1 * x,
                        a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, e * (x * x - y * y),
                        -f * y * (3 * x * x - y * y), h * x * y * z, -s * y * (4 * z * z - x * x - y * y),
                        t * z * (2 * z * z - 3 * x * x - 3 * y * y), -s * x * (4 * z * z - x * x - y * y),
                        u * z * (x * x - y * y), -f * x * (x * x - 3 * y * y)], -1)


def torch_render(t, cam, pre):
    """t: dict of float64 leaf tensors.  Discrete decisions (visibility, box,
    depth order) come from the oracle; everything continuous is autograd."""
    W = torch.tensor(np.asarray(cam.world_to_cam, np.float64))
    m = t["means"] + t["dmu"]
    qh = t["quats"] / t["quats"].norm(dim=-1, keepdim=True)
    dh = t["dq"] / t["dq"].norm(dim=-1, keepdim=True)
    qp = _hamilton(qh, dh)
    Rp, Rh = _rotation(qp), _rotation(qh)
    S = torch.diag_embed(torch.exp(t["log_scales"]))
    M = Rp @ S
    Sig = M @ M.transpose(-1, -2)
    tc = m @ W[:, :3].T + W[:, 3]
    tx, ty, tz = tc.unbind(-1)
    limx = 1.3 * 0.5 * cam.width / cam.fx
    limy = 1.3 * 0.5 * cam.height / cam.fy
    txc = torch.clamp(tx / tz, -limx, limx)
    tyc = torch.clamp(ty / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([cam.fx / tz, zero, -cam.fx * txc / tz], -1),
                     torch.stack([zero, cam.fy / tz, -cam.fy * tyc / tz], -1)], -2)
    T = J @ W[:, :3]
    S2 = T @ Sig @ T.transpose(-1, -2) + 0.3 * torch.eye(2, dtype=torch.float64)
    conic = torch.linalg.inv(S2)
    u = cam.fx * tx / tz + cam.cx
    v = cam.fy * ty / tz + cam.cy
    op = torch.sigmoid(t["opacity_logits"])
    wv = m - torch.tensor(np.asarray(cam.cam_pos, np.float64))
    dirv = wv / wv.norm(dim=-1, keepdim=True)
    Mloc = Rh @ Rp.transpose(-1, -2)
    dloc = (Mloc @ dirv.unsqueeze(-1)).squeeze(-1)
    Y = _sh_basis(dloc)[:, :t["sh"].shape[1]]
    rgb = torch.relu((Y.unsqueeze(-1) * t["sh"]).sum(1) + 0.5)
    H, Wd = cam.height, cam.width
    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(Wd, dtype=torch.float64),
                            indexing="ij")
    Tr = torch.ones(H, Wd, dtype=torch.float64)
    col = torch.zeros(3, H, Wd, dtype=torch.float64)
    done = torch.zeros(H, Wd, dtype=torch.bool)
    vis = np.nonzero(pre["visible"])[0]
    order = vis[np.lexsort((vis, pre["key"][vis]))]
    for i in order:
        x0, y0, x1, y1 = pre["box"][i]
        inbox = (xs >= x0) & (xs <= x1) & (ys >= y0) & (ys <= y1)
        dx, dy = xs - u[i], ys - v[i]
        power = -0.5 * (conic[i, 0, 0] * dx * dx + conic[i, 1, 1] * dy * dy) - conic[i, 0, 1] * dx * dy
        alpha = torch.clamp(op[i] * torch.exp(power), max=0.99)
        with torch.no_grad():
            cand = inbox & ~done & (power <= 0) & (alpha >= 1 / 255)
            stop = cand & (Tr * (1 - alpha) < 1e-4)
            act = cand & ~stop
            done = done | stop
        col = col + torch.where(act, alpha * Tr, torch.zeros_like(Tr)).unsqueeze(0) * rgb[i].view(3, 1, 1)
        Tr = torch.where(act, Tr * (1 - alpha), Tr)
    bg = torch.tensor(np.asarray(cam.bg, np.float64)).view(3, 1, 1)
    return col + Tr.unsqueeze(0) * bg


def test_adjoint_matches_torch_autograd():
    g, cam, dmu, dq = fd_scene(n=10, size=24, seed=7)
    pre = orc.preprocess(g, cam, dmu, dq)
    t = {k: torch.tensor(np.asarray(a, np.float64), requires_grad=True) for k, a in _arrays(g, dmu, dq).items()}
    img = torch_render(t, cam, pre)
    ref = orc.render(g, cam, dmu, dq)
    np.testing.assert_allclose(img.detach().numpy(), ref["image"], atol=1e-12)
    w = np.random.default_rng(2).normal(size=img.shape)
    (img * torch.tensor(w)).sum().backward()
    grads = orc.render_backward(g, cam, w, dmu, dq)
    for k in GRAD_KEYS:
        a = t[k].grad.numpy()
        b = grads["d_" + k]
        np.testing.assert_allclose(b, a, atol=1e-10 * (1 + np.abs(a).max()), err_msg=k)


def test_adjoint_matches_torch_autograd_with_clamped_jacobian():
    """The independent renderer clamps x/z and y/z with torch.clamp, whose
    gradient through a clamped coordinate is zero: the oracle's image and
    adjoint agree on a scene where a third or more of the Gaussians are
    clamped (a dropped clamp moves both)."""
    g, cam, dmu, dq = clamp_scene(n=12, size=24, seed=8)
    cl = clamped_mask(g, cam, dmu)
    assert cl.sum() >= g.n // 3, cl.sum()
    pre = orc.preprocess(g, cam, dmu, dq)
    t = {k: torch.tensor(np.asarray(a, np.float64), requires_grad=True) for k, a in _arrays(g, dmu, dq).items()}
    img = torch_render(t, cam, pre)
    ref = orc.render(g, cam, dmu, dq)
    np.testing.assert_allclose(img.detach().numpy(), ref["image"], atol=1e-12)
    w = np.random.default_rng(3).normal(size=img.shape)
    (img * torch.tensor(w)).sum().backward()
    grads = orc.render_backward(g, cam, w, dmu, dq)
    for k in GRAD_KEYS:
        a = t[k].grad.numpy()
        b = grads["d_" + k]
        np.testing.assert_allclose(b, a, atol=1e-10 * (1 + np.abs(a).max()), err_msg=k)
        # the clamped Gaussians carry real gradient (they are not just culled)
        assert np.abs(a[cl]).max() > 1e-6, k
