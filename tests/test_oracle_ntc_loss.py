"""Pins of the NTC, loss and optimiser oracles (CPU only)."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

from oracle import loss as oloss
from oracle import ntc as ontc
from oracle import optim as oopt
from paper_2403_01444_amd import synth


@pytest.fixture(scope="module")
def spec():
    return ontc.NTCSpec(synth.NTCConfig())


def test_resolution_table():
    # b^5 = 4, b^10 = 16, b^15 = 64 exactly: a naive floor would give 63, 255, 1023
    assert synth.NTCConfig().resolutions() == [16, 21, 27, 36, 48, 64, 84, 111, 147, 194, 256, 337,
                                               445, 588, 776, 1024]
    sizes = synth.NTCConfig().level_sizes()
    assert sizes[:3] == [17 ** 3, 22 ** 3, 28 ** 3] and all(s == 2 ** 15 for s in sizes[3:])


def test_hash_vertex_reproduction_and_partition_of_unity(spec):
    rng = np.random.default_rng(0)
    table = rng.normal(size=(int(spec.offsets[-1]), spec.F))
    # a point on a level-0 lattice vertex returns that vertex's entry exactly
    N = spec.res[0]
    v = np.array([[3, 5, 7]])
    x = (v / N) / spec.inv_ext.astype(np.float64) + spec.aabb_min
    x32 = x.astype(np.float32)
    inside, rows, wts = ontc.corners(spec, x32)
    w = wts[0][0]
    assert abs(w.sum() - 1) < 1e-12
    k = int(np.argmax(w))
    assert w[k] > 1 - 1e-5
    assert rows[0][0, k] == 3 + 17 * (5 + 17 * 7)
    # weights sum to one at random points and every level
    pts = rng.uniform(-1.1, 1.1, size=(500, 3)).astype(np.float32)
    inside, rows, wts = ontc.corners(spec, pts)
    for l in range(spec.L):
        np.testing.assert_allclose(wts[l].sum(1), 1.0, atol=1e-12)
        assert rows[l].min() >= spec.offsets[l] and rows[l].max() < spec.offsets[l + 1]


def test_dense_index_injective(spec):
    N = spec.res[2]
    g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    idx = g[:, 0] + (N + 1) * (g[:, 1] + (N + 1) * g[:, 2])
    assert len(np.unique(idx)) == (N + 1) ** 3


def test_encoding_continuous_across_cell_faces(spec):
    rng = np.random.default_rng(1)
    table = rng.normal(size=(int(spec.offsets[-1]), spec.F))
    N = spec.res[4]
    base = np.array([0.37, 0.52, 0.61])
    face = (np.floor(base * N) + 1) / N          # x lies on a face of level 4's lattice
    pts = []
    for eps in (-1e-6, 1e-6):
        xn = np.array([face[0] + eps, base[1], base[2]])
        pts.append(xn / spec.inv_ext.astype(np.float64) + spec.aabb_min)
    enc, *_ = ontc.encode(spec, table, np.asarray(pts, np.float32))
    lvl = slice(2 * 4, 2 * 5)
    assert np.abs(enc[0, lvl] - enc[1, lvl]).max() < 1e-3 * np.abs(table).max()


def test_gather_scatter_dot_product(spec):
    """<E(table), g> = <table, E^T(g)> for the (linear) encoding map E."""
    rng = np.random.default_rng(2)
    cfg = synth.NTCConfig()
    params = synth.ntc_init_params(cfg, 0).astype(np.float64)
    params[:spec.n_table] = rng.normal(size=spec.n_table)
    table, *_ = spec.split(params)
    pts = rng.uniform(-1.2, 1.2, size=(300, 3)).astype(np.float32)
    enc, inside, rows, wts = ontc.encode(spec, table, pts)
    gr = rng.normal(size=enc.shape)
    gr[~inside] = 0
    dt = np.zeros_like(table)
    for l in range(spec.L):
        for c in range(8):
            np.add.at(dt, rows[l][:, c], wts[l][:, c:c + 1] * gr[:, 2 * l:2 * l + 2])
    assert abs(np.sum(enc * gr) - np.sum(table * dt)) < 1e-9 * np.abs(np.sum(enc * gr)).max()


def test_ntc_forward_backward_vs_torch_autograd(spec):
    cfg = synth.NTCConfig()
    rng = np.random.default_rng(3)
    params = synth.ntc_init_params(cfg, 1).astype(np.float64)
    params[:spec.n_table] = rng.normal(scale=0.1, size=spec.n_table)
    pts = rng.uniform(-1.3, 1.3, size=(400, 3)).astype(np.float32)    # some outside the AABB
    dmu, dq, cache = ontc.forward(spec, params, pts)
    d_dmu, d_dq = rng.normal(size=dmu.shape), rng.normal(size=dq.shape)
    grad = ontc.backward(spec, params, cache, d_dmu, d_dq)
    # independent formulation: gather with torch indexing, linear layers, autograd
    P = torch.tensor(params, requires_grad=True)
    table_t, W1, W2, W3 = P[:spec.n_table].view(-1, 2), *[None] * 3
    k = spec.n_table
    W1 = P[k:k + 64 * 32].view(64, 32); k += 64 * 32
    W2 = P[k:k + 64 * 64].view(64, 64); k += 64 * 64
    W3 = P[k:k + 7 * 64].view(7, 64)
    inside, rows, wts = ontc.corners(spec, pts)
    enc = torch.cat([sum(torch.tensor(wts[l][:, c:c + 1]) * table_t[torch.tensor(rows[l][:, c])]
                         for c in range(8)) for l in range(spec.L)], dim=1)
    out = Fnn.linear(Fnn.relu(Fnn.linear(Fnn.relu(Fnn.linear(enc, W1)), W2)), W3)
    ins = torch.tensor(inside)
    np.testing.assert_allclose(dmu[inside], out[ins, :3].detach().numpy(), atol=1e-12)
    np.testing.assert_allclose(dq[inside], out[ins, 3:].detach().numpy(), atol=1e-12)
    assert np.all(dmu[~inside] == 0) and np.all(dq[~inside] == [1, 0, 0, 0])
    g = torch.cat([torch.tensor(d_dmu), torch.tensor(d_dq)], 1) * ins[:, None]
    (out * g).sum().backward()
    np.testing.assert_allclose(grad, P.grad.numpy(), atol=1e-10)


def test_storage_rounding():
    x = np.array([1.0 + 2 ** -12, 1.0 + 3 * 2 ** -12, 3e-5, 1.0 / 3])
    h = ontc.round_storage(x, "f16")
    assert h[0] == 1.0 and h[1] == 1.0 + 2 ** -10           # round half to even
    assert np.all(ontc.round_storage(h, "f16") == h)
    b = ontc.round_storage(x, "bf16")
    assert np.all(ontc.round_storage(b, "bf16") == b) and b[0] == 1.0
    s = ontc.round_significand(np.array([1e-9 * (1 + 2 ** -12)]), "f16")
    assert s[0] == 1e-9 * 1.0 or abs(s[0] / 1e-9 - 1) <= 2 ** -11


# ---------------------------------------------------------------------------
# loss (Eq. 6)
# ---------------------------------------------------------------------------

def torch_ssim(x, y):
    g = torch.exp(-(torch.arange(11, dtype=torch.float64) - 5) ** 2 / (2 * 1.5 ** 2))
    g = g / g.sum()
    w = (g[:, None] * g[None, :]).expand(3, 1, 11, 11).contiguous()
    f = lambda a: Fnn.conv2d(a[None], w, padding=5, groups=3)[0]
    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def test_ssim_identities_and_torch_reference():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(3, 23, 31))
    y = np.clip(x + rng.normal(scale=0.1, size=x.shape), 0, 1)
    d, _ = oloss.dssim(x, x)
    assert abs(d) < 1e-12
    assert oloss.l1(x, x)[0] == 0
    xt = torch.tensor(x, requires_grad=True)
    s = torch_ssim(xt, torch.tensor(y)).mean()
    (1 - s).backward()
    d, gd = oloss.dssim(x, y)
    assert abs(d - (1 - s.item())) < 1e-12
    np.testing.assert_allclose(gd, xt.grad.numpy(), atol=1e-13)
    L, gL = oloss.stage1_loss(x, y, 0.2)
    assert abs(L - (0.8 * np.abs(x - y).mean() + 0.2 * d)) < 1e-14


# ---------------------------------------------------------------------------
# Adam and warm-up (Eq. 7)
# ---------------------------------------------------------------------------

def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p, g = rng.normal(size=100), rng.normal(size=100)
    p1, m, v = oopt.adam(p, g, np.zeros(100), np.zeros(100), 1, 0.002, 0.9, 0.99, 1e-15)
    np.testing.assert_allclose(p1, p - 0.002 * g / (np.abs(g) + 1e-15), rtol=1e-12)
    # second step against torch.optim.Adam
    t = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([t], lr=0.002, betas=(0.9, 0.99), eps=1e-15)
    g2 = rng.normal(size=100)
    for gg in (g, g2):
        opt.zero_grad()
        t.grad = torch.tensor(gg)
        opt.step()
    p2, _, _ = oopt.adam(p1, g2, m, v, 2, 0.002, 0.9, 0.99, 1e-15)
    np.testing.assert_allclose(p2, t.detach().numpy(), rtol=1e-10, atol=1e-15)


def test_warmup_fixed_point_and_gradient():
    n = 50
    dmu = np.zeros((n, 3))
    dq = np.zeros((n, 4))
    dq[:, 0] = np.where(np.arange(n) % 2, 1.5, -0.7)       # +-Q, any length
    L, gm, gq = oopt.warmup_loss(dmu, dq)
    assert L == -1.0 and np.all(gq == 0)
    rng = np.random.default_rng(1)
    dmu, dq = rng.normal(size=(n, 3)), rng.normal(size=(n, 4))
    a, b = torch.tensor(dmu, requires_grad=True), torch.tensor(dq, requires_grad=True)
    cos = b[:, 0] / b.norm(dim=1)
    Lt = a.abs().sum(1).mean() - (cos * cos).mean()
    Lt.backward()
    L, gm, gq = oopt.warmup_loss(dmu, dq)
    assert abs(L - Lt.item()) < 1e-13
    np.testing.assert_allclose(gm, a.grad.numpy(), atol=1e-15)
    np.testing.assert_allclose(gq, b.grad.numpy(), atol=1e-14)
