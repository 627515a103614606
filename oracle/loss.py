"""Stage-1 loss oracle, float64 numpy (test infrastructure only).

Eq. 6: L = (1 - lambda) L1 + lambda L_D-SSIM with lambda = 0.2 (Sec. 4.1).
Readings where the paper is silent: L1 is the mean absolute difference over
the 3 x H x W image (subgradient sign(0) = 0); D-SSIM = 1 - mean SSIM, SSIM
computed per channel with an 11 x 11 Gaussian window of sigma 1.5, zero
padding ("same" output size), C1 = 0.01^2, C2 = 0.03^2 (the 3DG-S
convention the paper follows).
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    k = np.arange(size) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def filter2d(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """'same' 2D correlation of an (H, W) image with zero padding."""
    r = w.shape[0] // 2
    H, W = img.shape
    p = np.zeros((H + 2 * r, W + 2 * r))
    p[r:r + H, r:r + W] = img
    out = np.zeros((H, W))
    for dy in range(w.shape[0]):
        for dx in range(w.shape[1]):
            out += w[dy, dx] * p[dy:dy + H, dx:dx + W]
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray):
    """Per-channel local statistics and the SSIM map of (3, H, W) images."""
    w = window()
    mx = np.stack([filter2d(c, w) for c in x])
    my = np.stack([filter2d(c, w) for c in y])
    sxx = np.stack([filter2d(c, w) for c in x * x]) - mx * mx
    syy = np.stack([filter2d(c, w) for c in y * y]) - my * my
    sxy = np.stack([filter2d(c, w) for c in x * y]) - mx * my
    a1 = 2 * mx * my + C1
    a2 = 2 * sxy + C2
    b1 = mx * mx + my * my + C1
    b2 = sxx + syy + C2
    return dict(mx=mx, my=my, a1=a1, a2=a2, b1=b1, b2=b2, ssim=(a1 * a2) / (b1 * b2))


def l1(x, y):
    d = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    return np.abs(d).mean(), np.sign(d) / d.size


def dssim(x, y):
    """(1 - mean SSIM, its gradient with respect to x)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    t = ssim_terms(x, y)
    S = t["ssim"]
    a1, a2, b1, b2, mx, my = t["a1"], t["a2"], t["b1"], t["b2"], t["mx"], t["my"]
    # SSIM at a pixel as a function of the filtered maps mu_x, E[x^2], E[xy]
    dS_da1 = a2 / (b1 * b2)
    dS_da2 = a1 / (b1 * b2)
    dS_db1 = -S / b1
    dS_db2 = -S / b2
    # a1 = 2 mx my + C1; a2 = 2 (Exy - mx my) + C2; b1 = mx^2 + my^2 + C1;
    # b2 = (Exx - mx^2) + (Eyy - my^2) + C2
    d_mx = dS_da1 * 2 * my + dS_da2 * (-2 * my) + dS_db1 * 2 * mx + dS_db2 * (-2 * mx)
    d_exx = dS_db2
    d_exy = dS_da2 * 2
    w = window()
    n = x.size
    gx = np.stack([filter2d(d_mx[c], w) + 2 * x[c] * filter2d(d_exx[c], w) + y[c] * filter2d(d_exy[c], w)
                   for c in range(x.shape[0])])
    return 1.0 - S.mean(), -gx / n


def stage1_loss(x, y, lam: float = 0.2):
    """(L, dL/dx) for L = (1 - lam) L1 + lam D-SSIM; lam = 0 gives plain L1."""
    a, ga = l1(x, y)
    if lam == 0.0:
        return a, ga
    b, gb = dssim(x, y)
    return (1 - lam) * a + lam * b, (1 - lam) * ga + lam * gb
