"""Adam and the NTC warm-up loss, float64 numpy (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def adam(param, grad, m, v, step: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam step with bias correction (Kingma & Ba); returns (param, m, v).

    The NTC is trained with Adam at lr 0.002 (Suppl. Sec. A); the betas and
    epsilon are not stated there and are arguments here.
    """
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def warmup_loss(dmu, dq):
    """Eq. 7 averaged over points: mean ||dmu||_1 - mean cos^2(norm(dq), Q).

    Q = (1, 0, 0, 0) is the identity quaternion, so cos(norm(dq), Q) is
    dq_w / ||dq||; squaring removes the double cover (Sec. 4.1).  A zero dq
    contributes cos^2 = 0 and no gradient.  Returns (L, dL/ddmu, dL/ddq).
    """
    dmu = np.asarray(dmu, np.float64)
    dq = np.asarray(dq, np.float64)
    n = dmu.shape[0]
    n2 = (dq * dq).sum(axis=1)
    ok = n2 > 0
    cos2 = np.where(ok, dq[:, 0] ** 2 / np.where(ok, n2, 1.0), 0.0)
    L = np.abs(dmu).sum(axis=1).mean() - cos2.mean()
    g_mu = np.sign(dmu) / n
    g_q = np.zeros_like(dq)
    safe = np.where(ok, n2, 1.0)
    w = dq[:, 0]
    g_q[:, 0] = 2 * w * (n2 - w * w) / (safe * safe)
    for k in range(1, 4):
        g_q[:, k] = -2 * w * w * dq[:, k] / (safe * safe)
    g_q[~ok] = 0.0
    g_q = -g_q / n
    return L, g_mu, g_q
