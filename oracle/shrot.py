"""SH rotation and the per-frame transform bake, float64 numpy (test
infrastructure only).

Suppl. Sec. B: rotating a vector before projecting it onto the SH gives the
same as projecting first and rotating the SH, M P(N) = P(R N).  With
A = [P(N_0), ..., P(N_{2l})] for 2l+1 fixed directions, M = [P(R N_0), ...,
P(R N_{2l})] A^{-1}.  The paper uses band 1 with N = e_x, e_y, e_z; the same
construction is applied here to each band l <= 3 with 2l+1 directions that
make A invertible (reading A3).  The coefficient vector of band l is turned
by M_l(dR), dR = R(q') R(q^)^T, so that the colour in direction d after the
bake equals the colour before it in direction dR^T d.
"""
from __future__ import annotations

import numpy as np

from . import raster as orc


def band_directions(l: int) -> np.ndarray:
    """2l+1 unit directions used for band l (e_x, e_y, e_z for band 1)."""
    if l == 1:
        return np.eye(3)
    # golden-angle spiral with an asymmetric start (offset 0.2): the
    # symmetric choice 0.5 makes A singular for band 3; with 0.2 the
    # condition numbers are about 11 (band 2) and 6 (band 3)
    k = 2 * l + 1
    i = np.arange(k) + 0.2
    z = 1 - 2 * i / k
    phi = np.pi * (1 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def band_basis(l: int, dirs: np.ndarray) -> np.ndarray:
    """(2l+1) x len(dirs) matrix of the band-l basis at the directions."""
    cols = []
    for d in dirs:
        Y, _ = orc.sh_basis(3, d / np.linalg.norm(d))
        cols.append(Y[l * l:(l + 1) * (l + 1)])
    return np.stack(cols, axis=1)


def band_matrix(l: int, R: np.ndarray) -> np.ndarray:
    """M_l(R) with M_l(R) P_l(N) = P_l(R N)."""
    if l == 0:
        return np.ones((1, 1))
    N = band_directions(l)
    A = band_basis(l, N)
    B = band_basis(l, N @ np.asarray(R, np.float64).T)
    return B @ np.linalg.inv(A)


def bake(g, dmu, dq):
    """Transformed means, rotations and SH of a Gaussian set (float64)."""
    n = g.n
    K = (g.sh_degree + 1) ** 2
    mu = g.means.astype(np.float64) + (0 if dmu is None else np.asarray(dmu, np.float64))
    q = g.quats.astype(np.float64)
    qh = q / np.linalg.norm(q, axis=1, keepdims=True)
    out_q = np.zeros((n, 4))
    out_sh = g.sh.astype(np.float64).copy()
    for i in range(n):
        if dq is None:
            out_q[i] = qh[i]
            continue
        d = np.asarray(dq[i], np.float64)
        dh = d / max(np.linalg.norm(d), 1e-12)
        qp = orc.quat_mul(qh[i], dh)
        out_q[i] = qp
        dR = orc.quat_rot(qp) @ orc.quat_rot(qh[i]).T
        for l in range(1, g.sh_degree + 1):
            M = band_matrix(l, dR)
            out_sh[i, l * l:(l + 1) * (l + 1), :] = M @ out_sh[i, l * l:(l + 1) * (l + 1), :]
    return mu, out_q, out_sh
