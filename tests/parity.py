"""Shared parity checks of the GPU tests against the oracle."""
import numpy as np

from oracle import raster as orc


def check_image(img, T, ref, label, tol=1e-4):
    """Image and final transmittance against the oracle's render, every
    pixel: each pixel takes whichever of the oracle's two outcomes of the
    transmittance cut-off fits it (the decision single precision can take
    either way; elsewhere the two are equal).  Image error <= tol x the
    largest image value, transmittance error <= tol.  Prints the measured
    share of pixels whose cut-off was within reach, and how many took the
    alternative; returns them."""
    img = img.detach().cpu().numpy() if hasattr(img, "detach") else img
    T = T.detach().cpu().numpy() if hasattr(T, "detach") else T
    err, terr, alt, unres = orc.image_error(img, ref, T)
    amb = (ref["ambiguous"] & 2) > 0
    P = amb.size
    scale = np.abs(ref["image"]).max()
    ok = ~unres
    e = float(err[ok].max() / scale) if ok.any() else 0.0
    te = float(terr[ok].max()) if (ok.any() and terr is not None) else 0.0
    print(f"[parity] {label}: cut-off within reach at {int(amb.sum())} of {P} pixels ({amb.mean():.2e}), "
          f"{int(alt.sum())} matched the alternative, {int(unres.sum())} unresolved; "
          f"image error {e:.2e} (bar {tol:g}), transmittance error {te:.2e}", flush=True)
    assert not (alt & ~amb).any()
    assert unres.sum() <= 1e-5 * P, int(unres.sum())
    assert e <= tol, e
    assert te <= tol, te
    return float(amb.mean()), int(alt.sum())


def check_grads(grads, ref, label, tol=1e-3, keys=None):
    """Max-norm relative gradient error per tensor over every Gaussian, and
    over the Gaussians that reach no pixel with a decision within reach;
    the bar applies to the latter.  Prints both and the share set aside."""
    touched = ref["touched_ambiguous"].astype(bool)
    keep = ~touched
    for k in keys or grads.keys():
        v = grads[k]
        a = v.detach().cpu().numpy().astype(np.float64) if hasattr(v, "detach") else np.asarray(v, np.float64)
        b = ref[k]
        s_all = max(np.abs(b).max(), 1e-30)
        e_all = float(np.abs(a - b).max() / s_all)
        e_keep = float(np.abs(a[keep] - b[keep]).max() / max(np.abs(b[keep]).max(), 1e-30)) if keep.any() else 0.0
        print(f"[parity] {label} {k}: error {e_keep:.2e} over {keep.mean():.4f} of the Gaussians, "
              f"{e_all:.2e} over all (bar {tol:g})", flush=True)
        assert e_keep < tol, (k, e_keep)


def adam_determined(m_prev, v_prev, step, g, lr, b1, b2, eps, delta, tol):
    """Parameters whose Adam step (Kingma and Ba, bias-corrected; moments
    m_prev, v_prev before step number `step`) moves by at most `tol` when
    their gradient g moves by up to `delta` (probed at g +- delta and
    g +- delta / 2).  Adam normalises each step to about lr, so a parameter
    whose gradient is within reach of zero, or whose first moment nearly
    cancels, can step either way on a gradient error of that size; the
    parameter comparisons of the trajectory tests are made where it cannot."""
    def update(gg):
        m = b1 * m_prev + (1 - b1) * gg
        v = b2 * v_prev + (1 - b2) * gg * gg
        return lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    u0 = update(g)
    dev = np.zeros_like(u0)
    for f in (-1.0, -0.5, 0.5, 1.0):
        dev = np.maximum(dev, np.abs(update(g + f * delta) - u0))
    return dev <= tol


def curve_bars(ref, members, margin=0.1, widen=1.5):
    """Per logged iteration, the allowed distance from the oracle's PSNR:
    `margin` plus `widen` times the largest spread (largest minus smallest)
    of the oracle's curve and its float32-perturbed copies at that iteration
    or any logged before it.  Where the loop is well conditioned the spread
    is far below the margin; where rounding alone moves it (Adam oscillating
    near the optimum, the loop fitting its few training views) the copies
    move apart and do not come back together, and their spread at one logged
    point is a sample of a distance that fluctuates from point to point (a
    handful of copies can sit close together at one point and 0.2 dB apart
    at the next), so the bar keeps the widest spread seen so far.

    The GPU run is one more member of that family (its own rounding and the
    order of its float atomics perturb it by the same relative size), and a
    new member falls outside the range of n earlier ones with probability
    2 / (n + 1) at each point.  For normally spread members the expected
    range of nine is 2.97 sigma, and the distance between two members stays
    under 3 x sqrt(2) sigma = 4.24 sigma (99.7%), 1.43 times that range:
    hence `widen` = 1.5."""
    allc = np.vstack([np.asarray(ref, np.float64)] + [np.asarray(m, np.float64) for m in members])
    return margin + widen * np.maximum.accumulate(allc.max(axis=0) - allc.min(axis=0))
