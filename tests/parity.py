"""Comparison of GPU pixels against the oracle's branch sets.

The oracle lists every valid result of a pixel (branch 0 follows every FP64
decision; others flip decisions that lie within the single-precision error
margin of their threshold).  A GPU pixel passes if it matches one branch on
all outputs at once:
  RGB channels and alpha within 2e-4 absolute (the renderer's tolerance);
  depth (sum of w z) within 2e-4 times the pixel's mean depth (at least
  1 m): a weight error e moves the depth by at most e times the largest
  depth, and the mean depth bounds it within the pixel's few layers.
"""
import numpy as np

TOL_RGB = 2e-4
TOL_ALPHA = 2e-4
TOL_DEPTH_REL = 2e-4


def branch_errors(gpu, res):
    """gpu: (n, 5) float array (R, G, B, depth, alpha) for the oracle's
    pixels.  Returns (ok mask, best normalised error per pixel, skipped mask)
    where the normalised error is max over outputs of |diff| / tolerance.
    A pixel whose branch list overflowed the oracle's fork cap (skipped) is
    not complete, so it counts as a failure."""
    br = res.branches                                    # (n, cap, 5)
    nb = res.nbranch
    cap = br.shape[1]
    valid = np.arange(cap)[None, :] < nb[:, None]
    d = np.abs(gpu[:, None, :].astype(np.float64) - br)
    zbar = np.maximum(1.0, br[:, :, 3] / np.maximum(br[:, :, 4], 1e-6))
    e = np.maximum.reduce([d[:, :, 0] / TOL_RGB, d[:, :, 1] / TOL_RGB, d[:, :, 2] / TOL_RGB,
                           d[:, :, 4] / TOL_ALPHA, d[:, :, 3] / (TOL_DEPTH_REL * zbar)])
    e = np.where(valid, e, np.inf)
    best = e.min(axis=1)
    skipped = res.flags != 0
    ok = (best <= 1.0) & ~skipped
    return ok, best, skipped


def gpu_pixels(rgb, depth, alpha, px, py):
    """Gather (R, G, B, depth, alpha) of pixels (px, py) from planar images."""
    rgb = np.asarray(rgb); depth = np.asarray(depth); alpha = np.asarray(alpha)
    return np.stack([rgb[0, py, px], rgb[1, py, px], rgb[2, py, px], depth[py, px], alpha[py, px]], axis=1)


def summary(ok, best, skipped):
    fin = best[np.isfinite(best)]
    return (f"pixels={ok.size} fail={int((~ok).sum())} skipped={int(skipped.sum())} "
            f"worst={float(fin.max()) if fin.size else 0:.3g}x tol")
