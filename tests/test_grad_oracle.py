"""Pins of the FP64 gradient oracle (CPU): its forward render equals the C
oracle's; its gradients equal central differences of the C oracle's forward
render for every parameter kind (mean, scale, rotation, opacity, SH up to
degree 3); closed forms for one isotropic Gaussian."""
import math

import numpy as np
import pytest
import torch

from oracle import grad as G
from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, make_random_box, yaw_camera


def _scene(n, seed, deg=3, box=(1.2, 1.2, 1.2)):
    s = make_random_box(n, seed=seed, box=box)
    rng = np.random.default_rng(seed + 100)
    K = (deg + 1) ** 2
    sh = np.zeros((n, K, 3), np.float32)
    sh[:, 0, :] = np.asarray(s.sh, np.float32).reshape(n, -1, 3)[:, 0, :] * 0.6
    sh[:, 1:, :] = rng.normal(0, 0.08, size=(n, K - 1, 3))
    s.scales[:] = np.exp(rng.uniform(np.log(0.03), np.log(0.15), size=(n, 3))).astype(np.float32)
    return Scene(s.means, s.scales, s.quats, s.opacity, sh.reshape(n, K * 3), deg)


def _cam(w=40, h=32, f=40.0):
    return yaw_camera(w, h, f, (0.6, -1.4, 0.6), math.pi / 2)


def _c_forward(scene, cam, with_nalg=False):
    res, _, _ = O.render(scene, cam, O.MODE_THRESHOLD, 1.0)
    return (res.primary, res.flags, res.nalg) if with_nalg else (res.primary, res.flags)


def test_forward_equals_the_c_oracle():
    scene = _scene(120, 1)
    cam = _cam()
    prim, flags = _c_forward(scene, cam)
    p = G.leaf_params(scene)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    rgb, depth, alpha, cap = G.render(p, scene.sh_degree, cam, xx.ravel(), yy.ravel())
    ok = flags == 0
    assert ok.mean() > 0.95
    np.testing.assert_allclose(rgb.detach().numpy()[ok], prim[ok, :3], rtol=0, atol=1e-11)
    np.testing.assert_allclose(depth.detach().numpy()[ok], prim[ok, 3], rtol=0, atol=1e-10)
    np.testing.assert_allclose(alpha.detach().numpy()[ok], prim[ok, 4], rtol=0, atol=1e-11)
    assert alpha.detach().numpy().max() > 0.5


def _loss_c(scene, cam, g):
    """Loss and the per-pixel decision record (fork flags, pairs that pass
    q <= 9): a perturbation that changes either crosses a discontinuity."""
    prim, flags, nalg = _c_forward(scene, cam, with_nalg=True)
    return (float((prim[:, :3] * g[0]).sum() + (prim[:, 3] * g[1]).sum() + (prim[:, 4] * g[2]).sum()),
            (flags, nalg))


def _perturbed(scene, field, i, j, h):
    arrs = {k: np.array(getattr(scene, k), np.float64) for k in ("means", "scales", "quats", "opacity", "sh")}
    a = arrs[field]
    if a.ndim == 1:
        a[i] += h
    else:
        a[i, j] += h
    return Scene(*(arrs[k] for k in ("means", "scales", "quats", "opacity", "sh")), scene.sh_degree)


@pytest.mark.parametrize("seed", [2, 3])
def test_gradients_equal_central_differences(seed):
    """The C oracle reads float32 inputs: each step h is a power of two 2^-12
    of the parameter's binade, so v +- h is exact in float32.  Perturbations
    that change a decision (a fork flag or a pixel's count of pairs with
    q <= 9) cross a discontinuity and are skipped; at least three checks per
    parameter kind remain."""
    scene = _scene(40, seed, box=(0.8, 0.8, 0.8))
    cam = _cam(24, 20, 24.0)
    rng = np.random.default_rng(seed)
    n = scene.n
    g = (rng.normal(size=(cam.width * cam.height, 3)), rng.normal(size=cam.width * cam.height),
         rng.normal(size=cam.width * cam.height))
    grads, cap = G.gradients(scene, cam, *g)
    assert not cap.any()
    base, rec0 = _loss_c(scene, cam, g)
    assert (rec0[0] == 0).all()
    done = {k: 0 for k in ("means", "scales", "quats", "opacity", "sh")}
    K = (scene.sh_degree + 1) ** 2
    checks = [("means", 3), ("scales", 3), ("quats", 4), ("opacity", 0), ("sh", 3 * K)]
    for field, width in checks:
        for _ in range(12):
            i = int(rng.integers(n))
            j = int(rng.integers(width)) if width else 0
            val = np.asarray(getattr(scene, field), np.float64)
            v = val[i] if val.ndim == 1 else val[i, j]
            h = 2.0 ** math.floor(math.log2(max(abs(v), 1e-2))) * 2.0 ** -12
            lp, rp = _loss_c(_perturbed(scene, field, i, j, h), cam, g)
            lm, rm = _loss_c(_perturbed(scene, field, i, j, -h), cam, g)
            if any((a != b).any() for r in (rp, rm) for a, b in zip(r, rec0)):
                continue                                  # a decision changed
            fd = (lp - lm) / (2 * h)
            ga = grads[field][i] if field == "opacity" else grads[field].reshape(n, -1)[i, j]
            assert abs(fd - ga) <= 1e-3 * abs(ga) + 1e-4 * max(1.0, abs(fd)), (field, i, j, fd, ga)
            done[field] += 1
    assert all(v >= 3 for v in done.values()), done


def test_single_gaussian_closed_forms():
    """An isotropic Gaussian of opacity o on the optical axis, centred on a
    pixel centre: that pixel's alpha is o, so d alpha / d o = 1 and its
    colour gradient w.r.t. the DC coefficient is o Y_00; moving the mean
    along the axis changes only the depth output there (d D / d z = o)."""
    W = H = 9
    cam = yaw_camera(W, H, 20.0, (0.0, -2.0, 0.0), math.pi / 2)
    # world point seen at the centre of pixel (4, 4): on the optical axis
    o = float(np.float32(0.6))
    sh = np.zeros((1, 3), np.float32)
    sh[0] = 0.3
    s = Scene(np.array([[0.0, 0.0, 0.0]], np.float32), np.full((1, 3), 0.05, np.float32),
              np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), np.array([o], np.float32), sh, 0)
    npx = W * H
    c = 4 * W + 4
    g_a = np.zeros(npx); g_a[c] = 1.0
    grads, _ = G.gradients(s, cam, np.zeros((npx, 3)), np.zeros(npx), g_a)
    assert abs(grads["opacity"][0] - 1.0) < 1e-12
    assert np.abs(grads["means"][0]).max() < 1e-12          # q is at its minimum
    g_c = np.zeros((npx, 3)); g_c[c, 0] = 1.0
    grads, _ = G.gradients(s, cam, g_c, np.zeros(npx), np.zeros(npx))
    assert abs(grads["sh"][0, 0, 0] - o * 0.28209479177387814) < 1e-12
    g_d = np.zeros(npx); g_d[c] = 1.0
    grads, _ = G.gradients(s, cam, np.zeros((npx, 3)), g_d, np.zeros(npx))
    fwd = np.asarray(cam.R, np.float64).reshape(3, 3)[2]      # camera forward in world
    np.testing.assert_allclose(grads["means"][0], o * fwd, rtol=0, atol=1e-12)
