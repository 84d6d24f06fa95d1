"""FP64 gradients of the forward render (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests compare the GPU's backward pass with it;
the renderer never imports it.

What it differentiates is the oracle's forward render (``oracle.c``), restated
here with plain PyTorch CPU operations in float64 so that autograd supplies
the derivatives (NavGSim reconstructs its scenes by optimising the Gaussians'
parameters against captured images, Sec. III-B; the renderer's backward pass
serves that optimisation):

  projection: Sigma = R S S^T R^T from the normalised quaternion; camera
    mean t = W (mu - o); Jacobian J of the pinhole map at t with x/z and y/z
    clamped to the image's tangent range widened by 15 % of its size per
    side; Sigma' = J W Sigma W^T J^T + 0.3 I; conic = Sigma'^-1; 2D mean
    (fx tx/tz + cx, fy ty/tz + cy); colour clamp(0.5 + sum_k f_k Y_k(d), 0, 1)
    with d the unit vector from the camera to the mean;
  compositing per pixel centre, over the Gaussians with t_z > znear and a
    positive 2D determinant, in ascending (single-precision depth, id)
    order: q = d^T conic d; a Gaussian takes part when q <= 9 and
    alpha = min(0.99, o e^{-q/2}) >= 1/255; the pixel stops before the first
    Gaussian that would bring T (1 - alpha) below 1e-4; C = sum c alpha T +
    T_end bg, D = sum z alpha T, A = 1 - T_end (constants as single-precision
    values).

The discrete decisions (which Gaussians take part, the stop, the alpha cap)
are taken without gradient; everything else is differentiated.
"""
from __future__ import annotations

import numpy as np
import torch

ALPHA_CAP = float(np.float32(0.99))
ALPHA_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))
LOWPASS = 0.3
Q_MAX = 9.0

# real SH constants (Condon-Shortley phase), index l*l + l + m
_K00 = 0.28209479177387814
_K1 = 0.48860251190291992
_K2A, _K2B, _K2C = 1.0925484305920792, 0.31539156525252005, 0.54627421529603959
_K3A, _K3B, _K3C, _K3D, _K3E = (0.59004358992664352, 2.8906114426405538, 0.45704579946446572,
                                0.3731763325901154, 1.4453057213202769)


def _sh_basis(d, deg):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = [torch.full_like(x, _K00)]
    if deg >= 1:
        Y += [-_K1 * y, _K1 * z, -_K1 * x]
    if deg >= 2:
        Y += [_K2A * x * y, -_K2A * y * z, _K2B * (3 * z * z - 1), -_K2A * x * z, _K2C * (x * x - y * y)]
    if deg >= 3:
        Y += [-_K3A * y * (3 * x * x - y * y), _K3B * x * y * z, -_K3C * y * (5 * z * z - 1),
              _K3D * z * (5 * z * z - 3), -_K3C * x * (5 * z * z - 1), _K3E * z * (x * x - y * y),
              -_K3A * x * (x * x - 3 * y * y)]
    return torch.stack(Y, 1)


def _rotation(q):
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)


def project(means, scales, quats, opacity, sh, sh_degree, cam):
    """Per Gaussian: u, v, conic (A, B, C), opacity, colour (n, 3), depth
    z, single-precision depth key and validity (no gradient)."""
    W = torch.tensor(np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3), dtype=torch.float64)
    o = torch.tensor([float(np.float32(c)) for c in cam.position], dtype=torch.float64)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    Wd, Hd = float(cam.width), float(cam.height)
    d = means - o
    t = d @ W.T
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    xlo, xhi = (-cx - 0.15 * Wd) / fx, (Wd - cx + 0.15 * Wd) / fx
    ylo, yhi = (-cy - 0.15 * Hd) / fy, (Hd - cy + 0.15 * Hd) / fy
    xr = torch.clamp(tx / tz, xlo, xhi)
    yr = torch.clamp(ty / tz, ylo, yhi)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * xr / tz], 1),
                     torch.stack([zero, fy / tz, -fy * yr / tz], 1)], 1)          # (n, 2, 3)
    R = _rotation(quats)
    M = (J @ W) @ R * scales[:, None, :]                                          # J W R S
    S2 = M @ M.transpose(1, 2)
    s00 = S2[:, 0, 0] + LOWPASS
    s01 = S2[:, 0, 1]
    s11 = S2[:, 1, 1] + LOWPASS
    det = s00 * s11 - s01 * s01
    with torch.no_grad():
        valid = (tz > float(np.float32(cam.znear))) & (det > 0)
        zkey = tz.detach().numpy().astype(np.float32)
    safe = torch.where(valid, det, torch.ones_like(det))
    A, B, C = s11 / safe, -s01 / safe, s00 / safe
    u = fx * tx / tz + cx
    v = fy * ty / tz + cy
    dn = d / torch.linalg.norm(d, dim=1, keepdim=True)
    Y = _sh_basis(dn, sh_degree)                                                  # (n, K)
    K = Y.shape[1]
    raw = 0.5 + torch.einsum("nk,nkc->nc", Y, sh[:, :K, :])
    col = torch.clamp(raw, 0.0, 1.0)
    return dict(u=u, v=v, A=A, B=B, C=C, opacity=opacity, col=col, z=tz, zkey=zkey, valid=valid, raw=raw.detach())


def render(params, sh_degree, cam, px, py, chunk=2048, upstream=None):
    """Forward render of pixels (px, py): (rgb (P, 3), depth (P,), alpha
    (P,)) as float64 tensors carrying the graph to `params` (dict of leaf
    tensors means, scales, quats, opacity, sh).  With upstream = (g_rgb,
    g_depth, g_alpha) the loss sum(g . outputs) is back-propagated chunk by
    chunk and the outputs are returned detached.  Also returns per-pixel
    flags: 1 where some Gaussian's unclamped alpha is within 1e-6 of the 0.99
    cap (the gradient changes discontinuously there)."""
    pr = project(params["means"], params["scales"], params["quats"], params["opacity"], params["sh"], sh_degree,
                 cam)
    valid = np.nonzero(pr["valid"].numpy())[0]
    order = valid[np.lexsort((valid, pr["zkey"][valid]))]
    idx = torch.from_numpy(order)
    u, v = pr["u"][idx], pr["v"][idx]
    A, B, C = pr["A"][idx], pr["B"][idx], pr["C"][idx]
    op, col, z = pr["opacity"][idx], pr["col"][idx], pr["z"][idx]
    bg = torch.tensor([float(np.float32(b)) for b in cam.bg], dtype=torch.float64)
    outs, flags = [], []
    px = np.asarray(px); py = np.asarray(py)
    for s in range(0, px.size, chunk):
        x = torch.from_numpy(px[s:s + chunk].astype(np.float64) + 0.5)[:, None]
        y = torch.from_numpy(py[s:s + chunk].astype(np.float64) + 0.5)[:, None]
        dx, dy = x - u[None, :], y - v[None, :]
        q = A[None] * dx * dx + 2.0 * B[None] * dx * dy + C[None] * dy * dy
        a_raw = op[None] * torch.exp(-0.5 * q)
        with torch.no_grad():
            inq = q <= Q_MAX
            capped = a_raw >= ALPHA_CAP
            a_val = torch.where(capped, torch.full_like(a_raw, ALPHA_CAP), a_raw)
            keep = inq & (a_val >= ALPHA_MIN)
            ak = torch.where(keep, a_val, torch.zeros_like(a_val))
            Tex = torch.cumprod(torch.cat([torch.ones_like(ak[:, :1]), 1 - ak[:, :-1]], 1), 1)
            stop = keep & (Tex * (1 - ak) < T_MIN)
            live = torch.cumsum(stop.to(torch.int64), 1) == 0
            use = keep & live
            near_cap = (use & ((a_raw - ALPHA_CAP).abs() <= 1e-6)).any(1)
        alpha = torch.where(use, torch.where(capped, torch.full_like(a_raw, ALPHA_CAP), a_raw), torch.zeros_like(a_raw))
        one_minus = 1 - alpha
        T = torch.cumprod(torch.cat([torch.ones_like(alpha[:, :1]), one_minus[:, :-1]], 1), 1)
        w = alpha * T
        T_end = torch.prod(one_minus, 1)
        rgb = w @ col + T_end[:, None] * bg[None, :]
        depth = w @ z
        alp = 1 - T_end
        if upstream is not None:
            g_rgb, g_d, g_a = (torch.from_numpy(np.asarray(g, np.float64)[s:s + chunk]) for g in upstream)
            loss = (rgb * g_rgb).sum() + (depth * g_d).sum() + (alp * g_a).sum()
            loss.backward(retain_graph=True)
            rgb, depth, alp = rgb.detach(), depth.detach(), alp.detach()
        outs.append((rgb, depth, alp))
        flags.append(near_cap.numpy())
    rgb = torch.cat([o[0] for o in outs]); depth = torch.cat([o[1] for o in outs]); alp = torch.cat([o[2] for o in outs])
    return rgb, depth, alp, np.concatenate(flags) if flags else np.zeros(0, bool)


def leaf_params(scene, ids=None):
    """float64 leaf tensors (requires_grad) of the scene's Gaussians `ids`
    (all when None); sh as (n, K, 3)."""
    ids = np.arange(scene.n) if ids is None else np.asarray(ids)
    K = (scene.sh_degree + 1) ** 2
    t = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=torch.float64, requires_grad=True)  # noqa: E731
    return {"means": t(scene.means[ids]), "scales": t(scene.scales[ids]), "quats": t(scene.quats[ids]),
            "opacity": t(scene.opacity[ids]), "sh": t(np.asarray(scene.sh[ids], np.float64).reshape(len(ids), K, 3))}


def gradients(scene, cam, g_rgb, g_depth, g_alpha, ids=None):
    """Gradients of sum(g_rgb . rgb + g_depth depth + g_alpha alpha) over a
    full frame (row-major pixels; g_rgb (H*W, 3)) with respect to the
    Gaussians `ids` (all of a flat scene when None): dict of numpy arrays
    means (n, 3), scales (n, 3), quats (n, 4), opacity (n,), sh (n, K, 3);
    and the per-pixel cap flags of render()."""
    p = leaf_params(scene, ids)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    _, _, _, flags = render(p, scene.sh_degree, cam, xx.ravel(), yy.ravel(), upstream=(g_rgb, g_depth, g_alpha))
    return {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape)) for k, v in p.items()}, flags
