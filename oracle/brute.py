"""Untiled brute-force renderer in pure Python (tiny scenes only).

TEST INFRASTRUCTURE ONLY.  A second, independently written statement of the
same forward render as ``oracle.c`` (NavGSim Eq. (1), Sigma = R S S^T R^T from
the Supplementary Material, and the compositing reading of the project), used
to pin the oracle: every pixel tests every Gaussian, no bounding boxes, no
row lists, SH evaluated from its Cartesian polynomials rather than a
Legendre recursion, covariance built from rotated axes rather than matrix
products.  Follows the FP64 decision at every threshold (no forks).
"""
from __future__ import annotations

import math
import struct

ALPHA_CAP = struct.unpack("f", struct.pack("f", 0.99))[0]
ALPHA_MIN = struct.unpack("f", struct.pack("f", 1.0 / 255.0))[0]
T_MIN = struct.unpack("f", struct.pack("f", 1e-4))[0]


def _f32(x: float) -> float:
    return struct.unpack("f", struct.pack("f", x))[0]


def _qrot(q, v):
    """Rotate v by the unit quaternion q = (w, x, y, z): q v q*."""
    w, x, y, z = q
    # t = 2 (q_vec x v); v' = v + w t + q_vec x t
    tx = 2.0 * (y * v[2] - z * v[1])
    ty = 2.0 * (z * v[0] - x * v[2])
    tz = 2.0 * (x * v[1] - y * v[0])
    return (v[0] + w * tx + (y * tz - z * ty),
            v[1] + w * ty + (z * tx - x * tz),
            v[2] + w * tz + (x * ty - y * tx))


def _sh_cartesian(x, y, z):
    """Real SH (Condon-Shortley phase) l <= 3 as Cartesian polynomials,
    index l*l + l + m."""
    pi = math.pi
    return [
        0.5 * math.sqrt(1 / pi),
        -math.sqrt(3 / (4 * pi)) * y,
        math.sqrt(3 / (4 * pi)) * z,
        -math.sqrt(3 / (4 * pi)) * x,
        0.5 * math.sqrt(15 / pi) * x * y,
        -0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),
        -0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
        0.5 * math.sqrt(105 / pi) * x * y * z,
        -0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1),
        0.25 * math.sqrt(7 / pi) * z * (5 * z * z - 3),
        -0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1),
        0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ]


def project_one(mean, scale, quat, opacity, sh, cam):
    """Return None if culled, else dict(u, v, conic, cov, colour, z, zkey, o)."""
    o = [float(c) for c in cam.position]
    Rv = [[float(cam.R[i][j]) for j in range(3)] for i in range(3)]
    d = [float(mean[i]) - o[i] for i in range(3)]
    t = [(Rv[i][0] * d[0] + Rv[i][1] * d[1]) + Rv[i][2] * d[2] for i in range(3)]
    if not t[2] > float(cam.znear):
        return None
    qn = math.sqrt(sum(float(c) ** 2 for c in quat))
    q = [float(c) / qn for c in quat]
    # Sigma = sum_k s_k^2 a_k a_k^T, a_k = rotated k-th axis
    axes = [_qrot(q, e) for e in ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))]
    Sig = [[sum(float(scale[k]) ** 2 * axes[k][i] * axes[k][j] for k in range(3))
            for j in range(3)] for i in range(3)]
    fx, fy = float(cam.fx), float(cam.fy)
    W, H, cx, cy = float(cam.width), float(cam.height), float(cam.cx), float(cam.cy)
    tz = t[2]
    xr = min(max(t[0] / tz, (-cx - 0.15 * W) / fx), (W - cx + 0.15 * W) / fx)
    yr = min(max(t[1] / tz, (-cy - 0.15 * H) / fy), (H - cy + 0.15 * H) / fy)
    # rows of J W: derivative of (fx x/z, fy y/z) in world coordinates
    g0 = [fx / tz * Rv[0][j] - fx * xr / tz * Rv[2][j] for j in range(3)]
    g1 = [fy / tz * Rv[1][j] - fy * yr / tz * Rv[2][j] for j in range(3)]

    def quad(a, b):
        return sum(a[i] * Sig[i][j] * b[j] for i in range(3) for j in range(3))

    s00 = quad(g0, g0) + 0.3
    s01 = quad(g0, g1)
    s11 = quad(g1, g1) + 0.3
    det = s00 * s11 - s01 * s01
    if not det > 0:
        return None
    dn = math.sqrt(sum(c * c for c in d))
    Y = _sh_cartesian(d[0] / dn, d[1] / dn, d[2] / dn)
    K = len(sh)
    col = []
    for c in range(3):
        v = 0.5 + sum(float(sh[k][c]) * Y[k] for k in range(K))
        col.append(min(max(v, 0.0), 1.0))
    return dict(u=fx * t[0] / tz + float(cam.cx), v=fy * t[1] / tz + float(cam.cy),
                conic=(s11 / det, -s01 / det, s00 / det), cov=(s00, s01, s11),
                colour=col, z=tz, zkey=_f32(tz), o=float(opacity))


def render(scene, cam):
    """(rgb as [H][W][3], depth [H][W], alpha [H][W]) lists, FP64."""
    P = []
    for g in range(scene.n):
        p = project_one(scene.means[g], scene.scales[g], scene.quats[g], scene.opacity[g],
                        scene.sh[g], cam)
        if p is not None:
            P.append((p["zkey"], g, p))
    P.sort(key=lambda e: (e[0], e[1]))
    bg = [_f32(float(c)) for c in cam.bg]   # cameras hold single precision
    rgb = [[None] * cam.width for _ in range(cam.height)]
    dep = [[0.0] * cam.width for _ in range(cam.height)]
    alp = [[0.0] * cam.width for _ in range(cam.height)]
    for j in range(cam.height):
        for i in range(cam.width):
            x, y = i + 0.5, j + 0.5
            T, C, D = 1.0, [0.0, 0.0, 0.0], 0.0
            for _, _, p in P:
                A, B, Cc = p["conic"]
                dx, dy = x - p["u"], y - p["v"]
                q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
                if q > 9.0:
                    continue
                a = min(ALPHA_CAP, p["o"] * math.exp(-0.5 * q))
                if a < ALPHA_MIN:
                    continue
                Tn = T * (1 - a)
                if Tn < T_MIN:
                    break
                for c in range(3):
                    C[c] += p["colour"][c] * a * T
                D += p["z"] * a * T
                T = Tn
            rgb[j][i] = [C[c] + T * bg[c] for c in range(3)]
            dep[j][i] = D
            alp[j][i] = 1 - T
    return rgb, dep, alp
