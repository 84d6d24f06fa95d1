"""Bottom-up 8-ary Gaussian hierarchy over Morton order (input preparation).

The paper's scene is a tree whose leaves hold the fine Gaussians and whose
internal nodes aggregate them into coarser ones (Sec. III-B); how parents are
formed is not given.  This builder uses the reading documented with the
project: groups of 8 consecutive nodes in Morton order share a parent whose
Gaussian matches the weighted mixture's first two moments, with weight
w = opacity * (s1 s2 + s2 s3 + s1 s3).  Every node also carries a bounding
sphere that encloses the 3-sigma spheres of all leaves below it.

Layout: node k is Gaussian k; ids are level-major with the root level first
and the leaves last; children of a node are contiguous and ordered like their
parents, so a level-synchronous traversal that compacts stably produces
ascending ids.
"""
from __future__ import annotations

import numpy as np

from .scenes import Scene, _rotmat_to_quat

FANOUT = 8


def _quat_to_rotmat(q):
    """(n,4) (w,x,y,z) -> (n,3,3), normalising first."""
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - w * z); R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y); R[:, 2, 1] = 2 * (y * z + w * x); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariances(scales, quats):
    """Per-Gaussian 3x3 covariance in FP64 from FP32 scales and quaternions."""
    R = _quat_to_rotmat(quats.astype(np.float64))
    s2 = scales.astype(np.float64) ** 2
    return np.einsum("nij,nj,nkj->nik", R, s2, R)


def morton_codes(p, lo, hi):
    """30-bit Morton codes of points p (n,3) in the box [lo, hi]."""
    t = (p - lo) / np.maximum(hi - lo, 1e-12)
    c = np.clip((t * 1024).astype(np.int64), 0, 1023)

    def spread(v):
        v = (v | (v << 16)) & 0x030000FF
        v = (v | (v << 8)) & 0x0300F00F
        v = (v | (v << 4)) & 0x030C30C3
        v = (v | (v << 2)) & 0x09249249
        return v

    return (spread(c[:, 0]) << 2) | (spread(c[:, 1]) << 1) | spread(c[:, 2])


def _round_up_f32(x):
    f = x.astype(np.float32)
    low = f.astype(np.float64) < x
    f[low] = np.nextafter(f[low], np.float32(np.inf))
    return f


def build_hierarchy(leaves: Scene) -> Scene:
    """Build the hierarchy above a flat scene of leaves (see module doc)."""
    n0 = leaves.n
    lo = leaves.means.min(0).astype(np.float64)
    hi = leaves.means.max(0).astype(np.float64)
    order = np.argsort(morton_codes(leaves.means.astype(np.float64), lo, hi), kind="stable")
    # Per level (deepest first): FP64 moments and the stored FP32 attributes.
    lv_mean = [leaves.means[order].astype(np.float32)]
    lv_scale = [leaves.scales[order].astype(np.float32)]
    lv_quat = [leaves.quats[order].astype(np.float32)]
    lv_op = [leaves.opacity[order].astype(np.float32)]
    lv_sh = [leaves.sh[order].astype(np.float32)]
    lv_rad = [_round_up_f32(3.0 * lv_scale[0].astype(np.float64).max(1))]
    cov = covariances(lv_scale[0], lv_quat[0])
    while lv_mean[-1].shape[0] > 1:
        m = lv_mean[-1].astype(np.float64)
        s = lv_scale[-1].astype(np.float64)
        o = lv_op[-1].astype(np.float64)
        n = m.shape[0]
        starts = np.arange(0, n, FANOUT)
        w = o * (s[:, 0] * s[:, 1] + s[:, 1] * s[:, 2] + s[:, 0] * s[:, 2])
        W = np.add.reduceat(w, starts)
        mu = np.add.reduceat(w[:, None] * m, starts) / W[:, None]
        second = np.add.reduceat(w[:, None, None] * (cov + m[:, :, None] * m[:, None, :]), starts)
        P = second / W[:, None, None] - mu[:, :, None] * mu[:, None, :]
        P = 0.5 * (P + np.transpose(P, (0, 2, 1)))
        lam, V = np.linalg.eigh(P)
        lam = np.maximum(lam, 1e-12)
        V[np.linalg.det(V) < 0, :, 0] *= -1.0
        q = _rotmat_to_quat(V).astype(np.float32)
        sc = np.sqrt(lam).astype(np.float32)
        op = np.minimum(np.add.reduceat(w * o, starts) / W, 0.99).astype(np.float32)
        sh = (np.add.reduceat(w[:, None, None] * lv_sh[-1].astype(np.float64), starts)
              / W[:, None, None]).astype(np.float32)
        mu32 = mu.astype(np.float32)
        # Enclosing sphere of the children's spheres, in the stored precision.
        parent_of = np.repeat(np.arange(starts.size), np.diff(np.append(starts, n)))
        dist = np.linalg.norm(m - mu32.astype(np.float64)[parent_of], axis=1)
        reach = dist + lv_rad[-1].astype(np.float64)
        rad = _round_up_f32(np.maximum.reduceat(reach, starts))
        lv_mean.append(mu32); lv_scale.append(sc); lv_quat.append(q)
        lv_op.append(op); lv_sh.append(sh); lv_rad.append(rad)
        cov = covariances(sc, q)
    # Re-order: root level first.
    lv_mean.reverse(); lv_scale.reverse(); lv_quat.reverse(); lv_op.reverse()
    lv_sh.reverse(); lv_rad.reverse()
    sizes = np.array([a.shape[0] for a in lv_mean], dtype=np.int64)
    level_offset = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    N = int(level_offset[-1])
    parent = np.full(N, -1, np.int32)
    first_child = np.full(N, -1, np.int32)
    child_count = np.zeros(N, np.int32)
    for L in range(len(sizes) - 1):
        nc = int(sizes[L + 1])
        base_p, base_c = int(level_offset[L]), int(level_offset[L + 1])
        j = np.arange(sizes[L])
        first_child[base_p + j] = base_c + FANOUT * j
        child_count[base_p + j] = np.minimum(FANOUT, nc - FANOUT * j)
        parent[base_c + np.arange(nc)] = base_p + np.arange(nc) // FANOUT
    means = np.concatenate(lv_mean)
    bound = np.concatenate([means, np.concatenate(lv_rad)[:, None]], axis=1).astype(np.float32)
    return Scene(means, np.concatenate(lv_scale), np.concatenate(lv_quat),
                 np.concatenate(lv_op), np.concatenate(lv_sh), leaves.sh_degree,
                 parent=parent, first_child=first_child, child_count=child_count,
                 bound=bound, level_offset=level_offset,
                 meta=dict(leaves.meta, hierarchy="morton8_moment"))
