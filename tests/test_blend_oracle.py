"""Pins of the oracle's level-of-detail blending (CPU): the blend weight from
the parent's projected size, the two ends of the transition (t = 0: the
parent's projection; t = 1: the node's own), and intermediate weights
against an explicitly built blended Gaussian projected by the plain
oracle."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, workloads as W


@pytest.fixture(scope="module")
def plan():
    scene, cams = W.plan2m(scale=0.2, n_poses=6)
    return scene, cams


def _t(scene, ids, cam, tau):
    f2 = 2.0 * max(float(cam.fx), float(cam.fy))
    o = np.array([float(np.float32(c)) for c in cam.position])
    p = scene.parent[ids]
    t = np.ones(ids.size)
    has = p >= 0
    b = scene.bound[p[has]].astype(np.float64)
    d = np.sqrt(((b[:, :3] - o) ** 2).sum(axis=1))
    sp = f2 * b[:, 3] / d
    t[has] = np.clip((sp - tau) / tau, 0.0, 1.0)
    return t


def test_blend_weight_follows_the_parents_projected_size(plan):
    scene, cams = plan
    cam = cams[2]
    inside = 0
    for tau in (1.0, 64.0, 96.0, 128.0):
        ids = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
        _, t = O.project_blend(scene, ids, cam, tau, with_t=True)
        np.testing.assert_allclose(t, _t(scene, ids, cam, tau), rtol=1e-12, atol=1e-12)
        inside += int(((t > 0) & (t < 1)).sum())
    assert inside > 0


def test_zero_weight_is_the_parents_projection(plan):
    """t = 0 (tau far above every projected size): each node is drawn as its
    parent, bit for bit."""
    scene, cams = plan
    cam = cams[1]
    ids = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    ids = ids[scene.parent[ids] >= 0]
    out, t = O.project_blend(scene, ids, cam, 1e9, with_t=True)
    assert np.all(t == 0)
    par = O.project(scene, scene.parent[ids].astype(np.int32), cam)
    np.testing.assert_array_equal(out, par)


def test_unit_weight_is_the_nodes_own_projection(plan):
    """t = 1 (tau far below every projected size): the node's own
    projection up to the rounding of p + (g - p)."""
    scene, cams = plan
    cam = cams[3]
    ids = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    out, t = O.project_blend(scene, ids, cam, 1e-9, with_t=True)
    assert np.all(t == 1)
    own = O.project(scene, ids, cam)
    np.testing.assert_array_equal(out[:, 0], own[:, 0])
    v = own[:, 0] == 1
    np.testing.assert_allclose(out[v], own[v], rtol=1e-9, atol=1e-9)


def test_intermediate_weight_equals_the_blended_gaussian(plan):
    """For weights strictly inside (0, 1): build each blended Gaussian
    (mean, covariance, opacity and SH interpolated; covariance turned back
    into scales and a quaternion by an eigendecomposition), project it as a
    flat scene with the plain oracle, and compare."""
    scene, cams = plan
    cam = cams[4]
    tau = 128.0
    ids = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
    t = _t(scene, ids, cam, tau)
    sel = ids[(t > 0.05) & (t < 0.95)][:300]
    assert sel.size > 20
    ts = _t(scene, sel, cam, tau)
    p = scene.parent[sel]

    def sigma(k):
        q = scene.quats[k].astype(np.float64)
        R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()
        return np.einsum("nij,nj,nkj->nik", R, scene.scales[k].astype(np.float64) ** 2, R)

    S = sigma(p) + ts[:, None, None] * (sigma(sel) - sigma(p))
    w, V = np.linalg.eigh(S)
    V[np.linalg.det(V) < 0, :, 0] *= -1                      # proper rotations
    quat = Rotation.from_matrix(V).as_quat()                  # (x, y, z, w)
    mu = scene.means[p].astype(np.float64) + ts[:, None] * (scene.means[sel] - scene.means[p]).astype(np.float64)
    op = scene.opacity[p] + ts * (scene.opacity[sel] - scene.opacity[p])
    sh = scene.sh[p].astype(np.float64) + ts[:, None, None] * (scene.sh[sel] - scene.sh[p]).astype(np.float64)
    flat = Scene(means=mu, scales=np.sqrt(w), quats=np.concatenate([quat[:, 3:], quat[:, :3]], 1), opacity=op,
                 sh=sh, sh_degree=scene.sh_degree)
    want = O.project(flat, np.arange(sel.size, dtype=np.int32), cam)
    got = O.project_blend(scene, sel, cam, tau)
    # the flat scene's inputs pass through single precision: compare loosely
    v = want[:, O.PF["valid"]] == 1
    assert v.sum() > 10
    for f, rt in (("u", 1e-5), ("v", 1e-5), ("z", 1e-6), ("S00", 1e-4), ("S11", 1e-4), ("opacity", 1e-6)):
        np.testing.assert_allclose(got[v, O.PF[f]], want[v, O.PF[f]], rtol=rt, atol=1e-4, err_msg=f)
    np.testing.assert_allclose(got[v, O.PF["r"]:O.PF["b"] + 1], want[v, O.PF["r"]:O.PF["b"] + 1], atol=2e-6)
