"""Pins of the oracle's level-of-detail blending (CPU): the blend weight from
the parent's and the node's projected sizes, the two ends of the transition
(t = 0: the first child is the parent's projection, the others are
transparent; t = 1: the node's own), intermediate weights against an
explicitly built blended Gaussian projected by the plain oracle, and the
continuity of the image across a refine decision along a camera sweep."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, workloads as W


@pytest.fixture(scope="module")
def plan():
    scene, cams = W.plan2m(scale=0.2, n_poses=6)
    return scene, cams


def _size(scene, nodes, cam):
    """Projected size 2 f r / |c - o| of the nodes' bounding spheres."""
    f2 = 2.0 * max(float(cam.fx), float(cam.fy))
    o = np.array([float(np.float32(c)) for c in cam.position])
    b = scene.bound[nodes].astype(np.float64)
    return f2 * b[:, 3] / np.sqrt(((b[:, :3] - o) ** 2).sum(axis=1))


def _t(scene, ids, cam, tau):
    p = scene.parent[ids]
    t = np.ones(ids.size)
    has = p >= 0
    sp, sg = _size(scene, p[has], cam), _size(scene, ids[has], cam)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(sg < sp, np.clip((sp - tau) / (sp - sg), 0.0, 1.0), 1.0)
    t[has] = w
    return t


def _first(scene, ids, cut):
    """Whether each node is the first of its parent's children in the cut."""
    in_cut = set(int(k) for k in cut)
    out = np.ones(ids.size, bool)
    for i, g in enumerate(ids):
        p = int(scene.parent[g])
        if p >= 0:
            out[i] = not any(q in in_cut for q in range(int(scene.first_child[p]), int(g)))
    return out


def test_blend_weight_follows_the_projected_sizes(plan):
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
    """t = 0 (tau far above every projected size): the first of a parent's
    children in the cut is drawn as the parent, bit for bit; its siblings
    are drawn at the parent's place with opacity 0."""
    scene, cams = plan
    cam = cams[1]
    cut = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    ids = cut[scene.parent[cut] >= 0]
    ids = ids[_size(scene, ids, cam) < _size(scene, scene.parent[ids], cam)]
    out, t = O.project_blend(scene, ids, cam, 1e9, with_t=True, cut_ids=cut)
    assert np.all(t == 0)
    par = O.project(scene, scene.parent[ids].astype(np.int32), cam)
    first = _first(scene, ids, cut)
    assert first.any() and (~first).any()
    np.testing.assert_array_equal(out[first], par[first])
    op = O.PF["opacity"]
    np.testing.assert_array_equal(out[~first][:, op], 0.0)
    rest = [k for k in range(out.shape[1]) if k != op]
    np.testing.assert_array_equal(out[~first][:, rest], par[~first][:, rest])


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
    first = _first(scene, sel, ids)
    assert first.any() and (~first).any()

    def sigma(k):
        q = scene.quats[k].astype(np.float64)
        R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()
        return np.einsum("nij,nj,nkj->nik", R, scene.scales[k].astype(np.float64) ** 2, R)

    S = sigma(p) + ts[:, None, None] * (sigma(sel) - sigma(p))
    w, V = np.linalg.eigh(S)
    V[np.linalg.det(V) < 0, :, 0] *= -1                      # proper rotations
    quat = Rotation.from_matrix(V).as_quat()                  # (x, y, z, w)
    mu = scene.means[p].astype(np.float64) + ts[:, None] * (scene.means[sel] - scene.means[p]).astype(np.float64)
    op = np.where(first, scene.opacity[p] + ts * (scene.opacity[sel] - scene.opacity[p]), ts * scene.opacity[sel])
    sh = scene.sh[p].astype(np.float64) + ts[:, None, None] * (scene.sh[sel] - scene.sh[p]).astype(np.float64)
    flat = Scene(means=mu, scales=np.sqrt(w), quats=np.concatenate([quat[:, 3:], quat[:, :3]], 1), opacity=op,
                 sh=sh, sh_degree=scene.sh_degree)
    want = O.project(flat, np.arange(sel.size, dtype=np.int32), cam)
    got = O.project_blend(scene, sel, cam, tau, cut_ids=ids)
    # the flat scene's inputs pass through single precision: compare loosely
    v = want[:, O.PF["valid"]] == 1
    assert v.sum() > 10
    for f, rt in (("u", 1e-5), ("v", 1e-5), ("z", 1e-6), ("S00", 1e-4), ("S11", 1e-4), ("opacity", 1e-6)):
        np.testing.assert_allclose(got[v, O.PF[f]], want[v, O.PF[f]], rtol=rt, atol=1e-4, err_msg=f)
    np.testing.assert_allclose(got[v, O.PF["r"]:O.PF["b"] + 1], want[v, O.PF["r"]:O.PF["b"] + 1], atol=2e-6)


def _refine_step(scene, cam, node, tau, lam_lo, lam_hi):
    """Adjacent single-precision camera positions along the view direction,
    the node in the cut at the first and refined at the second."""
    import copy
    fwd = np.asarray(cam.R, np.float64)[2]
    p0 = np.asarray(cam.position, np.float64)

    def at(lam):
        c = copy.copy(cam)
        c.position = (p0 + lam * fwd).astype(np.float32)
        return c

    def refined(lam):
        return node not in set(O.cut(scene, at(lam), O.MODE_THRESHOLD, tau).tolist())

    assert not refined(lam_lo) and refined(lam_hi)
    for _ in range(80):
        mid = 0.5 * (lam_lo + lam_hi)
        if np.array_equal(at(mid).position, at(lam_lo).position) or \
                np.array_equal(at(mid).position, at(lam_hi).position):
            break
        if refined(mid):
            lam_hi = mid
        else:
            lam_lo = mid
    return at(lam_lo), at(lam_hi)


def refine_events(scene, cams, tau=40.0, n_cand=12):
    """(node, a, b, cut at a, cut at b) for refine events found along sweeps
    toward the largest interior nodes of a 240x136 view's cut: a and b are
    adjacent single-precision camera positions, only the node's refinement
    (the node leaves the cut, some of its children enter) tells the two
    cuts apart."""
    from paper_2603_15186_amd.synth import yaw_camera
    base = cams[2]
    cam = yaw_camera(240, 136, 900.0 * 240 / 1280, base.position, np.arctan2(base.R[2][1], base.R[2][0]))
    cut = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
    proj = O.project(scene, cut, cam)
    s = _size(scene, cut, cam)
    vis = (proj[:, O.PF["valid"]] == 1) & (scene.child_count[cut] > 0) & (s > 0.5 * tau)
    vis &= (proj[:, O.PF["u"]] > 20) & (proj[:, O.PF["u"]] < 220) & (proj[:, O.PF["v"]] > 20) & (proj[:, O.PF["v"]] < 116)
    cand = cut[vis][np.argsort(-s[vis])][:n_cand]
    assert cand.size
    out = []
    for node in cand:
        node = int(node)
        dist = float(np.linalg.norm(scene.bound[node, :3].astype(np.float64) - cam.position))
        try:
            a, b = _refine_step(scene, cam, node, tau, 0.0, 0.9 * dist)
        except AssertionError:
            continue
        ca = O.cut(scene, a, O.MODE_THRESHOLD, tau)
        cb = O.cut(scene, b, O.MODE_THRESHOLD, tau)
        kids = set(range(int(scene.first_child[node]), int(scene.first_child[node] + scene.child_count[node])))
        if set(ca.tolist()) - set(cb.tolist()) != {node} or not set(cb.tolist()) - set(ca.tolist()) <= kids:
            continue
        out.append((node, a, b, ca, cb))
    return out


def test_image_is_continuous_where_a_node_is_refined(plan):
    """Along a camera sweep toward a node, at the single-precision step where
    the node is refined (its children replace it in the cut), the blended
    image barely changes -- the first child is drawn as the node, its
    siblings are transparent -- while the plain cut's image jumps."""
    scene, cams = plan
    tau = 40.0
    checked = 0
    for node, a, b, ca, cb in refine_events(scene, cams, tau):
        # both cuts drawn from the second position: the difference is the
        # cut's change alone, not the camera's one-ulp move
        ia = O.image(O.render(scene, b, O.MODE_THRESHOLD, tau, blend=True, ids=ca)[0], b)[0]
        ib = O.image(O.render(scene, b, O.MODE_THRESHOLD, tau, blend=True, ids=cb)[0], b)[0]
        pa = O.image(O.render(scene, b, O.MODE_THRESHOLD, tau, ids=ca)[0], b)[0]
        pb = O.image(O.render(scene, b, O.MODE_THRESHOLD, tau, ids=cb)[0], b)[0]
        jump = np.abs(pa - pb).max()
        smooth = np.abs(ia - ib)
        print(f"node {node}: plain jump {jump:.4f}, blended max {smooth.max():.2e}, mean {smooth.mean():.2e}")
        assert smooth.max() < 1e-6
        checked += jump > 0.02
    assert checked >= 2
