"""Pins of the oracle's learned level-of-detail cut (CPU) with networks whose
logit is a known function: constant logits give the threshold cut or the
threshold cut stopped at every candidate; one-feature networks split the
candidates by opacity, child count, level and projected size exactly where
those quantities, read from the scene, say; linear one-feature networks split
them by camera depth, children's colour variance, view angle to the thinnest
axis and the parent's projected size, each computed independently here with
numpy and scipy; a zero logit leaves every candidate undecided, and flips are
honoured only for undecided ones."""
import math

import numpy as np
import pytest

from oracle import oracle as O, mlp as M
from paper_2603_15186_amd.synth import workloads as W

S_HI = 4096.0


@pytest.fixture(scope="module")
def plan():
    scene, cams = W.plan2m(scale=0.02, n_poses=6)
    return scene, cams


def _net(b3=0.0, feature=None, weight=1.0):
    """Parameters of a network with logit b3 (+ weight * relu(relu(x_f))
    with feature f passed through hidden unit 0 of both layers)."""
    q = {"W1": np.zeros((32, 8)), "b1": np.zeros(32), "W2": np.zeros((32, 32)), "b2": np.zeros(32),
         "w3": np.zeros(32), "b3": b3}
    if feature is not None:
        q["W1"][0, feature] = 1.0
        q["W2"][0, 0] = 1.0
        q["w3"][0] = weight
    return M.pack(q)


def _band(scene, cam, tau=1.0):
    """Internal nodes the threshold refines with projected size <= S_HI
    (same FP64 expressions as the cut's test)."""
    o = np.array([float(np.float32(c)) for c in cam.position])
    b = scene.bound.astype(np.float64)
    d = b[:, :3] - o
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    a = 2.0 * max(float(cam.fx), float(cam.fy)) * b[:, 3]
    lhs = a * a
    return (scene.child_count > 0) & (lhs > tau * tau * d2) & (lhs <= S_HI * S_HI * d2)


def _walk(scene, thr, cut):
    """Per threshold-cut node: its ancestor-or-self in `cut` (exactly one)."""
    in_cut = np.zeros(scene.n, bool)
    in_cut[cut] = True
    first = np.full(thr.size, -1)
    hits = np.zeros(thr.size, int)
    cur = thr.astype(np.int64)
    while (cur >= 0).any():
        alive = cur >= 0
        h = alive & in_cut[np.where(alive, cur, 0)]
        hits += h
        first = np.where(h & (first < 0), cur, first)
        cur = np.where(alive, scene.parent[np.where(alive, cur, 0)], -1)
    assert np.all(hits == 1)
    return first


def _learned(scene, cam, params, p_star=0.5, margin=1e-12, **kw):
    return O.cut_learned(scene, cam, params, np.zeros(8), np.ones(8), p_star, S_HI, margin=margin, **kw)


def test_constant_logits(plan):
    scene, cams = plan
    for cam in cams[1:4]:
        thr = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
        ids, amb = _learned(scene, cam, _net(b3=1.0))
        assert amb.size == 0
        np.testing.assert_array_equal(ids, thr)
        ids, amb = _learned(scene, cam, _net(b3=-1.0))
        assert amb.size == 0
        first = _walk(scene, thr, ids)
        band = _band(scene, cam)
        # each kept node is the highest band node above its leaves, or the
        # threshold node itself when no band node is above it
        for k, f in zip(thr[:2000], first[:2000]):
            anc = []
            a = int(k)
            while a >= 0:
                anc.append(a)
                a = int(scene.parent[a])
            top = [a for a in anc[::-1] if band[a]]
            assert f == (top[0] if top else k)
        assert ids.size < thr.size


@pytest.mark.parametrize("feature,cut_at", [(2, 0.94), (3, 4.5), (6, 4.5)])
def test_one_feature_networks(plan, feature, cut_at):
    """logit = x_f - c: a candidate is refined iff its feature f (opacity,
    child count, level) is at least c."""
    scene, cams = plan
    cam = cams[2]
    lvl = np.zeros(scene.n, int)
    for l in range(len(scene.level_offset) - 1):
        lvl[scene.level_offset[l]:scene.level_offset[l + 1]] = l
    value = {2: scene.opacity.astype(np.float64), 3: scene.child_count.astype(np.float64), 6: lvl.astype(np.float64)}
    ids, amb = _learned(scene, cam, _net(b3=-cut_at, feature=feature))
    assert amb.size == 0
    thr = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    first = _walk(scene, thr, ids)
    band = _band(scene, cam)
    in_cut = np.zeros(scene.n, bool)
    in_cut[ids] = True
    kept = band & in_cut
    assert kept.any()
    assert np.all(value[feature][kept] < cut_at)
    # expanded band nodes: band ancestors (strict) of the nodes reached
    reached = set()
    for f in np.unique(first):
        a = int(scene.parent[f])
        while a >= 0:
            reached.add(a)
            a = int(scene.parent[a])
    exp = np.array(sorted(k for k in reached if band[k]), dtype=np.int64)
    assert exp.size and np.all(value[feature][exp] >= cut_at)


def test_projected_size_feature(plan):
    """logit = log(2 f r / |c - o|) - log(s): refined iff the projected size
    reaches s (closed form from the bounding spheres)."""
    scene, cams = plan
    cam = cams[3]
    o = np.array([float(np.float32(c)) for c in cam.position])
    b = scene.bound.astype(np.float64)
    size = 2.0 * max(float(cam.fx), float(cam.fy)) * b[:, 3] / np.linalg.norm(b[:, :3] - o, axis=1)
    band = _band(scene, cam)
    s = float(np.median(size[band]))
    ids, amb = _learned(scene, cam, _net(b3=-math.log(s), feature=0))
    in_cut = np.zeros(scene.n, bool)
    in_cut[ids] = True
    kept = band & in_cut & ~np.isin(np.arange(scene.n), amb)
    assert kept.any() and np.all(size[kept] < s)
    assert np.any(band & ~in_cut & (size >= s))


def test_zero_logit_is_undecided_and_flips(plan):
    scene, cams = plan
    cam = cams[1]
    ids, amb = _learned(scene, cam, _net(b3=0.0))
    thr = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    np.testing.assert_array_equal(ids, thr)          # z = z* refines
    band = _band(scene, cam)
    assert amb.size > 0 and np.all(band[amb])
    # flipping the first undecided candidate keeps it and drops its subtree
    u = int(amb[0])
    ids2, _ = _learned(scene, cam, _net(b3=0.0), flip=[u])
    assert u in set(ids2.tolist()) and u not in set(ids.tolist())
    _walk(scene, thr, ids2)
    # a decided candidate cannot be flipped
    _, amb_d = _learned(scene, cam, _net(b3=1.0))
    assert amb_d.size == 0
    with pytest.raises(ValueError):
        _learned(scene, cam, _net(b3=1.0), flip=[u])


def _net_linear(feature, c):
    """Parameters of a network whose logit is exactly x_f - c: hidden unit 0
    carries relu(x_f - c), unit 1 relu(c - x_f), both passed through the
    second layer, and the output is their difference."""
    q = {"W1": np.zeros((32, 8)), "b1": np.zeros(32), "W2": np.zeros((32, 32)), "b2": np.zeros(32),
         "w3": np.zeros(32), "b3": 0.0}
    q["W1"][0, feature], q["b1"][0] = 1.0, -c
    q["W1"][1, feature], q["b1"][1] = -1.0, c
    q["W2"][0, 0] = q["W2"][1, 1] = 1.0
    q["w3"][0], q["w3"][1] = 1.0, -1.0
    return M.pack(q)


def _features_numpy(scene, cam, feature):
    """Feature `feature` of every node seen from `cam`, computed here from the
    scene arrays with numpy and scipy (Sec. III-B nodes; the feature list of
    the learned rule): 1 log camera depth of the bounding-sphere centre
    (floored at znear), 4 variance of the children's DC colour, 5 |cos|
    between the view ray and the thinnest axis, 7 log projected size of the
    parent (a root's own)."""
    from scipy.spatial.transform import Rotation

    o = np.asarray(cam.position, np.float32).astype(np.float64)
    Rv = np.asarray(cam.R, np.float32).astype(np.float64)
    b = scene.bound.astype(np.float64)
    d = b[:, :3] - o
    f = 2.0 * max(float(cam.fx), float(cam.fy))
    if feature == 1:
        depth = d @ Rv[2]                       # forward row of world -> camera
        return np.log(np.maximum(depth, float(np.float32(cam.znear))))
    if feature == 4:
        C0 = 1.0 / (2.0 * math.sqrt(math.pi))   # degree-0 real harmonic
        out = np.zeros(scene.n)
        dc = scene.sh[:, 0, :].astype(np.float64)
        for k in np.nonzero(scene.child_count > 1)[0]:
            kids = dc[scene.first_child[k]:scene.first_child[k] + scene.child_count[k]]
            out[k] = C0 * C0 * float(np.var(kids, axis=0).sum())
        return out
    if feature == 5:
        q = scene.quats.astype(np.float64)
        rot = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()        # scipy takes (x, y, z, w)
        thin = np.argmin(scene.scales, axis=1)
        axis = rot[np.arange(scene.n), :, thin]                            # column of the least scale
        return np.abs(np.einsum("ij,ij->i", d, axis)) / np.linalg.norm(d, axis=1)
    if feature == 7:
        size = f * b[:, 3] / np.linalg.norm(d, axis=1)
        par = np.where(scene.parent >= 0, scene.parent, np.arange(scene.n))
        return np.log(size[par])
    raise ValueError(feature)


@pytest.mark.parametrize("feature", [1, 4, 5, 7])
def test_feature_pins(plan, feature):
    """logit = x_f - c with the feature computed independently here: a
    candidate is refined iff its feature reaches c.  The split value lies
    halfway between two neighbouring feature values of the candidates, so a
    misread feature (a wrong coefficient stride, the largest axis for the
    thinnest, the node's own size for its parent's, the distance for the
    depth) puts candidates on the wrong side."""
    scene, cams = plan
    lvl = np.zeros(scene.n, int)
    for l in range(len(scene.level_offset) - 1):
        lvl[scene.level_offset[l]:scene.level_offset[l + 1]] = l
    for cam in cams[2:4]:
        value = _features_numpy(scene, cam, feature)
        band = _band(scene, cam)
        # split value from the candidates of the deepest level holding
        # candidates, so that some of them are reached and kept whichever
        # feature decides (for the parent's size the level above decides
        # whether they are reached at all)
        deep = band & (lvl == lvl[band].max())
        vals = np.unique(value[deep])
        assert vals.size > 20
        gaps = np.diff(vals)
        # widest gap among the middle half of the sorted values
        lo, hi = vals.size // 4, 3 * vals.size // 4
        i = lo + int(np.argmax(gaps[lo:hi]))
        assert gaps[i] > 1e-9 * max(1.0, abs(vals[i]))
        c = 0.5 * (vals[i] + vals[i + 1])
        ids, amb = _learned(scene, cam, _net_linear(feature, c))
        assert amb.size == 0
        thr = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
        first = _walk(scene, thr, ids)
        in_cut = np.zeros(scene.n, bool)
        in_cut[ids] = True
        kept = band & in_cut
        assert kept.any()
        assert np.all(value[kept] < c)
        reached = set()
        for fnode in np.unique(first):
            a = int(scene.parent[fnode])
            while a >= 0:
                reached.add(a)
                a = int(scene.parent[a])
        exp = np.array(sorted(k for k in reached if band[k]), dtype=np.int64)
        assert exp.size and np.all(value[exp] >= c)
