"""GPU level-of-detail transition blending (NavGSim Sec. III-B: transition
regions between levels are smoothly interpolated) against the FP64 oracle,
through the C ABI.

The reading: a cut node g with parent p is drawn as p + t (g - p) (mean,
covariance, SH), t = clamp((s_p - tau) / (s_p - s_g), 0, 1) with s_p, s_g
the parent's and the node's projected bounding-sphere sizes; the first of
p's children in the view's cut takes opacity o_p + t (o_g - o_p), the
others t o_g.  Scene: the floor plan at a tenth of its leaves (457k nodes);
thresholds of 64 and 128 px put most cut nodes inside the transition band,
0.01 px puts none there.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15186_amd.synth import workloads as W, yaw_camera
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_15186_amd import hgs
    r = hgs.Renderer(0)
    yield r
    r.close()


@pytest.fixture(scope="module")
def plan():
    return W.plan2m(scale=0.2, n_poses=6)


def _hgs():
    from paper_2603_15186_amd import hgs
    return hgs


def _render(R, scene, cams, tau, blend):
    hgs = _hgs()
    R.load_scene(scene)
    R.set_cameras(cams)
    R.set_lod(1, tau)
    R.set_option(hgs.HGS_OPT_LOD_BLEND, 1 if blend else 0)
    try:
        outs = R.render()
        torch.cuda.synchronize()
    finally:
        R.set_option(hgs.HGS_OPT_LOD_BLEND, 0)
    return [(a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()) for a, b, c in outs]


def _small_cam(c, W_=200, H_=117):
    return yaw_camera(W_, H_, 900.0 * W_ / 1280.0, c.position, math.atan2(c.R[2][1], c.R[2][0]))


@pytest.mark.parametrize("tau", [64.0, 128.0])
def test_blended_projection_matches_oracle(R, plan, tau):
    """Per cut entry of four 1280x720 views: validity, 2D mean, conic,
    depth key (bit-exact), colour and opacity of the blended Gaussian."""
    scene, cams = plan
    views = list(cams[1:5])
    _render(R, scene, views, tau, blend=True)
    interior = 0
    for v, cam in enumerate(views):
        ids = R.get_cut(v)
        assert np.array_equal(ids, O.cut(scene, cam, O.MODE_THRESHOLD, tau))
        g = R.get_projected(v)
        pr, t = O.project_blend(scene, ids, cam, tau, with_t=True)
        interior += int(((t > 0) & (t < 1)).sum())
        valid = g[:, 11] > 0
        assert np.array_equal(valid, pr[:, 0] > 0), v
        pv, gv = pr[valid], g[valid]
        for k, f in ((0, "u"), (1, "v")):
            err = np.abs(gv[:, k] - pv[:, O.PF[f]])
            assert np.all(err <= 1e-4 + 1.2e-7 * np.abs(pv[:, O.PF[f]])), (v, f, err.max())
        scale = np.sqrt(pv[:, O.PF["A"]] * pv[:, O.PF["C"]])
        for k, f in ((2, "A"), (3, "B"), (4, "C")):
            err = np.abs(gv[:, k] - pv[:, O.PF[f]]) / scale
            assert err.max() <= 1e-5, (v, f, err.max())
        np.testing.assert_array_equal(gv[:, 8], pv[:, O.PF["zkey"]].astype(np.float32))
        np.testing.assert_allclose(gv[:, 9], pv[:, O.PF["opacity"]], rtol=1e-6, atol=1e-7)
        # later siblings (opacity t o_g) are present, in every view
        par = scene.parent[ids]
        prev = np.r_[-1, ids[:-1]]
        later = (par >= 0) & (prev >= scene.first_child[np.maximum(par, 0)]) & (prev < ids)
        assert ((t < 1) & later).sum() > 100, v
        vis = gv[:, 10] > 0
        for k, f in ((5, "r"), (6, "g"), (7, "b")):
            np.testing.assert_allclose(gv[vis, k], pv[vis, O.PF[f]], atol=2e-6)
    assert interior > 1000


@pytest.mark.parametrize("tau,cam_i", [(64.0, 2), (128.0, 3)])
def test_blended_full_frame_parity(R, plan, tau, cam_i):
    """Every pixel of a 200x117 view (ragged tiles) within the renderer's
    tolerance of one of the oracle's branches."""
    scene, cams = plan
    cam = _small_cam(cams[cam_i])
    img = _render(R, scene, [cam], tau, blend=True)[0]
    res, ids, _ = O.render(scene, cam, O.MODE_THRESHOLD, tau, blend=True)
    assert np.array_equal(R.get_cut(0), ids)
    g = parity.gpu_pixels(*img, res.px, res.py)
    ok, best, skipped = parity.branch_errors(g, res)
    msg = parity.summary(ok, best, skipped)
    print(msg, flush=True)
    assert ok.all(), msg
    assert not skipped.any(), msg
    # blending changes the picture at this threshold
    plain = _render(R, scene, [cam], tau, blend=False)[0]
    assert np.abs(plain[0] - img[0]).max() > 1e-2


def test_weights_of_one_leave_the_image_unchanged(R, plan):
    """At a 0.01 px threshold every parent spans more than twice the
    threshold (t = 1): blending on and off give the same image bitwise."""
    scene, cams = plan
    views = [_small_cam(cams[1], 160, 96), _small_cam(cams[4], 96, 64)]
    on = _render(R, scene, views, 0.01, blend=True)
    off = _render(R, scene, views, 0.01, blend=False)
    for v in range(len(views)):
        for a, b in zip(on[v], off[v]):
            assert np.array_equal(a, b), v


def test_blending_is_independent_of_batching(R, plan):
    """Blended views rendered together equal the same views rendered alone."""
    scene, cams = plan
    views = [_small_cam(cams[1], 320, 240), _small_cam(cams[3], 128, 72), _small_cam(cams[5], 33, 17)]
    batch = _render(R, scene, views, 96.0, blend=True)
    for v, cam in enumerate(views):
        single = _render(R, scene, [cam], 96.0, blend=True)[0]
        for a, b in zip(batch[v], single):
            assert np.array_equal(a, b), v


def test_blended_image_is_continuous_where_a_node_is_refined(R, plan):
    """The GPU renders the two sides of a refine event (adjacent
    single-precision camera positions, only one node refined between them):
    the blended images differ by little more than the camera's one-ulp move
    makes, the plain ones jump."""
    from tests.test_blend_oracle import refine_events
    scene, cams = plan
    tau = 40.0
    seen = 0
    for node, a, b, ca, cb in refine_events(scene, cams, tau):
        on = _render(R, scene, [a, b], tau, blend=True)
        assert np.array_equal(R.get_cut(0), ca) and np.array_equal(R.get_cut(1), cb)
        off = _render(R, scene, [a, b], tau, blend=False)
        jump = np.abs(off[0][0] - off[1][0])
        step = np.abs(on[0][0] - on[1][0])
        print(f"node {node}: plain max {jump.max():.4f} mean {jump.mean():.2e}; "
              f"blended max {step.max():.4f} mean {step.mean():.2e}", flush=True)
        if jump.max() > 0.02:
            assert step.max() < 0.2 * jump.max() and step.mean() < 0.05 * jump.mean()
            seen += 1
    assert seen >= 2
