"""GPU backward pass through the C ABI against the FP64 gradient oracle.

Upstream gradients are random per pixel and zero at pixels where a forward
decision lies within the oracle's fork margins or an alpha is within 1e-6
of the 0.99 cap (the gradient is discontinuous there and either side is
valid).  Tolerance per parameter kind: |gpu - oracle| <= 1e-4 |oracle| +
5e-5 max|oracle| (FP32 per-pixel arithmetic and atomic sums against FP64;
the errors seen are about 1e-6 of the largest gradient).
"""
import math

import numpy as np
import pytest

from oracle import grad as G
from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, make_random_box, workloads as W, yaw_camera

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELDS = ("means", "scales", "quats", "opacity", "sh")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_15186_amd import hgs
    r = hgs.Renderer(0)
    yield r
    r.close()


def _scene(n, seed, deg=3, box=(1.2, 1.2, 1.2)):
    s = make_random_box(n, seed=seed, box=box)
    rng = np.random.default_rng(seed + 100)
    K = (deg + 1) ** 2
    sh = np.zeros((n, K, 3), np.float32)
    sh[:, 0, :] = np.asarray(s.sh, np.float32).reshape(n, -1, 3)[:, 0, :] * 0.6
    sh[:, 1:, :] = rng.normal(0, 0.06, size=(n, K - 1, 3))
    s.scales[:] = np.exp(rng.uniform(np.log(0.02), np.log(0.12), size=(n, 3))).astype(np.float32)
    return Scene(s.means, s.scales, s.quats, s.opacity, sh.reshape(n, K * 3), deg)


def _upstream(scene, cam, rng, ids=None):
    """Random image gradients, zero where the oracle's decisions are
    ambiguous; returns (g_rgb (P, 3), g_depth, g_alpha) as float32."""
    res, _, _ = O.render(scene, cam, O.MODE_THRESHOLD, 1.0, ids=ids)
    p = G.leaf_params(scene, ids)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    _, _, _, cap = G.render(p, scene.sh_degree, cam, xx.ravel(), yy.ravel())
    bad = (res.flags != 0) | cap
    P = cam.width * cam.height
    g = [rng.normal(size=(P, 3)), rng.normal(size=P) * 0.2, rng.normal(size=P)]
    for a in g:
        a[bad] = 0.0
    return [a.astype(np.float32).astype(np.float64) for a in g], bad


def _to_gpu(cam, g):
    H, Wd = cam.height, cam.width
    return (torch.from_numpy(np.ascontiguousarray(g[0].T.reshape(3, H, Wd), dtype=np.float32)).cuda(),
            torch.from_numpy(g[1].reshape(H, Wd).astype(np.float32)).cuda(),
            torch.from_numpy(g[2].reshape(H, Wd).astype(np.float32)).cuda())


def _compare(got, want, label=""):
    for f in FIELDS:
        gg = got[f].cpu().numpy().astype(np.float64).reshape(want[f].shape)
        ww = want[f]
        scale = np.abs(ww).max()
        err = np.abs(gg - ww)
        lim = 1e-4 * np.abs(ww) + 5e-5 * scale
        worst = float((err / np.maximum(lim, 1e-30)).max())
        print(f"{label} {f}: max|g| {scale:.3g}, worst {worst:.3g}x tol", flush=True)
        assert scale > 0, f
        assert np.all(err <= lim), (f, worst)


def _colours_away_from_clamp(scene, cam, ids=None):
    p = G.leaf_params(scene, ids)
    pr = G.project(p["means"], p["scales"], p["quats"], p["opacity"], p["sh"], scene.sh_degree, cam)
    raw = pr["raw"].numpy()[pr["valid"].numpy()]
    return np.all((np.abs(raw) > 1e-4) & (np.abs(raw - 1) > 1e-4))


@pytest.mark.parametrize("keep", [0, 1])
@pytest.mark.parametrize("seed,W_,H_", [(5, 72, 56), (6, 100, 45)])
def test_flat_scene_gradients_match_oracle(R, seed, W_, H_, keep):
    """keep = 1: the render keeps its pixel states and the backward pass
    reads them; keep = 0: the backward pass replays the forward walk."""
    from paper_2603_15186_amd import hgs
    scene = _scene(400, seed)
    cam = yaw_camera(W_, H_, 0.9 * W_, (0.6, -1.3, 0.6), math.pi / 2)
    assert _colours_away_from_clamp(scene, cam)
    rng = np.random.default_rng(seed)
    g, bad = _upstream(scene, cam, rng)
    assert bad.mean() < 0.02
    want, _ = G.gradients(scene, cam, *g)
    R.load_scene(scene)
    R.set_cameras([cam])
    R.set_option(hgs.HGS_OPT_KEEP_STATE, keep)
    try:
        R.render()
        got = R.backward([_to_gpu(cam, g)])
        torch.cuda.synchronize()
    finally:
        R.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
    _compare(got, want, f"seed {seed} keep {keep}")


@pytest.mark.parametrize("batch,persistent", [(128, 0), (256, 0), (64, 1)])
def test_kept_states_leave_images_and_gradients_unchanged(R, batch, persistent):
    """Images are bit-identical with and without kept pixel states, and the
    backward pass from kept states equals the replaying one up to the
    order of its atomic sums (each compositor variant keeps the states)."""
    from paper_2603_15186_amd import hgs
    scene, cams = W.plan2m(scale=0.02, n_poses=6)
    views = [yaw_camera(160, 90, 900.0 * 160 / 1280, c.position, math.atan2(c.R[2][1], c.R[2][0]))
             for c in cams[:3]]
    R.load_scene(scene)
    R.set_cameras(views)
    R.set_lod(1, 1.0)
    gen = torch.Generator(device="cuda").manual_seed(3)
    res = {}
    R.set_option(hgs.HGS_OPT_BATCH_DEPTH, batch)
    R.set_option(hgs.HGS_OPT_PERSISTENT, persistent)
    try:
        for keep in (0, 1):
            R.set_option(hgs.HGS_OPT_KEEP_STATE, keep)
            outs = R.render()
            grads = [tuple(torch.randn(t.shape, generator=gen.manual_seed(7 + v), device="cuda") for t in o)
                     for v, o in enumerate(outs)]
            got = R.backward(grads)
            torch.cuda.synchronize()
            res[keep] = ([tuple(t.cpu().numpy() for t in o) for o in outs], {k: v.cpu().numpy() for k, v in got.items()})
    finally:
        R.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
        R.set_option(hgs.HGS_OPT_BATCH_DEPTH, 256)
        R.set_option(hgs.HGS_OPT_PERSISTENT, 0)
    for a, b in zip(res[0][0], res[1][0]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    for f in FIELDS:
        a, b = res[0][1][f], res[1][1][f]
        scale = np.abs(a).max()
        assert scale > 0, f
        np.testing.assert_allclose(b, a, rtol=1e-4, atol=1e-5 * scale, err_msg=f)


def test_two_views_sum_their_gradients(R):
    scene = _scene(300, 7)
    cams = [yaw_camera(64, 48, 60.0, (0.6, -1.3, 0.6), math.pi / 2),
            yaw_camera(48, 40, 45.0, (-1.0, 0.5, 0.7), 0.1)]
    rng = np.random.default_rng(7)
    want = None
    gpu_in = []
    for cam in cams:
        assert _colours_away_from_clamp(scene, cam)
        g, _ = _upstream(scene, cam, rng)
        w, _ = G.gradients(scene, cam, *g)
        want = w if want is None else {k: want[k] + w[k] for k in FIELDS}
        gpu_in.append(_to_gpu(cam, g))
    R.load_scene(scene)
    R.set_cameras(cams)
    R.render()
    got = R.backward(gpu_in)
    torch.cuda.synchronize()
    _compare(got, want, "two views")
    # accumulation into given arrays
    got2 = R.backward(gpu_in, out={k: v.clone() for k, v in got.items()})
    torch.cuda.synchronize()
    for k in FIELDS:
        np.testing.assert_allclose(got2[k].cpu().numpy(), 2 * got[k].cpu().numpy(), rtol=1e-5, atol=1e-6)


def test_hierarchy_cut_gradients_match_oracle(R):
    """The threshold cut of a reduced floor plan: gradients land on the
    cut's nodes only and match the oracle's gradients of the same cut."""
    scene, cams = W.plan2m(scale=0.02, n_poses=6)
    c = cams[2]
    cam = yaw_camera(96, 64, 900.0 * 96 / 1280, c.position, math.atan2(c.R[2][1], c.R[2][0]))
    ids = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
    rng = np.random.default_rng(8)
    g, bad = _upstream(scene, cam, rng, ids=ids)
    want, _ = G.gradients(scene, cam, *g, ids=ids)
    from paper_2603_15186_amd import hgs
    R.load_scene(scene)
    R.set_cameras([cam])
    R.set_lod(1, 1.0)
    R.set_option(hgs.HGS_OPT_KEEP_STATE, 1)
    try:
        R.render()
        assert np.array_equal(R.get_cut(0), ids)
        got = R.backward([_to_gpu(cam, g)])
        torch.cuda.synchronize()
    finally:
        R.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
    sub = {k: v.cpu()[torch.from_numpy(ids.astype(np.int64))] for k, v in got.items()}
    _compare(sub, want, "plan cut")
    mask = np.ones(scene.n, bool)
    mask[ids] = False
    for k in FIELDS:
        assert not got[k].cpu().numpy()[mask].any(), k


def test_backward_preconditions(R):
    from paper_2603_15186_amd import hgs
    scene = _scene(50, 9)
    r = hgs.Renderer(0)
    try:
        r.load_scene(scene)
        cam = yaw_camera(32, 32, 30.0, (0.6, -1.3, 0.6), math.pi / 2)
        r.set_cameras([cam])
        with pytest.raises(hgs.HgsError) as ei:
            r.backward([(None, None, None)])
        assert ei.value.status == hgs.HGS_E_STATE
        r.render()
        with pytest.raises(ValueError):
            r.backward([])
        out = r.backward([(None, None, None)])
        torch.cuda.synchronize()
        assert all(not out[k].any() for k in FIELDS)
    finally:
        r.close()


def test_kept_states_through_graph_replays(R):
    """Renders replayed from a captured hipGraph keep their pixel states:
    the backward pass after each replay equals the one after an eager
    render (up to the order of its atomic sums), replay after replay."""
    from paper_2603_15186_amd import hgs
    scene, cams = W.plan2m(scale=0.02, n_poses=6)
    views = [yaw_camera(128, 72, 900.0 * 128 / 1280, c.position, math.atan2(c.R[2][1], c.R[2][0]))
             for c in cams[2:4]]
    R.load_scene(scene)
    R.set_cameras(views)
    R.set_lod(1, 1.0)
    gen = torch.Generator(device="cuda")
    try:
        R.set_option(hgs.HGS_OPT_KEEP_STATE, 1)
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        outs = R.render()
        grads = [tuple(torch.randn(t.shape, generator=gen.manual_seed(11 + v), device="cuda") for t in o)
                 for v, o in enumerate(outs)]
        want = {k: v.cpu().numpy() for k, v in R.backward(grads).items()}
        torch.cuda.synchronize()
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 1)
        for rep in range(3):
            R.render(outs)
            got = R.backward(grads)
            torch.cuda.synchronize()
            for f in FIELDS:
                scale = np.abs(want[f]).max()
                assert scale > 0, f
                np.testing.assert_allclose(got[f].cpu().numpy(), want[f], rtol=1e-4, atol=1e-5 * scale,
                                           err_msg=f"{f} replay {rep}")
        assert R.stats()["graph_launches"] >= 3
    finally:
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        R.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
