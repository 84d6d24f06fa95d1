"""Edge cases of the GPU path against the oracle: a single Gaussian, images
of one pixel, one row, one column and exactly one tile, a Gaussian behind
the camera, views batched with very different sizes, the backward
pass of a one-Gaussian scene, and SH degrees 0 to 2 forward and backward."""
import math

import numpy as np
import pytest

from oracle import grad as G
from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, make_random_box, yaw_camera
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


def _one(o=0.7, at=(0.0, 0.0, 0.0), scale=0.05):
    sh = np.array([[0.4, -0.2, 0.1]], np.float32)
    return Scene(np.array([at], np.float32), np.full((1, 3), scale, np.float32),
                 np.array([[0.9, 0.1, -0.2, 0.3]], np.float32), np.array([o], np.float32), sh, 0)


def _check(R, scene, cams):
    R.load_scene(scene)
    R.set_cameras(cams)
    outs = R.render()
    torch.cuda.synchronize()
    for cam, (rgb, dep, alp) in zip(cams, outs):
        res, _, _ = O.render(scene, cam)
        g = parity.gpu_pixels(rgb.cpu().numpy(), dep.cpu().numpy(), alp.cpu().numpy(), res.px, res.py)
        ok, best, skipped = parity.branch_errors(g, res)
        assert ok.all(), (cam.width, cam.height, parity.summary(ok, best, skipped))


@pytest.mark.parametrize("W_,H_", [(1, 1), (1, 40), (40, 1), (16, 16), (17, 33)])
def test_single_gaussian_tiny_images(R, W_, H_):
    """One Gaussian seen from 2 m, the principal point at the image centre:
    it covers the centre of every image size."""
    cam = yaw_camera(W_, H_, 30.0, (0.0, -2.0, 0.0), math.pi / 2, bg=(0.2, 0.3, 0.4))
    _check(R, _one(), [cam])


def test_gaussian_behind_the_camera_leaves_background(R):
    cam = yaw_camera(24, 16, 20.0, (0.0, -2.0, 0.0), -math.pi / 2, bg=(0.5, 0.25, 0.125))
    scene = _one()
    R.load_scene(scene)
    R.set_cameras([cam])
    rgb, dep, alp = (t.cpu().numpy() for t in R.render()[0])
    assert np.all(alp == 0) and np.all(dep == 0)
    np.testing.assert_array_equal(rgb[:, 0, 0], np.array([0.5, 0.25, 0.125], np.float32))
    _check(R, scene, [cam])


def test_batch_of_very_different_views(R):
    scene = make_random_box(3000, seed=11, box=(2.0, 2.0, 2.0))
    cams = [yaw_camera(1, 1, 1.0, (1.0, -1.0, 1.0), math.pi / 2),
            yaw_camera(300, 200, 250.0, (1.0, -1.5, 1.0), math.pi / 2),
            yaw_camera(16, 48, 20.0, (3.0, 1.0, 1.0), math.pi),
            yaw_camera(47, 3, 40.0, (1.0, 1.0, 1.0), 0.3)]
    _check(R, scene, cams)


def test_backward_of_one_gaussian(R):
    scene = _one(o=0.6)
    cam = yaw_camera(20, 14, 24.0, (0.0, -2.0, 0.0), math.pi / 2)
    rng = np.random.default_rng(1)
    P = cam.width * cam.height
    g = [rng.normal(size=(P, 3)), rng.normal(size=P), rng.normal(size=P)]
    g = [a.astype(np.float32).astype(np.float64) for a in g]
    res, _, _ = O.render(scene, cam)
    assert (res.flags == 0).all()
    want, _ = G.gradients(scene, cam, *g)
    R.load_scene(scene)
    R.set_cameras([cam])
    R.render()
    got = R.backward([(torch.from_numpy(np.ascontiguousarray(g[0].T.reshape(3, cam.height, cam.width),
                                                             dtype=np.float32)).cuda(),
                       torch.from_numpy(g[1].reshape(cam.height, cam.width).astype(np.float32)).cuda(),
                       torch.from_numpy(g[2].reshape(cam.height, cam.width).astype(np.float32)).cuda())])
    torch.cuda.synchronize()
    # the Gaussian is isotropic: its rotation gradient is rounding noise on
    # both sides, so the absolute floor comes from the largest gradient
    top = max(np.abs(w).max() for w in want.values())
    for k, w in want.items():
        gk = got[k].cpu().numpy().astype(np.float64).reshape(w.shape)
        np.testing.assert_allclose(gk, w, rtol=1e-4, atol=5e-5 * top, err_msg=k)


@pytest.mark.parametrize("deg", [1, 2])
def test_sh_degrees_one_and_two(R, deg):
    """Scenes of SH degree 1 and 2 (the projection kernel is instantiated per
    degree, and the coefficient loads differ: 16-byte loads for degree 1,
    scalar loads for degree 2) against the oracle, full frame."""
    base = make_random_box(2500, seed=20 + deg, box=(2.0, 2.0, 2.0))
    rng = np.random.default_rng(30 + deg)
    K = (deg + 1) ** 2
    sh = np.zeros((base.n, K, 3), np.float32)
    sh[:, 0, :] = np.asarray(base.sh, np.float32).reshape(base.n, -1, 3)[:, 0, :]
    sh[:, 1:, :] = rng.normal(0, 0.15, size=(base.n, K - 1, 3))
    scene = Scene(base.means, base.scales, base.quats, base.opacity, sh.reshape(base.n, K * 3), deg)
    cams = [yaw_camera(96, 64, 80.0, (1.0, -1.2, 1.0), math.pi / 2),
            yaw_camera(80, 80, 70.0, (3.2, 1.0, 1.0), math.pi)]
    _check(R, scene, cams)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_backward_sh_degrees_zero_to_two(R, deg):
    """The backward pass of scenes of SH degree 0, 1 and 2 (its kernels are
    instantiated per degree) against the FP64 gradient oracle."""
    base = make_random_box(300, seed=40 + deg, box=(1.2, 1.2, 1.2))
    rng = np.random.default_rng(50 + deg)
    K = (deg + 1) ** 2
    sh = np.zeros((base.n, K, 3), np.float32)
    sh[:, 0, :] = np.asarray(base.sh, np.float32).reshape(base.n, -1, 3)[:, 0, :] * 0.6
    if K > 1:
        sh[:, 1:, :] = rng.normal(0, 0.06, size=(base.n, K - 1, 3))
    scales = np.exp(rng.uniform(np.log(0.02), np.log(0.12), size=(base.n, 3))).astype(np.float32)
    scene = Scene(base.means, scales, base.quats, base.opacity, sh.reshape(base.n, K * 3), deg)
    cam = yaw_camera(64, 48, 58.0, (0.6, -1.3, 0.6), math.pi / 2)
    res, _, _ = O.render(scene, cam, O.MODE_THRESHOLD, 1.0)
    P = cam.width * cam.height
    g = [rng.normal(size=(P, 3)), rng.normal(size=P) * 0.2, rng.normal(size=P)]
    p = G.leaf_params(scene)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    _, _, _, cap = G.render(p, scene.sh_degree, cam, xx.ravel(), yy.ravel())
    bad = (res.flags != 0) | cap
    for a in g:
        a[bad] = 0.0
    g = [a.astype(np.float32).astype(np.float64) for a in g]
    want, _ = G.gradients(scene, cam, *g)
    R.load_scene(scene)
    R.set_cameras([cam])
    R.render()
    got = R.backward([(torch.from_numpy(np.ascontiguousarray(g[0].T.reshape(3, cam.height, cam.width),
                                                             dtype=np.float32)).cuda(),
                       torch.from_numpy(g[1].reshape(cam.height, cam.width).astype(np.float32)).cuda(),
                       torch.from_numpy(g[2].reshape(cam.height, cam.width).astype(np.float32)).cuda())])
    torch.cuda.synchronize()
    for k, w in want.items():
        gk = got[k].cpu().numpy().astype(np.float64).reshape(w.shape)
        top = np.abs(w).max()
        assert top > 0, k
        np.testing.assert_allclose(gk, w, rtol=1e-4, atol=5e-5 * top, err_msg=f"{k} degree {deg}")


@pytest.mark.parametrize("n16", [1, 255, 1024, 1025, (1 << 20) + 3])
def test_stream_copy_probe(R, n16):
    """The bandwidth probe copies exactly (sizes in 16-byte words, including
    ragged tails of its 4 KiB chunks) and rejects unaligned sizes."""
    from paper_2603_15186_amd import hgs
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (4 * n16,), dtype=torch.int32, device="cuda")
    dst = torch.zeros(4 * n16 + 4, dtype=torch.int32, device="cuda")
    R.stream_copy(src, dst[:4 * n16])
    torch.cuda.synchronize()
    assert torch.equal(src, dst[:4 * n16])
    assert int(dst[4 * n16:].abs().sum()) == 0
    odd = torch.zeros(3, dtype=torch.int32, device="cuda")
    with pytest.raises(hgs.HgsError) as ei:
        R.stream_copy(odd, odd.clone())
    assert ei.value.status == hgs.HGS_E_INVALID
