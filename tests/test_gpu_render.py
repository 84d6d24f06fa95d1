"""GPU parity of the HIP renderer against the FP64 oracle, through the C ABI.

Sizes: the 20k-Gaussian random box at 256x256 (16 x 16 tiles) in full; the
floor-plan scene at reduced leaf counts in full frames with a ragged tile
edge; the 2M-leaf floor plan at 1280x720 on sampled pixels and bit-exact
cuts.  The radix sort is checked bit-exactly against numpy's stable sort.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15186_amd.synth import workloads as W, yaw_camera
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _hgs():
    from paper_2603_15186_amd import hgs
    return hgs


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _hgs().Renderer(0)
    yield r
    r.close()


def _render(r, scene, cams, mode=1, tau=1.0, **opts):
    hgs = _hgs()
    r.load_scene(scene)
    r.set_cameras(cams)
    if scene.parent is not None:
        r.set_lod(mode, tau)
    for k, v in opts.items():
        r.set_option(getattr(hgs, "HGS_OPT_" + k.upper()), v)
    outs = r.render()
    torch.cuda.synchronize()
    return [(a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()) for a, b, c in outs]


def _check_full(img, scene, cam, mode=O.MODE_THRESHOLD, tau=1.0, ids=None):
    res, _, _ = O.render(scene, cam, mode, tau, ids=ids)
    px, py = res.px, res.py
    g = parity.gpu_pixels(*img, px, py)
    ok, best, skipped = parity.branch_errors(g, res)
    msg = parity.summary(ok, best, skipped)
    print(msg, flush=True)
    assert ok.all(), msg
    assert not skipped.any(), msg
    return res


# ------------------------------------------------------------------ sort

# sizes around the 8192-element histogram groups, past 1024 groups (a
# workgroup then owns several groups) and past 8192 * 8192 elements (groups
# then grow to keep at most 8192)
@pytest.mark.parametrize("n,bits,digit", [(1, 8, 11), (1000, 8, 8), (300001, 12, 11), (300001, 12, 6),
                                          (300001, 19, 11), (300001, 19, 8), (2_000_003, 32, 11),
                                          (2_000_003, 32, 8), (5_000_000, 17, 11), (5_000_000, 17, 9),
                                          (8191, 10, 9), (8192, 10, 9), (8193, 13, 6),
                                          (8_388_608, 18, 6), (9_000_005, 18, 8), (9_000_005, 32, 10),
                                          (70_000_001, 18, 6)])
def test_radix_sort_bit_exact(R, n, bits, digit):
    hgs = _hgs()
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)   # bits above key_bits ignored
    if n > 10:
        keys[: n // 10] = keys[0]            # many equal keys: stability matters
    vals = np.arange(n, dtype=np.uint32)
    kd = torch.from_numpy(keys.view(np.int32)).cuda()
    vd = torch.from_numpy(vals.view(np.int32)).cuda()
    R.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, digit)
    R.sort_pairs(kd, vd, bits)
    R.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, 8)
    torch.cuda.synchronize()
    masked = keys & np.uint32((1 << bits) - 1) if bits < 32 else keys
    order = np.argsort(masked, kind="stable")
    np.testing.assert_array_equal(vd.cpu().numpy().view(np.uint32), vals[order])
    np.testing.assert_array_equal(kd.cpu().numpy().view(np.uint32), keys[order])


# ------------------------------------------------------------------ flat scene

@pytest.fixture(scope="module")
def box():
    return W.box20k()


def test_box20k_full_frame_parity(R, box):
    scene, cams = box
    img = _render(R, scene, cams, count_nalg=1)[0]
    res = _check_full(img, scene, cams[0])
    st = R.stats()
    assert st["cut_size"] == scene.n
    # the GPU evaluates the same pixel/Gaussian pairs up to forks
    assert abs(st["n_alg"] - res.nalg.sum()) <= 0.001 * res.nalg.sum()


def test_box20k_centre_camera_parity(R, box):
    scene, _ = box
    cam = W.box_camera(center_view=True)
    img = _render(R, scene, [cam])[0]
    _check_full(img, scene, cam)


def test_projection_stage_parity(R, box):
    scene, cams = box
    _render(R, scene, cams)
    g = R.get_projected(0)
    ids = np.arange(scene.n)
    pr = O.project(scene, ids, cams[0])
    valid = g[:, 11] > 0
    assert np.array_equal(valid, pr[:, 0] > 0)
    pv = pr[valid]
    gv = g[valid]
    # the 2D mean is read back rounded to single precision
    for k, f in ((0, "u"), (1, "v")):
        assert np.all(np.abs(gv[:, k] - pv[:, O.PF[f]]) <= 1e-4 + 1.2e-7 * np.abs(pv[:, O.PF[f]])), f
    # conic from single-precision factors: relative to its scale sqrt(A C)
    scale = np.sqrt(pv[:, O.PF["A"]] * pv[:, O.PF["C"]])
    for k, f in ((2, "A"), (3, "B"), (4, "C")):
        err = np.abs(gv[:, k] - pv[:, O.PF[f]]) / scale
        assert err.max() <= 1e-5, (f, err.max())
    np.testing.assert_array_equal(gv[:, 8], pv[:, O.PF["zkey"]].astype(np.float32))
    vis = gv[:, 10] > 0
    for k, f in ((5, "r"), (6, "g"), (7, "b")):
        np.testing.assert_allclose(gv[vis, k], pv[vis, O.PF[f]], atol=2e-6)


def test_invariance_across_launch_choices(R, box):
    """Bitwise identical output for every batch depth, with and without exact
    tile binning, persistent compositing, and across repeated renders."""
    scene, cams = box
    ref = _render(R, scene, cams, batch_depth=256, exact_tiles=1, persistent=0)[0]
    again = _render(R, scene, cams)[0]
    for a, b in zip(ref, again):
        assert np.array_equal(a, b)
    for opts in ({"batch_depth": 64}, {"batch_depth": 128}, {"batch_depth": 64, "persistent": 1}, {"exact_tiles": 0},
                 {"persistent": 1}, {"sort_digit_bits": 11}, {"sort_digit_bits": 6}):
        img = _render(R, scene, cams, **opts)[0]
        for a, b in zip(ref, img):
            assert np.array_equal(a, b), opts
    _render(R, scene, cams, batch_depth=256, exact_tiles=1, persistent=0, sort_digit_bits=8)


def test_background_when_nothing_visible(R, box):
    scene, _ = box
    cam = yaw_camera(100, 37, 90.0, (2.0, -1.0, 1.5), -math.pi / 2, bg=(0.25, 0.5, 0.75))
    rgb, dep, alp = _render(R, scene, [cam])[0]
    np.testing.assert_array_equal(rgb[0], np.float32(0.25))
    np.testing.assert_array_equal(rgb[2], np.float32(0.75))
    assert not alp.any() and not dep.any()


def test_capacity_regrow_gives_identical_image(R, box):
    scene, cams = box
    hgs = _hgs()
    ref = _render(R, scene, cams)[0]
    R.set_option(hgs.HGS_OPT_INITIAL_CAPACITY, 1024)
    img = _render(R, scene, cams)[0]
    assert R.stats()["regrows"] >= 1
    R.set_option(hgs.HGS_OPT_INITIAL_CAPACITY, 0)
    for a, b in zip(ref, img):
        assert np.array_equal(a, b)


def test_depths_outside_the_key_range_fall_back_to_full_keys(R, box):
    """The depth sort's key width comes from each batch's depth range (the
    views' znear to the far corner of the means' bounding box), which holds
    for rotation matrices.  A camera matrix scaled by 3 (accepted: only its
    finiteness is checked) triples every depth and leaves that range: the
    render reports it, is redone with full 32-bit depth keys, and matches
    the oracle on the full frame."""
    import dataclasses
    scene, cams = box
    cam = dataclasses.replace(cams[0], R=(np.asarray(cams[0].R, np.float32) * 3).astype(np.float32))
    img = _render(R, scene, [cam])[0]
    assert R.stats()["regrows"] >= 1
    _check_full(img, scene, cam)


def test_capacity_error_without_regrow(R, box):
    scene, cams = box
    hgs = _hgs()
    R.load_scene(scene)
    R.set_cameras(cams)
    R.set_option(hgs.HGS_OPT_INITIAL_CAPACITY, 1024)
    R.set_option(hgs.HGS_OPT_AUTO_REGROW, 0)
    with pytest.raises(hgs.HgsError) as ei:
        R.render()
    assert ei.value.status == hgs.HGS_E_CAPACITY
    R.set_option(hgs.HGS_OPT_AUTO_REGROW, 1)
    R.set_option(hgs.HGS_OPT_INITIAL_CAPACITY, 0)
    R.render()


# ------------------------------------------------------------------ hierarchy

@pytest.fixture(scope="module")
def plan_small():
    return W.plan2m(scale=0.02, n_poses=12)


def _small_cam(c, W_=200, H_=117):
    """A smaller camera with the pose of c (ragged tiles: 200 = 12.5 x 16)."""
    return yaw_camera(W_, H_, 900.0 * W_ / 1280.0, c.position, math.atan2(c.R[2][1], c.R[2][0]))


@pytest.mark.parametrize("tau", [0.5, 1.0, 2.0, 4.0, 16.0])
def test_cut_bit_exact_small_plan(R, plan_small, tau):
    scene, cams = plan_small
    R.load_scene(scene)
    R.set_cameras(cams[:4])
    R.set_lod(1, tau)
    R.render()
    for v in range(4):
        got = R.get_cut(v)
        want = O.cut(scene, cams[v], O.MODE_THRESHOLD, tau)
        assert np.array_equal(got, want), (v, tau, got.size, want.size)


@pytest.mark.parametrize("tau", [1.0, 8.0])
def test_plan_full_frame_parity(R, plan_small, tau):
    scene, cams = plan_small
    cam = _small_cam(cams[3])
    img = _render(R, scene, [cam], tau=tau)[0]
    _check_full(img, scene, cam, tau=tau)


def test_all_leaves_mode_parity(R, plan_small):
    scene, cams = plan_small
    cam = _small_cam(cams[5], 96, 80)
    img = _render(R, scene, [cam], mode=0)[0]
    assert np.array_equal(R.get_cut(0), scene.leaf_ids())
    _check_full(img, scene, cam, mode=O.MODE_ALL_LEAVES)


def test_batched_views_equal_single_views(R, plan_small):
    scene, cams = plan_small
    views = [_small_cam(cams[1], 320, 240), _small_cam(cams[4], 128, 72), cams[7], _small_cam(cams[9], 33, 17)]
    batch = _render(R, scene, views)
    for v, cam in enumerate(views):
        single = _render(R, scene, [cam])[0]
        for a, b in zip(batch[v], single):
            assert np.array_equal(a, b), v


def test_very_large_batch_equals_single_views(R, plan_small):
    """Far more views than fit above the depth bits of the sort keys (a
    stable view pass then follows the depth sort, reading each entry's view
    from the cut) and than the cut's count pass stages in LDS (64), in many
    groups of 32 views.  Tiny views; sampled views equal their single-view
    renders bitwise and the last view's cut equals the oracle's."""
    scene, cams = plan_small
    n_levels = len(scene.level_offset) - 1
    n_views = 8192 // n_levels + 64
    assert n_views > 64
    views = [_small_cam(cams[v % len(cams)], 24 + (v % 3) * 8, 16 + (v % 5) * 4) for v in range(n_views)]
    batch = _render(R, scene, views)
    assert np.array_equal(R.get_cut(n_views - 1), O.cut(scene, views[-1], O.MODE_THRESHOLD, 1.0))
    for v in list(range(0, n_views, 97)) + [n_views - 1]:
        single = _render(R, scene, [views[v]])[0]
        for a, b in zip(batch[v], single):
            assert np.array_equal(a, b), v


def test_view_groups_keep_each_views_cut(R, plan_small):
    """A batch of 40 views: two groups of 32 and 8 views whose frontiers are
    node-major (a node's views next to each other), views staged in LDS by
    the count pass.  Every view's cut equals the oracle's, in ascending id
    order, and sampled views equal their single-view renders bitwise."""
    scene, cams = plan_small
    views = [_small_cam(cams[v % len(cams)], 120 + (v % 4) * 20, 68 + (v % 3) * 12) for v in range(40)]
    batch = _render(R, scene, views)
    for v, cam in enumerate(views):
        assert np.array_equal(R.get_cut(v), O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)), v
    for v in (0, 31, 32, 39):
        single = _render(R, scene, [views[v]])[0]
        for a, b in zip(batch[v], single):
            assert np.array_equal(a, b), v


def test_multi_pass_batches_equal_one_pass(R, plan_small):
    """A batch split into passes (at most 2 views, then 1 view per pass)
    gives the one-pass images bitwise, also replayed from a captured graph;
    the last pass keeps its cut, earlier passes' intermediates are gone."""
    scene, cams = plan_small
    hgs = _hgs()
    views = [_small_cam(cams[1], 320, 240), _small_cam(cams[4], 128, 72), cams[7], _small_cam(cams[9], 33, 17),
             _small_cam(cams[2], 200, 117)]
    one = _render(R, scene, views, pass_views=0)
    assert R.stats()["passes"] == 1
    try:
        for pv, n_pass in ((2, 3), (1, 5)):
            got = _render(R, scene, views, pass_views=pv)
            assert R.stats()["passes"] == n_pass
            for v in range(len(views)):
                for a, b in zip(one[v], got[v]):
                    assert np.array_equal(a, b), (pv, v)
        last = len(views) - 1
        assert np.array_equal(R.get_cut(last), O.cut(scene, views[last], O.MODE_THRESHOLD, 1.0))
        with pytest.raises(hgs.HgsError):
            R.get_cut(0)
        outs = R.alloc_outputs()
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 1)
        for rep in range(3):
            R.render(outs)
            torch.cuda.synchronize()
            for v in range(len(views)):
                for a, b in zip(one[v], outs[v]):
                    assert np.array_equal(a, b.cpu().numpy()), (rep, v)
        assert R.stats()["graph_launches"] >= 3
    finally:
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        R.set_option(hgs.HGS_OPT_PASS_VIEWS, 0)


def test_two_lanes_give_identical_images(R, plan_small):
    """Passes alternating between two work sets and two streams give the
    one-lane images bitwise, eagerly and replayed from a captured graph; the
    last pass's intermediates stay readable."""
    scene, cams = plan_small
    hgs = _hgs()
    views = [_small_cam(cams[1], 320, 240), _small_cam(cams[4], 128, 72), cams[7], _small_cam(cams[9], 33, 17),
             _small_cam(cams[2], 200, 117)]
    one = _render(R, scene, views)
    try:
        R.set_option(hgs.HGS_OPT_LANES, 2)
        for pv in (0, 1):
            got = _render(R, scene, views, pass_views=pv)
            assert R.stats()["passes"] >= 2
            for v in range(len(views)):
                for a, b in zip(one[v], got[v]):
                    assert np.array_equal(a, b), (pv, v)
        last = len(views) - 1
        assert np.array_equal(R.get_cut(last), O.cut(scene, views[last], O.MODE_THRESHOLD, 1.0))
        outs = R.alloc_outputs()
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 1)
        for rep in range(3):
            R.render(outs)
            torch.cuda.synchronize()
            for v in range(len(views)):
                for a, b in zip(one[v], outs[v]):
                    assert np.array_equal(a, b.cpu().numpy()), (rep, v)
    finally:
        R.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        R.set_option(hgs.HGS_OPT_PASS_VIEWS, 0)
        R.set_option(hgs.HGS_OPT_LANES, 1)


LAUNCH_SHAPES = [(8, 8, 1), (16, 8, 1), (16, 8, 2), (16, 16, 1), (16, 16, 2), (16, 16, 4), (32, 8, 1), (32, 8, 2),
                 (32, 16, 1), (32, 16, 2), (32, 16, 4)]


def test_tile_shapes_and_pixels_per_thread_give_identical_images(R, plan_small, box):
    """Every tile shape (8x8 .. 32x16), pixels per compositing thread (1, 2,
    4) and batch depth renders the default launch's images bit for bit: a
    floor-plan batch of views whose sizes are not multiples of the tiles,
    and the 20k box.  One 32-wide shape is also checked against the oracle
    on a full frame; unsupported shapes and kept pixel states with a
    non-default shape are refused."""
    hgs = _hgs()
    scene, cams = plan_small
    views = [_small_cam(cams[1], 200, 117), cams[7], _small_cam(cams[9], 33, 17), _small_cam(cams[4], 97, 211)]
    bs, bc = box
    try:
        ref = _render(R, scene, views, batch_depth=256, persistent=0)
        ref_box = _render(R, bs, bc)[0]
        for tw, th, px in LAUNCH_SHAPES:
            R.set_tile_shape(tw, th, px)
            for b in (64, 128, 256):
                img = _render(R, scene, views, batch_depth=b)
                for v in range(len(views)):
                    for a, c in zip(ref[v], img[v]):
                        assert np.array_equal(a, c), (tw, th, px, b, v)
            img = _render(R, bs, bc, batch_depth=256)[0]
            for a, c in zip(ref_box, img):
                assert np.array_equal(a, c), (tw, th, px, "box")
        R.set_tile_shape(32, 16, 4)
        _check_full(_render(R, bs, bc)[0], bs, bc[0])
        with pytest.raises(hgs.HgsError) as ei:
            R.set_option(hgs.HGS_OPT_KEEP_STATE, 1)
        assert ei.value.status == hgs.HGS_E_UNSUPPORTED
        for bad in ((24 << 16) | 8, (16 << 16) | 32, (4 << 16) | 4):
            with pytest.raises(hgs.HgsError) as ei:
                R.set_option(hgs.HGS_OPT_TILE_SHAPE, bad)
            assert ei.value.status == hgs.HGS_E_INVALID
        R.set_tile_shape(32, 8, 2)
        with pytest.raises(hgs.HgsError) as ei:
            R.set_option(hgs.HGS_OPT_PIXELS_PER_THREAD, 4)
        assert ei.value.status == hgs.HGS_E_INVALID
    finally:
        R.set_tile_shape(16, 16, 1)
        R.set_option(hgs.HGS_OPT_BATCH_DEPTH, 256)


def test_autotune_keeps_images_and_caches_the_plan(R, plan_small, tmp_path):
    """The autotuner's plan renders the same images bitwise; a second call
    with the same cache file applies the stored plan without timing."""
    scene, cams = plan_small
    hgs = _hgs()
    views = [_small_cam(cams[1], 320, 240), cams[7], _small_cam(cams[9], 33, 17)]
    ref = _render(R, scene, views, batch_depth=256, persistent=0, sort_digit_bits=8)
    cache = tmp_path / "plans.txt"
    try:
        plan = R.autotune(cache, reps=2)
        print("plan:", plan, flush=True)
        assert plan["batch_depth"] in (64, 128, 256) and plan["persistent"] in (0, 1)
        assert 6 <= plan["sort_digit_bits"] <= 11 and plan["from_cache"] == 0
        assert 0 < plan["ms"] <= plan["ms_default"]
        outs = R.render()
        torch.cuda.synchronize()
        for v in range(len(views)):
            for a, b in zip(ref[v], outs[v]):
                assert np.array_equal(a, b.cpu().numpy()), v
        again = R.autotune(cache, reps=2)
        assert again["from_cache"] == 1
        fields = ("batch_depth", "persistent", "sort_digit_bits", "lanes", "tile_w", "tile_h", "pixels_per_thread")
        assert [again[k] for k in fields] == [plan[k] for k in fields]
        outs = R.render()
        torch.cuda.synchronize()
        for v in range(len(views)):
            for a, b in zip(ref[v], outs[v]):
                assert np.array_equal(a, b.cpu().numpy()), v
        assert plan["lanes"] in (1, 2)
        assert len(cache.read_text().splitlines()) == 1
    finally:
        R.set_tile_shape(16, 16, 1)
        R.set_option(hgs.HGS_OPT_BATCH_DEPTH, 256)
        R.set_option(hgs.HGS_OPT_PERSISTENT, 0)
        R.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, 8)
        R.set_option(hgs.HGS_OPT_LANES, 1)


# ---------------------------------------------------------- full-size scene

@pytest.fixture(scope="module")
def plan_full():
    return W.plan2m(n_poses=200)


def test_plan2m_cut_bit_exact(R, plan_full):
    scene, cams = plan_full
    R.load_scene(scene)
    sel = [0, 57, 123, 199]
    R.set_cameras([cams[i] for i in sel])
    for tau in (1.0, 2.0, 4.0):
        R.set_lod(1, tau)
        R.render()
        for v, i in enumerate(sel):
            got = R.get_cut(v)
            want = O.cut(scene, cams[i], O.MODE_THRESHOLD, tau)
            assert np.array_equal(got, want), (i, tau, got.size, want.size)


def test_plan2m_sampled_pixel_parity(R, plan_full):
    """1280x720 frames of the 2M-leaf scene at tau = 1 in the bench's launch
    configuration; 3,000 sampled pixels per frame plus two full rows."""
    scene, cams = plan_full
    rng = np.random.default_rng(7)
    for i in (10, 150):
        cam = cams[i]
        img = _render(R, scene, [cam])[0]
        ids = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
        assert np.array_equal(R.get_cut(0), ids)
        px = np.concatenate([rng.integers(0, 1280, 3000), np.arange(1280), np.arange(1280)])
        py = np.concatenate([rng.integers(0, 720, 3000), np.full(1280, 360), np.full(1280, 719)])
        proj = O.project(scene, ids, cam)
        res = O.render_pixels(proj, cam, px, py)
        g = parity.gpu_pixels(*img, px, py)
        ok, best, skipped = parity.branch_errors(g, res)
        msg = parity.summary(ok, best, skipped)
        print(i, msg, flush=True)
        assert ok.all(), msg
        assert not skipped.any(), msg


def test_graph_replays_match_eager_render(R, plan_small):
    """The render captured in a hipGraph and replayed several times, with
    eager work and synchronisations between replays, gives the eager
    result every time; changing the LOD threshold re-captures."""
    scene, cams = plan_small
    hgs = _hgs()
    views = [_small_cam(cams[1], 320, 240), _small_cam(cams[6], 200, 117), cams[8]]
    ref = _render(R, scene, views, tau=1.0, use_graph=0)
    outs = R.alloc_outputs()
    R.set_option(hgs.HGS_OPT_USE_GRAPH, 1)
    side = torch.arange(100000, dtype=torch.int32, device="cuda")
    for rep in range(5):
        R.render(outs)
        torch.cuda.synchronize()
        for v in range(len(views)):
            for a, b in zip(ref[v], outs[v]):
                assert np.array_equal(a, b.cpu().numpy()), (rep, v)
        # eager work between replays: a sort and a torch op
        k = (side * 7919 % 1000).contiguous()
        R.sort_pairs(k, side.clone(), 10)
        side = side + 1
        torch.cuda.synchronize()
    assert R.stats()["graph_launches"] >= 5
    R.set_lod(hgs.HGS_LOD_THRESHOLD, 8.0)
    R.render(outs)
    torch.cuda.synchronize()
    ref8 = _render(R, scene, views, tau=8.0, use_graph=0)
    for v in range(len(views)):
        for a, b in zip(ref8[v], outs[v]):
            assert np.array_equal(a, b.cpu().numpy()), v


# ------------------------------------------- 8M-leaf plan, 256 mixed views

@pytest.fixture(scope="module")
def plan8m():
    return W.plan8m()


@pytest.mark.timeout(600)
def test_plan8m_mixed_resolution_batch(R, plan8m):
    """The 256-view batch (128 @ 320x240, 96 @ 640x480, 32 @ 1280x720) of the
    8M-leaf plan in one render call at tau = 1.  Its cut has more entries
    than the 2^28-entry index space, so the renderer splits the batch into
    passes by itself.  One view of each resolution equals its single-view
    render bitwise; that render's cut is bit-exact and its sampled pixels
    match the oracle."""
    scene, views = plan8m
    assert len(views) == 256
    R.load_scene(scene)
    R.set_cameras(views)
    R.set_lod(1, 1.0)
    outs = R.render()
    torch.cuda.synchronize()
    st = R.stats()
    print("plan8m batch:", st, flush=True)
    assert st["passes"] >= 2 and st["cut_size"] > (1 << 28)
    picks = [5, 128 + 17, 224 + 9]
    imgs = {v: tuple(t.cpu().numpy() for t in outs[v]) for v in picks}
    del outs
    rng = np.random.default_rng(3)
    for v in picks:
        cam = views[v]
        R.set_cameras([cam])
        single = R.render()[0]
        torch.cuda.synchronize()
        for a, b in zip(imgs[v], single):
            assert np.array_equal(a, b.cpu().numpy()), v
        want = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
        assert np.array_equal(R.get_cut(0), want), v
        px = rng.integers(0, cam.width, 800)
        py = rng.integers(0, cam.height, 800)
        res = O.render_pixels(O.project(scene, want, cam), cam, px, py)
        g = parity.gpu_pixels(*imgs[v], px, py)
        ok, best, skipped = parity.branch_errors(g, res)
        msg = parity.summary(ok, best, skipped)
        print(v, cam.width, cam.height, msg, flush=True)
        assert ok.all(), msg
