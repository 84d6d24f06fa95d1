"""GPU GS-slice occupancy through the C ABI against the FP64 oracle: every
cell the oracle decides (free or occupied) must agree; cells it reports as
undecided (a test within 1e-9 relative of its threshold) may go either way."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15186_amd.synth import make_random_box, workloads as W

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


def _compare(gpu, want):
    decided = want != 2
    bad = decided & (gpu.astype(np.int8) != want)
    assert not bad.any(), f"{int(bad.sum())} of {int(decided.sum())} decided cells differ"


def _leaves(scene):
    ids = scene.leaf_ids()
    return scene.means[ids], scene.scales[ids], scene.quats[ids], scene.opacity[ids]


def test_random_gaussians_match_oracle(R):
    """3,000 Gaussians of a random box (scales 4 mm - 0.3 m, random
    rotations), a ragged 45 x 37 grid of 5 cm cells, seven planes."""
    rng = np.random.default_rng(0)
    scene = make_random_box(3000, seed=4, box=(2.0, 2.0, 2.0))
    scene.scales[:] = np.exp(rng.uniform(np.log(0.004), np.log(0.3), size=scene.scales.shape)).astype(np.float32)
    R.load_scene(scene)
    heights = np.array([0.1, 0.4, 0.7, 1.0, 1.3, 1.6, 1.9], np.float32)
    occ, m = R.slice_occupancy(-0.1, 0.05, 0.05, 45, 37, heights, rho_min=0.5)
    torch.cuda.synchronize()
    g = occ.cpu().numpy()
    want = O.slice_occupancy(*_leaves(scene), -0.1, 0.05, 0.05, 45, 37, heights, rho_min=0.5)
    _compare(g, want)
    assert (want == 1).sum() > 100
    np.testing.assert_array_equal(m.cpu().numpy(), g.max(axis=0))
    _, m2 = R.slice_occupancy(-0.1, 0.05, 0.05, 45, 37, heights, rho_min=0.5, occ=False)
    np.testing.assert_array_equal(m2.cpu().numpy(), m.cpu().numpy())
    # a higher threshold marks a subset
    occ9, _ = R.slice_occupancy(-0.1, 0.05, 0.05, 45, 37, heights, rho_min=0.9)
    assert np.all(occ9.cpu().numpy() <= g)


@pytest.fixture(scope="module")
def plan_oracle():
    """The 2M-leaf plan and the oracle's planes for it: 15 planes from 0.1
    to 1.5 m over its 20 x 15 m extent at 5 cm (404 x 304 cells)."""
    scene, cams, fp = W.plan2m(n_poses=200, with_plan=True)
    heights = np.arange(0.1, 1.55, 0.1).astype(np.float32)
    want = O.slice_occupancy(*_leaves(scene), -0.1, -0.1, 0.05, 404, 304, heights, rho_min=0.5)
    return scene, cams, heights, want


def test_floor_plan_collision_map_matches_oracle(R, plan_oracle):
    """Walls and clutter occupy, the floor and ceiling sheets (far from
    every plane) do not."""
    scene, _, heights, want = plan_oracle
    R.load_scene(scene)
    occ, m = R.slice_occupancy(-0.1, -0.1, 0.05, 404, 304, heights, rho_min=0.5)
    torch.cuda.synchronize()
    g = occ.cpu().numpy()
    _compare(g, want)
    frac = g.max(axis=0).mean()
    print("occupied fraction", frac, "undecided", int((want == 2).sum()), flush=True)
    assert 0.02 < frac < 0.6
    np.testing.assert_array_equal(m.cpu().numpy(), g.max(axis=0))


def test_slice_arguments_are_checked(R):
    from paper_2603_15186_amd import hgs
    scene = make_random_box(100, seed=1)
    R.load_scene(scene)
    for kw in ({"rho_min": 0.0}, {"rho_min": 1.0}):
        with pytest.raises(hgs.HgsError) as ei:
            R.slice_occupancy(0, 0, 0.05, 10, 10, [0.5], **kw)
        assert ei.value.status == hgs.HGS_E_INVALID
    with pytest.raises(hgs.HgsError):
        R.slice_occupancy(0, 0, 0.0, 10, 10, [0.5])
    with pytest.raises(hgs.HgsError):
        R.slice_occupancy(0, 0, 0.05, 0, 10, [0.5])


def test_disc_collision_matches_oracle(R):
    """Disc robots against random maps and against the plan's collision map:
    every decided query agrees with the oracle's brute force over all cells;
    queries off the grid see free space."""
    scene = make_random_box(10, seed=2)
    R.load_scene(scene)
    rng = np.random.default_rng(9)
    for ny, nx, p in ((37, 53, 0.03), (128, 96, 0.002)):
        m = (rng.uniform(size=(ny, nx)) < p).astype(np.uint8)
        xy = np.stack([rng.uniform(-0.3, nx * 0.05 + 0.3, 4000), rng.uniform(-0.3, ny * 0.05 + 0.3, 4000)], 1)
        for radius in (0.0, 0.07, 0.3):
            got = R.disc_collision(torch.from_numpy(m).cuda(), 0.0, 0.0, 0.05, torch.from_numpy(xy).cuda(),
                                   radius).cpu().numpy()
            want = O.disc_collision(m, 0.0, 0.0, 0.05, xy, radius)
            _compare(got, want)
    far = R.disc_collision(torch.from_numpy(m).cuda(), 0.0, 0.0, 0.05,
                           torch.tensor([[-5.0, -5.0], [100.0, 2.0]], dtype=torch.float64).cuda(), 0.5)
    assert far.cpu().numpy().tolist() == [0, 0]


def test_robot_poses_against_the_plan_collision_map(R, plan_oracle):
    """The 2M-leaf plan's union map (15 planes, 5 cm) and 20,000 random
    positions for a 0.25 m robot: GPU (on its own map) = oracle (on the
    oracle's map, which has no undecided cell) on every decided query; the
    trajectory poses of the generator (0.3 m clearance) are free."""
    scene, cams, heights, planes = plan_oracle
    mo = planes.max(axis=0)
    assert not (mo == 2).any()
    R.load_scene(scene)
    _, m = R.slice_occupancy(-0.1, -0.1, 0.05, 404, 304, heights)
    assert np.array_equal(m.cpu().numpy(), mo)
    rng = np.random.default_rng(10)
    xy = rng.uniform([-0.1, -0.1], [20.1, 15.1], size=(20000, 2))
    got = R.disc_collision(m, -0.1, -0.1, 0.05, torch.from_numpy(xy).cuda(), 0.25).cpu().numpy()
    want = O.disc_collision(mo.astype(np.uint8), -0.1, -0.1, 0.05, xy, 0.25)
    _compare(got, want)
    print("colliding fraction", got.mean(), flush=True)
    assert 0.05 < got.mean() < 0.95
    path = np.array([[c.position[0], c.position[1]] for c in cams], np.float64)
    free = R.disc_collision(m, -0.1, -0.1, 0.05, torch.from_numpy(path).cuda(), 0.2).cpu().numpy()
    print("trajectory poses colliding at 0.2 m:", int(free.sum()), "of", free.size, flush=True)
    assert free.mean() < 0.05
