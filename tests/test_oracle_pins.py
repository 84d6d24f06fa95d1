"""Pins of the FP64 oracle against closed forms, library routines, an
independently written brute force, and invariants (CPU only).

Each test names what fixes the expected value.  Passages: NavGSim
(arXiv 2603.15186) Eq. (1) (Gaussian kernel), Supplementary Material
(Sigma = R S S^T R^T), Sec. III-A (render from intrinsics and extrinsics).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy import special

from oracle import brute
from oracle import oracle as O
from paper_2603_15186_amd.synth import Scene, yaw_camera

F32 = lambda x: float(np.float32(x))  # noqa: E731
CAP, AMIN, TMIN = F32(0.99), F32(1.0 / 255.0), F32(1e-4)
Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _scene(means, scales, quats, opac, sh, deg=0):
    return Scene(np.asarray(means, np.float32), np.asarray(scales, np.float32),
                 np.asarray(quats, np.float32), np.asarray(opac, np.float32),
                 np.asarray(sh, np.float32), deg)


def _axis_cam(W=64, H=64, f=64.0, bg=(0.0, 0.0, 0.0)):
    # camera at the origin looking along +y: camera (x, y, z) = world (x, -z, y)
    return yaw_camera(W, H, f, (0.0, 0.0, 0.0), math.pi / 2, bg=bg)


def _full(scene, cam, **kw):
    res, ids, proj = O.render(scene, cam, **kw)
    return res, proj


# ---------------------------------------------------------------- closed forms

def test_single_isotropic_gaussian_closed_form():
    """A single isotropic Gaussian at camera-space (0,0,z): the projected
    covariance is ((f s / z)^2 + 0.3) I exactly and the pixel value is
    c * alpha + (1 - alpha) * bg with alpha = min(0.99f, o exp(-q/2)) inside
    q <= 9 and alpha >= 1/255f (Eq. (1) on the image plane)."""
    z, s, o, f = 2.0, 0.05, 0.8, 64.0
    rgb = np.array([0.9, 0.4, 0.1])
    bg = (0.2, 0.3, 0.1)
    cam = _axis_cam(f=f, bg=bg)
    bg = tuple(F32(b) for b in bg)           # the camera holds single precision
    sc = _scene([[0.0, z, 0.0]], [[s, s, s]], [[1, 0, 0, 0]], [o], ((rgb - 0.5) / Y00)[None, None, :])
    res, proj = _full(sc, cam)
    var = (f * F32(s) / z) ** 2 + 0.3        # inputs are single precision
    assert proj[0, O.PF["S00"]] == pytest.approx(var, rel=1e-13)
    assert proj[0, O.PF["S11"]] == pytest.approx(var, rel=1e-13)
    assert abs(proj[0, O.PF["S01"]]) < 1e-13
    col = np.clip(Y00 * sc.sh[0, 0].astype(np.float64) + 0.5, 0, 1)   # stored coefficients
    checked = 0
    for k in range(res.px.size):
        dx, dy = res.px[k] + 0.5 - 32.0, res.py[k] + 0.5 - 32.0
        q = (dx * dx + dy * dy) / var
        a = min(CAP, F32(o) * math.exp(-0.5 * q))
        if abs(q - 9) < 1e-3 or abs(a - AMIN) < 1e-6:
            continue
        if q <= 9 and a >= AMIN:
            want = np.concatenate([col * a + (1 - a) * np.array(bg), [z * a, a]])
        else:
            want = np.array(list(bg) + [0.0, 0.0])
        got = res.primary[k]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
        checked += 1
    assert checked > 4000


def test_two_gaussians_closed_form():
    """Two Gaussians on the optical axis: C = c1 a1 + c2 a2 (1 - a1), with the
    nearer one first whatever their order in the input."""
    f = 64.0
    cam = _axis_cam(f=f)
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    means = [[0.0, 3.0, 0.0], [0.0, 2.0, 0.0]]   # the second is nearer
    sh = np.stack([(c1 - 0.5) / Y00, (c2 - 0.5) / Y00])[:, None, :]
    sc = _scene(means, [[0.1] * 3, [0.05] * 3], [[1, 0, 0, 0]] * 2, [0.7, 0.6], sh)
    res, proj = _full(sc, cam)
    c1, c2 = np.clip(Y00 * sc.sh[:, 0].astype(np.float64) + 0.5, 0, 1)
    k = 32 * 64 + 33   # pixel (33, 32): centre offset (1.5, 0.5)
    d2 = 1.5 ** 2 + 0.5 ** 2
    v_near = (f * F32(0.05) / 2.0) ** 2 + 0.3
    v_far = (f * F32(0.1) / 3.0) ** 2 + 0.3
    a_near = min(CAP, F32(0.6) * math.exp(-0.5 * d2 / v_near))
    a_far = min(CAP, F32(0.7) * math.exp(-0.5 * d2 / v_far))
    want_rgb = c2 * a_near + c1 * a_far * (1 - a_near)
    np.testing.assert_allclose(res.primary[k, :3], want_rgb, atol=1e-12)
    assert res.primary[k, 3] == pytest.approx(2.0 * a_near + 3.0 * a_far * (1 - a_near), abs=1e-12)
    assert res.primary[k, 4] == pytest.approx(1 - (1 - a_near) * (1 - a_far), abs=1e-12)


def test_capped_stack_single_contribution():
    """Layers that each reach the 0.99f cap: after the first, T = 1 - 0.99f;
    a second would give T' = (1-0.99f)^2 < 1e-4f, so it is not added and the
    pixel holds exactly one contribution.  (With decimal 0.99 and 1e-4 the
    second layer would be added: T' = 1.0000000000000018e-4.)"""
    assert (1 - CAP) ** 2 < TMIN
    assert (1 - 0.99) ** 2 >= 1e-4
    cam = _axis_cam()
    cols = np.array([[0.2, 0.9, 0.5], [0.8, 0.1, 0.3], [0.4, 0.4, 0.9]])
    means = [[0.0, 2.0, 0.0], [0.0, 2.5, 0.0], [0.0, 3.0, 0.0]]
    sc = _scene(means, [[0.3] * 3] * 3, [[1, 0, 0, 0]] * 3, [1.0] * 3, ((cols - 0.5) / Y00)[:, None, :])
    res, _ = _full(sc, cam)
    k = 31 * 64 + 31   # pixel centre (31.5, 31.5): q < 0.0125, o exp(-q/2) > 0.99
    c0 = np.clip(Y00 * sc.sh[0, 0].astype(np.float64) + 0.5, 0, 1)
    np.testing.assert_allclose(res.primary[k, :3], c0 * CAP, atol=1e-12)
    assert res.primary[k, 4] == pytest.approx(CAP, abs=1e-15)
    assert res.nalg[k] == 2


def _proj_rows(rows):
    """Hand-built projected entries (isotropic, variance var) for the
    compositing stage: (u, v, var, rgb, z, opacity)."""
    out = np.zeros((len(rows), len(O.PROJ_FIELDS)))
    for i, (u, v, var, rgb, z, o) in enumerate(rows):
        r = out[i]
        r[O.PF["valid"]] = 1; r[O.PF["u"]] = u; r[O.PF["v"]] = v
        r[O.PF["A"]] = 1 / var; r[O.PF["C"]] = 1 / var
        r[O.PF["S00"]] = var; r[O.PF["S11"]] = var
        r[O.PF["r"]:O.PF["b"] + 1] = rgb
        r[O.PF["z"]] = z; r[O.PF["zkey"]] = F32(z); r[O.PF["opacity"]] = o
    return out


def test_fork_at_exact_three_sigma():
    """A pixel centre exactly on the 3-sigma ellipse (q = 9) is a
    near-threshold decision: both outcomes are reported."""
    cam = _axis_cam()
    proj = _proj_rows([(34.5, 32.5, 4.0, (0.4, 0.4, 0.4), 2.0, 1.0)])   # dx = 6, sigma = 2
    res = O.render_pixels(proj, cam, np.array([40]), np.array([32]))
    assert res.nbranch[0] == 2
    a = math.exp(-4.5)
    assert res.branches[0, 0, 4] == pytest.approx(a, rel=1e-14)    # q <= 9 holds in FP64
    assert res.branches[0, 1, 4] == 0.0
    res = O.render_pixels(proj, cam, np.array([41]), np.array([32]))  # q = 12.25: clear
    assert res.nbranch[0] == 1 and res.branches[0, 0, 4] == 0.0


def test_fork_at_alpha_minimum():
    """alpha exactly at 1/255f: used and skipped are both valid."""
    cam = _axis_cam()
    proj = _proj_rows([(32.5, 32.5, 4.0, (1.0, 0.0, 0.0), 2.0, AMIN)])
    res = O.render_pixels(proj, cam, np.array([32]), np.array([32]))
    assert res.nbranch[0] == 2
    assert sorted(res.branches[0, :2, 4]) == pytest.approx([0.0, AMIN], abs=1e-15)


def test_fork_at_transmittance_minimum():
    """A second layer that takes T to 1e-4f exactly: stopping before it and
    adding it are both valid."""
    cam = _axis_cam()
    a2 = 1 - TMIN / (1 - CAP)
    proj = _proj_rows([(32.5, 32.5, 1e4, (1.0, 0.0, 0.0), 2.0, 1.0),
                       (32.5, 32.5, 1e4, (0.0, 1.0, 0.0), 3.0, a2)])
    res = O.render_pixels(proj, cam, np.array([32]), np.array([32]))
    assert res.nbranch[0] == 2
    g = sorted(res.branches[0, :2, 1])
    assert g[0] == 0.0
    assert g[1] == pytest.approx(a2 * (1 - CAP), rel=1e-12)


# ---------------------------------------------------------- projection pins

def _rand_scene(rng, n, deg, box=((-1, 1), (1.5, 4), (-1, 1))):
    lo = np.array([b[0] for b in box]); hi = np.array([b[1] for b in box])
    means = rng.uniform(lo, hi, size=(n, 3))
    scales = np.exp(rng.normal(-2.5, 0.6, size=(n, 3)))
    q = rng.normal(size=(n, 4))
    op = rng.uniform(0.05, 1.0, size=n)
    K = (deg + 1) ** 2
    sh = rng.normal(0, 0.6, size=(n, K, 3))
    return _scene(means, scales, q, op, sh, deg)


def test_projection_matches_finite_difference_jacobian_and_scipy_rotation():
    """Sigma' - 0.3 I = (dpi/dx) Sigma (dpi/dx)^T where dpi/dx is the FP64
    central-difference Jacobian of the pinhole map and Sigma comes from
    scipy's quaternion rotation (Supplementary Material: Sigma = R S S^T R^T)."""
    rng = np.random.default_rng(5)
    sc = _rand_scene(rng, 50, 0, box=((-0.5, 0.5), (2, 4), (-0.5, 0.5)))
    cam = yaw_camera(200, 150, 180.0, (0.1, -0.2, 0.05), math.pi / 2 + 0.1)
    proj = O.project(sc, np.arange(sc.n), cam)
    R = cam.R.astype(np.float64); o = cam.position.astype(np.float64)

    def pi(x):
        t = R @ (x - o)
        return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])

    for g in range(sc.n):
        mu = sc.means[g].astype(np.float64)
        h = 1e-5
        Jn = np.stack([(pi(mu + h * e) - pi(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        w, x, y, z = sc.quats[g].astype(np.float64)
        Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
        Sig = Rq @ np.diag(sc.scales[g].astype(np.float64) ** 2) @ Rq.T
        want = Jn @ Sig @ Jn.T
        got = np.array([[proj[g, O.PF["S00"]] - 0.3, proj[g, O.PF["S01"]]],
                        [proj[g, O.PF["S01"]], proj[g, O.PF["S11"]] - 0.3]])
        np.testing.assert_allclose(got, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())
        np.testing.assert_allclose([proj[g, O.PF["u"]], proj[g, O.PF["v"]]], pi(mu), rtol=1e-13)
        # conic is the inverse of Sigma'
        S = np.array([[proj[g, O.PF["S00"]], proj[g, O.PF["S01"]]],
                      [proj[g, O.PF["S01"]], proj[g, O.PF["S11"]]]])
        Cn = np.array([[proj[g, O.PF["A"]], proj[g, O.PF["B"]]], [proj[g, O.PF["B"]], proj[g, O.PF["C"]]]])
        np.testing.assert_allclose(Cn @ S, np.eye(2), atol=1e-12)
        assert np.all(np.linalg.eigvalsh(S) >= 0.3 - 1e-12)


def test_isotropic_gaussian_is_quaternion_invariant():
    rng = np.random.default_rng(6)
    n = 20
    q = rng.normal(size=(n, 4))
    sc = _scene(np.tile([[0.3, 2.5, -0.2]], (n, 1)), np.full((n, 3), 0.07), q, np.full(n, 0.5),
                np.zeros((n, 1, 3)))
    proj = O.project(sc, np.arange(n), _axis_cam())
    for f in ("S00", "S01", "S11"):
        np.testing.assert_allclose(proj[:, O.PF[f]], proj[0, O.PF[f]], rtol=1e-12, atol=1e-14)


def test_near_plane_culls_on_the_mean():
    cam = _axis_cam()
    sc = _scene([[0, 0.1999, 0], [0, 0.2001, 0], [0, -1.0, 0]], [[0.01] * 3] * 3, [[1, 0, 0, 0]] * 3,
                [0.5] * 3, np.zeros((3, 1, 3)))
    proj = O.project(sc, np.arange(3), cam)
    assert list(proj[:, 0]) == [0.0, 1.0, 0.0]


# ------------------------------------------------------------------ SH pins

def test_sh_degree0_is_constant():
    rng = np.random.default_rng(1)
    cam = _axis_cam()
    n = 30
    sc = _rand_scene(rng, n, 0)
    proj = O.project(sc, np.arange(n), cam)
    want = np.clip(Y00 * sc.sh[:, 0, :].astype(np.float64) + 0.5, 0, 1)
    ok = proj[:, 0] > 0
    np.testing.assert_allclose(proj[ok][:, O.PF["r"]:O.PF["b"] + 1], want[ok], atol=1e-14)


def test_sh_addition_theorem():
    """sum_m Y_lm(d)^2 = (2l+1) / (4 pi) for every unit d and l = 0..3."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        Y = O.sh_basis(d)
        for l in range(4):
            assert np.sum(Y[l * l:(l + 1) * (l + 1)] ** 2) == pytest.approx((2 * l + 1) / (4 * math.pi), rel=1e-12)


def test_sh_matches_scipy_complex_harmonics():
    """Real SH from scipy's complex Y_l^m (which carries the Condon-Shortley
    phase): Y_l0 = Y_l^0, Y_lm = sqrt2 Re Y_l^m (m>0), sqrt2 Im Y_l^|m| (m<0)."""
    rng = np.random.default_rng(3)
    for _ in range(30):
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        theta = math.acos(d[2]); phi = math.atan2(d[1], d[0])
        Y = O.sh_basis(d)
        for l in range(4):
            for m in range(-l, l + 1):
                c = special.sph_harm_y(l, abs(m), theta, phi)
                want = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
                assert Y[l * l + l + m] == pytest.approx(want, abs=1e-12)


# ------------------------------------------------------ compositing vs brute

@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_oracle_matches_untiled_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    deg = seed % 4
    sc = _rand_scene(rng, 40, deg)
    # seeds 4 and 5: off-centre principal point (window cameras)
    cx, cy = (5.0, 15.0) if seed >= 4 else (None, None)
    cam = yaw_camera(24, 20, 22.0, (0.05, 0.0, 0.1), math.pi / 2 + 0.05 * seed,
                     bg=(0.1, 0.0, 0.2) if seed % 2 else (0, 0, 0), cx=cx, cy=cy)
    res, _ = _full(sc, cam)
    rgb, dep, alp = brute.render(sc, cam)
    k = 0
    for j in range(cam.height):
        for i in range(cam.width):
            want = np.array(rgb[j][i] + [dep[j][i], alp[j][i]])
            br = res.branches[k, :res.nbranch[k]]
            err = np.abs(br - want[None]).max(axis=1)
            assert err.min() < 1e-9, (seed, i, j, err)
            if res.nbranch[k] == 1:
                assert err[0] < 1e-9
            k += 1


def test_permutation_invariance():
    rng = np.random.default_rng(11)
    sc = _rand_scene(rng, 200, 1)
    cam = yaw_camera(48, 40, 40.0, (0.0, 0.0, 0.0), math.pi / 2)
    res, _ = _full(sc, cam)
    perm = rng.permutation(sc.n)
    sp = _scene(sc.means[perm], sc.scales[perm], sc.quats[perm], sc.opacity[perm], sc.sh[perm], 1)
    res2, _ = _full(sp, cam)
    np.testing.assert_allclose(res2.primary, res.primary, atol=1e-12)


def test_transmittance_bounds_on_random_scene():
    """T is a product of factors in (0,1] and the walk stops before it would
    drop below 1e-4f: 0 <= alpha <= 1 - 1e-4f, and colour <= 1 - T."""
    rng = np.random.default_rng(12)
    sc = _rand_scene(rng, 400, 0)
    cam = yaw_camera(64, 48, 50.0, (0.0, 0.0, 0.0), math.pi / 2)
    res, _ = _full(sc, cam)
    for b in range(res.branches.shape[1]):
        valid = res.nbranch > b
        a = res.branches[valid, b, 4]
        assert np.all(a >= 0) and np.all(a <= 1 - TMIN + 1e-15)
        assert np.all(res.branches[valid, b, :3] <= a[:, None] + 1e-12)
    assert (res.primary[:, 4] > 0.99).mean() > 0.1   # some pixels are opaque


# ---------------------------------------------------------------- cut pins

@pytest.fixture(scope="module")
def small_plan():
    from paper_2603_15186_amd.synth import workloads as W
    scene, cams = W.plan2m(scale=0.01, n_poses=6, use_cache=False)
    return scene, cams


def _ancestors(scene, k):
    out = [k]
    while scene.parent[out[-1]] >= 0:
        out.append(int(scene.parent[out[-1]]))
    return out


def _outside(scene, cam, k):
    """Sphere k entirely outside the frustum, by normalised plane distances
    (division and square roots, unlike the oracle's squared form)."""
    c = scene.bound[k, :3].astype(np.float64); r = float(scene.bound[k, 3])
    p = cam.R.astype(np.float64) @ (c - cam.position.astype(np.float64))
    W, H = cam.width, cam.height
    planes = [np.array([0, 0, 1.0]), np.array([cam.fx, 0, cam.cx]), np.array([-cam.fx, 0, W - cam.cx]),
              np.array([0, cam.fy, cam.cy]), np.array([0, -cam.fy, H - cam.cy])]
    dists = [p[2] - cam.znear] + [float(n @ p) / np.linalg.norm(n) for n in planes[1:]]
    return min(dists) < -r, min(dists) >= -r * (1 - 1e-9)


def test_cut_small_tau_is_all_visible_leaves_and_large_tau_is_root(small_plan):
    scene, cams = small_plan
    cam = cams[0]
    fine = O.cut(scene, cam, O.MODE_THRESHOLD, 1e-6)
    assert np.all(scene.child_count[fine] == 0)
    for k in scene.leaf_ids()[::7]:
        anc = _ancestors(scene, int(k))
        out = [_outside(scene, cam, a) for a in anc]
        culled = any(o[0] for o in out)
        clear = all(o[1] for o in out)
        if k in set(fine.tolist()):
            assert not culled
        elif clear:
            pytest.fail(f"leaf {k} visible but not in the fine cut")
    coarse = O.cut(scene, cam, O.MODE_THRESHOLD, 1e9)
    assert list(coarse) == [0]


def test_cut_is_a_valid_antichain_and_monotone_in_tau(small_plan):
    scene, cams = small_plan
    for cam in cams[:3]:
        fine = O.cut(scene, cam, O.MODE_THRESHOLD, 1e-6)
        prev = fine
        for tau in (0.5, 1.0, 2.0, 4.0, 16.0, 64.0):
            cut = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
            assert np.all(np.diff(cut) > 0)                   # ascending, unique
            s = set(cut.tolist())
            for k in fine:                                    # each visible leaf: one cut node
                assert sum(a in s for a in _ancestors(scene, int(k))) == 1
            for k in prev:                                    # coarsening of the finer cut
                assert sum(a in s for a in _ancestors(scene, int(k))) == 1
            assert len(cut) <= len(prev)
            prev = cut


def test_cut_expand_rule_matches_projected_size(small_plan):
    """An emitted internal node has projected size 2 f r / |c - o| <= tau;
    every strict ancestor of a cut node has size > tau (sqrt and division
    here, squared products in the oracle)."""
    scene, cams = small_plan
    cam = cams[1]
    f = max(cam.fx, cam.fy)
    for tau in (2.0, 8.0, 32.0):
        cut = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
        c = scene.bound[:, :3].astype(np.float64); r = scene.bound[:, 3].astype(np.float64)
        size = 2 * f * r / np.linalg.norm(c - cam.position.astype(np.float64), axis=1)
        internal = cut[scene.child_count[cut] > 0]
        assert np.all(size[internal] <= tau * (1 + 1e-12))
        for k in cut[::5]:
            for a in _ancestors(scene, int(k))[1:]:
                assert size[a] > tau * (1 - 1e-12)


def test_all_leaves_mode(small_plan):
    scene, cams = small_plan
    ids = O.cut(scene, cams[0], O.MODE_ALL_LEAVES, 1.0)
    np.testing.assert_array_equal(ids, scene.leaf_ids())
