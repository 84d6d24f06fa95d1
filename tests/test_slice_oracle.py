"""Pins of the GS-slice occupancy oracle (CPU): the slice of a 3D Gaussian by a
horizontal plane against the conditional-Gaussian identities, the density
identity at random points, exact occupancy of axis-aligned ellipses, and
brute-force occupancy of rotated ones."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as O


def _random(n, seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    s = np.exp(rng.uniform(np.log(0.004), np.log(0.3), size=(n, 3))).astype(np.float32)
    mu = rng.uniform(0, 2, size=(n, 3)).astype(np.float32)
    o = rng.uniform(0.3, 1.0, size=n).astype(np.float32)
    return mu, s, q, o


def _sigma(s, q):
    """Covariance R diag(s^2) R^T with R from scipy (quaternion (w, x, y, z))."""
    qd = q.astype(np.float64)
    R = Rotation.from_quat(np.concatenate([qd[:, 1:], qd[:, :1]], axis=1)).as_matrix()
    return np.einsum("nij,nj,nkj->nik", R, s.astype(np.float64) ** 2, R)


def test_slice_parameters_are_the_conditional_gaussian():
    """lambda = 1 / Sigma_zz, C_xy^-1 = Sigma_xy - Sigma_xy,z Sigma_z,xy /
    Sigma_zz (Schur complement) and mu(z) = mu_xy + Sigma_xy,z / Sigma_zz (z -
    mu_z), i.e. (alpha, beta) = -Sigma_xy,z / Sigma_zz."""
    _, s, q, _ = _random(200, 0)
    P = O.slice_params(s, q)
    S = _sigma(s, q)
    szz = S[:, 2, 2]
    np.testing.assert_allclose(P[:, 2], 1.0 / szz, rtol=1e-9)
    np.testing.assert_allclose(P[:, 0], -S[:, 0, 2] / szz, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(P[:, 1], -S[:, 1, 2] / szz, rtol=1e-7, atol=1e-9)
    schur = S[:, :2, :2] - np.einsum("ni,nj->nij", S[:, :2, 2], S[:, :2, 2]) / szz[:, None, None]
    Cxy = np.stack([np.stack([P[:, 3], P[:, 4]], 1), np.stack([P[:, 4], P[:, 5]], 1)], 1)
    np.testing.assert_allclose(np.linalg.inv(Cxy), schur, rtol=1e-7, atol=1e-12)


def test_slice_reproduces_the_3d_density_on_the_plane():
    """exp(-1/2 d^T Sigma^-1 d) at (x, y, z) equals exp(-1/2 lambda dz^2)
    exp(-1/2 (xy - mu(z))^T C_xy (xy - mu(z))) -- with the -1/2 in the
    second factor that the printed formula drops."""
    mu, s, q, _ = _random(100, 1)
    P = O.slice_params(s, q)
    S = _sigma(s, q)
    rng = np.random.default_rng(2)
    for g in range(100):
        p = mu[g].astype(np.float64) + rng.normal(scale=s[g].max(), size=(20, 3))
        d = p - mu[g]
        full = np.exp(-0.5 * np.einsum("ni,ij,nj->n", d, np.linalg.inv(S[g]), d))
        dz = d[:, 2]
        m = mu[g, :2].astype(np.float64)[None, :] - dz[:, None] * P[g, :2][None, :]
        e = p[:, :2] - m
        C = np.array([[P[g, 3], P[g, 4]], [P[g, 4], P[g, 5]]])
        sl = np.exp(-0.5 * P[g, 2] * dz * dz) * np.exp(-0.5 * np.einsum("ni,ij,nj->n", e, C, e))
        np.testing.assert_allclose(sl, full, rtol=1e-7, atol=1e-300)


def _cells(x0, y0, cell, nx, ny):
    i = np.arange(nx)
    j = np.arange(ny)
    return x0 + i * cell, y0 + j * cell


def test_axis_aligned_ellipse_occupancy_is_exact():
    """For an axis-aligned Gaussian the least q over a cell sits at the mean
    clamped into the cell, so the occupied set has a closed form; the solid
    radius is r^2 = 2 ln(o a(z) / rho_min) with a(z) = exp(-(z-mu_z)^2 /
    (2 s_z^2))."""
    mu = np.array([[1.013, 0.977, 0.8]], np.float32)
    s = np.array([[0.11, 0.23, 0.07]], np.float32)
    q = np.array([[1.0, 0.0, 0.0, 0.0]], np.float32)
    o = np.array([0.93], np.float32)
    heights = np.array([0.8, 0.83, 0.87, 0.95, 1.1], np.float32)
    x0, y0, cell, nx, ny = 0.0, 0.0, 0.05, 41, 41
    occ = O.slice_occupancy(mu, s, q, o, x0, y0, cell, nx, ny, heights, rho_min=0.5)
    xs, ys = _cells(x0, y0, cell, nx, ny)
    m = mu[0].astype(np.float64)
    sd = s[0].astype(np.float64)
    for k, z in enumerate(heights.astype(np.float64)):
        A = float(o[0]) * np.exp(-0.5 * (z - m[2]) ** 2 / sd[2] ** 2)
        want = np.zeros((ny, nx), np.int8)
        if A > 0.5:
            r2 = 2 * np.log(A / 0.5)
            cx = np.clip(m[0], xs, xs + cell)
            cy = np.clip(m[1], ys, ys + cell)
            qq = ((cx[None, :] - m[0]) / sd[0]) ** 2 + ((cy[:, None] - m[1]) / sd[1]) ** 2
            want = (qq <= r2).astype(np.int8)
        assert (occ[k] == 2).sum() == 0
        np.testing.assert_array_equal(occ[k], want, err_msg=f"plane {k}")
    assert occ[0].sum() > 20 and occ[-1].sum() == 0


@pytest.mark.parametrize("seed", [3, 4])
def test_rotated_ellipse_occupancy_against_brute_force(seed):
    """A rotated Gaussian: a cell is occupied iff some point of the closed
    square lies in the solid ellipse; brute force samples each square's
    interior and edges densely, so it may only miss cells the ellipse just
    grazes."""
    rng = np.random.default_rng(seed)
    mu = np.array([[1.0 + rng.uniform(-0.03, 0.03), 1.0 + rng.uniform(-0.03, 0.03), 0.5]], np.float32)
    s = np.array([[0.25, 0.06, 0.12]], np.float32)
    q = rng.normal(size=(1, 4)).astype(np.float32)
    o = np.array([0.95], np.float32)
    heights = np.array([0.45, 0.5, 0.56], np.float32)
    x0, y0, cell, nx, ny = 0.0, 0.0, 0.05, 40, 40
    occ = O.slice_occupancy(mu, s, q, o, x0, y0, cell, nx, ny, heights)
    P = O.slice_params(s, q)[0]
    C = np.array([[P[3], P[4]], [P[4], P[5]]])
    t = np.linspace(0.0, 1.0, 41)
    for k, z in enumerate(heights.astype(np.float64)):
        dz = z - float(mu[0, 2])
        A = float(o[0]) * np.exp(-0.5 * P[2] * dz * dz)
        if A <= 0.5:
            assert occ[k].sum() == 0
            continue
        r2 = 2 * np.log(A / 0.5)
        m = mu[0, :2].astype(np.float64) - dz * P[:2]
        for j in range(ny):
            for i in range(nx):
                px = x0 + (i + t) * cell
                py = y0 + (j + t) * cell
                X, Y = np.meshgrid(px, py)
                dx, dy = X - m[0], Y - m[1]
                qq = C[0, 0] * dx * dx + 2 * C[0, 1] * dx * dy + C[1, 1] * dy * dy
                qmin = qq.min()
                if qmin <= r2:
                    assert occ[k, j, i] == 1, (k, j, i)
                elif qmin > r2 * 1.02 + 1e-3:
                    assert occ[k, j, i] == 0, (k, j, i, qmin, r2)


def test_opacity_below_threshold_and_far_planes_leave_the_map_empty():
    mu, s, q, o = _random(50, 5)
    heights = np.array([0.9, 1.0, 1.1], np.float32)
    thin = O.slice_occupancy(mu, s, q, np.full_like(o, 0.49), 0, 0, 0.05, 40, 40, heights, rho_min=0.5)
    assert thin.sum() == 0
    far = O.slice_occupancy(mu, s, q, o, 0, 0, 0.05, 40, 40, np.array([10.0], np.float32))
    assert far.sum() == 0
    near = O.slice_occupancy(mu, s, q, o, 0, 0, 0.05, 40, 40, heights)
    assert (near == 1).sum() > 0


def test_vertical_sheet_occupies_a_line_of_cells():
    """A wall: Gaussians on the plane x = 1.0 (thin in x, 5 cm apart in y and
    z); every plane between its bottom and top marks the cells whose x-range
    reaches 1.0 and no cell more than one cell away."""
    ys = np.arange(0.2, 1.8, 0.05)
    zs = np.arange(0.1, 1.5, 0.05)
    Y, Z = np.meshgrid(ys, zs)
    n = Y.size
    mu = np.stack([np.full(n, 1.0), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    s = np.tile(np.array([[0.005, 0.035, 0.035]], np.float32), (n, 1))
    q = np.tile(np.array([[1.0, 0.0, 0.0, 0.0]], np.float32), (n, 1))
    o = np.full(n, 0.95, np.float32)
    occ = O.slice_occupancy(mu, s, q, o, 0.0, 0.0, 0.05, 40, 40, np.array([0.5, 1.0], np.float32))
    for k in range(2):
        cols = np.nonzero(occ[k].any(axis=0))[0]
        assert set(cols.tolist()) <= {19, 20}
        assert occ[k][6:34, 19].all() or occ[k][6:34, 20].all()


def test_disc_collision_single_cell_closed_form():
    """One occupied cell [1.0, 1.05] x [2.0, 2.05]: a disc collides iff its
    centre is within the radius of the square (distance to the clamped
    point); cells outside the grid count as free."""
    m = np.zeros((60, 40), np.uint8)
    m[40, 20] = 1                       # x0 = 0, y0 = 0, cell 0.05
    rng = np.random.default_rng(6)
    xy = rng.uniform([0.5, 1.5], [1.6, 2.6], size=(2000, 2))
    got = O.disc_collision(m, 0.0, 0.0, 0.05, xy, 0.2)
    cx = np.clip(xy[:, 0], 1.0, 1.05)
    cy = np.clip(xy[:, 1], 2.0, 2.05)
    d = np.hypot(xy[:, 0] - cx, xy[:, 1] - cy)
    np.testing.assert_array_equal(got == 1, d < 0.2 * (1 - 1e-9))
    assert set(np.unique(got[np.abs(d - 0.2) > 1e-6])) <= {0, 1}
    far = O.disc_collision(m, 0.0, 0.0, 0.05, np.array([[5.0, 5.0], [-3.0, 1.0]]), 0.5)
    assert np.all(far == 0)


def test_disc_collision_against_sampled_discs():
    """Random maps: a sample point of the disc inside an occupied cell means
    collision; a collision means some occupied square is within the radius
    (checked on its corners' and edges' nearest points)."""
    rng = np.random.default_rng(7)
    m = (rng.uniform(size=(30, 30)) < 0.04).astype(np.uint8)
    xy = rng.uniform(0, 1.5, size=(300, 2))
    got = O.disc_collision(m, 0.0, 0.0, 0.05, xy, 0.12)
    t = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    rr = np.linspace(0, 0.12 * (1 - 1e-6), 12)
    for q in range(300):
        px = (xy[q, 0] + rr[:, None] * np.cos(t)[None, :]).ravel()
        py = (xy[q, 1] + rr[:, None] * np.sin(t)[None, :]).ravel()
        i = np.floor(px / 0.05).astype(int)
        j = np.floor(py / 0.05).astype(int)
        ok = (i >= 0) & (i < 30) & (j >= 0) & (j < 30)
        hit = bool(m[j[ok], i[ok]].any())
        if hit:
            assert got[q] == 1, q
        if got[q] == 1:
            jj, ii = np.nonzero(m)
            dx = np.maximum(np.maximum(ii * 0.05 - xy[q, 0], 0), xy[q, 0] - (ii + 1) * 0.05)
            dy = np.maximum(np.maximum(jj * 0.05 - xy[q, 1], 0), xy[q, 1] - (jj + 1) * 0.05)
            assert np.hypot(dx, dy).min() <= 0.12
