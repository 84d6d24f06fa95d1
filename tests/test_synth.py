"""Seeded input generators: determinism, hierarchy layout, moment matching
and bounding-sphere enclosure (CPU only)."""
import hashlib

import numpy as np
import pytest

from paper_2603_15186_amd.synth import build_hierarchy, covariances, make_floorplan, make_random_box
from paper_2603_15186_amd.synth import workloads as W


def _digest(*arrays):
    h = hashlib.sha1()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_random_box_is_seeded_and_matches_its_recipe():
    a = make_random_box(20000, seed=0)
    b = make_random_box(20000, seed=0)
    assert _digest(a.means, a.scales, a.quats, a.opacity, a.sh) == _digest(b.means, b.scales, b.quats, b.opacity, b.sh)
    assert a.means.min() >= 0 and a.means[:, 0].max() <= 4 and a.means[:, 2].max() <= 3
    ls = np.log(a.scales.astype(np.float64))
    assert abs(ls.mean() + 3.5) < 0.02 and abs(ls.std() - 0.5) < 0.02
    np.testing.assert_allclose(np.linalg.norm(a.quats, axis=1), 1, atol=1e-6)
    col = a.sh[:, 0, :] / (2 * np.sqrt(np.pi)) + 0.5
    assert col.min() >= -1e-6 and col.max() <= 1 + 1e-6


@pytest.fixture(scope="module")
def small():
    leaves, plan = make_floorplan(6000, (8.0, 6.0), 1, 3.0, 20, 3, seed=9)
    return leaves, build_hierarchy(leaves)


def test_floorplan_leaf_count_and_sheets(small):
    leaves, _ = small
    assert leaves.n == 6000
    assert np.all(leaves.scales[:, 2] == np.float32(0.005))
    assert leaves.sh.shape == (6000, 16, 3)


def test_hierarchy_layout(small):
    _, h = small
    n = h.n
    lo = h.level_offset
    assert lo[0] == 0 and lo[-1] == n
    assert np.all(h.parent[lo[0]:lo[1]] == -1)
    # children contiguous, in parent order, all one level down
    for L in range(h.n_levels - 1):
        ids = np.arange(lo[L], lo[L + 1])
        fc, cc = h.first_child[ids], h.child_count[ids]
        assert fc[0] == lo[L + 1]
        np.testing.assert_array_equal(fc[1:], fc[:-1] + cc[:-1])
        assert fc[-1] + cc[-1] == lo[L + 2]
        for k in ids[:50]:
            assert np.all(h.parent[h.first_child[k]:h.first_child[k] + h.child_count[k]] == k)
    assert np.all(h.child_count[lo[-2]:] == 0)
    assert np.all(h.child_count[:lo[-2]] > 0)


def test_parent_moments_and_enclosing_spheres(small):
    """Parent mean/covariance equal the weighted mixture moments with
    w = o (s1 s2 + s2 s3 + s1 s3); each sphere encloses its children's."""
    _, h = small
    cov = covariances(h.scales, h.quats)
    rng = np.random.default_rng(0)
    internal = np.nonzero(h.child_count > 0)[0]
    for k in rng.choice(internal, 200, replace=False):
        ch = np.arange(h.first_child[k], h.first_child[k] + h.child_count[k])
        s = h.scales[ch].astype(np.float64); o = h.opacity[ch].astype(np.float64)
        w = o * (s[:, 0] * s[:, 1] + s[:, 1] * s[:, 2] + s[:, 0] * s[:, 2])
        m = h.means[ch].astype(np.float64)
        mu = (w[:, None] * m).sum(0) / w.sum()
        d = m - mu
        P = (w[:, None, None] * (cov[ch] + d[:, :, None] * d[:, None, :])).sum(0) / w.sum()
        np.testing.assert_allclose(h.means[k], mu, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(cov[k], P, rtol=2e-5, atol=1e-7 * np.abs(P).max())
        c = h.bound[k, :3].astype(np.float64); r = float(h.bound[k, 3])
        reach = np.linalg.norm(h.bound[ch, :3].astype(np.float64) - c, axis=1) + h.bound[ch, 3]
        assert np.all(reach <= r)
    leaves = np.nonzero(h.child_count == 0)[0]
    np.testing.assert_array_equal(h.bound[leaves, 3] >= 3 * h.scales[leaves].max(1), True)


def test_workload_cameras():
    scene, cams = W.plan2m(scale=0.005, n_poses=10, use_cache=False)
    assert len(cams) == 10
    for c in cams:
        assert (c.width, c.height, c.fx) == (1280, 720, 900.0)
        assert abs(c.position[2] - 1.2) < 1e-6
        R = c.R.astype(np.float64)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
        np.testing.assert_allclose(np.cross(R[0], R[1]), R[2], atol=1e-6)
