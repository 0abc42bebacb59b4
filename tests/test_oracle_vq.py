"""Pins of the VQ oracle (Sec. 4.4) against hand-worked Lloyd iterations,
an independent nearest-centroid method, and properties of k-means."""
import numpy as np
import pytest

from oracle import vq as V


def test_assign_ties_take_the_lower_index_and_nonfinite_take_zero():
    c = np.array([0.0, 1.0, 4.0], np.float32)
    x = np.array([0.2, 0.5, 0.8, 2.5, 3.0, -7.0, 9.0, np.nan, np.inf], np.float32)
    # 0.5 and 2.5 are equidistant from two centroids: the lower index wins
    assert V.assign(x, c).tolist() == [0, 0, 1, 1, 2, 0, 2, 0, 0]


def test_assign_duplicate_centroids_take_the_first():
    c = np.array([1.0, 1.0, 1.0, 5.0], np.float32)
    assert V.assign(np.array([0.0, 1.0, 2.9, 3.1], np.float32), c).tolist() == [0, 0, 0, 3]


def test_assign_matches_voronoi_cells_from_midpoints():
    # independent method: for an ascending codebook the cell of centroid j is
    # the interval between the midpoints with its neighbours
    rng = np.random.default_rng(3)
    c = np.sort(rng.normal(size=37).astype(np.float32))
    x = rng.normal(scale=1.5, size=20000).astype(np.float32)
    mid = (c[1:].astype(np.float64) + c[:-1]) / 2
    ref = np.searchsorted(mid, x.astype(np.float64), side="left")
    # away from the midpoints both decide alike (FP32 versus exact rounding)
    gap = np.min(np.abs(x.astype(np.float64)[:, None] - mid[None, :]), axis=1)
    far = gap > 1e-5
    assert far.mean() > 0.99
    np.testing.assert_array_equal(V.assign(x, c)[far], ref[far])


def test_lloyd_hand_worked_two_clusters():
    x = np.array([0, 1, 2, 10, 11, 12], np.float32)
    # init: [min, max] = [0, 12] in 2 cells -> centres 3 and 9
    np.testing.assert_array_equal(V.init_codebook(x, 2), [3.0, 9.0])
    c, idx = V.fit(x, 2, 3)
    np.testing.assert_array_equal(c, [1.0, 11.0])  # the means of {0,1,2} and {10,11,12}
    assert idx.tolist() == [0, 0, 0, 1, 1, 1]


def test_lloyd_empty_cluster_keeps_its_centroid():
    x = np.array([0, 0, 10, 10], np.float32)
    c0 = V.init_codebook(x, 3)  # 10/3 * (0.5, 1.5, 2.5)
    np.testing.assert_allclose(c0, [5 / 3, 5, 25 / 3], rtol=1e-6)
    c1 = V.lloyd_step(x, c0)
    np.testing.assert_array_equal(c1, [0.0, 5.0, 10.0])  # the middle cluster received nothing


def test_lloyd_ignores_nonfinite_values():
    x = np.array([1.0, np.nan, 3.0, -np.inf], np.float32)
    c, idx = V.fit(x, 1, 2)
    np.testing.assert_array_equal(c, [2.0])
    assert idx.tolist() == [0, 0, 0, 0]


def test_all_equal_values_collapse_onto_one_centroid():
    x = np.full(100, 0.25, np.float32)
    c, idx = V.fit(x, 4, 3)
    np.testing.assert_array_equal(c, [0.25] * 4)  # zero-width range: every centre at the value
    assert (idx == 0).all()


def test_separated_clusters_are_recovered():
    rng = np.random.default_rng(11)
    # each true centre lies nearest its own initial cell centre, so Lloyd's
    # first assignment is already the true labelling
    centres = np.array([-3.0, -1.0, 1.0, 3.0, 5.0])
    labels = rng.integers(0, 5, size=5000)
    labels[:5] = np.arange(5)  # every cluster non-empty
    x = (centres[labels] + rng.uniform(-0.05, 0.05, size=5000)).astype(np.float32)
    c, idx = V.fit(x, 5, 20)
    assert idx.tolist() == labels.tolist()
    want = np.array([x[labels == j].astype(np.float64).mean() for j in range(5)], np.float32)
    np.testing.assert_array_equal(c, want)


def test_lloyd_objective_never_increases():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(0, 1, 3000), rng.exponential(2.0, 2000)]).astype(np.float32)
    c = V.init_codebook(x, 16)
    prev = V.objective(x, c, V.assign(x, c))
    for _ in range(10):
        c = V.lloyd_step(x, c)
        cur = V.objective(x, c, V.assign(x, c))
        assert cur <= prev * (1 + 1e-12)
        prev = cur
    assert np.all(np.diff(c) >= 0)


def test_quantize_uses_each_attributes_own_codebook():
    # attributes on disjoint ranges: a plane decoded through another
    # attribute's codebook would leave its range
    rng = np.random.default_rng(2)
    n = 3000
    planes = {
        "mean": rng.normal(size=(3, n)).astype(np.float32),
        "normal": rng.normal(size=(3, n)).astype(np.float32),
        "log_scale": rng.uniform(-6, -5, (3, n)).astype(np.float32),
        "quat": rng.uniform(10, 11, (4, n)).astype(np.float32),
        "opacity": rng.uniform(20, 21, (1, n)).astype(np.float32),
        "color": rng.uniform(30, 31, (3, n)).astype(np.float32),
        "shade": (rng.uniform(0, 1, (4, n)) + np.array([[40], [50], [60], [70]])).astype(np.float32),
    }
    q = V.quantize(planes, 16, 4)
    d = V.decode(q)
    np.testing.assert_array_equal(d["mean"], planes["mean"])
    np.testing.assert_array_equal(d["normal"], planes["normal"])
    for name in ("log_scale", "quat", "opacity", "color", "shade"):
        lo = planes[name].min(axis=1, keepdims=True) - 1e-3
        hi = planes[name].max(axis=1, keepdims=True) + 1e-3
        assert ((d[name] >= lo) & (d[name] <= hi)).all(), name
        # 16 centroids over a unit range: error within about a cell
        assert np.abs(d[name] - planes[name]).max() < 0.2, name
    # the four shading terms have separate codebooks: each reproduces its own band
    for r, base in enumerate((40, 50, 60, 70)):
        assert (np.floor(q["codebook"][4 + r]) == base).all()


@pytest.mark.parametrize("k", [1, 2, 256])
def test_codebook_stays_ascending(k):
    rng = np.random.default_rng(k)
    x = rng.standard_t(3, size=4000).astype(np.float32)
    c, idx = V.fit(x, k, 6)
    assert np.all(np.diff(c) >= 0)
    assert idx.max() < k
