"""The seeded input generators: shapes, ranges and the distribution laws the
paper states for its synthetic sets (Sec. 5.1) and weights (Sec. 5.1,
power diagrams)."""
import numpy as np
import pytest

from paper_2605_06408_amd import workloads as wl


@pytest.mark.parametrize("name", sorted(wl.CONFIGS))
def test_every_configuration_draws_in_its_box(name):
    xyz, w, box = wl.make(name, 3, 4000)
    assert xyz.shape == (4000, 3) and xyz.dtype == np.float32
    assert w is None or (w.shape == (4000,) and w.dtype == np.float32)
    if not name.startswith("surface"):  # the surface set's box is its far-field cube
        assert np.all(xyz >= box[:3]) and np.all(xyz <= box[3:])
    a = wl.make(name, 3, 4000)
    assert np.array_equal(a[0], xyz)  # seeded


def test_paper_gradient_density_is_linear_in_x():
    xyz, _, _ = wl.paper_gradient(400_000, 1)
    # p(x) ∝ x + 10 on [-10, 10]: the share of points below x is ((x + 10) / 20)^2
    for x in (-5.0, 0.0, 5.0):
        share = float(np.mean(xyz[:, 0] < x))
        assert share == pytest.approx(((x + 10.0) / 20.0) ** 2, abs=3e-3)
    assert float(np.mean(xyz[:, 1] < 0.0)) == pytest.approx(0.5, abs=3e-3)


def test_paper_clusters_split_evenly_with_sigma_0_1():
    xyz, _, _ = wl.paper_clusters(10_003, 2, k=10)
    # points come in 10 consecutive groups (the first 3 one longer), each a
    # Gaussian of sigma 0.1 (clamping aside)
    sizes = [1001] * 3 + [1000] * 7
    start = 0
    for c in sizes:
        g = xyz[start:start + c].astype(np.float64)
        start += c
        inside = np.all(np.abs(g) < 9.5, axis=1)
        if inside.mean() > 0.99:
            assert np.std(g, axis=0) == pytest.approx([0.1, 0.1, 0.1], rel=0.1)


def test_paper_weights_follow_the_nearest_neighbour_law():
    xyz, _, _ = wl.paper_uniform(3000, 4)
    w = wl.paper_weights(xyz, 4)
    p = xyz.astype(np.float64)
    d2 = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    dnn = float(np.median(np.sqrt(d2.min(axis=1))))  # brute force
    assert float(np.std(w)) == pytest.approx(dnn * dnn / 3.0, rel=0.05)
    assert abs(float(np.mean(w))) < 0.1 * dnn * dnn / 3.0
