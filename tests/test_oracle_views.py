"""Pins of the oracle's camera-clustering view sampler (Sec. 4.3).

The pins check what K-means and the batch rule must satisfy whatever the code:
the fixed point of Lloyd's algorithm (each camera nearest to its own centre,
centres equal to their members' means), a closed form for well separated
camera groups, one camera per cluster, the B = N case, and the features of a
hand-placed camera."""
import numpy as np

from oracle.views import camera_features, kmeans, view_batch
from paper_2504_12905_amd import synth


def ring_cameras():
    return synth.ellipse_cameras(150, 1264, 832, 70.0, 0)


def test_features_of_an_axis_camera():
    """Camera at (0, 0, -3) looking along +z next to one at (0, 0, 3) looking
    along -z: centres +-(0, 0, 1) after normalisation, directions +-z."""
    a = np.zeros(16, np.float32)
    a[0:9] = np.eye(3).reshape(-1)
    a[9:12] = [0, 0, 3]
    b = np.zeros(16, np.float32)
    b[0:9] = np.diag([1.0, -1.0, -1.0]).reshape(-1)   # 180 degrees about x: looks along -z
    b[9:12] = [0, 0, 3]                                  # centre -R^T t = (0, 0, 3)
    f = camera_features(np.stack([a, b]))
    np.testing.assert_allclose(f[0], [0, 0, -1, 0, 0, 1], atol=1e-12)
    np.testing.assert_allclose(f[1], [0, 0, 1, 0, 0, -1], atol=1e-12)


def test_lloyd_fixed_point():
    """150 cameras on the noisy ellipse, B = 16: every camera's nearest centre
    is its own, and every centre is the mean of its members."""
    f = camera_features(ring_cameras())
    labels, Cc = kmeans(f, 16, 7)
    D = ((f[:, None, :] - Cc[None, :, :]) ** 2).sum(axis=-1)
    assert np.array_equal(D.argmin(axis=1), labels)
    for c in range(16):
        np.testing.assert_allclose(Cc[c], f[labels == c].mean(axis=0), rtol=1e-12, atol=1e-15)
    assert np.bincount(labels, minlength=16).min() >= 1


def test_separated_groups_are_found():
    """Four tight groups of 10 cameras at the corners of a square (all looking
    at the origin), B = 4: the clusters are the groups, and every batch has one
    camera of each group."""
    rng = np.random.default_rng(2)
    cams, group = [], []
    for gi, ang in enumerate([0.0, 0.5 * np.pi, np.pi, 1.5 * np.pi]):
        for _ in range(10):
            pos = np.array([4 * np.cos(ang), 4 * np.sin(ang), 0.0]) + rng.normal(0, 0.05, 3)
            R, t = synth.look_at(pos, np.zeros(3))
            cams.append(synth.pack_camera(R, t, 64, 64, 60.0))
            group.append(gi)
    cams, group = np.stack(cams), np.array(group)
    f = camera_features(cams)
    for seed in range(5):
        labels, _ = kmeans(f, 4, seed)
        # a bijection between clusters and groups
        assert len({(int(l), int(g)) for l, g in zip(labels, group)}) == 4
        for it in range(3):
            ids = view_batch(labels, 4, seed, it)
            assert sorted(group[ids].tolist()) == [0, 1, 2, 3]


def test_every_camera_its_own_cluster_when_b_equals_n():
    cams = synth.sphere_cameras(12, 3.0, 64, 64, 60.0, 4)
    labels, _ = kmeans(camera_features(cams), 12, 1)
    assert sorted(labels.tolist()) == list(range(12))
    assert sorted(view_batch(labels, 12, 1, 5).tolist()) == list(range(12))


def test_batches_follow_the_counter():
    f = camera_features(ring_cameras())
    labels, _ = kmeans(f, 16, 3)
    a = view_batch(labels, 16, 3, 4)
    assert np.array_equal(a, view_batch(labels, 16, 3, 4))
    assert len(set(a.tolist())) == 16 and all(labels[a] == np.arange(16))
    assert not np.array_equal(a, view_batch(labels, 16, 3, 5))
