"""The library's host implementation of the camera-clustering view sampler
(Sec. 4.3; lmrs_view_clusters / lmrs_view_batch, plain C++ in liblmrs, no
device work) against the oracle's: same labels and the same batches."""
import ctypes as C

import numpy as np
import pytest

from oracle.views import camera_features, kmeans, view_batch
from paper_2504_12905_amd import synth


def ring_cameras():
    return synth.ellipse_cameras(150, 1264, 832, 70.0, 0)


@pytest.mark.parametrize("B,seed", [(8, 0), (16, 3), (32, 11)])
def test_library_matches_oracle(B, seed):
    """liblmrs' host K-means and batch draw give the oracle's labels and views."""
    from paper_2504_12905_amd import lmrs as L
    cams = np.ascontiguousarray(ring_cameras(), dtype=np.float32)
    labels = np.zeros(cams.shape[0], np.int32)
    st = L._lib.lmrs_view_clusters(C.c_void_p(cams.ctypes.data), cams.shape[0], B, seed,
                                   C.c_void_p(labels.ctypes.data))
    assert st == L.LMRS_OK
    ref, _ = kmeans(camera_features(cams), B, seed)
    assert np.array_equal(labels, ref)
    for it in (0, 1, 49, 50):
        ids = np.zeros(B, np.int32)
        assert L._lib.lmrs_view_batch(C.c_void_p(labels.ctypes.data), cams.shape[0], B, seed, it,
                                      C.c_void_p(ids.ctypes.data)) == L.LMRS_OK
        assert np.array_equal(ids, view_batch(ref, B, seed, it))


def test_library_rejects_bad_batches():
    from paper_2504_12905_amd import lmrs as L
    cams = np.ascontiguousarray(ring_cameras()[:5], dtype=np.float32)
    labels = np.zeros(5, np.int32)
    assert L._lib.lmrs_view_clusters(C.c_void_p(cams.ctypes.data), 5, 6, 0, C.c_void_p(labels.ctypes.data)) \
        == L.LMRS_EINVAL
    assert L._lib.lmrs_view_clusters(None, 5, 2, 0, C.c_void_p(labels.ctypes.data)) == L.LMRS_EINVAL
    labels[:] = [0, 0, 0, 0, 0]  # cluster 1 empty
    ids = np.zeros(2, np.int32)
    assert L._lib.lmrs_view_batch(C.c_void_p(labels.ctypes.data), 5, 2, 0, 0, C.c_void_p(ids.ctypes.data)) \
        == L.LMRS_EINVAL
