"""Host logic of the volume/lensing instrumentation (no GPU)."""
import numpy as np

from paper_1508_05856_amd import lensing


def test_plane_fractions_count_each_diagonal():
    t = np.array([[0, 0, 0], [1, 2, 1], [3, 3, 1], [2, 5, 5], [4, 0, 2]])
    f = lensing.plane_fractions(t)
    assert f == {"ik": 2 / 5, "kj": 2 / 5, "ij": 2 / 5}
    f1 = lensing.plane_fractions(t, width=1)
    assert f1 == {"ik": 2 / 5, "kj": 3 / 5, "ij": 3 / 5}
    assert lensing.plane_fractions(np.zeros((0, 3)))["ik"] == 0.0


def test_volume_percent_of_a_dense_product_is_100():
    n, b = 512, 32
    assert lensing.volume_percent((n // b) ** 3, n, b) == 100.0
    assert lensing.volume_percent(0, n, b) == 0.0
