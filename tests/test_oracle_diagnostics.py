"""Pins of the oracle's label ingestion and tumour diagnostics (sections 3.1,
3.2 and 3.5): hand-computed threshold and sampling cases, constant fields,
and closed-form diameters of boxes, balls and point pairs."""

import numpy as np
import pytest

from oracle import diagnostics as dg


def test_threshold_boundaries():
    # air <= 1 < white <= 115 < gray <= 240 < skull
    vals = np.array([0, 1, 2, 115, 116, 240, 241, 255], dtype=np.uint8)
    img = vals.reshape(1, 1, -1)
    lab = dg.labels_from_intensity(img, img.shape)
    assert lab.ravel().tolist() == [0, 0, 1, 1, 2, 2, 3, 3]


def test_other_thresholds_and_validation():
    img = np.arange(256, dtype=np.uint8).reshape(4, 8, 8)
    lab = dg.labels_from_intensity(img, img.shape, thresholds=(63, 127))
    assert np.array_equal(lab.ravel(), (np.arange(256) > 63).astype(int) + (np.arange(256) > 127))
    with pytest.raises(ValueError):
        dg.labels_from_intensity(img, img.shape, thresholds=(5, 5))
    with pytest.raises(ValueError):
        dg.labels_from_intensity(img.astype(np.int16), img.shape)


def test_sampling_identity_and_halving():
    # the same grid maps to itself; half the resolution takes the odd samples
    assert dg.sample_index(7, 7).tolist() == list(range(7))
    assert dg.sample_index(4, 8).tolist() == [1, 3, 5, 7]
    # 3 points over 10 samples: cell centres 10/6, 30/6, 50/6 -> 1, 5, 8
    assert dg.sample_index(3, 10).tolist() == [1, 5, 8]
    # more points than samples: repeat samples
    assert dg.sample_index(5, 2).tolist() == [0, 0, 1, 1, 1]


def test_sampled_volume_picks_the_right_voxels():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(6, 10, 12)).astype(np.uint8)
    lab = dg.labels_from_intensity(img, (3, 5, 4))
    for i, I in enumerate([1, 3, 5]):
        for j, J in enumerate([1, 3, 5, 7, 9]):
            for k, K in enumerate([1, 4, 7, 10]):
                v = int(img[I, J, K])
                assert lab[i, j, k] == (v > 1) + (v > 115) + (v > 240)


def test_volume_of_constant_and_mixed_fields():
    assert dg.tumour_volume(np.full((3, 4, 5), 0.25)) == pytest.approx(0.25)
    u = np.zeros((2, 2, 2))
    u[0, 0, 0] = 1.0
    assert dg.tumour_volume(u) == pytest.approx(1 / 8)


def test_diameter_closed_forms():
    u = np.zeros((9, 8, 7))
    assert dg.tumour_diameter_sq(u, 0.5) == -1
    u[2, 3, 4] = 1.0
    assert dg.tumour_diameter_sq(u, 0.5) == 0
    u[6, 1, 0] = 0.9
    assert dg.tumour_diameter_sq(u, 0.5) == 16 + 4 + 16
    assert dg.tumour_diameter_sq(u, 0.95) == 0  # the second point is below
    box = np.zeros((10, 10, 10))
    box[2:5, 1:8, 3:9] = 1.0  # 3 x 7 x 6 points
    assert dg.tumour_diameter_sq(box, 0.0) == 2**2 + 6**2 + 5**2
    # lattice ball of radius 4: the farthest points are antipodal axis points
    g = np.indices((11, 11, 11)) - 5
    ball = ((g**2).sum(axis=0) <= 16).astype(float)
    assert dg.tumour_diameter_sq(ball, 0.5) == 64


def test_diameter_blocks_agree():
    rng = np.random.default_rng(5)
    u = (rng.random((9, 7, 8)) > 0.9).astype(float)
    p = dg.tumour_points(u, 0.5)
    brute = max(int(((a - b) ** 2).sum()) for a in p for b in p)
    assert dg.tumour_diameter_sq(u, 0.5, block=7) == brute


def test_diameter_pair_is_the_smallest_maximiser():
    u = np.zeros((4, 4, 4))
    # corners (0,0,0), (3,3,3) and (0,3,3), (3,0,0): two pairs at d2 = 27
    for c in [(0, 0, 0), (3, 3, 3), (0, 3, 3), (3, 0, 0), (1, 1, 1)]:
        u[c] = 1.0
    d2, a, b = dg.tumour_diameter_pair(u, 0.5)
    assert d2 == 27
    assert (a, b) == (0, 63)  # (0,0,0)-(3,3,3) beats (0,3,3)-(3,0,0) = (15, 48)
    one = np.zeros((2, 3, 4))
    one[1, 2, 3] = 1.0
    assert dg.tumour_diameter_pair(one, 0.5) == (0, 23, 23)
    assert dg.tumour_diameter_pair(np.zeros((2, 2, 2)), 0.5) == (-1, -1, -1)
