"""Input generators of the paper's sweeps (no method arithmetic): the
detector locations of Sec. 6.1."""
import math

import numpy as np

import phantoms


def test_rotated_array_locations():
    a = phantoms.rotated_array_angles()
    assert a.shape == (384,) and np.all(np.diff(a) >= 0) and a.min() >= 0 and a.max() < 2 * math.pi
    base = phantoms.rotated_array_angles(n_rot=1)
    # one array: 64 elements, ends 172 degrees apart, centred on angle 0
    unwrapped = np.sort(np.angle(np.exp(1j * base)))
    assert len(base) == 64
    assert math.degrees(unwrapped[-1] - unwrapped[0]) == __import__("pytest").approx(172.0, abs=1e-9)
    assert abs(unwrapped[0] + unwrapped[-1]) < 1e-12


def test_uniform_subsets():
    a = phantoms.rotated_array_angles()
    for c in (16, 32, 64):
        s = phantoms.uniform_subset(a, c)
        assert len(np.unique(s)) == c and np.all(np.isin(s, a))
        gaps = np.diff(np.concatenate([s, [s[0] + 2 * math.pi]]))
        assert gaps.max() < 1.5 * 2 * math.pi / c and gaps.min() > 0.5 * 2 * math.pi / c
    assert np.array_equal(phantoms.uniform_subset(a, 384), a)
    xy = phantoms.detectors_xy(a[:3])
    assert np.allclose(np.hypot(xy[:, 0], xy[:, 1]), 1.2)
