"""The seeded input generators shared by the tests, the benchmark and the
oracle: deterministic, of the stated shapes, counter-clockwise curves, and
the tripod of the paper's examples (Section 8) with node 0 at x = (1, 0),
the observation point of the fictitious-frequency figure (Section 8.4)."""
import math

import numpy as np

import synthetic as sy


def _signed_area(p):
    q = np.roll(p, -1, axis=0)
    return 0.5 * np.sum(p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1])


def test_tripod_shape_and_observation_node():
    p = sy.tripod(400)
    assert p.shape == (400, 2)
    assert np.allclose(p[0], [1.0, 0.0], atol=1e-15)
    assert _signed_area(p) > 0
    # three lobes: radius (1 + 0.3 cos 3t) / 1.3 at the vertex angles
    t = np.arctan2(p[:, 1], p[:, 0])
    assert np.allclose(np.hypot(p[:, 0], p[:, 1]), (1.0 + 0.3 * np.cos(3 * t)) / 1.3, atol=1e-12)


def test_curves_are_counter_clockwise():
    for c in [sy.circle(64), sy.ellipse(100, 1.0, 0.5, angle=0.7)] + sy.multi_cavity(3, 8, 4096):
        assert _signed_area(c) > 0


def test_field_inputs_are_seeded():
    curves = [sy.tripod(300)]
    a, b, c = sy.field_targets(curves, 11), sy.field_targets(curves, 11), sy.field_targets(curves, 12)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.shape == (12 + 8 * 6 + 4, 2)
    x = sy.random_boundary_values(600, 3, 5)
    assert x.shape == (3, 600) and x.dtype == np.complex128
    assert np.array_equal(x, sy.random_boundary_values(600, 3, 5))


def test_plane_wave_angles():
    a = sy.plane_wave_angles(180)
    assert len(a) == 180 and a[0] == 0.0 and math.isclose(a[-1], math.radians(358.0))
