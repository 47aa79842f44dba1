"""The seeded input generators (shared by the oracle and the GPU tests;
they hold none of the method's arithmetic)."""
import numpy as np

from paper_1301_1704_amd import inputs as I


def test_moved_points_properties():
    p = I.uniform_points(301, 20000)
    q = I.moved_points(p, 302, 1e-3)
    assert q.dtype == np.float32 and q.shape == p.shape
    assert np.array_equal(q, I.moved_points(p, 302, 1e-3))          # seeded
    assert not np.array_equal(q, I.moved_points(p, 303, 1e-3))      # its own stream
    assert np.array_equal(I.moved_points(p, 302, 0.0), p)
    assert q.min() >= 0.0 and q.max() <= np.float32(1.0 - 2.0 ** -24)
    d = (q.astype(np.float64) - p)[(p > 0.01).all(1) & (p < 0.99).all(1)]
    assert abs(d.mean()) < 3e-5 and abs(d.std() / 1e-3 - 1.0) < 0.02
