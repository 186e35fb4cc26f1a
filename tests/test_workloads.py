"""Input generators: the tensor-grid evaluation of the smooth random fields
equals their pointwise definition."""

import numpy as np

import workloads as W
from workloads.fields import SmoothField


def test_smooth_field_grid_matches_pointwise():
    for seed, M in ((1, 16), (7, 64), (20240423, 128)):
        f = SmoothField(np.random.default_rng(seed))
        x = W.grid_coords(1.0, M)
        X, Y = np.meshgrid(x, x)
        ref = f(X, Y)
        got = f.grid(x, x)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        # rows are y, columns x
        assert abs(got[3, 5] - f(x[5], x[3])) <= 1e-13
