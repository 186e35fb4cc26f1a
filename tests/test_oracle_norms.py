"""Pins of the oracle's error norms (reading R18: the max norm and the root
mean square over inside nodes), by hand-computed values and the inequalities
between the two norms."""

import math

import numpy as np

from oracle.norms import max_norm, rms_norm


def test_hand_computed_values():
    err = np.array([[3.0, -4.0], [100.0, 0.0]])
    inside = np.array([[True, True], [False, True]])
    # inside errors 3, -4, 0: max 4, rms sqrt(25 / 3)
    assert max_norm(err, inside) == 4.0
    assert math.isclose(rms_norm(err, inside), math.sqrt(25.0 / 3.0), rel_tol=0, abs_tol=1e-15)


def test_complex_errors_use_the_modulus():
    err = np.array([3.0 + 4.0j, 0.0 + 1.0j, 7.0])
    inside = np.array([True, True, False])
    assert max_norm(err, inside) == 5.0
    assert math.isclose(rms_norm(err, inside), math.sqrt((25.0 + 1.0) / 2.0), rel_tol=0, abs_tol=1e-15)


def test_norm_inequalities_and_equality_case(rng):
    err = rng.standard_normal((17, 17)) + 1j * rng.standard_normal((17, 17))
    inside = rng.random((17, 17)) < 0.5
    n = int(inside.sum())
    mx, rms = max_norm(err, inside), rms_norm(err, inside)
    # rms <= max <= sqrt(n) rms
    assert rms <= mx <= math.sqrt(n) * rms * (1 + 1e-15)
    # constant modulus: the two norms agree
    const = 2.5 * np.exp(1j * rng.uniform(0, 2 * np.pi, (17, 17)))
    assert math.isclose(rms_norm(const, inside), 2.5, rel_tol=1e-15)
    assert math.isclose(max_norm(const, inside), 2.5, rel_tol=1e-15)


def test_no_inside_node():
    err = np.ones((3, 3))
    inside = np.zeros((3, 3), dtype=bool)
    assert max_norm(err, inside) == 0.0 and rms_norm(err, inside) == 0.0
