"""Pins of the oracle's five-point box solver (eq. 3.31, u = 0 on the box).

The fast route (sine transforms in x and y, divide by the eigenvalues) is
checked against a dense LU solve of the assembled matrix on tiny grids and
against the closed form on a discrete eigenvector.
"""

import numpy as np
import pytest

from oracle import boxsolve


@pytest.mark.parametrize("M", [8, 12, 16])
@pytest.mark.parametrize("kappa", [0.0, 37.5, 2.0e3, 3.0j * 64.0])
def test_fast_solve_equals_dense_lu(M, kappa, rng):
    h = 2.0 / M
    R = rng.standard_normal((M - 1, M - 1))
    if np.iscomplexobj(kappa):
        R = R + 1j * rng.standard_normal((M - 1, M - 1))
    U = boxsolve.solve(R, h, kappa)
    Ud = boxsolve.solve_dense(R, h, kappa)
    assert np.max(np.abs(U - Ud)) <= 1e-12 * np.max(np.abs(Ud))
    # and the residual of the difference equations themselves
    res = boxsolve.apply(U, h, kappa) - R
    assert np.max(np.abs(res)) <= 1e-10 * np.max(np.abs(R)) * (4.0 / (h * h) + abs(kappa)) * h * h


@pytest.mark.parametrize("M,k,l", [(16, 1, 1), (16, 3, 7), (32, 31, 2), (64, 17, 40)])
def test_eigenvector_closed_form(M, k, l):
    """sin(pi k i/M) sin(pi l j/M) is an eigenvector of Delta_h with
    eigenvalue -(4/h^2)(sin^2(pi k/2M) + sin^2(pi l/2M))."""
    h = 2.0 / M
    kappa = 5.0
    i = np.arange(1, M)
    E = np.sin(np.pi * l * i / M)[:, None] * np.sin(np.pi * k * i / M)[None, :]
    lam = -(4.0 / (h * h)) * (np.sin(np.pi * k / (2 * M)) ** 2
                              + np.sin(np.pi * l / (2 * M)) ** 2) - kappa
    U = boxsolve.solve(E, h, kappa)
    assert np.max(np.abs(U - E / lam)) <= 1e-14 * np.max(np.abs(E / lam)) * M


def test_dense_matrix_structure():
    """Row sums of the assembled operator: -kappa in the interior, and one
    1/h^2 fewer per missing (boundary) neighbour."""
    M, h, kappa = 6, 0.25, 3.0
    A = boxsolve.five_point_matrix(M, h, kappa)
    n = M - 1
    rs = A.sum(axis=1).reshape(n, n)
    assert np.isclose(rs[2, 2], -kappa)
    assert np.isclose(rs[0, 2], -kappa - 1.0 / h ** 2)
    assert np.isclose(rs[0, 0], -kappa - 2.0 / h ** 2)
    assert np.allclose(A, A.T)
