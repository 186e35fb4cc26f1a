"""Oracle five-point box solver (TEST INFRASTRUCTURE ONLY).

Solves the finite-difference system of eq. (3.31),

    (u_E + u_W + u_N + u_S - 4 u_P) / h^2 - kappa u_P = R_P,
    i, j = 1..M-1,  u = 0 on the box boundary,

exactly (up to rounding).  Two independent routes:

  solve        the paper's fast solver (section 3.4.2): transform the data to
               sine coefficients in both directions, divide by the
               eigenvalues of the five-point operator, transform back.  The
               DST-I here is scipy's (a library primitive).
  solve_dense  assembles the (M-1)^2 x (M-1)^2 matrix and calls a dense
               LU solve; used to pin `solve` on tiny grids.

Arrays are the (M-1) x (M-1) interior block indexed [j, i] (y row, x column).
kappa may be complex (the Schroedinger step).
"""

import numpy as np
import scipy.fft as sfft


def eigenvalues(M, h, kappa):
    """lambda[l, k] = -(4/h^2)(sin^2(pi k/2M) + sin^2(pi l/2M)) - kappa, the
    eigenvalue of Delta_h - kappa on sin(pi k i/M) sin(pi l j/M)."""
    s = np.sin(np.pi * np.arange(1, M) / (2.0 * M)) ** 2
    return -(4.0 / (h * h)) * (s[:, None] + s[None, :]) - kappa


def solve(R, h, kappa):
    M = R.shape[0] + 1
    assert R.shape == (M - 1, M - 1)
    Rhat = sfft.dstn(R, type=1)
    return sfft.idstn(Rhat / eigenvalues(M, h, kappa), type=1)


def five_point_matrix(M, h, kappa):
    n = M - 1
    N = n * n
    dtype = np.complex128 if np.iscomplexobj(kappa) else np.float64
    A = np.zeros((N, N), dtype=dtype)
    for j in range(n):
        for i in range(n):
            r = j * n + i
            A[r, r] = -4.0 / (h * h) - kappa
            if i > 0:
                A[r, r - 1] = 1.0 / (h * h)
            if i < n - 1:
                A[r, r + 1] = 1.0 / (h * h)
            if j > 0:
                A[r, r - n] = 1.0 / (h * h)
            if j < n - 1:
                A[r, r + n] = 1.0 / (h * h)
    return A


def solve_dense(R, h, kappa):
    M = R.shape[0] + 1
    A = five_point_matrix(M, h, kappa)
    return np.linalg.solve(A, R.ravel()).reshape(R.shape)


def apply(U, h, kappa):
    """(Delta_h - kappa) U on the interior block, U = 0 outside it."""
    P = np.pad(U, 1)
    return (P[1:-1, 2:] + P[1:-1, :-2] + P[2:, 1:-1] + P[:-2, 1:-1]
            - 4.0 * P[1:-1, 1:-1]) / (h * h) - kappa * U
