"""Pins of the oracle Richardson iteration (eq. 3.21) against closed forms
and a direct solve.

  * diagonal operator K = diag(lam): from phi_0 = 0 the iterate after k
    updates is exactly (1 - (1 - gamma lam)^k) b / lam, componentwise;
  * symmetric K: the residual contracts by at most rho = max |1 - gamma lam|
    per update, so the update count is at most ceil(log(tol) / log(rho));
  * the discrete second-kind equation of a small heat disk: the limit equals
    the direct (LU) solution of the assembled K, and the late contraction of
    the residual approaches the spectral radius of I - gamma K.
"""

import math

import numpy as np

import workloads as W
from oracle import bie
from oracle.geometry import Domain
from oracle.richardson import richardson


def test_diagonal_closed_form():
    rng = np.random.default_rng(1)
    lam = rng.uniform(0.2, 1.0, 40)
    b = rng.standard_normal(40)
    for gamma in (0.3, 0.9):
        for k in range(1, 6):
            phi, n, _, _ = richardson(lambda v: lam * v, b, gamma=gamma, fixed_iters=k)
            assert n == k
            ref = (1.0 - (1.0 - gamma * lam) ** k) * b / lam
            assert np.max(np.abs(phi - ref)) < 1e-13 * np.max(np.abs(ref))


def test_symmetric_contraction_bound():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    lam = rng.uniform(0.3, 0.9, 30)
    K = (Q * lam) @ Q.T
    b = rng.standard_normal(30)
    gamma, tol = 0.8, 1e-10
    rho = np.max(np.abs(1.0 - gamma * lam))
    phi, n, rel, conv = richardson(lambda v: K @ v, b, gamma=gamma, tol=tol)
    assert conv and rel <= tol
    assert n <= math.ceil(math.log(tol) / math.log(rho))
    assert np.allclose(phi, np.linalg.solve(K, b), rtol=0, atol=1e-8)


def test_bie_limit_and_rate():
    od = Domain(W.domain_c1_heat(32, Nb=64))
    kappa = 64.0
    K = bie.dense_operator(od, kappa)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(od.Nb)
    gamma = 1.0
    phi, n, rel, conv = richardson(lambda v: bie.matvec(od, kappa, v), b, gamma=gamma, tol=1e-11, max_iter=400)
    assert conv
    direct = np.linalg.solve(K, b)
    assert np.max(np.abs(phi - direct)) < 1e-9 * np.max(np.abs(direct))
    # late contraction of the residual against the spectral radius of I - gamma K
    rho = np.max(np.abs(1.0 - gamma * np.linalg.eigvals(K)))
    res = []
    x = np.zeros(od.Nb)
    for _ in range(60):
        r = b - K @ x
        res.append(np.linalg.norm(r))
        x = x + gamma * r
    ratio = (res[-1] / res[-11]) ** 0.1
    assert abs(ratio - rho) < 0.05 * rho
