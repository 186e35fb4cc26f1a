"""Pins of the oracle GMRES and Dirichlet BIE solve: a dense direct solve of
the assembled operator K, the true GMRES residual, closed-form Helmholtz
solutions (u = exp(ax+by) with a^2+b^2 = kappa, u = I0(sqrt(kappa) r) on the
disk) and the observed second-order convergence the method claims.
"""

import numpy as np
import pytest
import scipy.special

import workloads as W
from workloads import manufactured as mf
from oracle import bie
from oracle import geometry as G
from oracle.gmres import gmres


def test_gmres_matches_direct_solve_with_restarts(rng):
    n = 60
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, it, rel, conv = gmres(lambda v: A @ v, b, tol=1e-12, restart=7)
    assert conv and it > 7
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1.01e-12
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)


def test_gmres_complex_and_fixed_iterations(rng):
    n = 40
    A = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    calls = []

    def mv(v):
        calls.append(1)
        return A @ v
    x, it, rel, conv = gmres(mv, b, tol=1e-12, restart=50)
    assert conv and np.allclose(x, np.linalg.solve(A, b), atol=1e-10)
    calls.clear()
    x5, it5, _, _ = gmres(mv, b, fixed_iters=5)
    assert it5 == 5 and len(calls) == 5


@pytest.fixture(scope="module")
def small_disk():
    return G.Domain(W.domains.disk(0.5, 1.0, 32, 48))


def test_bie_gmres_matches_dense_operator(small_disk):
    d = small_disk
    kappa = 30.0
    K = bie.dense_operator(d, kappa)
    g = np.cos(d.theta) + 0.5 * np.sin(3 * d.theta)
    b = bie.rhs(d, kappa, None, None, g)
    phi_direct = np.linalg.solve(K, b)
    U, phi, st = bie.helmholtz_solve(d, kappa, None, None, g, tol=1e-13)
    assert st["converged"]
    assert np.max(np.abs(phi - phi_direct)) < 1e-10 * np.max(np.abs(phi_direct))
    assert np.linalg.norm(K @ phi - b) / np.linalg.norm(b) < 1e-12
    # K is a perturbation of 1/2 I + W: its spectrum sits in the right half plane
    ev = np.linalg.eigvals(K)
    assert ev.real.min() > 0.0


def _order(errs):
    return np.log2(errs[0] / errs[-1]) / (len(errs) - 1)


def test_bvp_exponential_solution_second_order():
    """lap u - kappa u = 0 with u = exp(ax+by), a^2 + b^2 = kappa, on the disk."""
    kappa, a = 64.0, 6.0
    b = np.sqrt(kappa - a * a)
    errs = []
    for M in (32, 64, 128, 256):
        d = G.Domain(W.domains.disk(0.5, 1.0, M, 2 * M))
        g = mf.helm_exp_u(d.colloc["x"], d.colloc["y"], a, b)
        U, _, st = bie.helmholtz_solve(d, kappa, None, None, g, tol=1e-12)
        errs.append(np.max(np.abs(U - mf.helm_exp_u(d.X, d.Y, a, b))[d.inside]))
    assert _order(errs) > 1.8, errs


def test_bvp_bessel_solution_on_disk():
    """u = I0(sqrt(kappa) r) solves lap u = kappa u."""
    kappa = 100.0
    errs = []
    for M in (32, 64, 128):
        d = G.Domain(W.domains.disk(0.45, 1.0, M, 2 * M))
        g = scipy.special.i0(np.sqrt(kappa) * np.hypot(d.colloc["x"], d.colloc["y"]))
        U, _, _ = bie.helmholtz_solve(d, kappa, None, None, g, tol=1e-12)
        ex = scipy.special.i0(np.sqrt(kappa) * np.hypot(d.X, d.Y))
        errs.append(np.max(np.abs(U - ex)[d.inside]) / np.max(np.abs(ex[d.inside])))
    assert _order(errs) > 1.8, errs


@pytest.mark.parametrize("kappa", [64.0, 512j])
def test_bvp_with_source_on_star_second_order(kappa):
    """u = sin(pi x) cos(pi y), f = lap u - kappa u, star domain; real and
    complex kappa (the Schroedinger coefficient is imaginary)."""
    errs = []
    for M in (64, 128, 256):
        d = G.Domain(W.domain_c2_wave(M))
        zx, zy = d.colloc["x"], d.colloc["y"]
        U, _, st = bie.helmholtz_solve(d, kappa, mf.helm_trig_f(d.X, d.Y, kappa),
                                       mf.helm_trig_f(zx, zy, kappa),
                                       mf.helm_trig_u(zx, zy), tol=1e-12)
        errs.append(np.max(np.abs(U - mf.helm_trig_u(d.X, d.Y))[d.inside]))
    assert _order(errs) > 1.5, errs
    assert errs[-1] < 5e-4
