"""Pins of the oracle Neumann solve (eqs. 3.19, 3.20 and the single-layer
interface problem 3.29): the normal-derivative extraction is exact for
piecewise quadratics, the assembled K_N is a second-kind operator (spectrum
in the right half plane, well conditioned at Nb = M), closed-form Helmholtz
solutions with du/dn data (exp(ax+by), I0 on the disk, a trigonometric
solution with a source, real and imaginary kappa) converge at second order,
the trace U+ converges to the exact boundary values, the Richardson form of
eq. 3.22 reaches the GMRES density, and Neumann time steps follow exact
solutions.
"""

import numpy as np
import pytest
import scipy.special

import workloads as W
from workloads import manufactured as mf
from oracle import bie
from oracle import geometry as G
from oracle import interface as I
from oracle.steppers import HeatStepper, WaveStepper

QP = np.array([1.0, 0.3, -0.2, 0.5, -0.7, 0.4])       # u+ coefficients
QJ = np.array([0.2, -0.1, 0.3, 0.25, 0.6, -0.35])     # u+ - u- (quadratic)


def _q(c, x, y):
    return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y


def _order(errs):
    return np.log2(errs[0] / errs[-1]) / (len(errs) - 1)


def _dn(grad, d):
    gx, gy = grad
    return gx * d.colloc["nx"] + gy * d.colloc["ny"]


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domain_c2_wave(128)])
def test_normal_extraction_exact_for_quadratics(desc):
    """u+ inside, u- = u+ - jq outside with the exact quadratic jumps at z:
    the extracted normal derivative equals n . grad u+(z) to rounding."""
    d = G.Domain(desc)
    X, Y = d.X, d.Y
    U = np.where(d.inside, _q(QP, X, Y), _q(QP, X, Y) - _q(QJ, X, Y))
    zx, zy = d.colloc["x"], d.colloc["y"]
    jz = {"u": _q(QJ, zx, zy),
          "ux": QJ[1] + 2 * QJ[3] * zx + QJ[4] * zy,
          "uy": QJ[2] + QJ[4] * zx + 2 * QJ[5] * zy,
          "uxx": np.full_like(zx, 2 * QJ[3]), "uxy": np.full_like(zx, QJ[4]),
          "uyy": np.full_like(zx, 2 * QJ[5])}
    got = I.extract(d, U, jz, d.st_weight_n)
    ex = (QP[1] + 2 * QP[3] * zx + QP[4] * zy) * d.colloc["nx"] + (QP[2] + QP[4] * zx + 2 * QP[5] * zy) * d.colloc["ny"]
    assert np.max(np.abs(got - ex)) < 1e-10


def test_normal_weights_are_normal_derivatives():
    """On linear data the weights give n . grad; they annihilate constants
    and the quadratic monomials (rows 1, 2 of the inverse Taylor system)."""
    d = G.Domain(W.domains.disk(0.5, 1.0, 64, 64))
    w = d.st_weight_n
    xi, eta = d.st_xi, d.st_eta
    assert np.max(np.abs(np.sum(w, axis=1))) < 1e-9
    assert np.max(np.abs(np.sum(w * xi, axis=1) - d.colloc["nx"])) < 1e-12
    assert np.max(np.abs(np.sum(w * eta, axis=1) - d.colloc["ny"])) < 1e-12
    for mono in (xi * xi, xi * eta, eta * eta):
        assert np.max(np.abs(np.sum(w * mono, axis=1))) < 1e-12


@pytest.mark.parametrize("desc", [W.domains.disk(0.5, 1.0, 48, 48), W.domains.star(0.5, 0.1, 5, 1.0, 64, 64)])
def test_neumann_operator_is_second_kind(desc):
    d = G.Domain(desc)
    K = bie.neumann_dense_operator(d, 25.0)
    ev = np.linalg.eigvals(K)
    assert ev.real.min() > 0.1 and ev.real.max() < 1.0, (ev.real.min(), ev.real.max())
    assert np.linalg.cond(K) < 10.0


def test_neumann_exponential_solution_second_order():
    """lap u - kappa u = 0, u = exp(ax+by) with a^2 + b^2 = kappa, du/dn
    given on the disk; the trace U+ converges too."""
    kappa, a = 64.0, 6.0
    b = np.sqrt(kappa - a * a)
    errs, terrs = [], []
    for M in (32, 64, 128, 256):
        d = G.Domain(W.domains.disk(0.5, 1.0, M, M))
        zx, zy = d.colloc["x"], d.colloc["y"]
        gn = _dn(mf.helm_exp_grad(zx, zy, a, b), d)
        U, _, Up, st = bie.neumann_solve(d, kappa, None, None, gn, tol=1e-12)
        assert st["converged"]
        ex = mf.helm_exp_u(d.X, d.Y, a, b)
        errs.append(np.max(np.abs(U - ex)[d.inside]) / np.max(np.abs(ex[d.inside])))
        terrs.append(np.max(np.abs(Up - mf.helm_exp_u(zx, zy, a, b))))
    assert _order(errs) > 1.8, errs
    assert _order(terrs) > 1.5, terrs


def test_neumann_bessel_solution_on_disk():
    """u = I0(sqrt(kappa) r): du/dn = sqrt(kappa) I1(sqrt(kappa) R) on r = R."""
    kappa, R = 100.0, 0.45
    k = np.sqrt(kappa)
    errs = []
    for M in (32, 64, 128):
        d = G.Domain(W.domains.disk(R, 1.0, M, M))
        gn = np.full(d.Nb, k * scipy.special.i1(k * R))
        U, _, _, _ = bie.neumann_solve(d, kappa, None, None, gn, tol=1e-12)
        ex = scipy.special.i0(k * np.hypot(d.X, d.Y))
        errs.append(np.max(np.abs(U - ex)[d.inside]) / np.max(np.abs(ex[d.inside])))
    assert _order(errs) > 1.8, errs


def test_neumann_star_second_order():
    """exp(3x + 4y) on the five-lobed star (kappa = 25): the error falls by
    more than 16 over two halvings of h (the single halvings vary)."""
    errs = []
    for M in (128, 256, 512):
        d = G.Domain(W.domains.star(0.5, 0.1, 5, 1.0, M, M))
        gn = _dn(mf.helm_exp_grad(d.colloc["x"], d.colloc["y"], 3.0, 4.0), d)
        U, _, _, _ = bie.neumann_solve(d, 25.0, None, None, gn, tol=1e-12)
        ex = mf.helm_exp_u(d.X, d.Y, 3.0, 4.0)
        errs.append(np.max(np.abs(U - ex)[d.inside]) / np.max(np.abs(ex[d.inside])))
    assert errs[0] / errs[-1] > 16.0, errs


@pytest.mark.parametrize("kappa", [64.0, 512j])
def test_neumann_with_source_second_order(kappa):
    """u = sin(pi x) cos(pi y), f = lap u - kappa u, du/dn on the star; real
    and imaginary kappa."""
    errs = []
    for M in (64, 128, 256):
        d = G.Domain(W.domain_c2_wave(M))
        zx, zy = d.colloc["x"], d.colloc["y"]
        U, _, _, st = bie.neumann_solve(d, kappa, mf.helm_trig_f(d.X, d.Y, kappa), mf.helm_trig_f(zx, zy, kappa),
                                        _dn(mf.helm_trig_grad(zx, zy), d), tol=1e-12)
        assert st["converged"]
        errs.append(np.max(np.abs(U - mf.helm_trig_u(d.X, d.Y))[d.inside]))
    assert _order(errs) > 1.5, errs
    assert errs[-1] < 2e-3


def test_neumann_richardson_reaches_gmres_density():
    """Eq. 3.22 (gamma = 1) converges to the GMRES density of the same K_N."""
    d = G.Domain(W.domains.star(0.5, 0.1, 5, 1.0, 64, 64))
    zx, zy = d.colloc["x"], d.colloc["y"]
    gn = _dn(mf.helm_exp_grad(zx, zy, 3.0, 4.0), d)
    _, p1, _, s1 = bie.neumann_solve(d, 25.0, None, None, gn, tol=1e-12)
    _, p2, _, s2 = bie.neumann_solve(d, 25.0, None, None, gn, tol=1e-11, solver="richardson", max_iter=2000)
    assert s1["converged"] and s2["converged"]
    assert np.max(np.abs(p1 - p2)) < 1e-8 * np.max(np.abs(p1))


def test_neumann_heat_steps_follow_exact_solution():
    """Crank-Nicolson with du/dn data: second order in (tau, h) together."""
    errs = []
    for M in (32, 64):
        desc = W.domains.disk(0.5, 1.0, M, M)
        d = G.Domain(desc)
        X, Y, zx, zy = d.X, d.Y, d.colloc["x"], d.colloc["y"]
        tau = 2.0 / M
        st = HeatStepper(d, tau, mf.heat_u(X, Y, 0), mf.heat_lap(X, Y, 0), mf.heat_u(zx, zy, 0),
                         mf.heat_lap(zx, zy, 0), tol=1e-12, bc="neumann")
        n = M // 8
        for k in range(n):
            U = st.step(_dn(mf.heat_grad(zx, zy, (k + 1) * tau), d), mf.heat_src(X, Y, k * tau)
                        + mf.heat_src(X, Y, (k + 1) * tau), mf.heat_src(zx, zy, k * tau)
                        + mf.heat_src(zx, zy, (k + 1) * tau))
        errs.append(np.max(np.abs(U - mf.heat_u(X, Y, n * tau))[d.inside]))
    assert errs[1] < errs[0] / 3.0, errs
    assert errs[1] < 1e-2, errs


def test_neumann_wave_steps_follow_exact_solution():
    """theta = 1/4 with du/dn data on the disk, tau = 4h (the stable range)."""
    errs = []
    for M in (32, 64):
        d = G.Domain(W.domains.disk(0.5, 1.0, M, M))
        X, Y, zx, zy = d.X, d.Y, d.colloc["x"], d.colloc["y"]
        tau = 4.0 * (2.0 / M)
        st = WaveStepper(d, tau, mf.wave_u(X, Y, 0), mf.wave_lap(X, Y, 0), mf.wave_u(zx, zy, 0),
                         mf.wave_lap(zx, zy, 0), mf.wave_u(X, Y, -tau), mf.wave_lap(X, Y, -tau),
                         mf.wave_u(zx, zy, -tau), mf.wave_lap(zx, zy, -tau), tol=1e-12, bc="neumann")
        n = M // 16
        for k in range(n):
            U = st.step(_dn(mf.wave_grad(zx, zy, (k + 1) * tau), d))
        errs.append(np.max(np.abs(U - mf.wave_u(X, Y, n * tau))[d.inside]))
    assert errs[1] < errs[0] / 3.0, errs
