"""Pins of the oracle interface solve: the jump relations of section 3.2.5
against analytic jumps, the corrections of section 3.2.4 against an exact
identity for piecewise quadratics, and the extraction of section 3.2.6
against exact recovery of a quadratic's interior limit.
"""

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import interface as I

A_, B_ = 1.3, -0.7          # u+ = exp(a x + b y), u- = 0


def _exp_case(d, th, kappa):
    """Analytic density, its theta-derivatives, psi = [u_n], psi_theta and
    f+ for u+ = exp(ax+by), u- = 0, at curve parameters th."""
    c = d.curve
    g, g1, g2 = c.derivs(th)
    fr = c.frame(th)
    e = np.exp(A_ * g[0] + B_ * g[1])
    lin1 = A_ * g1[0] + B_ * g1[1]
    lin2 = A_ * g2[0] + B_ * g2[1]
    phi, phi_t, phi_tt = e, lin1 * e, (lin1 * lin1 + lin2) * e
    dn = A_ * fr["nx"] + B_ * fr["ny"]
    dn_t = fr["sigma"] * (A_ * fr["dty"] - B_ * fr["dtx"])
    psi, psi_t = dn * e, dn_t * e + dn * phi_t
    f = (A_ * A_ + B_ * B_ - kappa) * e
    ref = {"u": e, "ux": A_ * e, "uy": B_ * e, "uxx": A_ * A_ * e,
           "uxy": A_ * B_ * e, "uyy": B_ * B_ * e}
    return phi, phi_t, phi_tt, psi, psi_t, f, fr, ref


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domain_c2_wave(64),
                                  W.domain_c3_schrodinger(64)])
@pytest.mark.parametrize("kappa", [0.0, 64.0])
def test_jump_relations_exact_with_exact_derivatives(desc, kappa):
    """Given exact phi, phi_theta, phi_thetatheta, psi, psi_theta and f,
    eq. (3.35) and the 3x3 system return the exact jumps."""
    d = G.Domain(desc)
    th = np.linspace(0.0, 2 * np.pi, 37)
    phi, phi_t, phi_tt, psi, psi_t, f, fr, ref = _exp_case(d, th, kappa)
    got = I.jumps(fr, phi, phi_t, phi_tt, f, kappa, psi, psi_t)
    for k in ref:
        assert np.max(np.abs(got[k] - ref[k])) < 1e-12 * np.max(np.abs(ref[k])) + 1e-13, k


def test_jumps_at_crossings_converge_fourth_order():
    """With only the collocation samples of phi, psi and f, the finite
    differences and cubic interpolation of reading R10 give the crossing
    jumps with an error falling ~16x per doubling of Nb."""
    errs = []
    for Nb in (128, 256, 512):
        d = G.Domain(W.domains.star(0.5, 0.1, 5, 1.0, 64, Nb))
        phi, _, _, psi, _, f, _, _ = _exp_case(d, d.theta, 10.0)
        bd = I.boundary_data(d, phi, f, psi)
        je = I.jumps_at_crossings(d, 10.0, bd)
        _, _, _, _, _, _, _, ref = _exp_case(d, d.edge_theta, 10.0)
        errs.append(max(np.max(np.abs(je[k] - ref[k])) / np.max(np.abs(ref[k])) for k in ref))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 8.0 and errs[1] / errs[2] > 8.0


def test_theta_derivatives_fourth_order():
    for N in (64, 128):
        th = 2 * np.pi * np.arange(N) / N
        v = np.exp(np.sin(3 * th))
        d1, d2 = I.theta_derivs(v, 2 * np.pi / N)
        r1 = 3 * np.cos(3 * th) * v
        r2 = (-9 * np.sin(3 * th) + 9 * np.cos(3 * th) ** 2) * v
        if N == 64:
            e1, e2 = np.max(np.abs(d1 - r1)), np.max(np.abs(d2 - r2))
        else:
            assert e1 / np.max(np.abs(d1 - r1)) > 12 and e2 / np.max(np.abs(d2 - r2)) > 12


def test_lagrange_exact_for_cubic_trig_free_samples():
    """Cubic interpolation reproduces a cubic in theta exactly (away from the
    periodic wrap)."""
    N = 64
    dth = 2 * np.pi / N
    th = dth * np.arange(N)
    cub = 0.3 - 0.2 * th + 0.05 * th ** 2 - 0.004 * th ** 3
    ts = np.array([1.05, 2.2, 3.9001, 4.5])
    got, = I.lagrange_at(ts, dth, [cub])
    ref = 0.3 - 0.2 * ts + 0.05 * ts ** 2 - 0.004 * ts ** 3
    assert np.max(np.abs(got - ref)) < 1e-13


# ---- corrections: exact identity for piecewise quadratics -------------------
QP = np.array([1.0, 0.3, -0.2, 0.5, -0.7, 0.4])       # u+ coefficients
QJ = np.array([0.2, -0.1, 0.3, 0.25, 0.6, -0.35])     # u+ - u- (quadratic)


def _q(c, x, y):
    return c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domain_c2_wave(128),
                                  W.domain_c3_schrodinger(96)])
def test_corrected_five_point_equation_exact_for_quadratics(desc):
    """If u+ and u- are quadratics whose difference is a quadratic, the
    Taylor jump term J is exact, so at every interior node
        Delta_h U = lap u(+/-) + C
    holds to rounding, with C the correction of reading R8."""
    d = G.Domain(desc)
    X, Y = d.X, d.Y
    U = np.where(d.inside, _q(QP, X, Y), _q(QP, X, Y) - _q(QJ, X, Y))
    ex, ey = d.edge_X, d.edge_Y
    je = {"u": _q(QJ, ex, ey),
          "ux": QJ[1] + 2 * QJ[3] * ex + QJ[4] * ey,
          "uy": QJ[2] + QJ[4] * ex + 2 * QJ[5] * ey,
          "uxx": np.full_like(ex, 2 * QJ[3]), "uxy": np.full_like(ex, QJ[4]),
          "uyy": np.full_like(ex, 2 * QJ[5])}
    C = I.corrections(d, je)
    h = d.h
    lapP = 2 * QP[3] + 2 * QP[5]
    lapM = lapP - (2 * QJ[3] + 2 * QJ[5])
    lhs = (U[1:-1, 2:] + U[1:-1, :-2] + U[2:, 1:-1] + U[:-2, 1:-1] - 4 * U[1:-1, 1:-1]) / h ** 2
    rhs = np.where(d.inside, lapP, lapM)[1:-1, 1:-1] + C[1:-1, 1:-1]
    assert np.max(np.abs(lhs - rhs)) < 1e-9 / h ** 2 * 1e-3
    # corrections vanish away from irregular nodes
    assert np.all(C[~d.irregular] == 0.0)
    assert np.count_nonzero(C) == np.count_nonzero(d.irregular)


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domain_c2_wave(128)])
def test_extraction_exact_for_quadratics(desc):
    """Grid values of u+ inside and u- = u+ - jq outside, with the exact
    quadratic jumps at z: the extracted U+(z) equals u+(z) to rounding."""
    d = G.Domain(desc)
    X, Y = d.X, d.Y
    U = np.where(d.inside, _q(QP, X, Y), _q(QP, X, Y) - _q(QJ, X, Y))
    zx, zy = d.colloc["x"], d.colloc["y"]
    jz = {"u": _q(QJ, zx, zy),
          "ux": QJ[1] + 2 * QJ[3] * zx + QJ[4] * zy,
          "uy": QJ[2] + QJ[4] * zx + 2 * QJ[5] * zy,
          "uxx": np.full_like(zx, 2 * QJ[3]), "uxy": np.full_like(zx, QJ[4]),
          "uyy": np.full_like(zx, 2 * QJ[5])}
    got = I.extract(d, U, jz)
    assert np.max(np.abs(got - _q(QP, zx, zy))) < 1e-12


def test_interface_solve_is_affine():
    """IS(f, phi) = IS(f, 0) + IS(0, phi) (the BIE split of reading R2)."""
    d = G.Domain(W.domain_c2_wave(64))
    rng = np.random.default_rng(3)
    kappa = 40.0
    f = rng.standard_normal(d.X.shape)
    fg = rng.standard_normal(d.Nb)
    phi = np.cos(3 * d.theta) + 0.1 * rng.standard_normal(d.Nb)
    U1, P1 = I.interface_solve(d, kappa, f, fg, phi)
    U2, P2 = I.interface_solve(d, kappa, f, fg, np.zeros(d.Nb))
    U3, P3 = I.interface_solve(d, kappa, None, None, phi)
    assert np.max(np.abs(U1 - U2 - U3)) < 1e-12 * np.max(np.abs(U1))
    assert np.max(np.abs(P1 - P2 - P3)) < 1e-12 * np.max(np.abs(P1))
