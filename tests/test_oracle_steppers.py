"""Pins of the oracle time steppers (section 3.1): observed second-order
convergence against manufactured exact solutions, the closed-form
Schroedinger solution with V = 0, the Crank-Nicolson B-step identity (3.10),
the recurrences against the five-point Laplacian at regular nodes, and the
theta-stability behaviour of the paper's Table 3.
"""

import json
import os

import numpy as np
import pytest

import workloads as W
from workloads import manufactured as mf
from oracle import boxsolve
from oracle.geometry import Domain
from oracle.norms import max_norm
from oracle.steppers import HeatStepper, SchrodingerStepper, WaveStepper

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _order(errs):
    return np.log2(errs[0] / errs[-1]) / (len(errs) - 1)


def run_heat(M, T=0.3125):
    d = Domain(W.domain_c1_heat(M))
    tau = d.h
    n = int(round(T / tau))
    zx, zy = d.colloc["x"], d.colloc["y"]
    st = HeatStepper(d, tau, mf.heat_u(d.X, d.Y, 0), mf.heat_lap(d.X, d.Y, 0),
                     mf.heat_u(zx, zy, 0), mf.heat_lap(zx, zy, 0))
    for k in range(n):
        t0, t1 = k * tau, (k + 1) * tau
        U = st.step(mf.heat_u(zx, zy, t1),
                    mf.heat_src(d.X, d.Y, t0) + mf.heat_src(d.X, d.Y, t1),
                    mf.heat_src(zx, zy, t0) + mf.heat_src(zx, zy, t1))
    return d, st, U, max_norm(U - mf.heat_u(d.X, d.Y, n * tau), d.inside)


def test_heat_crank_nicolson_second_order():
    errs = [run_heat(M)[3] for M in (32, 64, 128)]
    assert _order(errs) > 1.8, errs
    with open(os.path.join(GOLDEN, "paper_convergence_rates.json")) as f:
        t1 = json.load(f)["table1_heat_dirichlet"]["err_inf"]
    paper_order = _order(t1)
    assert 1.8 < paper_order < 2.6 and abs(_order(errs) - 2.0) < 0.4


def test_heat_recurrence_matches_five_point_laplacian():
    """At regular inside nodes the grid solution satisfies the five-point
    equation exactly, so G = 2 kappa U - F equals kappa U + Delta_h U there."""
    d, st, U, _ = run_heat(32, T=2 * (2.0 / 32))
    lapU = np.zeros_like(U)
    lapU[1:-1, 1:-1] = boxsolve.apply(U[1:-1, 1:-1], d.h, 0.0)
    reg = d.inside & ~d.irregular
    ref = st.kappa * U + lapU
    assert np.max(np.abs(st.G - ref)[reg]) < 1e-9 * np.max(np.abs(ref[reg]))


def run_wave(desc, c, T, theta=0.25):
    d = Domain(desc)
    tau = c * d.h
    n = int(round(T / tau))
    zx, zy = d.colloc["x"], d.colloc["y"]
    st = WaveStepper(d, tau, mf.wave_u(d.X, d.Y, 0), mf.wave_lap(d.X, d.Y, 0),
                     mf.wave_u(zx, zy, 0), mf.wave_lap(zx, zy, 0),
                     mf.wave_u(d.X, d.Y, -tau), mf.wave_lap(d.X, d.Y, -tau),
                     mf.wave_u(zx, zy, -tau), mf.wave_lap(zx, zy, -tau), theta=theta)
    for k in range(n):
        U = st.step(mf.wave_u(zx, zy, (k + 1) * tau))
    return max_norm(U - mf.wave_u(d.X, d.Y, n * tau), d.inside)


def test_wave_theta_scheme_second_order():
    """Star domain, Nb = M (the paper's collocation count), tau = 4h."""
    errs = [run_wave(W.domain_c2_wave(M, Nb=M), 4.0, 0.5) for M in (64, 128, 256)]
    assert _order(errs) > 1.8, errs


@pytest.mark.slow
def test_wave_theta_stability_as_in_table3():
    """Unit circle in [-1.2,1.2]^2, 256 grid, tau = 0.0625, T = 1 (Table 3):
    theta = 0.2 diverges, theta = 0.25 and 0.5 stay accurate."""
    with open(os.path.join(GOLDEN, "paper_table3_theta_stability.json")) as f:
        paper = json.load(f)["T1"]
    desc = W.domains.disk(1.0, 1.2, 256, 256)
    h = 2.4 / 256
    c = 0.0625 / h
    e02 = run_wave(desc, c, 1.0, theta=0.2)
    e025 = run_wave(desc, c, 1.0, theta=0.25)
    e05 = run_wave(desc, c, 1.0, theta=0.5)
    # our manufactured solution has a faster time scale than the paper's
    # (unstated) one, so the stable errors are larger in absolute terms; the
    # pin is the qualitative split between theta < 1/4 and theta >= 1/4
    assert paper["0.2"] > 1.0 and e02 > 1.0
    assert paper["0.25"] < 1e-2 and e025 < 0.1
    assert paper["0.5"] < 1e-2 and e05 < 0.1
    assert e02 > 50.0 * max(e025, e05)


def run_schr_free(M, T=0.125):
    d = Domain(W.domain_c3_schrodinger(M))
    tau = d.h / 2
    n = int(round(T / tau))
    zx, zy = d.colloc["x"], d.colloc["y"]
    st = SchrodingerStepper(d, tau, mf.schr_free_u(d.X, d.Y, 0), mf.schr_free_lap(d.X, d.Y, 0),
                            mf.schr_free_u(zx, zy, 0), mf.schr_free_lap(zx, zy, 0),
                            np.zeros_like(d.X), np.zeros_like(zx))
    for k in range(n):
        U = st.step(mf.schr_free_u(zx, zy, (k + 1) * tau))
    return max_norm(U - mf.schr_free_u(d.X, d.Y, n * tau), d.inside)


def test_schrodinger_free_closed_form_second_order():
    """V = 0, w = 0 on the ellipse: u = exp(i 2 pi^2 t) sin(pi x) sin(pi y)."""
    errs = [run_schr_free(M) for M in (64, 128, 256)]
    assert _order(errs) > 1.8, errs
    assert errs[-1] < 1e-4


def test_schrodinger_b_step_solves_crank_nicolson_equation():
    """The closed-form B-step satisfies the Crank-Nicolson equation (3.10)
    u** + i tau/2 (v + w|u**|^2) u** = u* - i tau/2 (v + w|u*|^2) u*."""
    rng = np.random.default_rng(7)
    d = Domain(W.domains.ellipse(0.6, 0.4, 1.0, 16, 32))
    tau, w = 0.01, 1.0
    v = rng.uniform(0, 80, d.X.shape)
    st = SchrodingerStepper(d, tau, np.zeros_like(d.X), np.zeros_like(d.X),
                            np.zeros(d.Nb), np.zeros(d.Nb), v, np.zeros(d.Nb), w=w)
    us = rng.standard_normal(d.X.shape) + 1j * rng.standard_normal(d.X.shape)
    uss = st._b_step(us, v)
    lhs = uss + 0.5j * tau * (v + w * np.abs(uss) ** 2) * uss
    rhs = us - 0.5j * tau * (v + w * np.abs(us) ** 2) * us
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(rhs))
    assert np.allclose(np.abs(uss), np.abs(us), rtol=1e-14)


def test_nonlinear_schrodinger_example_second_order():
    """The paper's nonlinear example (w = 1, v of eq. 4.3, exact solution
    eq. 4.4) on the three-lobed star in [-pi, pi]^2 with its time steps
    tau = 8/M, to T = 1, against the paper's Table 4.  The example leaves
    the star parameter c unstated; with c = 0.2 the max-norm errors agree
    with the table's within 2% at M = 32, 64, 128 (1.244e-1, 3.268e-2,
    8.303e-3 against 1.23e-1, 3.26e-2, 8.27e-3).  A B-step without the cubic
    term misses the exact solution by about 0.5."""
    errs = []
    for M in (32, 64, 128):
        d = Domain(W.domain_nls_example(M))
        X, Y, zx, zy = d.X, d.Y, d.colloc["x"], d.colloc["y"]
        tau = 8.0 / M
        st = SchrodingerStepper(d, tau, mf.nls_u(X, Y, 0), mf.nls_lap(X, Y, 0), mf.nls_u(zx, zy, 0),
                                mf.nls_lap(zx, zy, 0), mf.nls_potential(X, Y), mf.nls_potential(zx, zy), w=1.0,
                                tol=1e-12)
        n = int(round(1.0 / tau))
        for k in range(n):
            U = st.step(mf.nls_u(zx, zy, (k + 1) * tau))
        errs.append(np.max(np.abs(U - mf.nls_u(X, Y, n * tau))[d.inside]))
    with open(os.path.join(GOLDEN, "paper_convergence_rates.json")) as f:
        t4 = json.load(f)["table4_schrodinger_dirichlet"]["err_inf"]
    assert 1.8 < _order(t4[:3]) < 2.2
    assert abs(_order(errs) - 2.0) < 0.4, errs
    for e, p in zip(errs, t4[:3]):
        assert abs(e / p - 1.0) < 0.05, (errs, t4)


def test_godunov_split_is_backward_euler_for_the_free_equation():
    """Godunov splitting with v = 0, w = 0 is the backward Euler step of
    (3.11) over tau: for the eigenfunction phi = sin(pi x) sin(pi y)
    (lap phi = -2 pi^2 phi) its discrete solution is rho^n phi with
    rho = 1 / (1 - 2 pi^2 i tau).  Fed that Dirichlet data, the stepper
    reproduces rho^n phi up to the O(h^2) space error; fed the exact data
    exp(i 2 pi^2 t) phi, its error halves with tau (first order in time)."""
    e_be, e_ex = [], []
    for M in (64, 128):
        d = Domain(W.domain_c3_schrodinger(M))
        tau = d.h / 2
        zx, zy = d.colloc["x"], d.colloc["y"]
        phi_g = np.sin(np.pi * d.X) * np.sin(np.pi * d.Y)
        phi_b = np.sin(np.pi * zx) * np.sin(np.pi * zy)
        rho = 1.0 / (1.0 - 2j * np.pi ** 2 * tau)
        n = int(round(0.125 / tau))
        for data, out in ((lambda k: rho ** k * phi_b, e_be), (lambda k: mf.schr_free_u(zx, zy, k * tau), e_ex)):
            st = SchrodingerStepper(d, tau, phi_g + 0j, -2 * np.pi ** 2 * phi_g, phi_b + 0j,
                                    -2 * np.pi ** 2 * phi_b, np.zeros_like(d.X), np.zeros_like(zx),
                                    split="godunov", tol=1e-12)
            for k in range(n):
                U = st.step(data(k + 1))
            exact = rho ** n * phi_g if out is e_be else mf.schr_free_u(d.X, d.Y, n * tau)
            out.append(max_norm(U - exact, d.inside))
    assert e_be[-1] < 5e-5 and e_be[0] / e_be[1] > 2.8, e_be
    assert 1.8 < e_ex[0] / e_ex[1] < 2.2, e_ex
    assert e_ex[-1] > 100 * e_be[-1]


def test_godunov_split_nonlinear_example_first_order():
    """The paper's nonlinear example (w = 1, v of eq. 4.3, exact solution
    eq. 4.4, tau = 8/M, T = 1) with Godunov splitting: the error falls at
    about first order (ratios 1.54 and 1.60 from M = 32 to 128, rising toward
    2), and it stays well above the Strang splitting's -- the ordering the
    paper's comparison example reports (Table 5)."""
    errs, strang = [], []
    for M in (32, 64, 128):
        d = Domain(W.domain_nls_example(M))
        X, Y, zx, zy = d.X, d.Y, d.colloc["x"], d.colloc["y"]
        tau = 8.0 / M
        n = int(round(1.0 / tau))
        for split, out in (("godunov", errs), ("strang", strang)):
            st = SchrodingerStepper(d, tau, mf.nls_u(X, Y, 0), mf.nls_lap(X, Y, 0), mf.nls_u(zx, zy, 0),
                                    mf.nls_lap(zx, zy, 0), mf.nls_potential(X, Y), mf.nls_potential(zx, zy),
                                    w=1.0, tol=1e-12, split=split)
            for k in range(n):
                U = st.step(mf.nls_u(zx, zy, (k + 1) * tau))
            out.append(max_norm(U - mf.nls_u(X, Y, n * tau), d.inside))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(1.4 < r < 2.2 for r in ratios), errs
    assert ratios[1] > ratios[0]
    assert all(g > 3.0 * s for g, s in zip(errs[1:], strang[1:])), (errs, strang)
