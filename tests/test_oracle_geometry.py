"""Pins of the oracle geometry: classification (reading R5) against exact
integer / rational arithmetic, irregular nodes (section 3.2.4) by brute
force, crossings against closed forms, the curve frame against the circle's
closed form, and the six-point extraction weights (section 3.2.6) against
exact reproduction of quadratics.
"""

from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G


def test_c1_disk_classification_exact_integers():
    """Disk R = 1/2 on the 64-interval grid of [-1,1]^2: every coordinate is
    k/32 exactly, so inside <=> (i-32)^2 + (j-32)^2 < 16^2 in integers (a
    node on the circle counts as outside)."""
    d = G.Domain(W.domain_c1_heat())
    M = d.M
    exact = np.zeros((M + 1, M + 1), dtype=bool)
    on_gamma = 0
    for j in range(M + 1):
        for i in range(M + 1):
            v = (i - 32) ** 2 + (j - 32) ** 2 - 256
            exact[j, i] = v < 0
            on_gamma += v == 0
    assert np.array_equal(d.inside, exact)
    assert on_gamma == 4
    # irregular nodes and crossing edges by brute force on the exact classes
    irr = 0
    for j in range(1, M):
        for i in range(1, M):
            c = exact[j, i]
            if any(exact[j + dj, i + di] != c for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0))):
                irr += 1
    edges = sum(exact[j, i] != exact[j, i + 1] for j in range(M + 1) for i in range(M)) + \
        sum(exact[j, i] != exact[j + 1, i] for j in range(M) for i in range(M + 1))
    assert d.counts() == {"inside": int(exact.sum()), "irregular": irr, "edges": edges}
    assert d.counts() == {"inside": 793, "irregular": 180, "edges": 124}


def _poly_exact(desc, x, y):
    """The R5 polynomial in exact rational arithmetic of the double inputs;
    returns its sign convention: True = inside."""
    X, Y = Fraction(x) - Fraction(desc["cx"]), Fraction(y) - Fraction(desc["cy"])
    if desc["kind"] == "ellipse":
        a, b = Fraction(desc["a"]), Fraction(desc["b"])
        return b * b * X * X + a * a * Y * Y - a * a * b * b < 0
    r0, amp, m = Fraction(desc["r0"]), Fraction(desc["amp"]), desc["lobes"]
    if X == 0 and Y == 0:
        return True
    q = X * X + Y * Y
    pr, pi = Fraction(1), Fraction(0)
    for _ in range(m):
        pr, pi = pr * X - pi * Y, pr * Y + pi * X
    if m % 2:
        A = q ** ((m + 1) // 2) - amp * pi
        return A < 0 or A * A < r0 * r0 * q ** m
    C = r0 * q ** (m // 2) + amp * pi
    return C > 0 and q ** (m + 1) < C * C


@pytest.mark.parametrize("desc", [
    W.domain_c2_wave(128),
    W.domains.star(0.45, 0.09, 4, 1.0, 128, 256),
    W.domains.star(0.4, 0.08, 7, 1.0, 96, 192),
    W.domain_c3_schrodinger(128),
])
def test_classification_matches_exact_rational_and_geometry(desc):
    d = G.Domain(desc)
    # nodes within two cells of Gamma: exact rational sign of the same polynomial
    lev = d.curve.level(d.X, d.Y)
    near = np.argwhere(np.abs(lev) < 2.0 * d.h)
    assert len(near) > 50
    for j, i in near:
        assert d.inside[j, i] == _poly_exact(desc, d.x[i], d.y[j]), (i, j)
    # away from Gamma the polynomial test is the geometric test rho < r(theta)
    far = np.abs(lev) > 1e-9
    assert np.array_equal(d.inside[far], (lev < 0)[far])


def test_star_centre_is_inside():
    desc = W.domains.star(0.5, 0.1, 5, 1.0, 32, 64)
    assert bool(G.classify(desc, np.array([0.0]), np.array([0.0]))[0])
    desc = W.domains.star(0.5, 0.1, 4, 1.0, 32, 64)
    assert bool(G.classify(desc, np.array([0.0]), np.array([0.0]))[0])


def test_irregular_nodes_brute_force_star():
    d = G.Domain(W.domain_c2_wave(64))
    M = d.M
    expect = np.zeros_like(d.inside)
    for j in range(1, M):
        for i in range(1, M):
            c = d.inside[j, i]
            for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                if d.inside[j + dj, i + di] != c:
                    expect[j, i] = True
    assert np.array_equal(d.irregular, expect)
    assert np.array_equal(d.irr_index, np.flatnonzero(expect.ravel()))


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domains.disk(0.47, 1.0, 128, 256),
                                  W.domain_c3_schrodinger(128)])
def test_crossings_closed_form(desc):
    d = G.Domain(desc)
    for e in range(len(d.edge_p)):
        X, Y = d.edge_X[e], d.edge_Y[e]
        if desc["kind"] == "disk":
            R = desc["R"]
            if d.edge_axis[e] == 0:
                ref = np.sign(X) * np.sqrt(R * R - Y * Y)
                assert abs(X - ref) < 1e-14
            else:
                ref = np.sign(Y) * np.sqrt(R * R - X * X)
                assert abs(Y - ref) < 1e-14
        else:
            a, b = desc["a"], desc["b"]
            if d.edge_axis[e] == 0:
                ref = np.sign(X) * a * np.sqrt(1.0 - (Y / b) ** 2)
                assert abs(X - ref) < 1e-14
            else:
                ref = np.sign(Y) * b * np.sqrt(1.0 - (X / a) ** 2)
                assert abs(Y - ref) < 1e-14
        # the crossing lies between its two nodes
        xs, ys = d.X.ravel(), d.Y.ravel()
        p, q = d.edge_p[e], d.edge_q[e]
        if d.edge_axis[e] == 0:
            assert min(xs[p], xs[q]) <= X <= max(xs[p], xs[q]) and ys[p] == Y
        else:
            assert min(ys[p], ys[q]) <= Y <= max(ys[p], ys[q]) and xs[p] == X


def test_circle_frame_closed_form():
    R = 0.5
    c = G.Curve(W.domains.disk(R, 1.0, 16, 32))
    th = np.linspace(0, 2 * np.pi, 17)
    f = c.frame(th)
    assert np.allclose(f["tx"], -np.sin(th)) and np.allclose(f["ty"], np.cos(th))
    assert np.allclose(f["nx"], np.cos(th)) and np.allclose(f["ny"], np.sin(th))  # outward
    assert np.allclose(f["dtx"], -np.cos(th) / R) and np.allclose(f["dty"], -np.sin(th) / R)
    assert np.allclose(f["sigma"], R) and np.allclose(f["dsigma"], 0.0)


def test_star_frame_against_finite_differences():
    c = G.Curve(W.domain_c2_wave(64))
    th = np.linspace(0.1, 6.0, 9)
    e = 1e-5
    g0, g1, g2 = c.derivs(th)
    gp, _, _ = c.derivs(th + e)
    gm, _, _ = c.derivs(th - e)
    assert np.allclose((gp[0] - gm[0]) / (2 * e), g1[0], atol=1e-8)
    assert np.allclose((gp[1] - gm[1]) / (2 * e), g1[1], atol=1e-8)
    _, g1p, _ = c.derivs(th + e)
    _, g1m, _ = c.derivs(th - e)
    assert np.allclose((g1p[0] - g1m[0]) / (2 * e), g2[0], atol=1e-6)
    f, fp, fm = c.frame(th), c.frame(th + e), c.frame(th - e)
    ds = f["sigma"] * 2 * e
    assert np.allclose((fp["tx"] - fm["tx"]) / ds, f["dtx"], atol=1e-5)
    assert np.allclose((fp["sigma"] - fm["sigma"]) / (2 * e), f["dsigma"], atol=1e-6)


@pytest.mark.parametrize("desc", [W.domain_c1_heat(64), W.domain_c2_wave(128)])
def test_extraction_weights_reproduce_quadratics(desc, rng):
    d = G.Domain(desc)
    for _ in range(3):
        cf = rng.standard_normal(6)

        def q(x, y):
            return cf[0] + cf[1] * x + cf[2] * y + cf[3] * x * x + cf[4] * x * y + cf[5] * y * y
        vals = q(d.X.ravel()[d.st_node], d.Y.ravel()[d.st_node])
        got = np.sum(d.st_weight * vals, axis=1)
        ref = q(d.colloc["x"], d.colloc["y"])
        assert np.max(np.abs(got - ref)) < 1e-12
    # stencil shape: nearest node, its four neighbours and the diagonal toward z
    k = 5
    nodes = d.st_node[k]
    M = d.M
    ci, cj = nodes[0] % (M + 1), nodes[0] // (M + 1)
    assert abs(d.x[ci] - d.colloc["x"][k]) <= d.h / 2 + 1e-15
    assert abs(d.y[cj] - d.colloc["y"][k]) <= d.h / 2 + 1e-15
    offs = {(n % (M + 1) - ci, n // (M + 1) - cj) for n in nodes}
    assert {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)} <= offs and len(offs) == 6


def test_domain_too_close_to_box_is_rejected():
    with pytest.raises(ValueError):
        G.Domain(W.domains.disk(0.97, 1.0, 64, 128))
