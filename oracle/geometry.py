"""Oracle geometry (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

Follows Procedure 1 of the algorithm summary (section 3.3): discretise the
interface by quasi-uniform points, partition the box into a Cartesian grid
(section 3.2.4), identify regular / irregular nodes (section 3.2.4, the
definition after eq. 3.31) and find the intersections of Gamma with grid
lines.  The six-point extraction stencil of section 3.2.6 is built here too.

Readings taken (the paper is silent or the figure is missing):
  R5  inside <=> a fixed polynomial P(x, y) < 0, evaluated with +, -, * only,
      left to right, every operation rounded (numpy ufuncs never contract to
      FMA); a node exactly on Gamma counts as outside; the centre of a star
      counts as inside.
  R6  only the four five-point neighbours decide irregularity.
  R7  crossings by bisection of a smooth level function bracketed by the
      classification of the two end nodes.
  R12 stencil = nearest node c, c +- e_x, c +- e_y and the diagonal node
      c + s_x e_x + s_y e_y toward z.
"""

import numpy as np

TWO_PI = 2.0 * np.pi


class Curve:
    """Analytic counter-clockwise parametrisation gamma(theta) of Gamma."""

    def __init__(self, desc):
        self.kind = desc["kind"]
        self.cx = float(desc["cx"])
        self.cy = float(desc["cy"])
        self.R = float(desc["R"])
        self.a = float(desc["a"])
        self.b = float(desc["b"])
        self.r0 = float(desc["r0"])
        self.amp = float(desc["amp"])
        self.m = int(desc["lobes"])
        if self.kind not in ("disk", "ellipse", "star"):
            raise ValueError("unknown curve kind %r" % self.kind)

    # gamma, gamma', gamma'' -------------------------------------------------
    def derivs(self, th):
        """Return (g, g1, g2), each a pair of arrays: gamma and its first two
        theta-derivatives."""
        th = np.asarray(th, dtype=np.float64)
        c, s = np.cos(th), np.sin(th)
        if self.kind == "disk":
            R = self.R
            g = (self.cx + R * c, self.cy + R * s)
            g1 = (-R * s, R * c)
            g2 = (-R * c, -R * s)
        elif self.kind == "ellipse":
            a, b = self.a, self.b
            g = (self.cx + a * c, self.cy + b * s)
            g1 = (-a * s, b * c)
            g2 = (-a * c, -b * s)
        else:
            m = self.m
            r = self.r0 + self.amp * np.sin(m * th)
            r1 = self.amp * m * np.cos(m * th)
            r2 = -self.amp * m * m * np.sin(m * th)
            g = (self.cx + r * c, self.cy + r * s)
            g1 = (r1 * c - r * s, r1 * s + r * c)
            g2 = (r2 * c - 2.0 * r1 * s - r * c, r2 * s + 2.0 * r1 * c - r * s)
        return g, g1, g2

    def frame(self, th):
        """Geometry at parameter values th (section 3.2.5): point, speed
        sigma = |gamma'|, d sigma/d theta, unit tangent t, outward normal
        n = (t_y, -t_x) and dt/ds (s = arc length)."""
        g, g1, g2 = self.derivs(th)
        sig = np.sqrt(g1[0] * g1[0] + g1[1] * g1[1])
        tx, ty = g1[0] / sig, g1[1] / sig
        dsig = (g1[0] * g2[0] + g1[1] * g2[1]) / sig
        tg2 = tx * g2[0] + ty * g2[1]
        dtx = (g2[0] - tx * tg2) / (sig * sig)
        dty = (g2[1] - ty * tg2) / (sig * sig)
        return {"x": g[0], "y": g[1], "sigma": sig, "dsigma": dsig,
                "tx": tx, "ty": ty, "nx": ty, "ny": -tx, "dtx": dtx, "dty": dty}

    # smooth level function and parameter of a point on Gamma (R7) ---------
    def level(self, x, y):
        dx, dy = x - self.cx, y - self.cy
        if self.kind == "disk":
            return np.hypot(dx, dy) - self.R
        if self.kind == "ellipse":
            return (dx / self.a) ** 2 + (dy / self.b) ** 2 - 1.0
        th = np.arctan2(dy, dx)
        return np.hypot(dx, dy) - (self.r0 + self.amp * np.sin(self.m * th))

    def param(self, x, y):
        dx, dy = x - self.cx, y - self.cy
        if self.kind == "ellipse":
            th = np.arctan2(self.a * dy, self.b * dx)
        else:
            th = np.arctan2(dy, dx)
        return np.where(th < 0.0, th + TWO_PI, th)


def _powi(v, q):
    """v**q by repeated multiplication starting from 1 (R5)."""
    p = np.ones_like(v)
    for _ in range(q):
        p = p * v
    return p


def classify(desc, x, y):
    """Inside test of reading R5: True where the node is inside Omega.

    disk    (dx*dx + dy*dy) - R*R < 0
    ellipse (b*b)*(dx*dx) + (a*a)*(dy*dy) - (a*a)*(b*b) < 0
    star    rho < r0 + amp sin(m theta) rewritten without roots or
            transcendentals: with q = dx*dx + dy*dy and S = Im((dx+i dy)^m),
            odd m : A = q^((m+1)/2) - amp*S;  inside iff A < 0 or
                    A*A < (r0*r0)*q^m
            even m: C = r0*q^(m/2) + amp*S;   inside iff C > 0 and
                    q^(m+1) < C*C
            the centre itself is inside.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x - float(desc["cx"])
    dy = y - float(desc["cy"])
    kind = desc["kind"]
    if kind == "disk":
        R = float(desc["R"])
        return (dx * dx + dy * dy) - R * R < 0.0
    if kind == "ellipse":
        a, b = float(desc["a"]), float(desc["b"])
        return ((b * b) * (dx * dx) + (a * a) * (dy * dy)) - (a * a) * (b * b) < 0.0
    if kind != "star":
        raise ValueError(kind)
    r0, amp, m = float(desc["r0"]), float(desc["amp"]), int(desc["lobes"])
    q = dx * dx + dy * dy
    pr = np.ones_like(dx)
    pi = np.zeros_like(dx)
    for _ in range(m):
        pr, pi = pr * dx - pi * dy, pr * dy + pi * dx
    S = pi
    if m % 2 == 1:
        A = _powi(q, (m + 1) // 2) - amp * S
        inside = (A < 0.0) | (A * A < (r0 * r0) * _powi(q, m))
    else:
        C = r0 * _powi(q, m // 2) + amp * S
        inside = (C > 0.0) & (_powi(q, m + 1) < C * C)
    return inside | ((dx == 0.0) & (dy == 0.0))


class Domain:
    """Everything Procedure 1 sets up, for one descriptor.

    Grid arrays are indexed [j, i] (row j = y index, column i = x index);
    the linear index of node (i, j) is j*(M+1) + i.
    """

    def __init__(self, desc):
        self.desc = dict(desc)
        self.L = float(desc["L"])
        self.M = int(desc["M"])
        self.Nb = int(desc["Nb"])
        M, L = self.M, self.L
        self.h = (2.0 * L) / M
        self.x = -L + np.arange(M + 1, dtype=np.float64) * self.h
        self.y = self.x.copy()
        self.curve = Curve(desc)
        X, Y = np.meshgrid(self.x, self.y)          # X[j, i] = x_i
        self.X, self.Y = X, Y
        self.inside = classify(desc, X, Y)
        self._check_clearance()
        self._irregular()
        self._collocation()
        self._crossings()
        self._stencils()

    # Gamma must stay >= 3h away from the box boundary (R6) --------------
    def _check_clearance(self):
        M = self.M
        band = np.zeros_like(self.inside)
        band[:3, :] = band[-3:, :] = True
        band[:, :3] = band[:, -3:] = True
        if np.any(self.inside & band):
            raise ValueError("interface comes within 3h of the box boundary")
        th = np.linspace(0.0, TWO_PI, 4096, endpoint=False)
        g, _, _ = self.curve.derivs(th)
        lim = self.L - 3.0 * self.h
        if np.any(np.abs(g[0]) > lim) or np.any(np.abs(g[1]) > lim):
            raise ValueError("interface comes within 3h of the box boundary")
        del M

    # irregular nodes (section 3.2.4) ---------------------------------------
    def _irregular(self):
        ins = self.inside
        irr = np.zeros_like(ins)
        c = ins[1:-1, 1:-1]
        for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            nb = ins[1 + dj:ins.shape[0] - 1 + dj, 1 + di:ins.shape[1] - 1 + di]
            irr[1:-1, 1:-1] |= nb != c
        self.irregular = irr
        self.irr_index = np.flatnonzero(irr.ravel())      # sorted linear ids

    # collocation points (Procedure 1a) -------------------------------------
    def _collocation(self):
        Nb = self.Nb
        self.dtheta = TWO_PI / Nb
        self.theta = TWO_PI * np.arange(Nb, dtype=np.float64) / Nb
        self.colloc = self.curve.frame(self.theta)

    # grid-line crossings (Procedure 1d, reading R7) -----------------------
    def _crossings(self):
        ins, M = self.inside, self.M
        P, Q, axis = [], [], []
        # x-edges: (i, j) -- (i+1, j)
        jj, ii = np.nonzero(ins[:, :-1] != ins[:, 1:])
        P.append(jj * (M + 1) + ii)
        Q.append(jj * (M + 1) + ii + 1)
        axis.append(np.zeros(len(ii), dtype=np.int64))
        # y-edges: (i, j) -- (i, j+1)
        jj, ii = np.nonzero(ins[:-1, :] != ins[1:, :])
        P.append(jj * (M + 1) + ii)
        Q.append((jj + 1) * (M + 1) + ii)
        axis.append(np.ones(len(ii), dtype=np.int64))
        self.edge_p = np.concatenate(P)
        self.edge_q = np.concatenate(Q)
        self.edge_axis = np.concatenate(axis)
        xs, ys = self.X.ravel(), self.Y.ravel()
        insr = ins.ravel()
        pin = np.where(insr[self.edge_p], self.edge_p, self.edge_q)
        pout = np.where(insr[self.edge_p], self.edge_q, self.edge_p)
        lo_x, lo_y = xs[pin].copy(), ys[pin].copy()
        hi_x, hi_y = xs[pout].copy(), ys[pout].copy()
        for _ in range(64):                      # bisection to below one ulp
            mx, my = 0.5 * (lo_x + hi_x), 0.5 * (lo_y + hi_y)
            neg = self.curve.level(mx, my) < 0.0
            lo_x = np.where(neg, mx, lo_x)
            lo_y = np.where(neg, my, lo_y)
            hi_x = np.where(neg, hi_x, mx)
            hi_y = np.where(neg, hi_y, my)
        self.edge_X = 0.5 * (lo_x + hi_x)
        self.edge_Y = 0.5 * (lo_y + hi_y)
        self.edge_theta = self.curve.param(self.edge_X, self.edge_Y)
        self.edge_geom = self.curve.frame(self.edge_theta)

    # six-point extraction stencils (section 3.2.6, reading R12) ------------
    def _stencils(self):
        L, h, M, Nb = self.L, self.h, self.M, self.Nb
        zx, zy = self.colloc["x"], self.colloc["y"]
        ci = np.floor((zx + L) / h + 0.5).astype(np.int64)
        cj = np.floor((zy + L) / h + 0.5).astype(np.int64)
        sx = np.where(zx >= self.x[ci], 1, -1)
        sy = np.where(zy >= self.y[cj], 1, -1)
        di = np.stack([np.zeros_like(ci), np.ones_like(ci), -np.ones_like(ci),
                       np.zeros_like(ci), np.zeros_like(ci), sx], axis=1)
        dj = np.stack([np.zeros_like(cj), np.zeros_like(cj), np.zeros_like(cj),
                       np.ones_like(cj), -np.ones_like(cj), sy], axis=1)
        pi_ = ci[:, None] + di
        pj_ = cj[:, None] + dj
        self.st_node = pj_ * (M + 1) + pi_
        self.st_xi = self.x[pi_] - zx[:, None]
        self.st_eta = self.y[pj_] - zy[:, None]
        self.st_outside = ~self.inside[pj_, pi_]
        xi, eta = self.st_xi, self.st_eta
        A = np.stack([np.ones_like(xi), xi, eta, 0.5 * xi * xi, xi * eta,
                      0.5 * eta * eta], axis=2)               # (Nb, 6 nodes, 6)
        e0 = np.zeros((Nb, 6))
        e0[:, 0] = 1.0
        # U+(z) = e0^T A^{-1} U~  ->  weights w solve A^T w = e0
        self.st_weight = np.linalg.solve(np.transpose(A, (0, 2, 1)), e0[:, :, None])[:, :, 0]
        # the interior normal derivative n . (U_x+, U_y+) = (nx e1 + ny e2)^T
        # A^{-1} U~ (rows 1 and 2 of the same expansion; the Neumann problem)
        en = np.zeros((Nb, 6))
        en[:, 1] = self.colloc["nx"]
        en[:, 2] = self.colloc["ny"]
        self.st_weight_n = np.linalg.solve(np.transpose(A, (0, 2, 1)), en[:, :, None])[:, :, 0]
        del M, h

    def counts(self):
        return {"inside": int(self.inside.sum()),
                "irregular": int(self.irregular.sum()),
                "edges": int(len(self.edge_p))}
