"""Domain descriptors of the synthetic workloads.

A descriptor is a plain dict:

    kind    "disk" | "ellipse" | "star"
    cx, cy  centre of the curve
    R       disk radius
    a, b    ellipse semi-axes (x, y)
    r0, amp, lobes   star r(theta) = r0 + amp*sin(lobes*theta)
    L       the bounding box is [-L, L]^2
    M       number of grid intervals per axis (nodes 0..M)
    Nb      number of boundary collocation points

The shapes and sizes follow the workloads the method is measured on: a disk
of radius 0.5 with a 64-interval grid and 128 points (heat), a five-lobed
star 0.5+0.1 sin 5t on a 512 grid (wave), an ellipse 0.6/0.4 on a 1024 grid
(Schroedinger) and seeded random stars for the batched Helmholtz instances.
Apart from the heat disk, the collocation count is the paper's Nb = M
(section 4): with Nb = 2M the boundary is sampled finer than the grid
resolves, the discrete integral operator gains near-null high-frequency
modes, GMRES needs 3-40x more iterations and the theta = 1/4 wave
recurrence diverges.
"""

import numpy as np

BASE_SEED = 20240423


def grid_coords(L, M):
    """Node coordinates -L + i*h, h = 2L/M, i = 0..M (each op rounded)."""
    h = (2.0 * L) / M
    return -L + np.arange(M + 1, dtype=np.float64) * h


def _desc(kind, L, M, Nb, **kw):
    d = {"kind": kind, "cx": 0.0, "cy": 0.0, "R": 0.0, "a": 0.0, "b": 0.0,
         "r0": 0.0, "amp": 0.0, "lobes": 0, "L": float(L), "M": int(M),
         "Nb": int(Nb)}
    d.update(kw)
    return d


def disk(R, L, M, Nb, cx=0.0, cy=0.0):
    return _desc("disk", L, M, Nb, R=float(R), cx=float(cx), cy=float(cy))


def ellipse(a, b, L, M, Nb, cx=0.0, cy=0.0):
    return _desc("ellipse", L, M, Nb, a=float(a), b=float(b), cx=float(cx),
                 cy=float(cy))


def star(r0, amp, lobes, L, M, Nb, cx=0.0, cy=0.0):
    return _desc("star", L, M, Nb, r0=float(r0), amp=float(amp),
                 lobes=int(lobes), cx=float(cx), cy=float(cy))


def domain_c1_heat(M=64, Nb=None):
    """Disk of radius 0.5 in [-1,1]^2; 2M collocation points."""
    return disk(0.5, 1.0, M, 2 * M if Nb is None else Nb)


def domain_c2_wave(M=512, Nb=None):
    """Star r = 0.5 + 0.1 sin(5 theta) in [-1,1]^2; M collocation points
    (the paper's count, section 4) unless Nb is given."""
    return star(0.5, 0.1, 5, 1.0, M, M if Nb is None else Nb)


def domain_c3_schrodinger(M=1024, Nb=None):
    """Ellipse with semi-axes 0.6 / 0.4 in [-1,1]^2; M collocation points
    unless Nb is given."""
    return ellipse(0.6, 0.4, 1.0, M, M if Nb is None else Nb)


def domain_neumann_wave(M=512, Nb=None):
    """The eight-lobed star of the paper's Neumann wave example, r = 0.8 +
    0.2 sin(8 theta) (the example's (1-c) + c cos(8 theta), c = 0.2, turned
    by pi/16), in [-1.5, 1.5]^2; M collocation points unless Nb is given."""
    return star(0.8, 0.2, 8, 1.5, M, M if Nb is None else Nb)


def domain_nls_example(M=256, Nb=None):
    """The three-lobed star of the paper's nonlinear Schroedinger example,
    r = 1.2 + 0.3 sin(3 theta) (its 1.5[(1-c) + c cos(3 theta)] with c = 0.2,
    which the example leaves unstated, turned by pi/6), in [-pi, pi]^2; M
    collocation points unless Nb is given."""
    return star(1.2, 0.3, 3, np.pi, M, M if Nb is None else Nb)


def domain_c4_instance(index, grids=(128, 256, 512, 1024)):
    """One seeded batched-Helmholtz instance.

    Returns (descriptor, kappa, rng) where rng continues the instance's
    PCG64 stream (used for its random right-hand side and boundary data).
    Star radius r0 ~ U[0.3, 0.6], lobes ~ U{3..8}, amp = 0.2 r0,
    kappa ~ U[1, 1e4], M uniform over `grids`, Nb = M.
    """
    rng = np.random.default_rng(BASE_SEED + int(index))
    M = int(grids[rng.integers(0, len(grids))])
    r0 = float(rng.uniform(0.3, 0.6))
    lobes = int(rng.integers(3, 9))
    kappa = float(rng.uniform(1.0, 1.0e4))
    return star(r0, 0.2 * r0, lobes, 1.0, M, M), kappa, rng
