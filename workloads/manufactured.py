"""Manufactured exact solutions and initial data (problem data only).

Every function takes coordinate arrays x, y (any broadcastable shape) and
returns float64 / complex128 arrays.  Laplacians and gradients (the
`*_grad` functions, pairs (u_x, u_y) for Neumann data) are the analytic
ones.
"""

import numpy as np

PI = np.pi
SQRT2 = np.sqrt(2.0)


# ---- heat: u = exp(-t) sin(pi x) cos(pi y) with source s = u_t - lap u ----
def heat_u(x, y, t):
    return np.exp(-t) * np.sin(PI * x) * np.cos(PI * y)


def heat_lap(x, y, t):
    return -2.0 * PI * PI * heat_u(x, y, t)


def heat_grad(x, y, t):
    """(u_x, u_y), for Neumann data n . grad u."""
    e = np.exp(-t)
    return (PI * e * np.cos(PI * x) * np.cos(PI * y), -PI * e * np.sin(PI * x) * np.sin(PI * y))


def heat_src(x, y, t):
    """s = u_t - lap u = (2 pi^2 - 1) u."""
    return (2.0 * PI * PI - 1.0) * heat_u(x, y, t)


# ---- wave: u = cos(sqrt2 pi t) sin(pi x) sin(pi y), exact, no source -------
def wave_u(x, y, t):
    return np.cos(SQRT2 * PI * t) * np.sin(PI * x) * np.sin(PI * y)


def wave_lap(x, y, t):
    return -2.0 * PI * PI * wave_u(x, y, t)


def wave_grad(x, y, t):
    c = np.cos(SQRT2 * PI * t)
    return (PI * c * np.cos(PI * x) * np.sin(PI * y), PI * c * np.sin(PI * x) * np.cos(PI * y))


# ---- Schroedinger, i u_t = lap u + V u (w = 0) ------------------------------
def schr_free_u(x, y, t):
    """V = 0: u = exp(i 2 pi^2 t) sin(pi x) sin(pi y) solves i u_t = lap u."""
    return np.exp(1j * 2.0 * PI * PI * t) * np.sin(PI * x) * np.sin(PI * y)


def schr_free_lap(x, y, t):
    return -2.0 * PI * PI * schr_free_u(x, y, t)


def schr_free_grad(x, y, t):
    e = np.exp(1j * 2.0 * PI * PI * t)
    return (PI * e * np.cos(PI * x) * np.sin(PI * y), PI * e * np.sin(PI * x) * np.cos(PI * y))


# ---- nonlinear Schroedinger, w = 1 (the paper's Example 5) ----------------
def nls_potential(x, y):
    """v = 1 - cos^2 x cos^2 y (eq. 4.3)."""
    c = np.cos(x) * np.cos(y)
    return 1.0 - c * c


def nls_u(x, y, t):
    """exp(i t) cos x cos y (eq. 4.4): with v of eq. 4.3 and w = 1 it solves
    i u_t = lap u + v u + w |u|^2 u."""
    return np.exp(1j * t) * np.cos(x) * np.cos(y)


def nls_lap(x, y, t):
    return -2.0 * nls_u(x, y, t)


def packet_u0(x, y, width=0.1, k=(20.0, 0.0)):
    """Gaussian wave packet exp(-|x|^2/(2 w^2)) exp(i k.x), centred at 0."""
    s2 = width * width
    return np.exp(-(x * x + y * y) / (2.0 * s2)) * np.exp(1j * (k[0] * x + k[1] * y))


def packet_lap(x, y, width=0.1, k=(20.0, 0.0)):
    s2 = width * width
    ax = -x / s2 + 1j * k[0]
    ay = -y / s2 + 1j * k[1]
    return (ax * ax + ay * ay - 2.0 / s2) * packet_u0(x, y, width, k)


def harmonic_potential(x, y, strength=50.0):
    return strength * (x * x + y * y)


# ---- the Neumann wave example: a radial logistic bump at rest ----------------
def logistic_u0(x, y, r1=0.5, k=20.0):
    """1 / (1 + exp(k (r - r1))), r = |(x, y)|."""
    return 1.0 / (1.0 + np.exp(k * (np.hypot(x, y) - r1)))


def logistic_lap(x, y, r1=0.5, k=20.0, r_min=1e-3):
    """u'' + u'/r of the bump, with r >= r_min in the 1/r term (the bump has
    slope -k u (1 - u) ~ 1e-3 at r = 0, a kink whose Laplacian is
    unbounded there)."""
    u = logistic_u0(x, y, r1, k)
    d1 = -k * u * (1.0 - u)
    d2 = k * k * u * (1.0 - u) * (1.0 - 2.0 * u)
    return d2 + d1 / np.maximum(np.hypot(x, y), r_min)


# ---- modified Helmholtz BVP solutions (lap u - kappa u = f) -----------------
def helm_exp_u(x, y, a, b):
    """exp(a x + b y): lap u - kappa u = 0 when a^2 + b^2 = kappa."""
    return np.exp(a * x + b * y)


def helm_exp_grad(x, y, a, b):
    u = np.exp(a * x + b * y)
    return (a * u, b * u)


def helm_trig_u(x, y):
    return np.sin(PI * x) * np.cos(PI * y)


def helm_trig_grad(x, y):
    return (PI * np.cos(PI * x) * np.cos(PI * y), -PI * np.sin(PI * x) * np.sin(PI * y))


def helm_trig_f(x, y, kappa):
    """f = lap u - kappa u for u = sin(pi x) cos(pi y)."""
    return -(2.0 * PI * PI + kappa) * helm_trig_u(x, y)
