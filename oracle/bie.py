"""Oracle Dirichlet and Neumann BVP solves through the boundary integral
equations (TEST INFRASTRUCTURE ONLY).

For lap u - kappa u = f in Omega, u = g on Gamma (eq. 3.13), the density
phi of the double-layer potential solves the second-kind equation (3.17),
1/2 phi + W phi + Y f = g, and u = W phi + Y f (eq. 3.18).  Each of W phi
and Y f is the solution of an interface problem (3.24)/(3.27), so with
IS(f, phi) the interface solve of oracle.interface (reading R2):

    K v  = IS(0, v).U^+           (the discrete 1/2 I + W at Gamma)
    b    = g - IS(f, 0).U^+
    phi  = GMRES(K, b)            (reading R1)
    U    = IS(f, phi).U            on the grid; u = U at inside nodes.
"""

import numpy as np

from . import gmres as _gmres
from . import richardson as _richardson
from .interface import interface_solve


def matvec(dom, kappa, v):
    return interface_solve(dom, kappa, None, None, v)[1]


def rhs(dom, kappa, f_grid, f_gamma, g):
    if f_grid is None:
        return np.asarray(g).copy()
    return g - interface_solve(dom, kappa, f_grid, f_gamma,
                               np.zeros(dom.Nb, dtype=np.result_type(g, f_gamma, kappa)))[1]


def dense_operator(dom, kappa):
    """K assembled column by column (small Nb only)."""
    dtype = np.complex128 if np.iscomplexobj(kappa) else np.float64
    K = np.zeros((dom.Nb, dom.Nb), dtype=dtype)
    for k in range(dom.Nb):
        e = np.zeros(dom.Nb, dtype=dtype)
        e[k] = 1.0
        K[:, k] = matvec(dom, kappa, e)
    return K


def helmholtz_solve(dom, kappa, f_grid, f_gamma, g, phi0=None, tol=1e-10,
                    restart=50, max_iter=500, fixed_iters=None, solver="gmres", gamma=1.0):
    """Solve the Dirichlet problem.  Returns (U, phi, stats).  solver:
    "gmres" (reading R1) or "richardson" (eq. 3.21 with parameter gamma)."""
    cplx = any(np.iscomplexobj(v) for v in (kappa, f_grid, f_gamma, g, phi0)
               if v is not None)
    dtype = np.complex128 if cplx else np.float64
    g = np.asarray(g, dtype=dtype)
    b = rhs(dom, kappa, f_grid, f_gamma, g)
    if solver == "richardson":
        phi, iters, rel, conv = _richardson.richardson(
            lambda v: matvec(dom, kappa, v), b, phi0, gamma=gamma, tol=tol,
            max_iter=max_iter, fixed_iters=fixed_iters)
    else:
        phi, iters, rel, conv = _gmres.gmres(
            lambda v: matvec(dom, kappa, v), b, phi0, tol=tol, restart=restart,
            max_iter=max_iter, fixed_iters=fixed_iters)
    U, _ = interface_solve(dom, kappa, f_grid, f_gamma, phi)
    return U, phi, {"iters": iters, "rel_resid": rel, "converged": conv}


# ---- the Neumann problem ---------------------------------------------------
# lap u - kappa u = f in Omega, du/dn = g_N on Gamma (n outward).  The density
# psi of u = Yf - V psi (eq. 3.20) solves (3.19),
#     1/2 psi - d/dn (V psi) + d/dn (Yf) = g_N.
# -V psi is the interface problem (3.29) with [u_n] = psi (the table after
# eq. 3.30), whose interior normal derivative on Gamma is 1/2 psi - d/dn(V psi)
# (the jump [u_n] = psi split evenly about the direct value), and Yf is C^1
# across Gamma.  So with IS(f, phi, psi) the interface solve:
#     K_N v = IS(0, 0, v).dU+/dn,   b = g_N - IS(f, 0, 0).dU+/dn,
#     psi = GMRES(K_N, b),          U = IS(f, 0, psi).U.

def neumann_matvec(dom, kappa, v):
    v = np.asarray(v)
    return interface_solve(dom, kappa, None, None, np.zeros(dom.Nb, dtype=v.dtype), psi=v, normal=True)[2]


def neumann_rhs(dom, kappa, f_grid, f_gamma, gn):
    gn = np.asarray(gn)
    if f_grid is None:
        return gn.copy()
    zero = np.zeros(dom.Nb, dtype=np.result_type(gn, f_gamma, kappa))
    return gn - interface_solve(dom, kappa, f_grid, f_gamma, zero, normal=True)[2]


def neumann_dense_operator(dom, kappa):
    """K_N assembled column by column (small Nb only)."""
    dtype = np.complex128 if np.iscomplexobj(kappa) else np.float64
    K = np.zeros((dom.Nb, dom.Nb), dtype=dtype)
    for k in range(dom.Nb):
        e = np.zeros(dom.Nb, dtype=dtype)
        e[k] = 1.0
        K[:, k] = neumann_matvec(dom, kappa, e)
    return K


def neumann_solve(dom, kappa, f_grid, f_gamma, gn, psi0=None, tol=1e-10,
                  restart=50, max_iter=500, fixed_iters=None, solver="gmres", gamma=1.0):
    """Solve the Neumann problem.  Returns (U, psi, Uplus, stats): the grid
    solution, the density, the interior limit U+ at the collocation points
    (the trace of u on Gamma) and the iteration statistics.  solver: "gmres"
    (reading R1) or "richardson" (eq. 3.22 with parameter gamma)."""
    cplx = any(np.iscomplexobj(v) for v in (kappa, f_grid, f_gamma, gn, psi0)
               if v is not None)
    dtype = np.complex128 if cplx else np.float64
    gn = np.asarray(gn, dtype=dtype)
    b = neumann_rhs(dom, kappa, f_grid, f_gamma, gn)
    op = lambda v: neumann_matvec(dom, kappa, v)  # noqa: E731
    if solver == "richardson":
        psi, iters, rel, conv = _richardson.richardson(op, b, psi0, gamma=gamma, tol=tol, max_iter=max_iter,
                                                       fixed_iters=fixed_iters)
    else:
        psi, iters, rel, conv = _gmres.gmres(op, b, psi0, tol=tol, restart=restart, max_iter=max_iter,
                                             fixed_iters=fixed_iters)
    U, Uplus = interface_solve(dom, kappa, f_grid, f_gamma, np.zeros(dom.Nb, dtype=dtype), psi=psi)
    return U, psi, Uplus, {"iters": iters, "rel_resid": rel, "converged": conv}
