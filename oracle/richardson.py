"""Oracle Richardson iteration for the second-kind equation
(TEST INFRASTRUCTURE ONLY).

Section 3.2 solves 1/2 phi + W phi + Y f = g (eq. 3.17) by the Richardson
iteration of eq. 3.21,

    phi_{k+1} = (1 - gamma/2) phi_k + gamma [g - Y f - W phi_k],

with gamma in (0, 1) and an arbitrary initial density (the step list of
Procedure 3).  Here the discrete operators come as K = 1/2 I + W (a
function applying it) and b = g - Y f, so W phi_k = K phi_k - phi_k / 2.
The stopping test is the one the GMRES oracle uses (reading R1):
||b - K phi_k|| <= tol ||b||, or exactly fixed_iters updates.
"""

import numpy as np


def richardson(matvec, b, x0=None, gamma=1.0, tol=1e-10, max_iter=500, fixed_iters=None):
    """Return (phi, updates, relative residual of phi, converged)."""
    b = np.asarray(b)
    dtype = np.result_type(b, np.float64)
    phi = np.zeros(len(b), dtype=dtype) if x0 is None else np.array(x0, dtype=dtype)
    bnorm = np.linalg.norm(b)
    k = 0
    while True:
        Kphi = matvec(phi)
        rel = np.linalg.norm(b - Kphi) / bnorm if bnorm > 0 else np.linalg.norm(b - Kphi)
        if fixed_iters is not None:
            if k >= fixed_iters:
                return phi, k, rel, rel <= tol
        elif rel <= tol or k >= max_iter:
            return phi, k, rel, rel <= tol
        Wphi = Kphi - 0.5 * phi
        phi = (1.0 - 0.5 * gamma) * phi + gamma * (b - Wphi)
        k += 1
