"""Oracle restarted GMRES (TEST INFRASTRUCTURE ONLY).

The paper solves the boundary integral equation (3.17) by Richardson
iteration (3.21) and names GMRES as the better Krylov alternative in its
conclusion.  Reading R1 fixes the GMRES variant: GMRES(m) with m = 50,
modified Gram-Schmidt Arnoldi in the working precision, x0 = the caller's
warm start, stop when ||b - K x||_2 / ||b||_2 <= tol, at most max_iter
matrix-vector products; `fixed_iters` runs exactly that many products
whatever the residual (parity mode, reading R20).

The small least-squares problem min ||beta e1 - H y|| is solved by the
library's least-squares routine at every step (plain, not Givens-updated);
its residual norm is the GMRES residual estimate.
"""

import numpy as np


def _lsq(H, beta, j):
    """Solve the (j+2) x (j+1) least-squares problem; return (y, resid)."""
    Hj = H[:j + 2, :j + 1]
    rhs = np.zeros(j + 2, dtype=H.dtype)
    rhs[0] = beta
    y = np.linalg.lstsq(Hj, rhs, rcond=None)[0]
    return y, np.linalg.norm(rhs - Hj @ y)


def gmres(matvec, b, x0=None, tol=1e-10, restart=50, max_iter=500,
          fixed_iters=None):
    """Return (x, iterations, relative residual estimate, converged)."""
    b = np.asarray(b)
    dtype = np.result_type(b, np.float64)
    n = len(b)
    x = np.zeros(n, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0 and fixed_iters is None:
        return np.zeros(n, dtype=dtype), 0, 0.0, True
    limit = max_iter if fixed_iters is None else fixed_iters
    total = 0
    rel = np.inf
    while True:
        r = b - matvec(x) if np.any(x != 0) else b.astype(dtype)
        beta = np.linalg.norm(r)
        rel = beta / bnorm if bnorm > 0 else beta
        if fixed_iters is None and rel <= tol:
            return x, total, rel, True
        if total >= limit or beta == 0.0:
            return x, total, rel, rel <= tol
        m = min(restart, limit - total)
        V = np.zeros((n, m + 1), dtype=dtype)
        H = np.zeros((m + 1, m), dtype=dtype)
        V[:, 0] = r / beta
        y = None
        for j in range(m):
            w = matvec(V[:, j])
            total += 1
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            y, res = _lsq(H, beta, j)
            rel = res / bnorm if bnorm > 0 else res
            if (fixed_iters is None and rel <= tol) or total >= limit \
                    or H[j + 1, j] == 0.0:
                break
        x = x + V[:, :len(y)] @ y
        if (fixed_iters is None and rel <= tol) or total >= limit:
            return x, total, rel, rel <= tol
