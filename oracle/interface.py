"""Oracle interface-problem solve (TEST INFRASTRUCTURE ONLY).

One evaluation of Procedure 2 (section 3.3): for the unified interface
problem (3.30) with F = f~ (eq. 3.25), [u] = phi, [u_n] = psi and u = 0 on
the box boundary,

  a. jumps of u and its derivatives on Gamma (section 3.2.5, eq. 3.35 and
     the 3x3 system after it),
  b. correction of the five-point equations at irregular nodes (section
     3.2.4, C^+/C^- terms) and the grid solve (eq. 3.31),
  c. extraction of the interior limit U^+ at the collocation points
     (section 3.2.6, eq. 3.36), and for the Neumann problem of the interior
     normal derivative n . grad U^+ from the same expansion (its first-order
     coefficients).

Readings taken:
  R8  correction at node P for a crossing edge (P, Q) with intersection X on
      axis a: C(P) = -sigma(P) J / h^2, J = [u] + [u_a] d + [u_aa] d^2 / 2,
      d = Q_a - X_a, sigma = +1 inside, -1 outside (derived from the Taylor
      expansion; matches C^+ and C^- of section 3.2.4).
  R9  the second row of (3.35) has right-hand side psi (not psi_s).
  R10 phi_theta, phi_thetatheta at collocation points by periodic 4th-order
      central differences; values at a crossing parameter theta* by cubic
      Lagrange interpolation on nodes k-1..k+2, theta_k <= theta* < theta_k+1.
  R11 f on Gamma is supplied as a trace array f_gamma at the collocation
      points and interpolated like phi.
  R23 f~ = f at inside nodes, 0 outside.
"""

import numpy as np

from . import boxsolve


def theta_derivs(v, dtheta):
    """Periodic 4th-order central differences (R10): (v_theta, v_thetatheta)."""
    vp1, vp2 = np.roll(v, -1), np.roll(v, -2)
    vm1, vm2 = np.roll(v, 1), np.roll(v, 2)
    d1 = (-vp2 + 8.0 * vp1 - 8.0 * vm1 + vm2) / (12.0 * dtheta)
    d2 = (-vp2 + 16.0 * vp1 - 30.0 * v + 16.0 * vm1 - vm2) / (12.0 * dtheta * dtheta)
    return d1, d2


def lagrange_at(theta_star, dtheta, arrays):
    """Cubic Lagrange interpolation in theta (R10) of each periodic array in
    `arrays` at the parameters theta_star."""
    Nb = len(arrays[0])
    k = np.floor(theta_star / dtheta).astype(np.int64)
    k = np.minimum(k, Nb - 1)
    s = theta_star / dtheta - k
    w = [-s * (s - 1.0) * (s - 2.0) / 6.0,
         (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0,
         -(s + 1.0) * s * (s - 2.0) / 2.0,
         (s + 1.0) * s * (s - 1.0) / 6.0]
    out = []
    for a in arrays:
        acc = 0.0
        for o, wo in zip((-1, 0, 1, 2), w):
            acc = acc + wo * a[(k + o) % Nb]
        out.append(acc)
    return out


def jumps(geom, phi, phi_t, phi_tt, f, kappa, psi=0.0, psi_t=0.0):
    """Jumps of u, grad u and the Hessian across Gamma (section 3.2.5).

    phi, phi_t, phi_tt: the density and its theta-derivatives at the points;
    f: the trace of f on Gamma from inside; psi, psi_t: the normal-derivative
    jump and its theta-derivative (0 for the Dirichlet problem).
    """
    sig, dsig = geom["sigma"], geom["dsigma"]
    tx, ty, dtx, dty = geom["tx"], geom["ty"], geom["dtx"], geom["dty"]
    n = len(tx)
    dtype = np.result_type(phi, phi_t, phi_tt, f, kappa, psi, psi_t, tx)

    def full(v):
        return np.broadcast_to(np.asarray(v, dtype=dtype), (n,))

    phi, phi_t, phi_tt, f = full(phi), full(phi_t), full(phi_tt), full(f)
    psi, psi_t = full(psi), full(psi_t)
    phi_s = phi_t / sig
    phi_ss = (phi_tt - phi_s * dsig) / (sig * sig)
    psi_s = psi_t / sig
    # eq. (3.35) with right-hand side psi (R9); its matrix is its own inverse
    ux = tx * phi_s + ty * psi
    uy = ty * phi_s - tx * psi
    # the 3x3 system for [u_xx], [u_xy], [u_yy]
    A = np.zeros((n, 3, 3), dtype=dtype)
    A[:, 0, 0] = tx * tx
    A[:, 0, 1] = 2.0 * tx * ty
    A[:, 0, 2] = ty * ty
    A[:, 1, 0] = tx * ty
    A[:, 1, 1] = ty * ty - tx * tx
    A[:, 1, 2] = -tx * ty
    A[:, 2, 0] = 1.0
    A[:, 2, 2] = 1.0
    rhs = np.stack([phi_ss - (dtx * ux + dty * uy),
                    psi_s - dty * ux + dtx * uy,
                    f + kappa * phi], axis=1)
    sec = np.linalg.solve(A, rhs[:, :, None])[:, :, 0]
    return {"u": phi.copy(), "ux": ux, "uy": uy,
            "uxx": sec[:, 0], "uxy": sec[:, 1], "uyy": sec[:, 2]}


def boundary_data(dom, phi, f_gamma, psi=None):
    """phi, phi_theta, phi_thetatheta (and the same for f and psi) at the
    collocation points."""
    pt, ptt = theta_derivs(phi, dom.dtheta)
    out = {"phi": phi, "phi_t": pt, "phi_tt": ptt, "f": f_gamma}
    if psi is not None:
        out["psi"] = psi
        out["psi_t"], _ = theta_derivs(psi, dom.dtheta)
    return out


def jumps_at_collocation(dom, kappa, bd):
    psi = bd.get("psi", 0.0)
    psi_t = bd.get("psi_t", 0.0)
    return jumps(dom.colloc, bd["phi"], bd["phi_t"], bd["phi_tt"], bd["f"],
                 kappa, psi, psi_t)


def jumps_at_crossings(dom, kappa, bd):
    arrays = [bd["phi"], bd["phi_t"], bd["phi_tt"], bd["f"]]
    have_psi = "psi" in bd
    if have_psi:
        arrays += [bd["psi"], bd["psi_t"]]
    vals = lagrange_at(dom.edge_theta, dom.dtheta, arrays)
    psi, psi_t = (vals[4], vals[5]) if have_psi else (0.0, 0.0)
    return jumps(dom.edge_geom, vals[0], vals[1], vals[2], vals[3], kappa,
                 psi, psi_t)


def corrections(dom, je):
    """Correction grid C (M+1)x(M+1), nonzero only at irregular nodes (R8)."""
    M, h = dom.M, dom.h
    xs, ys = dom.X.ravel(), dom.Y.ravel()
    insr = dom.inside.ravel()
    dtype = np.result_type(je["u"], je["uxx"])
    C = np.zeros((M + 1) * (M + 1), dtype=dtype)
    ax = dom.edge_axis
    Xa = np.where(ax == 0, dom.edge_X, dom.edge_Y)
    ua = np.where(ax == 0, je["ux"], je["uy"])
    uaa = np.where(ax == 0, je["uxx"], je["uyy"])
    for node, other in ((dom.edge_p, dom.edge_q), (dom.edge_q, dom.edge_p)):
        d = np.where(ax == 0, xs[other], ys[other]) - Xa
        J = je["u"] + ua * d + 0.5 * uaa * d * d
        sgn = np.where(insr[node], 1.0, -1.0)
        np.add.at(C, node, -sgn * J / (h * h))
    return C.reshape(M + 1, M + 1)


def extract(dom, U, jz, weights=None):
    """U^+ at the collocation points from the grid solution U and the jumps
    at the collocation points (section 3.2.6).  weights: the six-point
    weights (default: those of U^+; dom.st_weight_n gives the interior
    normal derivative from the same corrected values)."""
    xi, eta = dom.st_xi, dom.st_eta
    J = (jz["u"][:, None] + jz["ux"][:, None] * xi + jz["uy"][:, None] * eta
         + 0.5 * jz["uxx"][:, None] * xi * xi + jz["uxy"][:, None] * xi * eta
         + 0.5 * jz["uyy"][:, None] * eta * eta)
    Ut = U.ravel()[dom.st_node] + np.where(dom.st_outside, J, 0.0)
    return np.sum((dom.st_weight if weights is None else weights) * Ut, axis=1)


def interface_solve(dom, kappa, f_grid, f_gamma, phi, psi=None, normal=False):
    """Solve the interface problem (3.30) with F = f~, [u] = phi, [u_n] = psi.

    f_grid: (M+1)x(M+1) array or None (f = 0); f_gamma: trace of f on Gamma at
    the collocation points (None when f = 0).  Returns (U, Uplus): the grid
    solution on all (M+1)^2 nodes (zero on the box boundary) and the interior
    limit U^+ at the collocation points; with normal=True also the interior
    normal derivative dU^+/dn there (U, Uplus, Unplus).
    """
    M, h = dom.M, dom.h
    cplx = any(np.iscomplexobj(v) for v in (kappa, f_grid, f_gamma, phi, psi)
               if v is not None)
    dtype = np.complex128 if cplx else np.float64
    phi = np.asarray(phi, dtype=dtype)
    if f_gamma is None:
        f_gamma = np.zeros(dom.Nb, dtype=dtype)
    bd = boundary_data(dom, phi, np.asarray(f_gamma, dtype=dtype),
                       None if psi is None else np.asarray(psi, dtype=dtype))
    je = jumps_at_crossings(dom, kappa, bd)
    jz = jumps_at_collocation(dom, kappa, bd)
    R = corrections(dom, je).astype(dtype)
    if f_grid is not None:
        R = R + np.where(dom.inside, f_grid, 0.0)          # f~ (R23)
    U = np.zeros((M + 1, M + 1), dtype=dtype)
    U[1:-1, 1:-1] = boxsolve.solve(R[1:-1, 1:-1], h, kappa)
    if normal:
        return U, extract(dom, U, jz), extract(dom, U, jz, dom.st_weight_n)
    return U, extract(dom, U, jz)
