"""Oracle time steppers (TEST INFRASTRUCTURE ONLY).

Each implicit step is one modified-Helmholtz solve (oracle.bie), Dirichlet
or Neumann, whose right-hand side comes from a recurrence, so that no
discrete Laplacian of the numerical solution is ever formed (section 3.1).
The same recurrence is carried on Gamma (reading R11), giving the trace of f
needed by the jump conditions; it takes u = g there for the Dirichlet
problem and the extracted interior limit U+ for the Neumann problem (g is
then du/dn).

Heat, Crank-Nicolson (eqs. 3.1-3.4, with a source s and diffusivity c,
reading R13):  kappa = 2c/tau,
    F^{n+1} = G^n + s^n + s^{n+1},   G^n = kappa u^n + lap u^n,
    lap u^{n+1} - kappa u^{n+1} = -F^{n+1},
    G^{n+1} = 2 kappa u^{n+1} - F^{n+1}      (= 4/tau u - F for c = 1).

Wave, implicit theta-scheme (eqs. 3.5-3.7, general theta, reading R15):
    kappa = 1/(theta tau^2),
    F^1 = (2u^0 - u^-1)/(theta tau^2) + (1-2theta)/theta lap u^0 + lap u^-1,
    F^0 = kappa u^0 - lap u^0,
    F^{n+2} = (kappa/theta) u^{n+1} - (1-2theta)/theta F^{n+1} - F^n
    (theta = 1/4 gives 16/tau^2 u - 2F - F, as in the paper).

Schroedinger, Strang splitting (eqs. 3.8-3.12 and the three-step algorithm
after them; i u_t = lap u + v u + w|u|^2 u as in eq. 2.2; reading R16):
    u*   = u^n - i tau/2 lap u^n   (= 2u^n - u**_prev for n >= 1),
    u**  = u* (1 - i beta)/(1 + i beta),  beta = tau/2 (v + w|u*|^2)
           (the Crank-Nicolson step of (3.10) solved in closed form; it
           keeps |u**| = |u*|, so the same beta holds on both sides),
    lap u^{n+1} - (2i/tau) u^{n+1} = -(2i/tau) u**.

Schroedinger, Godunov (Lie) splitting u^{n+1} = S^A(tau) S^B(tau) u^n (the
first-order splitting of section 1 and Example 7; reading R28): the B-step
is the same closed-form Crank-Nicolson step of (3.10) over tau, applied to
u^n itself; the A-step is the backward Euler step of (3.11) over the whole
step tau, u^{n+1} + i tau lap u^{n+1} = u**, i.e.
    lap u^{n+1} - (i/tau) u^{n+1} = -(i/tau) u**,
so no Laplacian of a numerical solution is needed and the carried state is
u^n (on Gamma its trace, g for the Dirichlet problem).
"""

import numpy as np

from .bie import helmholtz_solve, neumann_solve


class _Base:
    def __init__(self, dom, tol, restart, max_iter, bc="dirichlet"):
        if bc not in ("dirichlet", "neumann"):
            raise ValueError("bc must be 'dirichlet' or 'neumann'")
        self.dom = dom
        self.tol, self.restart, self.max_iter = tol, restart, max_iter
        self.bc = bc
        self.phi = None
        self.n = 0
        self.last_stats = None

    def _solve(self, f_grid, f_gamma, g, fixed_iters=None):
        """One implicit solve.  Returns (U, trace of u on Gamma): the trace is
        g for the Dirichlet problem and the extracted U+ for the Neumann one
        (g is then du/dn)."""
        if self.bc == "neumann":
            U, psi, trace, st = neumann_solve(self.dom, self.kappa, f_grid, f_gamma, g, psi0=self.phi,
                                              tol=self.tol, restart=self.restart, max_iter=self.max_iter,
                                              fixed_iters=fixed_iters)
            self.phi = psi
        else:
            U, phi, st = helmholtz_solve(self.dom, self.kappa, f_grid, f_gamma, g,
                                         phi0=self.phi, tol=self.tol,
                                         restart=self.restart,
                                         max_iter=self.max_iter,
                                         fixed_iters=fixed_iters)
            self.phi = phi
            trace = np.asarray(g)
        self.last_stats = st
        self.n += 1
        return U, trace


class HeatStepper(_Base):
    def __init__(self, dom, tau, u0, lap_u0, u0_gamma, lap_u0_gamma, c=1.0,
                 tol=1e-10, restart=50, max_iter=500, bc="dirichlet"):
        super().__init__(dom, tol, restart, max_iter, bc)
        self.tau = tau
        self.kappa = 2.0 * c / tau
        self.G = self.kappa * np.asarray(u0) + lap_u0
        self.G_gamma = self.kappa * np.asarray(u0_gamma) + lap_u0_gamma

    def step(self, g_next, src_grid=None, src_gamma=None, fixed_iters=None):
        F = self.G + (0.0 if src_grid is None else src_grid)
        Fg = self.G_gamma + (0.0 if src_gamma is None else src_gamma)
        U, tr = self._solve(-F, -Fg, g_next, fixed_iters)
        self.G = 2.0 * self.kappa * U - F
        self.G_gamma = 2.0 * self.kappa * tr - Fg
        return U


class WaveStepper(_Base):
    def __init__(self, dom, tau, u0, lap_u0, u0_gamma, lap_u0_gamma,
                 um1, lap_um1, um1_gamma, lap_um1_gamma, theta=0.25,
                 tol=1e-10, restart=50, max_iter=500, bc="dirichlet"):
        super().__init__(dom, tol, restart, max_iter, bc)
        self.tau, self.theta = tau, theta
        k = 1.0 / (theta * tau * tau)
        self.kappa = k
        c1 = (1.0 - 2.0 * theta) / theta
        self.F1 = k * (2.0 * u0 - um1) + c1 * lap_u0 + lap_um1
        self.F0 = k * u0 - lap_u0
        self.F1_gamma = k * (2.0 * u0_gamma - um1_gamma) + c1 * lap_u0_gamma + lap_um1_gamma
        self.F0_gamma = k * u0_gamma - lap_u0_gamma

    def step(self, g_next, fixed_iters=None):
        th, k = self.theta, self.kappa
        c1 = (1.0 - 2.0 * th) / th
        U, tr = self._solve(-self.F1, -self.F1_gamma, g_next, fixed_iters)
        F2 = (k / th) * U - c1 * self.F1 - self.F0
        F2g = (k / th) * tr - c1 * self.F1_gamma - self.F0_gamma
        self.F0, self.F1 = self.F1, F2
        self.F0_gamma, self.F1_gamma = self.F1_gamma, F2g
        return U


class SchrodingerStepper(_Base):
    def __init__(self, dom, tau, u0, lap_u0, u0_gamma, lap_u0_gamma,
                 v_grid, v_gamma, w=0.0, tol=1e-10, restart=50, max_iter=500, bc="dirichlet",
                 split="strang"):
        super().__init__(dom, tol, restart, max_iter, bc)
        if split not in ("strang", "godunov"):
            raise ValueError("split must be 'strang' or 'godunov'")
        self.tau, self.w, self.split = tau, w, split
        self.v, self.v_gamma = v_grid, v_gamma
        if split == "strang":
            # u* of the first step: the forward half step of the A part
            self.kappa = 2j / tau
            self.ustar = np.asarray(u0, dtype=np.complex128) - 0.5j * tau * lap_u0
            self.ustar_gamma = (np.asarray(u0_gamma, dtype=np.complex128)
                                - 0.5j * tau * lap_u0_gamma)
        else:
            # Godunov: the B-step acts on u^n itself
            self.kappa = 1j / tau
            self.ustar = np.array(u0, dtype=np.complex128)
            self.ustar_gamma = np.array(u0_gamma, dtype=np.complex128)

    def _b_step(self, us, v):
        beta = 0.5 * self.tau * (v + self.w * np.abs(us) ** 2)
        return us * (1.0 - 1j * beta) / (1.0 + 1j * beta)

    def step(self, g_next, fixed_iters=None):
        uss = self._b_step(self.ustar, self.v)
        uss_g = self._b_step(self.ustar_gamma, self.v_gamma)
        g_next = np.asarray(g_next, dtype=np.complex128)
        U, tr = self._solve(-self.kappa * uss, -self.kappa * uss_g, g_next,
                            fixed_iters)
        if self.split == "strang":
            # u* of the next step, u^{n+1} - i tau/2 lap u^{n+1}, from (3.12):
            # i tau/2 lap u^{n+1} = u** - u^{n+1}
            self.ustar = 2.0 * U - uss
            self.ustar_gamma = 2.0 * tr - uss_g
        else:
            self.ustar = U
            self.ustar_gamma = np.array(tr, dtype=np.complex128)
        return U
