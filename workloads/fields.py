"""Seeded smooth random fields for the batched Helmholtz instances.

f(x, y) = sum_{p,q=0}^{7} g_pq exp(-(p^2+q^2)/8) cos(p pi x/2 + alpha_pq)
                                              cos(q pi y/2 + beta_pq)
with g ~ N(0,1) and alpha, beta ~ U[0, 2 pi), drawn from the caller's PCG64
stream.  A field object is evaluated at any points.
"""

import numpy as np


class SmoothField:
    def __init__(self, rng, n=8):
        self.n = n
        self.g = rng.standard_normal((n, n))
        self.alpha = rng.uniform(0.0, 2.0 * np.pi, (n, n))
        self.beta = rng.uniform(0.0, 2.0 * np.pi, (n, n))

    def grid(self, x, y):
        """The field on the tensor grid F[j, i] = f(x[i], y[j]): each term is a
        product of a function of x and a function of y, so the sum is one
        (len(y) x n^2) @ (n^2 x len(x)) product."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        p = np.arange(self.n)[:, None]
        q = np.arange(self.n)[None, :]
        amp = (self.g * np.exp(-(p * p + q * q) / 8.0)).ravel()
        cx = np.cos(np.pi / 2.0 * np.multiply.outer(np.repeat(np.arange(self.n), self.n), x)
                    + self.alpha.ravel()[:, None])
        cy = np.cos(np.pi / 2.0 * np.multiply.outer(np.tile(np.arange(self.n), self.n), y)
                    + self.beta.ravel()[:, None])
        return (cy.T * amp) @ cx

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for p in range(self.n):
            for q in range(self.n):
                amp = self.g[p, q] * np.exp(-(p * p + q * q) / 8.0)
                out = out + amp * np.cos(p * np.pi * x / 2.0 + self.alpha[p, q]) \
                    * np.cos(q * np.pi * y / 2.0 + self.beta[p, q])
        return out
