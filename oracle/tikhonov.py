"""Generalised Tikhonov objective and its normal equation (eqs. obj, norm).

Readings:
  * The unknowns are relative maps q with dm_p = m0_p q_p, so that all five
    parameters have comparable scale; the misfit is divided by ||r||^2 so that
    lambda is dimensionless (the paper fixes neither).
  * Several problems (frequencies) stack their data: J q = [J_1 q; J_2 q; ...]
    and J* r = sum_f J_f* r_f.
  * L is either the identity (the paper's form of eq. obj) or the periodic,
    unscaled 5-point (2-D) or 7-point (3-D) Laplacian applied to each map (a
    generalised Tikhonov operator).
  * Real maps: the gradient and the normal operator take Re of J*.

    f(q)      = ||J q - r||^2 / ||r||^2 + lambda ||L q||^2
    grad f(q) = 2 Re J*(J q - r) / ||r||^2 + 2 lambda L^T L q
    (Re J*J / ||r||^2 + lambda L^T L) q = Re J* r / ||r||^2      (eq. norm)
"""

import numpy as np

from . import krylov


def laplacian(q):
    """Periodic 5-point Laplacian of each map of q [..., nz, nx], unscaled."""
    return (np.roll(q, 1, -1) + np.roll(q, -1, -1) + np.roll(q, 1, -2)
            + np.roll(q, -1, -2) - 4.0 * q)


def laplacian3(q):
    """Periodic 7-point Laplacian of each map of q [..., nz, ny, nx], unscaled."""
    return sum(np.roll(q, s, a) for a in (-1, -2, -3) for s in (1, -1)) - 6.0 * q


class Tikhonov:
    """The stacked linear problem of one DBI step.

    items: list of (LSProblem, ub [nsys,2,nz,nx], rec_ixz); m0: scales
    broadcastable to [5, nz, nx]; r: list of data arrays, one per item.
    """

    def __init__(self, items, m0, r, lam, reg="laplacian", tol=1e-12):
        self.items = items
        self.m0 = np.asarray(m0, dtype=float)
        self.r = [np.asarray(x) for x in r]
        self.rr = sum(float(np.vdot(x.ravel(), x.ravel()).real) for x in self.r)
        self.lam = float(lam)
        self.reg = reg
        self.tol = tol

    def _lap(self, q):
        # maps [nmaps, nz, nx] (2-D) or [nmaps, nz, ny, nx] (3-D)
        return laplacian3(q) if np.ndim(q) == 4 else laplacian(q)

    def L(self, q):
        return self._lap(q) if self.reg == "laplacian" else q

    def LtL(self, q):
        return self._lap(self._lap(q)) if self.reg == "laplacian" else q

    def J(self, q):
        dm = self.m0 * q
        return [P.frechet(ub, dm, rec, tol=self.tol) for (P, ub, rec) in self.items]

    def Jstar(self, d):
        g = 0.0
        for (P, ub, rec), dk in zip(self.items, d):
            g = g + P.adjoint(ub, dk, rec, tol=self.tol)
        return self.m0 * g

    def objective(self, q):
        res = [a - b for a, b in zip(self.J(q), self.r)]
        mis = sum(float(np.vdot(x.ravel(), x.ravel()).real) for x in res)
        Lq = self.L(q)
        return mis / self.rr + self.lam * float(np.sum(Lq * Lq))

    def gradient(self, q):
        res = [a - b for a, b in zip(self.J(q), self.r)]
        return 2.0 * np.real(self.Jstar(res)) / self.rr + 2.0 * self.lam * self.LtL(q)

    def normal_apply(self, q):
        return np.real(self.Jstar(self.J(q))) / self.rr + self.lam * self.LtL(q)

    def normal_rhs(self):
        return np.real(self.Jstar(self.r)) / self.rr

    def solve_cg(self, niter, q0=None):
        """`niter` CG iterations on eq. norm from q = 0; returns (q, residual norms)."""
        return krylov.cg(self.normal_apply, self.normal_rhs(), niter, x0=q0)
