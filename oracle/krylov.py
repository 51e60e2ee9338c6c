"""Textbook Krylov solvers used by the oracle.

The paper names CG, BiCGSTAB and GMRES for eq. axb without giving a tolerance,
restart or start vector.  The oracle uses:

* BiCGSTAB as published by van der Vorst (1992), unpreconditioned, x0 = 0
  unless given, stopping when the recursive residual satisfies
  ||r_k|| <= tol ||b||.  The true residual ||b - A x|| / ||b|| is reported
  as well.  Inner products are <a, b> = sum conj(a) b.
* CG (Hestenes and Stiefel 1952) for the real symmetric positive definite
  normal equation of eq. norm, run for a fixed number of iterations.
"""

import numpy as np


def vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def norm(a):
    return float(np.sqrt(np.real(vdot(a, a))))


class SolveInfo:
    """Per-solve record: iterations, recursive and true relative residual."""

    def __init__(self, iters, relres, true_relres, history):
        self.iters = iters
        self.relres = relres
        self.true_relres = true_relres
        self.history = history

    def __repr__(self):
        return (f"SolveInfo(iters={self.iters}, relres={self.relres:.3e}, "
                f"true_relres={self.true_relres:.3e})")


def bicgstab(apply, b, tol=1e-8, maxit=10000, x0=None):
    """Solve apply(x) = b by BiCGSTAB; returns (x, SolveInfo)."""
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=b.dtype)
    if bnorm == 0.0:
        return np.zeros_like(b), SolveInfo(0, 0.0, 0.0, [0.0])
    r = b - apply(x) if x0 is not None else b.copy()
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    hist = [norm(r) / bnorm]
    it = 0
    while hist[-1] > tol and it < maxit:
        it += 1
        rho = vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p)
        alpha = rho / vdot(rhat, v)
        s = r - alpha * v
        t = apply(s)
        tt = vdot(t, t)
        omega = vdot(t, s) / tt if tt != 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        hist.append(norm(r) / bnorm)
    true_rel = norm(b - apply(x)) / bnorm
    return x, SolveInfo(it, hist[-1], true_rel, hist)


def cg(apply, b, niter, x0=None):
    """Run `niter` CG iterations on a real SPD system; returns (x, residual norms)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=b.dtype)
    r = b - apply(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = float(np.vdot(r.ravel(), r.ravel()).real)
    hist = [np.sqrt(rr)]
    for _ in range(niter):
        Ap = apply(p)
        alpha = rr / float(np.vdot(p.ravel(), Ap.ravel()).real)
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.vdot(r.ravel(), r.ravel()).real)
        hist.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, hist
