"""The distorted-Born iterative (DBI) inversion at one frequency stage: the
iteration the paper builds around eqs. du, obj and norm (the DBI and
Frechet-derivative sections), with the stopping rule and the normalised data
error of its numerical examples.  Test infrastructure: used by the tests only.

One outer iteration k, with the background model m_b = homogeneous reference
+ contrast c_k, shared by every item (frequency) of the stage:
  1. u^b = A_b^-1 u0 for every item (eq. axb with the contrast c_k);
  2. r = d_obs - R u^b and eps_d = ||r|| / ||d_obs|| over all items (the
     normalised data error of the numerical examples);
  3. the stage ends when eps_d < tol or once max_outer updates were made;
  4. q = niter CG iterations on the normal equation (eq. norm) with lambda_k;
  5. c_{k+1} = c_k + m0 q (the background update of the DBI loop).

Readings (the paper names the scheme and cites it, without a formula):
  * self-adaptive cooling: lambda_k = lambda_0 eps_d,k / eps_d,0, so lambda
    falls with the data misfit and stays where it is when the misfit stalls;
  * the iteration limit of the stopping rule counts model updates: a stage
    makes at most max_outer updates and evaluates the misfit once more after
    the last one (eps_d has at most max_outer + 1 entries);
  * an exactly zero misfit also ends the stage (nothing is left to fit).
"""

import numpy as np

from . import operators, tikhonov


def data_error(res, d_obs):
    """eps_d = ||r|| / ||d_obs|| over lists of per-item data arrays."""
    rr = sum(float(np.vdot(x.ravel(), x.ravel()).real) for x in res)
    dd = sum(float(np.vdot(x.ravel(), x.ravel()).real) for x in d_obs)
    return float(np.sqrt(rr / dd))


def _sample(P, u, rec):
    """Receiver sampling of a 2-D or 3-D problem's fields."""
    if hasattr(P, "ny"):
        from .elastic3d import sample_3d
        return sample_3d(u, rec)
    return operators.sample(u, rec)


def background_data(items, contrast, solve_tol=1e-12):
    """u^b and R u^b of every item under one contrast (steps 1-2)."""
    fields, data = [], []
    for (P, src, f, rec, _) in items:
        P.set_contrast(contrast)
        ub, _ = P.solve(P.incident(src, f), tol=solve_tol)
        fields.append(ub)
        data.append(_sample(P, ub, rec))
    return fields, data


def dbi_stage(items, contrast, m0, lam0, niter, reg="identity", tol=1e-3, max_outer=10,
              solve_tol=1e-12):
    """Run one frequency stage of the DBI loop.

    items: list of (LSProblem, src_ixz, src_f, rec_ixz, d_obs), one per
    frequency of the stage, all on one grid; contrast: starting maps [5, nz,
    nx] (2-D) or [nmaps, nz, ny, nx] (3-D) in Pa and kg/m^3; m0: the
    parameter scales (dm_p = m0_p q_p).
    Returns (contrast, eps_d history, lambda of each update, last q or None).
    """
    c = np.array(contrast, dtype=float)
    m0b = np.asarray(m0, dtype=float).reshape((c.shape[0],) + (1,) * (c.ndim - 1))
    d_obs = [it[4] for it in items]
    eps_hist, lam_hist, q = [], [], None
    for k in range(max_outer + 1):
        fields, data = background_data(items, c, solve_tol)
        res = [d - dc for d, dc in zip(d_obs, data)]
        eps = data_error(res, d_obs)
        eps_hist.append(eps)
        if eps < tol or eps == 0.0 or k == max_outer:
            break
        lam = lam0 * eps / eps_hist[0]
        lam_hist.append(lam)
        T = tikhonov.Tikhonov([(P, ub, rec) for (P, _, _, rec, _), ub in zip(items, fields)],
                              m0b, res, lam, reg=reg, tol=solve_tol)
        q, _ = T.solve_cg(niter)
        c = c + m0b * q
    for (P, *_rest) in items:
        P.set_contrast(c)
    return c, eps_hist, lam_hist, q


def invert_sequential(stages, contrast, m0, lam0, niter, reg="identity", tol=1e-3, max_outer=10,
                      solve_tol=1e-12):
    """The sequential-frequency scheme of the numerical-examples section: the
    stages (one list of items per frequency, lowest first; items as for
    dbi_stage) are inverted one after the other, each starting from the model
    the previous stage ended with.  Returns (final contrast, per-stage
    (eps_d history, lambdas))."""
    c = np.array(contrast, dtype=float)
    records = []
    for items in stages:
        c, eps, lam, _ = dbi_stage(items, c, m0, lam0, niter, reg=reg, tol=tol, max_outer=max_outer,
                                   solve_tol=solve_tol)
        records.append((eps, lam))
    return c, records

