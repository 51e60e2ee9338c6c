"""Pins of the oracle's DBI stage (the distorted-Born iteration around eqs. du,
obj and norm) against what the mathematics fixes, independently of the
stage's own loop: a dense Gauss-Newton step built from the forward map alone,
the stop on exactly fitted data, and the descent of the data error."""

import numpy as np
import pytest

import workloads as W
from oracle import LSProblem, dbi, operators

N, DX, FREQ = 8, 10.0, 30.0
SRC = [(1, 1), (5, 2)]
SRC_F = [(0.0, 1.0), (1.0, 0.0)]
REC = [(ix, iz) for iz in (0, 4) for ix in range(N)]


def _setup():
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0)
    m0b = m0.reshape(5, 1, 1)
    c_true = m0b * W.smooth_maps(5, N, N, 1.5, 0.03)
    c_start = m0b * W.smooth_maps(6, N, N, 1.5, 0.01)
    P = LSProblem(N, N, DX, c0, rho0, FREQ, 0.02, c_true)
    u, _ = P.solve(P.incident(SRC, SRC_F), tol=1e-13)
    return P, m0, m0b, c_true, c_start, operators.sample(u, REC)


def _forward(P, c):
    """d(c) = R A(c)^-1 u0: the receiver data of the full forward problem."""
    P.set_contrast(c)
    u, _ = P.solve(P.incident(SRC, SRC_F), tol=1e-13)
    return operators.sample(u, REC).ravel()


def test_update_is_the_dense_gauss_newton_step():
    """One update with converged CG equals the regularised Gauss-Newton step
    q = (Re J^H J / ||r||^2 + lam I)^-1 Re J^H r / ||r||^2 with J taken column
    by column from central differences of the forward map (no Frechet code)."""
    P, m0, m0b, _, c_start, d_obs = _setup()
    lam = 20.0   # keeps the normal matrix's condition near 1e2: 100 CG steps converge
    c1, eps, lams, q = dbi.dbi_stage([(P, SRC, SRC_F, REC, d_obs)], c_start, m0, lam, 100, tol=0.0,
                                     max_outer=1, solve_tol=1e-13)
    assert len(eps) == 2 and lams == [lam]
    r = d_obs.ravel() - _forward(P, c_start)
    assert eps[0] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(d_obs), rel=1e-12)
    h = 1e-4
    cols = []
    for j in range(5 * N * N):
        dm = np.zeros(5 * N * N)
        dm[j] = 1.0
        dm = m0b * dm.reshape(5, N, N)
        cols.append((_forward(P, c_start + h * dm) - _forward(P, c_start - h * dm)) / (2 * h))
    J = np.array(cols).T
    rr = float(np.vdot(r, r).real)
    A = np.real(J.conj().T @ J) / rr + lam * np.eye(J.shape[1])
    q_gn = np.linalg.solve(A, np.real(J.conj().T @ r) / rr)
    assert np.linalg.norm(q.ravel() - q_gn) / np.linalg.norm(q_gn) < 1e-7
    step = (c1 - c_start).ravel()
    assert np.linalg.norm(step - (m0b * q_gn.reshape(5, N, N)).ravel()) / np.linalg.norm(step) < 1e-7
    # the misfit recorded after the update is that of the updated model
    r1 = d_obs.ravel() - _forward(P, c1)
    assert eps[1] == pytest.approx(np.linalg.norm(r1) / np.linalg.norm(d_obs), rel=1e-9)


def test_exactly_fitted_data_end_the_stage_without_update():
    P, m0, _, _, c_start, _ = _setup()
    d_fit = _forward(P, c_start).reshape(len(SRC), len(REC), 2)
    c1, eps, lams, q = dbi.dbi_stage([(P, SRC, SRC_F, REC, d_fit)], c_start, m0, 1e-3, 5, tol=1e-3,
                                     max_outer=10, solve_tol=1e-13)
    assert eps == [0.0] and lams == [] and q is None
    assert np.array_equal(c1, c_start)


def test_data_error_descends_and_lambda_cools():
    """In the Born regime each Gauss-Newton update lowers the misfit; the
    cooled lambda never rises while the misfit falls, and the stage makes at
    most max_outer updates."""
    P, m0, _, c_true, c_start, d_obs = _setup()
    c, eps, lams, _ = dbi.dbi_stage([(P, SRC, SRC_F, REC, d_obs)], c_start, m0, 1.0, 30, tol=0.0,
                                    max_outer=3, solve_tol=1e-13)
    assert len(eps) == 4 and len(lams) == 3
    assert all(b < a for a, b in zip(eps, eps[1:]))
    assert eps[-1] < 0.5 * eps[0]
    assert lams[0] == 1.0 and all(b <= a for a, b in zip(lams, lams[1:]))
    assert np.linalg.norm(c - c_true) < np.linalg.norm(c_start - c_true)


def test_sequential_scheme_chains_the_stages():
    """The sequential scheme's first stage is dbi_stage from the starting model
    and its second stage starts from the first stage's result."""
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0)
    m0b = m0.reshape(5, 1, 1)
    nx, nz = 16, 12
    c_true = m0b * W.smooth_maps(31, nz, nx, 2.0, 0.03)
    start = m0b * W.smooth_maps(32, nz, nx, 2.0, 0.01)
    src, srcf, rec = [(4, 1), (11, 1)], [(0.0, 1.0), (0.0, 1.0)], [(ix, 2) for ix in range(0, nx, 2)]
    stages = []
    for f in (20.0, 28.0):
        P = LSProblem(nx, nz, 10.0, c0, rho0, f, 0.02, c_true)
        u, _ = P.solve(P.incident(src, srcf), tol=1e-13)
        stages.append([(LSProblem(nx, nz, 10.0, c0, rho0, f, 0.02), src, srcf, rec, operators.sample(u, rec))])
    c_seq, recs = dbi.invert_sequential(stages, start, m0, 1.0, 4, tol=0.0, max_outer=1)
    c1, eps1, lam1, _ = dbi.dbi_stage(stages[0], start, m0, 1.0, 4, tol=0.0, max_outer=1)
    c2, eps2, lam2, _ = dbi.dbi_stage(stages[1], c1, m0, 1.0, 4, tol=0.0, max_outer=1)
    assert np.allclose(c_seq, c2, rtol=0, atol=1e-12 * np.abs(c2).max())
    assert recs[0][0] == eps1 and recs[1][0] == eps2
    # each stage lowers its own data error
    assert eps1[-1] < eps1[0] and eps2[-1] < eps2[0]
