"""Relative error of every result against the complex128 oracle, stated per
result (printed with -s): total and scattered fields, receiver data, J dm,
J* r, the Tikhonov gradient, for BiCGSTAB and GMRES solves to 1e-7 on a
96 x 64 VTI grid with two frequencies and three sources each.  Every error
must be <= 1e-4."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import LSProblem, tikhonov

pytestmark = pytest.mark.gpu

NX, NZ, NSYS, NREC, FREQS = 96, 64, 3, 12, (6.0, 11.0)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("krylov", ["bicgstab", "gmres"])
def test_relative_error_per_result(krylov):
    from paper_2402_02116_amd.plan import Plan
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0)
    maps = W.round_f32(m0 * W.random_layered(11, NZ, NX))
    src, f = W.surface_sources(NX, NSYS, iz=1)
    rec = W.surface_receivers(NX, NREC, iz=2)
    probs = [dict(nx=NX, nz=NZ, dx=10.0, c0=c0, rho0=rho0, freq_hz=fr, eta=0.02, nsys=NSYS) for fr in FREQS]
    plan = Plan(probs)
    for i in range(len(FREQS)):
        plan.set_contrast(i, maps)
        plan.set_receivers(i, rec)
    if krylov == "gmres":
        plan.set_krylov("gmres", restart=24)
    u0 = plan.incident(src * len(FREQS), f * len(FREQS))
    ub = plan.solve(u0, rtol=1e-7, maxit=3000).x
    q = W.round_f32(W.smooth_maps(12, NZ, NX, 4.0, 0.02))
    qt = torch.as_tensor(q, dtype=torch.float32).cuda()
    r_np = [W.round_f32(W.complex_normal(13 + k, (NSYS, NREC, 2))) for k in range(len(FREQS))]
    r = torch.as_tensor(np.concatenate([x.ravel() for x in r_np]).astype(np.complex64)).cuda()
    m0v = m0.ravel()
    d = plan.frechet_rel(ub, qt, m0v, rtol=1e-7).cpu().numpy()
    g = plan.adjoint_rel(ub, r, m0v, rtol=1e-7).cpu().numpy()
    fval, grad = plan.tikhonov_grad(ub, r, m0v, qt, lam=1e-3, reg="laplacian", rtol=1e-7)
    errs = {"u (total field)": [], "u - u0 (scattered)": [], "R u (receiver data)": []}
    items = []
    for i, fr in enumerate(FREQS):
        P = LSProblem(NX, NZ, 10.0, c0, rho0, fr, 0.02, maps)
        u0r = P.incident(src, f)
        uref, _ = P.solve(u0r, tol=1e-12)
        u = _np(plan.view(ub, i))
        errs["u (total field)"].append(_rel(u, uref))
        errs["u - u0 (scattered)"].append(_rel(u - _np(plan.view(u0, i)), uref - u0r))
        ri = np.asarray(rec)
        errs["R u (receiver data)"].append(_rel(u[:, :, ri[:, 1], ri[:, 0]], uref[:, :, ri[:, 1], ri[:, 0]]))
        items.append((P, uref, rec))
    T = tikhonov.Tikhonov(items, m0, r_np, lam=1e-3, reg="laplacian", tol=1e-12)
    errs["J (m0 q)"] = [_rel(d, np.concatenate([x.ravel() for x in T.J(q)]))]
    errs["m0 Re J* r"] = [_rel(g, np.real(T.Jstar(r_np)))]
    errs["Tikhonov gradient"] = [_rel(grad.cpu().numpy(), T.gradient(q))]
    errs["Tikhonov objective"] = [abs(fval - T.objective(q)) / abs(T.objective(q))]
    print(f"\n[accuracy] {krylov}, {NX}x{NZ}, {len(FREQS)} frequencies x {NSYS} sources, solves to 1e-7:")
    for k, v in errs.items():
        print(f"[accuracy]   {k:22s} max rel. error {max(v):.2e}")
    for k, v in errs.items():
        assert max(v) <= 1e-4, (k, v)
