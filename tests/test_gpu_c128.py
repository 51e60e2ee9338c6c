"""GPU parity of the complex128 build of the library (FWILS_C128: complex128
fields, float64 maps, the same kernels compiled in double precision) against
the complex128 CPU oracle.  With double-precision arithmetic the kernels must
agree with the oracle to near rounding (1e-12 for one operator application),
and solves to what their tolerance implies.  It also runs the complex64 path
against the complex128 GPU run, which is how the error of a large complex64
computation that the CPU oracle cannot reach is stated."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import LSProblem, dense, tikhonov

pytestmark = pytest.mark.gpu

OP_TOL = 1e-12


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _plan(problems, precision="c128"):
    from paper_2402_02116_amd.plan import Plan
    return Plan(problems, precision=precision)


def _vti(nx, nz, nsys, f=6.0, seed=3, amp=0.08, dx=8.0, symbol="spectral"):
    c0, rho0 = W.vti_background()
    maps = W.model_scales(c0, rho0) * W.smooth_maps(seed, nz, nx, 3.0, amp)
    return dict(nx=nx, nz=nz, dx=dx, c0=tuple(c0), rho0=rho0, freq_hz=f, eta=0.02, nsys=nsys,
                symbol=symbol), maps


def _oracle(p, maps):
    return LSProblem(p["nx"], p["nz"], p["dx"], p["c0"], p["rho0"], p["freq_hz"], p["eta"], maps,
                     symbol=p.get("symbol", "spectral"))


def test_iso32_blob_c128_bicgstab_matches_dense_solve():
    """32^2 isotropic background, Gaussian blob, one vertical force, 10 Hz:
    complex128 BiCGSTAB to 1e-8 against a dense direct solve of (I - G V) u = u0
    (2048 unknowns) with G from a direct DFT sum."""
    c = W.iso32_blob()
    p = dict(nx=32, nz=32, dx=c["dx"], c0=tuple(c["c0"]), rho0=c["rho0"], freq_hz=c["freq_hz"],
             eta=c["eta"], nsys=1)
    print("c128 iso32 blob", flush=True)
    plan = _plan([p])
    plan.set_contrast(0, c["maps"])
    u0 = plan.incident(c["src_ixz"], c["src_f"])
    assert u0.dtype == torch.complex128
    res = plan.solve(u0, rtol=1e-8, maxit=500)
    assert res.status == 0 and res.relres[0] <= 1e-8, (res.status, res.relres)
    P = _oracle(p, c["maps"])
    G = dense.green_matrix(P.Ghat)
    V = dense.contrast_operator(c["maps"], P.omega_t, 32, 32, c["dx"]).toarray()
    s = dense.point_source_vector(32, 32, c["dx"], 16, 16, 0.0, 1.0)
    u0d = G @ s
    assert _rel(_np(u0).ravel(), u0d) < OP_TOL
    ud = np.linalg.solve(np.eye(G.shape[0]) - G @ V, u0d)
    err = _rel(_np(res.x).ravel(), ud)
    assert err < 1e-7, err
    # the complex64 path on the same problem is two orders less accurate
    p64 = _plan([p], precision="c64")
    p64.set_contrast(0, W.round_f32(c["maps"]))
    r64 = p64.solve(p64.incident(c["src_ixz"], c["src_f"]), rtol=1e-7, maxit=500)
    assert _rel(_np(r64.x).ravel(), ud) < 1e-4


def test_c128_operators_match_oracle_to_rounding():
    """body force, G0 convolution, A u and the 2-D FFT on a two-problem plan with
    uneven grids (a 3 * 2^k size included)."""
    pa, ma = _vti(48, 32, 2, f=7.0, seed=5)
    pb, mb = _vti(64, 96, 3, f=4.0, seed=6, symbol="central")
    plan = _plan([pa, pb])
    plan.set_contrast(0, ma)
    plan.set_contrast(1, mb)
    rng = np.random.default_rng(11)
    parts = [rng.standard_normal((p["nsys"], 2, p["nz"], p["nx"]))
             + 1j * rng.standard_normal((p["nsys"], 2, p["nz"], p["nx"])) for p in (pa, pb)]
    u = plan.pack(parts)
    assert u.dtype == torch.complex128
    Au, b, g = plan.apply(u), plan.body_force(u), plan.convolve(u)
    for i, (p, m) in enumerate(((pa, ma), (pb, mb))):
        P = _oracle(p, m)
        assert _rel(_np(plan.view(Au, i)), P.apply(parts[i])) < OP_TOL
        assert _rel(_np(plan.view(b, i)), P.body_force(parts[i])) < OP_TOL
        assert _rel(_np(plan.view(g, i)), P.convolve(parts[i])) < OP_TOL
        F = plan.fft2(i, plan.view(u, i).contiguous())
        assert _rel(_np(F), np.fft.fft2(parts[i], axes=(-2, -1))) < OP_TOL


@pytest.mark.parametrize("krylov", ["bicgstab", "gmres"])
def test_c128_solve_batched_uneven_grids(krylov):
    pa, ma = _vti(48, 48, 3, f=6.0, seed=7, amp=0.1)
    pb, mb = _vti(96, 64, 2, f=9.0, seed=8, amp=0.1)
    plan = _plan([pa, pb])
    plan.set_contrast(0, ma)
    plan.set_contrast(1, mb)
    if krylov == "gmres":
        plan.set_krylov("gmres", restart=20)
    src, f = [], []
    for p in (pa, pb):
        s, ff = W.surface_sources(p["nx"], p["nsys"], iz=p["nz"] // 4)
        src += s
        f += ff
    print(f"c128 solve {krylov}", flush=True)
    u0 = plan.incident(src, f)
    res = plan.solve(u0, rtol=1e-10, maxit=3000)
    assert res.status == 0, (res.status, res.iters)
    assert np.all(res.relres <= 2e-10), res.relres
    k = 0
    for i, (p, m) in enumerate(((pa, ma), (pb, mb))):
        P = _oracle(p, m)
        ns = p["nsys"]
        uref, _ = P.solve(P.incident(src[k:k + ns], f[k:k + ns]), tol=1e-13)
        assert _rel(_np(plan.view(res.x, i)), uref) < 1e-8
        k += ns


def test_c128_frechet_adjoint_and_gradient_match_oracle():
    """J, J* and the Tikhonov gradient in complex128 against the oracle."""
    nx, nz, ns, nrec, freqs = 48, 32, 2, 6, (10.0, 14.0)
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0)
    maps = m0 * W.smooth_maps(31, nz, nx, 2.0, 0.08)
    src, f = W.surface_sources(nx, ns, iz=1)
    rec = W.surface_receivers(nx, nrec, iz=2)
    probs = [dict(nx=nx, nz=nz, dx=8.0, c0=tuple(c0), rho0=rho0, freq_hz=fr, eta=0.02, nsys=ns) for fr in freqs]
    plan = _plan(probs)
    for i in range(len(freqs)):
        plan.set_contrast(i, maps)
        plan.set_receivers(i, rec)
    ub = plan.solve(plan.incident(src * 2, f * 2), rtol=1e-12, maxit=2000).x
    items = []
    for fr in freqs:
        P = LSProblem(nx, nz, 8.0, c0, rho0, fr, 0.02, maps)
        ubr, _ = P.solve(P.incident(src, f), tol=1e-13)
        items.append((P, ubr, rec))
    for i in range(len(freqs)):
        assert _rel(_np(plan.view(ub, i)), items[i][1]) < 1e-10
    r_np = [W.complex_normal(40 + k, (ns, nrec, 2)) for k in range(len(freqs))]
    r = torch.as_tensor(np.concatenate([x.ravel() for x in r_np])).cuda()
    q = W.smooth_maps(33, nz, nx, 2.0, 0.02)
    qt = torch.as_tensor(q, dtype=torch.float64).cuda()
    T = tikhonov.Tikhonov(items, m0, r_np, lam=1e-3, reg="laplacian", tol=1e-13)
    d = plan.frechet_rel(ub, qt, m0.ravel(), rtol=1e-12).cpu().numpy()
    assert _rel(d, np.concatenate([x.ravel() for x in T.J(q)])) < 1e-9
    g = plan.adjoint_rel(ub, r, m0.ravel(), rtol=1e-12).cpu().numpy()
    assert _rel(g, np.real(T.Jstar(r_np))) < 1e-9
    fv, grad = plan.tikhonov_grad(ub, r, m0.ravel(), qt, lam=1e-3, reg="laplacian", rtol=1e-12)
    assert abs(fv - T.objective(q)) <= 1e-12 * abs(T.objective(q))
    assert _rel(grad.cpu().numpy(), T.gradient(q)) < 1e-9


def test_c64_normal_cg_against_c128_gpu_run():
    """The error of a complex64 normal-equation CG run stated against the same
    run in complex128 on the GPU (the reference used at sizes the CPU oracle
    cannot reach); here small enough to pin the complex128 run to the oracle.
    The data are those of a true perturbation, r = J q*, so that the normal
    operator Re J*J / ||r||^2 dominates lam and CG has work to do.  Partially
    converged CG iterates amplify operator differences by the conditioning of
    the Krylov basis, so the operators are compared tightly and the iterates
    after a few steps more loosely."""
    nx = nz = 48
    ns, nrec, freqs, niter = 3, 9, (4.0, 7.0), 3
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0)
    maps = W.round_f32(m0 * W.smooth_maps(7, nz, nx, 4.0, 0.08))
    qstar = W.round_f32(W.smooth_maps(8, nz, nx, 3.0, 0.02))
    src, f = W.surface_sources(nx, ns, iz=1)
    rec = W.surface_receivers(nx, nrec, iz=2)
    probs = [dict(nx=nx, nz=nz, dx=5.0, c0=tuple(c0), rho0=rho0, freq_hz=fr, eta=0.02, nsys=ns) for fr in freqs]
    items = []
    for fr in freqs:
        P = LSProblem(nx, nz, 5.0, c0, rho0, fr, 0.02, maps)
        ubr, _ = P.solve(P.incident(src, f), tol=1e-13)
        items.append((P, ubr, rec))
    r_np = tikhonov.Tikhonov(items, m0, [np.zeros((ns, nrec, 2))] * 2, lam=0.0, tol=1e-13).J(qstar)
    rr = sum(float(np.vdot(x.ravel(), x.ravel()).real) for x in r_np)
    out = {}
    for prec in ("c128", "c64"):
        print(f"normal CG {prec}", flush=True)
        plan = _plan(probs, precision=prec)
        for i in range(len(freqs)):
            plan.set_contrast(i, maps)
            plan.set_receivers(i, rec)
        tol = 1e-12 if prec == "c128" else 1e-7
        ub = plan.solve(plan.incident(src * 2, f * 2), rtol=tol, maxit=3000).x
        r = torch.as_tensor(np.concatenate([x.ravel() for x in r_np]).astype(
            np.complex128 if prec == "c128" else np.complex64)).cuda()
        qt = torch.as_tensor(qstar, dtype=plan.rdtype).cuda()
        Nq = plan.normal_apply(ub, m0.ravel(), rr, qt, lam=1e-3, reg="identity", rtol=tol)
        q, hist = plan.normal_cg(ub, r, m0.ravel(), niter=niter, lam=1e-3, reg="identity", rtol=tol)
        out[prec] = (q.double().cpu().numpy(), hist, Nq.double().cpu().numpy())
    T = tikhonov.Tikhonov(items, m0, r_np, lam=1e-3, reg="identity", tol=1e-13)
    q_ref, hist_ref = T.solve_cg(niter)
    assert hist_ref[-1] < 0.5 * hist_ref[0]   # CG does real work on this problem
    e128 = _rel(out["c128"][0], q_ref)
    assert _rel(out["c128"][2], T.normal_apply(qstar)) < 1e-9
    assert e128 < 1e-8, e128
    assert _rel(out["c128"][1], np.array(hist_ref)) < 1e-8
    # complex64 against the complex128 GPU run
    e_op = _rel(out["c64"][2], out["c128"][2])
    e_q = _rel(out["c64"][0], out["c128"][0])
    e_h = _rel(out["c64"][1], out["c128"][1])
    print(f"normal CG after {niter} steps: c128 vs oracle {e128:.2e}; c64 vs c128: N q {e_op:.2e}, "
          f"q {e_q:.2e}, residual history {e_h:.2e}", flush=True)
    assert e_op < 1e-5
    # measured 2.0e-6 (q) and 2.5e-7 (history) after 3 steps
    assert e_q < 2e-5 and e_h < 5e-6
