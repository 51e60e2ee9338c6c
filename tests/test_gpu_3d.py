"""GPU parity of the 3-D, generally anisotropic path (fwils_plan_create3)
against the complex128 3-D oracle (oracle/elastic3d.py): the 3-D FFT with
radix-5 lengths against numpy, the contrast stencil, convolution, operator,
incident field, batched BiCGSTAB and GMRES solves, J and J* in both the VTI
(C11, C13, C33, C55, C66, rho; App. C) and the general 21-constant
parametrisation (eq. dC), the one-cell-thick grid (d/dy = 0), the
complex128 build, and the 80 x 40 x 32 grid of the paper's 3-D example.
Tolerances as for 2-D: kernels <= 1e-5, solved fields and J / J* <= 1e-4."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import elastic3d as E3

pytestmark = pytest.mark.gpu

KERNEL_TOL = 1e-5
FIELD_TOL = 1e-4


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _case(nx, ny, nz, nsys, params="vti", freq=8.0, dx=10.0, seed=3, precision="c64"):
    from paper_2402_02116_amd.plan import Plan3
    if params == "vti":
        c21, rho = W.vti3d_background(gamma=0.1)
        maps = W.round_f32(W.contrast3(seed, nz, ny, nx, W.vti3d_scales(gamma=0.1), std=0.06))
    else:
        c21, rho = W.triclinic_background(seed)
        maps = W.round_f32(W.contrast3(seed, nz, ny, nx, W.general_scales(c21, rho), std=0.03))
    p = dict(nx=nx, ny=ny, nz=nz, dx=dx, c0=c21, rho0=rho, freq_hz=freq, eta=0.02, nsys=nsys, params=params)
    plan = Plan3([p], precision=precision)
    plan.set_contrast(0, maps)
    P = E3.LSProblem3D(nx, ny, nz, dx, c21, rho, freq, 0.02, maps=maps, params=params)
    return plan, p, maps, P


def _field(rng, nsys, nx, ny, nz):
    shape = (nsys, 3, nz, ny, nx)
    return W.round_f32(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2402_02116_amd import _lib
    _lib.load()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("nx,ny,nz", [(16, 16, 16), (20, 24, 40), (80, 40, 32), (48, 1, 64), (160, 20, 16)])
def test_fft3_matches_numpy(nx, ny, nz):
    """x rows, strided y and z passes, radix 2/3/4/5/8/16 (unnormalised both ways)."""
    plan, p, _, _ = _case(nx, ny, nz, 2)
    x = _field(np.random.default_rng(1), 2, nx, ny, nz)
    xt = torch.as_tensor(x.astype(np.complex64)).cuda()
    f = _np(plan.fft3(0, xt))
    ref = np.fft.fftn(x, axes=(-3, -2, -1))
    assert _rel(f, ref) < KERNEL_TOL
    b = _np(plan.fft3(0, torch.as_tensor(ref.astype(np.complex64)).cuda(), inverse=True))
    assert _rel(b, x * nx * ny * nz) < KERNEL_TOL


@pytest.mark.parametrize("params", ["vti", "general"])
def test_body_force_apply_incident_3d(params):
    nx, ny, nz = 24, 20, 16
    plan, p, maps, P = _case(nx, ny, nz, 2, params)
    u = _field(np.random.default_rng(2), 2, nx, ny, nz)
    ut = plan.pack([u])
    assert _rel(_np(plan.view(plan.body_force(ut), 0)), P.body_force(u)) < KERNEL_TOL
    assert _rel(_np(plan.view(plan.convolve(ut), 0)), P.convolve(u)) < KERNEL_TOL
    assert _rel(_np(plan.view(plan.apply(ut), 0)), P.apply(u)) < KERNEL_TOL
    assert torch.equal(plan.apply_noalloc(ut), plan.apply(ut))
    src = [(3, 5, 0), (20, 11, 9)]
    f = [(0.0, 0.0, 1.0), (0.3, -0.6, 0.7)]
    assert _rel(_np(plan.view(plan.incident(src, f), 0)), P.incident(src, f)) < KERNEL_TOL


@pytest.mark.parametrize("nx,ny,nz", [(24, 20, 16), (32, 40, 16), (32, 32, 16), (64, 24, 16)])
def test_marching_stencil_column_shapes(nx, ny, nz):
    """The z-marching stencil's column shapes (16 x 16 with and without
    overhang, 32 x 8) against the oracle's contrast stencil."""
    print(f"3-D stencil {nx}x{ny}x{nz}", flush=True)
    plan, p, maps, P = _case(nx, ny, nz, 2)
    u = _field(np.random.default_rng(4), 2, nx, ny, nz)
    ut = plan.pack([u])
    assert _rel(_np(plan.view(plan.body_force(ut), 0)), P.body_force(u)) < KERNEL_TOL


@pytest.mark.parametrize("params", ["vti", "general"])
def test_solve_3d_matches_oracle_batched_plain_gmres(params):
    nx, ny, nz = 24, 20, 16
    plan, p, maps, P = _case(nx, ny, nz, 3, params)
    src = [(4, 3, 0), (12, 10, 0), (20, 17, 2)]
    f = [(0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 0.6, 0.8)]
    u0 = plan.incident(src, f)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    res = plan.solve(u0, rtol=1e-6, maxit=800)
    assert res.status == 0 and np.all(res.relres <= 2e-6), (res.status, res.relres)
    u = _np(plan.view(res.x, 0))
    errs = [_rel(u[k], uref[k]) for k in range(3)]
    print(f"3-D {params} BiCGSTAB iters {res.iters.tolist()} field errors {errs}", flush=True)
    assert max(errs) < FIELD_TOL
    plain = plan.solve(u0, rtol=1e-6, maxit=800, plain=True)
    assert torch.equal(res.x, plain.x) and np.array_equal(res.iters, plain.iters)
    sc = plan.solve(u0, rtol=1e-6, maxit=800, scattered=True)
    assert torch.equal(sc.x, res.x - u0)
    plan.set_krylov("gmres", restart=20)
    g = plan.solve(u0, rtol=1e-6, maxit=800)
    assert g.status == 0
    ug = _np(plan.view(g.x, 0))
    assert max(_rel(ug[k], uref[k]) for k in range(3)) < FIELD_TOL


@pytest.mark.parametrize("params", ["vti", "general"])
def test_frechet_and_adjoint_3d_match_oracle(params):
    nx, ny, nz = 20, 16, 16
    plan, p, maps, P = _case(nx, ny, nz, 2, params, freq=7.0)
    src = [(5, 4, 0), (14, 11, 0)]
    f = [(0.0, 0.0, 1.0), (0.0, 1.0, 0.0)]
    # out of cell order, one cell twice (the adjoint scatter adds repeats)
    rec = list(reversed(W.surface_grid(nx, ny, 5, 4, iz=1)))
    rec.insert(3, rec[7])
    plan.set_receivers(0, rec)
    ub = plan.solve(plan.incident(src, f), rtol=1e-7, maxit=800).x
    ub_ref, _ = P.solve(P.incident(src, f), tol=1e-12)
    rng = np.random.default_rng(5)
    scales = W.vti3d_scales(0.1) if params == "vti" else W.general_scales(p["c0"], p["rho0"])
    dm = W.round_f32(W.contrast3(6, nz, ny, nx, scales, std=0.05))
    d = plan.frechet(ub, [torch.as_tensor(dm, dtype=torch.float32).cuda()], rtol=1e-7)
    d_ref = P.frechet(ub_ref, dm, rec, tol=1e-12)
    err_j = _rel(_np(plan.data_view(d, 0)), d_ref)
    r = W.round_f32(rng.standard_normal((2, len(rec), 3)) + 1j * rng.standard_normal((2, len(rec), 3)))
    g = _np(plan.adjoint(ub, torch.as_tensor(r.astype(np.complex64).ravel()).cuda(), rtol=1e-7)[0])
    g_ref = P.adjoint(ub_ref, r, rec, tol=1e-12)
    err_g = max(_rel(g[k], g_ref[k]) for k in range(g.shape[0]))
    lhs = np.vdot(r.ravel(), _np(d))
    rhs = np.vdot(g.ravel(), dm.ravel())
    print(f"3-D {params}: J {err_j:.2e}, J* worst map {err_g:.2e}, dot {abs(lhs - rhs) / abs(lhs):.2e}",
          flush=True)
    assert err_j < FIELD_TOL and err_g < FIELD_TOL
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_one_cell_thick_grid_general_medium():
    """ny = 1: the x-z plane with all three components coupled by a triclinic
    background and contrast."""
    nx, ny, nz = 48, 1, 32
    plan, p, maps, P = _case(nx, ny, nz, 2, "general", freq=9.0)
    src, f = [(7, 0, 0), (30, 0, 5)], [(0.0, 0.0, 1.0), (0.5, 0.5, 0.0)]
    res = plan.solve(plan.incident(src, f), rtol=1e-7, maxit=800)
    assert res.status == 0
    uref, _ = P.solve(P.incident(src, f), tol=1e-12)
    assert _rel(_np(plan.view(res.x, 0)), uref) < FIELD_TOL


def test_complex128_build_3d():
    nx, ny, nz = 20, 16, 24
    plan, p, maps, P = _case(nx, ny, nz, 2, "general", precision="c128")
    src, f = [(2, 3, 0), (15, 9, 4)], [(0.0, 0.0, 1.0), (1.0, 1.0, 0.0)]
    res = plan.solve(plan.incident(src, f), rtol=1e-11, maxit=1500)
    assert res.status == 0
    uref, _ = P.solve(P.incident(src, f), tol=1e-12)
    assert _rel(_np(plan.view(res.x, 0)), uref) < 1e-9


def test_many_systems_source_upload_3d():
    """128 systems: the cell indices and forces of every source reach the
    device intact (the forces follow the indices in the workspace), checked
    on the incident fields of the last systems."""
    nx, ny, nz = 16, 16, 16
    plan, p, maps, P = _case(nx, ny, nz, 128)
    src = [(k % nx, (3 * k) % ny, (5 * k) % nz) for k in range(128)]
    f = [(0.1 * (k % 3), 0.2, 1.0 - 0.01 * k) for k in range(128)]
    u0 = _np(plan.view(plan.incident(src, f), 0))
    for k in (0, 85, 100, 127):
        assert _rel(u0[k], P.incident([src[k]], [f[k]])[0]) < KERNEL_TOL, k


def test_hess3d_grid_sampled_against_oracle():
    """The 80 x 40 x 32 grid of 25 m cells of the paper's 3-D example, 100
    vertical surface forces at 7 Hz: every true residual <= 2e-6 and two
    systems against the oracle."""
    from paper_2402_02116_amd.plan import Plan3
    w = W.hess3d_vti()
    plan = Plan3([dict(nx=w["nx"], ny=w["ny"], nz=w["nz"], dx=w["dx"], c0=w["c0"], rho0=w["rho0"],
                       freq_hz=w["freq_hz"], eta=w["eta"], nsys=w["nsys"], params="vti")])
    plan.set_contrast(0, w["maps"])
    print("80x40x32 x 100 systems", flush=True)
    res = plan.solve(plan.incident(w["src_ixyz"], w["src_f"]), rtol=1e-6, maxit=1500)
    assert res.status == 0 and np.all(res.relres <= 2e-6), (res.status, res.relres.max())
    P = E3.LSProblem3D(w["nx"], w["ny"], w["nz"], w["dx"], w["c0"], w["rho0"], w["freq_hz"], w["eta"],
                       maps=w["maps"], params="vti")
    u = _np(plan.view(res.x, 0))
    for k in (0, 57):
        uref, _ = P.solve(P.incident([w["src_ixyz"][k]], [w["src_f"][k]]), tol=1e-10)
        err = _rel(u[k], uref[0])
        print(f"  system {k}: iters {res.iters[k]}, field error {err:.2e}", flush=True)
        assert err < FIELD_TOL


def test_tikhonov_normal_cg_and_dbi_update_3d():
    """3-D VTI plan of two frequencies on one grid: the Tikhonov objective and
    gradient with the 7-point Laplacian, three normal-equation CG iterations
    (L = I) and one distorted-Born update from the homogeneous background,
    each against the oracle (eqs. obj, norm and the DBI loop)."""
    from oracle import dbi, tikhonov
    from paper_2402_02116_amd.plan import Plan3
    nx, ny, nz, dx = 16, 16, 16, 10.0
    c21, rho = W.vti3d_background(gamma=0.1)
    m0 = W.vti3d_scales(gamma=0.1)
    maps = W.round_f32(W.contrast3(21, nz, ny, nx, m0, std=0.05))
    freqs, ns = (6.0, 9.0), 2
    src, f = [(4, 5, 0), (11, 10, 0)], [(0.0, 0.0, 1.0), (0.0, 0.5, 0.8)]
    rec = W.surface_grid(nx, ny, 4, 4, iz=1)
    probs = [dict(nx=nx, ny=ny, nz=nz, dx=dx, c0=c21, rho0=rho, freq_hz=fr, eta=0.02, nsys=ns, params="vti")
             for fr in freqs]
    plan = Plan3(probs)
    for i in range(2):
        plan.set_contrast(i, maps)
        plan.set_receivers(i, rec)
    ub = plan.solve(plan.incident(src * 2, f * 2), rtol=1e-7, maxit=800).x
    items = []
    for fr in freqs:
        P = E3.LSProblem3D(nx, ny, nz, dx, c21, rho, fr, 0.02, maps=maps, params="vti")
        items.append((P, P.solve(P.incident(src, f), tol=1e-12)[0], rec))
    rng = np.random.default_rng(22)
    r_np = [W.round_f32(rng.standard_normal((ns, len(rec), 3)) + 1j * rng.standard_normal((ns, len(rec), 3)))
            for _ in freqs]
    r = torch.as_tensor(np.concatenate([x.ravel() for x in r_np]).astype(np.complex64)).cuda()
    q = W.round_f32(W.contrast3(23, nz, ny, nx, np.ones((6, 1, 1, 1)), std=0.02))
    qt = torch.as_tensor(q, dtype=torch.float32).cuda()
    m0v = m0.ravel()
    T = tikhonov.Tikhonov(items, m0, r_np, lam=1e-3, reg="laplacian", tol=1e-12)
    fval, g = plan.tikhonov_grad(ub, r, m0v, qt, lam=1e-3, reg="laplacian", rtol=1e-7)
    e_g = _rel(g.double().cpu().numpy(), T.gradient(q))
    e_f = abs(fval - T.objective(q)) / abs(T.objective(q))
    Ti = tikhonov.Tikhonov(items, m0, r_np, lam=1e-3, reg="identity", tol=1e-12)
    qo, ho = Ti.solve_cg(3)
    qc, hc = plan.normal_cg(ub, r, m0v, niter=3, lam=1e-3, reg="identity", rtol=1e-7)
    e_q = _rel(qc.double().cpu().numpy(), qo)
    e_h = _rel(hc, np.array(ho))
    print(f"3-D Tikhonov: objective {e_f:.2e}, gradient {e_g:.2e}; CG q {e_q:.2e}, history {e_h:.2e}", flush=True)
    assert e_f < 1e-5 and e_g < 1e-4 and e_q < 1e-4 and e_h < 1e-4
    # one distorted-Born update from the homogeneous background towards `maps`
    d_obs = [E3.sample_3d(ub_ref, rec) for (_, ub_ref, _) in items]
    pd = Plan3(probs)
    for i in range(2):
        pd.set_receivers(i, rec)
    d_t = torch.as_tensor(np.concatenate([W.round_f32(x).ravel() for x in d_obs]).astype(np.complex64)).cuda()
    out = pd.dbi_run(src * 2, f * 2, d_t, m0v, lam0=1.0, niter=3, tol=0.0, max_outer=1, rtol=1e-7, maxit=800)
    zero = np.zeros_like(maps)
    its = [(E3.LSProblem3D(nx, ny, nz, dx, c21, rho, fr, 0.02, params="vti"), src, f, rec, W.round_f32(d))
           for fr, d in zip(freqs, d_obs)]
    c1, eps, _, _ = dbi.dbi_stage(its, zero, m0v, 1.0, 3, tol=0.0, max_outer=1, solve_tol=1e-12)
    step = pd.get_contrast(0).double().cpu().numpy()
    e_c = _rel(step, c1)
    e_e = _rel(np.array(out["eps"]), np.array(eps))
    print(f"3-D DBI update: eps {out['eps']} vs {eps}; model step {e_c:.2e}", flush=True)
    assert out["updates"] == 1 and e_c < 1e-3 and e_e < 1e-4
