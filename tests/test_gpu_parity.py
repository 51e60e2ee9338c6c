"""GPU parity: the HIP path (through the C ABI) against the complex128 CPU
oracle, element by element on seeded inputs, plus properties that hold at
any size.  Tolerances: complex64 FFT / stencil kernels <= 1e-5 relative
(fp32 rounding, a few ulp times log n), solved fields and J / J* <= 1e-4
relative (the field target), true residuals <= 2x the requested tolerance."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import LSProblem, operators

pytestmark = pytest.mark.gpu

KERNEL_TOL = 1e-5
FIELD_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2402_02116_amd import _lib
    _lib.load()          # fail loudly if the HIP library is missing
    yield
    torch.cuda.synchronize()


def _plan(problems):
    from paper_2402_02116_amd.plan import Plan
    return Plan(problems)


def _pd(nx, nz, dx, c0, rho0, f, nsys, eta=0.02, symbol="spectral"):
    return dict(nx=nx, nz=nz, dx=dx, c0=tuple(c0), rho0=rho0, freq_hz=f, eta=eta, nsys=nsys, symbol=symbol)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _oracle(p, maps):
    return LSProblem(p["nx"], p["nz"], p["dx"], p["c0"], p["rho0"], p["freq_hz"], p["eta"], maps,
                     symbol=p["symbol"])


def _vti_case(nx, nz, nsys, dx=8.0, f=6.0, seed=3, amp=0.08, ell=3.0, symbol="spectral"):
    c0, rho0 = W.vti_background()
    maps = W.round_f32(W.model_scales(c0, rho0) * W.smooth_maps(seed, nz, nx, ell, amp))
    return _pd(nx, nz, dx, c0, rho0, f, nsys, symbol=symbol), maps


def _cfield(rng, shape):
    return W.round_f32(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def _to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


# ------------------------------------------------------------------ FFT ----
FFT_SHAPES = [(16, 16), (24, 48), (32, 64), (48, 48), (64, 32), (96, 192), (128, 128), (192, 384),
              (256, 256), (384, 384), (512, 512), (768, 256), (1024, 1024), (1536, 64), (2048, 2048)]


@pytest.mark.parametrize("nx,nz", FFT_SHAPES)
def test_fft2_matches_numpy(nx, nz):
    """The Stockham row / column kernels give the unnormalised DFT (eq. FFT)."""
    p, _ = _vti_case(nx, nz, 1 if nx * nz > 512 * 512 else 2)
    plan = _plan([p])
    rng = np.random.default_rng(nx * 7 + nz)
    x = _cfield(rng, (p["nsys"], 2, nz, nx))
    xt = torch.as_tensor(x.astype(np.complex64)).cuda()
    X = _to_np(plan.fft2(0, xt))
    ref = np.fft.fft2(x, axes=(-2, -1))
    assert _rel(X, ref) < 2e-6
    Y = _to_np(plan.fft2(0, xt, inverse=True))
    refi = np.fft.ifft2(x, axes=(-2, -1)) * (nx * nz)
    assert _rel(Y, refi) < 2e-6


# ------------------------------------------------------------- operators --
OP_SHAPES = [(32, 32), (48, 24), (64, 128), (96, 96), (256, 128)]


@pytest.mark.parametrize("nx,nz", OP_SHAPES)
def test_body_force_matches_oracle(nx, nz):
    """Contrast stencil b = w~^2 drho u + div_h(dC : E_h u) (eqs. Ewave0, u_2)."""
    p, maps = _vti_case(nx, nz, 3, ell=1.0, amp=0.2)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    rng = np.random.default_rng(5)
    u = _cfield(rng, (3, 2, nz, nx))
    b = _to_np(plan.view(plan.body_force(plan.pack([u])), 0))
    ref = _oracle(p, maps).body_force(u)
    assert _rel(b, ref) < KERNEL_TOL


@pytest.mark.parametrize("nx,nz", OP_SHAPES)
def test_convolve_and_apply_match_oracle(nx, nz):
    """G0 conv f (eq. FFT with the Christoffel-inverse symbol) and A u (eq. A)."""
    p, maps = _vti_case(nx, nz, 2)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    P = _oracle(p, maps)
    rng = np.random.default_rng(6)
    u = _cfield(rng, (2, 2, nz, nx))
    ut = plan.pack([u])
    conv = _to_np(plan.view(plan.convolve(ut), 0))
    assert _rel(conv, P.convolve(u)) < KERNEL_TOL
    Au = _to_np(plan.view(plan.apply(ut), 0))
    assert _rel(Au, P.apply(u)) < KERNEL_TOL


def test_central_symbol_matches_oracle():
    p, maps = _vti_case(64, 48, 2, symbol="central")
    plan = _plan([p])
    plan.set_contrast(0, maps)
    rng = np.random.default_rng(7)
    u = _cfield(rng, (2, 2, 48, 64))
    Au = _to_np(plan.view(plan.apply(plan.pack([u])), 0))
    assert _rel(Au, _oracle(p, maps).apply(u)) < KERNEL_TOL


def test_incident_matches_oracle():
    """u0 = G0 conv s for point forces (eq. u0), several systems and directions."""
    p, maps = _vti_case(96, 64, 3)
    plan = _plan([p])
    src = [(5, 0), (50, 31), (95, 63)]
    force = [(0.0, 1.0), (1.0, 0.0), (0.6, -0.8)]
    u0 = _to_np(plan.view(plan.incident(src, force), 0))
    ref = _oracle(p, maps).incident(src, force)
    assert _rel(u0, ref) < KERNEL_TOL


def test_scattered_field_output_matches_oracle():
    """FWILS_SOLVE_SCATTERED: the library returns u_s = u - u0 (the split
    u = u0 + u_s of eq. delu), formed on the device; against the oracle's
    u - u0 per system, and in place over the incident field."""
    p, maps = _vti_case(96, 64, 3, amp=0.1)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(96, 3, iz=5)
    u0 = plan.incident(src, f)
    tot = plan.solve(u0, rtol=1e-7, maxit=500)
    sc = plan.solve(u0, rtol=1e-7, maxit=500, scattered=True)
    assert tot.status == 0 and sc.status == 0
    assert torch.equal(sc.x, tot.x - u0)        # the same solve, one fp32 subtraction
    buf = u0.clone()
    inplace = plan.solve(buf, rtol=1e-7, maxit=500, scattered=True, out=buf)
    assert torch.equal(inplace.x, sc.x)
    P = _oracle(p, maps)
    u0r = P.incident(src, f)
    uref, _ = P.solve(u0r, tol=1e-12)
    us = _to_np(plan.view(sc.x, 0))
    for k in range(3):
        assert _rel(us[k], uref[k] - u0r[k]) < FIELD_TOL, k


# ---------------------------------------------------------------- solves --
def test_solve_iso32_blob_matches_oracle():
    """32^2 isotropic background, Gaussian blob, 10 Hz: c64 BiCGSTAB vs the
    oracle's solution (itself pinned to a dense direct solve)."""
    c = W.iso32_blob()
    p = _pd(c["nx"], c["nz"], c["dx"], c["c0"], c["rho0"], c["freq_hz"], 1)
    plan = _plan([p])
    plan.set_contrast(0, c["maps"])
    u0 = plan.incident(c["src_ixz"], c["src_f"])
    res = plan.solve(u0, rtol=1e-7, maxit=200)
    assert res.status == 0 and res.relres[0] < 2e-7
    P = _oracle(p, c["maps"])
    uref, _ = P.solve(P.incident(c["src_ixz"], c["src_f"]), tol=1e-12)
    assert _rel(_to_np(plan.view(res.x, 0)), uref) < FIELD_TOL


@pytest.mark.parametrize("nx,nz,nsys", [(48, 96, 3), (128, 64, 2), (24, 24, 1)])
def test_solve_rectangular_vti_matches_oracle(nx, nz, nsys):
    p, maps = _vti_case(nx, nz, nsys, amp=0.1)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(nx, nsys, iz=nz // 3)
    u0 = plan.incident(src, f)
    res = plan.solve(u0, rtol=1e-6, maxit=500)
    assert res.status == 0
    assert np.all(res.relres < 2e-6)
    P = _oracle(p, maps)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    u = _to_np(plan.view(res.x, 0))
    for k in range(nsys):
        assert _rel(u[k], uref[k]) < FIELD_TOL


@pytest.mark.parametrize("nx,nz", [(2048, 16), (16, 2048)])
def test_solve_at_the_extreme_grid_shapes(nx, nz):
    """The longest supported rows and columns (2048 points) against the
    oracle, with the autotuner's choice of variants."""
    p, maps = _vti_case(nx, nz, 2, amp=0.08, seed=17)
    print(f"extreme shape {nx}x{nz}", flush=True)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    plan.autotune(reps=2)
    src = [(nx // 3, nz // 3), (2 * nx // 3, 2 * nz // 3)]
    f = [(0.0, 1.0), (1.0, 0.0)]
    res = plan.solve(plan.incident(src, f), rtol=1e-7, maxit=1000)
    assert res.status == 0
    P = _oracle(p, maps)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    u = _to_np(plan.view(res.x, 0))
    for k in range(2):
        assert _rel(u[k], uref[k]) < FIELD_TOL


def test_many_systems_on_a_small_grid():
    """256 systems of 32 x 32 (blocks, partial records and graph chunks at
    a large batch): every system converges; a sample matches the oracle."""
    nsys = 256
    p, maps = _vti_case(32, 32, nsys, amp=0.1, seed=19)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    src = [(s % 32, (s // 32) % 32) for s in range(nsys)]
    f = [(float(np.cos(s)), float(np.sin(s))) for s in range(nsys)]
    res = plan.solve(plan.incident(src, f), rtol=1e-6, maxit=500)
    assert res.status == 0 and np.all(res.relres < 2e-6)
    P = _oracle(p, maps)
    pick = [0, 97, 255]
    uref, _ = P.solve(P.incident([src[k] for k in pick], [f[k] for k in pick]), tol=1e-11)
    u = _to_np(plan.view(res.x, 0))
    for i, k in enumerate(pick):
        assert _rel(u[k], uref[i]) < FIELD_TOL


def test_solve_vti256_full_size_sampled():
    """256^2 VTI, 16 sources, 5 Hz at full size, batched c64 to 1e-6:
    every true residual <= 2e-6; three of the systems against the oracle."""
    c = W.vti256_layered()
    p = _pd(c["nx"], c["nz"], c["dx"], c["c0"], c["rho0"], c["freq_hz"], c["nsys"])
    plan = _plan([p])
    plan.set_contrast(0, c["maps"])
    u0 = plan.incident(c["src_ixz"], c["src_f"])
    res = plan.solve(u0, rtol=1e-6, maxit=500)
    assert res.status == 0
    assert np.all(res.relres <= 2e-6), res.relres
    P = _oracle(p, c["maps"])
    u = _to_np(plan.view(res.x, 0))
    for k in (0, 7, 15):
        uref, _ = P.solve(P.incident([c["src_ixz"][k]], [c["src_f"][k]]), tol=1e-10)
        assert _rel(u[k], uref[0]) < FIELD_TOL


def test_batched_equals_per_source_and_repeatable():
    """The batched graph solve, the non-graph solve and the plain per-source
    solve run the same kernels system by system: identical results."""
    p, maps = _vti_case(128, 128, 4, amp=0.1)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(128, 4)
    u0 = plan.incident(src, f)
    a = plan.solve(u0, rtol=1e-6, maxit=300)
    b = plan.solve(u0, rtol=1e-6, maxit=300)
    c = plan.solve(u0, rtol=1e-6, maxit=300, graph=False)
    d = plan.solve(u0, rtol=1e-6, maxit=300, plain=True)
    assert torch.equal(a.x, b.x)
    assert torch.equal(a.x, c.x)
    assert torch.equal(a.x, d.x)
    assert np.array_equal(a.iters, d.iters)


def test_zero_contrast_returns_incident_field():
    p, _ = _vti_case(64, 64, 2)
    plan = _plan([p])
    u0 = plan.incident([(3, 4), (40, 9)], [(0.0, 1.0), (1.0, 0.0)])
    res = plan.solve(u0, rtol=1e-6, maxit=10)
    assert res.status == 0 and np.all(res.iters <= 1)
    assert _rel(_to_np(res.x), _to_np(u0)) < 1e-6


def test_x0_warm_start_and_zero_rhs():
    p, maps = _vti_case(64, 64, 2, amp=0.1)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    u0 = plan.incident([(3, 0), (40, 0)], [(0.0, 1.0), (0.0, 1.0)])
    first = plan.solve(u0, rtol=1e-6, maxit=300)
    warm = plan.solve(u0, x0=first.x, rtol=1e-5, maxit=300)
    assert np.all(warm.iters == 0) and np.all(warm.relres < 2e-6)
    zero = plan.solve(plan.new_field(), rtol=1e-6, maxit=10)
    assert zero.status == 0 and np.all(zero.relres == 0) and not torch.any(zero.x != 0)


def test_maxit_reports_noconv():
    from paper_2402_02116_amd import _lib
    p, maps = _vti_case(64, 64, 2, amp=0.2)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    u0 = plan.incident([(3, 0), (40, 0)], [(0.0, 1.0), (0.0, 1.0)])
    res = plan.solve(u0, rtol=1e-12, maxit=2)
    assert res.status == _lib.FWILS_ENOCONV
    assert np.all(res.iters == 2)


def test_multi_problem_plan_matches_oracle():
    """Uneven grids and frequencies in one plan (one graph chunk covers all)."""
    c0, rho0 = W.vti_background()
    q = W.random_layered(2, 96, 96)
    cases = [(64, 64, 12.0, 6.0, 2), (96, 48, 8.0, 9.0, 3), (128, 128, 6.0, 5.0, 1)]
    probs, maps_l, src_l, f_l = [], [], [], []
    for nx, nz, dx, f, ns in cases:
        m = W.round_f32(W.model_scales(c0, rho0) * W.resample_periodic(q, nz, nx))
        probs.append(_pd(nx, nz, dx, c0, rho0, f, ns))
        maps_l.append(m)
        s, fv = W.surface_sources(nx, ns)
        src_l += s
        f_l += fv
    plan = _plan(probs)
    for i, m in enumerate(maps_l):
        plan.set_contrast(i, m)
    u0 = plan.incident(src_l, f_l)
    res = plan.solve(u0, rtol=1e-6, maxit=500)
    assert res.status == 0 and np.all(res.relres <= 2e-6)
    k = 0
    for i, (p, m) in enumerate(zip(probs, maps_l)):
        P = _oracle(p, m)
        ns = p["nsys"]
        uref, _ = P.solve(P.incident(src_l[k:k + ns], f_l[k:k + ns]), tol=1e-11)
        assert _rel(_to_np(plan.view(res.x, i)), uref) < FIELD_TOL
        k += ns


def test_solve_multigrid_full_size_oracle_residual():
    """Four grids (128^2 .. 384^2, 4 .. 12 Hz, 64 sources each) in one plan,
    batched c64 to 1e-6.  Every reported true residual <= 2e-6; on sampled
    systems of every grid the complex128 oracle operator gives the same
    bound for the returned field; the smallest grid is also solved by the
    oracle and compared field to field."""
    probs = W.four_grids()
    pds = [_pd(c["nx"], c["nz"], c["dx"], c["c0"], c["rho0"], c["freq_hz"], c["nsys"]) for c in probs]
    plan = _plan(pds)
    src, fv = [], []
    for i, c in enumerate(probs):
        plan.set_contrast(i, c["maps"])
        src += c["src_ixz"]
        fv += c["src_f"]
    u0 = plan.incident(src, fv)
    res = plan.solve(u0, rtol=1e-6, maxit=1500)
    assert res.status == 0, (res.status, res.iters)
    assert np.all(res.relres <= 2e-6), res.relres.max()
    for i, (c, p) in enumerate(zip(probs, pds)):
        P = _oracle(p, c["maps"])
        b = _to_np(plan.view(u0, i))
        x = _to_np(plan.view(res.x, i))
        for k in (0, c["nsys"] // 2, c["nsys"] - 1):
            rel = np.linalg.norm(b[k] - P.apply(x[k][None])[0]) / np.linalg.norm(b[k])
            assert rel <= 3e-6, (c["nx"], k, rel)
        if i == 0:
            uref, _ = P.solve(b[:1], tol=1e-10)
            assert _rel(x[0], uref[0]) < FIELD_TOL


def test_reciprocity_gpu():
    """G^b_ij(x, x') = G^b_ji(x', x) on a heterogeneous background (App. B)."""
    p, maps = _vti_case(96, 96, 4, amp=0.12)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    xa, xb = (10, 7), (70, 50)
    src = [xb, xb, xa, xa]
    force = [(1.0, 0.0), (0.0, 1.0), (1.0, 0.0), (0.0, 1.0)]
    res = plan.solve(plan.incident(src, force), rtol=1e-7, maxit=500)
    u = _to_np(plan.view(res.x, 0))
    for i in range(2):
        for j in range(2):
            gij = u[j][i, xa[1], xa[0]]        # force j at xb, component i at xa
            gji = u[2 + i][j, xb[1], xb[0]]    # force i at xa, component j at xb
            assert abs(gij - gji) <= 1e-4 * max(abs(gij), abs(gji))


# ------------------------------------------------------------ J and J* ----
def _jj_setup(nx=48, nz=32, nsys=2, nrec=6, seed=21):
    c0, rho0 = W.vti_background()
    maps = W.round_f32(W.model_scales(c0, rho0) * W.smooth_maps(seed, nz, nx, 2.0, 0.08))
    p = _pd(nx, nz, 8.0, c0, rho0, 12.0, nsys)
    plan = _plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(nx, nsys, iz=1)
    rec = W.surface_receivers(nx, nrec, iz=2)
    plan.set_receivers(0, rec)
    ub = plan.solve(plan.incident(src, f), rtol=1e-7, maxit=500).x
    return plan, p, maps, src, f, rec, ub, W.model_scales(c0, rho0)


def test_frechet_and_adjoint_match_oracle():
    plan, p, maps, src, f, rec, ub, m0 = _jj_setup()
    P = _oracle(p, maps)
    ub_ref, _ = P.solve(P.incident(src, f), tol=1e-12)
    rng = np.random.default_rng(3)
    dm = W.round_f32(m0 * W.smooth_maps(4, p["nz"], p["nx"], 2.0, 0.05))
    d = plan.frechet(ub, [torch.as_tensor(dm, dtype=torch.float32).cuda()], rtol=1e-7)
    d_ref = P.frechet(ub_ref, dm, rec, tol=1e-12)
    assert _rel(_to_np(plan.data_view(d, 0)), d_ref) < FIELD_TOL
    r = _cfield(rng, (p["nsys"], len(rec), 2))
    g = plan.adjoint(ub, torch.as_tensor(r.astype(np.complex64).ravel()).cuda(), rtol=1e-7)
    g_ref = P.adjoint(ub_ref, r, rec, tol=1e-12)
    gg = _to_np(g[0])
    for k in range(5):
        assert _rel(gg[k], g_ref[k]) < FIELD_TOL, k


def test_adjoint_dot_product_gpu():
    """<r, J dm> = <J* r, dm> for the HIP J and J* at 128^2 with 4 systems."""
    plan, p, maps, src, f, rec, ub, m0 = _jj_setup(128, 128, 4, 21, seed=9)
    rng = np.random.default_rng(11)
    dm = W.round_f32(m0 * rng.standard_normal((5, 128, 128)))
    r = _cfield(rng, (4, 21, 2))
    d = _to_np(plan.frechet(ub, [torch.as_tensor(dm, dtype=torch.float32).cuda()], rtol=1e-7))
    g = _to_np(plan.adjoint(ub, torch.as_tensor(r.astype(np.complex64).ravel()).cuda(), rtol=1e-7)[0])
    lhs = np.vdot(r.ravel(), d)
    rhs = np.vdot(g.ravel(), dm.ravel())
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_adjoint_with_repeated_receivers_matches_oracle():
    """J* with receivers listed out of cell order and several on one cell:
    the scatter sums each cell's receivers (R^T adds repeats, eq. ua0); the
    result against the oracle and against the same data pre-summed on the
    distinct receivers."""
    plan, p, maps, src, f, rec, ub, m0 = _jj_setup(nrec=6)
    rep = [rec[4], rec[1], rec[4], rec[0]] + list(reversed(rec))
    plan.set_receivers(0, rep)
    P = _oracle(p, maps)
    ub_ref, _ = P.solve(P.incident(src, f), tol=1e-12)
    rng = np.random.default_rng(17)
    r = _cfield(rng, (p["nsys"], len(rep), 2))
    g = _to_np(plan.adjoint(ub, torch.as_tensor(r.astype(np.complex64).ravel()).cuda(), rtol=1e-7)[0])
    g_ref = P.adjoint(ub_ref, r, rep, tol=1e-12)
    for k in range(5):
        assert _rel(g[k], g_ref[k]) < FIELD_TOL, k
    # the same data summed per distinct receiver cell
    uniq = sorted(set(map(tuple, rep)))
    rs = np.zeros((p["nsys"], len(uniq), 2), dtype=np.complex128)
    for j, c in enumerate(rep):
        rs[:, uniq.index(tuple(c))] += r[:, j].astype(np.complex64).astype(np.complex128)
    plan.set_receivers(0, uniq)
    g2 = _to_np(plan.adjoint(ub, torch.as_tensor(rs.astype(np.complex64).ravel()).cuda(), rtol=1e-7)[0])
    for k in range(5):
        assert _rel(g[k], g2[k]) < 1e-5, k
