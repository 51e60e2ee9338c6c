"""GPU parity of every kernel variant the autotuner chooses from: the LS
matvec with each stencil, row-transform and column-pass candidate against
the complex128 oracle, and a solve after autotuning (different radix orders
only change fp32 rounding)."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import LSProblem

pytestmark = pytest.mark.gpu

KERNEL_TOL = 1e-5


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _case(nx, nz, nsys, seed=5):
    c0, rho0 = W.vti_background()
    maps = W.round_f32(W.model_scales(c0, rho0) * W.smooth_maps(seed, nz, nx, 3.0, 0.08))
    p = dict(nx=nx, nz=nz, dx=8.0, c0=c0, rho0=rho0, freq_hz=6.0, eta=0.02, nsys=nsys)
    return p, maps


# (1024, 32): the radix-32 row variant; (64, 1024): the 1024-thread column
# variant and the longest columns of the shared / split variants; (512, 64):
# the 512-point rows (radix-32, 16- and 8-point variants) and the fused
# stencil + rows kernels of that width, which the 512^2 workload runs;
# (64, 512), (128, 16): the LDS-twiddle column variants at those lengths
@pytest.mark.parametrize("nx,nz", [(96, 64), (64, 96), (256, 384), (1024, 32), (64, 1024), (512, 64), (128, 256),
                                   (64, 512), (128, 16)])
def test_every_variant_matches_oracle(nx, nz):
    from paper_2402_02116_amd.plan import Plan
    p, maps = _case(nx, nz, 2)
    plan = Plan([p])
    plan.set_contrast(0, maps)
    rng = np.random.default_rng(7)
    u = W.round_f32(rng.standard_normal((2, 2, nz, nx)) + 1j * rng.standard_normal((2, 2, nz, nx)))
    ut = plan.pack([u])
    P = LSProblem(nx, nz, 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, maps)
    ref = P.apply(u)
    default = plan.tuning(0)
    seen = 0
    for kind in ("stencil", "rows", "cols", "fuse"):
        cands = plan.tuning_candidates(0, kind)
        # rows of more than 512 points have no fused stencil + rows variant
        assert len(cands) >= (1 if kind == "fuse" and nx > 512 else 2), kind
        for c in cands:
            plan.set_tuning(0, **c)
            out = plan.view(plan.apply(ut), 0).cpu().numpy().astype(np.complex128)
            err = _rel(out, ref)
            assert err < KERNEL_TOL, (kind, c, err)
            seen += 1
        plan.set_tuning(0, **{k: default[k] for k in c})
    print(f"{nx}x{nz}: {seen} variants checked", flush=True)


def test_autotune_then_solve_matches_oracle():
    from paper_2402_02116_amd.plan import Plan
    cases = [_case(96, 48, 2, seed=8), _case(128, 128, 2, seed=9)]
    plan = Plan([c[0] for c in cases])
    for i, (_, m) in enumerate(cases):
        plan.set_contrast(i, m)
    tun = plan.autotune(reps=3)
    for t in tun:
        assert all(x > 0 for x in t["time_us"]), t
    src, f = [], []
    for p, _ in cases:
        s, fv = W.surface_sources(p["nx"], p["nsys"])
        src += s
        f += fv
    u0 = plan.incident(src, f)
    res = plan.solve(u0, rtol=1e-6, maxit=500)
    assert res.status == 0 and np.all(res.relres <= 2e-6)
    k = 0
    for i, (p, m) in enumerate(cases):
        P = LSProblem(p["nx"], p["nz"], 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, m)
        uref, _ = P.solve(P.incident(src[k:k + p["nsys"]], f[k:k + p["nsys"]]), tol=1e-11)
        assert _rel(plan.view(res.x, i).cpu().numpy().astype(np.complex128), uref) < 1e-4
        k += p["nsys"]


@pytest.mark.parametrize("nx,nz", [(256, 64), (384, 48), (512, 48)])
def test_fused_solves_match_oracle_and_plain(nx, nz):
    """Every fused stencil+rows variant (and the separate stencil) through a
    whole BiCGSTAB solve, its direction-update modes included (the 512-thread
    form of the closing mode where it exists), with every row-transform
    variant in both row passes (so every Krylov epilogue of the inverse rows
    runs in each radix sequence), against the oracle; and the batched solve
    bit-identical to the per-source one under the same variants."""
    from paper_2402_02116_amd.plan import Plan
    p, maps = _case(nx, nz, 3, seed=11)
    plan = Plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(nx, 3, iz=nz // 4)
    u0 = plan.incident(src, f)
    P = LSProblem(nx, nz, 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, maps)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    fuse = plan.tuning_candidates(0, "fuse")
    rows = [r["row_points"] for r in plan.tuning_candidates(0, "rows")]
    assert len(fuse) >= 2 and len(rows) >= 2
    worst = 0.0
    for c in fuse:
        for rp in rows:
            plan.set_tuning(0, **dict(c, row_points=rp, row_points_inv=rp))
            print(f"{nx}x{nz}: fused points {c['fused_points']}, row points {rp}", flush=True)
            res = plan.solve(u0, rtol=1e-6, maxit=500)
            assert res.status == 0 and np.all(res.relres <= 2e-6), (c, rp, res.relres)
            x = plan.view(res.x, 0).cpu().numpy().astype(np.complex128)
            for k in range(3):
                err = _rel(x[k], uref[k])
                worst = max(worst, err)
                assert err < 1e-4, (c, rp, k, err)
            plain = plan.solve(u0, rtol=1e-6, maxit=500, plain=True)
            assert torch.equal(res.x, plain.x) and np.array_equal(res.iters, plain.iters), (c, rp)
    print(f"{nx}x{nz}: {len(fuse) * len(rows)} solves, worst field error {worst:.2e}", flush=True)


@pytest.mark.parametrize("nx,nz", [(128, 96), (96, 64)])
def test_marching_stencil_solves_match_oracle_and_plain(nx, nz):
    """The z-marching form of the separate stencil (stencil_sys = -1, 4- and
    8-row steps) in every BiCGSTAB update mode: several strips and row ranges
    per system (64- and 48-column strips), three systems, against the oracle,
    and the batched solve bit-identical to the per-source one."""
    from paper_2402_02116_amd.plan import Plan
    p, maps = _case(nx, nz, 3, seed=13)
    plan = Plan([p])
    plan.set_contrast(0, maps)
    src, f = W.surface_sources(nx, 3, iz=nz // 3)
    u0 = plan.incident(src, f)
    P = LSProblem(nx, nz, 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, maps)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    march = [c for c in plan.tuning_candidates(0, "stencil") if c["stencil_sys"] == -1]
    assert sorted(c["stencil_rows"] for c in march) == [4, 8]
    for c in march:
        plan.set_tuning(0, **dict(c, fused_points=0))
        res = plan.solve(u0, rtol=1e-6, maxit=500)
        assert res.status == 0 and np.all(res.relres <= 2e-6), (c, res.relres)
        x = plan.view(res.x, 0).cpu().numpy().astype(np.complex128)
        errs = [_rel(x[k], uref[k]) for k in range(3)]
        print(f"{nx}x{nz} marching stencil, {c['stencil_rows']}-row steps: iterations {res.iters.tolist()}, "
              f"field errors {max(errs):.2e}", flush=True)
        assert max(errs) < 1e-4, (c, errs)
        plain = plan.solve(u0, rtol=1e-6, maxit=500, plain=True)
        assert torch.equal(res.x, plain.x) and np.array_equal(res.iters, plain.iters), c


@pytest.mark.parametrize("nx,nz", [(96, 64), (64, 256)])
def test_lds_twiddle_column_solves_match_oracle_and_plain(nx, nz):
    """The column pass with the twiddle table in LDS (col_shared 4: 4- and
    8-point columns, 4 to 16 columns per block) through whole BiCGSTAB solves
    of three systems that stop at different iterations (so blocks of stopped
    systems exit while the others run), against the oracle, and the batched
    solve bit-identical to the per-source one."""
    from paper_2402_02116_amd.plan import Plan
    p, maps = _case(nx, nz, 3, seed=17)
    plan = Plan([p])
    plan.set_contrast(0, maps)
    src, _ = W.surface_sources(nx, 3, iz=nz // 5)
    f = [(0.0, 1.0), (1.0, 0.0), (0.6, -0.8)]   # different force directions: different iteration counts
    u0 = plan.incident(src, f)
    P = LSProblem(nx, nz, 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, maps)
    uref, _ = P.solve(P.incident(src, f), tol=1e-11)
    tw = [c for c in plan.tuning_candidates(0, "cols") if c["col_shared"] == 4]
    assert {c["col_points"] for c in tw} == {4, 8}, tw
    for c in tw:
        plan.set_tuning(0, **c)
        res = plan.solve(u0, rtol=1e-6, maxit=500)
        assert res.status == 0 and np.all(res.relres <= 2e-6), (c, res.relres)
        x = plan.view(res.x, 0).cpu().numpy().astype(np.complex128)
        errs = [_rel(x[k], uref[k]) for k in range(3)]
        print(f"{nx}x{nz} LDS-twiddle columns P={c['col_points']} W={c['col_width']}: iterations "
              f"{res.iters.tolist()}, field errors {max(errs):.2e}", flush=True)
        assert max(errs) < 1e-4, (c, errs)
        plain = plan.solve(u0, rtol=1e-6, maxit=500, plain=True)
        assert torch.equal(res.x, plain.x) and np.array_equal(res.iters, plain.iters), c
