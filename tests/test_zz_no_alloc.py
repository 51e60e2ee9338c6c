"""fwils_apply_noalloc, the LS matvec (eq. A) with the library's static
scratch, called through the raw C ABI and compared with fwils_apply on the
same plan: two calls in a row, the second on a smaller plan and the other
stencil form, each bit-identical to fwils_apply (the same kernels) and
within the kernel tolerance of the complex128 oracle; and the refusal of a
plan whose fields exceed the static scratch."""

import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import LSProblem

pytestmark = pytest.mark.gpu

KERNEL_TOL = 1e-5


def _case(nx, nz, nsys, seed, fused_points):
    from paper_2402_02116_amd.plan import Plan
    c0, rho0 = W.vti_background()
    maps = W.round_f32(W.model_scales(c0, rho0) * W.smooth_maps(seed, nz, nx, 3.0, 0.08))
    p = dict(nx=nx, nz=nz, dx=8.0, c0=c0, rho0=rho0, freq_hz=6.0, eta=0.02, nsys=nsys)
    plan = Plan([p])
    plan.set_contrast(0, maps)
    plan.set_tuning(0, fused_points=fused_points)
    rng = np.random.default_rng(seed)
    u = W.round_f32(rng.standard_normal((nsys, 2, nz, nx)) + 1j * rng.standard_normal((nsys, 2, nz, nx)))
    return plan, p, maps, u


def _noalloc(plan, ut):
    """One fwils_apply_noalloc call through ctypes; (status, output)."""
    out = torch.full_like(ut, float("nan"))
    plan._bind_stream()
    st = plan.lib.fwils_apply_noalloc(plan._h, ctypes.c_void_p(ut.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    torch.cuda.synchronize()
    return st, out


def test_noalloc_matvec_matches_apply_on_two_calls():
    assert torch.cuda.is_available()
    # first call: 256^2 x 16 systems (the bench workload's size) with the
    # fused stencil + rows kernel; second: a smaller plan with the separate
    # stencil (the second scratch buffer), after the first left its data
    for nx, nz, nsys, seed, fp in ((256, 256, 16, 1, 16), (96, 64, 2, 2, 0)):
        plan, p, maps, u = _case(nx, nz, nsys, seed, fp)
        ut = plan.pack([u])
        print(f"apply_noalloc {nx}x{nz} x {nsys} systems, fused_points {fp}", flush=True)
        st, out = _noalloc(plan, ut)
        assert st == 0, plan.lib.fwils_last_error()
        ref = plan.apply(ut)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        P = LSProblem(nx, nz, 8.0, p["c0"], p["rho0"], p["freq_hz"], 0.02, maps)
        k = nsys - 1
        got = plan.view(out, 0)[k].cpu().numpy().astype(np.complex128)
        want = P.apply(u[k][None])[0]
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        assert err < KERNEL_TOL, err
        del plan


def test_noalloc_refuses_fields_beyond_the_static_scratch():
    from paper_2402_02116_amd import _lib
    plan, p, maps, u = _case(256, 256, 40, 3, 0)     # 5.2 Mi complex elements > 4 Mi
    ut = plan.pack([u])
    st, out = _noalloc(plan, ut)
    assert st == _lib.FWILS_EINVAL
    assert b"static scratch" in plan.lib.fwils_last_error()
    assert torch.isnan(out.real).all()             # refused before any launch
