"""The timing entry of the BiCGSTAB direction-update pass: it runs the pass
with every system active, restores the solver's state, and refuses states
that are not those of a finished BiCGSTAB solve."""

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

NX = NZ = 64
NSYS = 4


def _plan(fused=True):
    from paper_2402_02116_amd.plan import Plan
    c0, rho0 = W.vti_background()
    m0 = W.model_scales(c0, rho0).reshape(5, 1, 1)
    plan = Plan([dict(nx=NX, nz=NZ, dx=10.0, c0=tuple(c0), rho0=rho0, freq_hz=20.0, eta=0.02, nsys=NSYS)])
    plan.set_contrast(0, W.round_f32(m0 * W.smooth_maps(3, NZ, NX, 3.0, 0.05)))
    fp = [c["fused_points"] for c in plan.tuning_candidates(0, "fuse") if c["fused_points"]]
    plan.set_tuning(0, fused_points=fp[0] if fused else 0)
    src = [(8 + 12 * i, 3 + i) for i in range(NSYS)]
    return plan, plan.incident(src, [(0.0, 1.0)] * NSYS)


@pytest.mark.parametrize("fused", [True, False])
def test_direction_update_pass_timing_restores_state(fused):
    print(f"time_krylov_pass fused={fused}", flush=True)
    from paper_2402_02116_amd._lib import FwilsError
    plan, u0 = _plan(fused)
    assert (plan.tuning(0)["fused_points"] != 0) == fused
    with pytest.raises(FwilsError):      # no solve yet
        plan.time_krylov_pass(3)
    res = plan.solve(u0, rtol=1e-12, maxit=6)
    it0, rr0 = plan.solve_stats()
    st0 = plan.solve_status()
    assert list(st0) == ["maxit"] * NSYS and np.all(it0 >= 6)
    us = plan.time_krylov_pass(5)
    assert np.isfinite(us) and us > 0.0
    it1, rr1 = plan.solve_stats()
    assert np.array_equal(it0, it1) and np.array_equal(rr0, rr1) and list(plan.solve_status()) == list(st0)
    # the next solve starts afresh and converges as before
    full = plan.solve(u0, rtol=1e-6, maxit=2000)
    ref_plan, ref_u0 = _plan(fused)
    ref = ref_plan.solve(ref_u0, rtol=1e-6, maxit=2000)
    assert full.status == 0 and torch.equal(full.x, ref.x)
    del res


def test_direction_update_pass_timing_refuses_gmres():
    from paper_2402_02116_amd._lib import FwilsError
    plan, u0 = _plan()
    plan.set_krylov("gmres", restart=8)
    plan.solve(u0, rtol=1e-12, maxit=6)
    with pytest.raises(FwilsError):
        plan.time_krylov_pass(3)
    plan.set_krylov("bicgstab")         # the workspace holds a GMRES state
    with pytest.raises(FwilsError):
        plan.time_krylov_pass(3)
