"""Sequential-frequency distorted-Born inversion: the frequencies of an
inversion are taken one after the other from the lowest, each stage starting
from the model the previous one ended with (the sequential scheme of the
paper's numerical examples).  Each stage is one fwils_dbi_run call on a
single-frequency plan; this module only hands the model from plan to plan."""


def invert_sequential(plans, src_ixz, src_f, d_obs, contrast, m0, lam0=1e-3, niter=10, reg="identity",
                      tol=1e-3, max_outer=10, rtol=1e-6, maxit=1000):
    """plans: one Plan per frequency (single problem, receivers set), in the
    order of inversion; d_obs: the matching device data.  contrast: starting
    maps [5, nz, nx] (numpy or device tensor).  Returns (final contrast on the
    device, per-stage records with the frequency, eps_d history, lambdas,
    number of updates and status)."""
    if len(plans) != len(d_obs):
        raise ValueError("one observed-data tensor per plan")
    stages = []
    cur = contrast
    for plan, d in zip(plans, d_obs):
        plan.set_contrast(0, cur)
        out = plan.dbi_run(src_ixz, src_f, d, m0, lam0=lam0, niter=niter, reg=reg, tol=tol,
                           max_outer=max_outer, rtol=rtol, maxit=maxit)
        cur = plan.get_contrast(0)
        stages.append(dict(freq_hz=plan.problems[0]["freq_hz"], eps=out["eps"], lam=out["lam"],
                           updates=out["updates"], status=out["status"]))
    return cur, stages
