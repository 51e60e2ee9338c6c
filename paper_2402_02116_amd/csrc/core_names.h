// The library core (capi.cpp and the kernels) is compiled once per
// precision.  In a core build the C entry points and the plan type carry the
// precision in their names (fwils_solve_c64, fwils_solve_c128, ...); the
// public names are defined once, in abi.cpp, and dispatch on the plan's
// precision.  Include before fwils.h, after common.h (which defines FW_NS).
#pragma once

#define FW_CORE_PASTE2(a, b) a##_##b
#define FW_CORE_PASTE(a, b) FW_CORE_PASTE2(a, b)
#define FW_CORE(n) FW_CORE_PASTE(n, FW_NS)

#define fwils_plan_s FW_CORE(fwils_plan_s)
#define fwils_plan_create FW_CORE(fwils_plan_create)
#define fwils_plan_destroy FW_CORE(fwils_plan_destroy)
#define fwils_workspace_size FW_CORE(fwils_workspace_size)
#define fwils_set_workspace FW_CORE(fwils_set_workspace)
#define fwils_set_stream FW_CORE(fwils_set_stream)
#define fwils_field_elems FW_CORE(fwils_field_elems)
#define fwils_set_contrast FW_CORE(fwils_set_contrast)
#define fwils_set_receivers FW_CORE(fwils_set_receivers)
#define fwils_incident FW_CORE(fwils_incident)
#define fwils_body_force FW_CORE(fwils_body_force)
#define fwils_convolve FW_CORE(fwils_convolve)
#define fwils_apply FW_CORE(fwils_apply)
#define fwils_apply_noalloc FW_CORE(fwils_apply_noalloc)
#define fwils_solve FW_CORE(fwils_solve)
#define fwils_frechet FW_CORE(fwils_frechet)
#define fwils_adjoint FW_CORE(fwils_adjoint)
#define fwils_apply_pass FW_CORE(fwils_apply_pass)
#define fwils_time_pass FW_CORE(fwils_time_pass)
#define fwils_time_krylov_pass FW_CORE(fwils_time_krylov_pass)
#define fwils_solve_stats FW_CORE(fwils_solve_stats)
#define fwils_solve_status FW_CORE(fwils_solve_status)
#define fwils_tikhonov_grad FW_CORE(fwils_tikhonov_grad)
#define fwils_normal_apply FW_CORE(fwils_normal_apply)
#define fwils_normal_cg FW_CORE(fwils_normal_cg)
#define fwils_frechet_rel FW_CORE(fwils_frechet_rel)
#define fwils_adjoint_rel FW_CORE(fwils_adjoint_rel)
#define fwils_laplacian FW_CORE(fwils_laplacian)
#define fwils_receiver_data FW_CORE(fwils_receiver_data)
#define fwils_get_contrast FW_CORE(fwils_get_contrast)
#define fwils_dbi_run FW_CORE(fwils_dbi_run)
#define fwils_fft2 FW_CORE(fwils_fft2)
#define fwils_gmres_workspace_size FW_CORE(fwils_gmres_workspace_size)
#define fwils_set_krylov FW_CORE(fwils_set_krylov)
#define fwils_autotune FW_CORE(fwils_autotune)
#define fwils_get_tuning FW_CORE(fwils_get_tuning)
#define fwils_set_tuning FW_CORE(fwils_set_tuning)
#define fwils_tuning_candidates FW_CORE(fwils_tuning_candidates)
