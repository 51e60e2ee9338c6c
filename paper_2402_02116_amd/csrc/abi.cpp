// The public C entry points of fwils.h.  The library core is compiled twice
// (complex64 and complex128); each build exports its entry points under
// precision-suffixed names (fwils_solve_c64, fwils_solve_c128, ...).  Every
// public function here forwards to the build that matches the plan's
// precision, which both plan types store as their first member.  The
// thread-local error text and the status strings live here, once.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/fwils.h"

// Every entry point that takes a plan (or creates one):
// X(return type, name without the fwils_ prefix, parameters, arguments).
#define FW_ABI_ENTRIES(X)                                                                                  \
    X(fwils_status, workspace_size, (fwils_plan plan, size_t* bytes), (plan, bytes))                     \
    X(fwils_status, set_workspace, (fwils_plan plan, void* dev, size_t bytes), (plan, dev, bytes))       \
    X(fwils_status, set_stream, (fwils_plan plan, void* hip_stream), (plan, hip_stream))                 \
    X(fwils_status, field_elems, (fwils_plan plan, int64_t* elems), (plan, elems))                       \
    X(fwils_status, set_contrast, (fwils_plan plan, int32_t iprob, const void* maps), (plan, iprob, maps)) \
    X(fwils_status, set_receivers, (fwils_plan plan, int32_t iprob, const int32_t* rec_ixz, int32_t nrec), \
      (plan, iprob, rec_ixz, nrec))                                                                        \
    X(fwils_status, incident, (fwils_plan plan, const int32_t* src_ixz, const double* src_f, void* u0),   \
      (plan, src_ixz, src_f, u0))                                                                          \
    X(fwils_status, body_force, (fwils_plan plan, const void* u, void* b), (plan, u, b))                 \
    X(fwils_status, convolve, (fwils_plan plan, const void* f, void* out), (plan, f, out))               \
    X(fwils_status, apply, (fwils_plan plan, const void* u, void* Au), (plan, u, Au))                    \
    X(fwils_status, apply_noalloc, (fwils_plan plan, const void* u, void* Au), (plan, u, Au))            \
    X(fwils_status, solve,                                                                                 \
      (fwils_plan plan, const void* rhs, void* x, double rtol, int32_t maxit, int32_t* iters,            \
       double* relres, uint32_t flags),                                                                    \
      (plan, rhs, x, rtol, maxit, iters, relres, flags))                                                   \
    X(fwils_status, frechet,                                                                               \
      (fwils_plan plan, const void* ub, const void* const* dm, void* d, double rtol, int32_t maxit),      \
      (plan, ub, dm, d, rtol, maxit))                                                                      \
    X(fwils_status, adjoint,                                                                               \
      (fwils_plan plan, const void* ub, const void* r, void* const* g, uint32_t flags, double rtol,       \
       int32_t maxit),                                                                                     \
      (plan, ub, r, g, flags, rtol, maxit))                                                                \
    X(fwils_status, apply_pass, (fwils_plan plan, int32_t pass, const void* u, void* Au),                 \
      (plan, pass, u, Au))                                                                                 \
    X(fwils_status, time_pass,                                                                             \
      (fwils_plan plan, int32_t pass, const void* u, void* Au, int32_t reps, float* us),                  \
      (plan, pass, u, Au, reps, us))                                                                       \
    X(fwils_status, time_krylov_pass, (fwils_plan plan, int32_t reps, float* us), (plan, reps, us))       \
    X(fwils_status, time_gmres_pass, (fwils_plan plan, int32_t kind, int32_t j, int32_t reps, float* us),  \
      (plan, kind, j, reps, us))                                                                           \
    X(fwils_status, solve_stats, (fwils_plan plan, int32_t* iters, double* relres), (plan, iters, relres)) \
    X(fwils_status, solve_status, (fwils_plan plan, int32_t* status), (plan, status))                    \
    X(fwils_status, tikhonov_grad,                                                                         \
      (fwils_plan plan, const void* ub, const void* r, const double* m0, double lam, int32_t reg,         \
       const void* q, void* grad, double* fval, void* dscratch, double rtol, int32_t maxit),              \
      (plan, ub, r, m0, lam, reg, q, grad, fval, dscratch, rtol, maxit))                                  \
    X(fwils_status, normal_apply,                                                                          \
      (fwils_plan plan, const void* ub, const double* m0, double rr, double lam, int32_t reg,             \
       const void* q_in, void* q_out, void* dscratch, double rtol, int32_t maxit),                        \
      (plan, ub, m0, rr, lam, reg, q_in, q_out, dscratch, rtol, maxit))                                   \
    X(fwils_status, normal_cg,                                                                             \
      (fwils_plan plan, const void* ub, const void* r, const double* m0, double lam, int32_t reg,         \
       int32_t niter, void* q, double* hist, void* dscratch, double rtol, int32_t maxit),                 \
      (plan, ub, r, m0, lam, reg, niter, q, hist, dscratch, rtol, maxit))                                 \
    X(fwils_status, normal_cg_steps,                                                                       \
      (fwils_plan plan, const void* ub, const void* r, const double* m0, double lam, int32_t reg,         \
       int32_t first, int32_t niter, void* q, double* hist, void* q_iters, void* dscratch, double rtol,  \
       int32_t maxit),                                                                                     \
      (plan, ub, r, m0, lam, reg, first, niter, q, hist, q_iters, dscratch, rtol, maxit))                 \
    X(fwils_status, frechet_rel,                                                                           \
      (fwils_plan plan, const void* ub, const void* q, const double* m0, void* d, double rtol,            \
       int32_t maxit),                                                                                     \
      (plan, ub, q, m0, d, rtol, maxit))                                                                   \
    X(fwils_status, adjoint_rel,                                                                           \
      (fwils_plan plan, const void* ub, const void* r, const double* m0, void* gq, double rtol,           \
       int32_t maxit),                                                                                     \
      (plan, ub, r, m0, gq, rtol, maxit))                                                                  \
    X(fwils_status, laplacian, (fwils_plan plan, const void* q, void* out), (plan, q, out))              \
    X(fwils_status, receiver_data, (fwils_plan plan, const void* u, void* d), (plan, u, d))              \
    X(fwils_status, get_contrast, (fwils_plan plan, int32_t iprob, void* maps), (plan, iprob, maps))     \
    X(fwils_status, dbi_run,                                                                               \
      (fwils_plan plan, const int32_t* src_ixz, const double* src_f, const void* d_obs, const double* m0, \
       double lam0, int32_t reg, int32_t niter, double tol, int32_t max_outer, void* ub, void* r, void* q, \
       void* dscratch, double* eps_hist, double* lam_hist, int32_t* updates, double rtol, int32_t maxit),  \
      (plan, src_ixz, src_f, d_obs, m0, lam0, reg, niter, tol, max_outer, ub, r, q, dscratch, eps_hist,   \
       lam_hist, updates, rtol, maxit))                                                                    \
    X(fwils_status, fft2, (fwils_plan plan, int32_t iprob, const void* in, void* out, int32_t inverse),  \
      (plan, iprob, in, out, inverse))                                                                     \
    X(fwils_status, gmres_workspace_size, (fwils_plan plan, int32_t restart, size_t* bytes),             \
      (plan, restart, bytes))                                                                              \
    X(fwils_status, set_krylov,                                                                            \
      (fwils_plan plan, int32_t method, int32_t restart, uint32_t flags, void* gws, size_t bytes),        \
      (plan, method, restart, flags, gws, bytes))                                                          \
    X(fwils_status, autotune, (fwils_plan plan, int32_t reps), (plan, reps))                             \
    X(fwils_status, get_tuning, (fwils_plan plan, int32_t iprob, fwils_tuning* out), (plan, iprob, out)) \
    X(fwils_status, set_tuning, (fwils_plan plan, int32_t iprob, const fwils_tuning* t), (plan, iprob, t)) \
    X(fwils_status, tuning_candidates,                                                                     \
      (fwils_plan plan, int32_t iprob, int32_t kind, fwils_tuning* out, int32_t cap, int32_t* count),     \
      (plan, iprob, kind, out, cap, count))

// The per-precision entry points (C linkage: only the names matter here).
#define FW_DECLARE(R, N, P, A) R fwils_##N##_c64 P; R fwils_##N##_c128 P;
extern "C" {
FW_ABI_ENTRIES(FW_DECLARE)
fwils_status fwils_plan_create_c64(const fwils_problem* probs, int32_t nprob, fwils_precision prec,
                                   fwils_plan* out);
fwils_status fwils_plan_create_c128(const fwils_problem* probs, int32_t nprob, fwils_precision prec,
                                    fwils_plan* out);
fwils_status fwils_plan_create3_c64(const fwils_problem3* probs, int32_t nprob, fwils_precision prec,
                                    fwils_plan* out);
fwils_status fwils_plan_create3_c128(const fwils_problem3* probs, int32_t nprob, fwils_precision prec,
                                     fwils_plan* out);
void fwils_plan_destroy_c64(fwils_plan plan);
void fwils_plan_destroy_c128(fwils_plan plan);
}
#undef FW_DECLARE

namespace {

thread_local std::string g_last_error;

void set_error(const char* msg) { g_last_error = msg; }

// A null plan goes to the complex64 build, which reports it.
bool is_c128(fwils_plan plan) { return plan && *reinterpret_cast<const int32_t*>(plan) == FWILS_C128; }

}  // namespace

extern "C" {

__attribute__((visibility("default"))) void fwils_internal_set_error(const char* msg) { set_error(msg); }

int32_t fwils_abi_version(void) { return FWILS_ABI_VERSION; }

const char* fwils_status_string(fwils_status s) {
    switch (s) {
        case FWILS_OK: return "ok";
        case FWILS_EINVAL: return "invalid argument";
        case FWILS_ENOMEM: return "workspace missing or too small";
        case FWILS_EDEVICE: return "HIP device error";
        case FWILS_ENOCONV: return "not converged";
        case FWILS_EBREAKDOWN: return "Krylov breakdown";
        case FWILS_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* fwils_last_error(void) { return g_last_error.c_str(); }

fwils_status fwils_plan_create(const fwils_problem* probs, int32_t nprob, fwils_precision prec,
                               fwils_plan* out) {
    if (prec == FWILS_C64) return fwils_plan_create_c64(probs, nprob, prec, out);
    if (prec == FWILS_C128) return fwils_plan_create_c128(probs, nprob, prec, out);
    set_error("plan_create: unknown precision");
    return FWILS_EINVAL;
}

fwils_status fwils_plan_create3(const fwils_problem3* probs, int32_t nprob, fwils_precision prec,
                                fwils_plan* out) {
    if (prec == FWILS_C64) return fwils_plan_create3_c64(probs, nprob, prec, out);
    if (prec == FWILS_C128) return fwils_plan_create3_c128(probs, nprob, prec, out);
    set_error("plan_create3: unknown precision");
    return FWILS_EINVAL;
}

void fwils_plan_destroy(fwils_plan plan) {
    if (!plan) return;
    if (is_c128(plan)) fwils_plan_destroy_c128(plan);
    else fwils_plan_destroy_c64(plan);
}

#define FW_DISPATCH(R, N, P, A) \
    R fwils_##N P { return is_c128(plan) ? fwils_##N##_c128 A : fwils_##N##_c64 A; }
FW_ABI_ENTRIES(FW_DISPATCH)
#undef FW_DISPATCH

}  // extern "C"
