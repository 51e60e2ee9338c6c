/*
 * fwils.h -- C ABI of the MI355X library for the matrix-free elastic
 * Lippmann-Schwinger (LS) solve and the Frechet / adjoint operators of the
 * distorted-Born method of Xiang, Jakobsen, Shekhar, Eikrem and Naevdal,
 * arXiv 2402.02116.
 *
 * Problem.  A 2-D (x-z) periodic grid of nx * nz square cells of size dx
 * carries a homogeneous background stiffness C0 (Voigt C11, C13, C33, C55;
 * VTI or isotropic) and density rho0 (eq. decom), a contrast dC(x), drho(x),
 * and one frequency f with complex frequency w~ = 2 pi f (1 + i eta).  The
 * displacement u solves eq. u_2 written as A u = u0 (eqs. A, axb):
 *
 *     A u = u - G0 conv b(u),   b(u) = w~^2 drho u + div_h( dC : E_h u ),
 *
 * where E_h is the Voigt strain built from 2nd-order central differences,
 * div_h = -E_h^T is the matching divergence (the integration by parts of eq.
 * dgv, exact on the torus), and G0 conv f = IFFT2( G_hat(k) FFT2(f) ) is the
 * circular convolution of eq. FFT with the wavenumber-domain Green's tensor
 * G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1 (Fourier transform of eq. Green;
 * Gamma is the Christoffel matrix of C0).  For even n, products of two
 * different wavenumber components use k = 0 at the Nyquist index so that
 * G_hat is even in k and G0 symmetric.
 *
 * One plan holds one or more problems ("grids"); each has nsys systems
 * (sources) that share its grid, background, frequency and contrast.
 *
 * Precision.  A plan is complex64 (FWILS_C64: complex64 fields and data,
 * float32 maps) or complex128 (FWILS_C128: complex128 fields and data,
 * float64 maps, the FP64 reference of the same path).  Krylov scalars, inner
 * products and norms are FP64 in both.  "complex" and "real" below are the
 * plan's types.
 *
 * Memory layout (all row-major, x fastest):
 *   field      complex [nsys][2][nz][nx], component 0 = u_x, 1 = u_z,
 *              interleaved (re, im).  A plan-level field is the
 *              concatenation of its problems' fields in problem order;
 *              fwils_field_elems gives its length in complex elements.
 *   maps       real [5][nz][nx], absolute units, order
 *              (dC11, dC13, dC33, dC55, drho) in Pa and kg/m^3.
 *   data       complex [nsys][nrec][2] per problem, concatenated.
 *   sources,   host int32 [n][2] as (ix, iz); forces host double [n][2]
 *   receivers  as (fx, fz) in newtons.
 *
 * Ownership and execution.
 *   All field, map and data pointers are DEVICE pointers owned by the caller
 *   and must stay valid until the stream has finished the call.  Index and
 *   force arrays are host pointers copied during the call.  The plan owns
 *   small host metadata only; device scratch is the caller-provided
 *   workspace (fwils_workspace_size / fwils_set_workspace), which the plan
 *   uses until it is destroyed or given another workspace.  Every call is
 *   asynchronous on the plan's stream (fwils_set_stream; default: the null
 *   stream) unless stated otherwise.  A plan is not thread-safe; separate
 *   plans are independent.
 *
 * Errors.  Every call returns fwils_status.  Argument errors (FWILS_EINVAL)
 * are detected before any work is enqueued and leave no side effects.  HIP
 * runtime failures give FWILS_EDEVICE; fwils_last_error() returns a
 * thread-local text with details.  Non-convergence is not an abort: outputs
 * are written and FWILS_ENOCONV is returned.
 */
#ifndef FWILS_H
#define FWILS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWILS_ABI_VERSION 8

typedef enum {
    FWILS_OK = 0,
    FWILS_EINVAL = 1,        /* bad argument, shape or state                  */
    FWILS_ENOMEM = 2,        /* workspace missing or too small                */
    FWILS_EDEVICE = 3,       /* HIP runtime error                             */
    FWILS_ENOCONV = 4,       /* some system did not reach the tolerance       */
    FWILS_EBREAKDOWN = 5,    /* Krylov breakdown or non-finite residual       */
    FWILS_EUNSUPPORTED = 6   /* valid request the library does not implement   */
} fwils_status;

typedef enum {
    FWILS_C64 = 0,           /* complex64 fields, fp32 maps, FP64 reductions  */
    FWILS_C128 = 1           /* complex128 fields, fp64 maps (FP64 reference) */
} fwils_precision;

typedef enum {
    FWILS_SYMBOL_SPECTRAL = 0,   /* exact wavenumbers in Gamma(k)              */
    FWILS_SYMBOL_CENTRAL = 1     /* k -> sin(k dx)/dx: G0 inverts the discrete
                                    background operator exactly (eq. Ewave)    */
} fwils_symbol;

/* One (grid, frequency) problem. */
typedef struct {
    int32_t nx, nz;      /* cells; each 2^a 3^b with 16 <= n <= 2048        */
    double  dx;          /* cell size (m), both axes                        */
    double  c0[4];       /* background Voigt C11, C13, C33, C55 (Pa)        */
    double  rho0;        /* background density (kg/m^3)                     */
    double  freq_hz;     /* frequency f (Hz)                                */
    double  damping;     /* eta in w~ = 2 pi f (1 + i eta); eta > 0         */
    int32_t nsys;        /* systems (sources) on this problem, >= 1         */
    int32_t symbol;      /* fwils_symbol                                    */
} fwils_problem;

/* One 3-D (grid, frequency) problem with a general anisotropic background
 * (the 21 elastic constants of the abbreviated subscript section; eq. decom)
 * and a contrast in one of two parametrisations (eq. dC):
 *   FWILS_PARAMS_VTI:     maps [6][nz][ny][nx] = (dC11, dC13, dC33, dC55, dC66,
 *                         drho) with App. C's B matrices (dC12 = dC11 - 2 dC66,
 *                         dC22 = dC11, dC23 = dC13, dC44 = dC55);
 *   FWILS_PARAMS_GENERAL: maps [22][nz][ny][nx] = the 21 constants of the upper
 *                         triangle of the 6 x 6 matrix in row-major order (C11,
 *                         C12, ..., C16, C22, ..., C66), then drho.
 * Fields of a 3-D plan are complex [nsys][3][nz][ny][nx] (u_x, u_y, u_z);
 * sources, forces and receivers are [n][3] as (ix, iy, iz) and (fx, fy, fz),
 * a point force F is F / dx^3 at its cell; data are [nsys][nrec][3].  The
 * operator is eq. A with the six-strain Voigt stencil, G_hat(k) the inverse of
 * the damped 3 x 3 Christoffel matrix of the background (products of two
 * different wavenumber components use k = 0 at an even axis's Nyquist
 * index).  Axis lengths 2^a 3^b 5^c from 16 to 256 (16, 20, 24, 32, 40, 48,
 * 64, 80, 96, 128, 160, 192, 256); ny = 1 gives the 2-D plane with all three
 * displacement components (d/dy = 0). */
#define FWILS_PARAMS_VTI 0
#define FWILS_PARAMS_GENERAL 1
typedef struct {
    int32_t nx, ny, nz;  /* cells per axis                                  */
    double  dx;          /* cell size (m), all axes                         */
    double  c0[21];      /* background C11, C12, ..., C16, C22, ..., C66 (Pa);
                            the 6 x 6 matrix must be positive definite       */
    double  rho0;        /* background density (kg/m^3)                     */
    double  freq_hz;     /* frequency f (Hz)                                */
    double  damping;     /* eta in w~ = 2 pi f (1 + i eta); eta > 0         */
    int32_t nsys;        /* systems (sources) on this problem, >= 1         */
    int32_t symbol;      /* fwils_symbol                                    */
    int32_t params;      /* FWILS_PARAMS_VTI or FWILS_PARAMS_GENERAL        */
} fwils_problem3;

typedef struct fwils_plan_s* fwils_plan;

/* Solve flags. */
#define FWILS_SOLVE_X0       0x1u  /* x holds the initial guess (else x0 = 0)   */
#define FWILS_SOLVE_PLAIN    0x2u  /* per-source loop, host-synchronous
                                      convergence check every iteration (the
                                      plain baseline; same kernels, nsys = 1)  */
#define FWILS_SOLVE_NOGRAPH  0x4u  /* batched, but launched without HIP graphs */
#define FWILS_SOLVE_SCATTERED 0x8u /* x receives u - rhs instead of u: with
                                      rhs = u0 (fwils_incident) this is the
                                      scattered field u_s = u - u0 of eq.
                                      delu's decomposition u = u0 + u_s */

/* Adjoint flags. */
#define FWILS_ADJ_ACCUMULATE 0x1u  /* add into g instead of overwriting        */

/* Create a plan for nprob problems (validated; nothing is allocated on the
 * device).  On success *out receives the plan. */
fwils_status fwils_plan_create(const fwils_problem* probs, int32_t nprob,
                               fwils_precision prec, fwils_plan* out);
void fwils_plan_destroy(fwils_plan plan);
/* A plan of 3-D problems (all problems of a plan are 2-D or all 3-D).  The
 * same entry points apply to it with the 3-D layouts above: workspace,
 * stream, contrast, receivers, incident, body force, convolve, apply,
 * apply_noalloc, solve (BiCGSTAB or GMRES), frechet, adjoint (complex128 maps
 * [nmaps][nz][ny][nx]), receiver_data, get_contrast, field_elems, solve
 * statistics, fft2 (the 3-D transform) and the Tikhonov / normal-equation /
 * DBI entry points (maps [nmaps][nz][ny][nx], m0 [nmaps], the 7-point
 * Laplacian); fwils_apply_pass / fwils_time_pass time its passes (0: stencil,
 * 1: x transforms, 2: the y, z-with-Green and y transforms, 3: inverse x
 * transforms with the epilogue).  The tuning and Krylov-pass timing entry
 * points return FWILS_EUNSUPPORTED for it; fwils_autotune leaves its problems
 * unchanged. */
fwils_status fwils_plan_create3(const fwils_problem3* probs, int32_t nprob, fwils_precision prec,
                                fwils_plan* out);

/* Bytes of device workspace the plan needs (256-byte aligned start). */
fwils_status fwils_workspace_size(fwils_plan plan, size_t* bytes);
/* Hand the plan its workspace.  Synchronous: initialises constant tables and
 * zero contrasts in it. */
fwils_status fwils_set_workspace(fwils_plan plan, void* dev, size_t bytes);
/* Stream for all later work (a hipStream_t; NULL = null stream). */
fwils_status fwils_set_stream(fwils_plan plan, void* hip_stream);
/* Complex elements in one plan-level field: sum_p nsys_p * 2 * nz_p * nx_p. */
fwils_status fwils_field_elems(fwils_plan plan, int64_t* elems);

/* Contrast of problem iprob (eqs. decom, key): copies the five maps
 * [5][nz][nx] (device, fp32, absolute units) into the workspace. */
fwils_status fwils_set_contrast(fwils_plan plan, int32_t iprob, const void* maps);

/* Receivers of problem iprob: host int32 [nrec][2] (ix, iz), 1 <= nrec <= 65536.
 * Copied into the workspace (synchronous). */
fwils_status fwils_set_receivers(fwils_plan plan, int32_t iprob,
                                 const int32_t* rec_ixz, int32_t nrec);

/* Incident field u0 = G0 conv s (eq. u0) for one point force per system:
 * s = F / dx^2 at cell (ix, iz).  src_ixz, src_f: host [sum nsys][2].
 * u0: device field (output). */
fwils_status fwils_incident(fwils_plan plan, const int32_t* src_ixz,
                            const double* src_f, void* u0);

/* b(u) = w~^2 drho u + div_h(dC : E_h u): the contrast body force (the
 * right-hand side of eq. Ewave0 without S).  u, b: device fields. */
fwils_status fwils_body_force(fwils_plan plan, const void* u, void* b);

/* out = G0 conv f (eq. FFT).  f, out: device fields (may alias). */
fwils_status fwils_convolve(fwils_plan plan, const void* f, void* out);

/* Au = u - G0 conv b(u) (eq. A), one batched application.  u, Au: device
 * fields, must not alias. */
fwils_status fwils_apply(fwils_plan plan, const void* u, void* Au);

/* fwils_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same kernels and result as fwils_apply, with the FFT scratch field and the
 * separate stencil's output in a static device array of the library (64 MiB
 * per GPU and precision build, held until the process ends) instead of the
 * workspace's two scratch vectors.  Allocates nothing (no hipMalloc / free).
 * Needs 2 * align256(field bytes) <= 64 MiB: fields of at most 4 Mi complex
 * elements (complex64) or 2 Mi (complex128); FWILS_EINVAL beyond that, or if
 * the current device is not the plan's workspace's device.  The plan's
 * workspace still holds its constant tables and contrast.  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other plans, other threads) race and must be serialised by the
 * caller.  Nothing in the array needs clearing between calls. */
fwils_status fwils_apply_noalloc(fwils_plan plan, const void* u, void* Au);

/* Solve A x = rhs for every system by the plan's Krylov method (eq. axb;
 * BiCGSTAB unless fwils_set_krylov chose GMRES), vectors of the plan's
 * precision and FP64 inner products.  Stops each system when its recursive residual
 * satisfies ||r|| <= rtol ||rhs||, or after maxit iterations.  rhs, x:
 * device fields (x is output, and input with FWILS_SOLVE_X0; with
 * FWILS_SOLVE_SCATTERED the output is the solution minus rhs, formed on the
 * device; x may then alias rhs).  iters (int32)
 * and relres (double, TRUE residual ||rhs - A x|| / ||rhs||) are device
 * arrays [sum nsys] or NULL.  Returns FWILS_ENOCONV if any system stopped at
 * maxit and FWILS_EBREAKDOWN if any broke down; x is written in all cases.
 * Synchronises the stream before returning. */
fwils_status fwils_solve(fwils_plan plan, const void* rhs, void* x, double rtol,
                         int32_t maxit, int32_t* iters, double* relres,
                         uint32_t flags);

/* Frechet operator (eqs. F, YM, F0, uY): for every system
 *   d = R A_b^-1 G0 conv P_b(dm),
 *   P_b(dm) = w~^2 dm_rho u^b + div_h( dC(dm) : E_h u^b ),
 * with dC(dm) = sum_p B^(p) dm^(p) (eq. dC, App. C) and A_b the operator with
 * the plan's contrast.  ub: device field of background solutions u^b.
 * dm: host array of nprob device pointers to fp32 maps [5][nz][nx]
 * (absolute units; may repeat).  d: device data (output).  The one LS solve
 * per system uses rtol / maxit as fwils_solve. */
fwils_status fwils_frechet(fwils_plan plan, const void* ub, const void* const* dm,
                           void* d, double rtol, int32_t maxit);

/* Adjoint operator (eqs. ad1, ua, ua0; App. B): for every problem
 *   u^a = A_b^-1 G0 conv R^T conj(r),
 *   g_rho = sum_sys conj( w~^2 u^a . u^b ),
 *   g_p   = - sum_sys conj( (E_h u^a)^T B^(p) (E_h u^b) ),  p = C11, C13, C33, C55,
 * accumulated over systems in FP64.  r: device data.  g: host array of nprob
 * device pointers to complex128 maps [5][nz][nx] in BOTH precisions (output;
 * with FWILS_ADJ_ACCUMULATE added to).  Problems that share a g pointer are
 * summed when FWILS_ADJ_ACCUMULATE is set.  The maps are FP64 because in
 * absolute units their values lie far below the float32 normal range (fields
 * of O(1e-12) m/N give products of O(1e-40)); fwils_adjoint_rel gives the
 * same operator in relative units of the plan's real type. */
fwils_status fwils_adjoint(fwils_plan plan, const void* ub, const void* r,
                           void* const* g, uint32_t flags, double rtol, int32_t maxit);

/* One of the four passes of fwils_apply, on the plan's workspace scratch
 * field (the sequence 0, 1, 2, 3 computes exactly fwils_apply):
 *   pass 0: scratch = b(u)                 (contrast stencil)
 *   pass 1: scratch = FFT_x(scratch)       (forward row transforms)
 *   pass 2: scratch = IFFT_z(G_hat FFT_z(scratch))  (column transforms with
 *           the Green's multiply, normalisation 1/(nx nz) included)
 *   pass 3: Au = u - IFFT_x(scratch)       (inverse rows + LS epilogue)
 * u is read by passes 0 and 3, Au written by pass 3 (others ignore them).
 * Exists so that a caller can time each kernel of the matvec. */
fwils_status fwils_apply_pass(fwils_plan plan, int32_t pass, const void* u, void* Au);
/* Average duration in microseconds (*us, host) of pass `pass` of
 * fwils_apply_pass over reps (1..10000) back-to-back launches, measured with
 * HIP events on the plan's stream after one warm-up launch.  Synchronous. */
fwils_status fwils_time_pass(fwils_plan plan, int32_t pass, const void* u, void* Au, int32_t reps, float* us);
/* Average duration in microseconds (*us, host) of the BiCGSTAB iteration's
 * direction-update pass with every system of the plan running: the contrast
 * stencil whose input update closes the previous iteration (r = s - omega t,
 * x += alpha p_old + omega s) and forms p = r + beta (p_old - omega v), with
 * the forward row transforms (one kernel when fused).  It continues from the
 * state of this plan's most recent solve, which must be a BiCGSTAB solve that
 * completed at least one iteration on every system (e.g. one stopped by maxit),
 * with the stop tests switched off: one warm-up launch, then reps (1..10000)
 * back-to-back launches between HIP events on the plan's stream (each takes
 * the same decisions).  The solver's per-system state is restored afterwards; the
 * workspace's Krylov vectors are left changed (every solve initialises them).
 * FWILS_EINVAL for a GMRES plan, when the last solve was not such a solve, or
 * if some system stopped running during the timed launches.  Synchronous. */
fwils_status fwils_time_krylov_pass(fwils_plan plan, int32_t reps, float* us);

/* Average duration in microseconds (*us, host) of one GMRES Arnoldi-step
 * kernel over all problems of a GMRES plan with every system running, at
 * step j (0 <= j < restart): kind 0, the basis update w -= sum_{l <= j} c_l w_l
 * (reads j + 2 field vectors, writes one); kind 1, the re-orthogonalisation
 * projections <w_l, w> (reads j + 2); kind 2, the inverse row transform whose
 * epilogue forms w = A w_j and its projections on the j + 1 basis vectors
 * (reads the spectrum, w_j and j + 1 basis vectors, writes w).  reps
 * (1..10000) back-to-back launches between HIP events on the plan's stream
 * after one warm-up; the solver's per-system state is restored afterwards,
 * the GMRES basis is left changed.  Synchronous. */
fwils_status fwils_time_gmres_pass(fwils_plan plan, int32_t kind, int32_t j, int32_t reps, float* us);

/* Per-system results of the most recent Krylov solve of this plan (from
 * fwils_solve, fwils_frechet or fwils_adjoint): completed iterations and the
 * recursive relative residual ||r|| / ||rhs||.  Host arrays [sum nsys] or
 * NULL.  Synchronous. */
fwils_status fwils_solve_stats(fwils_plan plan, int32_t* iters, double* relres);
/* Per-system outcome of the most recent Krylov solve (host int32 [sum nsys]):
 * FWILS_SYS_CONVERGED, _MAXIT (iteration limit), _BREAKDOWN (a Krylov scalar
 * became exactly zero), _NONFINITE (NaN or overflow), _RUNNING (not finished,
 * e.g. the call failed).  Synchronous. */
#define FWILS_SYS_RUNNING 0
#define FWILS_SYS_CONVERGED 1
#define FWILS_SYS_MAXIT 2
#define FWILS_SYS_BREAKDOWN 3
#define FWILS_SYS_NONFINITE 4
fwils_status fwils_solve_status(fwils_plan plan, int32_t* status);

/* ---- Generalised Tikhonov step (eqs. obj, norm) ------------------------
 * Unknowns are relative maps q, real [5][nz][nx] on the device, with
 * dm_p = m0_p q_p (m0: host double[5], e.g. the background C11, C13, C33,
 * C55, rho0); in a 3-D plan [nmaps][nz][ny][nx] and m0[nmaps] (six VTI or
 * 22 general maps).  All problems of the plan must share one grid (nx, ny,
 * nz, dx, parametrisation); their data stack: J q = [J_1 q; J_2 q; ...],
 * J* r = sum_f J_f* r_f.  With rr = ||r||^2 and L = I or the periodic
 * unscaled 5-point (2-D) or 7-point (3-D) Laplacian:
 *   f(q)      = ||J q - r||^2 / rr + lam ||L q||^2
 *   grad f(q) = 2 m0 Re J*(J q - r) / rr + 2 lam L^T L q
 *   N q       = m0 Re J*(J q) / rr + lam L^T L q          (normal operator)
 * r: device data (complex, plan data layout); dscratch: device complex
 * buffer with the same number of elements as r; ub: background solutions.
 * Every J and J* application is one LS solve per system (rtol, maxit). */
#define FWILS_REG_IDENTITY  0
#define FWILS_REG_LAPLACIAN 1

/* grad (device real [5][nz][nx]) and, if fval != NULL, *fval = f(q).  Synchronous. */
fwils_status fwils_tikhonov_grad(fwils_plan plan, const void* ub, const void* r, const double* m0,
                                 double lam, int32_t reg, const void* q, void* grad, double* fval,
                                 void* dscratch, double rtol, int32_t maxit);

/* q_out = N q_in for a given rr (> 0).  Synchronous. */
fwils_status fwils_normal_apply(fwils_plan plan, const void* ub, const double* m0, double rr,
                                double lam, int32_t reg, const void* q_in, void* q_out,
                                void* dscratch, double rtol, int32_t maxit);

/* niter iterations (1..1000) of CG on N q = m0 Re J* r / rr (eq. norm) from q = 0,
 * FP64 scalars kept on the device; the iteration ends early once the squared
 * residual norm has dropped by 1e30 (converged to working precision).  q:
 * device output.  hist (host double [niter + 1] or NULL) receives the
 * normal-equation residual norm before each iteration and after the last
 * (repeated after an early end).  Synchronous. */
fwils_status fwils_normal_cg(fwils_plan plan, const void* ub, const void* r, const double* m0,
                             double lam, int32_t reg, int32_t niter, void* q, double* hist,
                             void* dscratch, double rtol, int32_t maxit);

/* fwils_normal_cg in steps, with every iterate: first = 0 starts from q = 0
 * exactly as fwils_normal_cg; first = k > 0 continues, for niter more
 * iterations, the run of k iterations this plan's last call left in its
 * workspace (same ub, r, m0, lam and reg; FWILS_EINVAL if the plan holds no
 * such run, e.g. after another Tikhonov call).  The steps of one run give
 * exactly the iterates and history of one call of their total length: a run
 * that has reached the floor of fwils_normal_cg stays there.  q_iters (device real [niter][5][nz][nx], or NULL)
 * receives the iterate after each of the niter iterations; hist (host double
 * [niter + 1] or NULL) the residual norms from iteration first on.  For runs
 * longer than one call should take (checkpoints, progress, comparisons of
 * iterates).  first + niter <= 1000.  Synchronous. */
fwils_status fwils_normal_cg_steps(fwils_plan plan, const void* ub, const void* r, const double* m0,
                                   double lam, int32_t reg, int32_t first, int32_t niter, void* q,
                                   double* hist, void* q_iters, void* dscratch, double rtol,
                                   int32_t maxit);

/* J and J* in the relative units of the Tikhonov step (single-grid plans):
 *   fwils_frechet_rel: d = J (m0 q)                     (q: device real [5][nz][nx])
 *   fwils_adjoint_rel: gq = m0 Re(J* r), summed over problems (gq: device real)
 * These are the forward and backward of the differentiable operator q -> J q. */
fwils_status fwils_frechet_rel(fwils_plan plan, const void* ub, const void* q, const double* m0,
                               void* d, double rtol, int32_t maxit);
fwils_status fwils_adjoint_rel(fwils_plan plan, const void* ub, const void* r, const double* m0,
                               void* gq, double rtol, int32_t maxit);

/* out = L q: periodic unscaled 5-point Laplacian of the 5 maps [5][nz][nx]
 * (single-grid plans).  Self-adjoint, so it is also L^T q. */
fwils_status fwils_laplacian(fwils_plan plan, const void* q, void* out);

/* d = R u: every system's field sampled at its problem's receivers (the
 * receiver operator of the data, eqs. du and F0).  u: device field; d:
 * device complex [sum nsys][nrec][2] in the plan's data layout.  Every
 * problem needs receivers.  Asynchronous on the plan's stream. */
fwils_status fwils_receiver_data(fwils_plan plan, const void* u, void* d);

/* Copies problem iprob's contrast maps (real [5][nz][nx], the layout and
 * units of fwils_set_contrast) to the device buffer maps.  Asynchronous. */
fwils_status fwils_get_contrast(fwils_plan plan, int32_t iprob, void* maps);

/* ---- Distorted-Born iteration (the DBI loop around eqs. du, obj, norm) --
 * One frequency stage of the inversion on a single-grid plan.  The plan's
 * contrast is the background model m_b (shared by all its problems: set the
 * same maps on each) and is updated in place.  Outer iteration k:
 *   u^b = A_b^-1 u0 for the point forces src_ixz, src_f (as fwils_incident);
 *     from k = 1 on, the solve starts from the previous model's u^b;
 *   r = d_obs - R u^b;  eps_d[k] = ||r|| / ||d_obs|| (normalised data error);
 *   stop if eps_d[k] < tol, eps_d[k] == 0 or k == max_outer;
 *   lam_k = lam0 eps_d[k] / eps_d[0] (self-adaptive cooling; lam_0 = lam0);
 *   q = niter CG iterations on eq. norm with lam_k (as fwils_normal_cg);
 *   contrast_p += m0_p q_p on every problem (the background update).
 * The paper's stage stops at eps_d < 1e-3 or after 10 iterations
 * (tol = 1e-3, max_outer = 10).
 * d_obs: device data (plan layout, non-zero); ub: device field, receives the
 * final model's background fields; r: device data, receives their residual;
 * q: device real [5][nz][nx], receives the last update (untouched without
 * one); dscratch: device complex buffer of the data's size.  eps_hist: host
 * double [max_outer + 1]; lam_hist: host double [max_outer] or NULL;
 * updates (host, or NULL): the number of model updates made.
 * niter 1..1000, max_outer 0..100, tol >= 0.  Returns the worst status of
 * its solves (ENOCONV if any stopped at maxit); EBREAKDOWN if the data error
 * became non-finite.  Synchronous. */
fwils_status fwils_dbi_run(fwils_plan plan, const int32_t* src_ixz, const double* src_f,
                           const void* d_obs, const double* m0, double lam0, int32_t reg,
                           int32_t niter, double tol, int32_t max_outer, void* ub, void* r,
                           void* q, void* dscratch, double* eps_hist, double* lam_hist,
                           int32_t* updates, double rtol, int32_t maxit);

/* 2-D FFT of every field of problem iprob with the library's own transform
 * kernels (unnormalised forward, exp(-i k.x); inverse with exp(+i k.x) and
 * no 1/(nx nz)).  A self-test entry point.  in, out: device, may alias. */
fwils_status fwils_fft2(fwils_plan plan, int32_t iprob, const void* in, void* out,
                        int32_t inverse);

/* ------------------------------------------------------- Krylov method ----
 * Every solve of the plan (fwils_solve, and the solves inside J, J*, the
 * Tikhonov gradient and the normal-equation CG) uses the plan's Krylov
 * method: BiCGSTAB (default; needs no extra memory) or restarted GMRES(m),
 * the method of the paper's numerical examples (section on numerical
 * examples), with Arnoldi by classical Gram-Schmidt with one
 * re-orthogonalisation pass (or one pass with FWILS_GMRES_CGS1) and the
 * Hessenberg least-squares problem solved by Givens rotations in FP64.
 * GMRES stops a cycle when its residual estimate reaches rtol and accepts
 * a system when the true residual ||b - A x|| / ||b|| at the next cycle start
 * is <= rtol, or <= 2 rtol after a cycle that reached rtol on its estimate
 * (BiCGSTAB likewise accepts a recursive residual <= rtol with a true one
 * <= 2 rtol); fwils_solve's iters count Arnoldi steps (one matvec each; a
 * BiCGSTAB iteration is two).  FWILS_SOLVE_PLAIN is BiCGSTAB only. */
#define FWILS_KRYLOV_BICGSTAB 0
#define FWILS_KRYLOV_GMRES 1
#define FWILS_GMRES_CGS1 0x1u

/* Bytes of device memory GMRES(restart), restart 1..32, needs for this plan:
 * (restart + 1) field-sized basis vectors plus per-system FP64 state. */
fwils_status fwils_gmres_workspace_size(fwils_plan plan, int32_t restart, size_t* bytes);
/* Select the Krylov method.  For FWILS_KRYLOV_GMRES, gws is caller-owned
 * device memory of at least fwils_gmres_workspace_size bytes, 256-byte
 * aligned, kept until the method changes or the plan is destroyed; the plan
 * workspace must already be set.  restart, flags and gws are ignored for
 * BiCGSTAB.  Synchronous. */
fwils_status fwils_set_krylov(fwils_plan plan, int32_t method, int32_t restart, uint32_t flags, void* gws,
                              size_t bytes);

/* ---------------------------------------------------------- autotuner ----
 * The batched schedule over uneven grids picks, per problem, one variant of
 * each hot kernel: the radix sequence of the row and column transforms
 * (points per thread), the column tile width and LDS sharing of the column
 * pass, the contrast-stencil tile height and systems per workgroup, and
 * whether the stencil is fused into the forward row transform.
 * Every variant computes the same operator; different radix orders round
 * differently (fp32 rounding level).  A new plan starts from built-in
 * defaults.  Changing a problem's variants drops the plan's cached graph. */
typedef struct {
    int32_t row_points;    /* row-transform points per thread (radix sequence) */
    int32_t col_points;    /* column-transform points per thread */
    int32_t col_width;     /* columns per column workgroup (power of two) */
    int32_t col_shared;    /* 1: the two components share one LDS buffer;
                              2: separate threads transform them;
                              3: as 1 in blocks of up to 1024 threads
                                 (complex64, power-of-two columns of 512 or
                                 more points, col_points 8);
                              4: as 0, with the twiddle table copied to
                                 LDS (complex64, power-of-two columns,
                                 col_points 4 or 8, col_width 4 to 16)     */
    int32_t stencil_rows;  /* contrast-stencil tile height: 4, 8 or 16 (with
                              stencil_sys = -1: rows per step, 4 or 8; complex128
                              plans 4) */
    int32_t stencil_sys;   /* systems per stencil workgroup, 0 = from the grid size (the
                              plain stencil; the Krylov update modes always take the
                              count from the grid size); -1 = the z-marching stencil
                              (one system per workgroup walking a column strip down a
                              range of rows, every mode) */
    int32_t fused_points;  /* 0: contrast stencil and forward row transform as two
                              kernels; else one fused kernel with this many points
                              per thread (rows of at most 512 points) */
    int32_t row_points_inv; /* inverse row-transform points per thread (its Krylov
                              epilogues hold more registers, so it is tuned on its
                              own); 0 in fwils_set_tuning: the same as row_points */
    float time_us[4];      /* autotuner's time over all systems of the problem of the
                              chosen stencil, forward row pass, column variant (with
                              the forward and inverse row passes on the spectrum
                              layout it sets: tiles as wide as its blocks) and
                              stencil + row kernels (0 if not tuned) */
} fwils_tuning;

#define FWILS_TUNE_STENCIL 0
#define FWILS_TUNE_ROWS 1
#define FWILS_TUNE_COLS 2
#define FWILS_TUNE_FUSE 3

/* Time every candidate variant of each kernel kind on the plan's workspace
 * (which must be set; its field vectors are overwritten), reps launches each
 * (1..1000) with HIP events on the plan's stream, and keep the fastest per
 * problem.  Synchronous. */
fwils_status fwils_autotune(fwils_plan plan, int32_t reps);
/* Current variants of problem iprob. */
fwils_status fwils_get_tuning(fwils_plan plan, int32_t iprob, fwils_tuning* out);
/* Set the variants of problem iprob (time_us ignored).  EINVAL, with nothing
 * changed, if any field is not a built variant for this grid. */
fwils_status fwils_set_tuning(fwils_plan plan, int32_t iprob, const fwils_tuning* t);
/* The candidates of one kernel kind (FWILS_TUNE_*) for problem iprob, each
 * the current variants with that kind's fields replaced.  Writes up to cap
 * entries to out (host) and the total number to *count. */
fwils_status fwils_tuning_candidates(fwils_plan plan, int32_t iprob, int32_t kind, fwils_tuning* out,
                                     int32_t cap, int32_t* count);

const char* fwils_status_string(fwils_status s);
const char* fwils_last_error(void);
int32_t fwils_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FWILS_H */
