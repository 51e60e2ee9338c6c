// C ABI of the fwils library: plan and workspace management, the batched
// BiCGSTAB driver (eq. axb) with HIP-graph iteration chunks, the Frechet
// operator J (eqs. YM, F0, uY) and its adjoint J* (eqs. ad1, ua, ua0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"
// after launch.h (which selects the precision): the entry points of this
// build carry the precision in their names; abi.cpp dispatches to them
#include "core_names.h"
#include "../../include/fwils.h"

using namespace fw;

extern "C" void fwils_internal_set_error(const char* msg);

namespace {

#ifdef FW_C128
constexpr fwils_precision kPrec = FWILS_C128;
#else
constexpr fwils_precision kPrec = FWILS_C64;
#endif

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fwils_internal_set_error(buf);
}

#define FW_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return FWILS_EDEVICE;                                                          \
        }                                                                                  \
    } while (0)

#define FW_TRY(expr)                          \
    do {                                      \
        fwils_status s_ = (expr);             \
        if (s_ != FWILS_OK) return s_;        \
    } while (0)

constexpr int kMaxRec = 65536;
// per problem: receiver cells [kMaxRec][3], then the receivers in stable cell
// order [kMaxRec] and the run lengths of receivers sharing a cell [kMaxRec]
constexpr int kRecInts = 5;
// Iterations per graph chunk (even: the p buffers alternate).  Each chunk
// boundary costs a graph launch and a state readback; each iteration of the
// last chunk past convergence costs six near-empty launches.  At the 16-18
// iterations of the 256^2 solves, six per chunk: 2.06 ms per batched solve
// against 2.14 (four), 2.13 (eight) and 2.24 ms (two); the 3-D, 1024^2 and
// DBI workloads are equal or faster with six than with four.
constexpr int kChunkIters = 6;
// A chunk that the host launches after seeing that the previous one, expected
// to be the last, was not, runs this many iterations when the residual trend
// says they suffice (even, like kChunkIters).
constexpr int kTailIters = 2;
constexpr int kNumVec = 11;           // field-sized workspace vectors
constexpr int kMaxRestarts = 3;       // restarts from the true residual per solve
constexpr double kTrueResFactor = 2.0; // restart when ||b - A x|| > 2 rtol ||b||
constexpr int kMaxCgIters = 1000;
constexpr int kMaxDbiUpdates = 100;
constexpr double kCgFloor = 1e-30;    // normal CG stops when ||res||^2 <= kCgFloor ||res_0||^2

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ProbHost {
    fwils_problem p;
    ProbDev dev;
    size_t field_off;     // complex elements into a plan-level field
    size_t n_per_sys;     // 2 nz nx
    size_t sys_off;       // first system index
    size_t map_off;       // floats into the maps region
    size_t data_off;      // complex elements into plan-level receiver data
    int nrec;
    int np_rows;          // partial records per system from the row epilogues
    int np_vec;           // partial records per system from vector kernels
    KernelCfg cfg;        // kernel variants (defaults, the autotuner's or the caller's)
    float tuned_us[4];    // autotune: stencil, row, column, stencil + rows time of the choice
    // dimensions of the field (2-D: ny = 1, two components, five maps)
    bool d3 = false;      // a 3-D problem (fwils_plan_create3)
    int ny = 1, ncomp = 2, nmaps = 5;
    int rps = 0;          // rows of nx points per system: ncomp nz ny
    size_t cells = 0;     // nx ny nz
    ProbDev3 dev3{};      // 3-D kernel constants
};

}  // namespace

struct fwils_plan_s {
    int32_t prec = kPrec;   // first member in both precisions: read by the dispatch
    std::vector<ProbHost> probs;
    bool d3 = false;        // a plan of 3-D problems
    int cstride = 2;        // ints per source / receiver cell index, doubles per force
    size_t total_field = 0, total_sys = 0, maps_floats = 0;
    int max_np = 0;
    hipStream_t stream = nullptr;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t off_tw = 0, off_state = 0, off_part = 0, part_bytes = 0, off_maps = 0, off_rec = 0,
           off_src = 0, off_vec = 0;
    cplx* tw = nullptr;
    SysState* state = nullptr;
    double *partV = nullptr, *partT = nullptr, *partXR = nullptr, *partB = nullptr;
    real* maps = nullptr;
    int32_t* rec = nullptr;
    int32_t* src_i = nullptr;
    double* src_f = nullptr;
    cplx *x = nullptr, *r = nullptr, *rhat = nullptr, *p = nullptr, *p2 = nullptr, *v = nullptr,
           *s = nullptr, *t = nullptr, *tmp = nullptr, *rhs = nullptr;
    cplx* tmp2 = nullptr;   // the separate contrast stencil's output (input of the forward rows)
    // model-map scratch of the Tikhonov step (single-grid plans only)
    size_t map_n = 0, off_mapws = 0;   // cells of each model map (0: no shared grid)
    int map_k = 5;                        // model maps (5 in 2-D, 6 or 22 in 3-D)
    real *mq_dm = nullptr, *mq_x = nullptr, *mq_res = nullptr, *mq_p = nullptr, *mq_Ap = nullptr,
          *mq_l1 = nullptr, *mq_l2 = nullptr;
    double2* mq_g = nullptr;   // FP64 J* accumulator (map units)
    double *mq_part = nullptr, *mq_sc = nullptr, *mq_hist = nullptr;
    int cg_done = -1;           // iterations of the normal-equation CG run the map workspace holds (-1: none)
    bool cg_floor = false;      // that run reached the floor (converged to working precision)
    double cg_rs0 = 0.0;        // that run's initial squared residual
    // graphs of one chunk of iterations over all problems (the first chunk of
    // a solve or restart starts from r)
    hipGraphExec_t chunk = nullptr, chunk_first = nullptr, chunk_tail = nullptr;
    // Krylov method; GMRES state lives in a caller-provided workspace
    int krylov = FWILS_KRYLOV_BICGSTAB;
    bool bicg_state = false;   // the workspace holds the state of a finished BiCGSTAB solve
    int gm_m = 0;
    bool gm_cgs2 = true;
    size_t gm_maxnb = 0;
    cplx* gm_V = nullptr;
    GmSys* gm_sys = nullptr;
    double *gm_part = nullptr, *gm_tot1 = nullptr, *gm_tot2 = nullptr, *gm_tot3 = nullptr;
    hipGraphExec_t gm_cycle = nullptr;
    double gm_rtol = 0.0;           // tolerance the cycle graph was built for
    SysState* host_state = nullptr;   // pinned
    // pinned copies of the state after two consecutive chunks, and the events
    // that mark their arrival (the host checks one chunk while the next runs)
    SysState* host_pipe = nullptr;
    hipEvent_t pipe_ev[2] = {nullptr, nullptr};
};

namespace {

// receiver cells of problem i in the workspace, then its receivers in stable
// cell order and the run lengths of receivers sharing a cell
int32_t* rec_at(fwils_plan plan, size_t i) { return plan->rec + i * (size_t)kMaxRec * kRecInts; }
int32_t* rec_perm(fwils_plan plan, size_t i) { return rec_at(plan, i) + (size_t)kMaxRec * 3; }
int32_t* rec_glen(fwils_plan plan, size_t i) { return rec_at(plan, i) + (size_t)kMaxRec * 4; }

ProbDev make_dev(const fwils_problem& p) {
    ProbDev d;
    const double w = 2.0 * M_PI * p.freq_hz, eta = p.damping;
    const double w2r = w * w * (1.0 - eta * eta), w2i = w * w * 2.0 * eta;
    const double rw2 = p.rho0 * w * w;
    d.nx = p.nx;
    d.nz = p.nz;
    d.nsys = p.nsys;
    d.symbol = p.symbol;
    d.tile_sh = 0;   // set with the column variant (col_tile_shift)
    d.inv4dx2 = (real)(1.0 / (4.0 * p.dx * p.dx));
    d.w2 = mkc((real)w2r, (real)w2i);
    d.gc11 = (real)(p.c0[0] / rw2);
    d.gc33 = (real)(p.c0[2] / rw2);
    d.gc55 = (real)(p.c0[3] / rw2);
    d.gc1355 = (real)((p.c0[1] + p.c0[3]) / rw2);
    d.ga = mkc((real)(1.0 - eta * eta), (real)(2.0 * eta));
    d.gscale = (real)(1.0 / (rw2 * (double)p.nx * (double)p.nz));
    d.dkx = (real)(2.0 * M_PI / (p.nx * p.dx));
    d.dkz = (real)(2.0 * M_PI / (p.nz * p.dx));
    d.dx = (real)p.dx;
    return d;
}

fwils_status check_plan(fwils_plan plan, bool need_ws = true) {
    if (!plan) {
        set_error("null plan");
        return FWILS_EINVAL;
    }
    if (need_ws && !plan->ws) {
        set_error("plan has no workspace (fwils_set_workspace)");
        return FWILS_ENOMEM;
    }
    return FWILS_OK;
}

// FWILS_EUNSUPPORTED for a plan of 3-D problems (entry points of the 2-D path only).
fwils_status only_2d(fwils_plan plan, const char* what) {
    if (plan && plan->d3) {
        set_error("%s: not available for 3-D plans", what);
        return FWILS_EUNSUPPORTED;
    }
    return FWILS_OK;
}

// Views of the plan-level vectors for problem i.
inline cplx* at(cplx* base, const ProbHost& P) { return base + P.field_off; }
inline const cplx* at(const void* base, const ProbHost& P) {
    return static_cast<const cplx*>(base) + P.field_off;
}
inline SysState* st_at(fwils_plan pl, const ProbHost& P) { return pl->state + P.sys_off; }
inline double* part_at(double* base, fwils_plan pl, const ProbHost& P) {
    return base + P.sys_off * (size_t)pl->max_np * kPartialNV;
}
inline real* maps_at(fwils_plan pl, const ProbHost& P) { return pl->maps + P.map_off; }

// The kernel constants of a 3-D problem for a view of d.nsys systems.
inline ProbDev3 view3(const ProbHost& P, const ProbDev& d) {
    ProbDev3 d3 = P.dev3;
    d3.nsys = d.nsys;
    return d3;
}

// The part of a convolution between the forward and the inverse x (row)
// transforms, in place on the spectrum tmp: 2-D, the column pass with the
// Green multiply; 3-D, the y transforms around the z pass with the 3 x 3
// Green multiply.  d: the view (its nsys systems from tmp on).
hipError_t spectral(fwils_plan pl, const ProbHost& P, const ProbDev& d, cplx* tmp, const SysState* st, hipStream_t s) {
    if (!P.d3) return launch_cols(COL_GREEN, P.cfg.col, tmp, d, st, pl->tw, s);
    const ProbDev3 d3 = view3(P, d);
    const int nx = d3.nx, ny = d3.ny, nz = d3.nz;
    hipError_t e = hipSuccess;
    if (ny > 1) e = launch_axis3(AX_FWD, ny, tmp, nx, d3.nsys * 3 * nz, 3 * nz, st, pl->tw, d3, s);
    if (e == hipSuccess) e = launch_axis3(AX_GREEN, nz, tmp, nx * ny, d3.nsys, 1, st, pl->tw, d3, s);
    if (e == hipSuccess && ny > 1) e = launch_axis3(AX_INV, ny, tmp, nx, d3.nsys * 3 * nz, 3 * nz, st, pl->tw, d3, s);
    return e;
}

// The contrast stencil of either dimension (vector update vm, a.b the output).
hipError_t stencil_any(const ProbHost& P, const ProbDev& d, int vm, const StencilArgs& a, SysState* st, hipStream_t s) {
    if (P.d3) return launch_stencil3(vm, a, view3(P, d), st, s);
    return launch_stencil(vm, P.cfg.st, a, d, st, s);
}

// y = G0 conv f for problem P (f read, out written; tmp is scratch).
hipError_t conv_problem(fwils_plan pl, const ProbHost& P, const cplx* f, cplx* out) {
    const int rows = P.p.nsys * P.rps;
    cplx* tmp = at(pl->tmp, P);
    hipError_t e = launch_rows_fwd(P.p.nx, P.cfg.row_p, f, tmp, rows, P.rps, tile_rows(P.dev), nullptr, pl->tw,
                                   pl->stream);
    if (e == hipSuccess) e = spectral(pl, P, P.dev, tmp, nullptr, pl->stream);
    if (e == hipSuccess)
        e = launch_rows_inv(P.p.nx, P.cfg.row_pi, EPI_STORE, tmp, nullptr, nullptr, out, nullptr, rows,
                            P.rps, tile_rows(P.dev), nullptr, pl->tw, pl->stream);
    return e;
}

// One LS matvec with an epilogue, for nsys systems starting at the given
// views (used both batched and per system).
// tmp2: the separate stencil's output; null = the workspace vector at
// tmp's offset (tmp is then a view of the workspace's FFT scratch).
hipError_t matvec(fwils_plan pl, const ProbHost& P, const ProbDev& d, const cplx* u, cplx* tmp,
                  const real* maps, int epi, const cplx* aux, cplx* out, double* part,
                  const SysState* st, hipStream_t s, const GmEpi* ge = nullptr, cplx* tmp2 = nullptr) {
    const int rows = d.nsys * P.rps;
    const KernelCfg& k = P.cfg;
    hipError_t e = hipSuccess;
    if (k.fuse_p) {
        const StencilArgs a{u, nullptr, nullptr, nullptr, nullptr, maps, nullptr, 0};
        e = launch_srows(0, k.fuse_p, a, tmp, d, const_cast<SysState*>(st), pl->tw, s);
    } else {   // the stencil into tmp2 (same views as tmp), then the rows into tmp
        if (!tmp2) tmp2 = pl->tmp2 + (tmp - pl->tmp);
        const StencilArgs a{u, nullptr, nullptr, nullptr, tmp2, maps, nullptr, 0};
        e = stencil_any(P, d, VM_NONE, a, const_cast<SysState*>(st), s);
        if (e == hipSuccess) e = launch_rows_fwd(d.nx, k.row_p, tmp2, tmp, rows, P.rps, tile_rows(d), st, pl->tw, s);
    }
    if (e == hipSuccess) e = spectral(pl, P, d, tmp, st, s);
    if (e == hipSuccess)
        e = launch_rows_inv(d.nx, k.row_pi, epi, tmp, u, aux, out, part, rows, P.rps, tile_rows(d), st, pl->tw, s,
                            ge);
    return e;
}

// Views of one problem restricted to systems [s0, s0 + ns).
// Partial buffers are laid out per problem as [nsys][nb][kPartialNV] with the
// producer's nb (np_vec for partXR / partB, np_rows for partV / partT), so
// a view of systems from s0 on starts s0 * nb records into the problem's region.
struct SysView {
    ProbDev d;
    size_t foff;     // complex offset of system s0 within the plan-level field
    size_t soff;     // state index
    size_t poff_vec; // doubles: partXR / partB records of system s0
    size_t poff_row; // doubles: partV / partT records of system s0
};

SysView make_view(fwils_plan pl, const ProbHost& P, int s0, int ns) {
    SysView v;
    v.d = P.dev;
    v.d.nsys = ns;
    v.foff = P.field_off + (size_t)s0 * P.n_per_sys;
    v.soff = P.sys_off + (size_t)s0;
    const size_t base = P.sys_off * (size_t)pl->max_np * kPartialNV;
    v.poff_vec = base + (size_t)s0 * P.np_vec * kPartialNV;
    v.poff_row = base + (size_t)s0 * P.np_rows * kPartialNV;
    return v;
}

// One BiCGSTAB iteration on a view (all kernels skip stopped systems): six
// kernels, five with the stencil fused into the forward rows.  The first
// contrast stencil takes the direction update p = r + beta (p_old - omega v)
// into its input and, past the first iteration of a (re)start, the previous
// iteration's closing updates r = s - omega t, x += alpha p_old + omega s
// (decided from the t-pass records, so a system that stops there gets only
// those); the second takes s = r - alpha v.  p alternates between two buffers
// with the iteration parity.  px_only: the direction-update stencil pass
// alone (a timing aid; needs !first).
hipError_t bicg_iteration(fwils_plan pl, const ProbHost& P, const SysView& V, int parity, bool first,
                          hipStream_t s, bool px_only = false) {
    const int ns = V.d.nsys;
    const int rows = ns * P.rps;
    cplx *x = pl->x + V.foff, *r = pl->r + V.foff, *rh = pl->rhat + V.foff, *v = pl->v + V.foff,
           *sv = pl->s + V.foff, *t = pl->t + V.foff, *tmp = pl->tmp + V.foff;
    cplx* pold = (parity ? pl->p2 : pl->p) + V.foff;
    cplx* pnew = (parity ? pl->p : pl->p2) + V.foff;
    SysState* st = pl->state + V.soff;
    double *pV = pl->partV + V.poff_row, *pT = pl->partT + V.poff_row, *pXR = pl->partXR + V.poff_vec;
    const real* maps = maps_at(pl, P);
    StencilArgs ap{r, pold, v, pnew, tmp, maps, pXR, P.np_vec, rh};
    if (!first) {
        ap = StencilArgs{sv, pold, v, pnew, tmp, maps, pT, P.np_rows, rh};
        ap.a3 = t;
        ap.xio = x;
        ap.rout = r;
    }
    const KernelCfg& k = P.cfg;
    // contrast stencil with the fused vector update, then the forward rows
    // (one fused kernel, or two)
    auto stencil_rows = [&](int vm, const StencilArgs& a) -> hipError_t {
        if (k.fuse_p) return launch_srows(vm, k.fuse_p, a, tmp, V.d, st, pl->tw, s);
        StencilArgs a2 = a;   // the separate stencil writes tmp2, the rows read it
        a2.b = pl->tmp2 + V.foff;
        hipError_t r = stencil_any(P, V.d, vm, a2, st, s);
        if (r == hipSuccess)
            r = launch_rows_fwd(V.d.nx, k.row_p, a2.b, tmp, rows, P.rps, tile_rows(V.d), st, pl->tw, s);
        return r;
    };
    hipError_t e = stencil_rows(first ? VM_P : VM_PX, ap);
    if (px_only) return e;
    if (e == hipSuccess) e = spectral(pl, P, V.d, tmp, st, s);
    if (e == hipSuccess)
        e = launch_rows_inv(V.d.nx, k.row_pi, EPI_BICG_V, tmp, pnew, rh, v, pV, rows, P.rps, tile_rows(V.d), st,
                            pl->tw, s);
    const StencilArgs as{r, v, nullptr, sv, tmp, maps, pV, P.np_rows};
    if (e == hipSuccess) e = stencil_rows(VM_S, as);
    if (e == hipSuccess) e = spectral(pl, P, V.d, tmp, st, s);
    if (e == hipSuccess)
        e = launch_rows_inv(V.d.nx, k.row_pi, EPI_BICG_T, tmp, sv, rh, t, pT, rows, P.rps, tile_rows(V.d), st,
                            pl->tw, s);
    return e;
}

// The t pass of an iteration alone: t = s - G0*b(s) from the spectrum in the
// scratch field, with its dot-product records (a timing aid).
hipError_t bicg_t_pass(fwils_plan pl, const ProbHost& P, const SysView& V, hipStream_t s) {
    const int rows = V.d.nsys * P.rps;
    return launch_rows_inv(V.d.nx, P.cfg.row_pi, EPI_BICG_T, pl->tmp + V.foff, pl->s + V.foff, pl->rhat + V.foff,
                           pl->t + V.foff, pl->partT + V.poff_row, rows, P.rps, tile_rows(V.d),
                           pl->state + V.soff, pl->tw, s);
}

// The end-of-chunk close kernel after an iteration of the given parity.
hipError_t bicg_close(fwils_plan pl, const ProbHost& P, const SysView& V, int parity, hipStream_t s) {
    cplx* pnew = (parity ? pl->p : pl->p2) + V.foff;
    return launch_bicg_close(pl->x + V.foff, pl->r + V.foff, pnew, pl->s + V.foff, pl->t + V.foff,
                             pl->partT + V.poff_row, P.np_rows, pl->state + V.soff, V.d.nsys,
                             (int)P.n_per_sys, s);
}

// One chunk of `iters` (even) iterations and the close kernel; `first` when
// the chunk starts a solve or a restart (its first iteration reads r).
hipError_t bicg_chunk(fwils_plan pl, const ProbHost& P, const SysView& V, bool first, hipStream_t s,
                      int iters = kChunkIters) {
    hipError_t e = hipSuccess;
    for (int it = 0; it < iters && e == hipSuccess; ++it)
        e = bicg_iteration(pl, P, V, it & 1, first && it == 0, s);
    if (e == hipSuccess) e = bicg_close(pl, P, V, (kChunkIters - 1) & 1, s);
    return e;
}

// Capture one launch sequence per problem, each on its own forked stream, into
// one graph (problems run concurrently; the graph ends when all have).
fwils_status capture_graph(fwils_plan pl, hipGraphExec_t* out,
                           const std::function<hipError_t(const ProbHost&, hipStream_t)>& body) {
    const int np = (int)pl->probs.size();
    std::vector<hipStream_t> ss(np, nullptr);
    std::vector<hipEvent_t> ev(np + 1, nullptr);
    for (int i = 0; i < np; ++i) FW_HIP(hipStreamCreateWithFlags(&ss[i], hipStreamNonBlocking));
    for (int i = 0; i <= np; ++i) FW_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    hipGraph_t g = nullptr;
    FW_HIP(hipStreamBeginCapture(ss[0], hipStreamCaptureModeThreadLocal));
    hipError_t e = hipEventRecord(ev[np], ss[0]);
    for (int i = 1; i < np && e == hipSuccess; ++i) e = hipStreamWaitEvent(ss[i], ev[np], 0);
    for (int i = 0; i < np && e == hipSuccess; ++i) {
        e = body(pl->probs[i], ss[i]);
        if (i > 0 && e == hipSuccess) e = hipEventRecord(ev[i], ss[i]);
    }
    for (int i = 1; i < np && e == hipSuccess; ++i) e = hipStreamWaitEvent(ss[0], ev[i], 0);
    hipError_t e2 = hipStreamEndCapture(ss[0], &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    for (auto& q : ss) (void)hipStreamDestroy(q);
    for (auto& q : ev) (void)hipEventDestroy(q);
    if (e != hipSuccess) {
        *out = nullptr;
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return FWILS_EDEVICE;
    }
    return FWILS_OK;
}

fwils_status build_chunk_graphs(fwils_plan pl) {
    for (int f = 0; f < 3; ++f) {   // chunk, first chunk, tail chunk
        hipGraphExec_t* g = f == 1 ? &pl->chunk_first : f == 2 ? &pl->chunk_tail : &pl->chunk;
        if (*g) continue;
        FW_TRY(capture_graph(pl, g, [pl, f](const ProbHost& P, hipStream_t s) -> hipError_t {
            return bicg_chunk(pl, P, make_view(pl, P, 0, P.p.nsys), f == 1, s, f == 2 ? kTailIters : kChunkIters);
        }));
    }
    return FWILS_OK;
}


// Solve A x = b where b and the result live in plan-level fields.  x_ws is
// the workspace solution vector (pl->x).  flags as fwils_solve.
fwils_status bicg_solve_ws(fwils_plan pl, const cplx* b, bool use_x0, double rtol, int maxit,
                           int32_t* iters, double* relres, uint32_t flags) {
    hipStream_t s = pl->stream;
    // initial residual, state
    for (const ProbHost& P : pl->probs) {
        const int n = (int)P.n_per_sys;
        const cplx* bp = b + P.field_off;
        if (use_x0) {
            FW_HIP(matvec(pl, P, P.dev, at(pl->x, P), at(pl->tmp, P), maps_at(pl, P), EPI_TRUERES, bp,
                          at(pl->r, P), part_at(pl->partT, pl, P), nullptr, s));
        }
        FW_HIP(launch_bicg_init(bp, use_x0 ? at(pl->r, P) : nullptr, at(pl->x, P), at(pl->r, P),
                                at(pl->rhat, P), at(pl->p, P), at(pl->v, P),
                                part_at(pl->partXR, pl, P), part_at(pl->partB, pl, P), P.p.nsys, n,
                                !use_x0, s));
        FW_HIP(launch_bicg_state_init(st_at(pl, P), part_at(pl->partXR, pl, P),
                                      part_at(pl->partB, pl, P), P.p.nsys, P.np_vec, rtol, maxit, s));
    }
    const size_t nst = pl->total_sys;
    // known: pl->host_state holds the current states (else the first chunk is
    // queued without a look: its kernels exit at once for stopped systems)
    auto iterate = [&](bool known) -> fwils_status {
        if (flags & FWILS_SOLVE_PLAIN) {
            // per-source loop, host-synchronous check after every iteration
            for (const ProbHost& P : pl->probs) {
                for (int sy = 0; sy < P.p.nsys; ++sy) {
                    const SysView V = make_view(pl, P, sy, 1);
                    if (pl->host_state[V.soff].status != ST_RUNNING) continue;
                    for (int it = 0; it <= maxit; ++it) {
                        FW_HIP(bicg_iteration(pl, P, V, it & 1, it == 0, s));
                        FW_HIP(bicg_close(pl, P, V, it & 1, s));
                        FW_HIP(hipMemcpyAsync(pl->host_state + V.soff, pl->state + V.soff, sizeof(SysState),
                                              hipMemcpyDeviceToHost, s));
                        FW_HIP(hipStreamSynchronize(s));
                        if (pl->host_state[V.soff].status != ST_RUNNING) break;
                    }
                }
            }
            return FWILS_OK;
        }
        const int max_chunks = maxit / kTailIters + 2;   // a bound: the device stops systems at maxit
        bool done = false;
        if (known) {
            done = true;
            for (size_t i = 0; i < nst; ++i)
                if (pl->host_state[i].status == ST_RUNNING) done = false;
            if (done) return FWILS_OK;
        }
        if (!(flags & FWILS_SOLVE_NOGRAPH)) FW_TRY(build_chunk_graphs(pl));
        // Chunk c + 1 is queued before the state after chunk c is inspected, so
        // the device does not wait for the host between chunks; a chunk queued
        // after every system stopped only runs kernels that exit at once.  The
        // speculation is skipped when the residual trend says the chunk just
        // queued is likely the last one; when that chunk then was not the last,
        // the next one is a short tail chunk if the trend says it suffices.
        SysState* hp[2] = {pl->host_pipe, pl->host_pipe + nst};
        std::vector<int> len(max_chunks + 1, kChunkIters);   // iterations of each chunk
        auto launch = [&](int c, bool tail) -> fwils_status {
            len[c] = tail ? kTailIters : kChunkIters;
            if (flags & FWILS_SOLVE_NOGRAPH) {
                for (const ProbHost& P : pl->probs)
                    FW_HIP(bicg_chunk(pl, P, make_view(pl, P, 0, P.p.nsys), c == 0, s, len[c]));
            } else {
                FW_HIP(hipGraphLaunch(c == 0 ? pl->chunk_first : tail ? pl->chunk_tail : pl->chunk, s));
            }
            FW_HIP(hipMemcpyAsync(hp[c & 1], pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
            FW_HIP(hipEventRecord(pl->pipe_ev[c & 1], s));
            return FWILS_OK;
        };
        std::vector<double> prev(nst);
        for (size_t i = 0; i < nst; ++i) prev[i] = known ? pl->host_state[i].rnorm2 : 0.0;
        int launched = 0;
        bool last_likely = false;
        FW_TRY(launch(0, false));
        launched = 1;
        for (int c = 0; c < max_chunks; ++c) {
            if (launched == c + 1 && c + 1 < max_chunks && !last_likely) {
                FW_TRY(launch(c + 1, false));
                ++launched;
            }
            FW_HIP(hipEventSynchronize(pl->pipe_ev[c & 1]));
            const SysState* h = hp[c & 1];
            done = true;
            last_likely = true;
            bool tail_enough = true;
            for (size_t i = 0; i < nst; ++i) {
                if (h[i].status != ST_RUNNING) continue;
                done = false;
                // geometric extrapolation of ||r||^2 at the rate of chunk c
                const double cur = h[i].rnorm2;
                const double rate = prev[i] > 0.0 && cur > 0.0 ? std::log(cur / prev[i]) / len[c] : 0.0;
                if (!(cur * std::exp(rate * kChunkIters) <= h[i].tol2)) last_likely = false;
                if (!(cur * std::exp(rate * kTailIters) <= h[i].tol2)) tail_enough = false;
                prev[i] = cur;
            }
            if (done) break;
            if (launched == c + 1 && c + 1 < max_chunks) {
                FW_TRY(launch(c + 1, tail_enough));
                ++launched;
            }
        }
        return FWILS_OK;
    };
    // Iterate; then check the true residual and restart, from it, systems whose
    // recursive residual drifted (bounded number of restarts per system).
    const double limit2 = (kTrueResFactor * rtol) * (kTrueResFactor * rtol);
    for (int round = 0;; ++round) {
        // the plain loop reads every system's state first; the batched one
        // starts the first round without a host round trip
        const bool look = round > 0 || (flags & FWILS_SOLVE_PLAIN);
        if (look) {
            FW_HIP(hipMemcpyAsync(pl->host_state, pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
            FW_HIP(hipStreamSynchronize(s));
        }
        FW_TRY(iterate(look));
        for (const ProbHost& P : pl->probs)
            FW_HIP(matvec(pl, P, P.dev, at(pl->x, P), at(pl->tmp, P), maps_at(pl, P), EPI_TRUERES,
                          b + P.field_off, at(pl->r, P), part_at(pl->partT, pl, P), nullptr, s));
        if (round == kMaxRestarts) break;
        for (const ProbHost& P : pl->probs)
            FW_HIP(launch_bicg_restart_mark(st_at(pl, P), part_at(pl->partT, pl, P), P.np_rows, P.p.nsys,
                                            limit2, kMaxRestarts, s));
        FW_HIP(hipMemcpyAsync(pl->host_state, pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
        FW_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (const ProbHost& P : pl->probs) {
            bool here = false;
            for (int sy = 0; sy < P.p.nsys; ++sy) here = here || pl->host_state[P.sys_off + sy].status == ST_RESTART;
            if (!here) continue;
            any = true;
            // r already holds b - A x; restart from it (converged systems are not touched again)
            FW_HIP(launch_bicg_init(b + P.field_off, at(pl->r, P), at(pl->x, P), at(pl->r, P), at(pl->rhat, P),
                                    at(pl->p, P), at(pl->v, P), part_at(pl->partXR, pl, P),
                                    part_at(pl->partB, pl, P), P.p.nsys, (int)P.n_per_sys, false, s));
            FW_HIP(launch_bicg_restart(st_at(pl, P), P.p.nsys, s));
        }
        if (!any) break;
    }
    for (const ProbHost& P : pl->probs)
        FW_HIP(launch_bicg_finish(st_at(pl, P), part_at(pl->partT, pl, P), P.np_rows, P.p.nsys,
                                  iters ? iters + P.sys_off : nullptr, relres ? relres + P.sys_off : nullptr, s));
    FW_HIP(hipMemcpyAsync(pl->host_state, pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    pl->bicg_state = true;
    bool noconv = false, brk = false;
    for (size_t i = 0; i < nst; ++i) {
        const int stt = st_code(pl->host_state[i].status);
        if (stt == ST_MAXIT || stt == ST_RUNNING) noconv = true;
        if (stt == ST_BREAKDOWN || stt == ST_NONFINITE) brk = true;
    }
    if (brk) {
        set_error("BiCGSTAB breakdown or non-finite residual in at least one system");
        return FWILS_EBREAKDOWN;
    }
    if (noconv) {
        set_error("at least one system did not reach rtol within maxit");
        return FWILS_ENOCONV;
    }
    return FWILS_OK;
}

// ------------------------------------------------------------- GMRES ----
void drop_graphs(fwils_plan pl) {
    if (pl->chunk) (void)hipGraphExecDestroy(pl->chunk);
    if (pl->chunk_first) (void)hipGraphExecDestroy(pl->chunk_first);
    if (pl->chunk_tail) (void)hipGraphExecDestroy(pl->chunk_tail);
    pl->chunk_first = nullptr;
    pl->chunk_tail = nullptr;
    if (pl->gm_cycle) (void)hipGraphExecDestroy(pl->gm_cycle);
    pl->chunk = nullptr;
    pl->gm_cycle = nullptr;
}

GmArgs gm_args(fwils_plan pl, const ProbHost& P) {
    GmArgs a;
    a.V = pl->gm_V + P.field_off;
    a.vstride = pl->total_field;
    a.gs = pl->gm_sys + P.sys_off;
    a.st = pl->state + P.sys_off;
    a.part = pl->gm_part + P.sys_off * pl->gm_maxnb * kGmRec;
    a.tot1 = pl->gm_tot1 + P.sys_off * kGmRec;
    a.tot2 = pl->gm_tot2 + P.sys_off * kGmRec;
    a.tot3 = pl->gm_tot3 + P.sys_off * kGmRec;
    a.nsys = P.p.nsys;
    a.n = (int)P.n_per_sys;
    return a;
}

// r = b - A x into basis slot 0 with ||r||^2, ||b||^2, then the cycle start.
hipError_t gm_start(fwils_plan pl, const ProbHost& P, const cplx* b, double rtol, bool first, hipStream_t s) {
    const GmArgs a = gm_args(pl, P);
    const GmEpi ge{nullptr, 0, 0, a.part};
    hipError_t e = matvec(pl, P, P.dev, at(pl->x, P), at(pl->tmp, P), maps_at(pl, P), EPI_GMRES_R0,
                          b + P.field_off, a.V, nullptr, a.st, s, &ge);
    if (e == hipSuccess) e = launch_gm_sum(a, GM_SUM_BEGIN, P.np_rows, 0, false, rtol, first, s);
    return e;
}

// One GMRES cycle of m Arnoldi steps, the solution update, and the start of
// the next cycle (true residual).  Systems that are not RUNNING skip.
// Per step: the matvec whose epilogue projects w on the basis, the sum of
// those projections, w -= W c, and (CGS2) the projections of the result,
// their sum and the second subtraction; the last subtraction leaves ||w||^2
// records, whose sum builds the Hessenberg column.
hipError_t gm_cycle(fwils_plan pl, const ProbHost& P, const cplx* b, double rtol, hipStream_t s) {
    const GmArgs a = gm_args(pl, P);
    const int nbv = gm_blocks_per_sys((int)P.n_per_sys);
    const bool cgs2 = pl->gm_cgs2;
    hipError_t e = hipSuccess;
    for (int j = 0; j < pl->gm_m && e == hipSuccess; ++j) {
        const GmEpi ge{a.V, a.vstride, j + 1, a.part};
        cplx* wj = a.V + (size_t)j * a.vstride;
        cplx* wn = a.V + (size_t)(j + 1) * a.vstride;
        e = matvec(pl, P, P.dev, wj, at(pl->tmp, P), maps_at(pl, P), EPI_ARNOLDI, nullptr, wn, nullptr, a.st, s,
                   &ge);
        if (e == hipSuccess) e = launch_gm_sum(a, GM_SUM_PROJ1, P.np_rows, j, cgs2, rtol, false, s);
        if (e == hipSuccess) e = launch_gm_update(a, j, 1, !cgs2, s);
        if (cgs2) {
            if (e == hipSuccess) e = launch_gm_dots(a, j, s);
            if (e == hipSuccess) e = launch_gm_sum(a, GM_SUM_PROJ2, nbv, j, cgs2, rtol, false, s);
            if (e == hipSuccess) e = launch_gm_update(a, j, 2, true, s);
        }
        if (e == hipSuccess) e = launch_gm_sum(a, GM_SUM_HESS, nbv, j, cgs2, rtol, false, s);
    }
    if (e == hipSuccess) e = launch_gm_finish_cycle(at(pl->x, P), a, s);
    if (e == hipSuccess) e = gm_start(pl, P, b, rtol, false, s);
    return e;
}

fwils_status gm_solve_ws(fwils_plan pl, const cplx* b, bool use_x0, double rtol, int maxit, int32_t* iters,
                         double* relres, uint32_t flags) {
    if (flags & FWILS_SOLVE_PLAIN) {
        set_error("solve: the per-source plain loop is a BiCGSTAB mode");
        return FWILS_EUNSUPPORTED;
    }
    hipStream_t s = pl->stream;
    // the cycle graph reads the right-hand side from the plan's rhs vector
    if (b != pl->rhs) FW_HIP(launch_copy(b, pl->rhs, pl->total_field, s));
    b = pl->rhs;
    for (const ProbHost& P : pl->probs) {
        const GmArgs a = gm_args(pl, P);
        if (!use_x0) FW_HIP(launch_zero(at(pl->x, P), (size_t)P.p.nsys * P.n_per_sys, s));
        FW_HIP(launch_gm_init(a.st, a.gs, a.nsys, maxit, pl->gm_m, s));
        FW_HIP(gm_start(pl, P, b, rtol, true, s));
    }
    const size_t nst = pl->total_sys;
    auto any_running = [&](bool& any) -> fwils_status {
        FW_HIP(hipMemcpyAsync(pl->host_state, pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
        FW_HIP(hipStreamSynchronize(s));
        any = false;
        for (size_t i = 0; i < nst; ++i)
            if (pl->host_state[i].status == ST_RUNNING) any = true;
        return FWILS_OK;
    };
    bool any = false;
    FW_TRY(any_running(any));
    const bool graph = !(flags & FWILS_SOLVE_NOGRAPH);
    if (any && graph && (!pl->gm_cycle || pl->gm_rtol != rtol)) {
        if (pl->gm_cycle) (void)hipGraphExecDestroy(pl->gm_cycle);
        pl->gm_cycle = nullptr;
        const cplx* rhs = pl->rhs;
        FW_TRY(capture_graph(pl, &pl->gm_cycle, [pl, rhs, rtol](const ProbHost& P, hipStream_t q) {
            return gm_cycle(pl, P, rhs, rtol, q);
        }));
        pl->gm_rtol = rtol;
    }
    for (int c = 0; any && c <= maxit; ++c) {
        if (graph) {
            FW_HIP(hipGraphLaunch(pl->gm_cycle, s));
        } else {
            for (const ProbHost& P : pl->probs) FW_HIP(gm_cycle(pl, P, b, rtol, s));
        }
        FW_TRY(any_running(any));
    }
    FW_HIP(launch_gm_report(pl->state, iters, relres, (int)nst, s));
    FW_HIP(hipMemcpyAsync(pl->host_state, pl->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    bool noconv = false, brk = false;
    for (size_t i = 0; i < nst; ++i) {
        const int stt = st_code(pl->host_state[i].status);
        if (stt == ST_MAXIT || stt == ST_RUNNING) noconv = true;
        if (stt == ST_BREAKDOWN || stt == ST_NONFINITE) brk = true;
    }
    if (brk) {
        set_error("GMRES breakdown or non-finite residual in at least one system");
        return FWILS_EBREAKDOWN;
    }
    if (noconv) {
        set_error("at least one system did not reach rtol within maxit");
        return FWILS_ENOCONV;
    }
    return FWILS_OK;
}

fwils_status solve_ws(fwils_plan pl, const cplx* b, bool use_x0, double rtol, int maxit, int32_t* iters,
                      double* relres, uint32_t flags) {
    pl->bicg_state = false;
    if (pl->krylov == FWILS_KRYLOV_GMRES) return gm_solve_ws(pl, b, use_x0, rtol, maxit, iters, relres, flags);
    return bicg_solve_ws(pl, b, use_x0, rtol, maxit, iters, relres, flags);
}

// Checks the point forces (one per system, host arrays as fwils_incident
// takes them) and copies them to the plan's device arrays.
fwils_status upload_sources(fwils_plan plan, const int32_t* src_ixz, const double* src_f, const char* what) {
    if (!src_ixz || !src_f) {
        set_error("%s: null source pointer", what);
        return FWILS_EINVAL;
    }
    const int cs = plan->cstride;
    for (const ProbHost& P : plan->probs) {
        for (int sy = 0; sy < P.p.nsys; ++sy) {
            const size_t k = P.sys_off + sy;
            const int ix = src_ixz[cs * k], iz = src_ixz[cs * k + cs - 1], iy = cs == 3 ? src_ixz[cs * k + 1] : 0;
            bool finite = true;
            for (int c = 0; c < cs; ++c) finite = finite && std::isfinite(src_f[cs * k + c]);
            if (ix < 0 || ix >= P.p.nx || iz < 0 || iz >= P.p.nz || iy < 0 || iy >= P.ny || !finite) {
                set_error("%s: source %zu at (%d, %d, %d) outside the grid or non-finite force", what, k, ix, iy, iz);
                return FWILS_EINVAL;
            }
        }
    }
    FW_HIP(hipStreamSynchronize(plan->stream));
    FW_HIP(hipMemcpy(plan->src_i, src_ixz, plan->total_sys * cs * sizeof(int32_t), hipMemcpyHostToDevice));
    FW_HIP(hipMemcpy(plan->src_f, src_f, plan->total_sys * cs * sizeof(double), hipMemcpyHostToDevice));
    return FWILS_OK;
}

// u0 = G0 conv s for the uploaded point forces (eq. u0); f: a field-sized
// buffer for the discrete sources, distinct from out and from tmp.
hipError_t incident_ws(fwils_plan plan, cplx* f, cplx* out) {
    for (const ProbHost& P : plan->probs) {
        hipError_t e = launch_zero(at(f, P), (size_t)P.p.nsys * P.n_per_sys, plan->stream);
        const int cs = plan->cstride;
        if (e == hipSuccess)
            e = P.d3 ? launch_point_sources3(at(f, P), plan->src_i + cs * P.sys_off, plan->src_f + cs * P.sys_off,
                                             P.dev3, plan->stream)
                     : launch_point_sources(at(f, P), plan->src_i + cs * P.sys_off, plan->src_f + cs * P.sys_off,
                                            P.dev, plan->stream);
        if (e == hipSuccess) e = conv_problem(plan, P, at(f, P), at(out, P));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

fwils_status check_field_ptrs(std::initializer_list<const void*> ptrs) {
    for (const void* q : ptrs)
        if (!q) {
            set_error("null device pointer");
            return FWILS_EINVAL;
        }
    return FWILS_OK;
}

// Offsets of every problem in the plan-level vectors, partial-record sizes
// and the workspace layout, from the problems' dimensions and variants.
void layout_plan(fwils_plan pl) {
    size_t foff = 0, soff = 0, moff = 0;
    pl->max_np = 0;
    for (ProbHost& P : pl->probs) {
        P.n_per_sys = (size_t)P.ncomp * P.cells;
        P.field_off = foff;
        P.sys_off = soff;
        P.map_off = moff;
        P.data_off = 0;
        P.nrec = 0;
        P.tuned_us[0] = P.tuned_us[1] = P.tuned_us[2] = P.tuned_us[3] = 0.f;
        P.np_rows = row_geom(P.p.nx, P.cfg.row_pi, P.rps).blocks_per_sys;   // the inverse pass's partials
        P.np_vec = vec_blocks_per_sys((int)P.n_per_sys);
        pl->max_np = std::max(pl->max_np, P.np_vec);
        {   // partial buffers fit every row-transform variant
            int cand[3];
            const int nc = row_candidates(P.p.nx, cand);
            for (int c = 0; c < nc; ++c)
                pl->max_np = std::max(pl->max_np, row_geom(P.p.nx, cand[c], P.rps).blocks_per_sys);
        }
        foff += (size_t)P.p.nsys * P.n_per_sys;
        soff += (size_t)P.p.nsys;
        moff += (size_t)P.nmaps * P.cells;
    }
    const int nprob = (int)pl->probs.size();
    pl->total_field = foff;
    pl->total_sys = soff;
    pl->maps_floats = moff;
    // workspace layout
    size_t o = 0;
    pl->off_tw = o;
    o = align256(o + twiddle_table_elems() * sizeof(cplx));
    pl->off_state = o;
    o = align256(o + pl->total_sys * sizeof(SysState));
    pl->off_part = o;
    pl->part_bytes = align256(pl->total_sys * (size_t)pl->max_np * kPartialNV * sizeof(double));
    o += 4 * pl->part_bytes;
    pl->off_maps = o;
    o = align256(o + pl->maps_floats * sizeof(real));
    pl->off_rec = o;
    o = align256(o + (size_t)nprob * kMaxRec * kRecInts * sizeof(int32_t));
    pl->off_src = o;   // source cells, then (256-byte aligned) source forces
    o = align256(o + align256(pl->total_sys * 3 * sizeof(int32_t)) + pl->total_sys * 3 * sizeof(double));
    pl->off_vec = o;
    o += kNumVec * align256(pl->total_field * sizeof(cplx));
    // the Tikhonov step's model-map scratch: plans whose problems share one
    // grid (and parametrisation)
    bool one_grid = true;
    for (int i = 1; i < nprob; ++i)
        one_grid = one_grid && pl->probs[i].p.nx == pl->probs[0].p.nx && pl->probs[i].p.nz == pl->probs[0].p.nz &&
                   pl->probs[i].ny == pl->probs[0].ny && pl->probs[i].nmaps == pl->probs[0].nmaps &&
                   pl->probs[i].p.dx == pl->probs[0].p.dx;
    pl->map_n = one_grid ? pl->probs[0].cells : 0;
    pl->map_k = pl->probs[0].nmaps;
    pl->off_mapws = o;
    const size_t mk = (size_t)pl->map_k;
    if (pl->map_n) {
        o += 7 * align256(mk * pl->map_n * sizeof(real)) + align256(mk * pl->map_n * sizeof(double2));
        o += align256(kDotPartials * sizeof(double)) + align256(16 * sizeof(double)) +
             align256(kMaxCgIters + 1) * sizeof(double);
    }
    pl->ws_bytes = o;
}

// Kernel constants of a 3-D problem.  The scaled Christoffel coefficients
// come from the general 4-index tensor C_ijkl = C[V(i,j)][V(k,l)]:
// Gamma_ik = sum_jl C_ijkl k_j k_l, so the coefficient of the monomial
// k_j k_l (j <= l) in entry (i, k) is C_ijkj for j = l and C_ijkl + C_ilkj
// otherwise, divided by rho0 w^2 (w real).
ProbDev3 make_dev3(const fwils_problem3& p) {
    ProbDev3 d{};
    const double w = 2.0 * M_PI * p.freq_hz, eta = p.damping;
    const double rw2 = p.rho0 * w * w;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.nsys = p.nsys;
    d.params = p.params == FWILS_PARAMS_GENERAL ? kParamsGeneral : kParamsVti;
    d.symbol = p.symbol;
    d.inv4dx2 = (real)(1.0 / (4.0 * p.dx * p.dx));
    d.w2 = mkc((real)(w * w * (1.0 - eta * eta)), (real)(w * w * 2.0 * eta));
    d.dx = (real)p.dx;
    double C[6][6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            C[i][j] = C[j][i] = p.c0[q];
            ++q;
        }
    const int V[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};   // Voigt index of (i, j)
    const int pr[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    for (int a = 0; a < 6; ++a) {
        const int i = pr[a][0], k = pr[a][1];
        for (int b = 0; b < 6; ++b) {
            const int j = pr[b][0], l = pr[b][1];
            double c = C[V[i][j]][V[k][l]];
            if (j != l) c += C[V[i][l]][V[k][j]];
            d.gq[a][b] = (real)(c / rw2);
        }
    }
    d.ga = mkc((real)(1.0 - eta * eta), (real)(2.0 * eta));
    d.gscale = (real)(1.0 / (rw2 * (double)p.nx * (double)p.ny * (double)p.nz));
    d.dk[0] = (real)(2.0 * M_PI / (p.nx * p.dx));
    d.dk[1] = (real)(2.0 * M_PI / (p.ny * p.dx));
    d.dk[2] = (real)(2.0 * M_PI / (p.nz * p.dx));
    return d;
}

// Whether a symmetric 6 x 6 matrix (21 constants) is positive definite
// (Cholesky in double).
bool spd21(const double* c21) {
    double A[6][6];
    int q = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            A[i][j] = A[j][i] = c21[q];
            ++q;
        }
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
        if (!(d > 0.0)) return false;
        A[j][j] = std::sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = A[i][j];
            for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
            A[i][j] = v / A[j][j];
        }
    }
    return true;
}

}  // namespace

extern "C" {

fwils_status fwils_plan_create(const fwils_problem* probs, int32_t nprob, fwils_precision prec,
                               fwils_plan* out) {
    if (!out || !probs || nprob < 1 || nprob > 64) {
        set_error("plan_create: need 1..64 problems and an output pointer");
        return FWILS_EINVAL;
    }
    if (prec != kPrec) {
        set_error("plan_create: precision %d reached the wrong library core", (int)prec);
        return FWILS_EINVAL;
    }
    for (int i = 0; i < nprob; ++i) {
        const fwils_problem& p = probs[i];
        if (!fft_size_supported(p.nx) || !fft_size_supported(p.nz)) {
            set_error("problem %d: nx=%d nz=%d not supported (2^a 3^b, 16..2048)", i, p.nx, p.nz);
            return FWILS_EINVAL;
        }
        if (!(p.dx > 0) || !(p.rho0 > 0) || !(p.freq_hz > 0) || !(p.damping > 0) ||
            !(p.c0[0] > 0) || !(p.c0[2] > 0) || !(p.c0[3] > 0) || !std::isfinite(p.c0[1])) {
            set_error("problem %d: dx, rho0, freq_hz, damping, C11, C33, C55 must be > 0", i);
            return FWILS_EINVAL;
        }
        if (p.nsys < 1 || (long long)p.nsys * 2 * p.nx * p.nz > (1LL << 31) * 4) {
            set_error("problem %d: nsys=%d out of range", i, p.nsys);
            return FWILS_EINVAL;
        }
        if (p.symbol != FWILS_SYMBOL_SPECTRAL && p.symbol != FWILS_SYMBOL_CENTRAL) {
            set_error("problem %d: unknown symbol %d", i, p.symbol);
            return FWILS_EINVAL;
        }
    }
    fwils_plan pl = new fwils_plan_s();
    for (int i = 0; i < nprob; ++i) {
        ProbHost P;
        P.p = probs[i];
        P.dev = make_dev(P.p);
        P.ny = 1;
        P.ncomp = 2;
        P.nmaps = 5;
        P.cells = (size_t)P.p.nz * P.p.nx;
        P.rps = 2 * P.p.nz;
        P.cfg = kernel_cfg_default(P.p.nx, P.p.nz);
        P.dev.tile_sh = col_tile_shift(P.p.nx, P.cfg.col.W);
        pl->probs.push_back(P);
    }
    layout_plan(pl);
    *out = pl;
    return FWILS_OK;
}

fwils_status fwils_plan_create3(const fwils_problem3* probs, int32_t nprob, fwils_precision prec,
                                fwils_plan* out) {
    if (!out || !probs || nprob < 1 || nprob > 64) {
        set_error("plan_create3: need 1..64 problems and an output pointer");
        return FWILS_EINVAL;
    }
    if (prec != kPrec) {
        set_error("plan_create3: precision %d reached the wrong library core", (int)prec);
        return FWILS_EINVAL;
    }
    for (int i = 0; i < nprob; ++i) {
        const fwils_problem3& p = probs[i];
        if (!axis3_size_supported(p.nx) || !axis3_size_supported(p.nz) ||
            !(p.ny == 1 || axis3_size_supported(p.ny))) {
            set_error("problem %d: %d x %d x %d not supported (each axis 2^a 3^b 5^c in 16..256, or ny = 1)", i, p.nx,
                      p.ny, p.nz);
            return FWILS_EINVAL;
        }
        if (!(p.dx > 0) || !(p.rho0 > 0) || !(p.freq_hz > 0) || !(p.damping > 0)) {
            set_error("problem %d: dx, rho0, freq_hz and damping must be > 0", i);
            return FWILS_EINVAL;
        }
        bool finite = true;
        for (int k = 0; k < 21; ++k) finite = finite && std::isfinite(p.c0[k]);
        if (!finite || !spd21(p.c0)) {
            set_error("problem %d: the background stiffness must be finite and positive definite", i);
            return FWILS_EINVAL;
        }
        if (p.params != FWILS_PARAMS_VTI && p.params != FWILS_PARAMS_GENERAL) {
            set_error("problem %d: unknown params %d", i, p.params);
            return FWILS_EINVAL;
        }
        if (p.symbol != FWILS_SYMBOL_SPECTRAL && p.symbol != FWILS_SYMBOL_CENTRAL) {
            set_error("problem %d: unknown symbol %d", i, p.symbol);
            return FWILS_EINVAL;
        }
        const long long cells = (long long)p.nx * p.ny * p.nz;
        if (p.nsys < 1 || (long long)p.nsys * 3 * cells > (1LL << 31) * 4 || (long long)p.nsys * 3 * p.nz * p.ny > (1LL << 30)) {
            set_error("problem %d: nsys=%d out of range", i, p.nsys);
            return FWILS_EINVAL;
        }
    }
    fwils_plan pl = new fwils_plan_s();
    pl->d3 = true;
    pl->cstride = 3;
    for (int i = 0; i < nprob; ++i) {
        const fwils_problem3& q = probs[i];
        ProbHost P;
        P.p = fwils_problem{};
        P.p.nx = q.nx;
        P.p.nz = q.nz;
        P.p.dx = q.dx;
        P.p.rho0 = q.rho0;
        P.p.freq_hz = q.freq_hz;
        P.p.damping = q.damping;
        P.p.nsys = q.nsys;
        P.p.symbol = q.symbol;
        P.dev = ProbDev{};
        P.dev.nx = q.nx;
        P.dev.nz = q.nz;
        P.dev.nsys = q.nsys;
        P.dev.symbol = q.symbol;
        P.dev.tile_sh = 0;   // row-major spectra
        P.dev.dx = (real)q.dx;
        P.dev3 = make_dev3(q);
        P.d3 = true;
        P.ny = q.ny;
        P.ncomp = 3;
        P.nmaps = q.params == FWILS_PARAMS_GENERAL ? 22 : 6;
        P.cells = (size_t)q.nx * q.ny * q.nz;
        P.rps = 3 * q.nz * q.ny;
        P.cfg.row_p = P.cfg.row_pi = row_points_default(q.nx);
        P.cfg.col = ColCfg{0, 0, 0};
        P.cfg.st = st_default();
        P.cfg.fuse_p = 0;
        pl->probs.push_back(P);
    }
    layout_plan(pl);
    *out = pl;
    return FWILS_OK;
}

void fwils_plan_destroy(fwils_plan plan) {
    if (!plan) return;
    drop_graphs(plan);
    if (plan->host_state) (void)hipHostFree(plan->host_state);
    if (plan->host_pipe) (void)hipHostFree(plan->host_pipe);
    for (auto& e : plan->pipe_ev)
        if (e) (void)hipEventDestroy(e);
    delete plan;
}

fwils_status fwils_workspace_size(fwils_plan plan, size_t* bytes) {
    FW_TRY(check_plan(plan, false));
    if (!bytes) {
        set_error("null output");
        return FWILS_EINVAL;
    }
    *bytes = plan->ws_bytes;
    return FWILS_OK;
}

fwils_status fwils_field_elems(fwils_plan plan, int64_t* elems) {
    FW_TRY(check_plan(plan, false));
    if (!elems) {
        set_error("null output");
        return FWILS_EINVAL;
    }
    *elems = (int64_t)plan->total_field;
    return FWILS_OK;
}

fwils_status fwils_set_stream(fwils_plan plan, void* hip_stream) {
    FW_TRY(check_plan(plan, false));
    plan->stream = (hipStream_t)hip_stream;
    return FWILS_OK;
}

fwils_status fwils_set_workspace(fwils_plan plan, void* dev, size_t bytes) {
    FW_TRY(check_plan(plan, false));
    if (!dev || bytes < plan->ws_bytes || ((uintptr_t)dev & 255) != 0) {
        set_error("set_workspace: need %zu bytes, 256-byte aligned (got %zu)", plan->ws_bytes, bytes);
        return FWILS_ENOMEM;
    }
    drop_graphs(plan);
    plan->bicg_state = false;
    if (!plan->host_state) {
        FW_HIP(hipHostMalloc((void**)&plan->host_state, plan->total_sys * sizeof(SysState),
                             hipHostMallocDefault));
        FW_HIP(hipHostMalloc((void**)&plan->host_pipe, 2 * plan->total_sys * sizeof(SysState),
                             hipHostMallocDefault));
        for (auto& e : plan->pipe_ev) FW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    char* w = (char*)dev;
    plan->ws = w;
    plan->tw = (cplx*)(w + plan->off_tw);
    plan->state = (SysState*)(w + plan->off_state);
    plan->partV = (double*)(w + plan->off_part);
    plan->partT = (double*)(w + plan->off_part + plan->part_bytes);
    plan->partXR = (double*)(w + plan->off_part + 2 * plan->part_bytes);
    plan->partB = (double*)(w + plan->off_part + 3 * plan->part_bytes);
    plan->maps = (real*)(w + plan->off_maps);
    plan->rec = (int32_t*)(w + plan->off_rec);
    plan->src_i = (int32_t*)(w + plan->off_src);
    // the forces follow the cells at the offset the layout reserves (three ints per system)
    plan->src_f = (double*)(w + plan->off_src + align256(plan->total_sys * 3 * sizeof(int32_t)));
    cplx** vecs[kNumVec] = {&plan->x, &plan->r, &plan->rhat, &plan->p, &plan->p2,
                              &plan->v, &plan->s, &plan->t, &plan->tmp, &plan->rhs, &plan->tmp2};
    const size_t vb = align256(plan->total_field * sizeof(cplx));
    for (int i = 0; i < kNumVec; ++i) *vecs[i] = (cplx*)(w + plan->off_vec + i * vb);
    if (plan->map_n) {
        char* m = w + plan->off_mapws;
        const size_t fb = align256((size_t)plan->map_k * plan->map_n * sizeof(real));
        real** fm[7] = {&plan->mq_dm, &plan->mq_x, &plan->mq_res, &plan->mq_p,
                         &plan->mq_Ap, &plan->mq_l1, &plan->mq_l2};
        for (int i = 0; i < 7; ++i) *fm[i] = (real*)(m + i * fb);
        m += 7 * fb;
        plan->mq_g = (double2*)m;
        m += align256((size_t)plan->map_k * plan->map_n * sizeof(double2));
        plan->mq_part = (double*)m;
        m += align256(kDotPartials * sizeof(double));
        plan->mq_sc = (double*)m;
        m += align256(16 * sizeof(double));
        plan->mq_hist = (double*)m;
    }
    std::vector<cplx> tw(twiddle_table_elems());
    twiddle_table_fill(tw.data());
    FW_HIP(hipMemcpy(plan->tw, tw.data(), tw.size() * sizeof(cplx), hipMemcpyHostToDevice));
    FW_HIP(hipMemset(plan->maps, 0, plan->maps_floats * sizeof(real)));
    FW_HIP(hipMemset(plan->state, 0, plan->total_sys * sizeof(SysState)));
    FW_HIP(hipDeviceSynchronize());
    return FWILS_OK;
}

fwils_status fwils_set_contrast(fwils_plan plan, int32_t iprob, const void* maps_) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const real* maps = static_cast<const real*>(maps_);
    FW_TRY(check_plan(plan));
    if (iprob < 0 || iprob >= (int)plan->probs.size() || !maps) {
        set_error("set_contrast: bad problem index or null maps");
        return FWILS_EINVAL;
    }
    const ProbHost& P = plan->probs[iprob];
    FW_HIP(hipMemcpyAsync(maps_at(plan, P), maps, (size_t)P.nmaps * P.cells * sizeof(real),
                          hipMemcpyDeviceToDevice, plan->stream));
    return FWILS_OK;
}

fwils_status fwils_set_receivers(fwils_plan plan, int32_t iprob, const int32_t* rec_ixz, int32_t nrec) {
    FW_TRY(check_plan(plan));
    if (iprob < 0 || iprob >= (int)plan->probs.size() || !rec_ixz || nrec < 1 || nrec > kMaxRec) {
        set_error("set_receivers: bad problem index, null pointer or nrec out of 1..%d", kMaxRec);
        return FWILS_EINVAL;
    }
    ProbHost& P = plan->probs[iprob];
    const int cs = plan->cstride;
    for (int r = 0; r < nrec; ++r) {
        const int ix = rec_ixz[cs * r], iz = rec_ixz[cs * r + cs - 1], iy = cs == 3 ? rec_ixz[cs * r + 1] : 0;
        if (ix < 0 || ix >= P.p.nx || iy < 0 || iy >= P.ny || iz < 0 || iz >= P.p.nz) {
            set_error("set_receivers: receiver %d at (%d, %d, %d) outside the %dx%dx%d grid", r, ix, iy, iz, P.p.nx,
                      P.ny, P.p.nz);
            return FWILS_EINVAL;
        }
    }
    // the receivers in stable order of their cells, and the length of each run
    // of receivers on one cell at its first entry (the adjoint scatter sums a
    // run in one thread, in receiver order)
    std::vector<int64_t> cell(nrec);
    for (int r = 0; r < nrec; ++r) {
        const int ix = rec_ixz[cs * r], iz = rec_ixz[cs * r + cs - 1], iy = cs == 3 ? rec_ixz[cs * r + 1] : 0;
        cell[r] = ((int64_t)iz * P.ny + iy) * P.p.nx + ix;
    }
    std::vector<int32_t> perm(nrec), glen(nrec, 0);
    for (int r = 0; r < nrec; ++r) perm[r] = r;
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return cell[a] < cell[b]; });
    for (int k = 0; k < nrec;) {
        int e = k + 1;
        while (e < nrec && cell[perm[e]] == cell[perm[k]]) ++e;
        glen[k] = e - k;
        k = e;
    }
    FW_HIP(hipStreamSynchronize(plan->stream));
    FW_HIP(hipMemcpy(rec_at(plan, iprob), rec_ixz, (size_t)nrec * cs * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    FW_HIP(hipMemcpy(rec_perm(plan, iprob), perm.data(), (size_t)nrec * sizeof(int32_t), hipMemcpyHostToDevice));
    FW_HIP(hipMemcpy(rec_glen(plan, iprob), glen.data(), (size_t)nrec * sizeof(int32_t), hipMemcpyHostToDevice));
    P.nrec = nrec;
    size_t doff = 0;
    for (ProbHost& Q : plan->probs) {
        Q.data_off = doff;
        doff += (size_t)Q.p.nsys * Q.nrec * Q.ncomp;
    }
    return FWILS_OK;
}

fwils_status fwils_incident(fwils_plan plan, const int32_t* src_ixz, const double* src_f, void* u0) {
    FW_TRY(check_plan(plan));
    if (!u0) {
        set_error("incident: null pointer");
        return FWILS_EINVAL;
    }
    FW_TRY(upload_sources(plan, src_ixz, src_f, "incident"));
    FW_HIP(incident_ws(plan, plan->rhs, static_cast<cplx*>(u0)));
    return FWILS_OK;
}

fwils_status fwils_body_force(fwils_plan plan, const void* u, void* b) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({u, b}));
    for (const ProbHost& P : plan->probs) {
        const StencilArgs a{at(u, P), nullptr, nullptr, nullptr, static_cast<cplx*>(b) + P.field_off,
                            maps_at(plan, P), nullptr, 0};
        FW_HIP(stencil_any(P, P.dev, VM_NONE, a, nullptr, plan->stream));
    }
    return FWILS_OK;
}

fwils_status fwils_convolve(fwils_plan plan, const void* f, void* out) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({f, out}));
    for (const ProbHost& P : plan->probs)
        FW_HIP(conv_problem(plan, P, at(f, P), static_cast<cplx*>(out) + P.field_off));
    return FWILS_OK;
}

fwils_status fwils_apply(fwils_plan plan, const void* u, void* Au) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({u, Au}));
    if (u == Au) {
        set_error("apply: u and Au must not alias");
        return FWILS_EINVAL;
    }
    for (const ProbHost& P : plan->probs)
        FW_HIP(matvec(plan, P, P.dev, at(u, P), at(plan->tmp, P), maps_at(plan, P), EPI_APPLY, nullptr,
                      static_cast<cplx*>(Au) + P.field_off, nullptr, nullptr, plan->stream));
    return FWILS_OK;
}

}  // extern "C"

namespace {

// Scratch of fwils_apply_noalloc: the column-tiled FFT scratch field and the
// separate contrast stencil's output, in place of the two workspace vectors
// fwils_apply uses.  Every GPU the library runs on holds one copy (per
// precision build) for the life of the process.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current; looked
// up once per device.  In host code the array's own name is not a device
// address: only the looked-up pointer is ever handed to kernels.
fwils_status noalloc_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("apply_noalloc: device %d beyond the %d devices the library tracks", dev, kMaxDevices);
        return FWILS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        FW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("apply_noalloc: no device address for the static scratch on device %d", dev);
            return FWILS_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FWILS_OK;
}

}  // namespace

extern "C" {

fwils_status fwils_apply_noalloc(fwils_plan plan, const void* u, void* Au) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({u, Au}));
    if (u == Au) {
        set_error("apply_noalloc: u and Au must not alias");
        return FWILS_EINVAL;
    }
    const size_t fb = align256(plan->total_field * sizeof(cplx));
    if (2 * fb > kNoAllocBytes) {
        set_error("apply_noalloc: the plan's fields (%zu complex elements) need %zu bytes of scratch; "
                  "the static scratch holds %zu (fields of at most %zu complex elements)",
                  plan->total_field, 2 * fb, kNoAllocBytes, kNoAllocBytes / 2 / sizeof(cplx));
        return FWILS_EINVAL;
    }
    int dev = -1;
    FW_HIP(hipGetDevice(&dev));
    hipPointerAttribute_t attr;
    FW_HIP(hipPointerGetAttributes(&attr, plan->ws));
    if (attr.device != dev) {
        set_error("apply_noalloc: the plan's workspace is on device %d, device %d is current", attr.device, dev);
        return FWILS_EINVAL;
    }
    void* base = nullptr;
    FW_TRY(noalloc_scratch(dev, &base));
    cplx* tmp = static_cast<cplx*>(base);
    cplx* tmp2 = reinterpret_cast<cplx*>(static_cast<char*>(base) + fb);
    // the scratch is written in full before it is read: nothing to clear
    for (const ProbHost& P : plan->probs)
        FW_HIP(matvec(plan, P, P.dev, at(u, P), tmp + P.field_off, maps_at(plan, P), EPI_APPLY, nullptr,
                      static_cast<cplx*>(Au) + P.field_off, nullptr, nullptr, plan->stream, nullptr,
                      tmp2 + P.field_off));
    return FWILS_OK;
}

fwils_status fwils_solve(fwils_plan plan, const void* rhs, void* x, double rtol, int32_t maxit,
                         int32_t* iters, double* relres, uint32_t flags) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({rhs, x}));
    if (!(rtol > 0) || maxit < 1 ||
        (flags & ~(FWILS_SOLVE_X0 | FWILS_SOLVE_PLAIN | FWILS_SOLVE_NOGRAPH | FWILS_SOLVE_SCATTERED))) {
        set_error("solve: need rtol > 0, maxit >= 1 and known flags");
        return FWILS_EINVAL;
    }
    hipStream_t s = plan->stream;
    const bool x0 = (flags & FWILS_SOLVE_X0) != 0;
    if (x0) FW_HIP(launch_copy(static_cast<const cplx*>(x), plan->x, plan->total_field, s));
    fwils_status st = solve_ws(plan, static_cast<const cplx*>(rhs), x0, rtol, maxit, iters, relres, flags);
    if (st == FWILS_EDEVICE) return st;
    if (flags & FWILS_SOLVE_SCATTERED)   // u_s = u - u0 (eq. delu), elementwise, so x may alias rhs
        FW_HIP(launch_diff(plan->x, static_cast<const cplx*>(rhs), static_cast<cplx*>(x), plan->total_field, s));
    else
        FW_HIP(launch_copy(plan->x, static_cast<cplx*>(x), plan->total_field, s));
    FW_HIP(hipStreamSynchronize(s));
    return st;
}

}  // extern "C"

namespace {

// d = R w for problem i (either dimension).
hipError_t gather_any(fwils_plan plan, size_t i, const cplx* w, cplx* d, hipStream_t s) {
    const ProbHost& P = plan->probs[i];
    const int32_t* rec = rec_at(plan, i);
    return P.d3 ? launch_gather3(w, d, rec, P.nrec, P.dev3, s) : launch_gather(w, d, rec, P.nrec, P.dev, s);
}

// J dm (validated arguments): one virtual source, one convolution and one
// gather per problem around one batched solve.
fwils_status frechet_ws(fwils_plan plan, const void* ub, const real* const* dm, void* d, double rtol,
                        int32_t maxit) {
    hipStream_t s = plan->stream;
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        // virtual source P_b(dm): the contrast stencil applied to u^b with dm
        const StencilArgs a{at(ub, P), nullptr, nullptr, nullptr, at(plan->s, P), dm[i], nullptr, 0};
        FW_HIP(stencil_any(P, P.dev, VM_NONE, a, nullptr, s));
        FW_HIP(conv_problem(plan, P, at(plan->s, P), at(plan->rhs, P)));
    }
    fwils_status st = solve_ws(plan, plan->rhs, false, rtol, maxit, nullptr, nullptr, 0);
    if (st == FWILS_EDEVICE) return st;
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        FW_HIP(gather_any(plan, i, at(plan->x, P), static_cast<cplx*>(d) + P.data_off, s));
    }
    return st;
}

// J* r (validated arguments): receiver scatter and convolution per problem,
// one batched solve, correlation with u^b per problem.
fwils_status adjoint_ws(fwils_plan plan, const void* ub, const void* r, void* const* g, bool accumulate,
                        double rtol, int32_t maxit, bool fp64_maps = false) {
    hipStream_t s = plan->stream;
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        cplx* f = at(plan->s, P);
        FW_HIP(launch_zero(f, (size_t)P.p.nsys * P.n_per_sys, s));
        if (P.d3)
            FW_HIP(launch_scatter_conj3(static_cast<const cplx*>(r) + P.data_off, f, rec_at(plan, i),
                                        rec_perm(plan, i), rec_glen(plan, i), P.nrec, P.dev3, s));
        else
            FW_HIP(launch_scatter_conj(static_cast<const cplx*>(r) + P.data_off, f, rec_at(plan, i),
                                       rec_perm(plan, i), rec_glen(plan, i), P.nrec, P.dev, s));
        FW_HIP(conv_problem(plan, P, f, at(plan->rhs, P)));
    }
    fwils_status st = solve_ws(plan, plan->rhs, false, rtol, maxit, nullptr, nullptr, 0);
    if (st == FWILS_EDEVICE) return st;
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        if (P.d3)
            FW_HIP(launch_correlate3(at(plan->x, P), at(ub, P), static_cast<double2*>(g[i]), P.dev3, accumulate, s));
        else if (fp64_maps)
            FW_HIP(launch_correlate_f64(at(plan->x, P), at(ub, P), static_cast<double2*>(g[i]), P.dev,
                                        accumulate, s));
        else
            FW_HIP(launch_correlate(at(plan->x, P), at(ub, P), static_cast<cplx*>(g[i]), P.dev,
                                    accumulate, s));
    }
    return st;
}

fwils_status check_jj(fwils_plan plan, double rtol, int32_t maxit, const char* what) {
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        if (plan->probs[i].nrec < 1) {
            set_error("%s: problem %zu has no receivers", what, i);
            return FWILS_EINVAL;
        }
    }
    if (!(rtol > 0) || maxit < 1) {
        set_error("%s: need rtol > 0 and maxit >= 1", what);
        return FWILS_EINVAL;
    }
    return FWILS_OK;
}

fwils_status worst(fwils_status a, fwils_status b) {
    if (a == FWILS_EBREAKDOWN || b == FWILS_EBREAKDOWN) return FWILS_EBREAKDOWN;
    if (a == FWILS_ENOCONV || b == FWILS_ENOCONV) return FWILS_ENOCONV;
    return a != FWILS_OK ? a : b;
}

// ---- Tikhonov step --------------------------------------------------------
fwils_status check_tik(fwils_plan plan, const double* m0, double lam, int32_t reg, double rtol,
                       int32_t maxit, const char* what) {
    FW_TRY(check_jj(plan, rtol, maxit, what));
    if (!plan->map_n) {
        set_error("%s: the plan's problems do not share one grid", what);
        return FWILS_EINVAL;
    }
    if (!m0 || !(lam >= 0) || (reg != FWILS_REG_IDENTITY && reg != FWILS_REG_LAPLACIAN)) {
        set_error("%s: need m0[%d], lam >= 0 and a known regulariser", what, plan->map_k);
        return FWILS_EINVAL;
    }
    for (int k = 0; k < plan->map_k; ++k)
        if (!std::isfinite(m0[k])) {
            set_error("%s: m0 must be finite", what);
            return FWILS_EINVAL;
        }
    return FWILS_OK;
}

size_t data_elems(fwils_plan plan) {
    size_t n = 0;
    for (const ProbHost& P : plan->probs) n += (size_t)P.p.nsys * P.nrec * P.ncomp;
    return n;
}

// reg_out = L^T L q (Laplacian) or q (identity) into mq_l2; also L q in mq_l1.
fwils_status regulariser(fwils_plan plan, int32_t reg, const real* q, const real** rq) {
    const ProbHost& P = plan->probs[0];
    if (reg == FWILS_REG_LAPLACIAN) {
        FW_HIP(launch_laplacian(q, plan->mq_l1, P.p.nx, P.ny, P.p.nz, plan->map_k, plan->stream));
        FW_HIP(launch_laplacian(plan->mq_l1, plan->mq_l2, P.p.nx, P.ny, P.p.nz, plan->map_k, plan->stream));
        *rq = plan->mq_l2;
    } else {
        *rq = q;
    }
    return FWILS_OK;
}

// out = N q for a given rr (the normal operator of eq. norm)
fwils_status normal_apply_ws(fwils_plan plan, const void* ub, const MapScales& m0, double rr, double lam,
                             int32_t reg, const real* q, real* out, void* dscratch, double rtol,
                             int32_t maxit) {
    hipStream_t s = plan->stream;
    const int n = (int)plan->map_n;
    FW_HIP(launch_map_scale(q, plan->mq_dm, m0, n, s));
    std::vector<const real*> dms(plan->probs.size(), plan->mq_dm);
    fwils_status st = frechet_ws(plan, ub, dms.data(), dscratch, rtol, maxit);
    if (st == FWILS_EDEVICE) return st;
    std::vector<void*> gs(plan->probs.size(), plan->mq_g);
    FW_HIP(launch_zero_d2(plan->mq_g, (size_t)plan->map_k * plan->map_n, s));
    fwils_status st2 = adjoint_ws(plan, ub, dscratch, gs.data(), true, rtol, maxit, true);
    if (st2 == FWILS_EDEVICE) return st2;
    const real* rq = nullptr;
    FW_TRY(regulariser(plan, reg, q, &rq));
    FW_HIP(launch_map_combine(plan->mq_g, rq, out, m0, 1.0 / rr, lam, n, s));
    return worst(st, st2);
}

MapScales scales(const double* m0, int nmaps) {
    MapScales m{};
    m.n = nmaps;
    for (int k = 0; k < nmaps; ++k) m.s[k] = m0[k];
    return m;
}

// niter CG iterations on eq. norm from q = 0 (validated arguments); hist:
// host [niter + 1] or NULL.
// CG on the normal equation.  first = 0: from q = 0 (right-hand side, first
// residual); first = k > 0: continue the run whose k iterations the plan's
// map workspace holds.  q_iters (or null): the iterate after each iteration.
fwils_status normal_cg_ws(fwils_plan plan, const void* ub, const void* r, const MapScales& ms, double lam,
                          int32_t reg, int32_t niter, real* q, double* hist, void* dscratch, double rtol,
                          int32_t maxit, int32_t first = 0, real* q_iters = nullptr) {
    hipStream_t s = plan->stream;
    const int n = (int)plan->map_n;
    const size_t nm = (size_t)plan->map_k * plan->map_n;
    double* sc = plan->mq_sc;
    // rr = ||r||^2 (the misfit's normalisation)
    FW_HIP(launch_norm2_complex(static_cast<const cplx*>(r), data_elems(plan), plan->mq_part, sc + 4, s));
    double rr = 0;
    FW_HIP(hipMemcpyAsync(&rr, sc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    if (!(rr > 0)) {
        set_error("normal_cg: ||r|| is zero");
        return FWILS_EINVAL;
    }
    fwils_status st = FWILS_OK;
    if (first == 0) {   // the right-hand side m0 Re J* r / rr and the first residual
        plan->cg_done = -1;
        plan->cg_floor = false;
        std::vector<void*> gs(plan->probs.size(), plan->mq_g);
        FW_HIP(launch_zero_d2(plan->mq_g, nm, s));
        st = adjoint_ws(plan, ub, r, gs.data(), true, rtol, maxit, true);
        if (st == FWILS_EDEVICE) return st;
        FW_HIP(launch_map_combine(plan->mq_g, nullptr, plan->mq_res, ms, 1.0 / rr, 0.0, n, s));
        FW_HIP(launch_zero_f(plan->mq_x, nm, s));
        FW_HIP(launch_copy_f(plan->mq_res, plan->mq_p, nm, s));
        FW_HIP(launch_dot_real(plan->mq_res, plan->mq_res, nm, plan->mq_part, sc + 2, s));
        FW_HIP(launch_cg_shift(sc, plan->mq_hist, 0, s));
        FW_HIP(hipMemcpyAsync(&plan->cg_rs0, sc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        FW_HIP(hipStreamSynchronize(s));
    }
    const double rs0 = plan->cg_rs0;
    // iterations run: fewer once the residual is at the floor (none when
    // continuing a run that reached it, as one longer run would have stopped)
    int done = plan->cg_floor ? 0 : niter;
    for (int it = 0; it < done; ++it) {
        fwils_status sa = normal_apply_ws(plan, ub, ms, rr, lam, reg, plan->mq_p, plan->mq_Ap, dscratch,
                                          rtol, maxit);
        if (sa == FWILS_EDEVICE) return sa;
        st = worst(st, sa);
        FW_HIP(launch_dot_real(plan->mq_p, plan->mq_Ap, nm, plan->mq_part, sc + 1, s));
        FW_HIP(launch_cg_xr(plan->mq_x, plan->mq_res, plan->mq_p, plan->mq_Ap, sc, nm, s));
        FW_HIP(launch_dot_real(plan->mq_res, plan->mq_res, nm, plan->mq_part, sc + 2, s));
        FW_HIP(launch_cg_p(plan->mq_p, plan->mq_res, sc, nm, s));
        FW_HIP(launch_cg_shift(sc, plan->mq_hist, first + it + 1, s));
        if (q_iters) FW_HIP(launch_copy_f(plan->mq_x, q_iters + (size_t)it * nm, nm, s));
        // converged to working precision: further iterations would only push
        // the direction vectors towards underflow
        double rs = 0.0;
        FW_HIP(hipMemcpyAsync(&rs, sc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        FW_HIP(hipStreamSynchronize(s));
        if (!(rs > kCgFloor * rs0)) {
            done = it + 1;
            plan->cg_floor = true;
            break;
        }
    }
    if (q_iters)
        for (int it = done; it < niter; ++it) FW_HIP(launch_copy_f(plan->mq_x, q_iters + (size_t)it * nm, nm, s));
    FW_HIP(launch_copy_f(plan->mq_x, q, nm, s));
    if (hist)
        FW_HIP(hipMemcpyAsync(hist, plan->mq_hist + first, (size_t)(done + 1) * sizeof(double), hipMemcpyDeviceToHost,
                              s));
    FW_HIP(hipStreamSynchronize(s));
    if (hist)
        for (int i = done + 1; i <= niter; ++i) hist[i] = hist[done];
    plan->cg_done = first + niter;
    return st;
}


}  // namespace

extern "C" {

fwils_status fwils_frechet(fwils_plan plan, const void* ub, const void* const* dm_, void* d,
                           double rtol, int32_t maxit) {
    const real* const* dm = reinterpret_cast<const real* const*>(dm_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, dm, d}));
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        if (!dm[i]) {
            set_error("frechet: problem %zu has a null dm pointer", i);
            return FWILS_EINVAL;
        }
    }
    FW_TRY(check_jj(plan, rtol, maxit, "frechet"));
    fwils_status st = frechet_ws(plan, ub, dm, d, rtol, maxit);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(hipStreamSynchronize(plan->stream));
    return st;
}

fwils_status fwils_adjoint(fwils_plan plan, const void* ub, const void* r, void* const* g,
                           uint32_t flags, double rtol, int32_t maxit) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, r, g}));
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        if (!g[i]) {
            set_error("adjoint: problem %zu has a null g pointer", i);
            return FWILS_EINVAL;
        }
    }
    FW_TRY(check_jj(plan, rtol, maxit, "adjoint"));
    if (flags & ~FWILS_ADJ_ACCUMULATE) {
        set_error("adjoint: unknown flags");
        return FWILS_EINVAL;
    }
    // complex128 maps in both precisions: absolute-unit products lie below
    // the float32 normal range at physical field scales
    fwils_status st = adjoint_ws(plan, ub, r, g, (flags & FWILS_ADJ_ACCUMULATE) != 0, rtol, maxit, true);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(hipStreamSynchronize(plan->stream));
    return st;
}

fwils_status fwils_normal_apply(fwils_plan plan, const void* ub, const double* m0, double rr, double lam,
                                int32_t reg, const void* q_in_, void* q_out_, void* dscratch, double rtol,
                                int32_t maxit) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const real* q_in = static_cast<const real*>(q_in_);
    real* q_out = static_cast<real*>(q_out_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, q_in, q_out, dscratch}));
    FW_TRY(check_tik(plan, m0, lam, reg, rtol, maxit, "normal_apply"));
    if (!(rr > 0) || q_in == q_out) {
        set_error("normal_apply: need rr > 0 and distinct q_in, q_out");
        return FWILS_EINVAL;
    }
    fwils_status st = normal_apply_ws(plan, ub, scales(m0, plan->map_k), rr, lam, reg, q_in, q_out, dscratch, rtol, maxit);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(hipStreamSynchronize(plan->stream));
    return st;
}

fwils_status fwils_tikhonov_grad(fwils_plan plan, const void* ub, const void* r, const double* m0, double lam,
                                 int32_t reg, const void* q_, void* grad_, double* fval, void* dscratch,
                                 double rtol, int32_t maxit) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const real* q = static_cast<const real*>(q_);
    real* grad = static_cast<real*>(grad_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, r, q, grad, dscratch}));
    FW_TRY(check_tik(plan, m0, lam, reg, rtol, maxit, "tikhonov_grad"));
    hipStream_t s = plan->stream;
    const MapScales ms = scales(m0, plan->map_k);
    const int n = (int)plan->map_n;
    const size_t nd = data_elems(plan);
    double* sc = plan->mq_sc;
    // rr = ||r||^2
    FW_HIP(launch_norm2_complex(static_cast<const cplx*>(r), nd, plan->mq_part, sc + 4, s));
    // residual J q - r and its norm
    FW_HIP(launch_map_scale(q, plan->mq_dm, ms, n, s));
    std::vector<const real*> dms(plan->probs.size(), plan->mq_dm);
    fwils_status st = frechet_ws(plan, ub, dms.data(), dscratch, rtol, maxit);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(launch_sub_complex(static_cast<cplx*>(dscratch), static_cast<const cplx*>(r), nd, s));
    FW_HIP(launch_norm2_complex(static_cast<const cplx*>(dscratch), nd, plan->mq_part, sc + 5, s));
    std::vector<void*> gs(plan->probs.size(), plan->mq_g);
    FW_HIP(launch_zero_d2(plan->mq_g, (size_t)plan->map_k * plan->map_n, s));
    fwils_status st2 = adjoint_ws(plan, ub, dscratch, gs.data(), true, rtol, maxit, true);
    if (st2 == FWILS_EDEVICE) return st2;
    const real* rq = nullptr;
    FW_TRY(regulariser(plan, reg, q, &rq));
    // ||L q||^2
    const real* lq = (reg == FWILS_REG_LAPLACIAN) ? plan->mq_l1 : q;
    FW_HIP(launch_dot_real(lq, lq, (size_t)plan->map_k * plan->map_n, plan->mq_part, sc + 6, s));
    double h[3];
    FW_HIP(hipMemcpyAsync(h, sc + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    if (!(h[0] > 0)) {
        set_error("tikhonov_grad: ||r|| is zero");
        return FWILS_EINVAL;
    }
    FW_HIP(launch_map_combine(plan->mq_g, rq, grad, ms, 2.0 / h[0], 2.0 * lam, n, s));
    FW_HIP(hipStreamSynchronize(s));
    if (fval) *fval = h[1] / h[0] + lam * h[2];
    return worst(st, st2);
}

fwils_status fwils_frechet_rel(fwils_plan plan, const void* ub, const void* q_, const double* m0, void* d,
                               double rtol, int32_t maxit) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const real* q = static_cast<const real*>(q_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, q, d}));
    FW_TRY(check_tik(plan, m0, 0.0, FWILS_REG_IDENTITY, rtol, maxit, "frechet_rel"));
    FW_HIP(launch_map_scale(q, plan->mq_dm, scales(m0, plan->map_k), (int)plan->map_n, plan->stream));
    std::vector<const real*> dms(plan->probs.size(), plan->mq_dm);
    fwils_status st = frechet_ws(plan, ub, dms.data(), d, rtol, maxit);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(hipStreamSynchronize(plan->stream));
    return st;
}

fwils_status fwils_adjoint_rel(fwils_plan plan, const void* ub, const void* r, const double* m0, void* gq_,
                               double rtol, int32_t maxit) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    real* gq = static_cast<real*>(gq_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, r, gq}));
    FW_TRY(check_tik(plan, m0, 0.0, FWILS_REG_IDENTITY, rtol, maxit, "adjoint_rel"));
    std::vector<void*> gs(plan->probs.size(), plan->mq_g);
    FW_HIP(launch_zero_d2(plan->mq_g, (size_t)plan->map_k * plan->map_n, plan->stream));
    fwils_status st = adjoint_ws(plan, ub, r, gs.data(), true, rtol, maxit, true);
    if (st == FWILS_EDEVICE) return st;
    FW_HIP(launch_map_combine(plan->mq_g, nullptr, gq, scales(m0, plan->map_k), 1.0, 0.0, (int)plan->map_n, plan->stream));
    FW_HIP(hipStreamSynchronize(plan->stream));
    return st;
}

fwils_status fwils_laplacian(fwils_plan plan, const void* q_, void* out_) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const real* q = static_cast<const real*>(q_);
    real* out = static_cast<real*>(out_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({q, out}));
    if (!plan->map_n || q == out) {
        set_error("laplacian: needs a single-grid plan and distinct q, out");
        return FWILS_EINVAL;
    }
    FW_HIP(launch_laplacian(q, out, plan->probs[0].p.nx, plan->probs[0].ny, plan->probs[0].p.nz, plan->map_k,
                            plan->stream));
    return FWILS_OK;
}

fwils_status fwils_normal_cg(fwils_plan plan, const void* ub, const void* r, const double* m0, double lam,
                             int32_t reg, int32_t niter, void* q_, double* hist, void* dscratch, double rtol,
                             int32_t maxit) {
    real* q = static_cast<real*>(q_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, r, q, dscratch}));
    FW_TRY(check_tik(plan, m0, lam, reg, rtol, maxit, "normal_cg"));
    if (niter < 1 || niter > kMaxCgIters) {
        set_error("normal_cg: niter must be 1..%d", kMaxCgIters);
        return FWILS_EINVAL;
    }
    return normal_cg_ws(plan, ub, r, scales(m0, plan->map_k), lam, reg, niter, q, hist, dscratch, rtol, maxit);
}

fwils_status fwils_normal_cg_steps(fwils_plan plan, const void* ub, const void* r, const double* m0, double lam,
                                   int32_t reg, int32_t first, int32_t niter, void* q_, double* hist, void* q_iters,
                                   void* dscratch, double rtol, int32_t maxit) {
    real* q = static_cast<real*>(q_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({ub, r, q, dscratch}));
    FW_TRY(check_tik(plan, m0, lam, reg, rtol, maxit, "normal_cg_steps"));
    if (niter < 1 || first < 0 || first + niter > kMaxCgIters) {
        set_error("normal_cg_steps: need niter >= 1, first >= 0 and first + niter <= %d", kMaxCgIters);
        return FWILS_EINVAL;
    }
    if (first > 0 && plan->cg_done != first) {
        set_error("normal_cg_steps: first = %d, but the plan holds a run of %d iterations", first, plan->cg_done);
        return FWILS_EINVAL;
    }
    return normal_cg_ws(plan, ub, r, scales(m0, plan->map_k), lam, reg, niter, q, hist, dscratch, rtol, maxit, first,
                        static_cast<real*>(q_iters));
}

fwils_status fwils_receiver_data(fwils_plan plan, const void* u, void* d) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({u, d}));
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        if (P.nrec < 1) {
            set_error("receiver_data: problem %zu has no receivers", i);
            return FWILS_EINVAL;
        }
    }
    for (size_t i = 0; i < plan->probs.size(); ++i) {
        const ProbHost& P = plan->probs[i];
        FW_HIP(gather_any(plan, i, at(u, P), static_cast<cplx*>(d) + P.data_off, plan->stream));
    }
    return FWILS_OK;
}

fwils_status fwils_get_contrast(fwils_plan plan, int32_t iprob, void* maps) {
    FW_TRY(check_plan(plan));
    if (iprob < 0 || iprob >= (int)plan->probs.size() || !maps) {
        set_error("get_contrast: bad problem index or null maps");
        return FWILS_EINVAL;
    }
    const ProbHost& P = plan->probs[iprob];
    FW_HIP(hipMemcpyAsync(maps, maps_at(plan, P), (size_t)P.nmaps * P.cells * sizeof(real),
                          hipMemcpyDeviceToDevice, plan->stream));
    return FWILS_OK;
}

fwils_status fwils_dbi_run(fwils_plan plan, const int32_t* src_ixz, const double* src_f, const void* d_obs_,
                           const double* m0, double lam0, int32_t reg, int32_t niter, double tol,
                           int32_t max_outer, void* ub_, void* r_, void* q_, void* dscratch, double* eps_hist,
                           double* lam_hist, int32_t* updates, double rtol, int32_t maxit) {
    if (plan) plan->cg_done = -1;   // the map workspace is reused: no CG run to continue
    const cplx* d_obs = static_cast<const cplx*>(d_obs_);
    cplx* ub = static_cast<cplx*>(ub_);
    cplx* r = static_cast<cplx*>(r_);
    real* q = static_cast<real*>(q_);
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({d_obs, ub, r, q, dscratch, eps_hist}));
    FW_TRY(check_tik(plan, m0, lam0, reg, rtol, maxit, "dbi_run"));
    if (niter < 1 || niter > kMaxCgIters || max_outer < 0 || max_outer > kMaxDbiUpdates || !(tol >= 0)) {
        set_error("dbi_run: need niter 1..%d, max_outer 0..%d and tol >= 0", kMaxCgIters, kMaxDbiUpdates);
        return FWILS_EINVAL;
    }
    FW_TRY(upload_sources(plan, src_ixz, src_f, "dbi_run"));
    hipStream_t s = plan->stream;
    const MapScales ms = scales(m0, plan->map_k);
    const size_t nd = data_elems(plan);
    double* sc = plan->mq_sc;
    double dd = 0.0;
    FW_HIP(launch_norm2_complex(d_obs, nd, plan->mq_part, sc + 9, s));
    FW_HIP(hipMemcpyAsync(&dd, sc + 9, sizeof(double), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    if (!(dd > 0) || !std::isfinite(dd)) {
        set_error("dbi_run: d_obs must be non-zero and finite");
        return FWILS_EINVAL;
    }
    fwils_status st = FWILS_OK;
    int made = 0;
    for (int k = 0;; ++k) {
        // background fields of the current model, warm-started from the
        // previous model's fields after the first update
        FW_HIP(incident_ws(plan, plan->s, plan->rhs));
        if (k > 0) FW_HIP(launch_copy(ub, plan->x, plan->total_field, s));
        const fwils_status ss = solve_ws(plan, plan->rhs, k > 0, rtol, maxit, nullptr, nullptr, 0);
        if (ss == FWILS_EDEVICE) return ss;
        st = worst(st, ss);
        FW_HIP(launch_copy(plan->x, ub, plan->total_field, s));
        // r = d_obs - R u^b and the normalised data error
        for (size_t i = 0; i < plan->probs.size(); ++i) {
            const ProbHost& P = plan->probs[i];
            FW_HIP(gather_any(plan, i, at(ub, P), r + P.data_off, s));
        }
        FW_HIP(launch_data_residual(r, d_obs, nd, s));
        double rr = 0.0;
        FW_HIP(launch_norm2_complex(r, nd, plan->mq_part, sc + 8, s));
        FW_HIP(hipMemcpyAsync(&rr, sc + 8, sizeof(double), hipMemcpyDeviceToHost, s));
        FW_HIP(hipStreamSynchronize(s));
        const double eps = std::sqrt(rr / dd);
        if (!std::isfinite(eps)) {
            set_error("dbi_run: non-finite data error after %d updates", made);
            if (updates) *updates = made;
            return FWILS_EBREAKDOWN;
        }
        eps_hist[k] = eps;
        if (eps < tol || eps == 0.0 || k == max_outer) break;
        // self-adaptive cooling: lambda follows the data error
        const double lam = lam0 * eps / eps_hist[0];
        if (lam_hist) lam_hist[k] = lam;
        const fwils_status sq = normal_cg_ws(plan, ub, r, ms, lam, reg, niter, q, nullptr, dscratch, rtol, maxit);
        if (sq == FWILS_EDEVICE || sq == FWILS_EINVAL) return sq;
        st = worst(st, sq);
        for (const ProbHost& P : plan->probs) FW_HIP(launch_map_update(maps_at(plan, P), q, ms, (int)plan->map_n, s));
        ++made;
    }
    FW_HIP(hipStreamSynchronize(s));
    if (updates) *updates = made;
    return st;
}

fwils_status fwils_apply_pass(fwils_plan plan, int32_t pass, const void* u, void* Au) {
    FW_TRY(check_plan(plan));
    if (pass < 0 || pass > 3 || ((pass == 0 || pass == 3) && !u) || (pass == 3 && (!Au || u == Au))) {
        set_error("apply_pass: pass must be 0..3 with u (passes 0, 3) and a distinct Au (pass 3)");
        return FWILS_EINVAL;
    }
    hipStream_t s = plan->stream;
    for (const ProbHost& P : plan->probs) {
        const int rows = P.p.nsys * P.rps;
        cplx* tmp = at(plan->tmp, P);
        if (P.d3) {   // stencil / x rows / y, z (Green) and y transforms / inverse x rows
            if (pass == 0) {
                const StencilArgs a{at(u, P), nullptr, nullptr, nullptr, at(plan->tmp2, P), maps_at(plan, P), nullptr, 0};
                FW_HIP(stencil_any(P, P.dev, VM_NONE, a, nullptr, s));
            } else if (pass == 1) {
                FW_HIP(launch_rows_fwd(P.p.nx, P.cfg.row_p, at(plan->tmp2, P), tmp, rows, P.rps, SpecLayout{}, nullptr,
                                       plan->tw, s));
            } else if (pass == 2) {
                FW_HIP(spectral(plan, P, P.dev, tmp, nullptr, s));
            } else {
                FW_HIP(launch_rows_inv(P.p.nx, P.cfg.row_pi, EPI_APPLY, tmp, at(u, P), nullptr,
                                       static_cast<cplx*>(Au) + P.field_off, nullptr, rows, P.rps, SpecLayout{}, nullptr,
                                       plan->tw, s));
            }
            continue;
        }
        switch (pass) {
            case 0:
                if (P.cfg.fuse_p) {
                    const StencilArgs a{at(u, P), nullptr, nullptr, nullptr, nullptr, maps_at(plan, P), nullptr, 0};
                    FW_HIP(launch_srows(0, P.cfg.fuse_p, a, tmp, P.dev, nullptr, plan->tw, s));
                } else {
                    FW_HIP(launch_body_force(P.cfg.st, at(u, P), at(plan->tmp2, P), maps_at(plan, P), P.dev, nullptr, s));
                }
                break;
            case 1:   // part of pass 0 when the stencil and the rows are fused
                if (!P.cfg.fuse_p)
                    FW_HIP(launch_rows_fwd(P.p.nx, P.cfg.row_p, at(plan->tmp2, P), tmp, rows, P.rps,
                                           tile_rows(P.dev), nullptr, plan->tw, s));
                break;
            case 2: FW_HIP(launch_cols(COL_GREEN, P.cfg.col, tmp, P.dev, nullptr, plan->tw, s)); break;
            default:
                FW_HIP(launch_rows_inv(P.p.nx, P.cfg.row_pi, EPI_APPLY, tmp, at(u, P), nullptr,
                                       static_cast<cplx*>(Au) + P.field_off, nullptr, rows, P.rps, tile_rows(P.dev),
                                       nullptr, plan->tw, s));
        }
    }
    return FWILS_OK;
}

fwils_status fwils_time_pass(fwils_plan plan, int32_t pass, const void* u, void* Au, int32_t reps, float* us) {
    if (!us || reps < 1 || reps > 10000) {
        set_error("time_pass: need reps 1..10000 and an output");
        return FWILS_EINVAL;
    }
    FW_TRY(fwils_apply_pass(plan, pass, u, Au));   // validates, and warms up
    hipEvent_t e0, e1;
    FW_HIP(hipEventCreate(&e0));
    FW_HIP(hipEventCreate(&e1));
    fwils_status st = FWILS_OK;
    hipError_t he = hipEventRecord(e0, plan->stream);
    for (int r = 0; r < reps && he == hipSuccess && st == FWILS_OK; ++r) st = fwils_apply_pass(plan, pass, u, Au);
    if (he == hipSuccess) he = hipEventRecord(e1, plan->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FWILS_OK) return st;
    if (he != hipSuccess) {
        set_error("time_pass: %s", hipGetErrorString(he));
        return FWILS_EDEVICE;
    }
    *us = ms * 1e3f / (float)reps;
    return FWILS_OK;
}

fwils_status fwils_time_krylov_pass(fwils_plan plan, int32_t reps, float* us) {
    FW_TRY(only_2d(plan, "time_krylov_pass"));
    FW_TRY(check_plan(plan));
    if (!us || reps < 1 || reps > 10000) {
        set_error("time_krylov_pass: need reps 1..10000 and an output");
        return FWILS_EINVAL;
    }
    if (plan->krylov != FWILS_KRYLOV_BICGSTAB || !plan->bicg_state) {
        set_error("time_krylov_pass: needs a BiCGSTAB plan whose last solve was a finished BiCGSTAB solve");
        return FWILS_EINVAL;
    }
    hipStream_t s = plan->stream;
    const size_t nst = plan->total_sys;
    SysState* orig = plan->host_pipe;          // the solver's pinned staging, idle here
    SysState* run = plan->host_pipe + nst;
    FW_HIP(hipMemcpyAsync(orig, plan->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < nst; ++i) {
        if (orig[i].iter < 1 || !(orig[i].bnorm2 > 0.0) || !(orig[i].bnorm2 < 1e300)) {
            set_error("time_krylov_pass: system %zu has no completed BiCGSTAB iteration to continue from", i);
            return FWILS_EINVAL;
        }
        // every system keeps running: no convergence test, no iteration limit,
        // no restart with a fresh shadow residual
        run[i] = orig[i];
        run[i].status = ST_RUNNING;
        run[i].tol2 = 0.0;
        run[i].maxit = orig[i].iter + 1000000;
        run[i].fresh_at = 0;
    }
    // the records the pass reads (those of the last t pass; the solve's final
    // residual check reuses their buffer) are made again from s and t
    FW_HIP(hipMemcpyAsync(plan->state, run, nst * sizeof(SysState), hipMemcpyHostToDevice, s));
    for (const ProbHost& P : plan->probs) FW_HIP(bicg_t_pass(plan, P, make_view(plan, P, 0, P.p.nsys), s));
    // Back-to-back launches take the same decisions: a launch writes rho into
    // the slot of its own iteration parity and reads the other one, takes
    // omega from the t-pass records, which it does not write, and leaves the
    // iteration count alone; only x keeps accumulating its update.
    auto launch_all = [&]() -> hipError_t {
        for (const ProbHost& P : plan->probs) {
            const hipError_t e = bicg_iteration(plan, P, make_view(plan, P, 0, P.p.nsys), 0, false, s, true);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipEvent_t e0, e1;
    FW_HIP(hipEventCreate(&e0));
    FW_HIP(hipEventCreate(&e1));
    hipError_t he = launch_all();   // warm-up
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = launch_all();
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float total_ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&total_ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the last launch must have found every system running (else some blocks
    // skipped their work); then the solver's state goes back as it was
    bool all_ran = false;
    if (he == hipSuccess) he = hipMemcpyAsync(run, plan->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he == hipSuccess) {
        all_ran = true;
        for (size_t i = 0; i < nst; ++i)
            if (run[i].status != ST_RUNNING) all_ran = false;
        he = hipMemcpyAsync(plan->state, orig, nst * sizeof(SysState), hipMemcpyHostToDevice, s);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
        set_error("time_krylov_pass: %s", hipGetErrorString(he));
        return FWILS_EDEVICE;
    }
    if (!all_ran) {
        set_error("time_krylov_pass: a system left the running state during the timed launches");
        return FWILS_EINVAL;
    }
    *us = total_ms * 1e3f / (float)reps;
    return FWILS_OK;
}

fwils_status fwils_time_gmres_pass(fwils_plan plan, int32_t kind, int32_t j, int32_t reps, float* us) {
    FW_TRY(only_2d(plan, "time_gmres_pass"));
    FW_TRY(check_plan(plan));
    if (!us || reps < 1 || reps > 10000 || kind < 0 || kind > 2) {
        set_error("time_gmres_pass: need kind 0..2, reps 1..10000 and an output");
        return FWILS_EINVAL;
    }
    if (plan->krylov != FWILS_KRYLOV_GMRES || j < 0 || j >= plan->gm_m) {
        set_error("time_gmres_pass: needs a GMRES plan and 0 <= j < restart (%d)", plan->gm_m);
        return FWILS_EINVAL;
    }
    hipStream_t s = plan->stream;
    const size_t nst = plan->total_sys;
    SysState* orig = plan->host_pipe;   // the solver's pinned staging, idle here
    SysState* run = plan->host_pipe + nst;
    FW_HIP(hipMemcpyAsync(orig, plan->state, nst * sizeof(SysState), hipMemcpyDeviceToHost, s));
    FW_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < nst; ++i) {
        run[i] = orig[i];
        run[i].status = ST_RUNNING;
    }
    FW_HIP(hipMemcpyAsync(plan->state, run, nst * sizeof(SysState), hipMemcpyHostToDevice, s));
    auto launch_all = [&]() -> hipError_t {
        for (const ProbHost& P : plan->probs) {
            const GmArgs a = gm_args(plan, P);
            hipError_t e;
            if (kind == 0) {
                e = launch_gm_update(a, j, 1, false, s);
            } else if (kind == 1) {
                e = launch_gm_dots(a, j, s);
            } else {
                const GmEpi ge{a.V, a.vstride, j + 1, a.part};
                const int rows = P.p.nsys * P.rps;
                e = launch_rows_inv(P.p.nx, P.cfg.row_pi, EPI_ARNOLDI, at(plan->tmp, P), a.V + (size_t)j * a.vstride,
                                    nullptr, a.V + (size_t)(j + 1) * a.vstride, nullptr, rows, P.rps, tile_rows(P.dev),
                                    a.st, plan->tw, s, &ge);
            }
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipEvent_t e0, e1;
    FW_HIP(hipEventCreate(&e0));
    FW_HIP(hipEventCreate(&e1));
    hipError_t he = launch_all();   // warm-up
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = launch_all();
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float total_ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&total_ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (he == hipSuccess) he = hipMemcpyAsync(plan->state, orig, nst * sizeof(SysState), hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
        set_error("time_gmres_pass: %s", hipGetErrorString(he));
        return FWILS_EDEVICE;
    }
    *us = total_ms * 1e3f / (float)reps;
    return FWILS_OK;
}

fwils_status fwils_solve_status(fwils_plan plan, int32_t* status) {
    FW_TRY(check_plan(plan));
    if (!status) {
        set_error("solve_status: null output");
        return FWILS_EINVAL;
    }
    FW_HIP(hipStreamSynchronize(plan->stream));
    FW_HIP(hipMemcpy(plan->host_state, plan->state, plan->total_sys * sizeof(SysState), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < plan->total_sys; ++i) {
        switch (st_code(plan->host_state[i].status)) {
            case ST_CONVERGED: status[i] = FWILS_SYS_CONVERGED; break;
            case ST_MAXIT: status[i] = FWILS_SYS_MAXIT; break;
            case ST_BREAKDOWN: status[i] = FWILS_SYS_BREAKDOWN; break;
            case ST_NONFINITE: status[i] = FWILS_SYS_NONFINITE; break;
            default: status[i] = FWILS_SYS_RUNNING; break;
        }
    }
    return FWILS_OK;
}

fwils_status fwils_solve_stats(fwils_plan plan, int32_t* iters, double* relres) {
    FW_TRY(check_plan(plan));
    FW_HIP(hipStreamSynchronize(plan->stream));
    FW_HIP(hipMemcpy(plan->host_state, plan->state, plan->total_sys * sizeof(SysState),
                     hipMemcpyDeviceToHost));
    for (size_t i = 0; i < plan->total_sys; ++i) {
        const SysState& z = plan->host_state[i];
        if (iters) iters[i] = z.iter;
        if (relres) relres[i] = z.bnorm2 > 0 ? std::sqrt(z.rnorm2 / z.bnorm2) : 0.0;
    }
    return FWILS_OK;
}

}  // extern "C"

namespace {

// Layout of the GMRES workspace for restart length m.
struct GmLayout {
    size_t basis, sys, part, tot, total, maxnb;
};
GmLayout gm_layout(fwils_plan pl, int m) {
    GmLayout L;
    L.maxnb = 0;
    for (const ProbHost& P : pl->probs) {
        int cand[3];
        const int nc = row_candidates(P.p.nx, cand);
        for (int c = 0; c < nc; ++c)
            L.maxnb = std::max(L.maxnb, (size_t)row_geom(P.p.nx, cand[c], P.rps).blocks_per_sys);
        L.maxnb = std::max(L.maxnb, (size_t)gm_blocks_per_sys((int)P.n_per_sys));
    }
    size_t o = 0;
    L.basis = o;
    o = align256(o + (size_t)(m + 1) * pl->total_field * sizeof(cplx));
    L.sys = o;
    o = align256(o + pl->total_sys * sizeof(GmSys));
    L.part = o;
    o = align256(o + pl->total_sys * L.maxnb * kGmRec * sizeof(double));
    L.tot = o;
    o = align256(o + 3 * pl->total_sys * kGmRec * sizeof(double));
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

fwils_status fwils_gmres_workspace_size(fwils_plan plan, int32_t restart, size_t* bytes) {
    FW_TRY(check_plan(plan, false));
    if (!bytes || restart < 1 || restart > kGmMax) {
        set_error("gmres_workspace_size: restart must be 1..%d", kGmMax);
        return FWILS_EINVAL;
    }
    *bytes = gm_layout(plan, restart).total;
    return FWILS_OK;
}

fwils_status fwils_set_krylov(fwils_plan plan, int32_t method, int32_t restart, uint32_t flags, void* gws,
                              size_t bytes) {
    FW_TRY(check_plan(plan, false));
    if (flags & ~(uint32_t)FWILS_GMRES_CGS1) {
        set_error("set_krylov: unknown flags");
        return FWILS_EINVAL;
    }
    if (method == FWILS_KRYLOV_BICGSTAB) {
        drop_graphs(plan);
        plan->krylov = method;
        return FWILS_OK;
    }
    if (method != FWILS_KRYLOV_GMRES) {
        set_error("set_krylov: unknown method %d", method);
        return FWILS_EINVAL;
    }
    if (restart < 1 || restart > kGmMax) {
        set_error("set_krylov: restart must be 1..%d", kGmMax);
        return FWILS_EINVAL;
    }
    const GmLayout L = gm_layout(plan, restart);
    if (!gws || bytes < L.total || ((uintptr_t)gws & 255) != 0) {
        set_error("set_krylov: GMRES needs %zu bytes, 256-byte aligned (got %zu)", L.total, bytes);
        return FWILS_ENOMEM;
    }
    if (!plan->ws) {
        set_error("set_krylov: set the plan workspace first");
        return FWILS_ENOMEM;
    }
    char* w = static_cast<char*>(gws);
    drop_graphs(plan);
    plan->krylov = method;
    plan->gm_m = restart;
    plan->gm_cgs2 = !(flags & FWILS_GMRES_CGS1);
    plan->gm_maxnb = L.maxnb;
    plan->gm_V = reinterpret_cast<cplx*>(w + L.basis);
    plan->gm_sys = reinterpret_cast<GmSys*>(w + L.sys);
    plan->gm_part = reinterpret_cast<double*>(w + L.part);
    plan->gm_tot1 = reinterpret_cast<double*>(w + L.tot);
    plan->gm_tot2 = plan->gm_tot1 + plan->total_sys * kGmRec;
    plan->gm_tot3 = plan->gm_tot2 + plan->total_sys * kGmRec;
    return FWILS_OK;
}

}  // extern "C"

// ------------------------------------------------------------ autotuner --
namespace {

fwils_tuning to_tuning(const ProbHost& P) {
    fwils_tuning t;
    t.row_points = P.cfg.row_p;
    t.row_points_inv = P.cfg.row_pi;
    t.col_points = P.cfg.col.P;
    t.col_width = P.cfg.col.W;
    t.col_shared = P.cfg.col.seq;
    t.stencil_rows = P.cfg.st.TZ;
    t.stencil_sys = P.cfg.st.S;
    t.fused_points = P.cfg.fuse_p;
    for (int k = 0; k < 4; ++k) t.time_us[k] = P.tuned_us[k];
    return t;
}

KernelCfg from_tuning(const fwils_tuning& t) {
    KernelCfg k;
    k.row_p = t.row_points;
    k.row_pi = t.row_points_inv ? t.row_points_inv : t.row_points;
    k.col = ColCfg{t.col_points, t.col_width, t.col_shared};
    k.st = StCfg{t.stencil_rows, t.stencil_sys};
    k.fuse_p = t.fused_points;
    return k;
}

bool fuse_ok(const ProbHost& P, int fp) {
    if (fp == 0) return true;
    if (!row_points_ok(P.p.nx, fp)) return false;
    for (int vm = VM_NONE; vm <= VM_PX; ++vm) {   // every mode the solver launches
        const int F = srows_rows(P.p.nx, P.p.nz, fp, vm);
        if (F == 0 || srows_lds(P.p.nx, F) > kMaxLds) return false;
    }
    return true;
}

bool cfg_ok(const ProbHost& P, const KernelCfg& k) {
    return row_points_ok(P.p.nx, k.row_p) && row_points_ok(P.p.nx, k.row_pi) && col_cfg_ok(P.p.nz, P.p.nx, k.col) &&
           st_cfg_ok(P.p.nx, P.p.nz, k.st) && fuse_ok(P, k.fuse_p);
}

void apply_cfg(fwils_plan pl, ProbHost& P, const KernelCfg& k) {
    P.cfg = k;
    P.dev.tile_sh = col_tile_shift(P.p.nx, k.col.W);   // the spectrum follows the column blocks
    P.np_rows = row_geom(P.p.nx, k.row_pi, 2 * P.p.nz).blocks_per_sys;
    drop_graphs(pl);
}

// Candidates of one kind: the problem's current variants with that kind's
// fields replaced.
std::vector<KernelCfg> candidates(const ProbHost& P, int kind) {
    std::vector<KernelCfg> out;
    if (kind == FWILS_TUNE_STENCIL) {
        StCfg c[32];
        const int n = st_candidates(P.p.nx, P.p.nz, c, 32);
        for (int i = 0; i < n; ++i) {
            KernelCfg k = P.cfg;
            k.st = c[i];
            out.push_back(k);
        }
    } else if (kind == FWILS_TUNE_ROWS) {
        int c[3];
        const int n = row_candidates(P.p.nx, c);
        for (int i = 0; i < n; ++i) {
            KernelCfg k = P.cfg;
            k.row_p = k.row_pi = c[i];   // both row passes in this variant
            out.push_back(k);
        }
    } else if (kind == FWILS_TUNE_COLS) {
        ColCfg c[64];
        const int n = col_candidates(P.p.nz, P.p.nx, c, 64);
        for (int i = 0; i < n; ++i) {
            KernelCfg k = P.cfg;
            k.col = c[i];
            out.push_back(k);
        }
    } else if (kind == FWILS_TUNE_FUSE) {
        KernelCfg k = P.cfg;
        k.fuse_p = 0;
        out.push_back(k);
        int c[3];
        const int n = row_candidates(P.p.nx, c);
        for (int i = 0; i < n; ++i) {
            if (!fuse_ok(P, c[i])) continue;
            k.fuse_p = c[i];
            out.push_back(k);
        }
    }
    return out;
}

// The inverse row pass as an extra timing kind of the autotuner (with the
// Krylov v-epilogue: an input field, r^ and two-sum partial records).
constexpr int kTuneRowsInv = 100;

// One launch of the kernel of the given kind, variant k, over all systems of
// problem P (fields from the workspace vectors; every system active).
hipError_t tune_launch(fwils_plan pl, const ProbHost& P, int kind, const KernelCfg& k) {
    const int rows = P.p.nsys * 2 * P.p.nz;
    cplx* u = at(pl->x, P);
    cplx* tmp = at(pl->tmp, P);
    if (kind == kTuneRowsInv)
        return launch_rows_inv(P.p.nx, k.row_pi, EPI_BICG_V, tmp, u, at(pl->rhat, P), at(pl->v, P),
                               part_at(pl->partV, pl, P), rows, 2 * P.p.nz, tile_rows(P.dev), nullptr, pl->tw,
                               pl->stream);
    if (kind == FWILS_TUNE_STENCIL) return launch_body_force(k.st, u, tmp, maps_at(pl, P), P.dev, nullptr, pl->stream);
    cplx* tmp2 = at(pl->tmp2, P);
    if (kind == FWILS_TUNE_ROWS)
        return launch_rows_fwd(P.p.nx, k.row_p, tmp2, tmp, rows, 2 * P.p.nz, tile_rows(P.dev), nullptr, pl->tw,
                               pl->stream);
    if (kind == FWILS_TUNE_FUSE) {
        // the stencil and the forward rows, fused or as two kernels
        if (k.fuse_p) {
            const StencilArgs a{u, nullptr, nullptr, nullptr, nullptr, maps_at(pl, P), nullptr, 0};
            return launch_srows(0, k.fuse_p, a, tmp, P.dev, nullptr, pl->tw, pl->stream);
        }
        hipError_t e = launch_body_force(k.st, u, tmp2, maps_at(pl, P), P.dev, nullptr, pl->stream);
        if (e == hipSuccess)
            e = launch_rows_fwd(P.p.nx, k.row_p, tmp2, tmp, rows, 2 * P.p.nz, tile_rows(P.dev), nullptr, pl->tw,
                                pl->stream);
        return e;
    }
    // A column variant also fixes the spectrum layout (tiles as wide as its
    // blocks) that both row passes write and read: it is timed with them, as
    // the three passes of one convolution.
    ProbDev d = P.dev;
    d.tile_sh = col_tile_shift(P.p.nx, k.col.W);
    hipError_t e = launch_rows_fwd(P.p.nx, k.row_p, tmp2, tmp, rows, 2 * P.p.nz, tile_rows(d), nullptr, pl->tw,
                                   pl->stream);
    if (e == hipSuccess) e = launch_cols(COL_GREEN, k.col, tmp, d, nullptr, pl->tw, pl->stream);
    if (e == hipSuccess)
        e = launch_rows_inv(P.p.nx, k.row_pi, EPI_STORE, tmp, nullptr, nullptr, tmp2, nullptr, rows, 2 * P.p.nz,
                            tile_rows(d), nullptr, pl->tw, pl->stream);
    return e;
}

}  // namespace

extern "C" {

fwils_status fwils_autotune(fwils_plan plan, int32_t reps) {
    if (plan && plan->d3) return check_plan(plan);   // 3-D problems: one variant per kernel
    FW_TRY(check_plan(plan));
    if (reps < 1 || reps > 1000) {
        set_error("autotune: reps must be 1..1000");
        return FWILS_EINVAL;
    }
    hipStream_t s = plan->stream;
    hipEvent_t e0, e1;
    FW_HIP(hipEventCreate(&e0));
    FW_HIP(hipEventCreate(&e1));
    fwils_status st = FWILS_OK;
    for (ProbHost& P : plan->probs) {
        // finite inputs for every candidate
        hipError_t he = launch_zero(at(plan->x, P), (size_t)P.p.nsys * P.n_per_sys, s);
        if (he == hipSuccess) he = launch_zero(at(plan->tmp, P), (size_t)P.p.nsys * P.n_per_sys, s);
        if (he != hipSuccess) {
            set_error("autotune: %s", hipGetErrorString(he));
            st = FWILS_EDEVICE;
            break;
        }
        KernelCfg best = P.cfg;
        float best_us[4] = {0.f, 0.f, 0.f, 0.f};
        for (int kind = 0; kind < 4 && st == FWILS_OK; ++kind) {
            float tbest = 0.f;
            if (kind == FWILS_TUNE_FUSE) best.fuse_p = 0;
            P.cfg = best;   // later kinds are timed with the earlier choices
            P.dev.tile_sh = col_tile_shift(P.p.nx, best.col.W);
            float tbest_inv = 0.f;
            auto time_us = [&](int knd, const KernelCfg& k, float& us) -> hipError_t {
                float ms = 0.f;
                hipError_t e = tune_launch(plan, P, knd, k);   // warm-up (and first-use set-up)
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = tune_launch(plan, P, knd, k);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                us = ms * 1e3f / (float)reps;
                return e;
            };
            for (const KernelCfg& k : candidates(P, kind)) {
                float us = 0.f, us_inv = 0.f;
                he = time_us(kind, k, us);
                // the row variant is chosen for each direction on its own
                if (he == hipSuccess && kind == FWILS_TUNE_ROWS) he = time_us(kTuneRowsInv, k, us_inv);
                if (he != hipSuccess) {
                    set_error("autotune: %s", hipGetErrorString(he));
                    st = FWILS_EDEVICE;
                    break;
                }
                if (tbest == 0.f || us < tbest) {
                    tbest = us;
                    if (kind == FWILS_TUNE_STENCIL) best.st = k.st;
                    else if (kind == FWILS_TUNE_ROWS) best.row_p = k.row_p;
                    else if (kind == FWILS_TUNE_COLS) best.col = k.col;
                    else best.fuse_p = k.fuse_p;
                }
                if (kind == FWILS_TUNE_ROWS && (tbest_inv == 0.f || us_inv < tbest_inv)) {
                    tbest_inv = us_inv;
                    best.row_pi = k.row_pi;
                }
            }
            best_us[kind] = tbest;
        }
        if (st != FWILS_OK) break;
        apply_cfg(plan, P, best);
        for (int k = 0; k < 4; ++k) P.tuned_us[k] = best_us[k];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

fwils_status fwils_get_tuning(fwils_plan plan, int32_t iprob, fwils_tuning* out) {
    FW_TRY(only_2d(plan, "get_tuning"));
    FW_TRY(check_plan(plan, false));
    if (!out || iprob < 0 || iprob >= (int)plan->probs.size()) {
        set_error("get_tuning: bad problem index or null output");
        return FWILS_EINVAL;
    }
    *out = to_tuning(plan->probs[iprob]);
    return FWILS_OK;
}

fwils_status fwils_set_tuning(fwils_plan plan, int32_t iprob, const fwils_tuning* t) {
    FW_TRY(only_2d(plan, "set_tuning"));
    FW_TRY(check_plan(plan, false));
    if (!t || iprob < 0 || iprob >= (int)plan->probs.size()) {
        set_error("set_tuning: bad problem index or null input");
        return FWILS_EINVAL;
    }
    ProbHost& P = plan->probs[iprob];
    const KernelCfg k = from_tuning(*t);
    if (!cfg_ok(P, k)) {
        set_error("set_tuning: not a built variant for %dx%d (rows %d, cols %d/%d/%d, stencil %d/%d, fused %d)",
                  P.p.nz, P.p.nx, t->row_points, t->col_points, t->col_width, t->col_shared,
                  t->stencil_rows, t->stencil_sys, t->fused_points);
        return FWILS_EINVAL;
    }
    apply_cfg(plan, P, k);
    P.tuned_us[0] = P.tuned_us[1] = P.tuned_us[2] = P.tuned_us[3] = 0.f;
    return FWILS_OK;
}

fwils_status fwils_tuning_candidates(fwils_plan plan, int32_t iprob, int32_t kind, fwils_tuning* out,
                                     int32_t cap, int32_t* count) {
    FW_TRY(only_2d(plan, "tuning_candidates"));
    FW_TRY(check_plan(plan, false));
    if (!count || iprob < 0 || iprob >= (int)plan->probs.size() || kind < 0 || kind > 3 || cap < 0 ||
        (cap > 0 && !out)) {
        set_error("tuning_candidates: bad arguments");
        return FWILS_EINVAL;
    }
    const ProbHost& P = plan->probs[iprob];
    const std::vector<KernelCfg> c = candidates(P, kind);
    *count = (int32_t)c.size();
    for (int i = 0; i < (int)c.size() && i < cap; ++i) {
        ProbHost Q = P;
        Q.cfg = c[i];
        Q.tuned_us[0] = Q.tuned_us[1] = Q.tuned_us[2] = Q.tuned_us[3] = 0.f;
        out[i] = to_tuning(Q);
    }
    return FWILS_OK;
}

fwils_status fwils_fft2(fwils_plan plan, int32_t iprob, const void* in, void* out, int32_t inverse) {
    FW_TRY(check_plan(plan));
    FW_TRY(check_field_ptrs({in, out}));
    if (iprob < 0 || iprob >= (int)plan->probs.size()) {
        set_error("fft2: bad problem index");
        return FWILS_EINVAL;
    }
    const ProbHost& P = plan->probs[iprob];
    const int rows = P.p.nsys * P.rps;
    const cplx* src = static_cast<const cplx*>(in);
    cplx* dst = static_cast<cplx*>(out);
    hipStream_t s = plan->stream;
    if (P.d3) {   // x rows, then the y and z axes in place (unnormalised, separable)
        const ProbDev3& d = P.dev3;
        const int nx = d.nx, ny = d.ny, nz = d.nz, ns = P.p.nsys;
        const int px = row_points_default(nx);
        if (!inverse)
            FW_HIP(launch_rows_fwd(nx, px, src, dst, rows, P.rps, SpecLayout{}, nullptr, plan->tw, s));
        else
            FW_HIP(launch_rows_inv(nx, px, EPI_STORE, src, nullptr, nullptr, dst, nullptr, rows, P.rps, SpecLayout{},
                                   nullptr, plan->tw, s));
        const int mode = inverse ? AX_INV : AX_FWD;
        if (ny > 1) FW_HIP(launch_axis3(mode, ny, dst, nx, ns * 3 * nz, 3 * nz, nullptr, plan->tw, d, s));
        FW_HIP(launch_axis3(mode, nz, dst, nx * ny, ns * 3, 3, nullptr, plan->tw, d, s));
        return FWILS_OK;
    }
    ProbDev nat = P.dev;   // the transform itself: row-major in and out
    nat.tile_sh = 0;
    if (!inverse) {
        FW_HIP(launch_rows_fwd(P.p.nx, row_points_default(P.p.nx), src, dst, rows, 2 * P.p.nz, SpecLayout{}, nullptr,
                               plan->tw, s));
        FW_HIP(launch_cols(COL_FWD, col_default(P.p.nz, P.p.nx), dst, nat, nullptr, plan->tw, s));
    } else {
        FW_HIP(launch_rows_inv(P.p.nx, row_points_default(P.p.nx), EPI_STORE, src, nullptr, nullptr, dst,
                               nullptr, rows, 2 * P.p.nz, SpecLayout{}, nullptr, plan->tw, s));
        FW_HIP(launch_cols(COL_INV, col_default(P.p.nz, P.p.nx), dst, nat, nullptr, plan->tw, s));
    }
    return FWILS_OK;
}

}  // extern "C"
