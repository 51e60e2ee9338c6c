// Host-side launchers of the fwils kernels (internal interface between the
// C ABI in capi.cpp and the HIP translation units).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

FW_BEGIN
// Epilogues of the inverse row transform that ends a convolution y = G0 conv b.
enum RowEpilogue : int {
    EPI_STORE = 0,     // out = y
    EPI_APPLY = 1,     // out = u - y                          (A u)
    EPI_BICG_V = 2,    // out = u - y;  partial <aux, out>      (v = A p, <r^, v>)
    EPI_BICG_T = 3,    // out = u - y;  partials <out, u>, ||out||^2, ||u||^2, <aux, u>, <aux, out>
                       //   (t = A s, aux = r^); block 0 of each system counts the iteration
    EPI_TRUERES = 4,   // out = aux - (u - y); partial ||out||^2       (r = b - A x)
    EPI_ARNOLDI = 5,   // out = u - y = w; partial <basis_l, w>, l < nv
    EPI_GMRES_R0 = 6,  // out = aux - (u - y); partial ||out||^2, ||aux||^2
};

// Extra arguments of the GMRES epilogues (unused by the others).
struct GmEpi {
    const cplx* V;   // basis vector 0, indexed like the transform's output
    size_t vstride;    // complex elements between basis vectors
    int nv;            // basis vectors to project on
    double* part;      // [sys][blocks][kGmRec] partial records
};

enum ColMode : int { COL_GREEN = 0, COL_FWD = 1, COL_INV = 2 };

// FFT sizes the library has kernels for: 2^a 3^b, 16 <= n <= 2048.
bool fft_size_supported(int n);

constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

// Kernel variants of one problem (chosen by the autotuner or the caller).
struct ColCfg {
    int P;     // points per thread
    int W;     // columns per block
    int seq;   // 1: the two components share one LDS buffer; 2: they are
               // transformed by separate threads (Green pass only); 3: as 1 in
               // blocks of up to 1024 threads; 4: as 0 with the twiddle
               // table in LDS and W a compile-time constant (Green pass only)
};
struct StCfg {
    int TZ;    // tile height (rows), or the rows of a step of the z-marching kernel
    int S;     // systems per block, 0 = chosen from the grid size, kStMarch = the
               // z-marching kernel (one system per block)
};
constexpr int kStMarch = -1;
struct KernelCfg {
    int row_p;   // forward row-transform points per thread
    int row_pi;  // inverse row-transform points per thread (its epilogues hold more registers)
    ColCfg col;
    StCfg st;
    int fuse_p;  // 0: separate stencil and forward row pass; else the fused
                 // stencil + row kernel with this many points per thread
};

// Launch geometry of a variant (also used to size partial buffers).
struct RowGeom { int F; int threads; int blocks_per_sys; };
RowGeom row_geom(int n, int P, int nrows_per_sys);
struct ColGeom { int threads; int slots; size_t lds; };
ColGeom col_geom(int nz, int nx, const ColCfg& c);

// Variants: defaults, validity, and the candidate lists of the autotuner.
int row_points_default(int n);
bool row_points_ok(int n, int P);
int row_candidates(int n, int* out);          // at most 3
ColCfg col_default(int nz, int nx);
bool col_cfg_ok(int nz, int nx, const ColCfg& c);
int col_candidates(int nz, int nx, ColCfg* out, int cap);
StCfg st_default();
bool st_cfg_ok(int nx, int nz, const StCfg& c);
int st_candidates(int nx, int nz, StCfg* out, int cap);
KernelCfg kernel_cfg_default(int nx, int nz);

// Twiddle table tw[m] = exp(-2 pi i m / n), m < n, for every supported n,
// packed back to back; offset of size n in complex elements.
size_t twiddle_table_elems();
size_t twiddle_offset(int n);
void twiddle_table_fill(cplx* host);

// Row transforms over nrows rows of length n (rows_per_sys rows per system;
// a block never straddles systems).  st (may be null): systems whose status is
// not RUNNING are skipped.
// P is the points-per-thread variant (row_points_ok).  lay: the layout of
// the spectrum side (the forward pass's output, the inverse pass's input):
// row-major (nz = 0) or tiles of 2^sh columns (needs distinct in / out).
struct SpecLayout {
    int nz = 0, sh = 0;
};
hipError_t launch_rows_fwd(int n, int P, const cplx* in, cplx* out, int nrows, int rows_per_sys, SpecLayout lay,
                           const SysState* st, const cplx* tw, hipStream_t s);
hipError_t launch_rows_inv(int n, int P, int epi, const cplx* in, const cplx* u, const cplx* aux,
                           cplx* out, double* partials, int nrows, int rows_per_sys, SpecLayout lay,
                           const SysState* st, const cplx* tw, hipStream_t s, const GmEpi* ge = nullptr);
// The spectrum layout of problem d's convolutions.
inline SpecLayout tile_rows(const ProbDev& d) { return d.tile_sh ? SpecLayout{d.nz, d.tile_sh} : SpecLayout{}; }
// Column-tile shift for a column pass of W-column blocks on rows of nx points:
// tiles as wide as the block (4 to 32 columns), row-major for narrower blocks.
inline int col_tile_shift(int nx, int W) {
    if (W < 4 || nx % W != 0 || (W & (W - 1)) != 0) return 0;
    int sh = 0;
    while ((1 << sh) < W) ++sh;
    return sh;
}
// Column pass over [nsys][2][nz][nx] in place (column-tiled when pd.tile_sh).
// COL_FWD / COL_INV exist in the default points-per-thread variant with
// shared LDS only.
hipError_t launch_cols(int mode, const ColCfg& c, cplx* data, const ProbDev& pd, const SysState* st,
                       const cplx* tw, hipStream_t s);

// Body force b = w~^2 drho u + div_h(dC : E_h u) of one problem.
hipError_t launch_body_force(const StCfg& c, const cplx* u, cplx* b, const real* maps,
                             const ProbDev& pd, const SysState* st, hipStream_t s);
// Vector update fused into a stencil's load of its input field:
//   VM_NONE: the input is u itself;
//   VM_P:    p = r + beta (p_old - omega v)   (BiCGSTAB direction update)
//   VM_S:    s = r - alpha v                  (BiCGSTAB intermediate residual)
//   VM_PX:   the previous iteration's closing updates folded into the next
//            direction update: r = s - omega t, x += alpha p_old + omega s
//            (own cells), then p = r + beta (p_old - omega v)
enum StencilVec : int { VM_NONE = 0, VM_P = 1, VM_S = 2, VM_PX = 3 };

// The stencil with a BiCGSTAB vector update fused into its input (vm: 0 none,
// 1 p = r + beta (p_old - omega v) [u = r, a1 = p_old, a2 = v, wout = p_new,
// part = <rhat, r> records], 2 s = r - alpha v [u = r, a1 = v, wout = s,
// part = <rhat, v> records], 3 the previous iteration's r = s - omega t and
// x += alpha p_old + omega s, then p = r + beta (p_old - omega v) [u = s,
// a1 = p_old, a2 = v, a3 = t, xio = x, rout = r, wout = p_new, part = the
// t-pass records]).
struct StencilArgs {
    const cplx* u;
    const cplx* a1;
    const cplx* a2;
    cplx* wout;
    cplx* b;
    const real* maps;
    const double* part;
    int np;
    cplx* rhat = nullptr;        // vm 1, 3: shadow residual, set to r when the iteration restarts
    const cplx* a3 = nullptr;    // vm 3: t
    cplx* xio = nullptr;         // vm 3: x (updated)
    cplx* rout = nullptr;        // vm 3: r (written)
};
hipError_t launch_stencil(int vm, const StCfg& c, const StencilArgs& a, const ProbDev& pd, SysState* st,
                          hipStream_t s);
// The BiCGSTAB update of a stencil's input (vm = VM_P, VM_PX or VM_S, the
// fields of StencilArgs as for launch_stencil) as a streaming pass over the n
// complex values per system of nsys systems, writing the updated input to
// a.wout (and r, x, r^ as the fused modes do); the plain stencil follows.
hipError_t launch_bicg_update(int vm, const StencilArgs& a, long long n, int nsys, SysState* st, hipStream_t s);
// The stencil fused with the forward row transform: b (of the updated input,
// vm as above, a.b unused) row-transformed into out.  Rows up to kSrowsMaxN.
constexpr int kSrowsMaxN = 512;
int srows_rows(int nx, int nz, int P, int vm);  // rows per block in mode vm, 0 if unavailable
size_t srows_lds(int nx, int F);
hipError_t launch_srows(int vm, int P, const StencilArgs& a, cplx* out, const ProbDev& pd, SysState* st,
                        const cplx* tw, hipStream_t s);

// ------------------------------------------------------------- 3-D ------
// A 3-D problem: fields [nsys][3][nz][ny][nx] (u_x, u_y, u_z), a general
// background given by its 21 Voigt constants, and the contrast as VTI maps
// [6][nz][ny][nx] (dC11, dC13, dC33, dC55, dC66, drho) or general maps
// [22][nz][ny][nx] (the 21 constants of the upper triangle of the 6 x 6
// matrix in row-major order, then drho).
constexpr int kParamsVti = 0;
constexpr int kParamsGeneral = 1;
struct ProbDev3 {
    int nx, ny, nz, nsys;
    int params;           // kParamsVti or kParamsGeneral
    int symbol;           // 0 spectral, 1 central-difference wavenumbers
    real inv4dx2;         // 1 / (4 dx^2)
    cplx w2;              // w~^2
    real dx;
    // Green's symbol in units of rho0 w^2 (w real): the scaled Christoffel
    // entry Gamma'_p, p in (xx, yy, zz, yz, xz, xy), is sum_q gq[p][q] mono_q
    // with mono = (kx^2, ky^2, kz^2, ky kz, kx kz, kx ky)
    real gq[6][6];
    cplx ga;              // (1 + i eta)^2
    real gscale;          // 1 / (rho0 w^2 nx ny nz)
    real dk[3];           // 2 pi / (n dx) per axis
};
enum AxisMode : int { AX_FWD = 0, AX_INV = 1, AX_GREEN = 2 };
bool axis3_size_supported(int n);   // 3-D axis lengths: 2^a 3^b 5^c from 16 to 256 (see kernels_3d.hip)
int axis_points(int n);
// Contrast stencil of a 3-D problem with the vector update of StencilArgs.
hipError_t launch_stencil3(int vm, const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s);
// Strided-axis transforms in place: [nslab][n][S] (AX_FWD / AX_INV; system of
// a slab = slab / slabs_per_sys) or [nsys][3][n][S] (AX_GREEN, nslab = nsys,
// the z pass with the 3 x 3 Green multiply and the 1 / (nx ny nz) scale).
hipError_t launch_axis3(int mode, int n, cplx* data, int S, int nslab, int slabs_per_sys, const SysState* st,
                        const cplx* tw, const ProbDev3& pd, hipStream_t s);
hipError_t launch_point_sources3(cplx* f, const int32_t* src_ixyz, const double* src_f, const ProbDev3& pd,
                                 hipStream_t s);
hipError_t launch_gather3(const cplx* w, cplx* d, const int32_t* rec, int nrec, const ProbDev3& pd, hipStream_t s);
// f += R^T conj(d); perm / glen: the receivers in stable cell order and the
// run lengths of receivers sharing a cell (at each run's first entry, else 0).
hipError_t launch_scatter_conj3(const cplx* d, cplx* f, const int32_t* rec, const int32_t* perm,
                                const int32_t* glen, int nrec, const ProbDev3& pd, hipStream_t s);
// J* correlation of eq. ad1 into FP64 complex maps [NS + 1][nz][ny][nx].
hipError_t launch_correlate3(const cplx* ua, const cplx* ub, double2* g, const ProbDev3& pd, bool accumulate,
                             hipStream_t s);

// BiCGSTAB pieces (one problem; n = 2 nz nx complex per system).
int vec_blocks_per_sys(int n);
hipError_t launch_bicg_init(const cplx* b, const cplx* r0, cplx* x, cplx* r, cplx* rhat,
                            cplx* p, cplx* v, double* partXR, double* partB, int nsys, int n,
                            bool zero_x, hipStream_t s);
hipError_t launch_bicg_state_init(SysState* st, const double* partXR, const double* partB,
                                  int nsys, int npart, double rtol, int maxit, hipStream_t s);
hipError_t launch_bicg_close(cplx* x, cplx* r, const cplx* p, const cplx* sv, const cplx* t,
                             const double* partT, int npT, SysState* st, int nsys, int n, hipStream_t s);
hipError_t launch_bicg_restart_mark(SysState* st, const double* partTR, int npTR, int nsys, double limit2,
                                    int max_restarts, hipStream_t s);
hipError_t launch_bicg_restart(SysState* st, int nsys, hipStream_t s);
hipError_t launch_bicg_finish(const SysState* st, const double* partTR, int npTR, int nsys,
                              int32_t* iters, double* relres, hipStream_t s);

// Batched restarted GMRES (one problem).
struct GmArgs {
    cplx* V;          // basis slot 0 of this problem (system 0)
    size_t vstride;     // complex elements between basis slots
    GmSys* gs;          // per-system FP64 state
    SysState* st;       // per-system status / iteration count
    double* part;       // [sys][blocks][kGmRec] partial records
    double* tot1;       // [sys][kGmRec] projections of the Arnoldi epilogue
    double* tot2;       // [sys][kGmRec] projections of the re-orthogonalisation
    double* tot3;       // [sys][kGmRec] norms
    int nsys;
    int n;              // complex elements per system
};
int gm_blocks_per_sys(int n);
hipError_t launch_gm_init(SysState* st, GmSys* gs, int nsys, int maxit, int m, hipStream_t s);
// Sums of the per-block records (nb per system) of the previous GMRES kernel:
// GM_SUM_PROJ1 / GM_SUM_PROJ2 into tot1 / tot2 (2 (j + 1) values),
// GM_SUM_HESS ||w||^2 into tot3 and then Hessenberg column j, Givens
// rotation and stopping test, GM_SUM_BEGIN ||r||^2, ||b||^2 into tot3 and
// then the cycle-start test (first: also sets ||b||).
enum GmSum : int { GM_SUM_PROJ1 = 0, GM_SUM_PROJ2 = 1, GM_SUM_HESS = 2, GM_SUM_BEGIN = 3 };
hipError_t launch_gm_sum(const GmArgs& a, int mode, int nb, int j, bool cgs2, double rtol, bool first,
                         hipStream_t s);
hipError_t launch_gm_update(const GmArgs& a, int j, int pass, bool final, hipStream_t s);
hipError_t launch_gm_dots(const GmArgs& a, int j, hipStream_t s);
hipError_t launch_gm_finish_cycle(cplx* x, const GmArgs& a, hipStream_t s);
hipError_t launch_gm_report(const SysState* st, int32_t* iters, double* relres, int nsys, hipStream_t s);

// Sources, receivers, correlation.
hipError_t launch_point_sources(cplx* f, const int32_t* src_ixz, const double* src_f,
                                const ProbDev& pd, hipStream_t s);
hipError_t launch_gather(const cplx* w, cplx* d, const int32_t* rec_ixz, int nrec,
                         const ProbDev& pd, hipStream_t s);
hipError_t launch_scatter_conj(const cplx* d, cplx* f, const int32_t* rec_ixz, const int32_t* perm,
                               const int32_t* glen, int nrec, const ProbDev& pd, hipStream_t s);
hipError_t launch_correlate(const cplx* ua, const cplx* ub, cplx* g, const ProbDev& pd,
                            bool accumulate, hipStream_t s);
// The same correlation into FP64 complex maps (the Tikhonov step's
// accumulator: for fields in m/N the absolute J* r lies below fp32's range).
hipError_t launch_correlate_f64(const cplx* ua, const cplx* ub, double2* g, const ProbDev& pd,
                                bool accumulate, hipStream_t s);
hipError_t launch_zero_d2(double2* dst, size_t n, hipStream_t s);
hipError_t launch_copy(const cplx* src, cplx* dst, size_t n, hipStream_t s);
hipError_t launch_diff(const cplx* a, const cplx* b, cplx* out, size_t n, hipStream_t s);
hipError_t launch_zero(cplx* dst, size_t n, hipStream_t s);

// Tikhonov-step model maps (5 maps of one grid).
struct MapScales { double s[22]; int n; };   // per-map scales m0 and the map count
hipError_t launch_map_scale(const real* q, real* out, const MapScales& m0, int n, hipStream_t s);
hipError_t launch_laplacian(const real* q, real* out, int nx, int ny, int nz, int nmaps, hipStream_t s);
hipError_t launch_map_combine(const double2* g, const real* reg, real* out, const MapScales& m0,
                              double cj, double cl, int n, hipStream_t s);
constexpr int kDotPartials = 512;
hipError_t launch_dot_real(const real* a, const real* b, size_t n, double* part, double* out,
                           hipStream_t s);
hipError_t launch_norm2_complex(const cplx* a, size_t n, double* part, double* out, hipStream_t s);
hipError_t launch_cg_xr(real* x, real* res, const real* p, const real* Ap, const double* sc, size_t n,
                        hipStream_t s);
hipError_t launch_cg_p(real* p, const real* res, const double* sc, size_t n, hipStream_t s);
hipError_t launch_cg_shift(double* sc, double* hist, int it, hipStream_t s);
hipError_t launch_copy_f(const real* a, real* b, size_t n, hipStream_t s);
hipError_t launch_zero_f(real* b, size_t n, hipStream_t s);
hipError_t launch_sub_complex(cplx* d, const cplx* r, size_t n, hipStream_t s);
hipError_t launch_data_residual(cplx* r, const cplx* d_obs, size_t n, hipStream_t s);
hipError_t launch_map_update(real* maps, const real* q, const MapScales& m0, int n, hipStream_t s);

FW_END