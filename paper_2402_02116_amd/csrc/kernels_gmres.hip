// Batched restarted GMRES(m) for the LS system A u = u0 (eq. axb): the
// Arnoldi orthogonalisation by classical Gram-Schmidt with one
// re-orthogonalisation pass (CGS2), FP64 projections and norms, and the
// Hessenberg least-squares problem solved with Givens rotations in FP64 on the
// device, one system per thread.
//
// The basis is kept unnormalised: vector i is stored as w_i = n_i v_i with
// n_i = ||w_i||, so no pass rescales it.  For w = A w_j the projection
// coefficient on w_l is c_l = <w_l, w> / n_l^2, and the Hessenberg entries of
// the normalised basis are h_lj = c_l n_l / n_j, h_{j+1,j} = n_{j+1} / n_j.
// The update x += sum_l y_l v_l becomes x += sum_l (y_l / n_l) w_l.
#include <cmath>

#include "launch.h"

FW_BEGIN
constexpr int kGmThreads = 256;
constexpr int kGmEPT = 4;

int gm_blocks_per_sys(int n) { return (n + kGmThreads * kGmEPT - 1) / (kGmThreads * kGmEPT); }
__device__ __forceinline__ int gm_nb(int n) { return (n + kGmThreads * kGmEPT - 1) / (kGmThreads * kGmEPT); }

struct GmView {
    int sys, bi, i0;
};
__device__ __forceinline__ GmView gm_idx(int nb) {
    GmView v;
    v.sys = blockIdx.x / nb;
    v.bi = blockIdx.x - v.sys * nb;
    v.i0 = v.bi * kGmThreads * kGmEPT;
    return v;
}

// ---------------------------------------------------------------- set-up --
__global__ void k_gm_init(SysState* __restrict__ st, GmSys* __restrict__ gs, int nsys, int maxit, int m) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys) return;
    SysState& z = st[sys];
    z.rho_re[0] = z.rho_re[1] = z.rho_im[0] = z.rho_im[1] = 0.0;
    z.alpha_re = z.alpha_im = z.omega_re = z.omega_im = 0.0;
    z.bnorm2 = z.tol2 = z.rnorm2 = 0.0;
    z.iter = 0;
    z.maxit = maxit;
    z.restarts = 0;
    z.status = ST_RUNNING;
    gs[sys].j = 0;
    gs[sys].m = m;
    gs[sys].cycles = 0;
    gs[sys].est_conv = 0;
}

// Start of a cycle, after r = b - A x was written to basis slot 0 with
// ||r||^2 = r2 and ||b||^2 = b2: convergence test on the true residual, else
// g = (||r||, 0, ...).
__device__ void gm_begin(SysState& z, GmSys& g, double r2, double b2, double rtol, int first) {
    if (first) {
        z.bnorm2 = b2;
        z.tol2 = rtol * rtol * b2;
    }
    z.rnorm2 = r2;
    g.n2[0] = r2;
    g.j = 0;
    // accepted when the true residual meets rtol, or 2 rtol after a cycle that
    // met rtol on its own residual estimate (the finite-precision gap between
    // the two, as for the recursive residual of BiCGSTAB)
    const bool est = !first && g.est_conv;
    g.est_conv = 0;
    if (!(r2 == r2) || r2 > 1e300) z.status = ST_NONFINITE;
    else if (z.bnorm2 == 0.0 || r2 <= z.tol2 || (est && r2 <= 4.0 * z.tol2)) z.status = ST_CONVERGED;
    else if (z.iter >= z.maxit) z.status = ST_MAXIT;
    else {
        g.gre[0] = sqrt(r2);
        g.gim[0] = 0.0;
        for (int i = 1; i <= kGmMax; ++i) g.gre[i] = g.gim[i] = 0.0;
    }
}

// ------------------------------------------------- Gram-Schmidt passes ----
// Projection coefficients c_l = tot[2l] + i tot[2l+1] divided by n_l^2.
__device__ __forceinline__ void load_coeffs(cplx* c, const double* tot, const GmSys& g, int nv) {
    for (int l = threadIdx.x; l < nv; l += blockDim.x) {
        const double inv = 1.0 / g.n2[l];
        c[l] = mkc((real)(tot[2 * l] * inv), (real)(tot[2 * l + 1] * inv));
    }
    __syncthreads();
}

// Hessenberg column j from the two projection passes and n_{j+1}^2, Givens
// rotations, and the stopping test (one thread).  hre / him: kGmMax + 1
// doubles each of LDS for the column (a private array indexed at run time
// would live in scratch memory).
__device__ void gm_hessenberg(SysState& z, GmSys& g, const double* tot1, const double* tot2, double n2next,
                              double* hre, double* him) {
    const int j = g.j;
    const int ld = kGmMax + 1;
    g.n2[j + 1] = n2next;
    const double nj = sqrt(g.n2[j]);
    for (int l = 0; l <= j; ++l) {
        const double s = sqrt(g.n2[l]) / (g.n2[l] * nj);   // n_l / (n_l^2 n_j)
        hre[l] = (tot1[2 * l] + (tot2 ? tot2[2 * l] : 0.0)) * s;
        him[l] = (tot1[2 * l + 1] + (tot2 ? tot2[2 * l + 1] : 0.0)) * s;
    }
    hre[j + 1] = sqrt(n2next) / nj;
    him[j + 1] = 0.0;
    // previous rotations: [a; b] <- [c a + s b; -conj(s) a + c b]
    for (int l = 0; l < j; ++l) {
        const double c = g.cs[l], sr = g.sre[l], si = g.sim[l];
        const double ar = hre[l], ai = him[l], br = hre[l + 1], bi = him[l + 1];
        hre[l] = c * ar + (sr * br - si * bi);
        him[l] = c * ai + (sr * bi + si * br);
        hre[l + 1] = -(sr * ar + si * ai) + c * br;
        him[l + 1] = -(sr * ai - si * ar) + c * bi;
    }
    // new rotation zeroing h_{j+1}
    const double ar = hre[j], ai = him[j], br = hre[j + 1], bi = him[j + 1];
    const double aa = sqrt(ar * ar + ai * ai), bb = sqrt(br * br + bi * bi);
    const double rho = sqrt(aa * aa + bb * bb);
    if (!(rho > 0.0) || !(rho == rho)) {
        z.status = (rho == rho) ? ST_BREAKDOWN : ST_NONFINITE;
        return;
    }
    double c, sr, si, rr, ri;
    if (aa == 0.0) {
        c = 0.0;
        sr = br / bb;
        si = -bi / bb;       // conj(b) / |b|
        rr = bb;
        ri = 0.0;
    } else {
        c = aa / rho;
        const double ur = ar / aa, ui = ai / aa;   // a / |a|
        sr = (ur * br + ui * bi) / rho;            // (a/|a|) conj(b) / rho
        si = (ui * br - ur * bi) / rho;
        rr = ur * rho;
        ri = ui * rho;
    }
    g.cs[j] = c;
    g.sre[j] = sr;
    g.sim[j] = si;
    for (int l = 0; l < j; ++l) {
        g.rre[j * ld + l] = hre[l];
        g.rim[j * ld + l] = him[l];
    }
    g.rre[j * ld + j] = rr;
    g.rim[j * ld + j] = ri;
    // g_{j+1} = -conj(s) g_j, g_j = c g_j
    const double gr = g.gre[j], gi = g.gim[j];
    g.gre[j + 1] = -(sr * gr + si * gi);
    g.gim[j + 1] = -(sr * gi - si * gr);
    g.gre[j] = c * gr;
    g.gim[j] = c * gi;
    g.j = j + 1;
    z.iter += 1;
    const double res2 = g.gre[j + 1] * g.gre[j + 1] + g.gim[j + 1] * g.gim[j + 1];
    z.rnorm2 = res2;
    if (!(res2 == res2)) z.status = ST_NONFINITE;
    else if (res2 <= z.tol2 || g.j == g.m || z.iter >= z.maxit || !(n2next > 0.0)) {
        z.status = ST_CYCLE_DONE;
        g.est_conv = res2 <= z.tol2 ? 1 : 0;
    }
}

// w <- w - sum_{l <= j} c_l w_l in basis slot j + 1, with c from tot (pass 1:
// the epilogue's projections, pass 2: the re-orthogonalisation's).  With
// `final`, also a partial ||w||^2 record per block.
__global__ __launch_bounds__(kGmThreads) void k_gm_update(GmArgs a, int j, int pass, int final) {
    __shared__ cplx c[kGmMax + 1];
    __shared__ double red[4 * 4];
    const int nb = gm_nb(a.n);
    const GmView vi = gm_idx(nb);
    if (a.st[vi.sys].status != ST_RUNNING) return;
    const GmSys& g = a.gs[vi.sys];
    const double* tot = (pass == 1 ? a.tot1 : a.tot2) + (size_t)vi.sys * kGmRec;
    load_coeffs(c, tot, g, j + 1);
    const size_t off = (size_t)vi.sys * a.n;
    cplx* w = a.V + (size_t)(j + 1) * a.vstride + off;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kGmEPT; ++e) {
        const int i = vi.i0 + e * kGmThreads + threadIdx.x;
        if (i < a.n) {
            cplx x = w[i];
            for (int l = 0; l <= j; ++l) x = csub(x, cmul(c[l], a.V[(size_t)l * a.vstride + off + i]));
            st_wt(w + i, x);
            acc[0] += (double)x.x * x.x + (double)x.y * x.y;
        }
    }
    if (!final) return;
    block_allreduce<4, kGmThreads>(acc, red);
    if (threadIdx.x == 0) a.part[((size_t)vi.sys * nb + vi.bi) * kGmRec] = acc[0];
}

// tot2 = <w_l, w>, l <= j, for w in slot j + 1 (the re-orthogonalisation's
// projections), summed by each system's last block.
__global__ __launch_bounds__(kGmThreads) void k_gm_dots(GmArgs a, int j) {
    __shared__ double red[4 * 4];
    const int nb = gm_nb(a.n);
    const GmView vi = gm_idx(nb);
    if (a.st[vi.sys].status != ST_RUNNING) return;
    const size_t off = (size_t)vi.sys * a.n;
    const cplx* w = a.V + (size_t)(j + 1) * a.vstride + off;
    cplx x[kGmEPT];
#pragma unroll
    for (int e = 0; e < kGmEPT; ++e) {
        const int i = vi.i0 + e * kGmThreads + threadIdx.x;
        x[e] = (i < a.n) ? w[i] : mkc(0.f, 0.f);
    }
    double* rec = a.part + ((size_t)vi.sys * nb + vi.bi) * kGmRec;
    for (int l0 = 0; l0 <= j; l0 += 2) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int l = l0 + k;
            if (l > j) break;
            const cplx* v = a.V + (size_t)l * a.vstride + off;
#pragma unroll
            for (int e = 0; e < kGmEPT; ++e) {
                const int i = vi.i0 + e * kGmThreads + threadIdx.x;
                if (i < a.n) {
                    const cplx b = v[i];
                    acc[2 * k] += (double)b.x * x[e].x + (double)b.y * x[e].y;
                    acc[2 * k + 1] += (double)b.x * x[e].y - (double)b.y * x[e].x;
                }
            }
        }
        block_allreduce<4, kGmThreads>(acc, red);
        if (threadIdx.x == 0) {
            for (int k = 0; k < 4 && 2 * l0 + k < 2 * (j + 1); ++k) rec[2 * l0 + k] = acc[k];
        }
    }
}

// One block per system: sum the previous kernel's records, then (by mode)
// the Hessenberg column or the cycle-start test.
// One block per system has few blocks on the chip, so the records are summed
// by 16 groups of 64 lanes (a 384^2 system has 288 norm records): the
// four-grid GMRES(16) solve took 364.6-366.4 ms against 372.9-373.5 ms with
// 4 groups.
constexpr int kGmSumThreads = 1024;
__global__ __launch_bounds__(kGmSumThreads) void k_gm_sum(GmArgs a, int mode, int nb, int j, int cgs2,
                                                      double rtol, int first) {
    __shared__ double sm[kGmSumThreads];
    __shared__ double hcol[2 * (kGmMax + 1)];
    const int sys = blockIdx.x;
    SysState& z = a.st[sys];
    if (z.status != ST_RUNNING) return;
    const double* rec = a.part + (size_t)sys * nb * kGmRec;
    double* tot = (mode == GM_SUM_PROJ1 ? a.tot1 : mode == GM_SUM_PROJ2 ? a.tot2 : a.tot3) + (size_t)sys * kGmRec;
    const int nval = (mode == GM_SUM_HESS) ? 1 : (mode == GM_SUM_BEGIN) ? 2 : 2 * (j + 1);
    sum_records(rec, nb, kGmRec, nval, tot, sm);
    if (threadIdx.x != 0) return;
    if (mode == GM_SUM_HESS)
        gm_hessenberg(z, a.gs[sys], a.tot1 + (size_t)sys * kGmRec, cgs2 ? a.tot2 + (size_t)sys * kGmRec : nullptr,
                      tot[0], hcol, hcol + kGmMax + 1);
    else if (mode == GM_SUM_BEGIN)
        gm_begin(z, a.gs[sys], tot[0], tot[1], rtol, first);
}

// ------------------------------------------------------------ cycle end --
// R y = g by back substitution (k = steps of the cycle); stores y_l / n_l.
__global__ void k_gm_solve(const SysState* __restrict__ st, GmSys* __restrict__ gs, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys || st[sys].status != ST_CYCLE_DONE) return;
    GmSys& g = gs[sys];
    const int k = g.j, ld = kGmMax + 1;
    for (int i = k - 1; i >= 0; --i) {
        double sr = g.gre[i], si = g.gim[i];
        for (int l = i + 1; l < k; ++l) {
            const double ar = g.rre[l * ld + i], ai = g.rim[l * ld + i];
            sr -= ar * g.yre[l] - ai * g.yim[l];
            si -= ar * g.yim[l] + ai * g.yre[l];
        }
        const double dr = g.rre[i * ld + i], di = g.rim[i * ld + i];
        const double d = dr * dr + di * di;
        g.yre[i] = (sr * dr + si * di) / d;
        g.yim[i] = (si * dr - sr * di) / d;
    }
    for (int i = 0; i < k; ++i) {
        const double s = 1.0 / sqrt(g.n2[i]);
        g.yre[i] *= s;
        g.yim[i] *= s;
    }
}

// x += sum_{l < k} (y_l / n_l) w_l for systems at the end of a cycle.
__global__ __launch_bounds__(kGmThreads) void k_gm_xupdate(cplx* __restrict__ x, GmArgs a) {
    __shared__ cplx c[kGmMax];
    const int nb = gm_nb(a.n);
    const GmView vi = gm_idx(nb);
    if (a.st[vi.sys].status != ST_CYCLE_DONE) return;
    const GmSys& g = a.gs[vi.sys];
    const int k = g.j;
    for (int l = threadIdx.x; l < k; l += blockDim.x) c[l] = mkc((real)g.yre[l], (real)g.yim[l]);
    __syncthreads();
    const size_t off = (size_t)vi.sys * a.n;
#pragma unroll
    for (int e = 0; e < kGmEPT; ++e) {
        const int i = vi.i0 + e * kGmThreads + threadIdx.x;
        if (i < a.n) {
            cplx s = x[off + i];
            for (int l = 0; l < k; ++l) s = cadd(s, cmul(c[l], a.V[(size_t)l * a.vstride + off + i]));
            st_wt(x + off + i, s);
        }
    }
}

// Systems at the end of a cycle go back to RUNNING for the true-residual test.
__global__ void k_gm_next(SysState* __restrict__ st, GmSys* __restrict__ gs, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys || st[sys].status != ST_CYCLE_DONE) return;
    st[sys].status = ST_RUNNING;
    gs[sys].cycles += 1;
}

// Per-system outputs: iterations and the true relative residual of the last
// cycle start.
__global__ void k_gm_report(const SysState* __restrict__ st, int32_t* iters, double* relres, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys) return;
    if (iters) iters[sys] = st[sys].iter;
    if (relres) relres[sys] = st[sys].bnorm2 > 0.0 ? sqrt(st[sys].rnorm2 / st[sys].bnorm2) : 0.0;
}

// ------------------------------------------------------------- launchers --
static dim3 per_sys_grid(int nsys) { return dim3((nsys + 63) / 64); }

hipError_t launch_gm_init(SysState* st, GmSys* gs, int nsys, int maxit, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_init, per_sys_grid(nsys), dim3(64), 0, s, st, gs, nsys, maxit, m);
    return hipGetLastError();
}

hipError_t launch_gm_sum(const GmArgs& a, int mode, int nb, int j, bool cgs2, double rtol, bool first,
                         hipStream_t s) {
    if (mode < GM_SUM_PROJ1 || mode > GM_SUM_BEGIN || j < 0 || j >= kGmMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gm_sum, dim3(a.nsys), dim3(kGmSumThreads), 0, s, a, mode, nb, j, cgs2 ? 1 : 0, rtol,
                       first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gm_update(const GmArgs& a, int j, int pass, bool final, hipStream_t s) {
    if (j < 0 || j >= kGmMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gm_update, dim3(a.nsys * gm_blocks_per_sys(a.n)), dim3(kGmThreads), 0, s, a, j, pass,
                       final ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gm_dots(const GmArgs& a, int j, hipStream_t s) {
    if (j < 0 || j >= kGmMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gm_dots, dim3(a.nsys * gm_blocks_per_sys(a.n)), dim3(kGmThreads), 0, s, a, j);
    return hipGetLastError();
}

hipError_t launch_gm_report(const SysState* st, int32_t* iters, double* relres, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_report, per_sys_grid(nsys), dim3(64), 0, s, st, iters, relres, nsys);
    return hipGetLastError();
}

hipError_t launch_gm_finish_cycle(cplx* x, const GmArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_solve, per_sys_grid(a.nsys), dim3(64), 0, s, a.st, a.gs, a.nsys);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gm_xupdate, dim3(a.nsys * gm_blocks_per_sys(a.n)), dim3(kGmThreads), 0, s, x, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gm_next, per_sys_grid(a.nsys), dim3(64), 0, s, a.st, a.gs, a.nsys);
    return hipGetLastError();
}

FW_END