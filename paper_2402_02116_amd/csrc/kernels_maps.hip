// Model-map kernels of the generalised Tikhonov step (eqs. obj, norm):
// relative maps q [nmaps][cells] (five 2-D maps, six or 22 3-D ones; the
// plan's real type), dm = m0 q, the periodic 5- or 7-point Laplacian, the combination of J* output into gradient / normal-operator
// maps, FP64 inner products and the CG updates with device-resident scalars;
// the data residual and background update of the distorted-Born loop.
#include "launch.h"

FW_BEGIN
constexpr int kMapThreads = 256;

// out[p][i] = m0[p] q[p][i]
__global__ void k_map_scale(const real* __restrict__ q, real* __restrict__ out, MapScales m0,
                            int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (i < n) out[(size_t)p * n + i] = (real)(m0.s[p] * (double)q[(size_t)p * n + i]);
}

hipError_t launch_map_scale(const real* q, real* out, const MapScales& m0, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_map_scale, dim3((n + kMapThreads - 1) / kMapThreads, m0.n), dim3(kMapThreads), 0, s,
                       q, out, m0, n);
    return hipGetLastError();
}

// Periodic, unscaled Laplacian of nmaps maps [nmaps][nz][ny][nx]: the
// 5-point stencil in x-z for ny = 1 (2-D maps), the 7-point one otherwise.
__global__ void k_laplacian(const real* __restrict__ q, real* __restrict__ out, int nx, int ny, int nz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    const int n = nx * ny * nz;
    if (i >= n) return;
    const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    const real* a = q + (size_t)p * n;
    const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
    const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
    const int row = nx * ny;
    real v = a[i - x + xp] + a[i - x + xm] + a[zp * row + y * nx + x] + a[zm * row + y * nx + x] - 4.0f * a[i];
    if (ny > 1) {
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        v += a[z * row + yp * nx + x] + a[z * row + ym * nx + x] - 2.0f * a[i];
    }
    out[(size_t)p * n + i] = v;
}

hipError_t launch_laplacian(const real* q, real* out, int nx, int ny, int nz, int nmaps, hipStream_t s) {
    const int n = nx * ny * nz;
    hipLaunchKernelGGL(k_laplacian, dim3((n + kMapThreads - 1) / kMapThreads, nmaps), dim3(kMapThreads), 0,
                       s, q, out, nx, ny, nz);
    return hipGetLastError();
}

// out = c_j m0[p] Re(g[p]) + c_l reg[p]     (reg may be null: c_l ignored)
__global__ void k_map_combine(const double2* __restrict__ g, const real* __restrict__ reg,
                              real* __restrict__ out, MapScales m0, double cj, double cl, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (i >= n) return;
    const size_t k = (size_t)p * n + i;
    double v = cj * m0.s[p] * g[k].x;
    if (reg) v += cl * (double)reg[k];
    out[k] = (real)v;
}

hipError_t launch_map_combine(const double2* g, const real* reg, real* out, const MapScales& m0,
                              double cj, double cl, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_map_combine, dim3((n + kMapThreads - 1) / kMapThreads, m0.n), dim3(kMapThreads), 0, s,
                       g, reg, out, m0, cj, cl, n);
    return hipGetLastError();
}

// ------------------------------------------------------- FP64 reductions --
// part[block] = sum over the block's elements of a[i] * b[i] (real) or
// |a[i]|^2 (complex data).  Fixed-order, deterministic.
__global__ __launch_bounds__(256) void k_dot_real(const real* __restrict__ a, const real* __restrict__ b,
                                                  double* __restrict__ part, size_t n) {
    __shared__ double red[4 * 1];
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        acc[0] += (double)a[i] * (double)b[i];
    block_allreduce<1, 256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(256) void k_norm2_complex(const cplx* __restrict__ a,
                                                       double* __restrict__ part, size_t n) {
    __shared__ double red[4 * 1];
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        acc[0] += (double)a[i].x * a[i].x + (double)a[i].y * a[i].y;
    block_allreduce<1, 256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

constexpr int kDotBlocks = kDotPartials;

// out = sum(part[0..np)) with a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int np,
                                                      double* __restrict__ out) {
    __shared__ double red[4 * 1];
    double r[1];
    sum_partials<1, 256, 1>(part, np, r, red);
    if (threadIdx.x == 0) *out = r[0];
}

hipError_t launch_dot_real(const real* a, const real* b, size_t n, double* part, double* out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_dot_real, dim3(kDotBlocks), dim3(256), 0, s, a, b, part, n);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, kDotBlocks, out);
    return hipGetLastError();
}

hipError_t launch_norm2_complex(const cplx* a, size_t n, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2_complex, dim3(kDotBlocks), dim3(256), 0, s, a, part, n);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, kDotBlocks, out);
    return hipGetLastError();
}

// ---------------------------------------------------------- CG updates ----
// Device scalars (doubles): sc[0] = rs (current <res, res>), sc[1] = <p, Ap>,
// sc[2] = new <res, res>.  hist (may be null) receives sqrt(rs) per iteration.
// x += alpha p; res -= alpha Ap with alpha = rs / <p, Ap>
__global__ void k_cg_xr(real* __restrict__ x, real* __restrict__ res, const real* __restrict__ p,
                        const real* __restrict__ Ap, const double* __restrict__ sc, size_t n) {
    const double pap = sc[1];
    const double alpha = pap != 0.0 ? sc[0] / pap : 0.0;
    const real af = (real)alpha;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        x[i] += af * p[i];
        res[i] -= af * Ap[i];
    }
}

// p = res + beta p with beta = rs_new / rs; then rs = rs_new (one thread of
// block 0 after the block's update would race with other blocks, so the
// scalar shift happens in k_cg_shift).
__global__ void k_cg_p(real* __restrict__ p, const real* __restrict__ res, const double* __restrict__ sc,
                       size_t n) {
    const double beta = sc[0] != 0.0 ? sc[2] / sc[0] : 0.0;
    const real bf = (real)beta;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = res[i] + bf * p[i];
}

__global__ void k_cg_shift(double* __restrict__ sc, double* __restrict__ hist, int it) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc[0] = sc[2];
        if (hist) hist[it] = sqrt(sc[2]);
    }
}

hipError_t launch_cg_xr(real* x, real* res, const real* p, const real* Ap, const double* sc, size_t n,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_cg_xr, dim3(1024), dim3(256), 0, s, x, res, p, Ap, sc, n);
    return hipGetLastError();
}

hipError_t launch_cg_p(real* p, const real* res, const double* sc, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_p, dim3(1024), dim3(256), 0, s, p, res, sc, n);
    return hipGetLastError();
}

hipError_t launch_cg_shift(double* sc, double* hist, int it, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_shift, dim3(1), dim3(64), 0, s, sc, hist, it);
    return hipGetLastError();
}

__global__ void k_copy_f(const real* __restrict__ a, real* __restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}
__global__ void k_zero_f(real* __restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = 0.f;
}

// d -= r (complex data)
__global__ void k_sub_complex(cplx* __restrict__ d, const cplx* __restrict__ r, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = csub(d[i], r[i]);
}

hipError_t launch_sub_complex(cplx* d, const cplx* r, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_complex, dim3(256), dim3(256), 0, s, d, r, n);
    return hipGetLastError();
}

// r = d_obs - r: the data residual of a DBI step from the gathered R u^b
__global__ void k_data_residual(cplx* __restrict__ r, const cplx* __restrict__ d_obs, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        r[i] = csub(d_obs[i], r[i]);
}

hipError_t launch_data_residual(cplx* r, const cplx* d_obs, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_data_residual, dim3(256), dim3(256), 0, s, r, d_obs, n);
    return hipGetLastError();
}

// maps[p][i] += m0[p] q[p][i] (the DBI background update, in FP64 before
// rounding to the map precision)
__global__ void k_map_update(real* __restrict__ maps, const real* __restrict__ q, MapScales m0, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y;
    if (i < n) {
        const size_t k = (size_t)p * n + i;
        maps[k] = (real)((double)maps[k] + m0.s[p] * (double)q[k]);
    }
}

hipError_t launch_map_update(real* maps, const real* q, const MapScales& m0, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_map_update, dim3((n + kMapThreads - 1) / kMapThreads, m0.n), dim3(kMapThreads), 0, s,
                       maps, q, m0, n);
    return hipGetLastError();
}

hipError_t launch_copy_f(const real* a, real* b, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_f, dim3(1024), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}
hipError_t launch_zero_f(real* b, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f, dim3(1024), dim3(256), 0, s, b, n);
    return hipGetLastError();
}

FW_END