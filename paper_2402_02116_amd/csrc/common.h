// Shared device-side definitions for the fwils HIP kernels (gfx950).
//
// The library core is compiled twice from the same sources: complex64 fields
// with fp32 maps (namespace fw::c64, the product path) and, with FW_C128
// defined, complex128 fields with fp64 maps (namespace fw::c128, the FP64
// reference of the same path).  `cplx` / `real` are the field and map types
// of the build.  Fields are [nsys][2][nz][nx] complex with x fastest; maps are
// [5][nz][nx] real in the order (dC11, dC13, dC33, dC55, drho).  Krylov
// scalars, inner products and norms are FP64 in both builds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifdef FW_C128
#define FW_NS c128
#else
#define FW_NS c64
#endif
#define FW_BEGIN namespace fw { inline namespace FW_NS {
#define FW_END } }

FW_BEGIN

#ifdef FW_C128
using real = double;
using cplx = double2;
#else
using real = float;
using cplx = float2;
#endif

// ---------------------------------------------------------------- complex --
__host__ __device__ __forceinline__ cplx mkc(real re, real im) {
    cplx z;
    z.x = re;
    z.y = im;
    return z;
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return mkc(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return mkc(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cplx cscale(cplx a, real s) { return mkc(a.x * s, a.y * s); }
__device__ __forceinline__ cplx cconj(cplx a) { return mkc(a.x, -a.y); }
// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV>
__device__ __forceinline__ cplx mul_mi(cplx z) {
    return INV ? mkc(-z.y, z.x) : mkc(z.y, -z.x);
}

__device__ __forceinline__ real rsinpi(real x) {
#ifdef FW_C128
    return sinpi(x);
#else
    return sinpif(x);
#endif
}

// 1 / x for the Green's-tensor multiply: the hardware reciprocal (within 1
// ulp) in the complex64 build, the correctly rounded division in complex128.
__device__ __forceinline__ real green_rcp(real x) {
#ifdef FW_C128
    return 1.0 / x;
#else
    return __builtin_amdgcn_rcpf(x);
#endif
}

struct dcomplex { double re, im; };

// Store of one complex value.  complex64: a write-through store (system-
// coherent policy), so the kernel's output leaves no dirty L2 lines behind
// and the cache write-back at the kernel boundary has nothing to flush.  A
// relaxed atomic store at system scope is exactly that store on gfx950
// (global_store with sc0 sc1, no waits or fences), and the compiler sees it
// as a store: it tracks the store's register hazards and orders it only
// against accesses that may alias it.  complex128: a plain 16-byte store (an
// atomic store is at most 8 bytes, and two 8-byte write-through stores per
// lane write every cache line in two halves).
__device__ __forceinline__ void st_wt(cplx* p, cplx v) {
#ifdef FW_C128
    *p = v;
#else
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
#endif
}

// --------------------------------------------------------- problem consts --
// Per-problem constants, passed by value to every kernel of that problem.
// The spectrum between the row and the column passes of a convolution may be
// stored in column tiles as wide as a column block: each [nz][nx] plane as
// [nx / w][nz][w] (w = 2^sh), so that a column block reads and writes one
// contiguous run of memory instead of short segments of long rows.

// Offset of element (z, x) inside one spectrum plane: tiled when tile_nz (the
// plane's nz) is non-zero, row-major otherwise.
__host__ __device__ __forceinline__ size_t spec_off(int z, int x, int nx, int tile_nz, int sh) {
    return tile_nz ? ((size_t)(x >> sh) * tile_nz << sh) + ((size_t)z << sh) + (x & ((1 << sh) - 1))
                   : (size_t)z * nx + x;
}

struct ProbDev {
    int nx, nz, nsys, symbol;
    int tile_sh;          // the convolution's spectrum: tiles of 2^tile_sh columns, 0 = row-major
    real inv4dx2;         // 1 / (4 dx^2): both central differences of the stencil
    cplx w2;              // w~^2 = (2 pi f (1 + i eta))^2
    // Green's symbol in units of rho0 w^2 (w real): Gamma' = Gamma / (rho0 w^2)
    real gc11, gc33, gc55, gc1355;    // C11, C33, C55, C13 + C55 over rho0 w^2
    cplx ga;              // (1 + i eta)^2 = rho0 w~^2 / (rho0 w^2)
    real gscale;          // 1 / (rho0 w^2 nx nz): Green's scale and IFFT normalisation
    real dkx, dkz;        // 2 pi / (nx dx), 2 pi / (nz dx)
    real dx;
};

// --------------------------------------------------------- solver state ---
constexpr int kPartialNV = 8;   // doubles per partial-sum record

// A status word holds a SysStatus code in its low byte.  A stop decided inside
// a kernel whose blocks still owe the system its last solution update carries
// a tag above it (the kernel that decided it), so that the blocks of that
// kernel that read the status after the decision still do their part; a later
// kernel of the iteration removes the tag.
constexpr int kStampPx = 1;      // decided by a direction-update stencil
constexpr int kStampClose = 2;   // decided by the end-of-chunk close kernel
__host__ __device__ inline int st_code(int s) { return s & 0xFF; }
__host__ __device__ inline int st_tag(int s) { return s >> 8; }
__host__ __device__ inline int st_stamp(int code, int tag) { return code | (tag << 8); }

enum SysStatus : int {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAXIT = 2,
    ST_BREAKDOWN = 3,
    ST_NONFINITE = 4,
    ST_RESTART = 5,        // converged on the recursive residual, true residual too large
    ST_CYCLE_DONE = 6,     // GMRES: cycle finished, solution update pending
};

// Per-system BiCGSTAB scalars (FP64), one struct per system.
struct SysState {
    double rho_re[2], rho_im[2];   // rho_i by iteration parity
    double alpha_re, alpha_im;     // alpha_i of the current iteration
    double omega_re, omega_im;     // omega of the last completed iteration
    double bnorm2;                 // ||b||^2
    double tol2;                   // rtol^2 ||b||^2
    double rnorm2;                 // last recursive ||r||^2 seen by a check
    double best2;                  // smallest recursive ||r||^2 at a check
    int iter;                      // completed iterations
    int status;                    // SysStatus
    int maxit;
    int restarts;                  // restarts from the true residual so far
    int best_iter;                 // iteration of best2
    int fresh_at;                  // iteration that restarts with r^ = r (0: none)
};

// ------------------------------------------------------ block reductions --
// Sum NV doubles over a block of NT threads (NT a multiple of 64), in a fixed
// order: wave shuffles, then wave partials in index order.  Every thread
// receives the result.  smem needs NV * NT / 64 doubles.
template <int NV, int NT>
__device__ __forceinline__ void block_allreduce(double (&acc)[NV], double* smem) {
    static_assert(NT % 64 == 0, "block must be whole waves");
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) smem[wave * NV + k] = acc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += smem[w * NV + k];
        acc[k] = s;
    }
    __syncthreads();
}

// Sum the first NV doubles of np partial records (record i at
// part[i * STRIDE]) in a fixed order; every thread of the block receives the
// totals.  The first NR threads read the records (the others add zeros), so
// blocks of any size NT >= NR get bit-identical totals.
template <int NV, int NT, int STRIDE = kPartialNV, int NR = NT>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int np,
                                             double (&res)[NV], double* smem) {
    static_assert(NV <= STRIDE, "record too short");
    static_assert(NR <= NT && NR % 64 == 0, "readers");
#pragma unroll
    for (int k = 0; k < NV; ++k) res[k] = 0.0;
    for (int i = threadIdx.x; threadIdx.x < NR && i < np; i += NR) {
#pragma unroll
        for (int k = 0; k < NV; ++k) res[k] += part[(size_t)i * STRIDE + k];
    }
    block_allreduce<NV, NT>(res, smem);
}

// ------------------------------------------------------ record reduction --
// tot[k] = sum over records b < nb of rec[b * stride + k], k < nval, by one
// block: groups of 64 threads (one value per lane) add records q, q + G,
// q + 2G, ... and the G group sums are added in group order, so the result
// does not depend on timing.  blockDim.x must be a multiple of 64 and smem
// must hold blockDim.x doubles.
__device__ __forceinline__ void sum_records(const double* rec, int nb, int stride, int nval, double* tot,
                                            double* smem) {
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6, ngrp = blockDim.x >> 6;
    for (int k0 = 0; k0 < nval; k0 += 64) {
        const int k = k0 + lane;
        double s = 0.0;
        if (k < nval)
            for (int b = grp; b < nb; b += ngrp) s += rec[(size_t)b * stride + k];
        smem[threadIdx.x] = s;
        __syncthreads();
        if (grp == 0 && k < nval) {
            double t = 0.0;
            for (int q = 0; q < ngrp; ++q) t += smem[q * 64 + lane];
            tot[k] = t;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ GMRES state --
constexpr int kGmMax = 32;                      // largest restart length
constexpr int kGmRec = 2 * (kGmMax + 1) + 2;    // doubles per partial record

// Per-system FP64 state of restarted GMRES with an unnormalised Arnoldi basis
// (basis vector i stored as w_i = n_i v_i, n_i = ||w_i||).  R is the
// Hessenberg matrix after the Givens rotations, column-major with leading
// dimension kGmMax + 1.
struct GmSys {
    double n2[kGmMax + 1];                       // ||w_i||^2
    double rre[(kGmMax + 1) * kGmMax], rim[(kGmMax + 1) * kGmMax];
    double cs[kGmMax], sre[kGmMax], sim[kGmMax];   // rotations (c real, s complex)
    double gre[kGmMax + 1], gim[kGmMax + 1];       // rotated right-hand side
    double yre[kGmMax], yim[kGmMax];               // update coefficients y_i / n_i
    int j;                                          // Arnoldi steps of the current cycle
    int m;                                          // restart length
    int cycles;
    int est_conv;                                   // the cycle ended on its residual estimate
};

// Workgroup ids are dealt to the 8 XCDs round-robin (id % 8).  Remap so that
// each XCD works on one contiguous range of logical blocks: neighbouring
// tiles, which share cache lines and halos, then share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    const int full = nblk & ~7;
    if (bid >= full) return bid;
    return (bid & 7) * (full >> 3) + (bid >> 3);
}

FW_END
