// Kernel templates of the FFT passes of the LS matvec (eqs. A and FFT):
//   k_rows  - forward row transforms (after the contrast stencil), and
//             inverse row transforms fused with the LS / BiCGSTAB epilogues
//             and their FP64 partial inner products;
//   k_cols  - column transforms fused with the multiplication by the
//             wavenumber-domain Green's tensor G_hat(k), in place.
// Each translation unit that launches a (size, points-per-thread) variant
// instantiates it from here.
#pragma once

#include "fft.h"
#include "launch.h"

FW_BEGIN
// ------------------------------------------------------- block reduce ----
// Runtime block size (a multiple of 64, at most 256): fixed-order sum of
// NV doubles; thread 0 receives the total.
template <int NV>
__device__ __forceinline__ void block_sum_to0(double (&acc)[NV], double* smem) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) smem[wave * NV + k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += smem[w * NV + k];
            acc[k] = s;
        }
    }
}

// --------------------------------------------------------- row kernel ----
struct RowLds {
    cplx* p;
    __device__ __forceinline__ cplx& operator()(int, int pos) const { return p[lds_pad(pos)]; }
    __device__ __forceinline__ cplx& padded(int, int pp) const { return p[pp]; }
};

// Row transforms of F rows per block, P points per thread (T = N / P threads
// per row).  The spectrum side (the forward pass's output, the inverse pass's
// input) is in tiles of 2^tile_sh columns when tile_nz (= nz) is non-zero.  `in` and `out`
// may be the same array only with row-major spectra (in-place forward pass):
// every block reads all of its rows before its barriers and writes them after.
template <int N, int P, bool INV, int EPI>
__global__ __launch_bounds__(256) void k_rows(const cplx* in, cplx* out,
                                              const cplx* __restrict__ u,
                                              const cplx* __restrict__ aux,
                                              double* __restrict__ partials, int nrows,
                                              int rows_per_sys, int F, int tile_nz, int tile_sh,
                                              SysState* __restrict__ st,
                                              const cplx* __restrict__ tw, GmEpi ge) {
    using S = FftShape<N, P>;
    constexpr int T = S::T;
    constexpr int PL = PaddedLen<N>::value;
    extern __shared__ cplx lds_dyn[];
    __shared__ double red[4 * kPartialNV];

    const int tid = threadIdx.x;
    const int q = tid / T, t = tid % T;
    const int row0 = blockIdx.x * F;
    const int sys = row0 / rows_per_sys;
    if (st != nullptr && st[sys].status != ST_RUNNING) return;
    const int row = row0 + q;
    const bool active = (q < F) && (row < nrows);

    // spectrum positions of this row's points (tiled layout: plane, row in plane)
    size_t sbase = (size_t)row * N;
    int srow = 0;
    const bool tiled = tile_nz != 0;
    if (tiled) {
        srow = row % tile_nz;
        sbase = (size_t)(row / tile_nz) * tile_nz * N;
    }
    auto spos = [&](int x) -> size_t { return sbase + (tiled ? spec_off(srow, x, N, tile_nz, tile_sh) : (size_t)x); };

    cplx v[1][P];
    if (active) {
        if constexpr (INV) {
#pragma unroll
            for (int m = 0; m < P; ++m) v[0][m] = in[spos(t + T * m)];
        } else {
            const cplx* src = in + (size_t)row * N;
#pragma unroll
            for (int m = 0; m < P; ++m) v[0][m] = src[t + T * m];
        }
    } else {
#pragma unroll
        for (int m = 0; m < P; ++m) v[0][m] = mkc(0.f, 0.f);
    }
    // The epilogue's input vectors are loaded before the transform, so that
    // they are in flight during its passes instead of after them (inverse
    // rows at 256^2 x 16: 9.8 -> 7.1 us; at 1024^2 x 128: 4.47 -> 3.75 ms).
    constexpr bool kPre = INV && EPI != EPI_STORE;
    constexpr bool kPreA = INV && (EPI == EPI_BICG_V || EPI == EPI_BICG_T || EPI == EPI_TRUERES ||
                                   EPI == EPI_GMRES_R0);
    cplx upre[kPre ? P : 1], apre[kPreA ? P : 1];
    if constexpr (kPre) {
        if (active) {
#pragma unroll
            for (int m = 0; m < P; ++m) upre[m] = u[(size_t)row * N + t + T * m];
        }
    }
    if constexpr (kPreA) {
        if (active) {
#pragma unroll
            for (int m = 0; m < P; ++m) apre[m] = aux[(size_t)row * N + t + T * m];
        }
    }
    // idle threads (block padded to whole waves) work in a dummy slot F
    RowLds lds{lds_dyn + (size_t)(q < F ? q : F) * PL};
    fft_run<N, P, INV, 1>(v, t, tw, lds);

    double acc[kPartialNV] = {};
    if (active) {
        const size_t base = (size_t)row * N;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const size_t i = base + t + T * m;
            const cplx y = v[0][m];
            if constexpr (EPI == EPI_STORE) {
                st_wt(out + (INV ? i : spos(t + T * m)), y);
            } else {
                const cplx uu = kPre ? upre[kPre ? m : 0] : u[i];
                const cplx av = kPreA ? apre[kPreA ? m : 0] : mkc(0.f, 0.f);   // aux[i]
                const cplx o = csub(uu, y);
                if constexpr (EPI == EPI_APPLY) {
                    st_wt(out + i, o);
                } else if constexpr (EPI == EPI_BICG_V) {
                    st_wt(out + i, o);
                    const cplx a = av;
                    acc[0] += (double)a.x * o.x + (double)a.y * o.y;
                    acc[1] += (double)a.x * o.y - (double)a.y * o.x;
                } else if constexpr (EPI == EPI_BICG_T) {
                    st_wt(out + i, o);
                    const cplx h = av;
                    acc[0] += (double)o.x * uu.x + (double)o.y * uu.y;
                    acc[1] += (double)o.x * uu.y - (double)o.y * uu.x;
                    acc[2] += (double)o.x * o.x + (double)o.y * o.y;
                    acc[3] += (double)uu.x * uu.x + (double)uu.y * uu.y;
                    acc[4] += (double)h.x * uu.x + (double)h.y * uu.y;   // <r^, s>
                    acc[5] += (double)h.x * uu.y - (double)h.y * uu.x;
                    acc[6] += (double)h.x * o.x + (double)h.y * o.y;     // <r^, t>
                    acc[7] += (double)h.x * o.y - (double)h.y * o.x;
                } else if constexpr (EPI == EPI_TRUERES || EPI == EPI_GMRES_R0) {
                    const cplx b = av;
                    const cplx rr = csub(b, o);
                    st_wt(out + i, rr);
                    acc[0] += (double)rr.x * rr.x + (double)rr.y * rr.y;
                    if constexpr (EPI == EPI_GMRES_R0) acc[1] += (double)b.x * b.x + (double)b.y * b.y;
                } else if constexpr (EPI == EPI_ARNOLDI) {
                    st_wt(out + i, o);
                    v[0][m] = o;   // kept for the projections below
                }
            }
        }
    }
    if constexpr (EPI == EPI_ARNOLDI || EPI == EPI_GMRES_R0) {
        // GMRES: one partial record per block (summed by a later kernel)
        const int nb = rows_per_sys / F;
        const int bi = (row0 % rows_per_sys) / F;
        double* rec = ge.part + ((size_t)sys * nb + bi) * kGmRec;
        if constexpr (EPI == EPI_GMRES_R0) {
            block_sum_to0<kPartialNV>(acc, red);
            if (tid == 0) {
                rec[0] = acc[0];
                rec[1] = acc[1];
            }
        } else {
            const size_t base = (size_t)row * N;
            for (int l0 = 0; l0 < ge.nv; l0 += 2) {
                double a[4] = {0.0, 0.0, 0.0, 0.0};
                if (active) {
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const size_t i = base + t + T * m;
                        const cplx w = v[0][m];
#pragma unroll
                        for (int k = 0; k < 2; ++k) {
                            if (l0 + k < ge.nv) {
                                const cplx b = ge.V[(size_t)(l0 + k) * ge.vstride + i];
                                a[2 * k] += (double)b.x * w.x + (double)b.y * w.y;
                                a[2 * k + 1] += (double)b.x * w.y - (double)b.y * w.x;
                            }
                        }
                    }
                }
                block_sum_to0<4>(a, red);
                if (tid == 0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (2 * l0 + k < 2 * ge.nv) rec[2 * l0 + k] = a[k];
                }
                __syncthreads();
            }
        }
    } else if constexpr (EPI >= EPI_BICG_V) {
        block_sum_to0<kPartialNV>(acc, red);
        if (tid == 0) {
            const int nb = rows_per_sys / F;
            const int bi = (row0 % rows_per_sys) / F;
            double* dst = partials + ((size_t)sys * nb + bi) * kPartialNV;
#pragma unroll
            for (int k = 0; k < kPartialNV; ++k) dst[k] = acc[k];
            // the iteration is complete up to its solution update
            if constexpr (EPI == EPI_BICG_T) {
                if (bi == 0) st[sys].iter += 1;
            }
        }
    }
}

// ------------------------------------------------------ column kernel ----
struct ColLds {
    cplx* base;   // this thread's column (or its private dummy slot)
    int stride;     // W (columns interleaved) or 1 (dummy slot)
    int PL;
    __device__ __forceinline__ cplx& operator()(int f, int pos) const { return padded(f, lds_pad(pos)); }
    __device__ __forceinline__ cplx& padded(int f, int pp) const { return base[(f * PL + pp) * stride]; }
};

// (bx, bz) <- G_hat (bx, bz) with G_hat = gscale (Gamma' - ga I)^-1 for the
// real symmetric scaled Christoffel matrix Gamma' = [[gxx, gxz], [gxz, gzz]].
__device__ __forceinline__ void green_mul(cplx& bx, cplx& bz, real gxx, real gzz, real gxz,
                                          cplx ga, real gscale) {
    const cplx mxx = mkc(gxx - ga.x, -ga.y);
    const cplx mzz = mkc(gzz - ga.x, -ga.y);
    cplx det = cmul(mxx, mzz);
    det.x -= gxz * gxz;
    const real s = gscale * green_rcp(det.x * det.x + det.y * det.y);
    const cplx inv = mkc(det.x * s, -det.y * s);
    const cplx gx = cmul(inv, bx), gz = cmul(inv, bz);   // inv b
    const cplx ox = csub(cmul(mzz, gx), cscale(gz, gxz));
    const cplx oz = csub(cmul(mxx, gz), cscale(gx, gxz));
    bx = ox;
    bz = oz;
}

// Signed FFT index of i on an n-point axis (numpy fftfreq order).
__device__ __forceinline__ int fft_signed(int i, int n) { return (i < (n + 1) / 2) ? i : i - n; }

// u_hat = G_hat(k) b_hat(k) at the P points t + T*m of column ix of a
// transformed spectrum, with the IFFT normalisation folded in (eqs. u0 and A
// in the wavenumber domain).  The central-difference symbol sin(2 pi iz / N)
// / dx comes from the twiddle table (tw[iz] = exp(-2 pi i iz / N)).
template <int N, int P>
__device__ __forceinline__ void green_column(cplx (&v)[2][P], int t, int ix, const ProbDev& pd,
                                             const cplx* tw) {
    constexpr int T = N / P;
    const int nx = pd.nx;
    const int sx = fft_signed(ix, nx);
    const bool central = pd.symbol == 1;
    const real kx = central ? rsinpi(2.0f * (real)sx / (real)nx) / pd.dx : (real)sx * pd.dkx;
    const real kxo = ((nx % 2) == 0 && ix == nx / 2) ? 0.f : kx;
    const real kx2 = kx * kx;
    const real axx = pd.gc11 * kx2, azz = pd.gc55 * kx2, axz = pd.gc1355 * kxo;
    const real rdx = 1.0f / pd.dx;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int iz = t + T * m;
        const int sz = fft_signed(iz, N);
        const real kz = central ? -tw[iz].y * rdx : (real)sz * pd.dkz;
        const real kzo = ((N % 2) == 0 && iz == N / 2) ? 0.f : kz;
        green_mul(v[0][m], v[1][m], axx + pd.gc55 * kz * kz, azz + pd.gc33 * kz * kz, axz * kzo, pd.ga,
                  pd.gscale);
        __builtin_amdgcn_sched_barrier(0);   // one point at a time: bounded registers
    }
}

// Column transforms (with the Green multiply in COL_GREEN mode) of W columns
// per block, P points per thread.  SEQ: the two field components share one
// LDS buffer and go through each pass one after the other; otherwise each
// has its own buffer (twice the LDS, half the barriers).  NT: the block-size
// bound (1024 lets long columns use 16-column, 128-byte row segments).
template <int N, int P, int MODE, bool SEQ, int NT = 512>
__global__ __launch_bounds__(NT) void k_cols(cplx* __restrict__ data, ProbDev pd, int W,
                                              const SysState* __restrict__ st,
                                              const cplx* __restrict__ tw) {
    using S = FftShape<N, P>;
    constexpr int T = S::T;
    constexpr int PL = PaddedLen<N>::value;
    extern __shared__ cplx lds_dyn[];

    const int nx = pd.nx;
    const int tid = threadIdx.x;
    const int c = tid % W, t = tid / W;
    const int ntile = nx / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk / ntile;
    const int x0 = (blk % ntile) * W;
    if (st != nullptr && st[sys].status != ST_RUNNING) return;
    const bool active = t < T;

    // column x0 + c: row-major (stride nx) or column-tiled (stride: the tile width)
    const int cs = pd.tile_sh ? (1 << pd.tile_sh) : nx;
    cplx* base = data + (size_t)sys * 2 * N * nx + spec_off(0, x0 + c, nx, pd.tile_sh ? N : 0, pd.tile_sh);
    const size_t plane = (size_t)N * nx;
    cplx v[2][P];
    if (active) {
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) v[f][m] = base[f * plane + (size_t)(t + T * m) * cs];
    } else {
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) v[f][m] = mkc(0.f, 0.f);
    }
    ColLds lds{active ? lds_dyn + c : lds_dyn + (size_t)PL * W * (SEQ ? 1 : 2), active ? W : 1, PL};
    const int tt = active ? t : 0;

    if constexpr (MODE != COL_INV) {
        if constexpr (SEQ) fft_run_seq<N, P, false, 2>(v, tt, tw, lds);
        else fft_run<N, P, false, 2>(v, tt, tw, lds);
    }
    if constexpr (MODE == COL_GREEN) {
        green_column<N, P>(v, tt, x0 + c, pd, tw);
        __syncthreads();
    }
    if constexpr (MODE != COL_FWD) {
        // The inverse reads the same twiddle entries as the forward pass; an
        // opaque copy of the table pointer keeps the compiler from holding the
        // forward pass's twiddles in registers across the Green multiply.
        // Likewise for the LDS addresses, which are the same in both passes:
        // the opaque value is the offset into the LDS array, not the pointer,
        // so that the compiler still knows the accesses are LDS accesses (an
        // opaque pointer would turn them into flat memory instructions).
        // (The same for the twiddle table: an opaque zero offset keeps its
        // loads global loads.)
        int toff = 0;
        int ti = tt;
        int boff = (int)(lds.base - lds_dyn), bstride = lds.stride;
        asm volatile("" : "+s"(toff));
        asm volatile("" : "+v"(ti), "+v"(boff), "+v"(bstride));
        const cplx* twi = tw + toff;
        const ColLds ldi{lds_dyn + boff, bstride, PL};
        if constexpr (SEQ) fft_run_seq<N, P, true, 2>(v, ti, twi, ldi);
        else fft_run<N, P, true, 2>(v, ti, twi, ldi);
    }

    if (active) {
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) st_wt(base + f * plane + (size_t)(t + T * m) * cs, v[f][m]);
    }
}


// The Green-multiply column pass with the two field components on separate
// threads (twice the threads of k_cols, half the registers each): thread
// (comp, t, c) transforms component comp of column c; after the forward
// transform the components meet in LDS for the 2 x 2 Green multiply, and
// each thread keeps the output of its own component.
template <int N, int P>
__global__ __launch_bounds__(512) void k_cols_split(cplx* __restrict__ data, ProbDev pd, int W,
                                                     const SysState* __restrict__ st,
                                                     const cplx* __restrict__ tw) {
    using S = FftShape<N, P>;
    constexpr int T = S::T;
    constexpr int PL = PaddedLen<N>::value;
    extern __shared__ cplx lds_dyn[];

    const int nx = pd.nx;
    const int tid = threadIdx.x;
    const int wt = W * T;
    const int comp = tid / wt;                 // blockDim.x == 2 W T
    const int c = tid % W, t = (tid - comp * wt) / W;
    const int ntile = nx / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk / ntile;
    const int x0 = (blk % ntile) * W;
    if (st != nullptr && st[sys].status != ST_RUNNING) return;

    const size_t plane = (size_t)N * nx;
    const int cs = pd.tile_sh ? (1 << pd.tile_sh) : nx;   // column stride: row-major or column-tiled
    cplx* base = data + (size_t)sys * 2 * plane + comp * plane + spec_off(0, x0 + c, nx, pd.tile_sh ? N : 0, pd.tile_sh);
    cplx v[1][P];
#pragma unroll
    for (int m = 0; m < P; ++m) v[0][m] = base[(size_t)(t + T * m) * cs];
    const ColLds own{lds_dyn + (size_t)comp * PL * W + c, W, PL};
    const ColLds other{lds_dyn + (size_t)(1 - comp) * PL * W + c, W, PL};
    fft_run<N, P, false, 1>(v, t, tw, own);

    // exchange the transformed components through LDS
    __syncthreads();   // the last transform exchange is read
#pragma unroll
    for (int m = 0; m < P; ++m) own(0, t + T * m) = v[0][m];
    __syncthreads();
    const int ix = x0 + c;
    const int sx = fft_signed(ix, nx);
    const bool central = pd.symbol == 1;
    const real kx = central ? rsinpi(2.0f * (real)sx / (real)nx) / pd.dx : (real)sx * pd.dkx;
    const real kxo = ((nx % 2) == 0 && ix == nx / 2) ? 0.f : kx;
    const real kx2 = kx * kx;
    const real axx = pd.gc11 * kx2, azz = pd.gc55 * kx2, axz = pd.gc1355 * kxo;
    const real rdx = 1.0f / pd.dx;
    // the partner's values first, into registers (a select between a register
    // array element and an LDS address would force the array into memory)
    cplx o[P];
#pragma unroll
    for (int m = 0; m < P; ++m) o[m] = other(0, t + T * m);
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int iz = t + T * m;
        const int sz = fft_signed(iz, N);
        const real kz = central ? -tw[iz].y * rdx : (real)sz * pd.dkz;
        const real kzo = ((N % 2) == 0 && iz == N / 2) ? 0.f : kz;
        const cplx mine = v[0][m], theirs = o[m];
        cplx bx = comp == 0 ? mine : theirs;
        cplx bz = comp == 0 ? theirs : mine;
        green_mul(bx, bz, axx + pd.gc55 * kz * kz, azz + pd.gc33 * kz * kz, axz * kzo, pd.ga, pd.gscale);
        v[0][m] = comp == 0 ? bx : bz;
        __builtin_amdgcn_sched_barrier(0);   // one point at a time: bounded registers
    }
    __syncthreads();   // every partner value is read before the inverse writes LDS
    fft_run<N, P, true, 1>(v, t, tw, own);
#pragma unroll
    for (int m = 0; m < P; ++m) st_wt(base + (size_t)(t + T * m) * cs, v[0][m]);
}

// The Green-multiply column pass with the twiddle table in LDS and the tile
// width W fixed at compile time (LDS addresses then fold into the
// instructions' immediate offsets).  The table is copied once per block,
// after the block's column loads are issued; the transforms' twiddle reads
// are then LDS reads.  Blocks are exactly W x T threads (no idle threads).
template <int N, int P, int W>
__global__ __launch_bounds__(512) void k_cols_tw(cplx* __restrict__ data, ProbDev pd,
                                                  const SysState* __restrict__ st,
                                                  const cplx* __restrict__ tw) {
    using S = FftShape<N, P>;
    constexpr int T = S::T;
    constexpr int NT = W * T;
    constexpr int PL = PaddedLen<N>::value;
    constexpr int NTW = (N + NT - 1) / NT;   // table entries per thread
    extern __shared__ cplx lds_dyn[];

    const int nx = pd.nx;
    const int tid = threadIdx.x;
    const int c = tid % W, t = tid / W;
    const int ntile = nx / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk / ntile;
    if (st != nullptr && st[sys].status != ST_RUNNING) return;
    const int ix = (blk - sys * ntile) * W + c;

    const size_t plane = (size_t)N * nx;
    const int cs = pd.tile_sh ? (1 << pd.tile_sh) : nx;   // column stride: row-major or column-tiled
    cplx* base = data + (size_t)sys * 2 * plane + spec_off(0, ix, nx, pd.tile_sh ? N : 0, pd.tile_sh);
    cplx v[2][P];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int m = 0; m < P; ++m) v[f][m] = base[f * plane + (size_t)(t + T * m) * cs];
    cplx twv[NTW];
#pragma unroll
    for (int i = 0; i < NTW; ++i)
        if (tid + i * NT < N) twv[i] = tw[tid + i * NT];
#pragma unroll
    for (int i = 0; i < NTW; ++i)
        if (tid + i * NT < N) lds_dyn[tid + i * NT] = twv[i];
    const ColLds lds{lds_dyn + N + c, W, PL};
    __syncthreads();   // the twiddle table is in LDS

    fft_run<N, P, false, 2, true>(v, t, lds_dyn, lds);
    green_column<N, P>(v, t, ix, pd, lds_dyn);
    // as in k_cols: opaque copies keep the forward pass's twiddles and LDS
    // addresses from being held in registers across the Green multiply
    int toff = 0;
    int ti = t;
    int boff = c + N;
    asm volatile("" : "+v"(ti), "+v"(boff), "+v"(toff));
    const ColLds ldi{lds_dyn + boff, W, PL};
    fft_run<N, P, true, 2, true>(v, ti, lds_dyn + toff, ldi);
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int m = 0; m < P; ++m) st_wt(base + f * plane + (size_t)(t + T * m) * cs, v[f][m]);
}

// ----------------------------------------------------- launch helpers ----
// Dynamic LDS above the default limit must be enabled once per kernel.
template <class K>
inline hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N, int P, bool INV, int EPI>
inline hipError_t rows_launch(const cplx* in, cplx* out, const cplx* u, const cplx* aux,
                              double* part, int nrows, int rps, SpecLayout lay, const SysState* st,
                              const cplx* tw, hipStream_t s, const GmEpi* ge = nullptr) {
    if (lay.nz && (lay.sh < 1 || N % (1 << lay.sh) != 0 || in == out || rps != 2 * lay.nz))
        return hipErrorInvalidValue;
    const GmEpi gz{nullptr, 0, 0, nullptr};
    const RowGeom g = row_geom(N, P, rps);
    const int blocks = (nrows + g.F - 1) / g.F;
    const size_t lds = (size_t)(g.F + 1) * PaddedLen<N>::value * sizeof(cplx);
    hipError_t e = allow_lds(k_rows<N, P, INV, EPI>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_rows<N, P, INV, EPI>), dim3(blocks), dim3(g.threads), lds, s, in, out, u, aux,
                       part, nrows, rps, g.F, lay.nz, lay.sh, const_cast<SysState*>(st), tw, ge ? *ge : gz);
    return hipGetLastError();
}

template <int N, int P>
inline hipError_t cols_split_launch(cplx* data, const ProbDev& pd, int W, const SysState* st,
                                    const cplx* tw, hipStream_t s) {
    const ColGeom g = col_geom(N, pd.nx, ColCfg{P, W, 2});
    const int blocks = pd.nsys * (pd.nx / W);
    hipError_t e = allow_lds(k_cols_split<N, P>, g.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cols_split<N, P>), dim3(blocks), dim3(g.threads), g.lds, s, data, pd, W, st, tw);
    return hipGetLastError();
}

template <int N, int P, int MODE, bool SEQ, int NT = 512>
inline hipError_t cols_launch(cplx* data, const ProbDev& pd, int W, const SysState* st,
                              const cplx* tw, hipStream_t s) {
    const ColGeom g = col_geom(N, pd.nx, ColCfg{P, W, NT > 512 ? 3 : SEQ ? 1 : 0});
    if (g.threads > NT) return hipErrorInvalidValue;
    const int blocks = pd.nsys * (pd.nx / W);
    hipError_t e = allow_lds(k_cols<N, P, MODE, SEQ, NT>, g.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cols<N, P, MODE, SEQ, NT>), dim3(blocks), dim3(g.threads), g.lds, s, data, pd, W,
                       st, tw);
    return hipGetLastError();
}

// The LDS-twiddle pass: W from {4, 8, 16} as a template parameter.
template <int N, int P>
inline hipError_t cols_tw_launch(cplx* data, const ProbDev& pd, int W, const SysState* st, const cplx* tw,
                                 hipStream_t s) {
    const ColGeom g = col_geom(N, pd.nx, ColCfg{P, W, 4});
    if (g.threads != W * (N / P) || g.threads > 512) return hipErrorInvalidValue;
    const int blocks = pd.nsys * (pd.nx / W);
    auto go = [&](auto kernel) -> hipError_t {
        hipError_t e = allow_lds(kernel, g.lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(g.threads), g.lds, s, data, pd, st, tw);
        return hipGetLastError();
    };
    if (W == 4) return go(k_cols_tw<N, P, 4>);
    if (W == 8) return go(k_cols_tw<N, P, 8>);
    if (W == 16) return go(k_cols_tw<N, P, 16>);
    return hipErrorInvalidValue;
}

FW_END
