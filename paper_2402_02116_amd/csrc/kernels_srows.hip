// Contrast stencil fused with the forward row transform (eqs. u_2, A, FFT):
// a block owns F whole rows (both field components) of one system, loads
// them with a 2-row halo into LDS (applying the BiCGSTAB update of the input
// on the way, and for the own rows the previous iteration's r and x updates,
// as k_body_force does), forms
//     b = w~^2 drho u + (1 / 4 dx^2) div'(dC : e'),   e' = raw central differences,
// directly in the register layout of the row transform (each thread the
// positions t + T m of one row), transforms the 2F rows, and writes the
// row-transformed b.  One kernel and one HBM round trip of b fewer per matvec
// than the separate stencil and row passes.
#include "bicg.h"
#include "fft.h"

FW_BEGIN
namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Tile row (0..F+3, own rows 2..F+1) loaded at step lr of the load loop:
// the own rows top to bottom, then the two halo rows above and the two below.
__device__ __forceinline__ int srows_load_row(int lr, int F) {
    if (lr < F) return lr + 2;
    return lr - F < 2 ? lr - F : lr;
}

struct RowLdsF {
    cplx* p;
    __device__ __forceinline__ cplx& operator()(int, int pos) const { return p[lds_pad(pos)]; }
    __device__ __forceinline__ cplx& padded(int, int pp) const { return p[pp]; }
};

template <int N, int P, int VM, int NT>
__global__ __launch_bounds__(NT) void k_srows(const cplx* __restrict__ u, const cplx* __restrict__ a1,
                                               const cplx* __restrict__ a2, cplx* __restrict__ wout,
                                               cplx* __restrict__ rhat, cplx* __restrict__ out,
                                               const real* __restrict__ maps, ProbDev pd, int F,
                                               SysState* __restrict__ st, const double* __restrict__ part,
                                               int np, const cplx* __restrict__ tw,
                                               const cplx* __restrict__ a3, cplx* __restrict__ xio,
                                               cplx* __restrict__ rout) {
    using S = FftShape<N, P>;
    constexpr int T = S::T;
    constexpr int PL = PaddedLen<N>::value;
    extern __shared__ cplx lds_dyn[];
    __shared__ double red[NT / 64 * kPartialNV];

    const int nz = pd.nz;
    const size_t plane = (size_t)N * nz;
    const int bps = nz / F;                         // blocks per system
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk / bps;
    const int z0 = (blk - sys * bps) * F;
    if (st != nullptr) {   // uniform over the block
        const int stw = st[sys].status;
        if constexpr (VM == VM_PX) {
            if (!closing_enters(stw, kStampPx)) return;
        } else {
            if (stw != ST_RUNNING) {
                // the iteration's closing kernel is done: drop its tag
                if (VM == VM_S && st_tag(stw) != 0 && z0 == 0 && threadIdx.x == 0) st[sys].status = st_code(stw);
                return;
            }
        }
    }

    cplx c1 = mkc(0.f, 0.f), c2 = mkc(0.f, 0.f), c3 = mkc(0.f, 0.f);
    bool fresh = false;
    int step = SS_FULL;
    if constexpr (VM != VM_NONE) {
        step = stencil_scalars<VM, NT>(st, sys, part, np, red, z0 == 0 && threadIdx.x == 0, c1, c2, c3, fresh);
        if (step == SS_SKIP) return;
    }
    const size_t so = (size_t)sys * 2 * plane;
    // VM_PX on an own cell: r = s - omega t, x += alpha p_old + omega s
    auto close_iteration = [&](size_t gi) {
        const cplx sv = u[so + gi], tv = a3[so + gi], pv = a1[so + gi];
        const cplx rv = close_r(sv, tv, c2);
        st_wt(rout + so + gi, rv);
        st_wt(xio + so + gi, close_x(xio[so + gi], pv, sv, c3, c2));
        if (fresh) st_wt(rhat + so + gi, rv);
    };
    if constexpr (VM == VM_PX) {
        if (step == SS_XONLY) {   // stopped: the last solution update only
            const int own = 2 * F * N;
            for (int idx = threadIdx.x; idx < own; idx += blockDim.x) {
                const int c = idx / (F * N);
                const int rem = idx - c * F * N;
                close_iteration(c * plane + (size_t)z0 * N + rem);
            }
            return;
        }
    }
    // 1. the 2F + 8 rows (F + 4 per component) of the input into LDS, kB
    //    elements per thread at a time: every load of a batch is issued before
    //    its stores (out-of-range slots load element 0 and are dropped).
    //    Load order (both components of a row together): the own rows first,
    //    the four halo rows last, so that a halo row, which is an own row of
    //    the neighbouring block on the same XCD, is read after that block has
    //    brought it into the L2.
    const int HR = F + 4;
    cplx* su = lds_dyn;                           // [2][HR][N]
    const int total = 2 * HR * N;
    constexpr int kB = VM == VM_PX ? 4 : 8;
    for (int i0 = threadIdx.x; i0 < total; i0 += kB * NT) {
        size_t gi[kB];
        int li[kB];
        bool ok[kB], own[kB];
        cplx f[kB], sv[kB], pv[kB], rv[kB], xv[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int idx = i0 + j * NT;
            ok[j] = idx < total;
            const int id = ok[j] ? idx : 0;
            const int lr = id / (2 * N);
            const int c = (id / N) & 1;
            const int x = id - (id / N) * N;
            const int tr = srows_load_row(lr, F);
            gi[j] = so + c * plane + (size_t)wrapi(z0 - 2 + tr, nz) * N + x;
            li[j] = (c * HR + tr) * N + x;
            own[j] = ok[j] && tr >= 2 && tr < F + 2;
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const size_t g = gi[j];
            if constexpr (VM == VM_NONE) {
                f[j] = u[g];
            } else if constexpr (VM == VM_P) {
                const cplx r0 = u[g], p0 = a1[g], v0 = a2[g];
                f[j] = fresh ? r0 : cadd(r0, cmul(c1, csub(p0, cmul(c2, v0))));
            } else if constexpr (VM == VM_PX) {
                sv[j] = u[g];
                const cplx t0 = a3[g];
                pv[j] = a1[g];
                const cplx v0 = a2[g];
                xv[j] = own[j] ? xio[g] : mkc(0.f, 0.f);
                rv[j] = close_r(sv[j], t0, c2);
                f[j] = fresh ? rv[j] : cadd(rv[j], cmul(c1, csub(pv[j], cmul(c2, v0))));
            } else {
                f[j] = csub(u[g], cmul(c1, a1[g]));
            }
        }
#pragma unroll
        for (int j = 0; j < kB; ++j)
            if (ok[j]) su[li[j]] = f[j];
        if constexpr (VM != VM_NONE) {
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                if (!own[j]) continue;              // the block's own rows
                st_wt(wout + gi[j], f[j]);
                if constexpr (VM == VM_P) {
                    if (fresh) st_wt(rhat + gi[j], f[j]);
                } else if constexpr (VM == VM_PX) {
                    st_wt(rout + gi[j], rv[j]);
                    st_wt(xio + gi[j], close_x(xv[j], pv[j], sv[j], c3, c2));
                    if (fresh) st_wt(rhat + gi[j], rv[j]);
                }
            }
        }
    }
    __syncthreads();

    // 2. b on the own rows, in the transform's layout: row q = (component
    //    c = q / F, row z0 + q % F), thread t holds x = t + T m
    const int q = threadIdx.x / T, t = threadIdx.x - (threadIdx.x / T) * T;
    const bool active = q < 2 * F;
    const int c = active ? q / F : 0;
    const int zl = active ? q - c * F : 0;
    const int z = z0 + zl;
    const real sc = pd.inv4dx2;
    const real* mc11 = maps;
    const real* mc13 = maps + plane;
    const real* mc33 = maps + 2 * plane;
    const real* mc55 = maps + 3 * plane;
    const real* mrho = maps + 4 * plane;
    auto U = [&](int cc, int dz, int x) -> cplx { return su[(cc * HR + zl + 2 + dz) * N + wrapi(x, N)]; };
    const size_t zr = (size_t)z * N, zu = (size_t)wrapi(z - 1, nz) * N, zd = (size_t)wrapi(z + 1, nz) * N;
    // the map values of kG points are loaded before any of them is used
    constexpr int kG = P % 8 == 0 ? 8 : (P % 6 == 0 ? 6 : 4);
    static_assert(P % kG == 0, "points per thread");
    cplx v[1][P];
    if (active && c == 0) {
#pragma unroll
      for (int m0 = 0; m0 < P; m0 += kG) {
        real rh[kG], a11r[kG], a13r[kG], a11l[kG], a13l[kG], a55d[kG], a55u[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int m = g;
            const int x = t + T * (m0 + g), xl = wrapi(x - 1, N), xr = wrapi(x + 1, N);
            rh[m] = mrho[zr + x];
            a11r[m] = mc11[zr + xr];
            a13r[m] = mc13[zr + xr];
            a11l[m] = mc11[zr + xl];
            a13l[m] = mc13[zr + xl];
            a55d[m] = mc55[zd + x];
            a55u[m] = mc55[zu + x];
        }
#pragma unroll
        for (int m = 0; m < kG; ++m) {
            // sigma_1 at (z, x +- 1), sigma_5 at (z +- 1, x)
            const int x = t + T * (m0 + m);
            const cplx exr = csub(U(0, 0, x + 2), U(0, 0, x)), ezr = csub(U(1, 1, x + 1), U(1, -1, x + 1));
            const cplx exl = csub(U(0, 0, x), U(0, 0, x - 2)), ezl = csub(U(1, 1, x - 1), U(1, -1, x - 1));
            const cplx s1r = mkc(a11r[m] * exr.x + a13r[m] * ezr.x, a11r[m] * exr.y + a13r[m] * ezr.y);
            const cplx s1l = mkc(a11l[m] * exl.x + a13l[m] * ezl.x, a11l[m] * exl.y + a13l[m] * ezl.y);
            const cplx exzd = cadd(csub(U(0, 2, x), U(0, 0, x)), csub(U(1, 1, x + 1), U(1, 1, x - 1)));
            const cplx exzu = cadd(csub(U(0, 0, x), U(0, -2, x)), csub(U(1, -1, x + 1), U(1, -1, x - 1)));
            const cplx dx1 = csub(s1r, s1l);
            const cplx dz5 = csub(cscale(exzd, a55d[m]), cscale(exzu, a55u[m]));
            v[0][m0 + m] = cadd(cmul(cscale(pd.w2, rh[m]), U(0, 0, x)), cscale(cadd(dx1, dz5), sc));
        }
      }
    } else if (active) {
#pragma unroll
      for (int m0 = 0; m0 < P; m0 += kG) {
        real rh[kG], a13d[kG], a33d[kG], a13u[kG], a33u[kG], a55r[kG], a55l[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int m = g;
            const int x = t + T * (m0 + g), xl = wrapi(x - 1, N), xr = wrapi(x + 1, N);
            rh[m] = mrho[zr + x];
            a13d[m] = mc13[zd + x];
            a33d[m] = mc33[zd + x];
            a13u[m] = mc13[zu + x];
            a33u[m] = mc33[zu + x];
            a55r[m] = mc55[zr + xr];
            a55l[m] = mc55[zr + xl];
        }
#pragma unroll
        for (int m = 0; m < kG; ++m) {
            // sigma_5 at (z, x +- 1), sigma_3 at (z +- 1, x)
            const int x = t + T * (m0 + m);
            const cplx exzr = cadd(csub(U(0, 1, x + 1), U(0, -1, x + 1)), csub(U(1, 0, x + 2), U(1, 0, x)));
            const cplx exzl = cadd(csub(U(0, 1, x - 1), U(0, -1, x - 1)), csub(U(1, 0, x), U(1, 0, x - 2)));
            const cplx exd = csub(U(0, 1, x + 1), U(0, 1, x - 1)), ezd = csub(U(1, 2, x), U(1, 0, x));
            const cplx exu = csub(U(0, -1, x + 1), U(0, -1, x - 1)), ezu = csub(U(1, 0, x), U(1, -2, x));
            const cplx s3d = mkc(a13d[m] * exd.x + a33d[m] * ezd.x, a13d[m] * exd.y + a33d[m] * ezd.y);
            const cplx s3u = mkc(a13u[m] * exu.x + a33u[m] * ezu.x, a13u[m] * exu.y + a33u[m] * ezu.y);
            const cplx dx5 = csub(cscale(exzr, a55r[m]), cscale(exzl, a55l[m]));
            const cplx dz3 = csub(s3d, s3u);
            v[0][m0 + m] = cadd(cmul(cscale(pd.w2, rh[m]), U(1, 0, x)), cscale(cadd(dx5, dz3), sc));
        }
      }
    } else {
#pragma unroll
        for (int m = 0; m < P; ++m) v[0][m] = mkc(0.f, 0.f);
    }
    __syncthreads();   // the tile is read; its LDS now holds the transform's rows

    // 3. forward row transforms (idle threads work in a dummy slot)
    RowLdsF lds{lds_dyn + (size_t)(active ? q : 2 * F) * PL};
    fft_run<N, P, false, 1>(v, t, tw, lds);
    if (active) {   // the spectrum: row-major or column-tiled
        cplx* o = out + so + c * plane;
        const int tnz = pd.tile_sh ? nz : 0;
#pragma unroll
        for (int m = 0; m < P; ++m) st_wt(o + spec_off(z, t + T * m, N, tnz, pd.tile_sh), v[0][m]);
    }
}

}  // namespace

// Threads of the fused kernel: 512 (twice the rows per block, so a smaller
// share of halo rows) where a thread's row segment is short enough, for the
// heaviest input update, VM_PX, which reads four vectors in the halo, and for
// the plain mode on rows of 384 points or more (four own rows per block
// otherwise: 232 -> 228 us for the plain pass over the four grids 128^2 ..
// 384^2); 256 otherwise (measured: no gain for the lighter update modes).
constexpr bool srows_wide(int nx, int P, int vm) {
    return (vm == VM_PX && nx >= 256 && nx / P <= 32) || (vm == VM_NONE && nx >= 384 && nx / P <= 32);
}

// Rows per block (a power of two <= threads / 2T dividing nz) for n-point
// rows with P points per thread in stencil mode vm; 0 when the fused kernel
// does not apply.
int srows_rows(int nx, int nz, int P, int vm) {
#ifdef FW_C128
    (void)nx, (void)nz, (void)P, (void)vm;
    return 0;   // the complex128 build keeps the stencil and the row pass apart
#endif
    if (nx > kSrowsMaxN || nx % P != 0 || P > 24) return 0;   // no fused radix-32 variant
    const int T = nx / P;
    if (T > 128) return 0;
    int F = (srows_wide(nx, P, vm) ? 256 : 128) / T;
    while (F > 1 && nz % F != 0) F /= 2;
    return F;
}

size_t srows_lds(int nx, int F) {
    const size_t tile = (size_t)2 * (F + 4) * nx * sizeof(cplx);
    const size_t fft = (size_t)(2 * F + 1) * (nx + nx / 16 + 1) * sizeof(cplx);
    return tile > fft ? tile : fft;
}

template <int N, int P, int VM, int NT>
static hipError_t srows_launch_nt(const StencilArgs& a, cplx* out, const ProbDev& pd, SysState* st,
                                  const cplx* tw, hipStream_t s) {
    const int F = srows_rows(N, pd.nz, P, VM);
    if (F == 0) return hipErrorInvalidValue;
    const size_t lds = srows_lds(N, F);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_srows<N, P, VM, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = pd.nsys * (pd.nz / F);
    hipLaunchKernelGGL((k_srows<N, P, VM, NT>), dim3(blocks), dim3(NT), lds, s, a.u, a.a1, a.a2, a.wout, a.rhat,
                       out, a.maps, pd, F, st, a.part, a.np, tw, a.a3, a.xio, a.rout);
    return hipGetLastError();
}

template <int N, int P, int VM>
static hipError_t srows_launch(const StencilArgs& a, cplx* out, const ProbDev& pd, SysState* st,
                               const cplx* tw, hipStream_t s) {
    if constexpr (srows_wide(N, P, VM)) return srows_launch_nt<N, P, VM, 512>(a, out, pd, st, tw, s);
    else return srows_launch_nt<N, P, VM, 256>(a, out, pd, st, tw, s);
}

template <int N, int P>
static hipError_t srows_vm(int vm, const StencilArgs& a, cplx* out, const ProbDev& pd, SysState* st,
                           const cplx* tw, hipStream_t s) {
    if (vm == VM_NONE) return srows_launch<N, P, VM_NONE>(a, out, pd, st, tw, s);
    if (vm == VM_P) return srows_launch<N, P, VM_P>(a, out, pd, st, tw, s);
    if (vm == VM_PX) return srows_launch<N, P, VM_PX>(a, out, pd, st, tw, s);
    return srows_launch<N, P, VM_S>(a, out, pd, st, tw, s);
}

#ifdef FW_C128
#define FW_SROWS_VARIANTS(X)
#else
#define FW_SROWS_VARIANTS(X)                                                                         \
    X(16, 16) X(16, 8) X(24, 12) X(24, 24) X(32, 16) X(32, 8) X(48, 12) X(48, 24) X(64, 16) X(64, 8) \
    X(96, 12) X(96, 24) X(128, 16) X(128, 8) X(192, 12) X(192, 24) X(256, 16) X(256, 8) X(384, 12)  \
    X(384, 24) X(512, 16) X(512, 8)
#endif

hipError_t launch_srows(int vm, int P, const StencilArgs& a, cplx* out, const ProbDev& pd, SysState* st,
                        const cplx* tw, hipStream_t s) {
    if (vm < 0 || vm > 3 || (vm != VM_NONE && !st) || ((vm == VM_P || vm == VM_PX) && !a.rhat) ||
        (vm == VM_PX && (!a.a3 || !a.xio || !a.rout)))
        return hipErrorInvalidValue;
    if (!row_points_ok(pd.nx, P) || srows_rows(pd.nx, pd.nz, P, vm) == 0) return hipErrorInvalidValue;
    const cplx* t = tw + twiddle_offset(pd.nx);
#define FW_CASE(N, PP) \
    if (pd.nx == N && P == PP) return srows_vm<N, PP>(vm, a, out, pd, st, t, s);
    FW_SROWS_VARIANTS(FW_CASE)
#undef FW_CASE
    return hipErrorInvalidValue;
}

FW_END