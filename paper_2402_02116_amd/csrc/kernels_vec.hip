// Pointwise and stencil kernels of the LS solve, J and J*:
//   k_body_force   - contrast stencil b = w~^2 drho u + div_h(dC : E_h u)
//                    (eqs. Ewave0, u_2; abbreviated subscript section), also
//                    the virtual source P_b(dm) of eqs. YM / dC;
//   k_bicg_*       - batched BiCGSTAB vector updates with FP64 scalars;
//   k_point_sources, k_gather, k_scatter_conj - sources and receivers;
//   k_correlate    - adjoint correlation of eq. ad1 summed over systems (FP64
//                    sums; complex or FP64 complex output maps).
#include <algorithm>

#include "bicg.h"

FW_BEGIN
constexpr int kVecThreads = 256;
constexpr int kVecEPT = 4;   // complex elements per thread in vector kernels
constexpr int kStallIters = 150;   // iterations without halving ||r|| before a restart

// ------------------------------------------------------ contrast stencil --
// A block owns a TZ x TX tile of cells and loops over S systems of the same
// problem.  Threads are laid out 64 (x) by 4 (z); lanes x >= TX idle.  The
// contrast of the tile (and of its 1-cell halo) is loaded into registers
// together with the first displacement tile, and reused for every system.
// Per system:
//   1. the displacement tile with a 2-cell halo goes to LDS;
//   2. the stress s' = dC e (e = raw central differences, 2 dx times the
//      Voigt strain) is formed on the tile plus a 1-cell halo, in LDS;
//   3. b = w~^2 drho u + (1 / 4 dx^2) div'(s') on the tile.
constexpr int STX = 64, STZ = 8;

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// The vector update of the input (StencilVec, bicg.h) is written for the
// tile's own cells and used (halo included) as the stencil's input.  p is
// double-buffered by the caller because neighbouring tiles read p_old in
// their halos.

template <int TX, int TZ, int VM>
__global__ __launch_bounds__(256) void k_body_force(const cplx* __restrict__ u,
                                                    const cplx* __restrict__ a1,
                                                    const cplx* __restrict__ a2,
                                                    cplx* __restrict__ wout,
                                                    cplx* __restrict__ b,
                                                    const real* __restrict__ maps, ProbDev pd,
                                                    int S, SysState* __restrict__ st,
                                                    const double* __restrict__ part, int np,
                                                    cplx* __restrict__ rhat,
                                                    const cplx* __restrict__ a3,
                                                    cplx* __restrict__ xio,
                                                    cplx* __restrict__ rout) {
    static_assert(TX <= 64 && TZ % 4 == 0, "tile");
    constexpr int HX = TX + 4, HZ = TZ + 4, SX = TX + 2, SZ = TZ + 2;
    constexpr int KS = (SZ + 3) / 4;     // stress rows per thread
    constexpr int KB = TZ / 4;           // output rows per thread
    constexpr int KH = HZ / 4;           // displacement rows per thread
    __shared__ cplx su[2][HZ][HX];
    __shared__ cplx ss[3][SZ][SX];
    __shared__ double red[4 * kPartialNV];
    const int nx = pd.nx, nz = pd.nz;
    const size_t plane = (size_t)nx * nz;
    const int ntx = nx / TX;
    const int ntiles = ntx * (nz / TZ);
    // neighbouring blocks (on one XCD, resident together): the neighbouring
    // tiles of the same systems, which read each other's rows and columns as
    // their halos while those cache lines are still in the XCD's L2
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sg = blk / ntiles;
    const int tile = blk - sg * ntiles;
    const int sys0 = sg * S;
    const int z0 = (tile / ntx) * TZ, x0 = (tile % ntx) * TX;
    const int tx = threadIdx.x & 63, tg = threadIdx.x >> 6;
    const bool lane = tx < TX;
    const int hsx = (tx == 0) ? 0 : TX + 1;   // halo stress column of lanes 0 and 1
    const int hux = (tx < 2) ? tx : TX + tx;  // halo displacement column of lanes 0..3

    real m_in[KS][4], m_h[KS][4], rho[KB];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int sz = tg + 4 * k;
        const bool row = sz < SZ;
        const size_t gz = (size_t)wrap(z0 - 1 + sz, nz) * nx;
        const size_t gi = gz + (size_t)(x0 + (lane ? tx : 0));
        const size_t gh = gz + (size_t)wrap(x0 - 1 + hsx, nx);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            m_in[k][c] = (row && lane) ? maps[c * plane + gi] : 0.f;
            m_h[k][c] = (row && tx < 2) ? maps[c * plane + gh] : 0.f;
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
        rho[k] = lane ? maps[4 * plane + (size_t)(z0 + tg + 4 * k) * nx + x0 + tx] : 0.f;

    const real sc = pd.inv4dx2;
    for (int sys = sys0; sys < sys0 + S && sys < pd.nsys; ++sys) {
        if (st != nullptr) {   // uniform over the block
            const int stw = st[sys].status;
            if constexpr (VM == VM_PX) {
                if (!closing_enters(stw, kStampPx)) continue;
            } else {
                if (stw != ST_RUNNING) {
                    // the iteration's closing kernel is done: drop its tag
                    if (VM == VM_S && st_tag(stw) != 0 && tile == 0 && threadIdx.x == 0)
                        st[sys].status = st_code(stw);
                    continue;
                }
            }
        }
        cplx c1 = mkc(0.f, 0.f), c2 = mkc(0.f, 0.f), c3 = mkc(0.f, 0.f);
        bool fresh = false;
        int step = SS_FULL;
        if constexpr (VM != VM_NONE) {
            step = stencil_scalars<VM>(st, sys, part, np, red, tile == 0 && threadIdx.x == 0, c1, c2, c3, fresh);
            if (step == SS_SKIP) continue;
        }
        const size_t so = (size_t)sys * 2 * plane;
        cplx* bs = b + so;
        // VM_PX on an own cell: r = s - omega t, x += alpha p_old + omega s
        auto close_iteration = [&](size_t gi) {
            const cplx sv = u[so + gi], tv = a3[so + gi], pv = a1[so + gi];
            const cplx rv = close_r(sv, tv, c2);
            st_wt(rout + so + gi, rv);
            st_wt(xio + so + gi, close_x(xio[so + gi], pv, sv, c3, c2));
            if (fresh) rhat[so + gi] = rv;
        };
        if constexpr (VM == VM_PX) {
            if (step == SS_XONLY) {   // stopped: the last solution update only
                if (lane) {
#pragma unroll
                    for (int k = 0; k < KB; ++k) {
                        const size_t gi = (size_t)(z0 + tg + 4 * k) * nx + x0 + tx;
                        close_iteration(gi);
                        close_iteration(plane + gi);
                    }
                }
                continue;
            }
        }
        // input field value at global index gi of this system (comp offset included)
        auto field = [&](size_t gi) -> cplx {
            if constexpr (VM == VM_NONE) {
                return u[so + gi];
            } else if constexpr (VM == VM_P) {
                const cplx rv = u[so + gi];
                if (fresh) return rv;
                const cplx pv = a1[so + gi], vv = a2[so + gi];
                return cadd(rv, cmul(c1, csub(pv, cmul(c2, vv))));
            } else if constexpr (VM == VM_PX) {
                const cplx rv = close_r(u[so + gi], a3[so + gi], c2);
                if (fresh) return rv;
                const cplx pv = a1[so + gi], vv = a2[so + gi];
                return cadd(rv, cmul(c1, csub(pv, cmul(c2, vv))));
            } else {
                return csub(u[so + gi], cmul(c1, a1[so + gi]));
            }
        };
        __syncthreads();   // previous system's reads of su / ss are done
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            const int hz = tg + 4 * k;
            const size_t row = (size_t)wrap(z0 - 2 + hz, nz) * nx;
            if (lane) {
                const cplx f0 = field(row + x0 + tx), f1 = field(plane + row + x0 + tx);
                su[0][hz][tx + 2] = f0;
                su[1][hz][tx + 2] = f1;
                if constexpr (VM != VM_NONE) {
                    if (hz >= 2 && hz < TZ + 2) {     // the tile's own cells
                        st_wt(wout + so + row + x0 + tx, f0);
                        st_wt(wout + so + plane + row + x0 + tx, f1);
                        if constexpr (VM == VM_P) {
                            if (fresh) {              // p = r here
                                rhat[so + row + x0 + tx] = f0;
                                rhat[so + plane + row + x0 + tx] = f1;
                            }
                        } else if constexpr (VM == VM_PX) {
                            close_iteration(row + x0 + tx);
                            close_iteration(plane + row + x0 + tx);
                        }
                    }
                }
            }
            if (tx < 4) {
                const int gx = wrap(x0 - 2 + hux, nx);
                su[0][hz][hux] = field(row + gx);
                su[1][hz][hux] = field(plane + row + gx);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int sz = tg + 4 * k;
            if (sz < SZ) {
                const int hz = sz + 1;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h == 0 ? lane : (tx < 2)) {
                        const int sx = (h == 0) ? tx + 1 : hsx;
                        const int hx = sx + 1;
                        const real* m = (h == 0) ? m_in[k] : m_h[k];
                        const cplx ex = csub(su[0][hz][hx + 1], su[0][hz][hx - 1]);
                        const cplx ez = csub(su[1][hz + 1][hx], su[1][hz - 1][hx]);
                        const cplx exz = cadd(csub(su[0][hz + 1][hx], su[0][hz - 1][hx]),
                                                csub(su[1][hz][hx + 1], su[1][hz][hx - 1]));
                        ss[0][sz][sx] = mkc(m[0] * ex.x + m[1] * ez.x, m[0] * ex.y + m[1] * ez.y);
                        ss[1][sz][sx] = mkc(m[1] * ex.x + m[2] * ez.x, m[1] * ex.y + m[2] * ez.y);
                        ss[2][sz][sx] = cscale(exz, m[3]);
                    }
                }
            }
        }
        __syncthreads();
        if (lane) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int lz = tg + 4 * k;
                const int sz = lz + 1, sx = tx + 1;
                const cplx dx1 = csub(ss[0][sz][sx + 1], ss[0][sz][sx - 1]);
                const cplx dz5 = csub(ss[2][sz + 1][sx], ss[2][sz - 1][sx]);
                const cplx dx5 = csub(ss[2][sz][sx + 1], ss[2][sz][sx - 1]);
                const cplx dz3 = csub(ss[1][sz + 1][sx], ss[1][sz - 1][sx]);
                const cplx wr = cscale(pd.w2, rho[k]);
                const size_t gi = (size_t)(z0 + lz) * nx + x0 + tx;
                st_wt(bs + gi, cadd(cmul(wr, su[0][lz + 2][tx + 2]), cscale(cadd(dx1, dz5), sc)));
                st_wt(bs + plane + gi, cadd(cmul(wr, su[1][lz + 2][tx + 2]), cscale(cadd(dx5, dz3), sc)));
            }
        }
    }
}

// The same stencil marching along z: a block owns a TX-column strip over the
// row range [z0, z0 + ZR) of one system and walks it TZ rows at a time (TZ/4
// rows per thread).  LDS holds the input rows in a ring of RU rows and the
// stress rows in a ring of RS rows; the raw vectors of the input rows of the
// next one to three steps, and the maps of the next step's stress rows, are
// in flight in registers while a step computes.  Step at row z: the input rows z+2 ..
// z+TZ+1 enter the ring (own cells of the range write the updated vectors),
// the stress of rows z+1 .. z+TZ is formed, then b on rows z .. z+TZ-1.  Each
// input row of the range is read once, plus four halo rows per range, instead
// of the tiled kernel's TZ+4 rows per TZ.  The ring sizes keep every row a
// step reads alive until the next step's first barrier (RU >= 2 TZ + 2, RS
// >= TZ + 2), so a step needs two barriers.
template <int TZ>
struct MarchZ2 {
    static constexpr int KB = TZ / 4;                  // rows per thread per step
    static constexpr int RU = TZ == 4 ? 16 : 32;       // input ring rows
    static constexpr int RS = TZ == 4 ? 8 : 16;        // stress ring rows
    // steps of raw rows in flight: more where a step loads few bytes
    template <int VM>
    static constexpr int depth() { return TZ == 8 ? 1 : VM == VM_NONE ? 3 : VM == VM_PX ? 1 : 2; }
};

template <int TX, int TZ, int VM>
__global__ __launch_bounds__(256) void k_body_force_z(const cplx* __restrict__ u,
                                                      const cplx* __restrict__ a1,
                                                      const cplx* __restrict__ a2,
                                                      cplx* __restrict__ wout,
                                                      cplx* __restrict__ b,
                                                      const real* __restrict__ maps, ProbDev pd,
                                                      int ZR, SysState* __restrict__ st,
                                                      const double* __restrict__ part, int np,
                                                      cplx* __restrict__ rhat,
                                                      const cplx* __restrict__ a3,
                                                      cplx* __restrict__ xio,
                                                      cplx* __restrict__ rout, int SG) {
    static_assert(TX <= 64 && (TZ == 4 || TZ == 8), "tile");
    using Z = MarchZ2<TZ>;
    constexpr int KB = Z::KB, RU = Z::RU, RS = Z::RS;
    constexpr int HX = TX + 4, SX = TX + 2;
    constexpr int NV = VM == VM_NONE ? 1 : VM == VM_P ? 3 : VM == VM_PX ? 4 : 2;
    __shared__ cplx su[2][RU][HX];
    __shared__ cplx ss[3][RS][SX];
    __shared__ double red[4 * kPartialNV];
    const int nx = pd.nx, nz = pd.nz;
    const size_t plane = (size_t)nx * nz;
    const int ntx = nx / TX;
    const int ncol = ntx * (nz / ZR);
    // neighbouring blocks: the same strip and row range of SG systems (which
    // read the same maps), then the neighbouring strips and row ranges of
    // those systems (which read each other's cells as their halos)
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = blk / (ncol * SG), in = blk - grp * ncol * SG;
    const int col = in / SG;
    const int sys = grp * SG + (in - col * SG);
    const int x0 = (col % ntx) * TX, z0 = (col / ntx) * ZR, z1 = z0 + ZR;
    const int tx = threadIdx.x & 63, tg = threadIdx.x >> 6;
    const bool lane = tx < TX;
    const bool hlane = tx < 4;                // the x halo of the input rows
    const bool slane = tx < 2;                // the x halo of the stress rows
    const int hsx = (tx == 0) ? 0 : TX + 1;   // halo stress column of lanes 0 and 1
    const int hux = (tx < 2) ? tx : TX + tx;  // halo input column of lanes 0..3
    const int gxo = x0 + (lane ? tx : 0);                // own column
    const int gxh = wrap(x0 - 2 + hux, nx);              // input halo column
    const int gxs = wrap(x0 - 1 + hsx, nx);              // stress halo column

    if (st != nullptr) {   // uniform over the block
        const int stw = st[sys].status;
        if constexpr (VM == VM_PX) {
            if (!closing_enters(stw, kStampPx)) return;
        } else {
            if (stw != ST_RUNNING) {
                if (VM == VM_S && st_tag(stw) != 0 && col == 0 && threadIdx.x == 0) st[sys].status = st_code(stw);
                return;
            }
        }
    }
    cplx c1 = mkc(0.f, 0.f), c2 = mkc(0.f, 0.f), c3 = mkc(0.f, 0.f);
    bool fresh = false;
    int step = SS_FULL;
    if constexpr (VM != VM_NONE) {
        step = stencil_scalars<VM>(st, sys, part, np, red, col == 0 && threadIdx.x == 0, c1, c2, c3, fresh);
        if (step == SS_SKIP) return;
    }
    const size_t so = (size_t)sys * 2 * plane;
    auto rowoff = [&](int z) -> size_t { return (size_t)wrap(z, nz) * nx; };
    if constexpr (VM == VM_PX) {
        if (step == SS_XONLY) {   // stopped: the last solution update only
            if (lane)
                for (int z = z0 + tg; z < z1; z += 4)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const size_t gi = so + c * plane + rowoff(z) + gxo;
                        const cplx sv = u[gi], tv = a3[gi], pv = a1[gi];
                        const cplx rv = close_r(sv, tv, c2);
                        st_wt(rout + gi, rv);
                        st_wt(xio + gi, close_x(xio[gi], pv, sv, c3, c2));
                        if (fresh) rhat[gi] = rv;
                    }
            return;
        }
    }

    using Raw = cplx[NV][2];
    auto load_raw = [&](Raw& r, size_t g) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t gi = so + c * plane + g;
            r[0][c] = u[gi];
            if constexpr (VM == VM_P) {
                r[1][c] = a1[gi];
                r[2][c] = a2[gi];
            } else if constexpr (VM == VM_PX) {
                r[1][c] = a3[gi];
                r[2][c] = a1[gi];
                r[3][c] = a2[gi];
            } else if constexpr (VM == VM_S) {
                r[1][c] = a1[gi];
            }
        }
    };
    auto convert = [&](const Raw& r, cplx (&f)[2]) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if constexpr (VM == VM_NONE) {
                f[c] = r[0][c];
            } else if constexpr (VM == VM_P) {
                f[c] = fresh ? r[0][c] : cadd(r[0][c], cmul(c1, csub(r[1][c], cmul(c2, r[2][c]))));
            } else if constexpr (VM == VM_PX) {
                const cplx rv = close_r(r[0][c], r[1][c], c2);
                f[c] = fresh ? rv : cadd(rv, cmul(c1, csub(r[2][c], cmul(c2, r[3][c]))));
            } else {
                f[c] = csub(r[0][c], cmul(c1, r[1][c]));
            }
        }
    };
    // own cell of row z in the range: the updated vectors
    auto write_own = [&](const Raw& r, const cplx (&f)[2], const cplx (&xv)[2], int z) {
        if constexpr (VM != VM_NONE) {
            if (!lane || z < z0 || z >= z1) return;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const size_t gi = so + c * plane + rowoff(z) + gxo;
                st_wt(wout + gi, f[c]);
                if constexpr (VM == VM_P) {
                    if (fresh) rhat[gi] = f[c];
                } else if constexpr (VM == VM_PX) {
                    const cplx rv = close_r(r[0][c], r[1][c], c2);
                    st_wt(rout + gi, rv);
                    st_wt(xio + gi, close_x(xv[c], r[2][c], r[0][c], c3, c2));
                    if (fresh) rhat[gi] = rv;
                }
            }
        }
    };
    auto load_x = [&](cplx (&xv)[2], int z) {
        if constexpr (VM == VM_PX) {
            if (lane && z >= z0 && z < z1) {
                const size_t gi = so + rowoff(z) + gxo;
                xv[0] = xio[gi];
                xv[1] = xio[gi + plane];
            }
        }
    };
    // raw rows of one step (own and halo cells of this thread's rows)
    struct Rows {
        Raw o[KB], h[KB];
        cplx x[KB][2];
    };
    auto load_rows = [&](Rows& R, int zb) {   // rows zb + tg + 4k
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int z = zb + tg + 4 * k;
            const size_t ro = rowoff(z);
            if (lane) load_raw(R.o[k], ro + gxo);
            if (hlane) load_raw(R.h[k], ro + gxh);
            load_x(R.x[k], z);
        }
    };
    auto put_rows = [&](const Rows& R, int zb) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int z = zb + tg + 4 * k;
            const int slot = (z - z0 + 2 * RU) & (RU - 1);
            cplx f[2];
            if (lane) {
                convert(R.o[k], f);
                su[0][slot][tx + 2] = f[0];
                su[1][slot][tx + 2] = f[1];
                write_own(R.o[k], f, R.x[k], z);
            }
            if (hlane) {
                convert(R.h[k], f);
                su[0][slot][hux] = f[0];
                su[1][slot][hux] = f[1];
            }
        }
    };
    // stiffness maps (C11, C13, C33, C55) of a stress row at the own and halo column
    struct SMaps {
        real o[KB][4], h[KB][4];
    };
    auto load_smaps = [&](SMaps& m, int zb) {   // stress rows zb + tg + 4k
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const size_t ro = rowoff(zb + tg + 4 * k);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                m.o[k][c] = lane ? maps[c * plane + ro + gxo] : 0.f;
                m.h[k][c] = slane ? maps[c * plane + ro + gxs] : 0.f;
            }
        }
    };
    // stress of row z at stress column sx (input column sx + 1) into the ring
    auto stress_at = [&](int z, int sx, const real (&m)[4]) {
        const int hx = sx + 1;
        const int lo = (z - 1 - z0 + 2 * RU) & (RU - 1), mid = (z - z0 + 2 * RU) & (RU - 1),
                  hi = (z + 1 - z0 + 2 * RU) & (RU - 1);
        const cplx ex = csub(su[0][mid][hx + 1], su[0][mid][hx - 1]);
        const cplx ez = csub(su[1][hi][hx], su[1][lo][hx]);
        const cplx exz = cadd(csub(su[0][hi][hx], su[0][lo][hx]), csub(su[1][mid][hx + 1], su[1][mid][hx - 1]));
        const int s = (z - z0 + 2 * RS) & (RS - 1);
        ss[0][s][sx] = mkc(m[0] * ex.x + m[1] * ez.x, m[0] * ex.y + m[1] * ez.y);
        ss[1][s][sx] = mkc(m[1] * ex.x + m[2] * ez.x, m[1] * ex.y + m[2] * ez.y);
        ss[2][s][sx] = cscale(exz, m[3]);
    };

    // ---- prologue: input rows z0-2 .. z0+1 (one per thread group), stress
    // rows z0-1 and z0
    {
        const int z = z0 - 2 + tg;
        Raw ro, rh;
        cplx xv[2] = {};
        if (lane) load_raw(ro, rowoff(z) + gxo);
        if (hlane) load_raw(rh, rowoff(z) + gxh);
        load_x(xv, z);
        const int slot = (z - z0 + 2 * RU) & (RU - 1);
        cplx f[2];
        if (lane) {
            convert(ro, f);
            su[0][slot][tx + 2] = f[0];
            su[1][slot][tx + 2] = f[1];
            write_own(ro, f, xv, z);
        }
        if (hlane) {
            convert(rh, f);
            su[0][slot][hux] = f[0];
            su[1][slot][hux] = f[1];
        }
        real m[4], mh[4];
        if (tg < 2) {
            const size_t rm = rowoff(z0 - 1 + tg);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                m[c] = lane ? maps[c * plane + rm + gxo] : 0.f;
                mh[c] = slane ? maps[c * plane + rm + gxs] : 0.f;
            }
        }
        __syncthreads();
        if (tg < 2) {
            if (lane) stress_at(z0 - 1 + tg, tx + 1, m);
            if (slane) stress_at(z0 - 1 + tg, hsx, mh);
        }
    }
    // PD steps of raw rows in flight (buffers used in turn: the step loop is
    // unrolled by PD so that no register of a load in flight is moved)
    constexpr int PD = MarchZ2<TZ>::template depth<VM>();
    Rows R[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j)
        if (z0 + j * TZ < z1) load_rows(R[j], z0 + j * TZ + 2);
    SMaps mc, mn;
    load_smaps(mc, z0 + 1);
    real rc[KB], rn[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) rc[k] = lane ? maps[4 * plane + rowoff(z0 + tg + 4 * k) + gxo] : 0.f;
    const real sc = pd.inv4dx2;
    auto row_step = [&](int z, Rows& RA) {
        // the new input rows enter the ring; later rows and the next step's maps are issued
        put_rows(RA, z + 2);
        if (z + PD * TZ < z1) load_rows(RA, z + PD * TZ + 2);
        const bool more = z + TZ < z1;
        if (more) {
            load_smaps(mn, z + TZ + 1);
#pragma unroll
            for (int k = 0; k < KB; ++k) rn[k] = lane ? maps[4 * plane + rowoff(z + TZ + tg + 4 * k) + gxo] : 0.f;
        }
        __syncthreads();
        // stress of rows z+1 .. z+TZ
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int zs = z + 1 + tg + 4 * k;
            if (lane) stress_at(zs, tx + 1, mc.o[k]);
            if (slane) stress_at(zs, hsx, mc.h[k]);
        }
        __syncthreads();
        // b on rows z .. z+TZ-1
        if (lane) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int zo = z + tg + 4 * k;
                const int s = (zo - z0 + 2 * RS) & (RS - 1), sm = (zo - 1 - z0 + 2 * RS) & (RS - 1),
                          sp = (zo + 1 - z0 + 2 * RS) & (RS - 1);
                const int uo = (zo - z0 + 2 * RU) & (RU - 1);
                const int sx = tx + 1;
                const cplx dx1 = csub(ss[0][s][sx + 1], ss[0][s][sx - 1]);
                const cplx dz5 = csub(ss[2][sp][sx], ss[2][sm][sx]);
                const cplx dx5 = csub(ss[2][s][sx + 1], ss[2][s][sx - 1]);
                const cplx dz3 = csub(ss[1][sp][sx], ss[1][sm][sx]);
                const cplx wr = cscale(pd.w2, rc[k]);
                const size_t gi = so + rowoff(zo) + gxo;
                st_wt(b + gi, cadd(cmul(wr, su[0][uo][tx + 2]), cscale(cadd(dx1, dz5), sc)));
                st_wt(b + plane + gi, cadd(cmul(wr, su[1][uo][tx + 2]), cscale(cadd(dx5, dz3), sc)));
            }
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                rc[k] = rn[k];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    mc.o[k][c] = mn.o[k][c];
                    mc.h[k][c] = mn.h[k][c];
                }
            }
        }
    };
    for (int z = z0; z < z1; z += PD * TZ) {
#pragma unroll
        for (int j = 0; j < PD; ++j)
            if (z + j * TZ < z1) row_step(z + j * TZ, R[j]);   // uniform over the block
    }
}

// Tile width for nx: the largest of 64, 48, 32, 24, 16 dividing it.
static int tile_x(int nx) {
    const int cand[] = {64, 48, 32, 24, 16};
    for (int c : cand)
        if (nx % c == 0) return c;
    return 0;
}

StCfg st_default() { return StCfg{STZ, 0}; }

bool st_cfg_ok(int nx, int nz, const StCfg& c) {
    if (tile_x(nx) == 0) return false;
    if (c.S == kStMarch) {   // the z-marching kernel: 4- or 8-row steps
#ifdef FW_C128
        if (c.TZ != 4) return false;   // its 8-row rings exceed the static LDS limit
#else
        if (c.TZ != 4 && c.TZ != 8) return false;
#endif
        return nz % c.TZ == 0 && nz >= 2 * c.TZ;
    }
#ifdef FW_C128
    if (c.TZ != 4 && c.TZ != 8) return false;   // 16-row complex128 tiles exceed the static LDS limit
#else
    if (c.TZ != 4 && c.TZ != 8 && c.TZ != 16) return false;
#endif
    if (nz % c.TZ != 0) return false;
    return c.S == 0 || c.S == 1 || c.S == 2 || c.S == 4 || c.S == 8 || c.S == 16;
}

int st_candidates(int nx, int nz, StCfg* out, int cap) {
    int k = 0;
    const int tzs[3] = {8, 4, 16};
    const int ss[6] = {0, 1, 2, 4, 8, kStMarch};
    for (int tz : tzs)
        for (int sv : ss) {
            const StCfg c{tz, sv};
            if (st_cfg_ok(nx, nz, c) && k < cap) out[k++] = c;
        }
    return k;
}

// The BiCGSTAB update of a stencil's input on its own, as a streaming pass
// over the n complex values of each system's field: the same scalars, stop
// decisions and element arithmetic as the update fused into the stencil
// kernels (stencil_scalars, close_r, close_x), writing the updated input (p
// or s) that the plain stencil then reads.  bps blocks per system; block 0 of
// a system records its scalars and status.
template <int VM>
__global__ __launch_bounds__(256) void k_bicg_update(const cplx* __restrict__ u, const cplx* __restrict__ a1,
                                                 const cplx* __restrict__ a2, cplx* __restrict__ wout,
                                                 SysState* __restrict__ st, const double* __restrict__ part, int np,
                                                 cplx* __restrict__ rhat, const cplx* __restrict__ a3,
                                                 cplx* __restrict__ xio, cplx* __restrict__ rout, int n, int bps) {
    __shared__ double red[4 * kPartialNV];
    __shared__ int s_status;
    const int sys = blockIdx.x / bps, bi = blockIdx.x - sys * bps;
    const int t = threadIdx.x;
    if (t == 0) s_status = st[sys].status;
    __syncthreads();
    const int stw = s_status;
    __syncthreads();
    if constexpr (VM == VM_PX) {
        if (!closing_enters(stw, kStampPx)) return;
    } else {
        if (stw != ST_RUNNING) {
            if (VM == VM_S && st_tag(stw) != 0 && bi == 0 && t == 0) st[sys].status = st_code(stw);
            return;
        }
    }
    cplx c1 = mkc(0.f, 0.f), c2 = mkc(0.f, 0.f), c3 = mkc(0.f, 0.f);
    bool fresh = false;
    const int step = stencil_scalars<VM>(st, sys, part, np, red, bi == 0 && t == 0, c1, c2, c3, fresh);
    if (step == SS_SKIP) return;
    const size_t so = (size_t)sys * n;
    const cplx* __restrict__ us = u + so;
    const cplx* __restrict__ a1s = a1 + so;
    const cplx* __restrict__ a2s = a2 + so;
    const cplx* __restrict__ a3s = a3 + so;
    cplx* __restrict__ wos = wout + so;
    cplx* __restrict__ rhs = rhat + so;
    cplx* __restrict__ xs = xio + so;
    cplx* __restrict__ ros = rout + so;
    constexpr int U = 4;   // elements per thread in flight
    const int stride = bps * 256;
    for (int i0 = bi * 256 + t; i0 < n; i0 += U * stride) {
        cplx r0[U], r1[U], r2[U], r3[U], xv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = i0 + k * stride;
            if (i < n) {
                r0[k] = us[i];
                if constexpr (VM == VM_P) {
                    r1[k] = a1s[i];
                    r2[k] = a2s[i];
                } else if constexpr (VM == VM_PX) {
                    r1[k] = a3s[i];
                    r2[k] = a1s[i];
                    if (step == SS_FULL) r3[k] = a2s[i];
                    xv[k] = xs[i];
                } else if constexpr (VM == VM_S) {
                    r1[k] = a1s[i];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = i0 + k * stride;
            if (i >= n) continue;
            if constexpr (VM == VM_P) {
                const cplx f = fresh ? r0[k] : cadd(r0[k], cmul(c1, csub(r1[k], cmul(c2, r2[k]))));
                st_wt(wos + i, f);
                if (fresh) st_wt(rhs + i, f);
            } else if constexpr (VM == VM_PX) {
                const cplx rv = close_r(r0[k], r1[k], c2);
                st_wt(ros + i, rv);
                st_wt(xs + i, close_x(xv[k], r2[k], r0[k], c3, c2));
                if (step == SS_FULL) {
                    const cplx f = fresh ? rv : cadd(rv, cmul(c1, csub(r2[k], cmul(c2, r3[k]))));
                    st_wt(wos + i, f);
                    if (fresh) st_wt(rhs + i, rv);
                }
            } else if constexpr (VM == VM_S) {
                st_wt(wos + i, csub(r0[k], cmul(c1, r1[k])));
            }
        }
    }
}

hipError_t launch_bicg_update(int vm, const StencilArgs& a, long long n, int nsys, SysState* st, hipStream_t s) {
    if ((vm != VM_P && vm != VM_PX && vm != VM_S) || !st || !a.wout || n <= 0 || n > 0x7fffffffLL || nsys < 1 ||
        ((vm == VM_P || vm == VM_PX) && !a.rhat) || (vm == VM_PX && (!a.a3 || !a.xio || !a.rout)))
        return hipErrorInvalidValue;
    // blocks per system: at least 2048 blocks in the launch while every
    // thread has a few elements
    int bps = 1;
    while ((long long)bps * nsys < 2048 && (long long)bps * 2 * 256 * 4 <= n) bps *= 2;
    const dim3 grid((unsigned)(bps * nsys));
#define FW_UPD(V)                                                                                            \
    hipLaunchKernelGGL((k_bicg_update<V>), grid, dim3(256), 0, s, a.u, a.a1, a.a2, a.wout, st, a.part, a.np, \
                       a.rhat, a.a3, a.xio, a.rout, (int)n, bps)
    if (vm == VM_P) FW_UPD(VM_P);
    else if (vm == VM_PX) FW_UPD(VM_PX);
    else FW_UPD(VM_S);
#undef FW_UPD
    return hipGetLastError();
}

// Row range of the z-marching kernel: the whole column, halved (while it
// stays a multiple of the step and at least 32 rows) until the launch has
// 8192 workgroups.
static int march_rows(int nx, int tx, int nz, int tz, int nsys) {
    int zr = nz;
    while (zr % 2 == 0 && (zr / 2) % tz == 0 && zr / 2 >= 32 &&
           (long long)(nx / tx) * (nz / zr) * nsys < 8192)
        zr /= 2;
    return zr;
}

template <int TX, int TZ, int VM>
static void body_force_z_launch(const StencilArgs& a, const ProbDev& pd, SysState* st, hipStream_t s) {
    const int zr = march_rows(pd.nx, TX, pd.nz, TZ, pd.nsys);
    const long long blocks = (long long)(pd.nx / TX) * (pd.nz / zr) * pd.nsys;
    // systems per group of neighbouring blocks (the largest power of two up
    // to 16 that divides the system count): their blocks of one strip and
    // range read the same maps while those are in the XCD's L2.  1024^2 x 128
    // systems, plain pass: 3.74 -> 3.52 ms (one system per group: the maps
    // came from memory again for every system; all systems of a strip in one
    // group: 3.72 ms, the halo lines of neighbouring strips no longer shared)
    int sg = 1;
    while (sg * 2 <= 16 && pd.nsys % (sg * 2) == 0) sg *= 2;
    hipLaunchKernelGGL((k_body_force_z<TX, TZ, VM>), dim3((unsigned)blocks), dim3(256), 0, s, a.u, a.a1, a.a2,
                       a.wout, a.b, a.maps, pd, zr, st, a.part, a.np, a.rhat, a.a3, a.xio, a.rout, sg);
}

template <int TX, int TZ, int VM>
static hipError_t body_force_launch(const StCfg& c, const StencilArgs& a, const ProbDev& pd, SysState* st,
                                    hipStream_t s) {
    if constexpr (TZ == 4 || TZ == 8) {
        if (c.S == kStMarch) {
            body_force_z_launch<TX, TZ, VM>(a, pd, st, s);
            return hipGetLastError();
        }
    }
    const int ntiles = (pd.nx / TX) * (pd.nz / TZ);
    // the solver's update modes carry two to five vectors per system and take
    // the automatic count (the tuned count is timed in the plain mode)
    int S = VM == VM_NONE ? c.S : 0;
    if (S == 0) {
        // several systems per block once there are plenty of blocks
        S = 1;
        while (S < pd.nsys && (long long)ntiles * ((pd.nsys + 2 * S - 1) / (2 * S)) >= 2048) S *= 2;
    }
    S = std::min(S, std::max(pd.nsys, 1));
    const int blocks = ntiles * ((pd.nsys + S - 1) / S);
    hipLaunchKernelGGL((k_body_force<TX, TZ, VM>), dim3(blocks), dim3(256), 0, s, a.u, a.a1, a.a2, a.wout,
                       a.b, a.maps, pd, S, st, a.part, a.np, a.rhat, a.a3, a.xio, a.rout);
    return hipGetLastError();
}

template <int TX, int TZ>
static hipError_t body_force_vm(int vm, const StCfg& c, const StencilArgs& a, const ProbDev& pd, SysState* st,
                                hipStream_t s) {
    if (vm == VM_NONE) return body_force_launch<TX, TZ, VM_NONE>(c, a, pd, st, s);
    if (vm == VM_P) return body_force_launch<TX, TZ, VM_P>(c, a, pd, st, s);
    if (vm == VM_PX) return body_force_launch<TX, TZ, VM_PX>(c, a, pd, st, s);
    return body_force_launch<TX, TZ, VM_S>(c, a, pd, st, s);
}

template <int TX>
static hipError_t body_force_tz(int vm, const StCfg& c, const StencilArgs& a, const ProbDev& pd, SysState* st,
                                hipStream_t s) {
    if (c.TZ == 4) return body_force_vm<TX, 4>(vm, c, a, pd, st, s);
#ifndef FW_C128
    if (c.TZ == 16) return body_force_vm<TX, 16>(vm, c, a, pd, st, s);
#endif
    return body_force_vm<TX, 8>(vm, c, a, pd, st, s);
}

hipError_t launch_stencil(int vm, const StCfg& c, const StencilArgs& a, const ProbDev& pd, SysState* st,
                          hipStream_t s) {
    if (!st_cfg_ok(pd.nx, pd.nz, c) || vm < 0 || vm > 3 || (vm != 0 && !st) || ((vm == VM_P || vm == VM_PX) && !a.rhat) ||
        (vm == VM_PX && (!a.a3 || !a.xio || !a.rout)))
        return hipErrorInvalidValue;
    switch (tile_x(pd.nx)) {
        case 64: return body_force_tz<64>(vm, c, a, pd, st, s);
        case 48: return body_force_tz<48>(vm, c, a, pd, st, s);
        case 32: return body_force_tz<32>(vm, c, a, pd, st, s);
        case 24: return body_force_tz<24>(vm, c, a, pd, st, s);
        case 16: return body_force_tz<16>(vm, c, a, pd, st, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_body_force(const StCfg& c, const cplx* u, cplx* b, const real* maps,
                             const ProbDev& pd, const SysState* st, hipStream_t s) {
    StencilArgs a{u, nullptr, nullptr, nullptr, b, maps, nullptr, 0};
    return launch_stencil(VM_NONE, c, a, pd, const_cast<SysState*>(st), s);
}

KernelCfg kernel_cfg_default(int nx, int nz) {
    KernelCfg k;
    k.row_p = row_points_default(nx);
    k.row_pi = k.row_p;
    k.col = col_default(nz, nx);
    k.st = st_default();
    k.fuse_p = 0;
    return k;
}

// -------------------------------------------------------------- vectors --
int vec_blocks_per_sys(int n) { return (n + kVecThreads * kVecEPT - 1) / (kVecThreads * kVecEPT); }


// Block -> (system, block within system) for the vector kernels.
struct VecIdx {
    int sys, bi, i0;
};
__device__ __forceinline__ VecIdx vec_idx(int nb) {
    VecIdx v;
    v.sys = blockIdx.x / nb;
    v.bi = blockIdx.x - v.sys * nb;
    v.i0 = v.bi * kVecThreads * kVecEPT;
    return v;
}

// r = b (or r already holds b - A x0), x = 0 if zero_x, rhat = r, p = v = 0;
// partials <rhat, r>, ||r||^2 and ||b||^2.
__global__ __launch_bounds__(256) void k_bicg_init(const cplx* __restrict__ b,
                                                   const cplx* r0,   // may alias r
                                                   cplx* __restrict__ x, cplx* r,
                                                   cplx* __restrict__ rhat, cplx* __restrict__ p,
                                                   cplx* __restrict__ v,
                                                   double* __restrict__ partXR,
                                                   double* __restrict__ partB, int n, int nb,
                                                   int zero_x) {
    __shared__ double red[4 * 4];
    const VecIdx vi = vec_idx(nb);
    const size_t off = (size_t)vi.sys * n;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
        const int i = vi.i0 + e * kVecThreads + threadIdx.x;
        if (i < n) {
            const cplx bb = b[off + i];
            const cplx rr = r0 ? r0[off + i] : bb;
            if (zero_x) x[off + i] = mkc(0.f, 0.f);
            r[off + i] = rr;
            rhat[off + i] = rr;
            p[off + i] = mkc(0.f, 0.f);
            v[off + i] = mkc(0.f, 0.f);
            const double q = (double)rr.x * rr.x + (double)rr.y * rr.y;
            acc[0] += q;
            acc[2] += q;
            acc[3] += (double)bb.x * bb.x + (double)bb.y * bb.y;
        }
    }
    block_allreduce<4, 256>(acc, red);
    if (threadIdx.x == 0) {
        double* d = partXR + ((size_t)vi.sys * nb + vi.bi) * kPartialNV;
        d[0] = acc[0];
        d[1] = 0.0;
        d[2] = acc[2];
        d[3] = 0.0;
        partB[((size_t)vi.sys * nb + vi.bi) * kPartialNV] = acc[3];
    }
}

__global__ __launch_bounds__(256) void k_bicg_state_init(SysState* __restrict__ st,
                                                         const double* __restrict__ partXR,
                                                         const double* __restrict__ partB, int np,
                                                         double rtol, int maxit) {
    __shared__ double red[4 * 4];
    const int sys = blockIdx.x;
    double s[4];
    sum_partials<4, 256>(partB + (size_t)sys * np * kPartialNV, np, s, red);
    double q[4];
    sum_partials<4, 256>(partXR + (size_t)sys * np * kPartialNV, np, q, red);
    if (threadIdx.x == 0) {
        SysState z;
        z.rho_re[0] = 1.0; z.rho_im[0] = 0.0;
        z.rho_re[1] = 1.0; z.rho_im[1] = 0.0;
        z.alpha_re = 1.0; z.alpha_im = 0.0;
        z.omega_re = 1.0; z.omega_im = 0.0;
        z.bnorm2 = s[0];
        z.tol2 = rtol * rtol * s[0];
        z.rnorm2 = q[2];
        z.iter = 0;
        z.maxit = maxit;
        z.restarts = 0;
        z.best2 = q[2];
        z.best_iter = 0;
        z.fresh_at = 0;
        z.status = (s[0] == 0.0) ? ST_CONVERGED : ST_RUNNING;
        st[sys] = z;
    }
}


// End of a chunk of iterations: the stop decision of the last iteration from
// its t-pass records (so that the host sees every stopped system), with the
// closing updates x += alpha p + omega s, r = s - omega t owed to a stopped
// system.  A running system gets its stagnation bookkeeping only; its closing
// updates are left to the next direction-update stencil.
__global__ __launch_bounds__(256) void k_bicg_close(cplx* __restrict__ x, cplx* __restrict__ r,
                                                    const cplx* __restrict__ p,
                                                    const cplx* __restrict__ sv,
                                                    const cplx* __restrict__ t,
                                                    const double* __restrict__ partT, int npT,
                                                    SysState* __restrict__ st, int n, int nb) {
    __shared__ double red[4 * kPartialNV];
    const VecIdx vi = vec_idx(nb);
    if (!closing_enters(st[vi.sys].status, kStampClose)) return;   // uniform over the block
    double q[kPartialNV];
    sum_partials<kPartialNV, 256>(partT + (size_t)vi.sys * npT * kPartialNV, npT, q, red);
    SysState& z = st[vi.sys];
    const OmegaStep o = omega_step(q);
    const int code = close_code(z, o);
    const bool writer = vi.bi == 0 && threadIdx.x == 0;
    if (code == ST_RUNNING) {
        if (writer) {
            // stagnation: the best residual norm has not halved for kStallIters
            // iterations -> the next iteration restarts the recurrence (r^ = r)
            z.rnorm2 = o.rr;
            if (o.rr < 0.25 * z.best2) {
                z.best2 = o.rr;
                z.best_iter = z.iter;
            } else if (z.iter - z.best_iter >= kStallIters) {
                z.fresh_at = z.iter + 1;
                z.best2 = o.rr;
                z.best_iter = z.iter;
            }
        }
        return;
    }
    if (code != ST_NONFINITE) {
        const cplx af = toc(dcomplex{z.alpha_re, z.alpha_im}), of = toc(o.omega);
        const size_t off = (size_t)vi.sys * n;
#pragma unroll
        for (int e = 0; e < kVecEPT; ++e) {
            const int i = vi.i0 + e * kVecThreads + threadIdx.x;
            if (i < n) {
                const cplx svv = sv[off + i];
                st_wt(r + off + i, close_r(svv, t[off + i], of));
                st_wt(x + off + i, close_x(x[off + i], p[off + i], svv, af, of));
            }
        }
    }
    if (writer) {
        z.status = st_stamp(code, kStampClose);
        z.omega_re = o.omega.re;
        z.omega_im = o.omega.im;
        z.rnorm2 = o.rr;
    }
}

__global__ __launch_bounds__(256) void k_bicg_finish(const SysState* __restrict__ st,
                                                     const double* __restrict__ partTR, int np,
                                                     int32_t* __restrict__ iters,
                                                     double* __restrict__ relres) {
    __shared__ double red[4 * 4];
    const int sys = blockIdx.x;
    double q[4];
    sum_partials<4, 256>(partTR + (size_t)sys * np * kPartialNV, np, q, red);
    if (threadIdx.x == 0) {
        const double bb = st[sys].bnorm2;
        if (iters) iters[sys] = st[sys].iter;
        if (relres) relres[sys] = bb > 0.0 ? sqrt(q[0] / bb) : 0.0;
    }
}

// After a solve, systems are restarted from their current x (r = b - A x in
// partTR, fresh shadow residual r^ = r), at most max_restarts times each:
//   - converged on the recursive residual while the true residual ||b - A x||^2
//     exceeds limit2 ||b||^2 (the recursion drifted in finite precision);
//   - broken down (a BiCGSTAB scalar became exactly zero): x is the last
//     completed iterate, so restarting with r^ = r resumes the solve.
__global__ __launch_bounds__(256) void k_bicg_restart_mark(SysState* __restrict__ st,
                                                           const double* __restrict__ partTR, int np,
                                                           double limit2, int max_restarts) {
    __shared__ double red[4 * 4];
    const int sys = blockIdx.x;
    const int status = st_code(st[sys].status);
    if (status != ST_CONVERGED && status != ST_BREAKDOWN) return;
    double q[4];
    sum_partials<4, 256>(partTR + (size_t)sys * np * kPartialNV, np, q, red);
    if (threadIdx.x == 0 && st[sys].restarts < max_restarts &&
        (status == ST_BREAKDOWN || q[0] > limit2 * st[sys].bnorm2)) {
        st[sys].status = ST_RESTART;
        st[sys].restarts += 1;
    }
}

// Restart marked systems from the true residual now in r (the caller reran
// k_bicg_init with r0 = r): fresh BiCGSTAB scalars, iteration count kept.
__global__ void k_bicg_restart(SysState* __restrict__ st, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys || st[sys].status != ST_RESTART) return;
    SysState& z = st[sys];
    z.rho_re[0] = z.rho_re[1] = 1.0;
    z.rho_im[0] = z.rho_im[1] = 0.0;
    z.alpha_re = z.omega_re = 1.0;
    z.alpha_im = z.omega_im = 0.0;
    z.best2 = 1e300;
    z.best_iter = z.iter;
    z.fresh_at = 0;
    z.status = (z.iter >= z.maxit) ? ST_MAXIT : ST_RUNNING;
}

hipError_t launch_bicg_restart_mark(SysState* st, const double* partTR, int npTR, int nsys, double limit2,
                                    int max_restarts, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_restart_mark, dim3(nsys), dim3(256), 0, s, st, partTR, npTR, limit2,
                       max_restarts);
    return hipGetLastError();
}

hipError_t launch_bicg_restart(SysState* st, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_restart, dim3((nsys + 63) / 64), dim3(64), 0, s, st, nsys);
    return hipGetLastError();
}

hipError_t launch_bicg_init(const cplx* b, const cplx* r0, cplx* x, cplx* r, cplx* rhat,
                            cplx* p, cplx* v, double* partXR, double* partB, int nsys, int n,
                            bool zero_x, hipStream_t s) {
    const int nb = vec_blocks_per_sys(n);
    hipLaunchKernelGGL(k_bicg_init, dim3(nsys * nb), dim3(kVecThreads), 0, s, b, r0, x, r, rhat, p,
                       v, partXR, partB, n, nb, zero_x ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bicg_state_init(SysState* st, const double* partXR, const double* partB,
                                  int nsys, int npart, double rtol, int maxit, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_state_init, dim3(nsys), dim3(256), 0, s, st, partXR, partB, npart,
                       rtol, maxit);
    return hipGetLastError();
}

hipError_t launch_bicg_close(cplx* x, cplx* r, const cplx* p, const cplx* sv, const cplx* t,
                             const double* partT, int npT, SysState* st, int nsys, int n, hipStream_t s) {
    const int nb = vec_blocks_per_sys(n);
    hipLaunchKernelGGL(k_bicg_close, dim3(nsys * nb), dim3(kVecThreads), 0, s, x, r, p, sv, t, partT, npT, st, n,
                       nb);
    return hipGetLastError();
}

hipError_t launch_bicg_finish(const SysState* st, const double* partTR, int npTR, int nsys,
                              int32_t* iters, double* relres, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_finish, dim3(nsys), dim3(256), 0, s, st, partTR, npTR, iters, relres);
    return hipGetLastError();
}

// ------------------------------------------------------ copy and zero -----
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
__global__ __launch_bounds__(256) void k_zero(float4* __restrict__ dst, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// n complex elements, moved as 16-byte words (n is even for every field of
// this library).
constexpr size_t kCplxPerWord = 16 / sizeof(cplx);
hipError_t launch_copy(const cplx* src, cplx* dst, size_t n, hipStream_t s) {
    const size_t n4 = n / kCplxPerWord;
    const int blocks = (int)std::min<size_t>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n4);
    return hipGetLastError();
}
// out = a - b over n complex elements (out may alias a or b).
__global__ __launch_bounds__(256) void k_diff(const cplx* __restrict__ a, const cplx* b, cplx* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = csub(a[i], b[i]);
}
hipError_t launch_diff(const cplx* a, const cplx* b, cplx* out, size_t n, hipStream_t s) {
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_diff, dim3(blocks), dim3(256), 0, s, a, b, out, n);
    return hipGetLastError();
}
hipError_t launch_zero_d2(double2* dst, size_t n, hipStream_t s) {
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (float4*)dst, n);
    return hipGetLastError();
}
hipError_t launch_zero(cplx* dst, size_t n, hipStream_t s) {
    const size_t n4 = n / kCplxPerWord;
    const int blocks = (int)std::min<size_t>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (float4*)dst, n4);
    return hipGetLastError();
}

// ---------------------------------------------------- sources, receivers --
// f must be zero on entry: one force per system, F / dx^2 at (ix, iz).
__global__ void k_point_sources(cplx* __restrict__ f, const int32_t* __restrict__ ixz,
                                const double* __restrict__ force, ProbDev pd) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= pd.nsys) return;
    const size_t plane = (size_t)pd.nx * pd.nz;
    const int ix = ixz[2 * sys], iz = ixz[2 * sys + 1];
    const double inv = 1.0 / ((double)pd.dx * (double)pd.dx);
    cplx* fs = f + (size_t)sys * 2 * plane + (size_t)iz * pd.nx + ix;
    fs[0] = mkc((real)(force[2 * sys] * inv), 0.f);
    fs[plane] = mkc((real)(force[2 * sys + 1] * inv), 0.f);
}

hipError_t launch_point_sources(cplx* f, const int32_t* src_ixz, const double* src_f,
                                const ProbDev& pd, hipStream_t s) {
    hipLaunchKernelGGL(k_point_sources, dim3((pd.nsys + 63) / 64), dim3(64), 0, s, f, src_ixz, src_f, pd);
    return hipGetLastError();
}

// d[sys][rec][c] = w[sys][c][iz][ix]
__global__ void k_gather(const cplx* __restrict__ w, cplx* __restrict__ d,
                         const int32_t* __restrict__ rec, int nrec, ProbDev pd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = pd.nsys * nrec * 2;
    if (i >= total) return;
    const int c = i & 1;
    const int rr = (i >> 1) % nrec;
    const int sys = (i >> 1) / nrec;
    const size_t plane = (size_t)pd.nx * pd.nz;
    d[i] = w[(size_t)sys * 2 * plane + c * plane + (size_t)rec[2 * rr + 1] * pd.nx + rec[2 * rr]];
}

hipError_t launch_gather(const cplx* w, cplx* d, const int32_t* rec_ixz, int nrec,
                         const ProbDev& pd, hipStream_t s) {
    const int total = pd.nsys * nrec * 2;
    hipLaunchKernelGGL(k_gather, dim3((total + 255) / 256), dim3(256), 0, s, w, d, rec_ixz, nrec, pd);
    return hipGetLastError();
}

// f (zero on entry) += conj(d) at the receivers; one thread per (sys, c)
// walks the receivers in order, so repeated receivers add deterministically.
// f += R^T conj(d) (the adjoint source of eq. ua0).  Receivers are taken in
// the stable cell order the host built (perm) with the length of each run of
// receivers on one cell at the run's first entry (glen, 0 elsewhere): one
// thread per (system, run, component) sums its run in receiver order, so the
// result does not depend on the launch.
__global__ void k_scatter_conj(const cplx* __restrict__ d, cplx* __restrict__ f,
                               const int32_t* __restrict__ rec, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ glen, int nrec, ProbDev pd) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)pd.nsys * nrec * 2) return;
    const int c = (int)(i & 1);
    const size_t q = i >> 1;
    const int k = (int)(q % nrec), sys = (int)(q / nrec);
    const int n = glen[k];
    if (n == 0) return;
    const cplx* ds = d + (size_t)sys * nrec * 2 + c;
    const int r0 = perm[k];
    cplx acc = cconj(ds[2 * (size_t)r0]);
    for (int j = 1; j < n; ++j) acc = cadd(acc, cconj(ds[2 * (size_t)perm[k + j]]));
    const size_t plane = (size_t)pd.nx * pd.nz;
    cplx* fs = f + (size_t)sys * 2 * plane + c * plane;
    const size_t gi = (size_t)rec[2 * r0 + 1] * pd.nx + rec[2 * r0];
    fs[gi] = cadd(fs[gi], acc);
}

hipError_t launch_scatter_conj(const cplx* d, cplx* f, const int32_t* rec_ixz, const int32_t* perm,
                               const int32_t* glen, int nrec, const ProbDev& pd, hipStream_t s) {
    const size_t total = (size_t)pd.nsys * nrec * 2;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_conj, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, f, rec_ixz, perm,
                       glen, nrec, pd);
    return hipGetLastError();
}

// ------------------------------------------------------- correlation -----
// g_rho = conj(w~^2 sum_sys u^a . u^b); g_p = -conj(sum_sys eps^a . B^p eps^b),
// with the 2-D B matrices of the maps (C11, C13, C33, C55):
//   B11 -> e1 e1,  B13 -> e1 e3 + e3 e1,  B33 -> e3 e3,  B55 -> e5 e5.
// A block covers 64 cells; its four thread groups take every fourth system
// and their FP64 sums are added in group order (a fixed order: the result
// does not depend on the launch).
template <class OUT>
__global__ __launch_bounds__(256) void k_correlate(const cplx* __restrict__ ua,
                                                   const cplx* __restrict__ ub,
                                                   OUT* __restrict__ g, ProbDev pd, int accumulate) {
    constexpr int NA = 10;   // accumulators: rho, B11, B13, B33, B55 (re, im)
    __shared__ double red[3][NA][64];
    const int nx = pd.nx, nz = pd.nz;
    const size_t plane = (size_t)nx * nz;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int cell = blockIdx.x * 64 + lane;
    const bool live = cell < (int)plane;
    const int cc = live ? cell : 0;
    const int z = cc / nx, x = cc - z * nx;
    const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
    const int zp = (z + 1 == nz) ? 0 : z + 1, zm = (z == 0) ? nz - 1 : z - 1;
    const size_t ic = cc, ixp = (size_t)z * nx + xp, ixm = (size_t)z * nx + xm;
    const size_t izp = (size_t)zp * nx + x, izm = (size_t)zm * nx + x;
    double acc[NA] = {};
    for (int s = grp; s < pd.nsys; s += 4) {
        const cplx* A = ua + (size_t)s * 2 * plane;
        const cplx* B = ub + (size_t)s * 2 * plane;
        const cplx ax = A[ic], az = A[plane + ic], bx = B[ic], bz = B[plane + ic];
        acc[0] += (double)ax.x * bx.x - (double)ax.y * bx.y + (double)az.x * bz.x - (double)az.y * bz.y;
        acc[1] += (double)ax.x * bx.y + (double)ax.y * bx.x + (double)az.x * bz.y + (double)az.y * bz.x;
        const cplx e1a = csub(A[ixp], A[ixm]);
        const cplx e3a = csub(A[plane + izp], A[plane + izm]);
        const cplx e5a = cadd(csub(A[izp], A[izm]), csub(A[plane + ixp], A[plane + ixm]));
        const cplx e1b = csub(B[ixp], B[ixm]);
        const cplx e3b = csub(B[plane + izp], B[plane + izm]);
        const cplx e5b = cadd(csub(B[izp], B[izm]), csub(B[plane + ixp], B[plane + ixm]));
        acc[2] += (double)e1a.x * e1b.x - (double)e1a.y * e1b.y;
        acc[3] += (double)e1a.x * e1b.y + (double)e1a.y * e1b.x;
        acc[4] += (double)e1a.x * e3b.x - (double)e1a.y * e3b.y + (double)e3a.x * e1b.x - (double)e3a.y * e1b.y;
        acc[5] += (double)e1a.x * e3b.y + (double)e1a.y * e3b.x + (double)e3a.x * e1b.y + (double)e3a.y * e1b.x;
        acc[6] += (double)e3a.x * e3b.x - (double)e3a.y * e3b.y;
        acc[7] += (double)e3a.x * e3b.y + (double)e3a.y * e3b.x;
        acc[8] += (double)e5a.x * e5b.x - (double)e5a.y * e5b.y;
        acc[9] += (double)e5a.x * e5b.y + (double)e5a.y * e5b.x;
    }
    if (grp > 0) {
#pragma unroll
        for (int k = 0; k < NA; ++k) red[grp - 1][k][lane] = acc[k];
    }
    __syncthreads();
    if (grp > 0 || !live) return;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] += red[j][k][lane];
    const double rr = acc[0], ri = acc[1];
    const double s = (double)pd.inv4dx2;
    const double wr = pd.w2.x, wi = pd.w2.y;
    // conj(w2 * rho) ; -conj(a) * s
    const double out[5][2] = {{-acc[2] * s, acc[3] * s},
                              {-acc[4] * s, acc[5] * s},
                              {-acc[6] * s, acc[7] * s},
                              {-acc[8] * s, acc[9] * s},
                              {wr * rr - wi * ri, -(wr * ri + wi * rr)}};
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        OUT* dst = g + (size_t)p * plane + ic;
        OUT o = accumulate ? *dst : OUT{};
        o.x = (decltype(o.x))((double)o.x + out[p][0]);
        o.y = (decltype(o.y))((double)o.y + out[p][1]);
        *dst = o;
    }
}

hipError_t launch_correlate(const cplx* ua, const cplx* ub, cplx* g, const ProbDev& pd,
                            bool accumulate, hipStream_t s) {
    const int cells = pd.nx * pd.nz;
    hipLaunchKernelGGL(k_correlate<cplx>, dim3((cells + 63) / 64), dim3(256), 0, s, ua, ub, g, pd,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_correlate_f64(const cplx* ua, const cplx* ub, double2* g, const ProbDev& pd,
                                bool accumulate, hipStream_t s) {
    const int cells = pd.nx * pd.nz;
    hipLaunchKernelGGL(k_correlate<double2>, dim3((cells + 63) / 64), dim3(256), 0, s, ua, ub, g, pd,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

FW_END