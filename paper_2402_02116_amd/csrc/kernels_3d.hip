// Kernels of the 3-D, generally anisotropic LS solve, J and J* (the
// 21-constant form of eqs. decom, u_2 and dC; the six-strain vectors of the
// abbreviated subscript section; App. C for the VTI set):
//   k_stencil3        - contrast stencil b = w~^2 drho u + div_h(dC : E_h u) on
//                       [nsys][3][nz][ny][nx] fields, with the BiCGSTAB vector
//                       update of its input fused into the load (bicg.h);
//   k_axis            - FFT along y or z (a strided axis) in place, and the z
//                       pass that multiplies by the 3 x 3 Green's tensor
//                       G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1 between its
//                       forward and inverse transforms;
//   k_point_sources3, k_gather3, k_scatter_conj3 - sources and receivers;
//   k_correlate3      - the adjoint correlation of eq. ad1 summed over
//                       systems in FP64.
// The x transforms are the row kernels of the 2-D path (rows of nx points).
#include <algorithm>
#include <numeric>

#include "bicg.h"
#include "fft_kernels.h"

FW_BEGIN
__device__ __forceinline__ int wrapm(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// ------------------------------------------------------ contrast stencil --
// Number of stiffness maps of a parametrisation (the density map follows).
template <bool GEN>
struct Params3 { static constexpr int NS = GEN ? 21 : 5; };

// sigma = dC e for one cell: VTI maps (dC11, dC13, dC33, dC55, dC66), with
// dC12 = dC11 - 2 dC66, dC22 = dC11, dC23 = dC13, dC44 = dC55 (App. C), or
// the 21 constants of the upper triangle in row-major order.
template <bool GEN>
__device__ __forceinline__ void stress3(const real* m, int mstride, const cplx (&e)[6], cplx (&s)[6]) {
    if constexpr (!GEN) {
        const real c11 = m[0], c13 = m[mstride], c33 = m[2 * mstride], c55 = m[3 * mstride],
                   c66 = m[4 * mstride];
        const real c12 = c11 - 2.f * c66;
        s[0] = mkc(c11 * e[0].x + c12 * e[1].x + c13 * e[2].x, c11 * e[0].y + c12 * e[1].y + c13 * e[2].y);
        s[1] = mkc(c12 * e[0].x + c11 * e[1].x + c13 * e[2].x, c12 * e[0].y + c11 * e[1].y + c13 * e[2].y);
        s[2] = mkc(c13 * (e[0].x + e[1].x) + c33 * e[2].x, c13 * (e[0].y + e[1].y) + c33 * e[2].y);
        s[3] = cscale(e[3], c55);
        s[4] = cscale(e[4], c55);
        s[5] = cscale(e[5], c66);
    } else {
        real c[6][6];
        int p = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) {
                c[i][j] = m[p * mstride];
                c[j][i] = c[i][j];
                ++p;
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            real sx = 0, sy = 0;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                sx += c[i][j] * e[j].x;
                sy += c[i][j] * e[j].y;
            }
            s[i] = mkc(sx, sy);
        }
    }
}

// A block owns a TX x TY x TZ tile of cells and loops over S systems of the
// same problem.  The stiffness contrast of the tile plus a 1-cell halo and the
// density of the tile go to LDS once.  Per system:
//   1. the input field (the vector update applied) on the tile plus a 2-cell
//      halo goes to LDS; own cells write the updated vectors;
//   2. the stress s' = dC e' (e' = raw central differences, 2 dx times the
//      Voigt strain) on the tile plus a 1-cell halo, in LDS;
//   3. b = w~^2 drho u + (1 / 4 dx^2) div'(s') on the tile.
// Tiles may overhang the grid: loads wrap periodically and only in-grid
// cells are written.
template <int TX, int TY, int TZ>
struct Tile3 {
    static constexpr int HX = TX + 4, HY = TY + 4, HZ = TZ + 4, HC = HX * HY * HZ;
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2, SC = SX * SY * SZ;
    static constexpr int OC = TX * TY * TZ;
};

template <bool GEN, int TX, int TY, int TZ>
inline size_t stencil3_lds() {
    using T = Tile3<TX, TY, TZ>;
    return (size_t)(3 * T::HC + 6 * T::SC) * sizeof(cplx) +
           (size_t)(Params3<GEN>::NS * T::SC + T::OC) * sizeof(real);
}

template <int VM, bool GEN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_stencil3(const cplx* __restrict__ u, const cplx* __restrict__ a1,
                                                  const cplx* __restrict__ a2, cplx* __restrict__ wout,
                                                  cplx* __restrict__ b, const real* __restrict__ maps, ProbDev3 pd,
                                                  int S, SysState* __restrict__ st, const double* __restrict__ part,
                                                  int np, cplx* __restrict__ rhat, const cplx* __restrict__ a3,
                                                  cplx* __restrict__ xio, cplx* __restrict__ rout) {
    using T = Tile3<TX, TY, TZ>;
    constexpr int NS = Params3<GEN>::NS;
    extern __shared__ __align__(16) unsigned char lds3[];
    cplx* su = reinterpret_cast<cplx*>(lds3);          // [3][HC]
    cplx* ss = su + 3 * T::HC;                           // [6][SC]
    real* sm = reinterpret_cast<real*>(ss + 6 * T::SC);  // [NS][SC], then rho [OC]
    __shared__ double red[4 * kPartialNV];
    __shared__ int s_status;

    const int nx = pd.nx, ny = pd.ny, nz = pd.nz;
    const size_t cells = (size_t)nx * ny * nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    const int nsg = (pd.nsys + S - 1) / S;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = blk / nsg;
    const int sys0 = (blk - tile * nsg) * S;
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    auto gcell = [&](int dx_, int dy_, int dz_) -> size_t {
        return ((size_t)wrapm(z0 + dz_, nz) * ny + wrapm(y0 + dy_, ny)) * nx + wrapm(x0 + dx_, nx);
    };

    // contrast of the stress region and density of the tile
    for (int q = threadIdx.x; q < T::SC; q += 256) {
        const int sx = q % T::SX, sy = (q / T::SX) % T::SY, sz = q / (T::SX * T::SY);
        const size_t g = gcell(sx - 1, sy - 1, sz - 1);
#pragma unroll
        for (int p = 0; p < NS; ++p) sm[p * T::SC + q] = maps[(size_t)p * cells + g];
    }
    for (int o = threadIdx.x; o < T::OC; o += 256) {
        const int ox = o % TX, oy = (o / TX) % TY, oz = o / (TX * TY);
        sm[NS * T::SC + o] = maps[(size_t)NS * cells + gcell(ox, oy, oz)];
    }

    const real sc = pd.inv4dx2;
    for (int sys = sys0; sys < sys0 + S && sys < pd.nsys; ++sys) {
        if (st != nullptr) {
            // one read per block, broadcast: another block's writer may change
            // the word meanwhile, and every thread must take the same branch
            if (threadIdx.x == 0) s_status = st[sys].status;
            __syncthreads();
            const int stw = s_status;
            __syncthreads();
            if constexpr (VM == VM_PX) {
                if (!closing_enters(stw, kStampPx)) continue;
            } else {
                if (stw != ST_RUNNING) {
                    // the iteration's closing kernel is done: drop its tag
                    if (VM == VM_S && st_tag(stw) != 0 && tile == 0 && threadIdx.x == 0) st[sys].status = st_code(stw);
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
        const size_t so = (size_t)sys * 3 * cells;
        // VM_PX on an own cell: r = s - omega t, x += alpha p_old + omega s
        auto close_iteration = [&](size_t gi) {
            const cplx sv = u[so + gi], tv = a3[so + gi], pv = a1[so + gi];
            const cplx rv = close_r(sv, tv, c2);
            rout[so + gi] = rv;
            xio[so + gi] = close_x(xio[so + gi], pv, sv, c3, c2);
            if (fresh) rhat[so + gi] = rv;
        };
        if constexpr (VM == VM_PX) {
            if (step == SS_XONLY) {   // stopped: the last solution update only
                for (int o = threadIdx.x; o < T::OC; o += 256) {
                    const int ox = o % TX, oy = (o / TX) % TY, oz = o / (TX * TY);
                    if (x0 + ox >= nx || y0 + oy >= ny || z0 + oz >= nz) continue;
                    const size_t g = gcell(ox, oy, oz);
#pragma unroll
                    for (int c = 0; c < 3; ++c) close_iteration(c * cells + g);
                }
                continue;
            }
        }
        // input field value at index gi of this system (component offset included)
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
        __syncthreads();   // the previous system's reads of su / ss are done
        for (int h = threadIdx.x; h < T::HC; h += 256) {
            const int hx = h % T::HX, hy = (h / T::HX) % T::HY, hz = h / (T::HX * T::HY);
            const size_t g = gcell(hx - 2, hy - 2, hz - 2);
            const bool own = hx >= 2 && hx < TX + 2 && hy >= 2 && hy < TY + 2 && hz >= 2 && hz < TZ + 2 &&
                             x0 + hx - 2 < nx && y0 + hy - 2 < ny && z0 + hz - 2 < nz;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t gi = c * cells + g;
                const cplx f = field(gi);
                su[c * T::HC + h] = f;
                if constexpr (VM != VM_NONE) {
                    if (own) {
                        wout[so + gi] = f;
                        if constexpr (VM == VM_P) {
                            if (fresh) rhat[so + gi] = f;   // p = r here
                        } else if constexpr (VM == VM_PX) {
                            close_iteration(gi);
                        }
                    }
                }
            }
        }
        __syncthreads();
        constexpr int DY = T::HX, DZ = T::HX * T::HY;
        for (int q = threadIdx.x; q < T::SC; q += 256) {
            const int sx = q % T::SX, sy = (q / T::SX) % T::SY, sz = q / (T::SX * T::SY);
            const int h = ((sz + 1) * T::HY + sy + 1) * T::HX + sx + 1;
            cplx d[3][3];   // d[c][j]: raw difference of component c along axis j
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const cplx* w = su + c * T::HC + h;
                d[c][0] = csub(w[1], w[-1]);
                d[c][1] = csub(w[DY], w[-DY]);
                d[c][2] = csub(w[DZ], w[-DZ]);
            }
            const cplx e[6] = {d[0][0], d[1][1], d[2][2], cadd(d[1][2], d[2][1]), cadd(d[0][2], d[2][0]),
                               cadd(d[0][1], d[1][0])};
            cplx s[6];
            stress3<GEN>(sm + q, T::SC, e, s);
#pragma unroll
            for (int i = 0; i < 6; ++i) ss[i * T::SC + q] = s[i];
        }
        __syncthreads();
        constexpr int EY = T::SX, EZ = T::SX * T::SY;
        for (int o = threadIdx.x; o < T::OC; o += 256) {
            const int ox = o % TX, oy = (o / TX) % TY, oz = o / (TX * TY);
            if (x0 + ox >= nx || y0 + oy >= ny || z0 + oz >= nz) continue;
            const int q = ((oz + 1) * T::SY + oy + 1) * T::SX + ox + 1;
            auto dd = [&](int i, int off) { return csub(ss[i * T::SC + q + off], ss[i * T::SC + q - off]); };
            // b_i = sum_j D_j sigma_ij, Voigt (xx, yy, zz, yz, xz, xy) = (0..5)
            const cplx bx = cadd(cadd(dd(0, 1), dd(5, EY)), dd(4, EZ));
            const cplx by = cadd(cadd(dd(5, 1), dd(1, EY)), dd(3, EZ));
            const cplx bz = cadd(cadd(dd(4, 1), dd(3, EY)), dd(2, EZ));
            const int h = ((oz + 2) * T::HY + oy + 2) * T::HX + ox + 2;
            const cplx wr = cscale(pd.w2, sm[NS * T::SC + o]);
            const size_t g = so + gcell(ox, oy, oz);
            b[g] = cadd(cmul(wr, su[h]), cscale(bx, sc));
            b[g + cells] = cadd(cmul(wr, su[T::HC + h]), cscale(by, sc));
            b[g + 2 * cells] = cadd(cmul(wr, su[2 * T::HC + h]), cscale(bz, sc));
        }
    }
}

// The same stencil marching along z: a block owns a TX x TY column of cells
// over the z range [z0, z1) of one system and walks it plane by plane.  LDS
// holds the input (vector update applied) on three planes z, z+1, z+2 with a
// 2-cell xy halo, and the stress s' on planes z and z+1 with a 1-cell halo;
// the stress of plane z-1 at the thread's own cell stays in registers (only
// the z difference of the own column needs it).  Step z: load plane z+2 into
// the buffer of plane z-1, form the stress of plane z+1, then b on plane z.
// Every input plane of the range is loaded once (own cells write the updated
// vectors then), plus four halo planes per range: each input value is read
// (TX+4)(TY+4)/(TX TY) * (z1-z0+4)/(z1-z0) times instead of the tiled kernel's
// (TX+4)(TY+4)(TZ+4)/(TX TY TZ).
template <int TX, int TY>
struct March3 {
    static constexpr int HX = TX + 4, HY = TY + 4, HP = HX * HY;   // input plane with halo 2
    static constexpr int SX = TX + 2, SY = TY + 2, SP = SX * SY;   // stress plane with halo 1
    static constexpr int NT = TX * TY;                             // one thread per column
};

template <int TX, int TY>
inline size_t march3_lds() {
    using M = March3<TX, TY>;
    return (size_t)(3 * 3 * M::HP + 2 * 6 * M::SP) * sizeof(cplx);
}

template <int VM, bool GEN, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_stencil3z(const cplx* __restrict__ u, const cplx* __restrict__ a1,
                                                       const cplx* __restrict__ a2, cplx* __restrict__ wout,
                                                       cplx* __restrict__ b, const real* __restrict__ maps,
                                                       ProbDev3 pd, int ZC, SysState* __restrict__ st,
                                                       const double* __restrict__ part, int np,
                                                       cplx* __restrict__ rhat, const cplx* __restrict__ a3,
                                                       cplx* __restrict__ xio, cplx* __restrict__ rout) {
    using M = March3<TX, TY>;
    constexpr int NT = M::NT;
    static_assert(NT == 256, "the FP64 record sums of the Krylov scalars read with 256 threads");
    constexpr int NS = Params3<GEN>::NS;
    extern __shared__ __align__(16) unsigned char lds3[];
    cplx* su = reinterpret_cast<cplx*>(lds3);   // [3 planes][3 comps][HP]
    cplx* ss = su + 9 * M::HP;                  // [2 planes][6][SP]
    __shared__ double red[4 * kPartialNV];
    __shared__ int s_status;

    const int nx = pd.nx, ny = pd.ny, nz = pd.nz;
    const size_t cells = (size_t)nx * ny * nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, nzc = (nz + ZC - 1) / ZC;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk % pd.nsys;                 // neighbouring blocks: the same column, other systems
    const int col = blk / pd.nsys;
    const int x0 = (col % ntx) * TX, y0 = ((col / ntx) % nty) * TY, z0 = (col / (ntx * nty)) * ZC;
    const int z1 = min(z0 + ZC, nz);
    (void)nzc;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const bool own_xy = x0 + tx < nx && y0 + ty < ny;

    if (st != nullptr) {
        if (threadIdx.x == 0) s_status = st[sys].status;
        __syncthreads();
        const int stw = s_status;
        __syncthreads();
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
    const size_t so = (size_t)sys * 3 * cells;
    auto gidx = [&](int x, int y, int z) -> size_t {
        return ((size_t)wrapm(z, nz) * ny + wrapm(y, ny)) * nx + wrapm(x, nx);
    };
    auto close_iteration = [&](size_t gi) {
        const cplx sv = u[so + gi], tv = a3[so + gi], pv = a1[so + gi];
        const cplx rv = close_r(sv, tv, c2);
        rout[so + gi] = rv;
        xio[so + gi] = close_x(xio[so + gi], pv, sv, c3, c2);
        if (fresh) rhat[so + gi] = rv;
    };
    if constexpr (VM == VM_PX) {
        if (step == SS_XONLY) {   // stopped: the last solution update only
            if (own_xy)
                for (int z = z0; z < z1; ++z) {
                    const size_t g = gidx(x0 + tx, y0 + ty, z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) close_iteration(c * cells + g);
                }
            return;
        }
    }
    auto field = [&](size_t gi) -> cplx {
        if constexpr (VM == VM_NONE) {
            return u[so + gi];
        } else if constexpr (VM == VM_P) {
            const cplx rv = u[so + gi];
            if (fresh) return rv;
            return cadd(rv, cmul(c1, csub(a1[so + gi], cmul(c2, a2[so + gi]))));
        } else if constexpr (VM == VM_PX) {
            const cplx rv = close_r(u[so + gi], a3[so + gi], c2);
            if (fresh) return rv;
            return cadd(rv, cmul(c1, csub(a1[so + gi], cmul(c2, a2[so + gi]))));
        } else {
            return csub(u[so + gi], cmul(c1, a1[so + gi]));
        }
    };
    // input plane z (with the 2-cell xy halo) into buffer k; own cells of the
    // range write the updated vectors
    auto load_plane = [&](int k, int z) {
        const bool own_z = z >= z0 && z < z1;
        cplx* dst = su + k * 3 * M::HP;
        for (int h = threadIdx.x; h < M::HP; h += NT) {
            const int hx = h % M::HX, hy = h / M::HX;
            const size_t g = gidx(x0 - 2 + hx, y0 - 2 + hy, z);
            const bool own = own_z && hx >= 2 && hx < TX + 2 && hy >= 2 && hy < TY + 2 && x0 + hx - 2 < nx &&
                             y0 + hy - 2 < ny;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t gi = c * cells + g;
                const cplx f = field(gi);
                dst[c * M::HP + h] = f;
                if constexpr (VM != VM_NONE) {
                    if (own) {
                        wout[so + gi] = f;
                        if constexpr (VM == VM_P) {
                            if (fresh) rhat[so + gi] = f;
                        } else if constexpr (VM == VM_PX) {
                            close_iteration(gi);
                        }
                    }
                }
            }
        }
    };
    // raw strain at input-buffer position h of plane `mid` (z differences
    // from planes lo and hi), then the stress s' = dC e'
    auto stress_at = [&](const cplx* lo, const cplx* mid, const cplx* hi, int h, const real* mp, size_t mstride,
                         cplx (&sg)[6]) {
        cplx d[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cplx* w = mid + c * M::HP + h;
            d[c][0] = csub(w[1], w[-1]);
            d[c][1] = csub(w[M::HX], w[-M::HX]);
            d[c][2] = csub(hi[c * M::HP + h], lo[c * M::HP + h]);
        }
        const cplx e[6] = {d[0][0], d[1][1], d[2][2], cadd(d[1][2], d[2][1]), cadd(d[0][2], d[2][0]),
                           cadd(d[0][1], d[1][0])};
        real m[NS];
#pragma unroll
        for (int p = 0; p < NS; ++p) m[p] = mp[p * mstride];
        stress3<GEN>(m, 1, e, sg);
    };
    // stress of plane z (buffers lo = z-1, mid = z, hi = z+1) into stress buffer j
    auto stress_plane = [&](int j, const cplx* lo, const cplx* mid, const cplx* hi, int z) {
        cplx* dst = ss + j * 6 * M::SP;
        for (int q = threadIdx.x; q < M::SP; q += NT) {
            const int sx = q % M::SX, sy = q / M::SX;
            const int h = (sy + 1) * M::HX + sx + 1;
            cplx sg[6];
            stress_at(lo, mid, hi, h, maps + gidx(x0 - 1 + sx, y0 - 1 + sy, z), cells, sg);
#pragma unroll
            for (int i = 0; i < 6; ++i) dst[i * M::SP + q] = sg[i];
        }
    };

    // prologue: input planes z0-1, z0, z0+1; the own column's stress of plane
    // z0-1 (its z difference reads the own cell of plane z0-2 directly); the
    // stress plane z0
    int kb[3] = {0, 1, 2};   // buffers of planes z-1, z, z+1 (then z, z+1, z+2)
    load_plane(kb[0], z0 - 1);
    load_plane(kb[1], z0);
    load_plane(kb[2], z0 + 1);
    __syncthreads();
    const int hown = (ty + 2) * M::HX + tx + 2;
    const int qown = (ty + 1) * M::SX + tx + 1;
    cplx sprev[6];
    {
        const size_t g = gidx(x0 + tx, y0 + ty, z0 - 2);   // the own cell of plane z0-2
        cplx below[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) below[c] = field(c * cells + g);
        cplx d[3][3];
        const cplx* mid = su + kb[0] * 3 * M::HP;
        const cplx* hi = su + kb[1] * 3 * M::HP;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cplx* w = mid + c * M::HP + hown;
            d[c][0] = csub(w[1], w[-1]);
            d[c][1] = csub(w[M::HX], w[-M::HX]);
            d[c][2] = csub(hi[c * M::HP + hown], below[c]);
        }
        const cplx e[6] = {d[0][0], d[1][1], d[2][2], cadd(d[1][2], d[2][1]), cadd(d[0][2], d[2][0]),
                           cadd(d[0][1], d[1][0])};
        real m[NS];
        const real* mp = maps + gidx(x0 + tx, y0 + ty, z0 - 1);
#pragma unroll
        for (int p = 0; p < NS; ++p) m[p] = mp[p * cells];
        stress3<GEN>(m, 1, e, sprev);
    }
    int jc = 0;   // stress buffer of the current plane
    stress_plane(jc, su + kb[0] * 3 * M::HP, su + kb[1] * 3 * M::HP, su + kb[2] * 3 * M::HP, z0);
    __syncthreads();
    // now kb = {z0-1, z0, z0+1}: rotate so that kb = {z, z+1, (free)}
    const real sc = pd.inv4dx2;
    for (int z = z0; z < z1; ++z) {
        // buffers: kb[1] = plane z, kb[2] = plane z+1, kb[0] = plane z-1 (free now)
        load_plane(kb[0], z + 2);
        __syncthreads();
        const cplx* pz = su + kb[1] * 3 * M::HP;
        const cplx* pz1 = su + kb[2] * 3 * M::HP;
        const cplx* pz2 = su + kb[0] * 3 * M::HP;
        stress_plane(1 - jc, pz, pz1, pz2, z + 1);
        __syncthreads();
        const cplx* cur = ss + jc * 6 * M::SP;
        const cplx* nxt = ss + (1 - jc) * 6 * M::SP;
        if (own_xy) {
            auto dxy = [&](int i, int off) { return csub(cur[i * M::SP + qown + off], cur[i * M::SP + qown - off]); };
            auto dz = [&](int i) { return csub(nxt[i * M::SP + qown], sprev[i]); };
            const cplx bx = cadd(cadd(dxy(0, 1), dxy(5, M::SX)), dz(4));
            const cplx by = cadd(cadd(dxy(5, 1), dxy(1, M::SX)), dz(3));
            const cplx bz = cadd(cadd(dxy(4, 1), dxy(3, M::SX)), dz(2));
            const size_t g = gidx(x0 + tx, y0 + ty, z);
            const cplx wr = cscale(pd.w2, maps[(size_t)NS * cells + g]);
            b[so + g] = cadd(cmul(wr, pz[hown]), cscale(bx, sc));
            b[so + g + cells] = cadd(cmul(wr, pz[M::HP + hown]), cscale(by, sc));
            b[so + g + 2 * cells] = cadd(cmul(wr, pz[2 * M::HP + hown]), cscale(bz, sc));
#pragma unroll
            for (int i = 0; i < 6; ++i) sprev[i] = cur[i * M::SP + qown];
        }
        __syncthreads();   // plane z and stress plane z are read: their buffers are free
        const int k0 = kb[0];
        kb[0] = kb[1];
        kb[1] = kb[2];
        kb[2] = k0;
        jc = 1 - jc;
    }
}

template <int VM, bool GEN, int TX, int TY>
static hipError_t stencil3z_launch(const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    const int ntx = (pd.nx + TX - 1) / TX, nty = (pd.ny + TY - 1) / TY;
    // z ranges of at most 32 planes, more of them while the launch is small
    int ZC = std::min(pd.nz, 32);
    while (ZC > 8 && (long long)ntx * nty * ((pd.nz + ZC - 1) / ZC) * pd.nsys < 4096) ZC /= 2;
    const long long blocks = (long long)ntx * nty * ((pd.nz + ZC - 1) / ZC) * pd.nsys;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = march3_lds<TX, TY>();
    hipError_t e = allow_lds(k_stencil3z<VM, GEN, TX, TY>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stencil3z<VM, GEN, TX, TY>), dim3((unsigned)blocks), dim3(TX * TY), lds, s, a.u, a.a1,
                       a.a2, a.wout, a.b, a.maps, pd, ZC, st, a.part, a.np, a.rhat, a.a3, a.xio, a.rout);
    return hipGetLastError();
}

// Tile of the build: 8 x 8 x 4 cells (complex64), 4 x 4 x 4 (complex128,
// twice the bytes per value).
#ifdef FW_C128
constexpr int kT3X = 4, kT3Y = 4, kT3Z = 4;
#else
constexpr int kT3X = 8, kT3Y = 8, kT3Z = 4;
#endif

template <int VM, bool GEN>
static hipError_t stencil3_launch(const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    const int ntiles = ((pd.nx + kT3X - 1) / kT3X) * ((pd.ny + kT3Y - 1) / kT3Y) * ((pd.nz + kT3Z - 1) / kT3Z);
    int S = 1;
    while (S < pd.nsys && (long long)ntiles * ((pd.nsys + 2 * S - 1) / (2 * S)) >= 2048) S *= 2;
    S = std::min(S, std::max(pd.nsys, 1));
    const int blocks = ntiles * ((pd.nsys + S - 1) / S);
    const size_t lds = stencil3_lds<GEN, kT3X, kT3Y, kT3Z>();
    hipError_t e = allow_lds(k_stencil3<VM, GEN, kT3X, kT3Y, kT3Z>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stencil3<VM, GEN, kT3X, kT3Y, kT3Z>), dim3(blocks), dim3(256), lds, s, a.u, a.a1, a.a2,
                       a.wout, a.b, a.maps, pd, S, st, a.part, a.np, a.rhat, a.a3, a.xio, a.rout);
    return hipGetLastError();
}

// Column shape of the z-marching stencil (256 threads): 16 x 16 or 32 x 8
// cells, whichever overhangs the grid less; 0 for grids thinner than 8 cells
// in y, which take the tiled kernel.
static int march_shape(int nx, int ny) {
    if (ny < 8 || nx < 16) return 0;
    const long long a = (long long)((nx + 15) / 16) * 16 * ((ny + 15) / 16) * 16;
    const long long b = (long long)((nx + 31) / 32) * 32 * ((ny + 7) / 8) * 8;
    return a <= b ? 16 : 32;
}

template <int VM, bool GEN>
static hipError_t stencil3_any(const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    const int m = march_shape(pd.nx, pd.ny);
    if (m == 16) return stencil3z_launch<VM, GEN, 16, 16>(a, pd, st, s);
    if (m == 32) return stencil3z_launch<VM, GEN, 32, 8>(a, pd, st, s);
    return stencil3_launch<VM, GEN>(a, pd, st, s);
}

template <bool GEN>
static hipError_t stencil3_vm(int vm, const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    if (vm == VM_NONE) return stencil3_any<VM_NONE, GEN>(a, pd, st, s);
    if (vm == VM_P) return stencil3_any<VM_P, GEN>(a, pd, st, s);
    if (vm == VM_PX) return stencil3_any<VM_PX, GEN>(a, pd, st, s);
    return stencil3_any<VM_S, GEN>(a, pd, st, s);
}

hipError_t launch_stencil3(int vm, const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    if (vm < 0 || vm > 3 || (vm != 0 && !st) || ((vm == VM_P || vm == VM_PX) && !a.rhat) ||
        (vm == VM_PX && (!a.a3 || !a.xio || !a.rout)) || (vm != VM_NONE && !a.wout))
        return hipErrorInvalidValue;
    return pd.params == kParamsGeneral ? stencil3_vm<true>(vm, a, pd, st, s) : stencil3_vm<false>(vm, a, pd, st, s);
}

// ------------------------------------------------------ strided axes -----
// Transforms along an axis of length N with stride S (the product of the
// faster dimensions): the data is [nslab][N][S] (AX_FWD, AX_INV: one slab per
// (system, component, outer index)) or [nsys][3][N][S] (AX_GREEN: the z pass
// of the three components of one system).  A block takes W adjacent columns
// of one slab; thread (t, c) holds positions t + T m of column c.
struct AxisLds {
    cplx* base;
    int stride, PL;
    __device__ __forceinline__ cplx& operator()(int f, int pos) const {
        return base[(f * PL + lds_pad(pos)) * stride];
    }
};

// out = gscale (Gamma' - ga I)^-1 b for the real symmetric scaled
// Christoffel matrix Gamma' (entries xx, yy, zz, yz, xz, xy), by the
// adjugate of the complex symmetric 3 x 3 matrix.
__device__ __forceinline__ void green_mul3(cplx (&b)[3], const real (&g)[6], cplx ga, real gscale) {
    const cplx mxx = mkc(g[0] - ga.x, -ga.y), myy = mkc(g[1] - ga.x, -ga.y), mzz = mkc(g[2] - ga.x, -ga.y);
    const real myz = g[3], mxz = g[4], mxy = g[5];
    const cplx axx = mkc(cmul(myy, mzz).x - myz * myz, cmul(myy, mzz).y);
    const cplx ayy = mkc(cmul(mxx, mzz).x - mxz * mxz, cmul(mxx, mzz).y);
    const cplx azz = mkc(cmul(mxx, myy).x - mxy * mxy, cmul(mxx, myy).y);
    const cplx axy = csub(mkc(mxz * myz, 0.f), cscale(mzz, mxy));
    const cplx axz = csub(mkc(mxy * myz, 0.f), cscale(myy, mxz));
    const cplx ayz = csub(mkc(mxy * mxz, 0.f), cscale(mxx, myz));
    const cplx det = cadd(cmul(mxx, axx), cadd(cscale(axy, mxy), cscale(axz, mxz)));
    const real s = gscale / (det.x * det.x + det.y * det.y);
    const cplx inv = mkc(det.x * s, -det.y * s);
    const cplx gx = cmul(inv, b[0]), gy = cmul(inv, b[1]), gz = cmul(inv, b[2]);
    b[0] = cadd(cmul(axx, gx), cadd(cmul(axy, gy), cmul(axz, gz)));
    b[1] = cadd(cmul(axy, gx), cadd(cmul(ayy, gy), cmul(ayz, gz)));
    b[2] = cadd(cmul(axz, gx), cadd(cmul(ayz, gy), cmul(azz, gz)));
}

// Wavenumber of index i on an n-point axis: exact (dk * signed index) or the
// central-difference symbol sin(2 pi i / n) / dx.
__device__ __forceinline__ real axis_k(int i, int n, real dk, real dx, bool central) {
    const int si = fft_signed(i, n);
    return central ? rsinpi(2.0f * (real)si / (real)n) / dx : (real)si * dk;
}

template <int N, int P, int MODE>
__global__ __launch_bounds__(256) void k_axis(cplx* __restrict__ data, int S, int W, int slabs_per_sys,
                                              const SysState* __restrict__ st, const cplx* __restrict__ tw,
                                              ProbDev3 pd) {
    using FS = FftShape<N, P>;
    constexpr int T = FS::T;
    constexpr int PL = PaddedLen<N>::value;
    constexpr int NC = MODE == AX_GREEN ? 3 : 1;
    extern __shared__ cplx lds_dyn[];

    const int tid = threadIdx.x;
    const int c = tid % W, t = tid / W;
    const int ncb = S / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int slab = blk / ncb;
    const int col = (blk - slab * ncb) * W + c;
    const int sys = MODE == AX_GREEN ? slab : slab / slabs_per_sys;
    if (st != nullptr && st[sys].status != ST_RUNNING) return;
    const bool active = t < T;
    const size_t span = (size_t)N * S;
    cplx* base = data + (size_t)slab * NC * span + col;

    cplx v[NC][P];
#pragma unroll
    for (int f = 0; f < NC; ++f)
#pragma unroll
        for (int m = 0; m < P; ++m) v[f][m] = active ? base[f * span + (size_t)(t + T * m) * S] : mkc(0.f, 0.f);
    AxisLds lds{active ? lds_dyn + c : lds_dyn + (size_t)NC * PL * W, active ? W : 1, PL};
    const int tt = active ? t : 0;
    if constexpr (MODE != AX_INV) fft_run<N, P, false, NC>(v, tt, tw, lds);
    if constexpr (MODE == AX_GREEN) {
        const int ix = col % pd.nx, iy = col / pd.nx;
        const bool central = pd.symbol == 1;
        const real kx = axis_k(ix, pd.nx, pd.dk[0], pd.dx, central);
        const real ky = axis_k(iy, pd.ny, pd.dk[1], pd.dx, central);
        // products of two different components: 0 at an even axis's Nyquist index
        const real kxo = (pd.nx % 2 == 0 && ix == pd.nx / 2) ? 0.f : kx;
        const real kyo = (pd.ny % 2 == 0 && iy == pd.ny / 2) ? 0.f : ky;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int iz = tt + T * m;
            const real kz = axis_k(iz, N, pd.dk[2], pd.dx, central);
            const real kzo = (N % 2 == 0 && iz == N / 2) ? 0.f : kz;
            const real mono[6] = {kx * kx, ky * ky, kz * kz, kyo * kzo, kxo * kzo, kxo * kyo};
            real g[6];
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                real a = 0;
#pragma unroll
                for (int q = 0; q < 6; ++q) a += pd.gq[p][q] * mono[q];
                g[p] = a;
            }
            cplx b3[3] = {v[0][m], v[1][m], v[2][m]};
            green_mul3(b3, g, pd.ga, pd.gscale);
            v[0][m] = b3[0];
            v[1][m] = b3[1];
            v[2][m] = b3[2];
            __builtin_amdgcn_sched_barrier(0);   // one point at a time: bounded registers
        }
        __syncthreads();
    }
    if constexpr (MODE != AX_FWD) fft_run<N, P, true, NC>(v, tt, tw, lds);
    if (active) {
#pragma unroll
        for (int f = 0; f < NC; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) base[f * span + (size_t)(t + T * m) * S] = v[f][m];
    }
}

// Points per thread of the strided passes: radix-8 passes for 2^k, 12 for
// 3 * 2^k, 10 for 5 * 2^k.
int axis_points(int n) { return (n % 5 == 0) ? 10 : (n % 3 == 0) ? 12 : 8; }

#define FW_AXIS_SIZES(X) \
    X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256)

bool axis3_size_supported(int n) {
#define FW_IS(N) if (n == N) return true;
    FW_AXIS_SIZES(FW_IS)
#undef FW_IS
    return false;
}

template <int N, int MODE>
static hipError_t axis_launch(cplx* data, int S, int nslab, int slabs_per_sys, const SysState* st, const cplx* tw,
                              const ProbDev3& pd, hipStream_t s) {
    constexpr int P = (N % 5 == 0) ? 10 : (N % 3 == 0) ? 12 : 8;
    constexpr int T = N / P;
    constexpr int NC = MODE == AX_GREEN ? 3 : 1;
    int W = 16;
    while (W > 1 && (W * T > 256 || S % W != 0)) W /= 2;
    const int threads = ((W * T + 63) / 64) * 64;
    const size_t lds = (size_t)(NC * PaddedLen<N>::value * (W + 1)) * sizeof(cplx);
    hipError_t e = allow_lds(k_axis<N, P, MODE>, lds);
    if (e != hipSuccess) return e;
    const long long blocks = (long long)nslab * (S / W);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_axis<N, P, MODE>), dim3((unsigned)blocks), dim3(threads), lds, s, data, S, W,
                       slabs_per_sys, st, tw + twiddle_offset(N), pd);
    return hipGetLastError();
}

hipError_t launch_axis3(int mode, int n, cplx* data, int S, int nslab, int slabs_per_sys, const SysState* st,
                        const cplx* tw, const ProbDev3& pd, hipStream_t s) {
#define FW_AX(N)                                                                                             \
    if (n == N) {                                                                                            \
        if (mode == AX_FWD) return axis_launch<N, AX_FWD>(data, S, nslab, slabs_per_sys, st, tw, pd, s);     \
        if (mode == AX_INV) return axis_launch<N, AX_INV>(data, S, nslab, slabs_per_sys, st, tw, pd, s);     \
        if (mode == AX_GREEN) return axis_launch<N, AX_GREEN>(data, S, nslab, slabs_per_sys, st, tw, pd, s); \
    }
    FW_AXIS_SIZES(FW_AX)
#undef FW_AX
    return hipErrorInvalidValue;
}

// ---------------------------------------------------- sources, receivers --
// f must be zero on entry: one force per system, F / dx^3 at (ix, iy, iz).
__global__ void k_point_sources3(cplx* __restrict__ f, const int32_t* __restrict__ ixyz,
                                 const double* __restrict__ force, ProbDev3 pd) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= pd.nsys) return;
    const size_t cells = (size_t)pd.nx * pd.ny * pd.nz;
    const size_t g = ((size_t)ixyz[3 * sys + 2] * pd.ny + ixyz[3 * sys + 1]) * pd.nx + ixyz[3 * sys];
    const double inv = 1.0 / ((double)pd.dx * (double)pd.dx * (double)pd.dx);
#pragma unroll
    for (int c = 0; c < 3; ++c) f[(size_t)sys * 3 * cells + c * cells + g] = mkc((real)(force[3 * sys + c] * inv), 0.f);
}

hipError_t launch_point_sources3(cplx* f, const int32_t* src_ixyz, const double* src_f, const ProbDev3& pd,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_point_sources3, dim3((pd.nsys + 63) / 64), dim3(64), 0, s, f, src_ixyz, src_f, pd);
    return hipGetLastError();
}

// d[sys][rec][c] = w[sys][c][iz][iy][ix]
__global__ void k_gather3(const cplx* __restrict__ w, cplx* __restrict__ d, const int32_t* __restrict__ rec,
                          int nrec, ProbDev3 pd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pd.nsys * nrec * 3) return;
    const int c = i % 3, rr = (i / 3) % nrec, sys = i / (3 * nrec);
    const size_t cells = (size_t)pd.nx * pd.ny * pd.nz;
    const size_t g = ((size_t)rec[3 * rr + 2] * pd.ny + rec[3 * rr + 1]) * pd.nx + rec[3 * rr];
    d[i] = w[(size_t)sys * 3 * cells + c * cells + g];
}

hipError_t launch_gather3(const cplx* w, cplx* d, const int32_t* rec, int nrec, const ProbDev3& pd, hipStream_t s) {
    const int total = pd.nsys * nrec * 3;
    hipLaunchKernelGGL(k_gather3, dim3((total + 255) / 256), dim3(256), 0, s, w, d, rec, nrec, pd);
    return hipGetLastError();
}

// f (zero on entry) += conj(d) at the receivers; one thread per (sys, c) walks
// the receivers in order, so repeated receivers add deterministically.
__global__ void k_scatter_conj3(const cplx* __restrict__ d, cplx* __restrict__ f, const int32_t* __restrict__ rec,
                                int nrec, ProbDev3 pd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pd.nsys * 3) return;
    const int sys = i / 3, c = i % 3;
    const size_t cells = (size_t)pd.nx * pd.ny * pd.nz;
    cplx* fs = f + (size_t)sys * 3 * cells + c * cells;
    for (int r = 0; r < nrec; ++r) {
        const cplx dv = d[((size_t)sys * nrec + r) * 3 + c];
        const size_t g = ((size_t)rec[3 * r + 2] * pd.ny + rec[3 * r + 1]) * pd.nx + rec[3 * r];
        fs[g] = cadd(fs[g], cconj(dv));
    }
}

hipError_t launch_scatter_conj3(const cplx* d, cplx* f, const int32_t* rec, int nrec, const ProbDev3& pd,
                                hipStream_t s) {
    const int total = pd.nsys * 3;
    hipLaunchKernelGGL(k_scatter_conj3, dim3((total + 63) / 64), dim3(64), 0, s, d, f, rec, nrec, pd);
    return hipGetLastError();
}

// ------------------------------------------------------- correlation -----
// Per cell, summed over systems in FP64 (eq. ad1):
//   g_p   = -conj( sum_IJ e^a_I B^(p)_IJ e^b_J ) / (4 dx^2)   (raw differences e)
//   g_rho = conj( w~^2 sum_c u^a_c u^b_c ),
// for the VTI maps (C11, C13, C33, C55, C66) with App. C's B, or the 21
// constants with B^(IJ) = e_I e_J^T + e_J e_I^T (I != J), e_I e_I^T (I = J).
__device__ __forceinline__ void zacc(double& re, double& im, cplx a, cplx b, double w = 1.0) {
    re += w * ((double)a.x * b.x - (double)a.y * b.y);
    im += w * ((double)a.x * b.y + (double)a.y * b.x);
}

__device__ __forceinline__ void strain_raw3(const cplx* f, size_t cells, size_t c0, size_t xp, size_t xm, size_t yp,
                                            size_t ym, size_t zp, size_t zm, cplx (&e)[6]) {
    const cplx* ux = f;
    const cplx* uy = f + cells;
    const cplx* uz = f + 2 * cells;
    (void)c0;
    e[0] = csub(ux[xp], ux[xm]);
    e[1] = csub(uy[yp], uy[ym]);
    e[2] = csub(uz[zp], uz[zm]);
    e[3] = cadd(csub(uy[zp], uy[zm]), csub(uz[yp], uz[ym]));
    e[4] = cadd(csub(ux[zp], ux[zm]), csub(uz[xp], uz[xm]));
    e[5] = cadd(csub(ux[yp], ux[ym]), csub(uy[xp], uy[xm]));
}

template <bool GEN>
__global__ __launch_bounds__(256) void k_correlate3(const cplx* __restrict__ ua, const cplx* __restrict__ ub,
                                                    double2* __restrict__ g, ProbDev3 pd, int accumulate) {
    constexpr int NS = Params3<GEN>::NS;
    const int nx = pd.nx, ny = pd.ny, nz = pd.nz;
    const size_t cells = (size_t)nx * ny * nz;
    const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= cells) return;
    const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((size_t)nx * ny));
    auto at = [&](int xx, int yy, int zz) { return ((size_t)wrapm(zz, nz) * ny + wrapm(yy, ny)) * nx + wrapm(xx, nx); };
    const size_t xp = at(x + 1, y, z), xm = at(x - 1, y, z), yp = at(x, y + 1, z), ym = at(x, y - 1, z),
                 zp = at(x, y, z + 1), zm = at(x, y, z - 1);
    double acc[NS][2] = {};
    double rr = 0, ri = 0;
    for (int s = 0; s < pd.nsys; ++s) {
        const cplx* A = ua + (size_t)s * 3 * cells;
        const cplx* B = ub + (size_t)s * 3 * cells;
#pragma unroll
        for (int c = 0; c < 3; ++c) zacc(rr, ri, A[c * cells + cell], B[c * cells + cell]);
        cplx ea[6], eb[6];
        strain_raw3(A, cells, cell, xp, xm, yp, ym, zp, zm, ea);
        strain_raw3(B, cells, cell, xp, xm, yp, ym, zp, zm, eb);
        if constexpr (GEN) {
            int p = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = i; j < 6; ++j) {
                    zacc(acc[p][0], acc[p][1], ea[i], eb[j]);
                    if (i != j) zacc(acc[p][0], acc[p][1], ea[j], eb[i]);
                    ++p;
                }
        } else {
            const cplx sa = cadd(ea[0], ea[1]), sb = cadd(eb[0], eb[1]);
            zacc(acc[0][0], acc[0][1], sa, sb);                                  // B^11
            zacc(acc[1][0], acc[1][1], sa, eb[2]);                               // B^13
            zacc(acc[1][0], acc[1][1], ea[2], sb);
            zacc(acc[2][0], acc[2][1], ea[2], eb[2]);                            // B^33
            zacc(acc[3][0], acc[3][1], ea[3], eb[3]);                            // B^55
            zacc(acc[3][0], acc[3][1], ea[4], eb[4]);
            zacc(acc[4][0], acc[4][1], ea[5], eb[5]);                            // B^66
            zacc(acc[4][0], acc[4][1], ea[0], eb[1], -2.0);
            zacc(acc[4][0], acc[4][1], ea[1], eb[0], -2.0);
        }
    }
    const double sc = (double)pd.inv4dx2;
    const double wr = pd.w2.x, wi = pd.w2.y;
#pragma unroll
    for (int p = 0; p <= NS; ++p) {
        double2* dst = g + (size_t)p * cells + cell;
        double ore, oim;
        if (p < NS) {
            ore = -acc[p][0] * sc;     // -conj(a) / (4 dx^2)
            oim = acc[p][1] * sc;
        } else {
            ore = wr * rr - wi * ri;   // conj(w~^2 rho)
            oim = -(wr * ri + wi * rr);
        }
        double2 o = accumulate ? *dst : double2{0.0, 0.0};
        o.x += ore;
        o.y += oim;
        *dst = o;
    }
}

hipError_t launch_correlate3(const cplx* ua, const cplx* ub, double2* g, const ProbDev3& pd, bool accumulate,
                             hipStream_t s) {
    const size_t cells = (size_t)pd.nx * pd.ny * pd.nz;
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    if (pd.params == kParamsGeneral)
        hipLaunchKernelGGL(k_correlate3<true>, dim3(blocks), dim3(256), 0, s, ua, ub, g, pd, accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL(k_correlate3<false>, dim3(blocks), dim3(256), 0, s, ua, ub, g, pd, accumulate ? 1 : 0);
    return hipGetLastError();
}

FW_END
