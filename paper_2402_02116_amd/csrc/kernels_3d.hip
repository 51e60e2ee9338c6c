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
            st_wt(rout + so + gi, rv);
            st_wt(xio + so + gi, close_x(xio[so + gi], pv, sv, c3, c2));
            if (fresh) st_wt(rhat + so + gi, rv);
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
                        st_wt(wout + so + gi, f);
                        if constexpr (VM == VM_P) {
                            if (fresh) st_wt(rhat + so + gi, f);   // p = r here
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
            st_wt(b + g, cadd(cmul(wr, su[h]), cscale(bx, sc)));
            st_wt(b + g + cells, cadd(cmul(wr, su[T::HC + h]), cscale(by, sc)));
            st_wt(b + g + 2 * cells, cadd(cmul(wr, su[2 * T::HC + h]), cscale(bz, sc)));
        }
    }
}

// The same stencil (plain: b of the input u) marching along z: a block owns
// a TX x TY column of cells over the z range [z0, z1) of one system and walks
// it plane by plane.  Each thread owns one cell of the column (p0) and, for
// the first RING threads, one cell of the 2-cell xy halo ring around it (p1),
// and keeps the input of planes z, z+1, z+2 at those cells in registers.  LDS
// holds only plane z+1 of the input (for the x and y differences) and the
// stress s' of plane z with a 1-cell halo.  Step z: the stress of plane z+1
// at the own and inner ring cells (z differences from registers), then b on
// plane z (the z difference of the own column's stress from registers), then
// plane z+2 and the new stress replace the LDS planes; the next two planes
// are loads in flight meanwhile.  Every input plane of the range is read
// once, plus three halo planes and the own column of a fourth per range.
// The BiCGSTAB update modes run as a streaming pass before it
// (launch_bicg_update): fused into this kernel they held one or two waves
// per SIMD.
template <int TX, int TY>
struct March3 {
    static constexpr int HX = TX + 4, HY = TY + 4, HP = HX * HY;   // input plane with halo 2
    static constexpr int SX = TX + 2, SY = TY + 2, SP = SX * SY;   // stress plane with halo 1
    static constexpr int NT = TX * TY;                             // one thread per own cell
    static constexpr int RING = HP - NT;                           // halo cells of an input plane
};

template <int TX, int TY>
inline size_t march3_lds() {
    using M = March3<TX, TY>;
    return (size_t)(3 * M::HP + 6 * M::SP) * sizeof(cplx);
}

// Halo-ring cell k of a (TX+4) x (TY+4) plane: the two rows above, the two
// rows below, then the two columns left and right of the own rows.
template <int TX, int TY>
__device__ __forceinline__ void ring_cell(int k, int& hx, int& hy) {
    constexpr int HX = TX + 4;
    if (k < 2 * HX) {
        hy = k / HX;
        hx = k % HX;
    } else if (k < 4 * HX) {
        k -= 2 * HX;
        hy = TY + 2 + k / HX;
        hx = k % HX;
    } else if (k < 4 * HX + 2 * TY) {
        k -= 4 * HX;
        hy = 2 + k / 2;
        hx = k % 2;
    } else {
        k -= 4 * HX + 2 * TY;
        hy = 2 + k / 2;
        hx = TX + 2 + k % 2;
    }
}

template <bool GEN, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_stencil3z(const cplx* __restrict__ u, cplx* __restrict__ b,
                                                       const real* __restrict__ maps, ProbDev3 pd, int ZC,
                                                       const SysState* __restrict__ st) {
    using M = March3<TX, TY>;
    static_assert(M::RING <= M::NT, "one halo-ring cell per thread at most");
    constexpr int NS = Params3<GEN>::NS;
    extern __shared__ __align__(16) unsigned char lds3[];
    cplx* sp = reinterpret_cast<cplx*>(lds3);   // input plane [3][HP]
    cplx* ss = sp + 3 * M::HP;                  // stress plane [6][SP]
    __shared__ int s_status;

    const int nx = pd.nx, ny = pd.ny, nz = pd.nz;
    const size_t cells = (size_t)nx * ny * nz;
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    // neighbouring blocks (on one XCD, resident together): the neighbouring
    // columns and z ranges of the same system, which read each other's cells
    // as their halos while those cache lines are still in the XCD's L2
    const int ncol = ntx * nty * ((nz + ZC - 1) / ZC);
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int sys = blk / ncol;
    const int col = blk - sys * ncol;
    const int x0 = (col % ntx) * TX, y0 = ((col / ntx) % nty) * TY, z0 = (col / (ntx * nty)) * ZC;
    const int z1 = min(z0 + ZC, nz);
    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    const bool own_xy = x0 + tx < nx && y0 + ty < ny;

    if (st != nullptr) {
        if (t == 0) s_status = st[sys].status;
        __syncthreads();
        if (s_status != ST_RUNNING) return;
    }
    // this system's vectors; offsets within a system fit 32 bits (3 x 256^3)
    const size_t so = (size_t)sys * 3 * cells;
    const cplx* __restrict__ us = u + so;
    cplx* __restrict__ bs = b + so;
    const uint32_t cells32 = (uint32_t)cells, plane32 = (uint32_t)nx * (uint32_t)ny;
    // planes z0-2 .. z1+3 lie within one period of the axis
    auto zoff = [&](int z) -> uint32_t { return (uint32_t)(z < 0 ? z + nz : (z >= nz ? z - nz : z)) * plane32; };
    const uint32_t xy0 = (uint32_t)wrapm(y0 + ty, ny) * nx + wrapm(x0 + tx, nx);

    // the thread's halo-ring cell
    const bool has1 = t < M::RING;
    int hx1 = 2, hy1 = 2;
    if (has1) ring_cell<TX, TY>(t, hx1, hy1);
    const bool st1 = has1 && hx1 >= 1 && hx1 <= TX + 2 && hy1 >= 1 && hy1 <= TY + 2;   // inner ring: stress
    const uint32_t xy1 = (uint32_t)wrapm(y0 - 2 + hy1, ny) * nx + wrapm(x0 - 2 + hx1, nx);
    const int h0 = (ty + 2) * M::HX + tx + 2, h1 = hy1 * M::HX + hx1;
    const int q0 = (ty + 1) * M::SX + tx + 1, q1 = (hy1 - 1) * M::SX + hx1 - 1;

    using Raw = cplx[3];
    auto load_raw = [&](Raw& r, uint32_t g) {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = us[c * cells32 + g];
    };
    auto convert = [&](const Raw& r, cplx (&f)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = r[c];
    };
    auto load_maps = [&](real (&m)[NS], uint32_t g) {
#pragma unroll
        for (int p = 0; p < NS; ++p) m[p] = maps[p * cells32 + g];
    };
    // s' = dC e' at LDS input position h of the current plane; z differences
    // from the planes below (lo) and above (hi)
    auto stress_at = [&](int h, const cplx (&lo)[3], const cplx (&hi)[3], const real (&m)[NS], cplx (&sg)[6]) {
        cplx d[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cplx* w = sp + c * M::HP + h;
            d[c][0] = csub(w[1], w[-1]);
            d[c][1] = csub(w[M::HX], w[-M::HX]);
            d[c][2] = csub(hi[c], lo[c]);
        }
        const cplx e[6] = {d[0][0], d[1][1], d[2][2], cadd(d[1][2], d[2][1]), cadd(d[0][2], d[2][0]),
                           cadd(d[0][1], d[1][0])};
        stress3<GEN>(m, 1, e, sg);
    };
    auto put_plane = [&](const cplx (&f0)[3], const cplx (&f1)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sp[c * M::HP + h0] = f0[c];
            if (has1) sp[c * M::HP + h1] = f1[c];
        }
    };

    // ---- prologue: planes z0-2 (own column), z0-1, z0, z0+1, z0+2
    cplx fa0[3], fa1[3], fb0[3], fb1[3], fc0[3], fc1[3];
    cplx sold[6];
    {
        Raw r0, r1;
        cplx fm2[3], fm0[3], fm1[3];
        load_raw(r0, zoff(z0 - 2) + xy0);
        convert(r0, fm2);
        load_raw(r0, zoff(z0 - 1) + xy0);
        convert(r0, fm0);
        if (has1) {
            load_raw(r1, zoff(z0 - 1) + xy1);
            convert(r1, fm1);
        }
        load_raw(r0, zoff(z0) + xy0);
        convert(r0, fa0);
        if (has1) {
            load_raw(r1, zoff(z0) + xy1);
            convert(r1, fa1);
        }
        put_plane(fm0, fm1);
        real m[NS];
        load_maps(m, zoff(z0 - 1) + xy0);
        __syncthreads();
        stress_at(h0, fm2, fa0, m, sold);   // own stress of plane z0-1
        load_raw(r0, zoff(z0 + 1) + xy0);
        convert(r0, fb0);
        if (has1) {
            load_raw(r1, zoff(z0 + 1) + xy1);
            convert(r1, fb1);
        }
        __syncthreads();
        put_plane(fa0, fa1);
        __syncthreads();
        cplx sg[6];
        load_maps(m, zoff(z0) + xy0);
        stress_at(h0, fm0, fb0, m, sg);   // stress of plane z0
#pragma unroll
        for (int i = 0; i < 6; ++i) ss[i * M::SP + q0] = sg[i];
        if (st1) {
            load_maps(m, zoff(z0) + xy1);
            stress_at(h1, fm1, fb1, m, sg);
#pragma unroll
            for (int i = 0; i < 6; ++i) ss[i * M::SP + q1] = sg[i];
        }
        load_raw(r0, zoff(z0 + 2) + xy0);
        convert(r0, fc0);
        if (has1) {
            load_raw(r1, zoff(z0 + 2) + xy1);
            convert(r1, fc1);
        }
        __syncthreads();
        put_plane(fb0, fb1);
    }
    // in flight during a step: planes z+3 and z+4 (two buffers, used in
    // turn: the loop is unrolled by two so that no register of a load in
    // flight is moved) and the maps of plane z+2
    Raw rA0, rA1, rB0, rB1;
    load_raw(rA0, zoff(z0 + 3) + xy0);
    if (has1) load_raw(rA1, zoff(z0 + 3) + xy1);
    load_raw(rB0, zoff(z0 + 4) + xy0);
    if (has1) load_raw(rB1, zoff(z0 + 4) + xy1);
    // stiffness maps of plane z+1 (and, prefetched, z+2); the 21-constant
    // form loads them at the step instead (registers)
    constexpr int NPF = GEN ? 1 : NS;
    real mc0[NS], mc1[NS], mn0[NPF], mn1[NPF];
    if constexpr (!GEN) {
        load_maps(mc0, zoff(z0 + 1) + xy0);
        if (st1) load_maps(mc1, zoff(z0 + 1) + xy1);
        load_maps(mn0, zoff(z0 + 2) + xy0);
        if (st1) load_maps(mn1, zoff(z0 + 2) + xy1);
    }
    const real* rho = maps + (size_t)NS * cells;   // (uint32 offsets below)
    real rho_z = rho[zoff(z0) + xy0], rho_1 = rho[zoff(z0 + 1) + xy0], rho_2 = rho[zoff(z0 + 2) + xy0];
    __syncthreads();

    const real sc = pd.inv4dx2;
    // step z: b on plane z; rd holds plane z+3 and is refilled with z+5
    auto plane_step = [&](int z, Raw& rd0, Raw& rd1) {
        // stress of plane z+1 at the own and inner-ring cells
        cplx s0[6], s1[6];
        if constexpr (GEN) {
            load_maps(mc0, zoff(z + 1) + xy0);
            if (st1) load_maps(mc1, zoff(z + 1) + xy1);
        }
        stress_at(h0, fa0, fc0, mc0, s0);
        if (st1) stress_at(h1, fa1, fc1, mc1, s1);
        // b on plane z at the own cell
        if (own_xy) {
            auto dxy = [&](int i, int off) { return csub(ss[i * M::SP + q0 + off], ss[i * M::SP + q0 - off]); };
            const cplx bx = cadd(cadd(dxy(0, 1), dxy(5, M::SX)), csub(s0[4], sold[4]));
            const cplx by = cadd(cadd(dxy(5, 1), dxy(1, M::SX)), csub(s0[3], sold[3]));
            const cplx bz = cadd(cadd(dxy(4, 1), dxy(3, M::SX)), csub(s0[2], sold[2]));
            const uint32_t g = zoff(z) + xy0;
            const cplx wr = cscale(pd.w2, rho_z);
            st_wt(bs + g, cadd(cmul(wr, fa0[0]), cscale(bx, sc)));
            st_wt(bs + g + cells32, cadd(cmul(wr, fa0[1]), cscale(by, sc)));
            st_wt(bs + g + 2 * cells32, cadd(cmul(wr, fa0[2]), cscale(bz, sc)));
        }
        __syncthreads();   // the LDS planes z+1 (input) and z (stress) are read
#pragma unroll
        for (int i = 0; i < 6; ++i) {   // own stress of plane z for the next z difference
            sold[i] = ss[i * M::SP + q0];
            ss[i * M::SP + q0] = s0[i];
            if (st1) ss[i * M::SP + q1] = s1[i];
        }
        put_plane(fc0, fc1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            fa0[c] = fb0[c];
            fb0[c] = fc0[c];
            fa1[c] = fb1[c];
            fb1[c] = fc1[c];
        }
        convert(rd0, fc0);
        if (has1) convert(rd1, fc1);
        if constexpr (!GEN) {
#pragma unroll
            for (int p = 0; p < NS; ++p) {
                mc0[p] = mn0[p];
                mc1[p] = mn1[p];
            }
        }
        rho_z = rho_1;
        rho_1 = rho_2;
        if (z + 5 <= z1 + 1) {
            load_raw(rd0, zoff(z + 5) + xy0);
            if (has1) load_raw(rd1, zoff(z + 5) + xy1);
        }
        if (z + 3 <= z1) {
            if constexpr (!GEN) {
                load_maps(mn0, zoff(z + 3) + xy0);
                if (st1) load_maps(mn1, zoff(z + 3) + xy1);
            }
            rho_2 = rho[zoff(z + 3) + xy0];
        }
        __syncthreads();
    };
    int z = z0;
    for (; z + 1 < z1; z += 2) {
        plane_step(z, rA0, rA1);
        plane_step(z + 1, rB0, rB1);
    }
    if (z < z1) plane_step(z, rA0, rA1);
}

template <bool GEN, int TX, int TY>
static hipError_t stencil3z_launch(const StencilArgs& a, const ProbDev3& pd, const SysState* st, hipStream_t s) {
    const int ntx = (pd.nx + TX - 1) / TX, nty = (pd.ny + TY - 1) / TY;
    // z ranges of at most 32 planes, more of them while the launch is small
    int ZC = std::min(pd.nz, 32);
    while (ZC > 8 && (long long)ntx * nty * ((pd.nz + ZC - 1) / ZC) * pd.nsys < 1024) ZC /= 2;
    const long long blocks = (long long)ntx * nty * ((pd.nz + ZC - 1) / ZC) * pd.nsys;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = march3_lds<TX, TY>();
    hipError_t e = allow_lds(k_stencil3z<GEN, TX, TY>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stencil3z<GEN, TX, TY>), dim3((unsigned)blocks), dim3(TX * TY), lds, s, a.u, a.b, a.maps,
                       pd, ZC, st);
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
// in y, which take the tiled kernel.  (A 16 x 20 column, which loads a fifth
// fewer cells per plane at 80 x 40, was slower: five waves per block pack
// worse than four.)
static int march_shape(int nx, int ny) {
    if (ny < 8 || nx < 16) return 0;
    const long long a = (long long)((nx + 15) / 16) * 16 * ((ny + 15) / 16) * 16;
    const long long b = (long long)((nx + 31) / 32) * 32 * ((ny + 7) / 8) * 8;
    return a <= b ? 16 : 32;
}

template <int VM, bool GEN>
static hipError_t stencil3_any(const StencilArgs& a, const ProbDev3& pd, SysState* st, hipStream_t s) {
    const int m = march_shape(pd.nx, pd.ny);
    if (m == 0) return stencil3_launch<VM, GEN>(a, pd, st, s);   // the tiled kernel, update fused
    StencilArgs p = a;
    if constexpr (VM != VM_NONE) {
        // the vector update as its own streaming pass, then the plain
        // z-marching stencil on the updated input (the marching kernel with
        // the update fused held one or two waves per SIMD: 206 against
        // 217 ms for the 80 x 40 x 32 x 100-system step)
        hipError_t e = launch_bicg_update(VM, a, 3LL * pd.nx * pd.ny * pd.nz, pd.nsys, st, s);
        if (e != hipSuccess) return e;
        p.u = a.wout;
    }
    return m == 16 ? stencil3z_launch<GEN, 16, 16>(p, pd, st, s) : stencil3z_launch<GEN, 32, 8>(p, pd, st, s);
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
    __device__ __forceinline__ cplx& operator()(int f, int pos) const { return padded(f, lds_pad(pos)); }
    __device__ __forceinline__ cplx& padded(int f, int pp) const { return base[(f * PL + pp) * stride]; }
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
    const real s = gscale * green_rcp(det.x * det.x + det.y * det.y);
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
            for (int m = 0; m < P; ++m) st_wt(base + f * span + (size_t)(t + T * m) * S, v[f][m]);
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
// f += R^T conj(d) with the receivers in the host's stable cell order (perm,
// run lengths glen): one thread per (system, run, component), each run
// summed in receiver order.
__global__ void k_scatter_conj3(const cplx* __restrict__ d, cplx* __restrict__ f, const int32_t* __restrict__ rec,
                                const int32_t* __restrict__ perm, const int32_t* __restrict__ glen, int nrec,
                                ProbDev3 pd) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)pd.nsys * nrec * 3) return;
    const int c = (int)(i % 3);
    const size_t q = i / 3;
    const int k = (int)(q % nrec), sys = (int)(q / nrec);
    const int n = glen[k];
    if (n == 0) return;
    const cplx* ds = d + (size_t)sys * nrec * 3 + c;
    const int r0 = perm[k];
    cplx acc = cconj(ds[3 * (size_t)r0]);
    for (int j = 1; j < n; ++j) acc = cadd(acc, cconj(ds[3 * (size_t)perm[k + j]]));
    const size_t cells = (size_t)pd.nx * pd.ny * pd.nz;
    cplx* fs = f + (size_t)sys * 3 * cells + c * cells;
    const size_t g = ((size_t)rec[3 * r0 + 2] * pd.ny + rec[3 * r0 + 1]) * pd.nx + rec[3 * r0];
    fs[g] = cadd(fs[g], acc);
}

hipError_t launch_scatter_conj3(const cplx* d, cplx* f, const int32_t* rec, const int32_t* perm,
                                const int32_t* glen, int nrec, const ProbDev3& pd, hipStream_t s) {
    const size_t total = (size_t)pd.nsys * nrec * 3;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_conj3, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d, f, rec, perm, glen,
                       nrec, pd);
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
