// Device helpers of the batched BiCGSTAB shared by the stencil kernels:
// FP64 complex arithmetic, the stopping test, and the per-system scalars of
// the vector updates fused into a stencil's input.
#pragma once

#include "launch.h"

FW_BEGIN
__device__ __forceinline__ dcomplex zdiv(dcomplex a, dcomplex b) {
    const double d = b.re * b.re + b.im * b.im;
    return dcomplex{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ dcomplex zmul(dcomplex a, dcomplex b) {
    return dcomplex{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx toc(dcomplex a) { return mkc((real)a.re, (real)a.im); }
__device__ __forceinline__ bool zzero(dcomplex a) { return a.re == 0.0 && a.im == 0.0; }

// Convergence / limit / finiteness test of the recursive residual; returns
// true if the system must stop.  Block 0 records the status.
__device__ __forceinline__ bool bicg_stop(SysState* st, int sys, double rr, bool writer) {
    const SysState& s = st[sys];
    int status = ST_RUNNING;
    if (!(rr == rr) || rr > 1e300) status = ST_NONFINITE;
    else if (rr <= s.tol2) status = ST_CONVERGED;
    else if (s.iter >= s.maxit) status = ST_MAXIT;
    if (status != ST_RUNNING && writer) {
        st[sys].status = status;
        st[sys].rnorm2 = rr;
    }
    return status != ST_RUNNING;
}


constexpr double kOmegaLimit = 0.7;

// From the t-pass records q = (<t,s>, ||t||^2, ||s||^2, <r^,s>, <r^,t>):
// omega = <t,s> / ||t||^2, enlarged when t and s are far from parallel
// (|<t,s>| < 0.7 |t| |s|; the finite-precision safeguard of Sleijpen and van
// der Vorst, 1995, which keeps the BiCG part from stalling), and for the next
// residual r = s - omega t its norm ||r||^2 = ||s||^2 - 2 Re(conj(omega)
// <t,s>) + |omega|^2 ||t||^2 and <r^, r> = <r^,s> - omega <r^,t>.
struct OmegaStep {
    dcomplex omega;
    double rr;
    dcomplex rho;
};
__device__ __forceinline__ OmegaStep omega_step(const double (&q)[kPartialNV]) {
    OmegaStep o;
    o.omega = dcomplex{0.0, 0.0};
    if (q[2] != 0.0) {
        o.omega = dcomplex{q[0] / q[2], q[1] / q[2]};
        const double ts = sqrt(q[0] * q[0] + q[1] * q[1]);
        // |t| |s| as a product of roots: the product of the squares can
        // underflow for tiny fields
        const double c = (q[3] > 0.0) ? ts / (sqrt(q[2]) * sqrt(q[3])) : 1.0;
        if (c < kOmegaLimit && c > 0.0) {
            o.omega.re *= kOmegaLimit / c;
            o.omega.im *= kOmegaLimit / c;
        }
    }
    const double wr = o.omega.re, wi = o.omega.im;
    const double rr = q[3] - 2.0 * (wr * q[0] + wi * q[1]) + (wr * wr + wi * wi) * q[2];
    o.rr = rr > 0.0 ? rr : 0.0;
    o.rho = dcomplex{q[4] - (wr * q[6] - wi * q[7]), q[5] - (wr * q[7] + wi * q[6])};
    return o;
}

// Whether a block of a launch that closes iterations (tag kStampPx or
// kStampClose) has work for a system with status word s: the system runs, or
// another block of this very launch stopped it with its last solution update
// still owed.
__device__ __forceinline__ bool closing_enters(int s, int tag) {
    if (s == ST_RUNNING) return true;
    const int c = st_code(s);
    return (c == ST_CONVERGED || c == ST_MAXIT) && st_tag(s) == tag;
}

// The stop decision at the end of an iteration, from the t-pass records:
// non-finite, converged (||r||^2 <= tol2) or out of iterations; ST_RUNNING
// otherwise.
__device__ __forceinline__ int close_code(const SysState& z, const OmegaStep& o) {
    if (!(o.rr == o.rr) || o.rr > 1e300 || !(o.omega.re == o.omega.re) || !(o.omega.im == o.omega.im))
        return ST_NONFINITE;
    if (o.rr <= z.tol2) return ST_CONVERGED;
    if (z.iter >= z.maxit) return ST_MAXIT;
    return ST_RUNNING;
}

// The closing updates of an iteration on one element: r = s - omega t and
// x + alpha p + omega s.  Contraction is off so that every kernel that closes
// an iteration (stencils, close kernel) rounds it identically.
__device__ __forceinline__ cplx close_r(cplx sv, cplx tv, cplx omega) {
#pragma clang fp contract(off)
    return mkc(sv.x - (omega.x * tv.x - omega.y * tv.y), sv.y - (omega.x * tv.y + omega.y * tv.x));
}
__device__ __forceinline__ cplx close_x(cplx xv, cplx pv, cplx sv, cplx alpha, cplx omega) {
#pragma clang fp contract(off)
    const real ax = alpha.x * pv.x - alpha.y * pv.y, ay = alpha.x * pv.y + alpha.y * pv.x;
    const real wx = omega.x * sv.x - omega.y * sv.y, wy = omega.x * sv.y + omega.y * sv.x;
    return mkc(xv.x + (ax + wx), xv.y + (ay + wy));
}

enum StencilStep : int { SS_SKIP = 0, SS_FULL = 1, SS_XONLY = 2 };

// Scalars of the update of system sys from its producer's partial records
// (summed by every block in the same order).  VM_P -> c1 = beta, c2 = omega,
// and `fresh` when the recurrence restarts from the current iterate (r^ = r,
// p = r): scheduled after a stagnation, or forced by a zero scalar that would
// otherwise break the iteration down.  VM_S -> c1 = alpha.  VM_PX -> c1 =
// beta, c2 = omega, c3 = alpha; the stopping test is on the residual r = s -
// omega t, and a stopped system still receives its solution update
// (SS_XONLY).  Returns SS_SKIP if the system stops (converged, limit,
// breakdown) with nothing left to do; `writer` (one thread of one block per
// system) records scalars and status.  Every thread of the block (NT threads)
// must call it (block reduction); the totals do not depend on NT.
template <int VM, int NT = 256>
__device__ __forceinline__ int stencil_scalars(SysState* st, int sys, const double* part, int np, double* red,
                                               bool writer, cplx& c1, cplx& c2, cplx& c3, bool& fresh) {
    const SysState& z = st[sys];
    const int it = z.iter + 1;
    if constexpr (VM == VM_PX) {
        double q[kPartialNV];
        sum_partials<kPartialNV, NT, kPartialNV, 256>(part + (size_t)sys * np * kPartialNV, np, q, red);
        const OmegaStep o = omega_step(q);
        const dcomplex alpha{z.alpha_re, z.alpha_im};
        c2 = toc(o.omega);
        c3 = toc(alpha);
        const int code = close_code(z, o);
        if (code != ST_RUNNING) {
            if (writer) {
                st[sys].status = st_stamp(code, kStampPx);
                st[sys].omega_re = o.omega.re;
                st[sys].omega_im = o.omega.im;
                st[sys].rnorm2 = o.rr;
            }
            return code == ST_NONFINITE ? SS_SKIP : SS_XONLY;
        }
        dcomplex rho_i = o.rho;
        const dcomplex rho_prev{z.rho_re[(it - 1) & 1], z.rho_im[(it - 1) & 1]};
        fresh = (z.fresh_at == it) || zzero(rho_i) || zzero(rho_prev) || zzero(o.omega);
        if (fresh) {
            rho_i = dcomplex{o.rr, 0.0};   // <r, r>
            c1 = mkc(0.f, 0.f);
        } else {
            const dcomplex beta = zmul(zdiv(rho_i, rho_prev), zdiv(alpha, o.omega));
            c1 = mkc((real)beta.re, (real)beta.im);
        }
        if (writer) {
            st[sys].rho_re[it & 1] = rho_i.re;
            st[sys].rho_im[it & 1] = rho_i.im;
            st[sys].omega_re = o.omega.re;
            st[sys].omega_im = o.omega.im;
            st[sys].rnorm2 = o.rr;
        }
        return SS_FULL;
    } else {
        double q[4];
        sum_partials<4, NT, kPartialNV, 256>(part + (size_t)sys * np * kPartialNV, np, q, red);
        if constexpr (VM == VM_P) {
            if (bicg_stop(st, sys, q[2], writer)) return SS_SKIP;
            dcomplex rho_i{q[0], q[1]};
            const dcomplex rho_prev{z.rho_re[(it - 1) & 1], z.rho_im[(it - 1) & 1]};
            const dcomplex alpha{z.alpha_re, z.alpha_im}, omega{z.omega_re, z.omega_im};
            fresh = (z.fresh_at == it) || zzero(rho_i) || zzero(rho_prev) || zzero(omega);
            if (fresh) {
                rho_i = dcomplex{q[2], 0.0};   // <r, r>
                c1 = mkc(0.f, 0.f);
            } else {
                const dcomplex beta = zmul(zdiv(rho_i, rho_prev), zdiv(alpha, omega));
                c1 = mkc((real)beta.re, (real)beta.im);
            }
            c2 = mkc((real)omega.re, (real)omega.im);
            if (writer) {
                st[sys].rho_re[it & 1] = rho_i.re;
                st[sys].rho_im[it & 1] = rho_i.im;
            }
        } else {
            const dcomplex rho_i{z.rho_re[it & 1], z.rho_im[it & 1]};
            const dcomplex rv{q[0], q[1]};
            if (zzero(rv)) {
                if (writer) st[sys].status = ST_BREAKDOWN;
                return SS_SKIP;
            }
            const dcomplex alpha = zdiv(rho_i, rv);
            c1 = mkc((real)alpha.re, (real)alpha.im);
            if (writer) {
                st[sys].alpha_re = alpha.re;
                st[sys].alpha_im = alpha.im;
            }
        }
        return SS_FULL;
    }
}

FW_END