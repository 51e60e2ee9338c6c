// Device helpers of the batched BiCGSTAB shared by the stencil kernels:
// FP64 complex arithmetic, the stopping test, and the per-system scalars of
// the vector updates fused into a stencil's input.
#pragma once

#include "launch.h"

namespace fw {

__device__ __forceinline__ dcomplex zdiv(dcomplex a, dcomplex b) {
    const double d = b.re * b.re + b.im * b.im;
    return dcomplex{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ dcomplex zmul(dcomplex a, dcomplex b) {
    return dcomplex{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ float2 tof(dcomplex a) { return make_float2((float)a.re, (float)a.im); }
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

// Vector update fused into a stencil's load of its input field:
//   VM_NONE: the input is u itself;
//   VM_P:    p = r + beta (p_old - omega v)   (BiCGSTAB direction update)
//   VM_S:    s = r - alpha v                  (BiCGSTAB intermediate residual)
enum StencilVec : int { VM_NONE = 0, VM_P = 1, VM_S = 2 };

// Scalars of the update of system sys from its producer's partial records
// (summed by every block in the same order): VM_P -> c1 = beta, c2 = omega,
// and `fresh` when the recurrence restarts from the current iterate (r^ = r,
// p = r): scheduled after a stagnation, or forced by a zero scalar that would
// otherwise break the iteration down.  VM_S -> c1 = alpha.  Returns false if
// the system stops (converged, limit, breakdown); `writer` (one thread of one
// block per system) records scalars and status.  Every thread of the block
// must call it (block reduction).
template <int VM>
__device__ __forceinline__ bool stencil_scalars(SysState* st, int sys, const double* part, int np, double* red,
                                                bool writer, float2& c1, float2& c2, bool& fresh) {
    double q[4];
    sum_partials<4, 256>(part + (size_t)sys * np * kPartialNV, np, q, red);
    const SysState& z = st[sys];
    const int it = z.iter + 1;
    if constexpr (VM == VM_P) {
        if (bicg_stop(st, sys, q[2], writer)) return false;
        dcomplex rho_i{q[0], q[1]};
        const dcomplex rho_prev{z.rho_re[(it - 1) & 1], z.rho_im[(it - 1) & 1]};
        const dcomplex alpha{z.alpha_re, z.alpha_im}, omega{z.omega_re, z.omega_im};
        fresh = (z.fresh_at == it) || zzero(rho_i) || zzero(rho_prev) || zzero(omega);
        if (fresh) {
            rho_i = dcomplex{q[2], 0.0};   // <r, r>
            c1 = make_float2(0.f, 0.f);
        } else {
            const dcomplex beta = zmul(zdiv(rho_i, rho_prev), zdiv(alpha, omega));
            c1 = make_float2((float)beta.re, (float)beta.im);
        }
        c2 = make_float2((float)omega.re, (float)omega.im);
        if (writer) {
            st[sys].rho_re[it & 1] = rho_i.re;
            st[sys].rho_im[it & 1] = rho_i.im;
        }
    } else {
        const dcomplex rho_i{z.rho_re[it & 1], z.rho_im[it & 1]};
        const dcomplex rv{q[0], q[1]};
        if (zzero(rv)) {
            if (writer) st[sys].status = ST_BREAKDOWN;
            return false;
        }
        const dcomplex alpha = zdiv(rho_i, rv);
        c1 = make_float2((float)alpha.re, (float)alpha.im);
        if (writer) {
            st[sys].alpha_re = alpha.re;
            st[sys].alpha_im = alpha.im;
        }
    }
    return true;
}

}  // namespace fw
