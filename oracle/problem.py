"""One Lippmann-Schwinger problem: a periodic grid, a homogeneous background
(C0, rho0), one frequency and a contrast; its solves, the Frechet operator J
and its adjoint J*.

Paper passages:
  eqs. decom, Ewave0, u, u_2, A, axb  - the LS equation and its operator;
  eq. u0                              - the incident field;
  eqs. del, delu, u_3, du, dC, duB, F - the DBI linearisation and J;
  eqs. YM, F0, uYr, key, uY, uM0      - the matrix-free J via virtual sources;
  eqs. ad, ad1, ua, ua0, App. B       - the adjoint and its matrix-free form.

Readings (the paper is silent on these):
  * The heterogeneous reference model of the DBI step is the homogeneous
    background plus a reference contrast (eq. key); A_b is eq. A with that
    contrast.  The paper solves separate LS problems for u^(Y) and u^(M)
    (eq. uY); by linearity their weighted sum w^2 u^(Y) - u^(M) solves the
    same LS equation with the summed incident field, so one solve gives
    J dm = R A_b^-1 G0 conv P_b(dm) with the virtual source
        P_b(dm) = w~^2 dm_rho u^b + div_h( dC(dm) : E_h u^b ),
    where dC(dm) = sum_p B^(p) dm^(p) (eq. dC); the minus sign of eq. F0 is
    absorbed by the integration by parts (div_h = -E_h^T).
  * The adjoint follows eq. ad1: the back-propagated field solves the same
    LS equation with incident field G0 conv (R^T conj(r)) (eqs. ua, ua0,
    using the reciprocity G^b(x, r) = G^b(r, x)^T of App. B), and
        (J* r)_rho = conj( w~^2 u^a . u^b ),
        (J* r)_p   = -conj( E_h u^a . B^(p) E_h u^b ),
    summed over the systems (sources) of the problem.
  * Inner products are unweighted sums over cells, components, receivers
    and systems (the integrals of App. B up to a constant cell volume).
  * Model maps are absolute (Pa, kg/m^3) in the order (C11, C13, C33, C55, rho).
"""

import numpy as np

from . import green, krylov, media, operators


class LSProblem:
    """Background, frequency and reference contrast of one (grid, frequency)."""

    def __init__(self, nx, nz, dx, c0, rho0, freq_hz, eta=0.02, maps=None,
                 symbol="spectral"):
        self.nx, self.nz, self.dx = int(nx), int(nz), float(dx)
        self.c0 = tuple(float(c) for c in c0)        # (C11, C13, C33, C55)
        self.rho0 = float(rho0)
        self.freq_hz = float(freq_hz)
        self.eta = float(eta)
        self.omega_t = green.complex_frequency(self.freq_hz, self.eta)
        C11, C13, C33, C55 = self.c0
        self.C6 = media.voigt_2d(C11, C13, C33, C55)
        self.Ghat = green.green_symbol(self.C6, self.rho0, self.omega_t,
                                       self.nx, self.nz, self.dx, symbol)
        self.set_contrast(np.zeros((5, self.nz, self.nx)) if maps is None else maps)

    # ----- contrast -----------------------------------------------------
    def set_contrast(self, maps):
        maps = np.asarray(maps, dtype=float)
        assert maps.shape == (5, self.nz, self.nx)
        self.maps = maps
        self.dC6 = media.contrast_voigt_2d(*maps[:4])
        self.drho = maps[4]

    # ----- operators ----------------------------------------------------
    def body_force(self, u):
        return operators.body_force(u, self.dC6, self.drho, self.omega_t, self.dx)

    def convolve(self, f):
        return operators.convolve(self.Ghat, f)

    def apply(self, u):
        """A u = u - G0 conv b(u), eq. A."""
        return u - self.convolve(self.body_force(u))

    def incident(self, src_ixz, src_f):
        """u0 = G0 conv s for one point force per system, eq. u0."""
        s = operators.point_sources(len(src_ixz), self.nx, self.nz, self.dx,
                                    src_ixz, src_f)
        return self.convolve(s)

    def solve(self, rhs, tol=1e-10, maxit=10000):
        """Solve A u = rhs for every system (eq. axb); returns (u, [SolveInfo])."""
        rhs = np.asarray(rhs, dtype=complex)
        out = np.empty_like(rhs)
        infos = []
        for k in range(rhs.shape[0]):
            xk, info = krylov.bicgstab(lambda v: self.apply(v[None])[0], rhs[k],
                                       tol=tol, maxit=maxit)
            out[k] = xk
            infos.append(info)
        return out, infos

    # ----- Frechet operator and adjoint ---------------------------------
    def virtual_source(self, ub, dm):
        """P_b(dm) = w~^2 dm_rho u^b + div_h(dC(dm) : E_h u^b), eqs. YM / dC."""
        dm = np.asarray(dm)
        dC6 = media.contrast_voigt_2d(*dm[:4])
        return operators.body_force(ub, dC6, dm[4], self.omega_t, self.dx)

    def frechet_field(self, ub, dm, tol=1e-10):
        """The scattered field A_b^-1 G0 conv P_b(dm) for every system (eq. uY)."""
        w, _ = self.solve(self.convolve(self.virtual_source(ub, dm)), tol=tol)
        return w

    def frechet(self, ub, dm, rec_ixz, tol=1e-10):
        """J dm = R A_b^-1 G0 conv P_b(dm), [nsys, nrec, 2] (eqs. F0, uY)."""
        return operators.sample(self.frechet_field(ub, dm, tol), rec_ixz)

    def adjoint(self, ub, r, rec_ixz, tol=1e-10):
        """J* r as five complex maps [5, nz, nx] (eqs. ad1, ua, ua0)."""
        f = operators.sample_transpose(np.conj(r), rec_ixz, self.nx, self.nz)
        ua, _ = self.solve(self.convolve(f), tol=tol)
        return self.correlate(ua, ub)

    def correlate(self, ua, ub):
        """Sum over systems of the pointwise products of eq. ad1."""
        ea = operators.strain_voigt(ua, self.dx)
        eb = operators.strain_voigt(ub, self.dx)
        g = np.zeros((5, self.nz, self.nx), dtype=complex)
        for p, B in enumerate(media.map_B_matrices_2d()):
            prod = np.einsum("sIzx,IJ,sJzx->zx", ea, B, eb)
            g[p] = -np.conj(prod)
        g[4] = np.conj(self.omega_t ** 2 * np.einsum("sczx,sczx->zx", ua, ub))
        return g

    # ----- forward map used by the Jacobian pin ---------------------------
    def data(self, maps, u0, rec_ixz, tol=1e-12):
        """R A(maps)^-1 u0: the receiver data of the full forward problem."""
        saved = self.maps
        self.set_contrast(maps)
        try:
            u, _ = self.solve(u0, tol=tol)
        finally:
            self.set_contrast(saved)
        return operators.sample(u, rec_ixz)
