"""Three-dimensional, generally anisotropic form of the same method: media,
Green's symbol, finite-difference operators and one LS problem with its
solves, Frechet operator and adjoint.

TEST INFRASTRUCTURE (see the package docstring): plain numpy / scipy in
complex128, written from the paper; the HIP path shares nothing with it.

Paper passages:
  * the integral equation of the forward problem with all 21 elastic
    parameters and the density (Introduction, eqs. decom, u, u_2, A, axb);
  * eq. dC, delta C = sum_p B^(p) delta m^(p) over the 21 independent
    stiffness constants, with delta m^(0) = delta rho;
  * the abbreviated subscript section: the 6x6 stiffness matrix, the
    6-component engineering strain (d1u1, d2u2, d3u3, d2u3 + d3u2,
    d1u3 + d3u1, d1u2 + d2u1), the VTI matrix with C12 = C11 - 2 C66;
  * App. C: the VTI B matrices, B^66 with its -2 entries from C12;
  * App. A: the analytic 3-D isotropic Green's tensor (a loose pin only);
  * the modified 3-D VTI Hess example (six parameters C11, C33, C55, C66,
    C13, rho on an 80 x 40 x 32 grid of 25 m cells).

Conventions (0-based).  Tensor indices x = 0, y = 1, z = 2; Voigt indices
0..5 = (xx, yy, zz, yz, xz, xy).  Grids are [nz, ny, nx] with x fastest,
periodic in every direction, cell size dx on all three axes.  Fields are
[..., 3, nz, ny, nx] with components (u_x, u_y, u_z).

Readings (the paper is silent on these; the 2-D readings carry over):
  * G0 is the wavenumber-domain inverse of the damped 3x3 Christoffel
    matrix, G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1 with
    Gamma_ik = C_ijkl k_j k_l from the general 4-index tensor of a general
    (triclinic) background; products of two DIFFERENT wavenumber components
    take 0 at the Nyquist index of an even axis, squares keep (n/2)^2, so
    that G_hat stays even in k and G0 symmetric;
  * 2nd-order central differences, div_h = -E_h^T (exact summation by parts
    on the torus), as in 2-D;
  * parametrisations of the contrast:
      'general': the 21 constants of the upper triangle of the 6x6 matrix in
                 row-major order (C11, C12, ..., C16, C22, ..., C66), then
                 rho; B^(IJ) = e_I e_J^T + e_J e_I^T for I != J and e_I e_I^T
                 for I = J (the position of the constant in the symmetric
                 matrix, eq. dC);
      'vti':     (C11, C13, C33, C55, C66, rho) with the App. C matrices
                 (the order of the 2-D maps, C66 added before rho);
  * a point force F at cell (ix, iy, iz) is F / dx^3 at that cell.
"""

import numpy as np
import scipy.fft
import scipy.special

from . import krylov
from .media import VOIGT_INDEX, vti_B_matrices, voigt_to_tensor
from .operators import _WORKERS

#: Voigt pairs (I, J), I <= J, of the 21 independent constants, in order.
GENERAL_PAIRS = [(i, j) for i in range(6) for j in range(i, 6)]
GENERAL_NAMES = tuple(f"C{i + 1}{j + 1}" for i, j in GENERAL_PAIRS) + ("rho",)
VTI_NAMES = ("C11", "C13", "C33", "C55", "C66", "rho")
PARAM_NAMES = {"general": GENERAL_NAMES, "vti": VTI_NAMES}


# ------------------------------------------------------------------ media --
def voigt_from_21(c21):
    """Symmetric 6x6 Voigt matrix from the 21 constants in GENERAL_PAIRS order."""
    c21 = np.asarray(c21)
    C = np.zeros((6, 6) + c21.shape[1:], dtype=np.result_type(c21, 1.0))
    for p, (i, j) in enumerate(GENERAL_PAIRS):
        C[i, j] = c21[p]
        C[j, i] = c21[p]
    return C


def voigt_to_21(C6):
    """The 21 upper-triangle constants of a symmetric 6x6 matrix."""
    C6 = np.asarray(C6)
    return np.array([C6[i, j] for i, j in GENERAL_PAIRS])


def general_B_matrices():
    """The 21 constant B matrices of eq. dC for a general stiffness.

    B^(IJ) marks where the constant C_IJ sits in the symmetric 6x6 matrix:
    both (I, J) and (J, I) for an off-diagonal constant.
    """
    out = []
    for i, j in GENERAL_PAIRS:
        B = np.zeros((6, 6))
        B[i, j] = 1.0
        B[j, i] = 1.0
        out.append(B)
    return out


def vti_B_list():
    """App. C's B matrices in the order of the 'vti' maps (C11, C13, C33, C55, C66)."""
    B = vti_B_matrices()
    return [B["11"], B["13"], B["33"], B["55"], B["66"]]


def B_list(params):
    return general_B_matrices() if params == "general" else vti_B_list()


def contrast_voigt(maps, params):
    """delta C(x) = sum_p B^(p) delta m^(p)(x) (eq. dC) as a [6, 6, nz, ny, nx] field."""
    Bs = B_list(params)
    maps = np.asarray(maps, dtype=float)
    assert maps.shape[0] == len(Bs) + 1, "stiffness maps plus rho"
    return np.einsum("pIJ,p...->IJ...", np.array(Bs), maps[:-1])


def thomsen_vti_6x6(vp0, vs0, eps, delta, gamma, rho):
    """6x6 VTI stiffness from Thomsen's parameters; C66 = C55 (1 + 2 gamma)."""
    C33 = rho * vp0 ** 2
    C55 = rho * vs0 ** 2
    C11 = C33 * (1.0 + 2.0 * eps)
    C13 = np.sqrt(2.0 * delta * C33 * (C33 - C55) + (C33 - C55) ** 2) - C55
    C66 = C55 * (1.0 + 2.0 * gamma)
    from .media import vti_voigt
    return vti_voigt(C11, C33, C55, C66, C13)


def rotate_voigt(C6, R):
    """Stiffness of a rotated medium, C'_ijkl = R_ia R_jb R_kc R_ld C_abcd, as 6x6."""
    C = voigt_to_tensor(C6)
    Cr = np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, C)
    out = np.zeros((6, 6))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    out[VOIGT_INDEX[i, j], VOIGT_INDEX[k, l]] = Cr[i, j, k, l]
    return out


# ------------------------------------------------------- Green's symbol --
def wavenumbers_3d(nx, ny, nz, dx, symbol="spectral", odd=False):
    """(kx, ky, kz) on the [nz, ny, nx] FFT grid.

    symbol='central' replaces k by sin(k dx)/dx (the central-difference
    symbol).  odd=True gives the wavenumbers for products of two different
    components: zero at the Nyquist index of an even axis.
    """
    ks = []
    for n in (nx, ny, nz):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=dx)
        if symbol == "central":
            k = np.sin(k * dx) / dx
        elif symbol != "spectral":
            raise ValueError("symbol must be 'spectral' or 'central'")
        if odd and n % 2 == 0:
            k = k.copy()
            k[n // 2] = 0.0
        ks.append(k)
    KZ, KY, KX = np.meshgrid(ks[2], ks[1], ks[0], indexing="ij")
    return KX, KY, KZ


def christoffel_k(C6, K, Ko=None):
    """Gamma_ik = sum_jl C_ijkl k_j k_l from the general 4-index tensor at
    wavevectors K [3, ...]; Ko (default K) serves the products of two
    different components.  Returns [3, 3, ...]."""
    C = voigt_to_tensor(C6)
    K = [np.asarray(k, dtype=float) for k in K]
    Ko = K if Ko is None else [np.asarray(k, dtype=float) for k in Ko]
    ext = (None,) * K[0].ndim
    G = np.zeros((3, 3) + K[0].shape)
    for j in range(3):
        for l in range(3):
            kk = K[j] * K[l] if j == l else Ko[j] * Ko[l]
            G += C[:, j, :, l][(slice(None), slice(None)) + ext] * kk
    return G


def christoffel_3d(C6, nx, ny, nz, dx, symbol="spectral"):
    """Christoffel matrix on the [nz, ny, nx] FFT grid, [3, 3, nz, ny, nx]."""
    return christoffel_k(C6, wavenumbers_3d(nx, ny, nz, dx, symbol),
                         wavenumbers_3d(nx, ny, nz, dx, symbol, odd=True))


def green_symbol_3d(C6, rho0, omega_t, nx, ny, nz, dx, symbol="spectral"):
    """G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1, [3, 3, nz, ny, nx] (eq. Green transformed)."""
    Gam = christoffel_3d(C6, nx, ny, nz, dx, symbol).astype(complex)
    M = Gam - rho0 * omega_t ** 2 * np.eye(3)[:, :, None, None, None]
    Minv = np.linalg.inv(np.moveaxis(M, (0, 1), (-2, -1)))
    return np.moveaxis(Minv, (-2, -1), (0, 1))


def green_symbol_isotropic_3d(vp, vs, rho0, omega_t, KX, KY, KZ):
    """Textbook isotropic symbol: P part along k^, S part across it; G_hat(0) = -I/(rho0 w~^2)."""
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kn = np.sqrt(k2)
    safe = np.where(kn > 0, kn, 1.0)
    h = [np.where(kn > 0, K / safe, 0.0) for K in (KX, KY, KZ)]
    P = np.array([[h[i] * h[j] for j in range(3)] for i in range(3)])
    I = np.eye(3)[:, :, None, None, None] * np.ones_like(k2)
    gp = 1.0 / (rho0 * (vp ** 2 * k2 - omega_t ** 2))
    gs = 1.0 / (rho0 * (vs ** 2 * k2 - omega_t ** 2))
    return P * gp + (I - P) * gs


def green_analytic_3d(vp, vs, rho0, omega_t, r_vec):
    """App. A's 3-D isotropic Green's tensor (Aki and Richards) at offsets
    r_vec [3, ...] != 0, evaluated at the complex frequency w~.  The printed
    form with exp(+i w r / alpha) is the outgoing tensor of the exp(-i w t)
    convention used here, so it is taken as printed."""
    r = np.sqrt(np.sum(np.asarray(r_vec) ** 2, axis=0))
    g = np.asarray(r_vec) / r
    out = np.empty((3, 3) + r.shape, dtype=complex)
    ea = np.exp(1j * omega_t * r / vp) / (4.0 * np.pi * rho0 * vp ** 2 * r)
    eb = np.exp(1j * omega_t * r / vs) / (4.0 * np.pi * rho0 * vs ** 2 * r)
    qa = -vp / (1j * omega_t * r)
    qb = -vs / (1j * omega_t * r)
    for i in range(3):
        for j in range(3):
            d = 1.0 if i == j else 0.0
            gg = g[i] * g[j]
            t3 = 3.0 * gg - d
            out[i, j] = ea * (gg + t3 * qa + t3 * qa ** 2) - eb * ((gg - d) + t3 * qb + t3 * qb ** 2)
    return out


# ----------------------------------------------------------- operators --
def d_axis(f, dx, axis):
    """Periodic central difference along a field axis: -1 = x, -2 = y, -3 = z."""
    return (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)) / (2.0 * dx)


def strain_voigt_3d(u, dx):
    """Engineering Voigt strain [..., 6, nz, ny, nx] of u [..., 3, nz, ny, nx]."""
    D = [lambda f: d_axis(f, dx, -1), lambda f: d_axis(f, dx, -2), lambda f: d_axis(f, dx, -3)]
    c = [u[..., a, :, :, :] for a in range(3)]
    e = np.zeros(u.shape[:-4] + (6,) + u.shape[-3:], dtype=np.result_type(u, 1.0))
    for i in range(3):
        for j in range(i, 3):
            if i == j:
                e[..., VOIGT_INDEX[i, i], :, :, :] = D[i](c[i])
            else:
                e[..., VOIGT_INDEX[i, j], :, :, :] = D[j](c[i]) + D[i](c[j])
    return e


def divergence_voigt_3d(s, dx):
    """b_i = sum_j D_j sigma_ij of a Voigt stress field [..., 6, nz, ny, nx]."""
    out = np.zeros(s.shape[:-4] + (3,) + s.shape[-3:], dtype=s.dtype)
    for i in range(3):
        for j in range(3):
            out[..., i, :, :, :] += d_axis(s[..., VOIGT_INDEX[i, j], :, :, :], dx, -1 - j)
    return out


def body_force_3d(u, dC6, drho, omega_t, dx):
    """b(u) = w~^2 drho u + div_h(dC : E_h u) (eq. Ewave0's contrast terms)."""
    e = strain_voigt_3d(u, dx)
    s = np.einsum("IJ...,sJ...->sI...", dC6, e.reshape((-1,) + e.shape[-4:])).reshape(e.shape)
    return omega_t ** 2 * drho * u + divergence_voigt_3d(s, dx)


def convolve_3d(Ghat, f):
    """G0 conv f = ifftn(G_hat . fftn(f)) over the three grid axes (eq. FFT)."""
    F = scipy.fft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)
    H = np.einsum("ij...,sj...->si...", Ghat, F.reshape((-1,) + F.shape[-4:])).reshape(F.shape)
    return scipy.fft.ifftn(H, axes=(-3, -2, -1), workers=_WORKERS)


def point_sources_3d(nx, ny, nz, dx, src_ixyz, src_f):
    """One point force per system: F / dx^3 at cell (ix, iy, iz)."""
    s = np.zeros((len(src_ixyz), 3, nz, ny, nx), dtype=complex)
    for k, ((ix, iy, iz), f) in enumerate(zip(src_ixyz, src_f)):
        s[k, :, iz, iy, ix] += np.asarray(f, dtype=float) / dx ** 3
    return s


def sample_3d(w, rec_ixyz):
    """d[sys, rec, comp] = w[sys, comp, iz, iy, ix]."""
    r = np.asarray(rec_ixyz, dtype=int)
    return np.transpose(w[:, :, r[:, 2], r[:, 1], r[:, 0]], (0, 2, 1))


def sample_transpose_3d(d, rec_ixyz, nx, ny, nz):
    """R^T: receiver values back into a field, repeats added."""
    out = np.zeros((d.shape[0], 3, nz, ny, nx), dtype=np.result_type(d, 1j))
    for k, (ix, iy, iz) in enumerate(rec_ixyz):
        out[:, :, iz, iy, ix] += d[:, k, :]
    return out


# ------------------------------------------------------------- problem --
class LSProblem3D:
    """One (3-D grid, general background, frequency) problem with a contrast.

    c0: the background as a symmetric 6x6 Voigt matrix (or its 21 constants);
    maps: [nparams + 1, nz, ny, nx] contrast in the chosen parametrisation.
    """

    def __init__(self, nx, ny, nz, dx, c0, rho0, freq_hz, eta=0.02, maps=None, params="vti",
                 symbol="spectral"):
        self.nx, self.ny, self.nz, self.dx = int(nx), int(ny), int(nz), float(dx)
        c0 = np.asarray(c0, dtype=float)
        self.C6 = voigt_from_21(c0) if c0.shape == (21,) else c0
        assert self.C6.shape == (6, 6) and np.allclose(self.C6, self.C6.T)
        self.rho0, self.freq_hz, self.eta = float(rho0), float(freq_hz), float(eta)
        self.params = params
        self.nmaps = len(PARAM_NAMES[params])
        self.omega_t = 2.0 * np.pi * self.freq_hz * (1.0 + 1j * self.eta)
        self.Ghat = green_symbol_3d(self.C6, self.rho0, self.omega_t, nx, ny, nz, dx, symbol)
        self.set_contrast(np.zeros((self.nmaps, nz, ny, nx)) if maps is None else maps)

    def set_contrast(self, maps):
        maps = np.asarray(maps, dtype=float)
        assert maps.shape == (self.nmaps, self.nz, self.ny, self.nx)
        self.maps = maps
        self.dC6 = contrast_voigt(maps, self.params)
        self.drho = maps[-1]

    def body_force(self, u):
        return body_force_3d(u, self.dC6, self.drho, self.omega_t, self.dx)

    def convolve(self, f):
        return convolve_3d(self.Ghat, f)

    def apply(self, u):
        """A u = u - G0 conv b(u) (eq. A)."""
        return u - self.convolve(self.body_force(u))

    def incident(self, src_ixyz, src_f):
        """u0 = G0 conv s (eq. u0)."""
        return self.convolve(point_sources_3d(self.nx, self.ny, self.nz, self.dx, src_ixyz, src_f))

    def solve(self, rhs, tol=1e-10, maxit=10000):
        rhs = np.asarray(rhs, dtype=complex)
        out = np.empty_like(rhs)
        infos = []
        for k in range(rhs.shape[0]):
            xk, info = krylov.bicgstab(lambda v: self.apply(v[None])[0], rhs[k], tol=tol, maxit=maxit)
            out[k] = xk
            infos.append(info)
        return out, infos

    def virtual_source(self, ub, dm):
        """P_b(dm) = w~^2 dm_rho u^b + div_h(dC(dm) : E_h u^b) (eqs. YM, dC)."""
        dm = np.asarray(dm, dtype=float)
        return body_force_3d(ub, contrast_voigt(dm, self.params), dm[-1], self.omega_t, self.dx)

    def frechet(self, ub, dm, rec_ixyz, tol=1e-10):
        """J dm = R A_b^-1 G0 conv P_b(dm) (eqs. F0, uY), [nsys, nrec, 3]."""
        w, _ = self.solve(self.convolve(self.virtual_source(ub, dm)), tol=tol)
        return sample_3d(w, rec_ixyz)

    def adjoint(self, ub, r, rec_ixyz, tol=1e-10):
        """J* r as complex maps [nparams + 1, nz, ny, nx] (eqs. ad1, ua, ua0)."""
        f = sample_transpose_3d(np.conj(r), rec_ixyz, self.nx, self.ny, self.nz)
        ua, _ = self.solve(self.convolve(f), tol=tol)
        return self.correlate(ua, ub)

    def correlate(self, ua, ub):
        """Sum over systems of eq. ad1's pointwise products."""
        ea = strain_voigt_3d(ua, self.dx)
        eb = strain_voigt_3d(ub, self.dx)
        Bs = B_list(self.params)
        g = np.zeros((len(Bs) + 1, self.nz, self.ny, self.nx), dtype=complex)
        for p, B in enumerate(Bs):
            g[p] = -np.conj(np.einsum("sI...,IJ,sJ...->...", ea, B, eb))
        g[-1] = np.conj(self.omega_t ** 2 * np.einsum("sc...,sc...->...", ua, ub))
        return g

    def data(self, maps, u0, rec_ixyz, tol=1e-12):
        """R A(maps)^-1 u0: receiver data of the full forward problem."""
        saved = self.maps
        self.set_contrast(maps)
        try:
            u, _ = self.solve(u0, tol=tol)
        finally:
            self.set_contrast(saved)
        return sample_3d(u, rec_ixyz)
