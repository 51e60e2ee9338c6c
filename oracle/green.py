"""Green's tensor of the homogeneous background.

Paper passages: eq. Green (the defining PDE with a unit point source), eq. u0
(incident field by convolution with G0) and App. A (isotropic analytic forms).

The periodic grid needs G0 only through its discrete Fourier symbol.  Fourier
transforming eq. Green with a homogeneous C0, rho0 turns div(C0 : grad G) into
-Gamma(k) G_hat, with the Christoffel matrix Gamma_ik = C_ijkl k_j k_l, so that
(rho0 w~^2 - Gamma) G_hat = -I and

    G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1.

Here w~ = w (1 + i eta) carries the small damping that keeps the periodic
problem away from the real slowness surface.  The time convention is
exp(-i w t), so outgoing waves are exp(+i k r) and decay because Im w~ > 0.

This module computes Gamma from the general 4-index tensor (no VTI shortcut)
and inverts each 2x2 (x, z) block with numpy.linalg.inv.
"""

import numpy as np
import scipy.special

from .media import voigt_to_tensor


def angular_wavenumbers(n, dx):
    """Discrete angular wavenumbers 2 pi fftfreq(n, dx), in FFT order."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=dx)


def complex_frequency(freq_hz, eta):
    """w~ = 2 pi f (1 + i eta)."""
    return 2.0 * np.pi * freq_hz * (1.0 + 1j * eta)


def wavenumber_grid(nx, nz, dx, symbol="spectral"):
    """(kx, kz) on the [nz, nx] FFT grid.

    symbol='spectral' uses the exact discrete wavenumbers; symbol='central'
    replaces each k by sin(k dx)/dx, the Fourier symbol of the 2nd-order
    central difference, which makes G_hat the exact inverse of the discrete
    background operator (used by the PDE-equivalence pin).
    """
    kx = angular_wavenumbers(nx, dx)
    kz = angular_wavenumbers(nz, dx)
    if symbol == "central":
        kx = np.sin(kx * dx) / dx
        kz = np.sin(kz * dx) / dx
    elif symbol != "spectral":
        raise ValueError("symbol must be 'spectral' or 'central'")
    KX, KZ = np.meshgrid(kx, kz, indexing="xy")
    return KX, KZ


def odd_wavenumber_grid(nx, nz, dx, symbol="spectral"):
    """The wavenumbers used in products of two DIFFERENT components.

    For even n the Nyquist index -n/2 has no partner +n/2, so a term odd in
    one component (such as kx kz) would make G_hat lose its evenness in k and
    the discrete G0 its symmetry.  Such products therefore take the value zero
    at the Nyquist index; squares keep (n/2)^2.  The central-difference symbol
    vanishes there already.
    """
    KX, KZ = wavenumber_grid(nx, nz, dx, symbol)
    if nx % 2 == 0:
        KX = KX.copy()
        KX[:, nx // 2] = 0.0
    if nz % 2 == 0:
        KZ = KZ.copy()
        KZ[nz // 2, :] = 0.0
    return KX, KZ


def christoffel_2d(C6, KX, KZ, KXo=None, KZo=None):
    """In-plane Christoffel matrix Gamma_ik = sum_jl C_ijkl k_j k_l.

    k = (kx, 0, kz); terms with j != l use the odd-product wavenumbers
    (KXo, KZo) (see odd_wavenumber_grid).  Returns the (x, z) block as
    [2, 2, nz, nx].
    """
    C = voigt_to_tensor(C6)
    KXo = KX if KXo is None else KXo
    KZo = KZ if KZo is None else KZo
    K = np.stack([KX, np.zeros_like(KX), KZ])        # [3, nz, nx]
    Ko = np.stack([KXo, np.zeros_like(KX), KZo])
    G3 = np.zeros((3, 3) + KX.shape)
    for j in range(3):
        for l in range(3):
            kk = K[j] * K[l] if j == l else Ko[j] * Ko[l]
            G3 += C[:, j, :, l][:, :, None, None] * kk
    sel = [0, 2]
    return G3[np.ix_(sel, sel)]


def green_symbol(C6, rho0, omega_t, nx, nz, dx, symbol="spectral"):
    """G_hat(k) = (Gamma(k) - rho0 w~^2 I)^-1 on the FFT grid, [2, 2, nz, nx]."""
    KX, KZ = wavenumber_grid(nx, nz, dx, symbol)
    KXo, KZo = odd_wavenumber_grid(nx, nz, dx, symbol)
    Gam = christoffel_2d(C6, KX, KZ, KXo, KZo).astype(complex)
    M = Gam - rho0 * omega_t ** 2 * np.eye(2)[:, :, None, None]
    Minv = np.linalg.inv(np.moveaxis(M, (0, 1), (-2, -1)))
    return np.moveaxis(Minv, (-2, -1), (0, 1))


def green_symbol_isotropic(vp, vs, rho0, omega_t, KX, KZ):
    """Closed-form isotropic symbol (Helmholtz split into P and S parts).

    G_hat = k^ k^T / (rho0 (vp^2 k^2 - w~^2)) + (I - k^ k^T)/(rho0 (vs^2 k^2 - w~^2)),
    and G_hat(0) = -I / (rho0 w~^2).
    """
    k2 = KX ** 2 + KZ ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        kn = np.sqrt(k2)
        hx = np.where(kn > 0, KX / np.where(kn > 0, kn, 1), 0.0)
        hz = np.where(kn > 0, KZ / np.where(kn > 0, kn, 1), 0.0)
    P = np.array([[hx * hx, hx * hz], [hz * hx, hz * hz]])
    I = np.eye(2)[:, :, None, None] * np.ones_like(k2)
    gp = 1.0 / (rho0 * (vp ** 2 * k2 - omega_t ** 2))
    gs = 1.0 / (rho0 * (vs ** 2 * k2 - omega_t ** 2))
    G = P * gp + (I - P) * gs
    return G


def green_analytic_2d(vp, vs, rho0, omega_t, rx, rz):
    """Analytic 2-D isotropic Green's tensor, App. A, in the exp(-i w t) form.

    App. A prints the exp(+i w t) form with second-kind Hankel functions and
    a 1/(8 i rho) prefactor.  Its complex conjugate (first-kind Hankel
    functions, prefactor i/(8 rho)) is the outgoing Green's tensor for the
    convention used here, evaluated at complex w~:

        G_ij = i/(8 rho) { A delta_ij - B (2 g_i g_j - delta_ij) },
        A = H0(w r/a)/a^2 + H0(w r/b)/b^2,  B = H2(w r/a)/a^2 - H2(w r/b)/b^2,

    with g = (x - x')/r.  Returns [2, 2, ...] over the offsets (rx, rz) != 0.
    """
    r = np.hypot(rx, rz)
    gx, gz = rx / r, rz / r
    H0a = scipy.special.hankel1(0, omega_t * r / vp)
    H0b = scipy.special.hankel1(0, omega_t * r / vs)
    H2a = scipy.special.hankel1(2, omega_t * r / vp)
    H2b = scipy.special.hankel1(2, omega_t * r / vs)
    A = H0a / vp ** 2 + H0b / vs ** 2
    B = H2a / vp ** 2 - H2b / vs ** 2
    g = [gx, gz]
    out = np.empty((2, 2) + np.shape(r), dtype=complex)
    for i in range(2):
        for j in range(2):
            d = 1.0 if i == j else 0.0
            out[i, j] = 1j / (8.0 * rho0) * (A * d - B * (2.0 * g[i] * g[j] - d))
    return out
