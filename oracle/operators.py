"""Discrete operators of the Lippmann-Schwinger equation on a periodic grid.

Paper passages: eqs. u and u_2 (the integral equation and its form after the
integration by parts of eq. dgv), eq. A (the operator), eq. axb, eq. FFT
(circular convolution by FFT) and eq. u0 (incident field); the abbreviated
subscript section for the Voigt strain vector.

Discretisation (the paper leaves the stencil unspecified; these are the
readings used throughout):
  * grid [nz, nx], spacing dx on both axes, every index periodic;
  * derivatives are 2nd-order central differences
        (D_x f)[j, i] = (f[j, i+1] - f[j, i-1]) / (2 dx),  D_z likewise along j;
  * the strain is the Voigt engineering strain built from D_x and D_z;
  * the term -int grad'G0 . [dC : grad u] of eq. u_2 is evaluated as
    G0 conv (div_h sigma) with div_h built from the same central differences.
    On the torus summation by parts is exact (div_h = -E_h^T), so the
    surface term of eq. dgv vanishes identically;
  * G0 conv f = ifft2(G_hat * fft2(f)); the cell-volume factor of the
    integral and the 1/dx^2 of the sampled Green's function cancel.

Field arrays are [..., 2, nz, nx] with component 0 = x and 1 = z.
"""

import os

import numpy as np
import scipy.fft

# threads for scipy.fft: the host cores, at most 16 (one GPU's share of a box)
_WORKERS = max(1, min(os.cpu_count() or 1, 16))


def ddx(f, dx):
    """Central difference along x (last axis), periodic."""
    return (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1)) / (2.0 * dx)


def ddz(f, dx):
    """Central difference along z (second-last axis), periodic."""
    return (np.roll(f, -1, axis=-2) - np.roll(f, 1, axis=-2)) / (2.0 * dx)


def strain_voigt(u, dx):
    """Voigt engineering strain of an in-plane field, [..., 6, nz, nx].

    (d1u1, d2u2, d3u3, d2u3+d3u2, d1u3+d3u1, d1u2+d2u1) with u_y = 0 and
    d/dy = 0, so entries 1, 3 and 5 vanish.
    """
    ux, uz = u[..., 0, :, :], u[..., 1, :, :]
    e = np.zeros(u.shape[:-3] + (6,) + u.shape[-2:], dtype=np.result_type(u, 1.0))
    e[..., 0, :, :] = ddx(ux, dx)
    e[..., 2, :, :] = ddz(uz, dx)
    e[..., 4, :, :] = ddz(ux, dx) + ddx(uz, dx)
    return e


def stress_voigt(C6f, e):
    """sigma_I = sum_J C_IJ e_J for a Voigt field C6f [6, 6, nz, nx]."""
    if C6f.ndim == 4:
        return np.einsum("IJzx,...Jzx->...Izx", C6f, e)
    return np.einsum("IJ,...Jzx->...Izx", C6f, e)


def divergence_voigt(s, dx):
    """In-plane divergence b_i = sum_j d_j sigma_ij of a Voigt stress field.

    The stress tensor is rebuilt from the Voigt vector (sigma_xx = s0,
    sigma_zz = s2, sigma_xz = s4); with d/dy = 0 only d_x and d_z act.
    """
    from .media import VOIGT_INDEX
    comps = (0, 2)                      # tensor indices of x and z
    out = np.zeros(s.shape[:-3] + (2,) + s.shape[-2:], dtype=s.dtype)
    for a, i in enumerate(comps):
        sx = s[..., VOIGT_INDEX[i, 0], :, :]
        sz = s[..., VOIGT_INDEX[i, 2], :, :]
        out[..., a, :, :] = ddx(sx, dx) + ddz(sz, dx)
    return out


def body_force(u, dC6, drho, omega_t, dx):
    """Equivalent body force of the contrast, eq. Ewave0 right-hand side:

        b(u) = w~^2 drho u + div_h( dC : E_h u ).

    The LS equation (eq. u_2 after the integration by parts) is u = u0 + G0 conv b(u).
    """
    e = strain_voigt(u, dx)
    s = stress_voigt(dC6, e)
    return omega_t ** 2 * drho * u + divergence_voigt(s, dx)


def convolve(Ghat, f):
    """G0 conv f = ifft2( G_hat(k) . fft2(f)(k) ), eq. FFT; f is [..., 2, nz, nx]."""
    F = scipy.fft.fft2(f, axes=(-2, -1), workers=_WORKERS)
    H = np.einsum("ijzx,...jzx->...izx", Ghat, F)
    return scipy.fft.ifft2(H, axes=(-2, -1), workers=_WORKERS)


def ls_apply(u, Ghat, dC6, drho, omega_t, dx):
    """The operator of eq. A applied to u: A u = u - G0 conv b(u)."""
    return u - convolve(Ghat, body_force(u, dC6, drho, omega_t, dx))


def point_sources(nsys, nx, nz, dx, src_ixz, src_f):
    """Discrete source field for one point force per system, eq. u_int.

    A force F (newtons, components (fx, fz)) at cell (ix, iz) is the delta
    function sampled as F / dx^2 at that cell.
    """
    s = np.zeros((nsys, 2, nz, nx), dtype=complex)
    for k in range(nsys):
        ix, iz = int(src_ixz[k][0]), int(src_ixz[k][1])
        s[k, 0, iz, ix] += src_f[k][0] / dx ** 2
        s[k, 1, iz, ix] += src_f[k][1] / dx ** 2
    return s


def sample(w, rec_ixz):
    """Receiver sampling R: d[sys, rec, comp] = w[sys, comp, iz_rec, ix_rec]."""
    ix = np.array([r[0] for r in rec_ixz], dtype=int)
    iz = np.array([r[1] for r in rec_ixz], dtype=int)
    return np.transpose(w[:, :, iz, ix], (0, 2, 1))


def sample_transpose(d, rec_ixz, nx, nz):
    """R^T: place receiver values back into a field (adding repeats)."""
    nsys = d.shape[0]
    out = np.zeros((nsys, 2, nz, nx), dtype=np.result_type(d, 1j))
    for r, (ix, iz) in enumerate(rec_ixz):
        out[:, :, iz, ix] += d[:, r, :]
    return out
