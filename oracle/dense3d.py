"""Explicit 3-D matrices for pinning the 3-D oracle on tiny grids.

TEST INFRASTRUCTURE.  Nothing here uses an FFT or the roll stencils of
elastic3d.py:

* green_matrix_3d: the dense periodic Green's matrix from a direct DFT sum,
  g_ij(n) = (1/N) sum_k G_hat_ij(k) exp(2 pi i k.n / N), placed at row
  (i, x), column (j, x') as g_ij(x - x');
* strain_operator_3d: E_h (the six engineering Voigt strains) as a sparse
  matrix assembled from explicit circulant difference matrices by Kronecker
  products;
* stiffness_operator_3d: the per-cell 6x6 stiffness as a block matrix built
  entry by entry from the symmetric matrix;
* contrast_operator_3d / elastic_operator_3d: V = w~^2 drho - E_h^T dC E_h
  and the discrete eq. Ewave, w~^2 rho - E_h^T C E_h, so that the
  divergence enters only as the transpose of E_h.

Vectors are fields [3, nz, ny, nx] flattened in C order.
"""

import numpy as np
import scipy.sparse as sp


def _inverse_dft(n):
    m = np.arange(n)
    return np.exp(2j * np.pi * np.outer(m, m) / n)


def green_real_space_3d(Ghat):
    """g_ij[z, y, x] = (1/N) sum_k G_hat_ij[kz, ky, kx] exp(2 pi i k.n)."""
    _, _, nz, ny, nx = Ghat.shape
    Ez, Ey, Ex = _inverse_dft(nz), _inverse_dft(ny), _inverse_dft(nx)
    return np.einsum("za,yb,xc,ijabc->ijzyx", Ez, Ey, Ex, Ghat) / (nz * ny * nx)


def green_matrix_3d(Ghat):
    """Dense [3 N, 3 N] matrix of the periodic convolution with G0."""
    _, _, nz, ny, nx = Ghat.shape
    g = green_real_space_3d(Ghat)
    N = nz * ny * nx
    iz, iy, ix = np.unravel_index(np.arange(N), (nz, ny, nx))
    dz = (iz[:, None] - iz[None, :]) % nz
    dy = (iy[:, None] - iy[None, :]) % ny
    dxx = (ix[:, None] - ix[None, :]) % nx
    G = np.empty((3 * N, 3 * N), dtype=complex)
    for i in range(3):
        for j in range(3):
            G[i * N:(i + 1) * N, j * N:(j + 1) * N] = g[i, j][dz, dy, dxx]
    return G


def _derivative_1d(n, dx):
    """Circulant central difference (f[m+1] - f[m-1]) / (2 dx); zero for n = 1."""
    if n == 1:
        return sp.csr_matrix((1, 1))
    rows = np.arange(n)
    data = np.concatenate([np.full(n, 1.0 / (2 * dx)), np.full(n, -1.0 / (2 * dx))])
    cols = np.concatenate([(rows + 1) % n, (rows - 1) % n])
    return sp.csr_matrix((data, (np.concatenate([rows, rows]), cols)), shape=(n, n)).tocsr()


def strain_operator_3d(nx, ny, nz, dx):
    """E_h: [6 N, 3 N]; rows (e_xx, e_yy, e_zz, e_yz, e_xz, e_xy), columns (u_x, u_y, u_z)."""
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Dx = sp.kron(sp.kron(Iz, Iy), _derivative_1d(nx, dx))
    Dy = sp.kron(sp.kron(Iz, _derivative_1d(ny, dx)), Ix)
    Dz = sp.kron(sp.kron(_derivative_1d(nz, dx), Iy), Ix)
    Z = sp.csr_matrix((nx * ny * nz, nx * ny * nz))
    return sp.bmat([[Dx, Z, Z],
                    [Z, Dy, Z],
                    [Z, Z, Dz],
                    [Z, Dz, Dy],
                    [Dz, Z, Dx],
                    [Dy, Dx, Z]]).tocsr()


def stiffness_operator_3d(C6field, n):
    """Block [6 N, 6 N] matrix of a per-cell symmetric 6x6 stiffness (C6field [6, 6, ...] or [6, 6])."""
    blocks = [[None] * 6 for _ in range(6)]
    for I in range(6):
        for J in range(6):
            v = np.broadcast_to(np.asarray(C6field[I][J], dtype=float).ravel(), (n,)).copy()
            blocks[I][J] = sp.diags(v)
    return sp.bmat(blocks).tocsr()


def contrast_operator_3d(dC6, drho, omega_t, nx, ny, nz, dx):
    """V = w~^2 drho - E_h^T dC E_h, sparse [3 N, 3 N]."""
    n = nx * ny * nz
    E = strain_operator_3d(nx, ny, nz, dx)
    D = stiffness_operator_3d(dC6, n)
    R = sp.diags(np.tile(np.asarray(drho, dtype=float).ravel(), 3))
    return (omega_t ** 2 * R - E.T @ D @ E).tocsr()


def elastic_operator_3d(C6_0, rho0, dC6, drho, omega_t, nx, ny, nz, dx):
    """Discrete eq. Ewave in 3-D: w~^2 rho - E_h^T C E_h with C = C0 + dC, rho = rho0 + drho."""
    n = nx * ny * nz
    C = np.asarray(dC6, dtype=float) + np.asarray(C6_0, dtype=float)[:, :, None, None, None]
    E = strain_operator_3d(nx, ny, nz, dx)
    D = stiffness_operator_3d(C, n)
    R = sp.diags(np.tile((rho0 + np.asarray(drho, dtype=float)).ravel(), 3))
    return (omega_t ** 2 * R - E.T @ D @ E).tocsr()


def point_source_vector_3d(nx, ny, nz, dx, ix, iy, iz, f):
    """Flattened source vector: F / dx^3 at cell (ix, iy, iz)."""
    n = nx * ny * nz
    s = np.zeros(3 * n, dtype=complex)
    cell = (iz * ny + iy) * nx + ix
    for c in range(3):
        s[c * n + cell] = f[c] / dx ** 3
    return s
