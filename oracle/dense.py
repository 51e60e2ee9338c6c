"""Explicit matrices for pinning the oracle on tiny grids.

Nothing here uses an FFT or the stencil code of operators.py:

* green_matrix builds the dense periodic Green's matrix from a direct DFT sum
  g_ij(n) = (1/N) sum_k G_hat_ij(k) exp(2 pi i k.n / N), then places
  g_ij(x - x') in row (i, x), column (j, x');
* strain_operator builds E_h (the Voigt strain restricted to
  (e_xx, e_zz, e_xz)) as a sparse matrix from explicit stencil coefficients;
* contrast_operator builds V = w~^2 drho - E_h^T dC E_h with the reduced 3x3
  Voigt stiffness per cell, so that the divergence enters only through the
  transpose of E_h;
* elastic_operator builds the discrete version of eq. Ewave,
  w~^2 rho - E_h^T C E_h, for the full medium.

Vectors are fields [2, nz, nx] flattened C-order (index c nz nx + z nx + x).
"""

import numpy as np
import scipy.sparse as sp


def _inverse_dft(n):
    m = np.arange(n)
    return np.exp(2j * np.pi * np.outer(m, m) / n)


def green_real_space(Ghat):
    """g_ij[z, x] = (1/(nz nx)) sum_k G_hat_ij[kz, kx] exp(2 pi i (kz z/nz + kx x/nx))."""
    _, _, nz, nx = Ghat.shape
    Ez, Ex = _inverse_dft(nz), _inverse_dft(nx)
    return np.einsum("zk,ijkl,xl->ijzx", Ez, Ghat, Ex) / (nz * nx)


def green_matrix(Ghat):
    """Dense [2 nz nx, 2 nz nx] matrix of the periodic convolution with G0."""
    _, _, nz, nx = Ghat.shape
    g = green_real_space(Ghat)
    z = np.arange(nz)
    x = np.arange(nx)
    dz = (z[:, None] - z[None, :]) % nz           # [z, z']
    dxi = (x[:, None] - x[None, :]) % nx          # [x, x']
    N = nz * nx
    G = np.empty((2 * N, 2 * N), dtype=complex)
    for i in range(2):
        for j in range(2):
            blk = g[i, j][dz[:, None, :, None], dxi[None, :, None, :]]   # [z, x, z', x']
            G[i * N:(i + 1) * N, j * N:(j + 1) * N] = blk.reshape(N, N)
    return G


def _derivative_1d(n, dx):
    """Circulant central difference: (f[m+1] - f[m-1]) / (2 dx)."""
    rows = np.arange(n)
    data = np.concatenate([np.full(n, 1.0 / (2 * dx)), np.full(n, -1.0 / (2 * dx))])
    cols = np.concatenate([(rows + 1) % n, (rows - 1) % n])
    return sp.csr_matrix((data, (np.concatenate([rows, rows]), cols)), shape=(n, n))


def strain_operator(nx, nz, dx):
    """E_h: [3 N, 2 N], rows (e_xx, e_zz, e_xz), columns (u_x, u_z)."""
    Dx = sp.kron(sp.identity(nz), _derivative_1d(nx, dx))
    Dz = sp.kron(_derivative_1d(nz, dx), sp.identity(nx))
    Z = sp.csr_matrix((nz * nx, nz * nx))
    return sp.bmat([[Dx, Z], [Z, Dz], [Dz, Dx]]).tocsr()


def _stiffness_blocks(C11, C13, C33, C55, n):
    """Block matrix of the reduced Voigt stiffness [[C11, C13, 0], [C13, C33, 0], [0, 0, C55]]."""
    def d(a):
        return sp.diags(np.broadcast_to(np.asarray(a, dtype=float).ravel(), (n,)).copy())
    Z = sp.csr_matrix((n, n))
    return sp.bmat([[d(C11), d(C13), Z], [d(C13), d(C33), Z], [Z, Z, d(C55)]]).tocsr()


def contrast_operator(maps, omega_t, nx, nz, dx):
    """V = w~^2 drho - E_h^T dC E_h as a sparse [2 N, 2 N] matrix."""
    n = nz * nx
    E = strain_operator(nx, nz, dx)
    D = _stiffness_blocks(maps[0], maps[1], maps[2], maps[3], n)
    R = sp.diags(np.tile(np.asarray(maps[4], dtype=float).ravel(), 2))
    return (omega_t ** 2 * R - E.T @ D @ E).tocsr()


def elastic_operator(c0, rho0, maps, omega_t, nx, nz, dx):
    """Discrete eq. Ewave: w~^2 rho - E_h^T C E_h for C = C0 + dC, rho = rho0 + drho."""
    n = nz * nx
    C11, C13, C33, C55 = c0
    E = strain_operator(nx, nz, dx)
    D = _stiffness_blocks(C11 + maps[0], C13 + maps[1], C33 + maps[2], C55 + maps[3], n)
    R = sp.diags(np.tile((rho0 + np.asarray(maps[4], dtype=float)).ravel(), 2))
    return (omega_t ** 2 * R - E.T @ D @ E).tocsr()


def point_source_vector(nx, nz, dx, ix, iz, fx, fz):
    """Flattened source vector: F / dx^2 at cell (ix, iz)."""
    s = np.zeros(2 * nz * nx, dtype=complex)
    s[0 * nz * nx + iz * nx + ix] = fx / dx ** 2
    s[1 * nz * nx + iz * nx + ix] = fz / dx ** 2
    return s
