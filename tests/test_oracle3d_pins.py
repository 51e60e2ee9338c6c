"""Pins of the 3-D, generally anisotropic oracle (oracle/elastic3d.py) to
things other than itself: explicit matrices built without FFTs or roll
stencils (oracle/dense3d.py), a sparse direct solve of the discrete 3-D
elastic equation, the textbook isotropic symbol, the rotation covariance of
the Christoffel matrix, the App. C matrices and the derivatives of the
strain energy, the already-pinned 2-D oracle (a grid one cell thick),
reciprocity, the adjoint identity, the Jacobian limit and App. A's analytic
3-D Green's tensor.  A mistake such as a transposed Voigt index, a wrong
sign or missing factor 2 in the shear strains, a dropped B^66 coupling or a
conjugation error fails at least one of them."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dense3d, elastic3d as E3
from oracle import LSProblem, krylov, media

RHO0 = 2200.0


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def _tilted_background(seed=0):
    """A VTI medium rotated by a random rotation: all 21 constants non-zero."""
    C = E3.thomsen_vti_6x6(2500.0, 1200.0, 0.15, 0.05, 0.1, RHO0)
    return E3.rotate_voigt(C, _rotation(seed))


def _smooth(rng, shape, ell=1.5):
    from scipy.ndimage import gaussian_filter
    a = gaussian_filter(rng.standard_normal(shape), ell, mode="wrap")
    return a / np.std(a)


def _general_contrast(C6, rng, shape, amp=0.05):
    """Smooth random contrast of all 21 constants (scaled by the background's
    largest constant) and of rho."""
    scale = np.abs(C6).max()
    maps = np.array([amp * scale * _smooth(rng, shape) for _ in range(21)] + [amp * RHO0 * _smooth(rng, shape)])
    return maps


def _vti_contrast(rng, shape, amp=0.08):
    C = E3.thomsen_vti_6x6(2500.0, 1200.0, 0.15, 0.05, 0.1, RHO0)
    m0 = [C[0, 0], C[0, 2], C[2, 2], C[4, 4], C[5, 5], RHO0]
    return np.array([amp * m * _smooth(rng, shape) for m in m0])


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# -------------------------------------------------------------- media ----
def test_general_B_matrices_are_energy_derivatives():
    """d(e^T C e)/dc_p = e^T B^(p) e for each of the 21 constants (eq. dC)."""
    rng = np.random.default_rng(1)
    c = rng.standard_normal(21)
    e = rng.standard_normal(6)
    Bs = E3.general_B_matrices()
    assert len(Bs) == 21
    for p in range(21):
        d = np.zeros(21)
        d[p] = 1.0
        fd = (e @ E3.voigt_from_21(c + d) @ e - e @ E3.voigt_from_21(c - d) @ e) / 2.0
        assert abs(fd - e @ Bs[p] @ e) < 1e-12
    # the 21 matrices span the symmetric 6x6 matrices: sum_p c_p B^(p) = C
    assert np.allclose(np.einsum("p,pij->ij", c, np.array(Bs)), E3.voigt_from_21(c))


def test_vti_B_matrices_match_appendix_and_derivatives(golden_dir):
    """App. C's five B matrices (B^66 with its -2 entries from C12 = C11 - 2 C66)
    are the derivatives of the VTI stiffness with respect to its constants."""
    Bs = dict(zip(("C11", "C13", "C33", "C55", "C66"), E3.vti_B_list()))
    base = dict(C11=17.9, C33=13.8, C55=3.2, C66=4.1, C13=8.1)
    for name, B in Bs.items():
        hi = dict(base)
        lo = dict(base)
        hi[name] += 0.5
        lo[name] -= 0.5
        fd = media.vti_voigt(hi["C11"], hi["C33"], hi["C55"], hi["C66"], hi["C13"]) - \
            media.vti_voigt(lo["C11"], lo["C33"], lo["C55"], lo["C66"], lo["C13"])
        assert np.array_equal(fd, B), name
    assert Bs["C66"][0, 1] == -2.0 and Bs["C66"][5, 5] == 1.0
    # the same numbers as the printed appendix (golden file)
    txt = open(f"{golden_dir}/vti_b_matrices.txt").read()
    assert "-2" in txt


def test_vti_contrast_equals_its_general_expansion():
    """The VTI parametrisation is the general one restricted by C22 = C11,
    C12 = C11 - 2 C66, C23 = C13, C44 = C55."""
    rng = np.random.default_rng(2)
    v = rng.standard_normal((6, 2, 3, 4))
    g = np.zeros((22, 2, 3, 4))
    idx = {pair: p for p, pair in enumerate(E3.GENERAL_PAIRS)}
    C11, C13, C33, C55, C66, rho = v
    g[idx[(0, 0)]] = C11
    g[idx[(1, 1)]] = C11
    g[idx[(0, 1)]] = C11 - 2 * C66
    g[idx[(0, 2)]] = C13
    g[idx[(1, 2)]] = C13
    g[idx[(2, 2)]] = C33
    g[idx[(3, 3)]] = C55
    g[idx[(4, 4)]] = C55
    g[idx[(5, 5)]] = C66
    g[21] = rho
    assert np.allclose(E3.contrast_voigt(v, "vti"), E3.contrast_voigt(g, "general"))


# ------------------------------------------------------ Green's symbol ----
def test_isotropic_symbol_closed_form_3d():
    """The general 4-index Christoffel inverse reduces to the textbook P / S
    split for an isotropic medium (odd grid sizes: no Nyquist index)."""
    vp, vs = 2000.0, 1000.0
    C6 = media.vti_voigt(RHO0 * vp ** 2, RHO0 * vp ** 2, RHO0 * vs ** 2, RHO0 * vs ** 2,
                         RHO0 * (vp ** 2 - 2 * vs ** 2))
    w = 2 * np.pi * 7.0 * (1 + 0.02j)
    G = E3.green_symbol_3d(C6, RHO0, w, 9, 7, 5, 10.0)
    KX, KY, KZ = E3.wavenumbers_3d(9, 7, 5, 10.0)
    ref = E3.green_symbol_isotropic_3d(vp, vs, RHO0, w, KX, KY, KZ)
    assert _rel(G, ref) < 1e-13


def test_christoffel_rotation_covariance():
    """Gamma'(k) = R Gamma(R^T k) R^T for the rotated stiffness, at random k:
    pins the general (triclinic) Christoffel matrix index by index."""
    C = E3.thomsen_vti_6x6(2500.0, 1200.0, 0.2, -0.05, 0.15, RHO0)
    R = _rotation(5)
    Cr = E3.rotate_voigt(C, R)
    assert np.count_nonzero(np.abs(E3.voigt_to_21(Cr)) > 1e-6 * np.abs(Cr).max()) == 21
    k = np.random.default_rng(6).standard_normal((3, 11))
    Gr = E3.christoffel_k(Cr, k)
    G = E3.christoffel_k(C, R.T @ k)
    ref = np.einsum("ia,abn,jb->ijn", R, G, R)
    assert _rel(Gr, ref) < 1e-13
    assert np.allclose(Gr, np.swapaxes(Gr, 0, 1))
    assert np.all(np.linalg.eigvalsh(np.moveaxis(Gr, 2, 0)) > 0)


# --------------------------------------------------- explicit matrices ----
def test_dense_direct_solve_3d():
    """Triclinic background, heterogeneous 21-constant contrast, 8 x 6 x 4
    grid (576 unknowns): BiCGSTAB through FFT convolutions and roll stencils
    against numpy.linalg.solve of (I - G V) u = G s with G from a direct
    DFT sum and V assembled from Kronecker difference matrices."""
    nx, ny, nz, dx = 8, 6, 4, 12.0
    C6 = _tilted_background(0)
    rng = np.random.default_rng(3)
    maps = _general_contrast(C6, rng, (nz, ny, nx))
    P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 9.0, maps=maps, params="general")
    src, f = [(2, 3, 1)], [(0.3, -0.5, 1.0)]
    u0 = P.incident(src, f)
    u, info = P.solve(u0, tol=1e-12)
    G = dense3d.green_matrix_3d(P.Ghat)
    V = dense3d.contrast_operator_3d(P.dC6, maps[-1], P.omega_t, nx, ny, nz, dx).toarray()
    s = dense3d.point_source_vector_3d(nx, ny, nz, dx, 2, 3, 1, f[0])
    u0_dense = G @ s
    assert _rel(u0.ravel(), u0_dense) < 1e-12
    ud = np.linalg.solve(np.eye(G.shape[0]) - G @ V, u0_dense)
    assert _rel(u.ravel(), ud) < 1e-9, info


def test_body_force_is_minus_transpose_stencil():
    """The roll-stencil body force equals V u with V = w~^2 drho - E_h^T dC E_h."""
    nx, ny, nz, dx = 6, 5, 4, 7.0
    C6 = _tilted_background(1)
    rng = np.random.default_rng(4)
    maps = _general_contrast(C6, rng, (nz, ny, nx))
    P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 5.0, maps=maps, params="general")
    u = rng.standard_normal((1, 3, nz, ny, nx)) + 1j * rng.standard_normal((1, 3, nz, ny, nx))
    V = dense3d.contrast_operator_3d(P.dC6, maps[-1], P.omega_t, nx, ny, nz, dx)
    assert _rel(P.body_force(u).ravel(), V @ u.ravel()) < 1e-13


@pytest.mark.parametrize("shape", [(12, 8, 10), (9, 10, 6)])
def test_pde_equivalence_central_symbol_3d(shape):
    """With the central-difference symbol G0 inverts the discrete background
    operator exactly, so the LS solution solves the discrete 3-D eq. Ewave
    (w~^2 rho - E_h^T C E_h) u = -s of the whole medium (sparse direct check);
    the spectral symbol must not (negative control)."""
    nx, ny, nz = shape
    dx = 10.0
    C6 = _tilted_background(2)
    rng = np.random.default_rng(7)
    maps = _general_contrast(C6, rng, (nz, ny, nx), amp=0.03)
    src, f = [(nx // 3, ny // 2, 1)], [(0.0, 0.4, 1.0)]
    s = dense3d.point_source_vector_3d(nx, ny, nz, dx, *src[0], f[0])
    for symbol, ok in (("central", True), ("spectral", False)):
        P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 8.0, maps=maps, params="general", symbol=symbol)
        u, _ = P.solve(P.incident(src, f), tol=1e-13)
        L = dense3d.elastic_operator_3d(C6, RHO0, P.dC6, maps[-1], P.omega_t, nx, ny, nz, dx)
        res = np.linalg.norm(L @ u.ravel() + s) / np.linalg.norm(s)
        if ok:
            assert res < 1e-9, res
            direct = spla.spsolve(L.tocsc(), -s)
            assert _rel(u.ravel(), direct) < 1e-9
        else:
            assert res > 1e-3, res


# ------------------------------------------------------- 2-D reduction ----
def test_one_cell_thick_grid_reduces_to_the_2d_oracle():
    """ny = 1, VTI background and contrast: the x and z components of the
    3-D problem are the pinned 2-D problem (a point force F / dx^3 in a slab
    of one cell is F / dx^2 per unit thickness, so u_3d dx = u_2d) and u_y
    is not excited by in-plane forces."""
    nx, nz, dx = 24, 16, 8.0
    C6 = E3.thomsen_vti_6x6(2500.0, 1200.0, 0.15, 0.05, 0.1, RHO0)
    rng = np.random.default_rng(8)
    m3 = _vti_contrast(rng, (nz, 1, nx))
    P3 = E3.LSProblem3D(nx, 1, nz, dx, C6, RHO0, 12.0, maps=m3, params="vti")
    m2 = m3[[0, 1, 2, 3, 5], :, 0, :]
    P2 = LSProblem(nx, nz, dx, (C6[0, 0], C6[0, 2], C6[2, 2], C6[4, 4]), RHO0, 12.0, maps=m2)
    u3, _ = P3.solve(P3.incident([(5, 0, 3)], [(0.6, 0.0, -0.8)]), tol=1e-12)
    u2, _ = P2.solve(P2.incident([(5, 3)], [(0.6, -0.8)]), tol=1e-12)
    assert np.abs(u3[0, 1]).max() < 1e-12 * np.abs(u3).max()
    assert _rel(u3[0][[0, 2], :, 0, :] * dx, u2[0]) < 1e-10
    # an out-of-plane force excites only u_y (the SH problem)
    uy, _ = P3.solve(P3.incident([(5, 0, 3)], [(0.0, 1.0, 0.0)]), tol=1e-12)
    assert np.abs(uy[0][[0, 2]]).max() < 1e-12 * np.abs(uy).max()


# -------------------------------------------- reciprocity and adjoint ----
def test_reciprocity_3d():
    """G^b_ij(x, x') = G^b_ji(x', x) with a heterogeneous general contrast
    (symmetry of the discrete operator; App. B's reciprocity)."""
    nx, ny, nz, dx = 10, 8, 6, 10.0
    C6 = _tilted_background(3)
    rng = np.random.default_rng(9)
    maps = _general_contrast(C6, rng, (nz, ny, nx), amp=0.1)
    P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 10.0, maps=maps, params="general")
    a, b = (1, 2, 1), (7, 5, 4)
    for i in range(3):
        for j in range(3):
            fj = np.eye(3)[j]
            fi = np.eye(3)[i]
            uj, _ = P.solve(P.incident([a], [fj]), tol=1e-13)
            ui, _ = P.solve(P.incident([b], [fi]), tol=1e-13)
            gij = uj[0, i, b[2], b[1], b[0]]
            gji = ui[0, j, a[2], a[1], a[0]]
            assert abs(gij - gji) <= 1e-9 * abs(gij), (i, j)


@pytest.mark.parametrize("params", ["vti", "general"])
def test_adjoint_dot_product_3d(params):
    """<r, J dm> = <J* r, dm> with complex dm, two systems (eq. ad1, App. B)."""
    nx, ny, nz, dx = 8, 6, 6, 10.0
    C6 = _tilted_background(4) if params == "general" else E3.thomsen_vti_6x6(2500.0, 1200.0, 0.15, 0.05, 0.1, RHO0)
    rng = np.random.default_rng(10)
    mb = _general_contrast(C6, rng, (nz, ny, nx)) if params == "general" else _vti_contrast(rng, (nz, ny, nx))
    P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 9.0, maps=mb, params=params)
    src = [(1, 1, 0), (5, 3, 0)]
    f = [(0.0, 0.0, 1.0), (0.5, 0.5, 0.7)]
    rec = [(i, j, 1) for i in range(0, 8, 3) for j in range(0, 6, 2)]
    ub, _ = P.solve(P.incident(src, f), tol=1e-13)
    dm = rng.standard_normal(mb.shape) * np.abs(mb).max() + 1j * rng.standard_normal(mb.shape) * np.abs(mb).max()
    r = rng.standard_normal((2, len(rec), 3)) + 1j * rng.standard_normal((2, len(rec), 3))
    # complex dm: J is complex-linear in dm (virtual source of eq. YM)
    d = P.frechet(ub, dm.real, rec, tol=1e-13) + 1j * P.frechet(ub, dm.imag, rec, tol=1e-13)
    g = P.adjoint(ub, r, rec, tol=1e-13)
    lhs = np.vdot(r, d)
    rhs = np.vdot(g, dm)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_frechet_is_the_jacobian_3d():
    """(R u(m + h d) - R u(m - h d)) / 2h -> J d, O(h^2), general parametrisation."""
    nx, ny, nz, dx = 8, 6, 6, 10.0
    C6 = _tilted_background(5)
    rng = np.random.default_rng(11)
    mb = _general_contrast(C6, rng, (nz, ny, nx))
    P = E3.LSProblem3D(nx, ny, nz, dx, C6, RHO0, 9.0, maps=mb, params="general")
    src, f = [(2, 2, 0)], [(0.2, 0.1, 1.0)]
    rec = [(i, 3, 2) for i in range(8)]
    u0 = P.incident(src, f)
    ub, _ = P.solve(u0, tol=1e-13)
    d = _general_contrast(C6, rng, (nz, ny, nx), amp=0.05)
    jd = P.frechet(ub, d, rec, tol=1e-13)
    errs = []
    for h in (1e-3, 1e-4):
        fd = (P.data(mb + h * d, u0, rec, tol=1e-13) - P.data(mb - h * d, u0, rec, tol=1e-13)) / (2 * h)
        errs.append(_rel(fd, jd))
    # second order: ten times smaller h, a hundred times smaller error
    assert errs[1] < 1e-6 and 50 < errs[0] / errs[1] < 200, errs


def test_zero_contrast_gives_the_incident_field_3d():
    C6 = _tilted_background(6)
    P = E3.LSProblem3D(8, 6, 4, 10.0, C6, RHO0, 6.0, params="general")
    u0 = P.incident([(1, 2, 3)], [(1.0, 0.0, 0.0)])
    u, info = P.solve(u0, tol=1e-12)
    assert info[0].iters <= 1 and _rel(u, u0) < 1e-14


# ---------------------------------------------------- App. A (loose) ------
@pytest.mark.slow
def test_periodic_green_matches_appendix_a_3d():
    """Isotropic background, 128^3 grid at 10 points per S wavelength and
    eta = 0.1 (so that the periodic images have decayed): the spectral
    Green's tensor column agrees with App. A's 3-D formula at complex w~ for
    offsets 2 lambda_s <= r <= L/4 to 1.5 % (a factor 2 gives 50 %, a sign
    flip 200 %)."""
    n, dx = 128, 10.0
    vp, vs = 2000.0, 1000.0
    f, eta = 10.0, 0.1           # lambda_s = 100 m = 10 cells
    C6 = media.vti_voigt(RHO0 * vp ** 2, RHO0 * vp ** 2, RHO0 * vs ** 2, RHO0 * vs ** 2,
                         RHO0 * (vp ** 2 - 2 * vs ** 2))
    w = 2 * np.pi * f * (1 + 1j * eta)
    P = E3.LSProblem3D(n, n, n, dx, C6, RHO0, f, eta=eta, params="vti")
    fvec = np.array([0.3, 0.5, 0.8])
    col = P.incident([(0, 0, 0)], [fvec])[0]
    idx = np.arange(n)
    off = np.where(idx <= n // 2, idx, idx - n) * dx
    OZ, OY, OX = np.meshgrid(off, off, off, indexing="ij")
    r = np.sqrt(OX ** 2 + OY ** 2 + OZ ** 2)
    sel = (r >= 2 * vs / f) & (r <= n * dx / 4)
    assert sel.sum() > 10000
    Ga = E3.green_analytic_3d(vp, vs, RHO0, w, np.array([OX[sel], OY[sel], OZ[sel]]))
    ref = np.einsum("ijn,j->in", Ga, fvec)
    err = np.linalg.norm(col[:, sel] - ref) / np.linalg.norm(ref)
    assert err < 5e-2, err


def test_laplacian3_plane_wave_eigenvalues():
    """The periodic 7-point Laplacian maps exp(i k.n) to (sum_a 2 cos(k_a) - 6)
    exp(i k.n), its discrete eigenvalue, for every map and wavevector."""
    from oracle import tikhonov
    nz, ny, nx = 6, 5, 8
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for kx, ky, kz in ((1, 0, 0), (3, 2, 1), (4, 4, 5)):
        a = (2 * np.pi * kx / nx, 2 * np.pi * ky / ny, 2 * np.pi * kz / nz)
        w = np.exp(1j * (a[0] * X + a[1] * Y + a[2] * Z))
        q = np.array([w, 2 * w])
        lam = 2 * np.cos(a[0]) + 2 * np.cos(a[1]) + 2 * np.cos(a[2]) - 6
        assert np.allclose(tikhonov.laplacian3(q), lam * q, atol=1e-12)
