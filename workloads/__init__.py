"""Seeded synthetic workloads for the elastic Lippmann-Schwinger hot path.

This module only makes inputs: background constants, contrast maps, source and
receiver positions and random data vectors.  It holds none of the method's
arithmetic, and both the CPU oracle and the GPU library consume what it makes.

The paper's own models (the 2-D VTI reservoir and Hess models) are not
available; these layered-plus-random VTI contrasts stand in for them.  Every
array is produced in float64 from numpy.random.default_rng(seed);
`round_f32` gives the float32-representable copy that both sides then use.

Recipes
-------
* Isotropic Voigt constants: C11 = C33 = rho vp^2, C55 = rho vs^2,
  C13 = C11 - 2 C55.
* VTI constants from Thomsen parameters: C33 = rho vp0^2, C55 = rho vs0^2,
  C11 = C33 (1 + 2 eps), C13 = sqrt(2 delta C33 (C33 - C55) + (C33 - C55)^2) - C55.
* Smooth random field: white N(0, 1) on the grid, periodic Gaussian filter of
  standard deviation `ell` cells, standardised to zero mean and unit standard
  deviation, times `std`.
* Random-layered relative contrast (one draw per map, in the order C11, C13,
  C33, C55, rho): 6 layer offsets U(-0.10, 0.10) with layer l covering rows
  [round(l nz / 6), round((l + 1) nz / 6)), plus a smooth random field of
  std 0.05 and ell 10 cells.  Absolute maps are q_p * m0_p.
* Sources: vertical unit forces at iz = 0, ix = floor((s + 1/2) nx / ns).
  Receivers: iz = 0, ix = round(r (nx - 1) / (nr - 1)).
"""

import math

import numpy as np
import scipy.ndimage

MAP_ORDER = ("C11", "C13", "C33", "C55", "rho")


# ---------------------------------------------------------------- media ----
def iso_voigt(vp, vs, rho):
    C11 = rho * vp * vp
    C55 = rho * vs * vs
    return (C11, C11 - 2.0 * C55, C11, C55)


def thomsen_voigt(vp0, vs0, eps, delta, rho):
    C33 = rho * vp0 * vp0
    C55 = rho * vs0 * vs0
    C11 = C33 * (1.0 + 2.0 * eps)
    C13 = math.sqrt(2.0 * delta * C33 * (C33 - C55) + (C33 - C55) ** 2) - C55
    return (C11, C13, C33, C55)


VTI_BACKGROUND = dict(vp0=2500.0, vs0=1200.0, eps=0.15, delta=0.05, rho=2200.0)


def vti_background():
    b = VTI_BACKGROUND
    return thomsen_voigt(b["vp0"], b["vs0"], b["eps"], b["delta"], b["rho"]), b["rho"]


def model_scales(c0, rho0):
    """m0 = (C11, C13, C33, C55, rho) of the background, shape [5, 1, 1]."""
    return np.array(list(c0) + [rho0], dtype=float)[:, None, None]


# --------------------------------------------------------------- fields ----
def smooth_random(rng, nz, nx, ell, std):
    w = rng.standard_normal((nz, nx))
    f = scipy.ndimage.gaussian_filter(w, sigma=ell, mode="wrap")
    f = (f - f.mean()) / f.std()
    return std * f


def random_layered(seed, nz, nx, nlayers=6, offset=0.10, std=0.05, ell=10):
    rng = np.random.default_rng(seed)
    q = np.empty((5, nz, nx))
    bounds = [int(round(l * nz / nlayers)) for l in range(nlayers + 1)]
    for p in range(5):
        o = rng.uniform(-offset, offset, size=nlayers)
        layer = np.empty(nz)
        for l in range(nlayers):
            layer[bounds[l]:bounds[l + 1]] = o[l]
        n = smooth_random(rng, nz, nx, ell, std)
        q[p] = layer[:, None] + n
    return q


def smooth_maps(seed, nz, nx, ell, std):
    rng = np.random.default_rng(seed)
    return np.stack([smooth_random(rng, nz, nx, ell, std) for _ in range(5)])


def gaussian_blob(nz, nx, cz, cx, sigma, peak):
    z = np.arange(nz)[:, None]
    x = np.arange(nx)[None, :]
    r2 = (z - cz) ** 2 + (x - cx) ** 2
    return peak * np.exp(-r2 / (2.0 * sigma * sigma))


def resample_periodic(q, nz, nx):
    """Periodic bilinear resampling of maps [..., NZ, NX] onto [..., nz, nx]."""
    NZ, NX = q.shape[-2:]
    zs = np.arange(nz) * (NZ / nz)
    xs = np.arange(nx) * (NX / nx)
    z0 = np.floor(zs).astype(int)
    x0 = np.floor(xs).astype(int)
    tz = (zs - z0)[:, None]
    tx = (xs - x0)[None, :]
    z1 = (z0 + 1) % NZ
    x1 = (x0 + 1) % NX
    a = q[..., z0[:, None], x0[None, :]]
    b = q[..., z0[:, None], x1[None, :]]
    c = q[..., z1[:, None], x0[None, :]]
    d = q[..., z1[:, None], x1[None, :]]
    return (1 - tz) * ((1 - tx) * a + tx * b) + tz * ((1 - tx) * c + tx * d)


def complex_normal(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def round_f32(a):
    """The float32 (or complex64) representable copy of a, kept in 64-bit."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return a.astype(np.complex64).astype(np.complex128)
    return a.astype(np.float32).astype(np.float64)


# ------------------------------------------------------ sources, receivers --
def surface_sources(nx, ns, iz=0, force=(0.0, 1.0)):
    ixz = [(int(math.floor((s + 0.5) * nx / ns)), iz) for s in range(ns)]
    f = [tuple(float(c) for c in force)] * ns
    return ixz, f


def surface_receivers(nx, nr, iz=0):
    if nr == 1:
        return [(0, iz)]
    return [(int(round(r * (nx - 1) / (nr - 1))), iz) for r in range(nr)]


# ------------------------------------------------------------ workloads ----
def problem_dict(nx, nz, dx, c0, rho0, freq_hz, eta, maps, src_ixz, src_f):
    return dict(nx=nx, nz=nz, dx=dx, c0=tuple(c0), rho0=rho0, freq_hz=freq_hz,
                eta=eta, maps=maps, src_ixz=src_ixz, src_f=src_f, nsys=len(src_ixz))


def iso32_blob():
    """32^2 isotropic, Gaussian blob contrast, one vertical force at the centre, 10 Hz."""
    nx = nz = 32
    c0 = iso_voigt(2000.0, 1000.0, 2000.0)
    rho0 = 2000.0
    q = gaussian_blob(nz, nx, 16, 16, 4.0, 0.10)
    maps = round_f32(model_scales(c0, rho0) * q[None])
    return problem_dict(nx, nz, 10.0, c0, rho0, 10.0, 0.02, maps, [(16, 16)], [(0.0, 1.0)])


def vti256_layered(nsrc=16):
    """256^2 VTI at 8 m, random-layered contrast (seed 1), 16 surface forces, 5 Hz."""
    nx = nz = 256
    c0, rho0 = vti_background()
    q = random_layered(1, nz, nx)
    maps = round_f32(model_scales(c0, rho0) * q)
    src, f = surface_sources(nx, nsrc)
    return problem_dict(nx, nz, 8.0, c0, rho0, 5.0, 0.02, maps, src, f)


FOUR_GRIDS = ((128, 37.5, 4.0), (192, 25.0, 6.0), (256, 18.75, 8.0), (384, 12.5, 12.0))


def four_grids(nsrc=64):
    """Four (grid, frequency) problems over one 4800 m square, 64 forces each."""
    c0, rho0 = vti_background()
    q384 = random_layered(2, 384, 384)
    out = []
    for n, dx, f in FOUR_GRIDS:
        q = q384 if n == 384 else resample_periodic(q384, n, n)
        maps = round_f32(model_scales(c0, rho0) * q)
        src, fv = surface_sources(n, nsrc)
        out.append(problem_dict(n, n, dx, c0, rho0, f, 0.02, maps, src, fv))
    return out


def vti512_jacobian(n=512, dx=5.0, nsrc=32, nrec=101, freqs=(5.0, 8.0)):
    """J / J* workload: reference contrast, perturbation, data and FD direction."""
    c0, rho0 = vti_background()
    qb = random_layered(3, n, n)
    maps = round_f32(model_scales(c0, rho0) * qb)
    src, fv = surface_sources(n, nsrc)
    rec = surface_receivers(n, nrec)
    probs = [problem_dict(n, n, dx, c0, rho0, f, 0.02, maps, src, fv) for f in freqs]
    dq = round_f32(smooth_maps(4, n, n, 10, 0.01))
    r = [round_f32(complex_normal(5 + 100 * k, (nsrc, nrec, 2))) for k in range(len(freqs))]
    d = round_f32(smooth_maps(6, n, n, 10, 1.0))
    return dict(problems=probs, rec_ixz=rec, dq=dq, r=r, d=d, lam=1e-3,
                reg="laplacian", m0=model_scales(c0, rho0))


def vti1024_normal(n=1024, dx=5.0, nsrc=128, nrec=201, freqs=(4.0, 7.0, 10.0)):
    """Normal-equation CG workload: smooth background contrast and truth."""
    c0, rho0 = vti_background()
    qb = smooth_maps(7, n, n, 20, 0.08)
    maps = round_f32(model_scales(c0, rho0) * qb)
    src, fv = surface_sources(n, nsrc)
    rec = surface_receivers(n, nrec)
    probs = [problem_dict(n, n, dx, c0, rho0, f, 0.02, maps, src, fv) for f in freqs]
    dq_true = round_f32(smooth_maps(8, n, n, 10, 0.02))
    return dict(problems=probs, rec_ixz=rec, dq_true=dq_true, lam=1e-3, reg="identity",
                m0=model_scales(c0, rho0), cg_iters=20)


def reservoir_dbi(nx=192, nz=48, dx=20.0, nsrc=48, nrec=96, freqs=(3.0, 5.0, 7.0, 9.0, 11.0, 13.0, 15.0, 17.0, 19.0),
                  seed=9, smooth=15.0):
    """Stand-in for the paper's 2-D VTI reservoir inversion (its model is not
    available): a VTI background with random-layered perturbations of all five
    parameters (seed 9: layer offsets within 10 %, 2 % smooth noise) on 192 x 48
    cells of 20 m (the 2^a 3^b grid nearest the example's 180 x 45), the
    starting model its periodic Gaussian smoothing with sigma 15 cells, 48
    vertical surface forces, 96 surface receivers and nine frequencies from
    3 to 19 Hz, inverted one after the other."""
    c0, rho0 = vti_background()
    m0 = model_scales(c0, rho0)
    q_true = random_layered(seed, nz, nx, nlayers=6, offset=0.10, std=0.02, ell=6)
    q_start = scipy.ndimage.gaussian_filter(q_true, sigma=(0, smooth, smooth), mode="wrap")
    src_ixz, src_f = surface_sources(nx, nsrc, iz=1)
    rec = surface_receivers(nx, nrec, iz=1)
    return dict(nx=nx, nz=nz, dx=dx, c0=c0, rho0=rho0, eta=0.02, freqs=tuple(freqs), m0=m0.ravel(),
                c_true=round_f32(m0 * q_true), c_start=round_f32(m0 * q_start), src_ixz=src_ixz, src_f=src_f,
                rec=rec)


# ------------------------------------------------------------------ 3-D ----
# Inputs of the 3-D problems: a general background given by the 21 constants
# of the upper triangle of its 6 x 6 Voigt matrix (row by row), contrast maps
# [nmaps, nz, ny, nx] and sources / receivers (ix, iy, iz).
#
# * VTI background from Thomsen parameters with C66 = C55 (1 + 2 gamma): the
#   6 x 6 matrix with C22 = C11, C12 = C11 - 2 C66, C23 = C13, C44 = C55.
# * A "triclinic" background: that VTI matrix plus a seeded random symmetric
#   perturbation of every entry (relative size `scale` of C33), kept only if
#   positive definite (redrawn otherwise).
# * Smooth random 3-D fields: the 2-D recipe with a 3-D periodic filter.
# * The stand-in for the paper's modified 3-D VTI Hess model (not available):
#   80 x 40 x 32 cells of 25 m, VTI background with C66 = C55, six contrast
#   maps (C11, C13, C33, C55, C66, rho) made of 4 flat layers (offsets
#   U(-0.10, 0.10)) plus smooth noise (std 0.03, ell 4 cells) relative to the
#   background constants, 100 vertical forces on a 10 x 10 surface grid and
#   400 receivers on a 20 x 20 surface grid.
def vti_voigt_upper(C11, C13, C33, C55, C66):
    """The 21 upper-triangle constants of a VTI stiffness."""
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = C11
    C[0, 1] = C[1, 0] = C11 - 2.0 * C66
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[2, 2] = C33
    C[3, 3] = C[4, 4] = C55
    C[5, 5] = C66
    return C[np.triu_indices(6)]


def vti3d_background(gamma=0.0):
    """21 constants and rho of the VTI background; C66 = C55 (1 + 2 gamma)."""
    (C11, C13, C33, C55), rho = vti_background()
    return vti_voigt_upper(C11, C13, C33, C55, C55 * (1.0 + 2.0 * gamma)), rho


def vti3d_scales(gamma=0.0):
    """(C11, C13, C33, C55, C66, rho) of the VTI background, shape [6, 1, 1, 1]."""
    (C11, C13, C33, C55), rho = vti_background()
    return np.array([C11, C13, C33, C55, C55 * (1.0 + 2.0 * gamma), rho])[:, None, None, None]


def triclinic_background(seed, scale=0.08):
    """21 constants of a positive definite 6 x 6 stiffness near the VTI one, and rho."""
    c21, rho = vti3d_background(gamma=0.1)
    C = np.zeros((6, 6))
    C[np.triu_indices(6)] = c21
    C = C + np.triu(C, 1).T
    rng = np.random.default_rng(seed)
    while True:
        R = rng.standard_normal((6, 6))
        Cp = C + scale * C[2, 2] * (R + R.T) / 2.0
        if np.all(np.linalg.eigvalsh(Cp) > 0.05 * C[2, 2]):
            return Cp[np.triu_indices(6)], rho


def smooth_random3(rng, nz, ny, nx, ell, std):
    w = rng.standard_normal((nz, ny, nx))
    f = scipy.ndimage.gaussian_filter(w, sigma=ell, mode="wrap")
    sd = f.std()
    f = (f - f.mean()) / (sd if sd > 0 else 1.0)
    return std * f


def contrast3(seed, nz, ny, nx, scales, ell=2.0, std=0.05):
    """Smooth random relative contrast times the per-map scales [nmaps, 1, 1, 1]."""
    rng = np.random.default_rng(seed)
    q = np.array([smooth_random3(rng, nz, ny, nx, ell, std) for _ in range(scales.shape[0])])
    return q * scales


def general_scales(c21, rho):
    """Per-map scale of a 21-constant contrast: C33 of the background for
    every constant (off-diagonal ones are often zero in the background), rho."""
    c33 = float(c21[12])
    return np.array([c33] * 21 + [rho])[:, None, None, None]


def surface_grid(nx, ny, n1, n2, iz=0):
    """n1 x n2 points evenly spread over the top face, (ix, iy, iz)."""
    xs = [int(math.floor((i + 0.5) * nx / n1)) for i in range(n1)]
    ys = [int(math.floor((j + 0.5) * ny / n2)) for j in range(n2)]
    return [(x, y, iz) for y in ys for x in xs]


def hess3d_vti(nsrc=(10, 10), nrec=(20, 20), freq_hz=7.0, seed=12):
    """80 x 40 x 32, 25 m cells: the stand-in for the modified 3-D VTI Hess example."""
    nx, ny, nz, dx = 80, 40, 32, 25.0
    c21, rho = vti3d_background(gamma=0.0)
    scales = vti3d_scales(gamma=0.0)
    rng = np.random.default_rng(seed)
    q = np.zeros((6, nz, ny, nx))
    for p in range(6):
        off = rng.uniform(-0.10, 0.10, 4)
        for layer in range(4):
            q[p, round(layer * nz / 4):round((layer + 1) * nz / 4)] += off[layer]
        q[p] += smooth_random3(rng, nz, ny, nx, 4.0, 0.03)
    maps = round_f32(q * scales)
    src = surface_grid(nx, ny, *nsrc)
    rec = surface_grid(nx, ny, *nrec, iz=1)
    return dict(nx=nx, ny=ny, nz=nz, dx=dx, c0=c21, rho0=rho, freq_hz=freq_hz, eta=0.02, params="vti",
                maps=maps, src_ixyz=src, src_f=[(0.0, 0.0, 1.0)] * len(src), rec_ixyz=rec, nsys=len(src),
                scales=scales)
