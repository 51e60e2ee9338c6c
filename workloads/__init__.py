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
