"""Slow, plain CPU oracle for the matrix-free elastic Lippmann-Schwinger method.

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it.  The product library never
calls into it and shares no code with it: the HIP path has its own kernels,
headers and constants, and the oracle has its own numpy/scipy implementation
written directly from the paper (Xiang, Jakobsen, Shekhar, Eikrem and Naevdal,
"Efficient scattering approach to seismic full-waveform inversion in
anisotropic elastic media with variable density", arXiv 2402.02116).

Everything here runs in complex128 / float64 on the CPU.  Functions cite the
section or equation label of the paper they restate.

Modules
-------
media      Voigt stiffness, the VTI matrix and the B matrices (abbreviated
           subscript section, App. C).
green      Wavenumber-domain Green's tensor from the general 4-index
           Christoffel matrix (eq. Green), the isotropic closed form and the
           analytic 2-D Hankel form (App. A).
operators  Finite-difference strain / divergence, body force, FFT
           convolution (eq. FFT), the LS operator (eqs. A, axb), incident field
           (eq. u0), receiver sampling.
krylov     Textbook BiCGSTAB and CG.
problem    One (grid, background, contrast) problem with its solves, the
           Frechet operator (eqs. F, YM, F0, uY) and the adjoint (eqs. ad1, ua).
tikhonov   Generalised Tikhonov objective, gradient and normal-equation CG
           (eqs. obj, norm).
dbi        One frequency stage of the distorted-Born iteration: background
           solve, normalised data error, normal-equation CG, model update,
           self-adaptive lambda cooling and the stopping rule.
dense      Explicit matrices for the pins: the dense Green's matrix from a
           direct DFT sum and the sparse discrete elastic operator (eq. Ewave).
elastic3d  The 3-D, generally anisotropic form: 21-constant stiffness and
           its B matrices (eq. dC), the VTI set with C66 (App. C), the 3x3
           Christoffel inverse, 6-strain stencils, one LS problem with its
           solves, J and J*.
dense3d    Explicit 3-D matrices for its pins (direct-DFT Green's matrix,
           Kronecker-assembled E_h, the discrete 3-D eq. Ewave).

Parity pins for every function live in tests/test_oracle_*.py.
"""

from . import media, green, operators, krylov, problem, tikhonov, dbi, dense, elastic3d, dense3d  # noqa: F401
from .problem import LSProblem  # noqa: F401
