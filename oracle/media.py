"""Stiffness in abbreviated-subscript (Voigt) form, the VTI matrix and the B
matrices of the stiffness decomposition.

Paper passages: the abbreviated subscript section (6x6 stiffness, Voigt strain
vector, VTI matrix with C12 = C11 - 2 C66), eq. dC (delta C = sum_p B^(p)
delta m^(p)) and App. C (the VTI B matrices).

Conventions (0-based): tensor indices x=0, y=1, z=2; Voigt indices
0..5 = (xx, yy, zz, yz, xz, xy).  Strains are engineering strains, so the
Voigt strain vector is (d1u1, d2u2, d3u3, d2u3+d3u2, d1u3+d3u1, d1u2+d2u1).

The 2-D problem lives in the x-z plane (u_y = 0, d/dy = 0), and the 2-D
parameter set is (C11, C13, C33, C55, rho), stored in that order.
"""

import numpy as np

#: Voigt index of the symmetric tensor pair (i, j).
VOIGT_INDEX = np.array([[0, 5, 4],
                        [5, 1, 3],
                        [4, 3, 2]])

#: Order of the 2-D model maps.
MAP_NAMES = ("C11", "C13", "C33", "C55", "rho")


def voigt_to_tensor(C6):
    """Expand a 6x6 Voigt matrix into the 4th-rank tensor C_ijkl.

    C6 may carry trailing field axes ([6, 6, ...]); the result is
    [3, 3, 3, 3, ...].  C_ijkl = C6[V(i,j), V(k,l)] uses the symmetries
    C_ijkl = C_jikl = C_ijlk (abbreviated subscript section).
    """
    C6 = np.asarray(C6)
    V = VOIGT_INDEX
    return C6[V[:, :, None, None], V[None, None, :, :]]


def vti_voigt(C11, C33, C55, C66, C13):
    """The 6x6 VTI stiffness of the abbreviated subscript section.

    Five independent constants; C12 = C11 - 2 C66 and C44 = C55.
    """
    C12 = C11 - 2.0 * C66
    C = np.zeros((6, 6), dtype=np.result_type(C11, C33, C55, C66, C13, 1.0))
    C[0, 0] = C[1, 1] = C11
    C[0, 1] = C[1, 0] = C12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[2, 2] = C33
    C[3, 3] = C[4, 4] = C55
    C[5, 5] = C66
    return C


def vti_B_matrices():
    """The constant B matrices of App. C for the VTI parameters.

    Returned as a dict keyed '11', '33', '55', '66', '13'.  Each is the
    derivative of the VTI stiffness matrix with respect to that constant
    (C12 = C11 - 2 C66 puts +1 entries into B^11 and -2 entries into B^66).
    """
    B = {k: np.zeros((6, 6)) for k in ("11", "33", "55", "66", "13")}
    B["11"][0:2, 0:2] = 1.0
    B["33"][2, 2] = 1.0
    B["55"][3, 3] = 1.0
    B["55"][4, 4] = 1.0
    B["66"][0, 1] = B["66"][1, 0] = -2.0
    B["66"][5, 5] = 1.0
    B["13"][0, 2] = B["13"][1, 2] = B["13"][2, 0] = B["13"][2, 1] = 1.0
    return B


def voigt_2d(C11, C13, C33, C55):
    """Background 6x6 stiffness for the 2-D parameter set.

    The in-plane (x-z) behaviour depends only on C11, C13, C33 and C55; C66
    only enters through C12, which multiplies the out-of-plane strain and is
    inert in 2-D.  We take C66 = C55 so that the matrix is a valid VTI one.
    """
    return vti_voigt(C11, C33, C55, C55, C13)


def contrast_voigt_2d(dC11, dC13, dC33, dC55):
    """Stiffness contrast field delta C(x) = sum_p B^(p) delta m^(p)(x), eq. dC.

    The four 2-D maps are combined with the App. C matrices B^11, B^13, B^33
    and B^55.  Returns a [6, 6, nz, nx] field.
    """
    B = vti_B_matrices()
    out = (B["11"][:, :, None, None] * np.asarray(dC11)[None, None]
           + B["13"][:, :, None, None] * np.asarray(dC13)[None, None]
           + B["33"][:, :, None, None] * np.asarray(dC33)[None, None]
           + B["55"][:, :, None, None] * np.asarray(dC55)[None, None])
    return out


def map_B_matrices_2d():
    """B matrices in the order of the 2-D stiffness maps (C11, C13, C33, C55)."""
    B = vti_B_matrices()
    return [B["11"], B["13"], B["33"], B["55"]]
