"""ctypes loader for libfwils.so and the C declarations of include/fwils.h.

Loading never falls back to anything: if the library is missing or cannot be
loaded, FwilsLibraryError is raised.
"""

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwils.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fwils.h")

c_int32, c_double, c_size_t, c_void_p, c_uint32, c_int64 = (
    ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int64)

FWILS_OK, FWILS_EINVAL, FWILS_ENOMEM, FWILS_EDEVICE, FWILS_ENOCONV, FWILS_EBREAKDOWN, FWILS_EUNSUPPORTED = range(7)
FWILS_C64 = 0
FWILS_C128 = 1
FWILS_SYMBOL_SPECTRAL, FWILS_SYMBOL_CENTRAL = 0, 1
FWILS_SOLVE_X0, FWILS_SOLVE_PLAIN, FWILS_SOLVE_NOGRAPH, FWILS_SOLVE_SCATTERED = 0x1, 0x2, 0x4, 0x8
FWILS_ADJ_ACCUMULATE = 0x1
FWILS_REG_IDENTITY, FWILS_REG_LAPLACIAN = 0, 1


class FwilsProblem(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("nz", c_int32), ("dx", c_double), ("c0", c_double * 4),
                ("rho0", c_double), ("freq_hz", c_double), ("damping", c_double),
                ("nsys", c_int32), ("symbol", c_int32)]


class FwilsProblem3(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("dx", c_double), ("c0", c_double * 21),
                ("rho0", c_double), ("freq_hz", c_double), ("damping", c_double), ("nsys", c_int32),
                ("symbol", c_int32), ("params", c_int32)]


FWILS_PARAMS_VTI, FWILS_PARAMS_GENERAL = 0, 1


class FwilsTuning(ctypes.Structure):
    _fields_ = [("row_points", c_int32), ("col_points", c_int32), ("col_width", c_int32),
                ("col_shared", c_int32), ("stencil_rows", c_int32), ("stencil_sys", c_int32),
                ("fused_points", c_int32), ("row_points_inv", c_int32), ("time_us", ctypes.c_float * 4)]

    FIELDS = ("row_points", "col_points", "col_width", "col_shared", "stencil_rows", "stencil_sys",
              "fused_points", "row_points_inv")

    def to_dict(self):
        d = {k: int(getattr(self, k)) for k in self.FIELDS}
        d["time_us"] = [float(x) for x in self.time_us]
        return d


FWILS_TUNE_STENCIL, FWILS_TUNE_ROWS, FWILS_TUNE_COLS, FWILS_TUNE_FUSE = 0, 1, 2, 3
FWILS_KRYLOV_BICGSTAB, FWILS_KRYLOV_GMRES = 0, 1
FWILS_GMRES_CGS1 = 0x1

P = c_void_p
SIGNATURES = {
    "fwils_plan_create": (c_int32, [ctypes.POINTER(FwilsProblem), c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "fwils_plan_create3": (c_int32, [ctypes.POINTER(FwilsProblem3), c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "fwils_plan_destroy": (None, [P]),
    "fwils_workspace_size": (c_int32, [P, ctypes.POINTER(c_size_t)]),
    "fwils_set_workspace": (c_int32, [P, P, c_size_t]),
    "fwils_set_stream": (c_int32, [P, P]),
    "fwils_field_elems": (c_int32, [P, ctypes.POINTER(c_int64)]),
    "fwils_set_contrast": (c_int32, [P, c_int32, P]),
    "fwils_set_receivers": (c_int32, [P, c_int32, ctypes.POINTER(c_int32), c_int32]),
    "fwils_incident": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_double), P]),
    "fwils_body_force": (c_int32, [P, P, P]),
    "fwils_convolve": (c_int32, [P, P, P]),
    "fwils_apply": (c_int32, [P, P, P]),
    "fwils_apply_noalloc": (c_int32, [P, P, P]),
    "fwils_solve": (c_int32, [P, P, P, c_double, c_int32, P, P, c_uint32]),
    "fwils_frechet": (c_int32, [P, P, ctypes.POINTER(c_void_p), P, c_double, c_int32]),
    "fwils_adjoint": (c_int32, [P, P, P, ctypes.POINTER(c_void_p), c_uint32, c_double, c_int32]),
    "fwils_fft2": (c_int32, [P, c_int32, P, P, c_int32]),
    "fwils_apply_pass": (c_int32, [P, c_int32, P, P]),
    "fwils_time_pass": (c_int32, [P, c_int32, P, P, c_int32, ctypes.POINTER(ctypes.c_float)]),
    "fwils_time_krylov_pass": (c_int32, [P, c_int32, ctypes.POINTER(ctypes.c_float)]),
    "fwils_time_gmres_pass": (c_int32, [P, c_int32, c_int32, c_int32, ctypes.POINTER(ctypes.c_float)]),
    "fwils_tikhonov_grad": (c_int32, [P, P, P, ctypes.POINTER(c_double), c_double, c_int32, P, P,
                                      ctypes.POINTER(c_double), P, c_double, c_int32]),
    "fwils_normal_apply": (c_int32, [P, P, ctypes.POINTER(c_double), c_double, c_double, c_int32, P, P, P,
                                     c_double, c_int32]),
    "fwils_normal_cg": (c_int32, [P, P, P, ctypes.POINTER(c_double), c_double, c_int32, c_int32, P,
                                  ctypes.POINTER(c_double), P, c_double, c_int32]),
    "fwils_normal_cg_steps": (c_int32, [P, P, P, ctypes.POINTER(c_double), c_double, c_int32, c_int32, c_int32, P,
                                        ctypes.POINTER(c_double), P, P, c_double, c_int32]),
    "fwils_frechet_rel": (c_int32, [P, P, P, ctypes.POINTER(c_double), P, c_double, c_int32]),
    "fwils_adjoint_rel": (c_int32, [P, P, P, ctypes.POINTER(c_double), P, c_double, c_int32]),
    "fwils_laplacian": (c_int32, [P, P, P]),
    "fwils_receiver_data": (c_int32, [P, P, P]),
    "fwils_get_contrast": (c_int32, [P, c_int32, P]),
    "fwils_dbi_run": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_double), P, ctypes.POINTER(c_double),
                                c_double, c_int32, c_int32, c_double, c_int32, P, P, P, P,
                                ctypes.POINTER(c_double), ctypes.POINTER(c_double), ctypes.POINTER(c_int32),
                                c_double, c_int32]),
    "fwils_solve_stats": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "fwils_solve_status": (c_int32, [P, ctypes.POINTER(c_int32)]),
    "fwils_autotune": (c_int32, [P, c_int32]),
    "fwils_gmres_workspace_size": (c_int32, [P, c_int32, ctypes.POINTER(c_size_t)]),
    "fwils_set_krylov": (c_int32, [P, c_int32, c_int32, c_uint32, P, c_size_t]),
    "fwils_get_tuning": (c_int32, [P, c_int32, ctypes.POINTER(FwilsTuning)]),
    "fwils_set_tuning": (c_int32, [P, c_int32, ctypes.POINTER(FwilsTuning)]),
    "fwils_tuning_candidates": (c_int32, [P, c_int32, c_int32, ctypes.POINTER(FwilsTuning), c_int32,
                                          ctypes.POINTER(c_int32)]),
    "fwils_status_string": (ctypes.c_char_p, [c_int32]),
    "fwils_last_error": (ctypes.c_char_p, []),
    "fwils_abi_version": (c_int32, []),
}


class FwilsLibraryError(RuntimeError):
    pass


class FwilsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


_LIB = None


def header_functions(path=HEADER):
    """Names of the functions declared in include/fwils.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fwils_[a-z0-9_]+)\s*\(", txt)))


def load(path=LIB_PATH):
    """Load libfwils.so (cached for the default path) and declare every entry point."""
    global _LIB
    if path == LIB_PATH and _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise FwilsLibraryError(
            f"{path} is not built; run `python -m paper_2402_02116_amd.build` (hipcc, gfx950)")
    try:
        lib = ctypes.CDLL(path)
    except OSError as e:
        raise FwilsLibraryError(f"cannot load {path}: {e}") from e
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _LIB = lib
    return lib


def check(status, what=""):
    """Raise FwilsError for any status other than FWILS_OK."""
    if status == FWILS_OK:
        return
    lib = load()
    msg = lib.fwils_last_error().decode(errors="replace")
    name = lib.fwils_status_string(status).decode()
    raise FwilsError(status, f"{what}: {name} ({status}): {msg}")
