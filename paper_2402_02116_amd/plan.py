"""Python binding of the fwils C ABI (include/fwils.h).

Argument marshalling only: every computation runs in the HIP kernels of
libfwils.so.  PyTorch supplies device memory (the workspace and the fields)
and the stream: each call enqueues on torch's current stream of the plan's
device.

Field tensors are flat complex CUDA tensors holding the plan-level field
(problems concatenated, each [nsys][2][nz][nx]); `view(t, i)` gives problem i
as a [nsys, 2, nz, nx] view.  A plan is complex64 with float32 maps
(precision "c64", the default) or complex128 with float64 maps ("c128", the
FP64 reference of the same kernels); `cdtype` / `rdtype` are its types.
"""

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check

SYMBOLS = {"spectral": _lib.FWILS_SYMBOL_SPECTRAL, "central": _lib.FWILS_SYMBOL_CENTRAL}
PRECISIONS = {"c64": (_lib.FWILS_C64, torch.complex64, torch.float32),
              "c128": (_lib.FWILS_C128, torch.complex128, torch.float64)}


@dataclass
class SolveResult:
    x: torch.Tensor           # flat field
    iters: np.ndarray         # [sum nsys] int32
    relres: np.ndarray        # [sum nsys] true relative residual
    status: int               # FWILS_OK / FWILS_ENOCONV / FWILS_EBREAKDOWN


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """One or more (grid, frequency) problems solved together."""

    CSTRIDE = 2   # ints per source / receiver cell, doubles per force

    def __init__(self, problems, device="cuda", precision="c64"):
        self.lib = _lib.load()
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        prec, self.cdtype, self.rdtype = PRECISIONS[precision]
        if not torch.cuda.is_available():
            raise RuntimeError("fwils needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.problems = [dict(p) for p in problems]
        n = len(self.problems)
        arr = (_lib.FwilsProblem * n)()
        for i, p in enumerate(self.problems):
            arr[i].nx, arr[i].nz = int(p["nx"]), int(p["nz"])
            arr[i].dx = float(p["dx"])
            for k in range(4):
                arr[i].c0[k] = float(p["c0"][k])
            arr[i].rho0 = float(p["rho0"])
            arr[i].freq_hz = float(p["freq_hz"])
            arr[i].damping = float(p.get("eta", p.get("damping", 0.02)))
            arr[i].nsys = int(p["nsys"])
            sym = p.get("symbol", "spectral")
            arr[i].symbol = SYMBOLS[sym] if isinstance(sym, str) else int(sym)
        h = ctypes.c_void_p()
        check(self.lib.fwils_plan_create(arr, n, prec, ctypes.byref(h)), "fwils_plan_create")
        self._attach(h)

    def _sys_elems(self, p):
        """Complex elements of one system's field."""
        return 2 * p["nz"] * p["nx"]

    def _attach(self, h):
        """Workspace, stream and the plan-level offsets of a created plan."""
        n = len(self.problems)
        self._h = h
        size = ctypes.c_size_t()
        check(self.lib.fwils_workspace_size(h, ctypes.byref(size)), "fwils_workspace_size")
        self.workspace_bytes = size.value
        with torch.cuda.device(self.device):
            raw = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._ws_raw = raw
        self._ws_ptr = raw.data_ptr() + off
        self._bind_stream()
        check(self.lib.fwils_set_workspace(h, ctypes.c_void_p(self._ws_ptr), size.value),
              "fwils_set_workspace")
        fe = ctypes.c_int64()
        check(self.lib.fwils_field_elems(h, ctypes.byref(fe)), "fwils_field_elems")
        self.field_elems = fe.value
        self.offsets, self.sys_offsets = [], []
        o = so = 0
        for p in self.problems:
            self.offsets.append(o)
            self.sys_offsets.append(so)
            o += p["nsys"] * self._sys_elems(p)
            so += p["nsys"]
        self.total_sys = so
        self.nrec = [0] * n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.fwils_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------ helpers --
    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.fwils_set_stream(self._h, ctypes.c_void_p(s)), "fwils_set_stream")

    def new_field(self):
        return torch.zeros(self.field_elems, dtype=self.cdtype, device=self.device)

    def _out_field(self):
        # an output the library writes in full (no fill kernel before the call)
        return torch.empty(self.field_elems, dtype=self.cdtype, device=self.device)

    def view(self, t, i):
        p = self.problems[i]
        n = p["nsys"] * self._sys_elems(p)
        return t[self.offsets[i]:self.offsets[i] + n].view(p["nsys"], *self._field_shape(p))

    def _field_shape(self, p):
        return (2, p["nz"], p["nx"])

    def pack(self, parts):
        """Concatenate per-problem [nsys, 2, nz, nx] arrays into a plan-level field."""
        flat = [torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x)
                .to(self.cdtype).reshape(-1) for x in parts]
        return torch.cat(flat).to(self.device).contiguous()

    def _field(self, t, name):
        _require_cuda(t, self.cdtype, name)
        if t.numel() != self.field_elems:
            raise ValueError(f"{name} has {t.numel()} elements, the plan's fields have {self.field_elems}")
        return t

    def data_elems(self):
        return sum(p["nsys"] * nr * 2 for p, nr in zip(self.problems, self.nrec))

    def data_view(self, d, i):
        p = self.problems[i]
        off = sum(q["nsys"] * nr * 2 for q, nr in zip(self.problems[:i], self.nrec[:i]))
        return d[off:off + p["nsys"] * self.nrec[i] * 2].view(p["nsys"], self.nrec[i], 2)

    # ---------------------------------------------------------- the ABI ----
    def set_contrast(self, i, maps):
        p = self.problems[i]
        m = torch.as_tensor(maps, dtype=self.rdtype).to(self.device).contiguous()
        if tuple(m.shape) != (5, p["nz"], p["nx"]):
            raise ValueError(f"maps must be [5, {p['nz']}, {p['nx']}]")
        self._bind_stream()
        check(self.lib.fwils_set_contrast(self._h, i, _ptr(m)), "fwils_set_contrast")
        torch.cuda.current_stream(self.device).synchronize()

    def set_receivers(self, i, rec_ixz):
        r = np.ascontiguousarray(np.asarray(rec_ixz, dtype=np.int32).reshape(-1, 2))
        self._bind_stream()
        check(self.lib.fwils_set_receivers(self._h, i, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           r.shape[0]), "fwils_set_receivers")
        self.nrec[i] = r.shape[0]

    def incident(self, src_ixz, src_f):
        s = np.ascontiguousarray(np.asarray(src_ixz, dtype=np.int32).reshape(-1, 2))
        f = np.ascontiguousarray(np.asarray(src_f, dtype=np.float64).reshape(-1, 2))
        if s.shape[0] != self.total_sys or f.shape[0] != self.total_sys:
            raise ValueError(f"need {self.total_sys} sources and forces")
        u0 = self._out_field()
        self._bind_stream()
        check(self.lib.fwils_incident(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(u0)),
              "fwils_incident")
        return u0

    def body_force(self, u, out=None):
        self._field(u, "u")
        out = self.new_field() if out is None else self._field(out, "out")
        self._bind_stream()
        check(self.lib.fwils_body_force(self._h, _ptr(u), _ptr(out)), "fwils_body_force")
        return out

    def convolve(self, f, out=None):
        self._field(f, "f")
        out = self.new_field() if out is None else self._field(out, "out")
        self._bind_stream()
        check(self.lib.fwils_convolve(self._h, _ptr(f), _ptr(out)), "fwils_convolve")
        return out

    def apply(self, u, out=None):
        self._field(u, "u")
        out = self.new_field() if out is None else self._field(out, "out")
        self._bind_stream()
        check(self.lib.fwils_apply(self._h, _ptr(u), _ptr(out)), "fwils_apply")
        return out

    def apply_noalloc(self, u, out=None):
        """apply() with the library's static scratch instead of the workspace's
        (fwils_apply_noalloc: no device allocation inside the call)."""
        self._field(u, "u")
        out = self.new_field() if out is None else self._field(out, "out")
        self._bind_stream()
        check(self.lib.fwils_apply_noalloc(self._h, _ptr(u), _ptr(out)), "fwils_apply_noalloc")
        return out

    def solve(self, rhs, x0=None, rtol=1e-6, maxit=1000, plain=False, graph=True, out=None,
              strict=False, scattered=False):
        """Krylov solve of A x = rhs with the plan's method (set_krylov); returns
        SolveResult (iters, true relres).  scattered=True: x is the solution
        minus rhs (the scattered field u - u0 when rhs = u0), formed by the
        library."""
        self._field(rhs, "rhs")
        flags = 0
        if x0 is not None:
            x = self._field(x0, "x0").clone() if out is None else out.copy_(x0)
            flags |= _lib.FWILS_SOLVE_X0
        else:
            x = self._out_field() if out is None else self._field(out, "out")
        if plain:
            flags |= _lib.FWILS_SOLVE_PLAIN
        if not graph:
            flags |= _lib.FWILS_SOLVE_NOGRAPH
        if scattered:
            flags |= _lib.FWILS_SOLVE_SCATTERED
        iters = torch.empty(self.total_sys, dtype=torch.int32, device=self.device)
        relres = torch.empty(self.total_sys, dtype=torch.float64, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_solve(self._h, _ptr(rhs), _ptr(x), float(rtol), int(maxit),
                                  _ptr(iters), _ptr(relres), flags)
        if st not in (_lib.FWILS_OK, _lib.FWILS_ENOCONV, _lib.FWILS_EBREAKDOWN) or (strict and st != 0):
            check(st, "fwils_solve")
        return SolveResult(x, iters.cpu().numpy(), relres.cpu().numpy(), st)

    def frechet(self, ub, dm, rtol=1e-6, maxit=1000):
        """J dm for every system; dm: list (one per problem) of rdtype [5, nz, nx]."""
        self._field(ub, "ub")
        dms = []
        for i, p in enumerate(self.problems):
            m = dm[i]
            _require_cuda(m, self.rdtype, f"dm[{i}]")
            if tuple(m.shape) != (5, p["nz"], p["nx"]):
                raise ValueError(f"dm[{i}] must be [5, {p['nz']}, {p['nx']}]")
            dms.append(m)
        arr = (ctypes.c_void_p * len(dms))(*[m.data_ptr() for m in dms])
        d = torch.empty(self.data_elems(), dtype=self.cdtype, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_frechet(self._h, _ptr(ub), arr, _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_frechet")
        return d

    def adjoint(self, ub, r, rtol=1e-6, maxit=1000, g=None, accumulate=False):
        """J* r: list (one per problem) of complex128 [5, nz, nx] maps (FP64 in
        both precisions: absolute-unit values lie below the float32 range)."""
        self._field(ub, "ub")
        _require_cuda(r, self.cdtype, "r")
        if r.numel() != self.data_elems():
            raise ValueError(f"r must hold {self.data_elems()} complex values")
        if g is None:
            if accumulate:
                raise ValueError("accumulate needs the g maps to add to")
            g = [torch.empty(5, p["nz"], p["nx"], dtype=torch.complex128, device=self.device)
                 for p in self.problems]
        for i, (gi, p) in enumerate(zip(g, self.problems)):
            _require_cuda(gi, torch.complex128, f"g[{i}]")
            if tuple(gi.shape) != (5, p["nz"], p["nx"]):
                raise ValueError(f"g[{i}] must be [5, {p['nz']}, {p['nx']}]")
        arr = (ctypes.c_void_p * len(g))(*[gi.data_ptr() for gi in g])
        self._bind_stream()
        st = self.lib.fwils_adjoint(self._h, _ptr(ub), _ptr(r), arr,
                                    _lib.FWILS_ADJ_ACCUMULATE if accumulate else 0,
                                    float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_adjoint")
        return g

    def apply_pass(self, k, u=None, out=None):
        """Pass k (0..3) of apply(); passes 0..3 in order compute apply(u)."""
        if u is not None:
            self._field(u, "u")
        if out is not None:
            self._field(out, "out")
        self._bind_stream()
        check(self.lib.fwils_apply_pass(self._h, int(k), None if u is None else _ptr(u),
                                        None if out is None else _ptr(out)), "fwils_apply_pass")
        return out

    def time_pass(self, k, u, out, reps=50):
        """Average duration (us) of pass k of apply() over reps back-to-back launches."""
        self._field(u, "u")
        self._field(out, "out")
        us = ctypes.c_float()
        self._bind_stream()
        check(self.lib.fwils_time_pass(self._h, int(k), _ptr(u), _ptr(out), int(reps), ctypes.byref(us)),
              "fwils_time_pass")
        return us.value

    def time_krylov_pass(self, reps=50):
        """Average duration (us) of the BiCGSTAB direction-update stencil pass
        with every system running, continuing from the last solve's state."""
        us = ctypes.c_float()
        self._bind_stream()
        check(self.lib.fwils_time_krylov_pass(self._h, int(reps), ctypes.byref(us)), "fwils_time_krylov_pass")
        return us.value

    GMRES_KINDS = {"update": 0, "dots": 1, "projections": 2}

    def time_gmres_pass(self, kind, j, reps=20):
        """Average duration (us) of one Arnoldi-step kernel ('update', 'dots' or
        'projections') at step j with every system running (GMRES plans)."""
        us = ctypes.c_float()
        self._bind_stream()
        check(self.lib.fwils_time_gmres_pass(self._h, self.GMRES_KINDS[kind], int(j), int(reps), ctypes.byref(us)),
              "fwils_time_gmres_pass")
        return us.value

    def solve_stats(self):
        """(iters, recursive relres) of the last Krylov solve, per system."""
        it = np.zeros(self.total_sys, dtype=np.int32)
        rr = np.zeros(self.total_sys, dtype=np.float64)
        check(self.lib.fwils_solve_stats(self._h, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "fwils_solve_stats")
        return it, rr

    SYS_STATUS = {0: "running", 1: "converged", 2: "maxit", 3: "breakdown", 4: "nonfinite"}

    def solve_status(self):
        """Per-system outcome of the last Krylov solve (names of SYS_STATUS)."""
        st = np.zeros(self.total_sys, dtype=np.int32)
        check(self.lib.fwils_solve_status(self._h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "fwils_solve_status")
        return [self.SYS_STATUS.get(int(v), "?") for v in st]

    # ------------------------------------------------- Tikhonov step ----
    REGS = {"identity": _lib.FWILS_REG_IDENTITY, "laplacian": _lib.FWILS_REG_LAPLACIAN}

    def _qshape(self):
        """Shape of the model maps of the Tikhonov step (the first problem's)."""
        p = self.problems[0]
        return (5, p["nz"], p["nx"])

    def _maps(self, q, name):
        _require_cuda(q, self.rdtype, name)
        if tuple(q.shape) != self._qshape():
            raise ValueError(f"{name} must be {list(self._qshape())}")
        return q

    def _m0(self, m0):
        a = np.ascontiguousarray(np.asarray(m0, dtype=np.float64).reshape(self._qshape()[0]))
        return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def _data(self, r, name):
        _require_cuda(r, self.cdtype, name)
        if r.numel() != self.data_elems():
            raise ValueError(f"{name} must hold {self.data_elems()} complex values")
        return r

    def frechet_rel(self, ub, q, m0, rtol=1e-6, maxit=1000):
        """d = J (m0 q) for relative maps q [5, nz, nx] (rdtype)."""
        self._field(ub, "ub")
        self._maps(q, "q")
        m, mp = self._m0(m0)
        d = torch.zeros(self.data_elems(), dtype=self.cdtype, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_frechet_rel(self._h, _ptr(ub), _ptr(q), mp, _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_frechet_rel")
        return d

    def adjoint_rel(self, ub, r, m0, rtol=1e-6, maxit=1000):
        """gq = m0 Re(J* r) summed over problems, rdtype [5, nz, nx]."""
        self._field(ub, "ub")
        self._data(r, "r")
        m, mp = self._m0(m0)
        p = self.problems[0]
        gq = torch.zeros(self._qshape(), dtype=self.rdtype, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_adjoint_rel(self._h, _ptr(ub), _ptr(r), mp, _ptr(gq), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_adjoint_rel")
        return gq

    def laplacian(self, q):
        self._maps(q, "q")
        out = torch.empty_like(q)
        self._bind_stream()
        check(self.lib.fwils_laplacian(self._h, _ptr(q), _ptr(out)), "fwils_laplacian")
        return out

    def tikhonov_grad(self, ub, r, m0, q, lam=1e-3, reg="laplacian", rtol=1e-6, maxit=1000):
        """(f(q), grad f(q)) of the generalised Tikhonov objective."""
        self._field(ub, "ub")
        self._data(r, "r")
        self._maps(q, "q")
        m, mp = self._m0(m0)
        grad = torch.empty_like(q)
        d = torch.empty_like(r)
        f = ctypes.c_double()
        self._bind_stream()
        st = self.lib.fwils_tikhonov_grad(self._h, _ptr(ub), _ptr(r), mp, float(lam), self.REGS[reg],
                                          _ptr(q), _ptr(grad), ctypes.byref(f), _ptr(d), float(rtol),
                                          int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_tikhonov_grad")
        return f.value, grad

    def normal_apply(self, ub, m0, rr, q, lam=1e-3, reg="identity", rtol=1e-6, maxit=1000):
        self._field(ub, "ub")
        self._maps(q, "q")
        m, mp = self._m0(m0)
        out = torch.empty_like(q)
        d = torch.zeros(self.data_elems(), dtype=self.cdtype, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_normal_apply(self._h, _ptr(ub), mp, float(rr), float(lam), self.REGS[reg],
                                         _ptr(q), _ptr(out), _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_normal_apply")
        return out

    def normal_cg(self, ub, r, m0, niter=20, lam=1e-3, reg="identity", rtol=1e-6, maxit=1000):
        """niter CG iterations on the normal equation from q = 0: (q, residual history)."""
        self._field(ub, "ub")
        self._data(r, "r")
        m, mp = self._m0(m0)
        p = self.problems[0]
        q = torch.empty(self._qshape(), dtype=self.rdtype, device=self.device)
        d = torch.empty_like(r)
        hist = np.zeros(niter + 1, dtype=np.float64)
        self._bind_stream()
        st = self.lib.fwils_normal_cg(self._h, _ptr(ub), _ptr(r), mp, float(lam), self.REGS[reg],
                                      int(niter), _ptr(q), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_normal_cg")
        return q, hist

    def normal_cg_steps(self, ub, r, m0, first, niter, lam=1e-3, reg="identity", rtol=1e-6, maxit=1000):
        """niter CG iterations on the normal equation, from q = 0 (first = 0) or
        continuing the plan's run of `first` iterations: (q, history of the
        residual norm from iteration `first` on, iterates [niter, 5, nz, nx])."""
        self._field(ub, "ub")
        self._data(r, "r")
        m, mp = self._m0(m0)
        p = self.problems[0]
        q = torch.empty(self._qshape(), dtype=self.rdtype, device=self.device)
        qi = torch.empty((niter,) + self._qshape(), dtype=self.rdtype, device=self.device)
        d = torch.empty_like(r)
        hist = np.zeros(niter + 1, dtype=np.float64)
        self._bind_stream()
        st = self.lib.fwils_normal_cg_steps(self._h, _ptr(ub), _ptr(r), mp, float(lam), self.REGS[reg], int(first),
                                            int(niter), _ptr(q), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _ptr(qi), _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_normal_cg_steps")
        return q, hist, qi

    def receiver_data(self, u, out=None):
        """d = R u: the fields sampled at every problem's receivers (plan data layout)."""
        self._field(u, "u")
        d = torch.empty(self.data_elems(), dtype=self.cdtype, device=self.device) if out is None \
            else self._data(out, "out")
        self._bind_stream()
        check(self.lib.fwils_receiver_data(self._h, _ptr(u), _ptr(d)), "fwils_receiver_data")
        return d

    def get_contrast(self, i):
        """Problem i's current contrast maps [5, nz, nx] (rdtype)."""
        p = self.problems[i]
        m = torch.empty(5, p["nz"], p["nx"], dtype=self.rdtype, device=self.device)
        self._bind_stream()
        check(self.lib.fwils_get_contrast(self._h, i, _ptr(m)), "fwils_get_contrast")
        torch.cuda.current_stream(self.device).synchronize()
        return m

    def dbi_run(self, src_ixz, src_f, d_obs, m0, lam0=1e-3, niter=10, reg="identity", tol=1e-3,
                max_outer=10, rtol=1e-6, maxit=1000):
        """One frequency stage of the distorted-Born inversion (fwils_dbi_run):
        updates the plan's contrast in place and returns a dict with the data
        error history eps_d, the cooled lambdas, the number of updates, the
        final background fields ub, their residual r, the last update q and
        the status of the worst solve."""
        s = np.ascontiguousarray(np.asarray(src_ixz, dtype=np.int32).reshape(-1, self.CSTRIDE))
        f = np.ascontiguousarray(np.asarray(src_f, dtype=np.float64).reshape(-1, self.CSTRIDE))
        if s.shape[0] != self.total_sys or f.shape[0] != self.total_sys:
            raise ValueError(f"need {self.total_sys} sources and forces")
        self._data(d_obs, "d_obs")
        m, mp = self._m0(m0)
        p = self.problems[0]
        ub = self.new_field()
        r = torch.empty_like(d_obs)
        d = torch.empty_like(d_obs)
        q = torch.zeros(self._qshape(), dtype=self.rdtype, device=self.device)
        eps = np.full(max_outer + 1, np.nan)
        lam = np.full(max(max_outer, 1), np.nan)
        upd = ctypes.c_int32(0)
        dbl = ctypes.POINTER(ctypes.c_double)
        self._bind_stream()
        st = self.lib.fwils_dbi_run(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    f.ctypes.data_as(dbl), _ptr(d_obs), mp, float(lam0), self.REGS[reg],
                                    int(niter), float(tol), int(max_outer), _ptr(ub), _ptr(r), _ptr(q), _ptr(d),
                                    eps.ctypes.data_as(dbl), lam.ctypes.data_as(dbl), ctypes.byref(upd),
                                    float(rtol), int(maxit))
        if st not in (_lib.FWILS_OK, _lib.FWILS_ENOCONV):
            check(st, "fwils_dbi_run")
        n = int(upd.value)
        return dict(eps=eps[:n + 1].tolist(), lam=lam[:n].tolist(), updates=n, ub=ub, r=r, q=q, status=st)

    # ------------------------------------------------- Krylov method ----
    def set_krylov(self, method="bicgstab", restart=20, cgs2=True):
        """Krylov method of every solve of this plan: 'bicgstab' (default) or
        'gmres' (restarted GMRES(restart), restart <= 32; allocates its basis)."""
        if method == "bicgstab":
            check(self.lib.fwils_set_krylov(self._h, _lib.FWILS_KRYLOV_BICGSTAB, 0, 0, None, 0),
                  "fwils_set_krylov")
            self._gm_raw = None
            self.krylov = ("bicgstab", 0)
            return
        if method != "gmres":
            raise ValueError(f"unknown Krylov method {method!r}")
        size = ctypes.c_size_t()
        check(self.lib.fwils_gmres_workspace_size(self._h, int(restart), ctypes.byref(size)),
              "fwils_gmres_workspace_size")
        with torch.cuda.device(self.device):
            raw = torch.empty(size.value + 256, dtype=torch.uint8, device=self.device)
        ptr = raw.data_ptr() + (-raw.data_ptr()) % 256
        self._bind_stream()
        check(self.lib.fwils_set_krylov(self._h, _lib.FWILS_KRYLOV_GMRES, int(restart),
                                        0 if cgs2 else _lib.FWILS_GMRES_CGS1, ctypes.c_void_p(ptr), size.value),
              "fwils_set_krylov")
        self._gm_raw = raw
        self.krylov = ("gmres", int(restart))

    # ----------------------------------------------------- autotuner ----
    TUNE_KINDS = {"stencil": _lib.FWILS_TUNE_STENCIL, "rows": _lib.FWILS_TUNE_ROWS, "cols": _lib.FWILS_TUNE_COLS,
                  "fuse": _lib.FWILS_TUNE_FUSE}

    def autotune(self, reps=20):
        """Time every kernel variant on this plan's workspace and keep the fastest
        per problem (overwrites the plan's field vectors).  Returns tuning()."""
        self._bind_stream()
        check(self.lib.fwils_autotune(self._h, int(reps)), "fwils_autotune")
        return [self.tuning(i) for i in range(len(self.problems))]

    def tuning(self, i):
        """Kernel variants of problem i (dict of the fwils_tuning fields)."""
        t = _lib.FwilsTuning()
        check(self.lib.fwils_get_tuning(self._h, int(i), ctypes.byref(t)), "fwils_get_tuning")
        return t.to_dict()

    def set_tuning(self, i, **fields):
        """Replace some variant fields of problem i (the others stay)."""
        cur = self.tuning(i)
        t = _lib.FwilsTuning()
        for k in _lib.FwilsTuning.FIELDS:
            setattr(t, k, int(fields.pop(k, cur[k])))
        if fields:
            raise ValueError(f"unknown tuning fields {sorted(fields)}")
        check(self.lib.fwils_set_tuning(self._h, int(i), ctypes.byref(t)), "fwils_set_tuning")

    def tuning_candidates(self, i, kind):
        """Candidate variants of one kernel kind ('stencil', 'rows', 'cols') for problem i."""
        k = self.TUNE_KINDS[kind]
        n = ctypes.c_int32(0)
        check(self.lib.fwils_tuning_candidates(self._h, int(i), k, None, 0, ctypes.byref(n)),
              "fwils_tuning_candidates")
        arr = (_lib.FwilsTuning * max(n.value, 1))()
        check(self.lib.fwils_tuning_candidates(self._h, int(i), k, arr, n.value, ctypes.byref(n)),
              "fwils_tuning_candidates")
        out = []
        for j in range(n.value):
            d = arr[j].to_dict()
            d.pop("time_us")
            out.append(d)
        return out

    def fft2(self, i, x, inverse=False, out=None):
        """2-D FFT (unnormalised) of every field of problem i; x: [nsys, 2, nz, nx]."""
        _require_cuda(x, self.cdtype, "x")
        out = torch.empty_like(x) if out is None else out
        self._bind_stream()
        check(self.lib.fwils_fft2(self._h, i, _ptr(x), _ptr(out), 1 if inverse else 0), "fwils_fft2")
        return out


class Plan3(Plan):
    """One or more 3-D problems with a general anisotropic background
    (fwils_plan_create3).  A problem dict holds nx, ny, nz, dx, c0 (the 21
    constants of the 6 x 6 stiffness, upper triangle row by row, or a 6 x 6
    array), rho0, freq_hz, nsys, and optionally eta / damping, symbol and
    params ('vti': maps C11, C13, C33, C55, C66, rho; 'general': the 21
    constants and rho).  Fields are [nsys, 3, nz, ny, nx]; sources and
    receivers (ix, iy, iz); forces (fx, fy, fz); data [nsys, nrec, 3]."""

    PARAMS = {"vti": _lib.FWILS_PARAMS_VTI, "general": _lib.FWILS_PARAMS_GENERAL}
    NMAPS = {"vti": 6, "general": 22}
    CSTRIDE = 3

    def __init__(self, problems, device="cuda", precision="c64"):
        self.lib = _lib.load()
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        prec, self.cdtype, self.rdtype = PRECISIONS[precision]
        if not torch.cuda.is_available():
            raise RuntimeError("fwils needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.problems = [dict(p) for p in problems]
        n = len(self.problems)
        arr = (_lib.FwilsProblem3 * n)()
        for i, p in enumerate(self.problems):
            p.setdefault("params", "vti")
            arr[i].nx, arr[i].ny, arr[i].nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
            arr[i].dx = float(p["dx"])
            c0 = np.asarray(p["c0"], dtype=np.float64)
            if c0.shape == (6, 6):
                c0 = c0[np.triu_indices(6)]
            if c0.shape != (21,):
                raise ValueError("c0 must hold 21 constants or be a 6 x 6 matrix")
            for k in range(21):
                arr[i].c0[k] = float(c0[k])
            arr[i].rho0 = float(p["rho0"])
            arr[i].freq_hz = float(p["freq_hz"])
            arr[i].damping = float(p.get("eta", p.get("damping", 0.02)))
            arr[i].nsys = int(p["nsys"])
            sym = p.get("symbol", "spectral")
            arr[i].symbol = SYMBOLS[sym] if isinstance(sym, str) else int(sym)
            arr[i].params = self.PARAMS[p["params"]]
        h = ctypes.c_void_p()
        check(self.lib.fwils_plan_create3(arr, n, prec, ctypes.byref(h)), "fwils_plan_create3")
        self._attach(h)

    def _sys_elems(self, p):
        return 3 * p["nz"] * p["ny"] * p["nx"]

    def _field_shape(self, p):
        return (3, p["nz"], p["ny"], p["nx"])

    def nmaps(self, i):
        return self.NMAPS[self.problems[i]["params"]]

    def _map_shape(self, i):
        p = self.problems[i]
        return (self.nmaps(i), p["nz"], p["ny"], p["nx"])

    def _qshape(self):
        return self._map_shape(0)

    def set_contrast(self, i, maps):
        m = torch.as_tensor(maps, dtype=self.rdtype).to(self.device).contiguous()
        if tuple(m.shape) != self._map_shape(i):
            raise ValueError(f"maps must be {list(self._map_shape(i))}")
        self._bind_stream()
        check(self.lib.fwils_set_contrast(self._h, i, _ptr(m)), "fwils_set_contrast")
        torch.cuda.current_stream(self.device).synchronize()

    def get_contrast(self, i):
        m = torch.empty(self._map_shape(i), dtype=self.rdtype, device=self.device)
        self._bind_stream()
        check(self.lib.fwils_get_contrast(self._h, i, _ptr(m)), "fwils_get_contrast")
        torch.cuda.current_stream(self.device).synchronize()
        return m

    def set_receivers(self, i, rec_ixyz):
        r = np.ascontiguousarray(np.asarray(rec_ixyz, dtype=np.int32).reshape(-1, 3))
        self._bind_stream()
        check(self.lib.fwils_set_receivers(self._h, i, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           r.shape[0]), "fwils_set_receivers")
        self.nrec[i] = r.shape[0]

    def incident(self, src_ixyz, src_f):
        s = np.ascontiguousarray(np.asarray(src_ixyz, dtype=np.int32).reshape(-1, 3))
        f = np.ascontiguousarray(np.asarray(src_f, dtype=np.float64).reshape(-1, 3))
        if s.shape[0] != self.total_sys or f.shape[0] != self.total_sys:
            raise ValueError(f"need {self.total_sys} sources and forces")
        u0 = self._out_field()
        self._bind_stream()
        check(self.lib.fwils_incident(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(u0)),
              "fwils_incident")
        return u0

    def data_elems(self):
        return sum(p["nsys"] * nr * 3 for p, nr in zip(self.problems, self.nrec))

    def data_view(self, d, i):
        p = self.problems[i]
        off = sum(q["nsys"] * nr * 3 for q, nr in zip(self.problems[:i], self.nrec[:i]))
        return d[off:off + p["nsys"] * self.nrec[i] * 3].view(p["nsys"], self.nrec[i], 3)

    def frechet(self, ub, dm, rtol=1e-6, maxit=1000):
        """J dm for every system; dm: list (one per problem) of rdtype [nmaps, nz, ny, nx]."""
        self._field(ub, "ub")
        for i, m in enumerate(dm):
            _require_cuda(m, self.rdtype, f"dm[{i}]")
            if tuple(m.shape) != self._map_shape(i):
                raise ValueError(f"dm[{i}] must be {list(self._map_shape(i))}")
        arr = (ctypes.c_void_p * len(dm))(*[m.data_ptr() for m in dm])
        d = torch.empty(self.data_elems(), dtype=self.cdtype, device=self.device)
        self._bind_stream()
        st = self.lib.fwils_frechet(self._h, _ptr(ub), arr, _ptr(d), float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_frechet")
        return d

    def adjoint(self, ub, r, rtol=1e-6, maxit=1000, g=None, accumulate=False):
        """J* r: list (one per problem) of complex128 [nmaps, nz, ny, nx] maps."""
        self._field(ub, "ub")
        _require_cuda(r, self.cdtype, "r")
        if r.numel() != self.data_elems():
            raise ValueError(f"r must hold {self.data_elems()} complex values")
        if g is None:
            if accumulate:
                raise ValueError("accumulate needs the g maps to add to")
            g = [torch.empty(self._map_shape(i), dtype=torch.complex128, device=self.device)
                 for i in range(len(self.problems))]
        for i, gi in enumerate(g):
            _require_cuda(gi, torch.complex128, f"g[{i}]")
            if tuple(gi.shape) != self._map_shape(i):
                raise ValueError(f"g[{i}] must be {list(self._map_shape(i))}")
        arr = (ctypes.c_void_p * len(g))(*[gi.data_ptr() for gi in g])
        self._bind_stream()
        st = self.lib.fwils_adjoint(self._h, _ptr(ub), _ptr(r), arr,
                                    _lib.FWILS_ADJ_ACCUMULATE if accumulate else 0, float(rtol), int(maxit))
        if st != _lib.FWILS_OK:
            check(st, "fwils_adjoint")
        return g

    def fft3(self, i, x, inverse=False, out=None):
        """3-D FFT (unnormalised) of every field of problem i; x: [nsys, 3, nz, ny, nx]."""
        _require_cuda(x, self.cdtype, "x")
        out = torch.empty_like(x) if out is None else out
        self._bind_stream()
        check(self.lib.fwils_fft2(self._h, i, _ptr(x), _ptr(out), 1 if inverse else 0), "fwils_fft2")
        return out
