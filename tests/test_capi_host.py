"""Host-only tests of the C ABI: the library loads, exports every declared
entry point, validates arguments before touching the device, and the Python
binding refuses to run without a GPU.  No compute calls."""

import ctypes
import re
import os

import pytest
import torch

from paper_2402_02116_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _prob(**kw):
    p = _lib.FwilsProblem()
    p.nx, p.nz, p.dx = kw.get("nx", 64), kw.get("nz", 32), kw.get("dx", 8.0)
    c0 = kw.get("c0", (1.7875e10, 8.0805e9, 1.375e10, 3.168e9))
    for k in range(4):
        p.c0[k] = c0[k]
    p.rho0, p.freq_hz, p.damping = kw.get("rho0", 2200.0), kw.get("freq_hz", 5.0), kw.get("damping", 0.02)
    p.nsys, p.symbol = kw.get("nsys", 3), kw.get("symbol", 0)
    return p


def _create(lib, probs, prec=0):
    arr = (_lib.FwilsProblem * len(probs))(*probs)
    h = ctypes.c_void_p()
    st = lib.fwils_plan_create(arr, len(probs), prec, ctypes.byref(h))
    return st, h


def test_library_exports_every_declared_symbol(lib):
    names = _lib.header_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES)
    ver = re.search(r"#define FWILS_ABI_VERSION (\d+)", open(_lib.HEADER).read())
    assert lib.fwils_abi_version() == int(ver.group(1))


def test_tuning_defaults_candidates_and_validation(lib):
    """Host-side autotuner bookkeeping (no device work): defaults, candidate
    lists, and rejection of variants that are not built for the grid."""
    st, h = _create(lib, [_prob(nx=384, nz=384, nsys=4), _prob(nx=256, nz=24, nsys=2)])
    assert st == 0
    try:
        t = _lib.FwilsTuning()
        assert lib.fwils_get_tuning(h, 0, ctypes.byref(t)) == 0
        assert (t.row_points, t.col_points, t.col_width, t.col_shared, t.stencil_rows) == (12, 12, 16, 1, 8)
        assert t.fused_points == 0
        assert list(t.time_us) == [0.0, 0.0, 0.0, 0.0]
        for kind, field in ((0, "stencil_rows"), (1, "row_points"), (2, "col_points"), (3, "fused_points")):
            n = ctypes.c_int32()
            assert lib.fwils_tuning_candidates(h, 0, kind, None, 0, ctypes.byref(n)) == 0
            arr = (_lib.FwilsTuning * n.value)()
            assert lib.fwils_tuning_candidates(h, 0, kind, arr, n.value, ctypes.byref(n)) == 0
            assert n.value >= 2
            for c in arr:
                assert lib.fwils_set_tuning(h, 0, ctypes.byref(c)) == 0
        # 24 rows: no 16-row stencil tiles; widths must divide nx; bad radix
        bad = _lib.FwilsTuning()
        assert lib.fwils_get_tuning(h, 1, ctypes.byref(bad)) == 0
        good = _lib.FwilsTuning.from_buffer_copy(bad)
        bad.stencil_rows = 16
        assert lib.fwils_set_tuning(h, 1, ctypes.byref(bad)) == _lib.FWILS_EINVAL
        bad = _lib.FwilsTuning.from_buffer_copy(good)
        bad.col_width = 3
        assert lib.fwils_set_tuning(h, 1, ctypes.byref(bad)) == _lib.FWILS_EINVAL
        bad = _lib.FwilsTuning.from_buffer_copy(good)
        bad.row_points = 7
        assert lib.fwils_set_tuning(h, 1, ctypes.byref(bad)) == _lib.FWILS_EINVAL
        after = _lib.FwilsTuning()
        assert lib.fwils_get_tuning(h, 1, ctypes.byref(after)) == 0
        assert bytes(after) == bytes(good)
        # autotune needs the workspace
        assert lib.fwils_autotune(h, 5) == _lib.FWILS_ENOMEM
    finally:
        lib.fwils_plan_destroy(h)


def test_status_strings(lib):
    for s in range(7):
        assert lib.fwils_status_string(s)
    assert b"unknown" in lib.fwils_status_string(99)


def test_problem_struct_layout_matches_header():
    assert ctypes.sizeof(_lib.FwilsProblem) == 80
    assert _lib.FwilsProblem.nsys.offset == 72


@pytest.mark.parametrize("bad", [
    dict(nx=17), dict(nz=4096), dict(nx=8), dict(nx=80), dict(dx=0.0), dict(rho0=-1.0),
    dict(freq_hz=0.0), dict(damping=0.0), dict(nsys=0), dict(symbol=2),
    dict(c0=(0.0, 1e9, 1e10, 1e9)), dict(c0=(1e10, float("nan"), 1e10, 1e9)),
])
def test_plan_create_rejects_bad_problems(lib, bad):
    st, h = _create(lib, [_prob(), _prob(**bad)])
    assert st == _lib.FWILS_EINVAL
    assert not h.value
    assert b"problem 1" in lib.fwils_last_error()


def test_plan_create_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.fwils_plan_create(None, 1, 0, ctypes.byref(h)) == _lib.FWILS_EINVAL
    arr = (_lib.FwilsProblem * 1)(_prob())
    assert lib.fwils_plan_create(arr, 0, 0, ctypes.byref(h)) == _lib.FWILS_EINVAL
    assert lib.fwils_plan_create(arr, 1, 0, None) == _lib.FWILS_EINVAL
    assert lib.fwils_plan_create(arr, 1, 7, ctypes.byref(h)) == _lib.FWILS_EINVAL
    assert b"precision" in lib.fwils_last_error()


@pytest.mark.parametrize("prec,csize", [(_lib.FWILS_C64, 8), (_lib.FWILS_C128, 16)])
def test_both_precisions_create_plans_and_dispatch(lib, prec, csize):
    """Each precision has its own library core; the public entry points route
    a plan to the core that created it (workspace scales with the element size)."""
    arr = (_lib.FwilsProblem * 1)(_prob(nx=64, nz=32, nsys=3))
    h = ctypes.c_void_p()
    assert lib.fwils_plan_create(arr, 1, prec, ctypes.byref(h)) == _lib.FWILS_OK and h.value
    try:
        fe, sz = ctypes.c_int64(), ctypes.c_size_t()
        assert lib.fwils_field_elems(h, ctypes.byref(fe)) == 0 and fe.value == 3 * 2 * 64 * 32
        assert lib.fwils_workspace_size(h, ctypes.byref(sz)) == 0
        assert sz.value >= 9 * fe.value * csize
        # errors raised inside either core reach the shared error text
        assert lib.fwils_apply(h, ctypes.c_void_p(256), ctypes.c_void_p(512)) == _lib.FWILS_ENOMEM
        assert b"workspace" in lib.fwils_last_error()
    finally:
        lib.fwils_plan_destroy(h)
    assert lib.fwils_apply(None, ctypes.c_void_p(256), ctypes.c_void_p(512)) == _lib.FWILS_EINVAL
    assert b"null plan" in lib.fwils_last_error()


def test_plan_metadata_without_device(lib):
    probs = [_prob(nx=64, nz=32, nsys=3), _prob(nx=96, nz=48, nsys=2), _prob(nx=2048, nz=16, nsys=1)]
    st, h = _create(lib, probs)
    assert st == _lib.FWILS_OK and h.value
    try:
        fe = ctypes.c_int64()
        assert lib.fwils_field_elems(h, ctypes.byref(fe)) == 0
        assert fe.value == 3 * 2 * 64 * 32 + 2 * 2 * 96 * 48 + 1 * 2 * 2048 * 16
        sz = ctypes.c_size_t()
        assert lib.fwils_workspace_size(h, ctypes.byref(sz)) == 0
        # nine Krylov / scratch vectors at least
        assert sz.value >= 9 * fe.value * 8
        assert lib.fwils_workspace_size(h, None) == _lib.FWILS_EINVAL
        # everything that needs device memory refuses before any launch
        assert lib.fwils_apply(h, ctypes.c_void_p(256), ctypes.c_void_p(512)) == _lib.FWILS_ENOMEM
        assert lib.fwils_solve(h, ctypes.c_void_p(256), ctypes.c_void_p(512), 1e-6, 10, None, None, 0) \
            == _lib.FWILS_ENOMEM
        assert lib.fwils_set_workspace(h, None, sz.value) == _lib.FWILS_ENOMEM
        assert lib.fwils_set_workspace(h, ctypes.c_void_p(256), sz.value - 1) == _lib.FWILS_ENOMEM
        assert lib.fwils_set_workspace(h, ctypes.c_void_p(257), sz.value) == _lib.FWILS_ENOMEM
        assert lib.fwils_set_stream(h, None) == _lib.FWILS_OK
        v = ctypes.c_void_p(256)
        assert lib.fwils_receiver_data(h, v, v) == _lib.FWILS_ENOMEM
        assert lib.fwils_get_contrast(h, 0, v) == _lib.FWILS_ENOMEM
        m0 = (ctypes.c_double * 5)(1, 1, 1, 1, 1)
        eps = (ctypes.c_double * 11)()
        assert lib.fwils_dbi_run(h, None, None, v, m0, 1e-3, 0, 5, 1e-3, 10, v, v, v, v, eps, None, None,
                                 1e-6, 100) == _lib.FWILS_ENOMEM
    finally:
        lib.fwils_plan_destroy(h)


def test_null_plan_is_rejected(lib):
    assert lib.fwils_apply(None, None, None) == _lib.FWILS_EINVAL
    assert lib.fwils_solve(None, None, None, 1e-6, 10, None, None, 0) == _lib.FWILS_EINVAL
    assert lib.fwils_receiver_data(None, None, None) == _lib.FWILS_EINVAL
    assert lib.fwils_get_contrast(None, 0, None) == _lib.FWILS_EINVAL
    assert lib.fwils_dbi_run(None, None, None, None, None, 0.0, 0, 1, 0.0, 1, None, None, None, None, None,
                             None, None, 1e-6, 10) == _lib.FWILS_EINVAL
    lib.fwils_plan_destroy(None)


def test_python_binding_fails_loudly_without_gpu():
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2402_02116_amd.plan import Plan
    with pytest.raises(RuntimeError, match="GPU"):
        Plan([dict(nx=32, nz=32, dx=10.0, c0=(8e9, 4e9, 8e9, 2e9), rho0=2000.0, freq_hz=10.0, nsys=1)])


def test_missing_library_raises(tmp_path):
    with pytest.raises(_lib.FwilsLibraryError, match="not built"):
        _lib.load(str(tmp_path / "libfwils.so"))


def _prob3(**kw):
    import workloads as W
    p = _lib.FwilsProblem3()
    p.nx, p.ny, p.nz = kw.get("n", (80, 40, 32))
    p.dx = 25.0
    c0 = kw.get("c0", W.vti3d_background()[0])
    for k in range(21):
        p.c0[k] = float(c0[k])
    p.rho0, p.freq_hz, p.damping = 2200.0, 7.0, 0.02
    p.nsys, p.symbol, p.params = kw.get("nsys", 4), 0, kw.get("params", _lib.FWILS_PARAMS_VTI)
    return p


def test_plan_create3_validates_on_the_host(lib):
    """3-D plans: supported axis lengths (2^a 3^b 5^c, 16..256, or ny = 1), a
    positive definite background, known parametrisations; field and workspace
    sizes follow [nsys][3][nz][ny][nx]; 3-D plans refuse the 2-D-only calls."""
    import workloads as W
    cases = [({}, 0), ({"n": (80, 1, 32)}, 0), ({"n": (80, 40, 33)}, _lib.FWILS_EINVAL),
             ({"n": (512, 16, 16)}, _lib.FWILS_EINVAL), ({"params": 7}, _lib.FWILS_EINVAL),
             ({"c0": -W.vti3d_background()[0]}, _lib.FWILS_EINVAL), ({"nsys": 0}, _lib.FWILS_EINVAL)]
    for kw, want in cases:
        arr = (_lib.FwilsProblem3 * 1)(_prob3(**kw))
        h = ctypes.c_void_p()
        assert lib.fwils_plan_create3(arr, 1, _lib.FWILS_C64, ctypes.byref(h)) == want, kw
        if want == 0:
            n = kw.get("n", (80, 40, 32))
            fe = ctypes.c_int64()
            assert lib.fwils_field_elems(h, ctypes.byref(fe)) == 0
            assert fe.value == 4 * 3 * n[0] * n[1] * n[2]
            t = _lib.FwilsTuning()
            assert lib.fwils_get_tuning(h, 0, ctypes.byref(t)) == _lib.FWILS_EUNSUPPORTED
            lib.fwils_plan_destroy(h)
    # precision reaches the right core; general parametrisation accepted
    arr = (_lib.FwilsProblem3 * 1)(_prob3(params=_lib.FWILS_PARAMS_GENERAL, n=(20, 24, 16)))
    h = ctypes.c_void_p()
    assert lib.fwils_plan_create3(arr, 1, _lib.FWILS_C128, ctypes.byref(h)) == 0
    lib.fwils_plan_destroy(h)
