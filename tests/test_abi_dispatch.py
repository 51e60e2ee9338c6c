"""Host-side consistency of the two-precision library: every public entry
point of include/fwils.h is defined once by the dispatch layer, each core build
renames exactly the entry points the dispatch layer forwards, and the shared
library exports the public names and both precision variants."""

import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_2402_02116_amd" / "csrc"
SHIM_ONLY = {"fwils_status_string", "fwils_last_error", "fwils_abi_version"}


def _public():
    h = (ROOT / "include" / "fwils.h").read_text()
    return set(re.findall(r"^(?:fwils_status|void|const char\*|int32_t)\s+(fwils_\w+)\s*\(", h, re.M))


def test_core_rename_list_matches_header():
    renamed = set(re.findall(r"^#define (fwils_\w+) FW_CORE\(\1\)", (CSRC / "core_names.h").read_text(), re.M))
    assert renamed - {"fwils_plan_s"} == _public() - SHIM_ONLY


def test_dispatch_list_matches_header():
    abi = (CSRC / "abi.cpp").read_text()
    forwarded = {"fwils_" + n for n in re.findall(r"^\s*X\(\w+, (\w+),", abi, re.M)}
    defined = forwarded | {"fwils_plan_create", "fwils_plan_create3", "fwils_plan_destroy"} | SHIM_ONLY
    assert defined == _public()


def test_library_exports_public_and_variant_symbols():
    lib = ROOT / "paper_2402_02116_amd" / "libfwils.so"
    if not lib.exists():
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", str(lib)], capture_output=True, text=True).stdout
    syms = set(re.findall(r" T (fwils_\w+)$", out, re.M))
    pub = _public()
    assert pub <= syms
    for n in pub - SHIM_ONLY:
        assert n + "_c64" in syms and n + "_c128" in syms, n
