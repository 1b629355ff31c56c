"""The C-ABI library builds for gfx950, loads, and exports every declared entry point.

No compute call is made here (no GPU in this environment).
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_2107_06640_amd", "libseis.so")


def declared(prefix="seis_"):
    """Functions declared in the headers of include/ whose names start with prefix."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(INCLUDE, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("seis_setup", "seis_predict", "seis_correct", "seis_read", "seis_write", "seis_step"):
        assert n in names
    fno = declared("fno_")
    for n in ("fno_gemm", "fno_adam", "fno_rel_l2", "fno_bias_act", "fno_gelu_backward", "fno_channel_sum"):
        assert n in fno


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s((?:seis|fno)_\w+)", out))
    missing = [n for n in declared() + declared("fno_") if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_declares_signatures():
    from paper_2107_06640_amd import seis
    lib = seis.load_library()
    for n in declared():
        assert hasattr(lib, n)
    assert sorted(seis.EXPORTED) == declared()
    from paper_2107_06640_amd import fno
    lib = fno._lib()
    for n in declared("fno_"):
        assert getattr(lib, n).restype is not None


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_carries_device_code():
    out = subprocess.run(["readelf", "-S", "-W", LIB], capture_output=True, text=True, check=True).stdout
    assert ".hip_fatbin" in out
