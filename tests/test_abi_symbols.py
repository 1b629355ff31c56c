"""The C-ABI library builds for gfx950, loads, and exports every declared entry point.

No compute call is made here (no GPU in this environment).
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seis.h")
LIB = os.path.join(ROOT, "paper_2107_06640_amd", "libseis.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(seis_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("seis_setup", "seis_predict", "seis_correct", "seis_read", "seis_write", "seis_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(seis_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_declares_signatures():
    from paper_2107_06640_amd import seis
    lib = seis.load_library()
    for n in declared():
        assert hasattr(lib, n)
    assert sorted(seis.EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_carries_device_code():
    out = subprocess.run(["readelf", "-S", "-W", LIB], capture_output=True, text=True, check=True).stdout
    assert ".hip_fatbin" in out
