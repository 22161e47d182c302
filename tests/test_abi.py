"""CPU-side checks of the C ABI: the header's declarations are all exported by the library."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vsaogm.h")
LIB = os.path.join(ROOT, "paper_2408_09066_amd", "libvsaogm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vsaogm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("vsaogm_encode", "vsaogm_decode", "vsaogm_classify", "vsaogm_map_create",
              "vsaogm_memories", "vsaogm_fuse"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (vsaogm_[a-z_0-9]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_binding_matches_header():
    from paper_2408_09066_amd import native
    L = native.load()
    assert L.vsaogm_version() >= 100
    assert set(native.EXPORTED) <= set(declared())
    for n in declared():
        getattr(L, n)
