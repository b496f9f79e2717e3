"""The C-ABI library builds for gfx950, loads, and exports every function
that include/hipperm.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hipperm.h")
LIB = os.path.join(ROOT, "paper_2509_20776_amd", "libhipperm.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2509_20776_amd import build
        build.build(verbose=False)
    return LIB


def test_header_declares_api():
    names = declared()
    for must in ("hp_create", "hp_permute_plan", "hp_spref_plan", "hp_spasgn_plan"):
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hp_[a-z0-9_]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


def test_library_loads_and_reports_status_strings(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.hp_status_string.restype = ctypes.c_char_p
    assert lib.hp_status_string(0) == b"HP_OK"
    assert lib.hp_status_string(3) == b"HP_ERR_NOT_PERMUTATION"


def test_library_is_gfx950(lib_path):
    data = open(lib_path, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
