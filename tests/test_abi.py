"""The C-ABI library loads on the CPU and exports every entry point that
include/sbr.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbr.h")
LIB = os.path.join(ROOT, "paper_2208_10006_amd", "libsbr.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sbr_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    names = declared()
    for n in ["sbr_scene_build", "sbr_trace", "sbr_receive", "sbr_channel"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.sbr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.sbr_version()


def test_binding_names_match_the_abi():
    """Every public function of the Python binding named sbr_* exists in the header."""
    src = open(os.path.join(ROOT, "paper_2208_10006_amd", "sbr.py")).read()
    py = set(re.findall(r"^def (sbr_[a-z_0-9]+)\(", src, flags=re.M))
    hdr = set(declared())
    extra = {n for n in py if n not in hdr and not n.endswith("_device")}
    assert not extra, extra
