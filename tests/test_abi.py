"""The C-ABI library loads on the CPU and exports every entry point that
include/sbr.h and include/sbr_nn.h declare (no compute call: there is no GPU
here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("sbr.h", "sbr_nn.h")]
LIB = os.path.join(ROOT, "paper_2208_10006_amd", "libsbr.so")


def declared(path=None):
    names = set()
    for h in [path] if path else HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(sbr_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_four_calls():
    names = declared(HEADERS[0])
    for n in ["sbr_scene_build", "sbr_trace", "sbr_receive", "sbr_channel"]:
        assert n in names


def test_nn_header_declares_the_surrogate_kernels():
    names = declared(HEADERS[1])
    for n in ["sbr_nn_gemm_bf16", "sbr_nn_im2col", "sbr_nn_col2im", "sbr_nn_fourier", "sbr_nn_adam",
              "sbr_nn_ensemble", "sbr_nn_mse"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsbr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.sbr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.sbr_version()


@pytest.mark.parametrize("module", ["sbr.py", "nn.py"])
def test_binding_names_match_the_abi(module):
    """Every public function of the Python bindings named sbr_* exists in a header."""
    src = open(os.path.join(ROOT, "paper_2208_10006_amd", module)).read()
    py = set(re.findall(r"^def (sbr_[a-z_0-9]+)\(", src, flags=re.M))
    hdr = set(declared())
    extra = {n for n in py if n not in hdr and not n.endswith("_device")}
    assert not extra, extra
    if module == "nn.py":
        sig = set(re.findall(r'"(sbr_nn_[a-z_0-9]+)"', src))
        assert sig == {n for n in hdr if n.startswith("sbr_nn_")}
