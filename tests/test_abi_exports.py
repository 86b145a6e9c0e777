"""The C ABI: libtsnmf.so loads without a GPU and exports every function that
include/tsnmf.h declares (no compute call is made here)."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsnmf.h")
LIB = os.path.join(ROOT, "paper_1402_6964_amd", "libtsnmf.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(tsnmf_[a-z0-9_]+)\s*\(",
                                 txt, flags=re.M)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, "-m", "paper_1402_6964_amd.build", "--incremental"], cwd=ROOT, check=True)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for fn in ("tsnmf_tsqr_r", "tsnmf_tsqr_r_batched", "tsnmf_gauss_proj", "tsnmf_select_spa",
               "tsnmf_select_xray", "tsnmf_select_gp", "tsnmf_nnls", "tsnmf_residual", "tsnmf_reserve"):
        assert fn in names


def test_every_declared_function_is_exported(so):
    missing = [fn for fn in declared() if not hasattr(so, fn)]
    assert not missing, f"not exported: {missing}"


def test_version_and_status_text(so):
    so.tsnmf_version.restype = ctypes.c_int
    so.tsnmf_status_string.restype = ctypes.c_char_p
    assert so.tsnmf_version() >= 100
    assert so.tsnmf_status_string(0) == b"success"
    assert so.tsnmf_status_string(-3) == b"invalid argument"


def test_binding_names_match_the_header():
    """The Python binding wraps every entry point under the same name."""
    src = open(os.path.join(ROOT, "paper_1402_6964_amd", "tsnmf.py")).read()
    for fn in declared():
        assert re.search(rf"^def {fn}\(", src, flags=re.M), fn
