"""The C-ABI library loads on a machine without a GPU and exports every
function that include/hs.h declares (no compute calls are made here)."""
import ctypes
import os
import re

from paper_2505_06703_amd import build as hsbuild
from paper_2505_06703_amd import hs

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[ \t]*(?:const\s+)?[A-Za-z_][\w]*[\s\*]+(hs_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def _lib():
    if not os.path.exists(hsbuild.LIB):
        hsbuild.build_library(force=True)
    return ctypes.CDLL(hsbuild.LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hs_pose_sample", "hs_scan_forward", "hs_skin", "hs_scan_backward",
                     "hs_plan_create", "hs_context_create", "hs_last_error"):
        assert required in names
    assert sorted(hs.SYMBOLS) == names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string_is_host_only_and_callable():
    lib = _lib()
    lib.hs_version.restype = ctypes.c_char_p
    assert lib.hs_version().decode().startswith("hs ")
