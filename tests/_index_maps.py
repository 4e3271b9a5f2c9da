"""The kernels' index maps (csrc/index_maps.h), compiled for the host with
g++ into a small library the CPU tests call through ctypes."""
import ctypes
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        out = os.path.join(tempfile.mkdtemp(prefix="tlt_index_"), "index_probe.so")
        subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I",
                        os.path.join(ROOT, "paper_2203_12339_amd", "csrc"),
                        os.path.join(ROOT, "tests", "_index_probe.cpp"), "-o", out], check=True)
        L = ctypes.CDLL(out)
        L.haar_row.restype = ctypes.c_longlong
        _LIB = L
    return _LIB
