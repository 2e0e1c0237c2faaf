"""Host builds of library headers for CPU-side checks."""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
_lib = None


def host_exact():
    """ctypes handle to the host build of exact.hpp (compiled on first use)."""
    global _lib
    if _lib is None:
        out = os.path.join(HERE, "libhost_exact.so")
        src = os.path.join(HERE, "host_exact.cpp")
        hdr = os.path.join(ROOT, "paper_1508_05931_amd", "csrc", "exact.hpp")
        if (not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src)
                or os.path.getmtime(out) < os.path.getmtime(hdr)):
            hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
            subprocess.check_call([
                hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                "--offload-arch=gfx950",
                "-I", os.path.join(ROOT, "paper_1508_05931_amd", "csrc"),
                "-o", out + ".tmp", src])
            os.replace(out + ".tmp", out)
        lib = ctypes.CDLL(out)
        d = ctypes.c_double
        for name in ("hx_orient", "hx_orient_exact"):
            getattr(lib, name).argtypes = [d] * 6
            getattr(lib, name).restype = ctypes.c_int
        lib.hx_angle_key.argtypes = [d] * 4
        lib.hx_angle_key.restype = ctypes.c_uint
        lib.hx_turn_key.argtypes = [d] * 4
        lib.hx_turn_key.restype = ctypes.c_uint
        lib.hx_key_at_least.argtypes = [d] * 5
        lib.hx_key_at_least.restype = ctypes.c_int
        _lib = lib
    return _lib
