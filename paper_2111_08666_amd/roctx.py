"""roctx ranges around the phases of a run, for rocprofv3 --marker-trace.

    from paper_2111_08666_amd.roctx import rng
    with rng("timed steps"):
        ...

The ranges come from ROCm's roctx library (rocprofiler-sdk); where it is not
installed they are no-ops, so the code that uses them runs unchanged.
"""
import contextlib
import ctypes
import os

_LIB = None
_TRIED = False


def _lib():
    global _LIB, _TRIED
    if not _TRIED:
        _TRIED = True
        rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4"):
            try:
                lib = ctypes.CDLL(os.path.join(rocm, "lib", name))
            except OSError:
                continue
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            lib.roctxRangePushA.restype = ctypes.c_int
            lib.roctxRangePop.restype = ctypes.c_int
            lib.roctxMarkA.argtypes = [ctypes.c_char_p]
            _LIB = lib
            break
    return _LIB


def available() -> bool:
    return _lib() is not None


@contextlib.contextmanager
def rng(name: str):
    """A nested roctx range named `name` around the with-block."""
    lib = _lib()
    if lib is not None:
        lib.roctxRangePushA(name.encode())
    try:
        yield
    finally:
        if lib is not None:
            lib.roctxRangePop()


def mark(name: str):
    lib = _lib()
    if lib is not None:
        lib.roctxMarkA(name.encode())
