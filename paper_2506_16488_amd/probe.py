"""The benchmark's scattered-access probe (libppsp_probe.so).

Measurement tooling, outside the search library and its C interface: the
round kernel is bound by scattered 8-16 byte accesses to the search state,
and this probe measures the device's rate for exactly those accesses, so the
benchmark can price a launch against it. The search path never loads it.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libppsp_probe.so")
_lib = None


def randbench(words, accesses, kind, device=0) -> float:
    """Kernel milliseconds (second of two runs) for `accesses` scattered
    16-byte loads (kind 0) or 64-bit atomicMin (kind 1) over a fresh table of
    `words` 64-bit words. Raises ValueError on bad arguments, RuntimeError on
    a device failure."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise ImportError("libppsp_probe.so is not built (run __graft_entry__.build())")
        import torch  # noqa: F401  (bind to torch's HIP runtime, as the search library does)
        _lib = ctypes.CDLL(SO_PATH)
        _lib.probe_randbench.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double)]
        _lib.probe_randbench.restype = ctypes.c_int
    ms = ctypes.c_double(0)
    rc = _lib.probe_randbench(device, int(words), int(accesses), int(kind), ctypes.byref(ms))
    if rc == -1:
        raise ValueError("probe_randbench: bad arguments")
    if rc != 0:
        raise RuntimeError("probe_randbench failed (%d)" % rc)
    return ms.value
