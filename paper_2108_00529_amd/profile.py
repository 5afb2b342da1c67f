"""Per-kernel device timing of libbgv launches (include/bgv_profile.h): start and stop
HIP events attached to library kernel launches while enabled."""
from __future__ import annotations

import ctypes as C

from ._lib import lib

lib.bgv_profile_enable.argtypes = [C.c_int]
lib.bgv_profile_enable.restype = None
lib.bgv_profile_filter.argtypes = [C.c_char_p]
lib.bgv_profile_filter.restype = None
lib.bgv_profile_sample.argtypes = [C.c_int]
lib.bgv_profile_sample.restype = None
lib.bgv_profile_reset.argtypes = []
lib.bgv_profile_reset.restype = None
lib.bgv_profile_count.argtypes = []
lib.bgv_profile_count.restype = C.c_int
lib.bgv_profile_get.argtypes = [C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
lib.bgv_profile_get.restype = C.c_int


lib.bgv_profile_counter.argtypes = [C.c_char_p, C.POINTER(C.c_uint64)]
lib.bgv_profile_counter.restype = C.c_int


def counter(name: str) -> int | None:
    """A device work counter (e.g. "bh_interactions"), or None if unknown."""
    v = C.c_uint64()
    return int(v.value) if lib.bgv_profile_counter(name.encode(), C.byref(v)) == 0 else None


def enable(on: bool = True) -> None:
    lib.bgv_profile_enable(1 if on else 0)


def only(kernel: str | None) -> None:
    """Record only kernels whose name starts with `kernel` (the name as stats() reports
    it, without the "k_" prefix); None records every kernel."""
    lib.bgv_profile_filter(None if not kernel else ("k_" + kernel).encode())


def sample(every: int) -> None:
    """Record one in `every` of the launches that pass the filter (1: all)."""
    lib.bgv_profile_sample(int(every))


def reset() -> None:
    lib.bgv_profile_reset()


def stats() -> dict:
    """{kernel name: {"launches": n, "total_ms": t}} since the last reset."""
    out = {}
    for i in range(lib.bgv_profile_count()):
        name = C.c_char_p()
        cnt = C.c_int64()
        ms = C.c_double()
        if lib.bgv_profile_get(i, C.byref(name), C.byref(cnt), C.byref(ms)) == 0:
            key = name.value.decode()
            key = key[2:] if key.startswith("k_") else key
            out[key] = {"launches": int(cnt.value), "total_ms": float(ms.value)}
    return out
