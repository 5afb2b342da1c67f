"""ctypes loader for libbgv.so (the HIP kernels and their C ABI, include/bgv.h).

torch is imported first so that the HIP runtime it ships is the one the library binds
to (both use the soname libamdhip64.so.7).  There is no fallback: if the library is
missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before libbgv.so)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbgv.so")


class BgvError(RuntimeError):
    pass


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2108_00529_amd/build.py` "
                      "(or __graft_entry__.build()) first")

lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

P = C.c_void_p
i32, i64, f32, u64 = C.c_int32, C.c_int64, C.c_float, C.c_uint64
SZ = C.c_size_t


class CdParams(C.Structure):
    _fields_ = [("threshold", i32), ("passes", i32), ("growth", i32), ("method", i32), ("chunk", i64),
                ("tie", i32), ("rule", i32)]


class SketchParams(C.Structure):
    _fields_ = [("rows", i32), ("cols", i32), ("coef1", P), ("coef2", P)]


class Fa2Params(C.Structure):
    _fields_ = [("iters", i32), ("exact", i32), ("theta", f32), ("kr", f32), ("kg", f32), ("tau", f32),
                ("ks", f32), ("ksmax", f32)]


def _sig(name, res, args):
    fn = getattr(lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


bgv_status_string = _sig("bgv_status_string", C.c_char_p, [i32])
bgv_last_error = _sig("bgv_last_error", C.c_char_p, [])
bgv_community_workspace = _sig("bgv_community_workspace", SZ, [i32, i64, C.POINTER(CdParams)])
bgv_community = _sig("bgv_community", i32, [i32, i64, P, C.POINTER(CdParams), P, P, P, P, SZ, P])
bgv_community_passes = _sig("bgv_community_passes", i32, [i32, i64, P, C.POINTER(CdParams), P, P, P, P, P, SZ, P])
bgv_community_resume = _sig("bgv_community_resume", i32, [i32, i64, P, C.POINTER(CdParams), i32, P, P, P, P, P,
                                                          SZ, P])
bgv_supergraph_workspace = _sig("bgv_supergraph_workspace", SZ, [i32, i64, C.POINTER(SketchParams)])
bgv_supergraph = _sig("bgv_supergraph", i32, [i32, i64, P, P, P, C.POINTER(SketchParams), C.POINTER(i32),
                                              C.POINTER(i64), P, P, P, P, P, P, P, P, P, SZ, P])
bgv_fa2_workspace = _sig("bgv_fa2_workspace", SZ, [i32, i64, C.POINTER(Fa2Params)])
bgv_fa2_layout = _sig("bgv_fa2_layout", i32, [i32, i64, P, P, P, P, P, P, C.POINTER(Fa2Params), P, SZ, P])
bgv_fa2_layout_static = _sig("bgv_fa2_layout_static", i32, [i32, i64, P, P, P, P, P, P, C.POINTER(Fa2Params), P])
BGV_FA2_STATIC_SCRATCH_BYTES = 64 << 20
bgv_fa2_energy_workspace = _sig("bgv_fa2_energy_workspace", SZ, [i32, i64])
bgv_fa2_energy = _sig("bgv_fa2_energy", i32, [i32, i64, P, P, P, P, f32, f32, P, P, SZ, P])
bgv_fa2_grad = _sig("bgv_fa2_grad", i32, [i32, i64, P, P, P, P, f32, f32, P, P, P, SZ, P])

bgv_batched_workspace = _sig("bgv_batched_workspace", SZ, [i32, i64, i64])
bgv_batched = _sig("bgv_batched", i32, [i32, i64, i64, P, P, P, P, C.POINTER(CdParams), C.POINTER(SketchParams),
                                        C.POINTER(Fa2Params), i32, i32, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P])

bgv_draw_workspace = _sig("bgv_draw_workspace", SZ, [i32])
bgv_draw_supernodes = _sig("bgv_draw_supernodes", i32, [i32, P, P, P, P, SZ, P])

bgv_validate_edges = _sig("bgv_validate_edges", i32, [i32, i64, P, P, P])
bgv_bh_tree_workspace = _sig("bgv_bh_tree_workspace", SZ, [i32])
bgv_bh_tree = _sig("bgv_bh_tree", i32, [i32, P, P, P, P, P, P, P, P, SZ, P])

EXPORTED = ["bgv_status_string", "bgv_last_error", "bgv_community_workspace", "bgv_community",
            "bgv_community_passes", "bgv_community_resume",
            "bgv_supergraph_workspace", "bgv_supergraph", "bgv_fa2_workspace", "bgv_fa2_layout", "bgv_fa2_layout_static",
            "bgv_fa2_energy_workspace", "bgv_fa2_energy", "bgv_fa2_grad",
            "bgv_profile_enable", "bgv_profile_filter", "bgv_profile_sample", "bgv_profile_reset", "bgv_profile_count", "bgv_profile_get",
            "bgv_profile_counter", "bgv_batched_workspace", "bgv_batched", "bgv_draw_workspace",
            "bgv_draw_supernodes", "bgv_validate_edges", "bgv_bh_tree_workspace", "bgv_bh_tree"]


BGV_E_RANGE = -2


def check(status: int, what: str) -> None:
    if status != 0:
        msg = bgv_last_error().decode(errors="replace")
        raise BgvError(f"{what}: {bgv_status_string(status).decode()} {msg}")
