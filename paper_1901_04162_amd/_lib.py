"""ctypes binding of libmomfill.so (argument marshalling only).

torch is imported first on purpose: it loads the HIP runtime that the library
then shares (both resolve libamdhip64 by the same soname).
"""

from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
# MOMFILL_SO names another build of the same sources (the host-sanitizer test
# loads one this way); default: the in-tree library.
SO_PATH = os.environ.get("MOMFILL_SO") or os.path.join(_HERE, "libmomfill.so")

MF_OK, MF_EINVAL, MF_EMESH, MF_ERANGE, MF_ENOMEM, MF_EHIP, MF_ENOTCONV = 0, -1, -2, -3, -4, -5, -6
MF_MODE_TABLE, MF_MODE_DIRECT = 0, 1
MF_PART_A, MF_PART_PHI = 0x10, 0x20
MF_C64, MF_C128 = 0, 1

EXPORTS = [
    "mf_last_error", "mf_mesh_create", "mf_mesh_destroy", "mf_mesh_n_edges", "mf_mesh_edges",
    "mf_mesh_n_touching", "mf_mesh_plan", "mf_r_range", "mf_build_tables", "mf_tables_destroy",
    "mf_tables_info", "mf_tables_get", "mf_tables_eval", "mf_fill_Z", "mf_fill_Z_backward",
    "mf_sync_status", "mf_set_timing", "mf_mesh_timings", "mf_batch_create", "mf_batch_fill",
    "mf_batch_destroy", "mf_near_create", "mf_near_info", "mf_near_pattern", "mf_fill_near",
    "mf_near_destroy", "mf_rhs_planewave", "mf_far_field", "mf_fill_mfie",
    "mf_rhs_planewave_mfie", "mf_fill_angular", "mf_angular_rmax", "mf_build_exp_table",
    "mf_batch_info", "mf_batch_set_choice", "mf_mesh_workspace_bytes", "mf_mesh_set_workspace",
    "mf_tables_workspace_bytes", "mf_exp_table_workspace_bytes", "mf_batch_workspace_bytes",
    "mf_near_workspace_bytes", "mf_near_set_workspace", "mf_r_range_static", "mf_mesh_tb_plan",
    "mf_fill_tune", "mf_fill_choice_name", "mf_mesh_fill_timings", "mf_mesh_set_fill_choice",
]


class MomfillError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"momfill error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(
                f"{SO_PATH} is missing: build it with `python -m paper_1901_04162_amd.build`")
        L = C.CDLL(SO_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.mf_last_error.restype = C.c_char_p
        L.mf_last_error.argtypes = []
        L.mf_mesh_create.argtypes = [C.c_int32, C.c_int32, ip, C.POINTER(vp)]
        L.mf_mesh_destroy.argtypes = [vp]
        L.mf_mesh_destroy.restype = None
        L.mf_mesh_n_edges.argtypes = [vp, ip]
        L.mf_mesh_edges.argtypes = [vp, ip]
        L.mf_mesh_n_touching.argtypes = [vp, C.POINTER(C.c_int64)]
        sp = C.POINTER(C.c_size_t)
        L.mf_mesh_workspace_bytes.argtypes = [vp, sp]
        L.mf_mesh_set_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.mf_tables_workspace_bytes.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                                sp]
        L.mf_exp_table_workspace_bytes.argtypes = [C.c_double, C.c_double, C.c_double, sp]
        L.mf_batch_workspace_bytes.argtypes = [C.c_int32, C.POINTER(vp), sp]
        L.mf_near_workspace_bytes.argtypes = [vp, sp]
        L.mf_near_set_workspace.argtypes = [vp, vp, C.c_size_t, vp]
        L.mf_batch_create.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(C.c_double), C.POINTER(vp), C.c_int, C.c_int,
                                      C.POINTER(vp), C.c_int, C.POINTER(C.c_int64), vp,
                                      C.c_size_t, C.POINTER(vp)]
        L.mf_batch_fill.argtypes = [vp, vp]
        L.mf_batch_destroy.argtypes = [vp]
        L.mf_batch_destroy.restype = None
        L.mf_near_create.argtypes = [vp, dp, C.c_double, C.POINTER(vp)]
        L.mf_near_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.mf_near_pattern.argtypes = [vp, C.POINTER(C.c_int64), ip]
        L.mf_fill_near.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, C.c_int, vp]
        L.mf_near_destroy.argtypes = [vp]
        L.mf_near_destroy.restype = None
        L.mf_rhs_planewave.argtypes = [vp, vp, C.c_double, C.c_int, dp, dp, vp, C.c_int, vp]
        L.mf_rhs_planewave_mfie.argtypes = [vp, vp, C.c_double, C.c_int, dp, dp, vp, C.c_int,
                                            vp]
        L.mf_batch_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_float)]
        L.mf_batch_set_choice.argtypes = [vp, C.c_int32]
        L.mf_fill_angular.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, C.c_int, vp, vp,
                                      C.c_int, C.c_int64, vp]
        L.mf_angular_rmax.argtypes = [vp, vp, C.c_int, dp, vp]
        L.mf_build_exp_table.argtypes = [C.c_double, C.c_double, C.c_double, vp, C.c_size_t,
                                         C.POINTER(vp), vp]
        L.mf_fill_mfie.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, C.c_int,
                                   C.c_int64, vp]
        L.mf_far_field.argtypes = [vp, vp, C.c_double, C.c_int, vp, C.c_int, C.c_int32, vp,
                                   C.c_double, vp, vp, vp]
        L.mf_mesh_plan.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int32)]
        L.mf_mesh_tb_plan.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.mf_r_range.argtypes = [vp, vp, C.c_int, dp, dp, vp]
        L.mf_r_range_static.argtypes = [vp, vp, C.c_int, dp, dp, vp]
        L.mf_fill_tune.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, C.c_int,
                                   C.c_int64, vp, ip, C.POINTER(C.c_float)]
        L.mf_fill_choice_name.argtypes = [C.c_int32]
        L.mf_fill_choice_name.restype = C.c_char_p
        L.mf_build_tables.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, vp,
                                      C.c_size_t, C.POINTER(vp), vp]
        L.mf_tables_destroy.argtypes = [vp]
        L.mf_tables_destroy.restype = None
        L.mf_tables_info.argtypes = [vp, ip, ip, ip, ip, dp, dp, dp, dp]
        L.mf_tables_get.argtypes = [vp, C.c_int, dp, dp, ip, vp]
        L.mf_tables_eval.argtypes = [vp, C.c_int, C.c_int64, vp, vp, vp]
        L.mf_fill_Z.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, C.c_int,
                                C.c_int64, vp]
        L.mf_fill_Z_backward.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, C.c_int,
                                         C.c_int64, vp, vp, vp]
        L.mf_sync_status.argtypes = [vp, vp]
        L.mf_set_timing.argtypes = [C.c_int]
        L.mf_set_timing.restype = None
        L.mf_mesh_timings.argtypes = [vp, C.POINTER(C.c_float)]
        L.mf_mesh_fill_timings.argtypes = [vp, C.POINTER(C.c_float)]
        L.mf_mesh_set_fill_choice.argtypes = [vp, C.c_int32]
        _lib = L
    return _lib


def check(rc: int):
    if rc != MF_OK:
        raise MomfillError(rc, lib().mf_last_error().decode())
    return rc
