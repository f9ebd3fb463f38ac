"""ctypes declarations of the C ABI in include/tlfea.h (argument marshalling only).

The shared library must have been built (``paper_2602_17002_amd/build.py``);
there is no fallback path: a missing library raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtlfea.so")

TLFEA_OK = 0
STATUS_NAMES = {0: "TLFEA_OK", -1: "TLFEA_E_INVALID", -2: "TLFEA_E_SHAPE", -3: "TLFEA_E_REF_JACOBIAN",
                -4: "TLFEA_E_NOMEM", -5: "TLFEA_E_DEVICE", -6: "TLFEA_E_UNSUPPORTED"}
T10, H8, Q27 = 0, 1, 2
SVK, MR, NH = 0, 1, 2
PLAIN, BATCHED, AUTOTUNE, KEEP_ORDER = 0, 1, 2, 4
KERNEL_IDS = ("forward_tile", "adjoint_tile", "tangent_tile", "halo", "batched_graph", "residual_tile",
              "newton_tile", "mass_tile")

EXPORTS = ("tlfea_create_mesh", "tlfea_destroy_mesh", "tlfea_get_mesh_info", "tlfea_internal_force",
           "tlfea_internal_force_vjp", "tlfea_tangent_jvp", "tlfea_last_error", "tlfea_set_profiling",
           "tlfea_get_profile", "tlfea_reset_profile", "tlfea_node_order", "tlfea_count_inverted",
           "tlfea_internal_force_noalloc", "tlfea_mass_action", "tlfea_step_residual", "tlfea_newton_operator",
           "tlfea_newton_workspace", "tlfea_newton_step", "tlfea_create_joints", "tlfea_destroy_joints",
           "tlfea_joint_values", "tlfea_joint_scatter")


class Block(C.Structure):
    _fields_ = [("elem", C.c_int32), ("law", C.c_int32), ("n_elem", C.c_int64),
                ("conn", C.POINTER(C.c_int32)), ("theta", C.c_double * 5),
                ("damped", C.c_int32), ("tile_elems", C.c_int32),
                ("nq", C.c_int32), ("reserved", C.c_int32),
                ("qp_w", C.POINTER(C.c_double)), ("dsdxi", C.POINTER(C.c_double)),
                ("rho", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elem", C.c_int64), ("n_qp", C.c_int64),
                ("n_tiles", C.c_int64), ("n_halo_nodes", C.c_int64), ("n_partials", C.c_int64),
                ("n_blocks", C.c_int32), ("flags", C.c_int32),
                ("tile_elems_t10", C.c_int32), ("tile_elems_h8", C.c_int32),
                ("tile_elems_q27", C.c_int32), ("reserved", C.c_int32),
                ("device_bytes", C.c_int64), ("graphs_built", C.c_int64), ("graphs_updated", C.c_int64)]


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("rtol", C.c_double)]


class KrylovInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("g_norm", C.c_double), ("res_norm", C.c_double)]


class Point(C.Structure):
    _fields_ = [("elem", C.c_int32), ("nodes", C.c_int32 * 27), ("xi", C.c_double * 3)]


class Revolute(C.Structure):
    _fields_ = [("P", Point), ("Q", Point), ("R", Point), ("S", Point), ("T", Point)]


class TlfeaError(RuntimeError):
    def __init__(self, status, what, msg):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {msg}")


_lib = None


def lib():
    """Load libtlfea.so (raises ImportError if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2602_17002_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.c_void_p
    L.tlfea_create_mesh.argtypes = [C.c_int64, C.POINTER(C.c_double), C.c_int32, C.POINTER(Block), C.c_int32,
                                    vp, C.POINTER(vp)]
    L.tlfea_create_mesh.restype = C.c_int
    L.tlfea_destroy_mesh.argtypes = [vp]
    L.tlfea_destroy_mesh.restype = None
    L.tlfea_get_mesh_info.argtypes = [vp, C.POINTER(MeshInfo)]
    L.tlfea_get_mesh_info.restype = C.c_int
    L.tlfea_internal_force.argtypes = [vp, dp, dp, dp, dp, vp]
    L.tlfea_internal_force.restype = C.c_int
    L.tlfea_internal_force_noalloc.argtypes = [vp, dp, dp, dp, dp, vp]
    L.tlfea_internal_force_noalloc.restype = C.c_int
    L.tlfea_internal_force_vjp.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.tlfea_internal_force_vjp.restype = C.c_int
    L.tlfea_tangent_jvp.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
    L.tlfea_tangent_jvp.restype = C.c_int
    L.tlfea_count_inverted.argtypes = [vp, dp, vp, vp]
    L.tlfea_mass_action.argtypes = [vp, dp, dp, vp]
    L.tlfea_mass_action.restype = C.c_int
    L.tlfea_step_residual.argtypes = [vp, dp, dp, dp, C.c_double, dp, dp, dp, vp]
    L.tlfea_step_residual.restype = C.c_int
    L.tlfea_newton_operator.argtypes = [vp, dp, dp, C.c_double, dp, dp, dp, vp]
    L.tlfea_newton_operator.restype = C.c_int
    L.tlfea_newton_workspace.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.tlfea_newton_workspace.restype = C.c_int
    L.tlfea_newton_step.argtypes = [vp, dp, dp, dp, C.c_double, dp, dp, C.POINTER(KrylovOpts), dp, dp, C.c_int64,
                                    C.POINTER(KrylovInfo), vp]
    L.tlfea_newton_step.restype = C.c_int
    L.tlfea_create_joints.argtypes = [C.c_int64, C.POINTER(C.c_double), C.c_int32, C.POINTER(Revolute), vp,
                                      C.POINTER(vp)]
    L.tlfea_create_joints.restype = C.c_int
    L.tlfea_destroy_joints.argtypes = [vp]
    L.tlfea_destroy_joints.restype = None
    L.tlfea_joint_values.argtypes = [vp, dp, dp, vp]
    L.tlfea_joint_values.restype = C.c_int
    L.tlfea_joint_scatter.argtypes = [vp, dp, dp, C.c_double, C.c_double, dp, C.c_int32, vp]
    L.tlfea_joint_scatter.restype = C.c_int
    L.tlfea_count_inverted.restype = C.c_int
    L.tlfea_last_error.argtypes = []
    L.tlfea_last_error.restype = C.c_char_p
    L.tlfea_set_profiling.argtypes = [vp, C.c_int32]
    L.tlfea_set_profiling.restype = C.c_int
    L.tlfea_get_profile.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.tlfea_get_profile.restype = C.c_int
    L.tlfea_reset_profile.argtypes = [vp]
    L.tlfea_reset_profile.restype = C.c_int
    L.tlfea_node_order.argtypes = [vp, C.POINTER(C.c_int32)]
    L.tlfea_node_order.restype = C.c_int
    _lib = L
    return L


def check(status, what):
    if status != TLFEA_OK:
        msg = lib().tlfea_last_error().decode(errors="replace")
        raise TlfeaError(status, what, msg)
