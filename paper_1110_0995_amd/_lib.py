"""ctypes view of the C ABI declared in include/lbmibm.h and include/magnet.h
(argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  -- load torch's HIP runtime first so the library binds to the same one

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmibm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_F64, LBM_F32, LBM_F32_DEV = 0, 1, 2
PRECISIONS = {"f64": LBM_F64, "f32": LBM_F32, "f32dev": LBM_F32_DEV}
ERRORS = {LBM_EINVAL: "EINVAL", LBM_ENOMEM: "ENOMEM", LBM_EHIP: "EHIP", LBM_ENONFINITE: "ENONFINITE",
          LBM_ESTATE: "ESTATE"}

# every symbol include/*.h declares
EXPORTS = ("lbm_plane_stride", "lbm_workspace_bytes", "lbm_init", "lbm_init_channels",
           "lbm_workspace_bytes_channels", "lbm_set_launch", "lbm_set_ibm_overlap", "lbm_set_node_records", "lbm_node_records_used", "lbm_run", "lbm_check_finite", "lbm_step",
           "lbm_step_timed", "ibm_rest_shape", "ibm_couple", "lbm_read_fields", "lbm_current", "lbm_store_f64", "lbm_load_f64", "ibm_force_jvp", "lbm_adjoint_step",
           "lbm_run_record", "lbm_adjoint_run", "lbm_destroy", "lbm_last_error",
           "mag_workspace_bytes", "mag_field", "mag_forces", "mag_run", "mag_run_static", "mag_freeze")
MAG_MAX_SHEETS = 8


class LbmParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic", C.c_int32 * 3),
                ("tau", C.c_double), ("body_force", C.c_double * 3), ("prec", C.c_int32),
                ("plane_stride", C.c_int64), ("solid", C.c_void_p), ("f_a", C.c_void_p), ("f_b", C.c_void_p),
                ("gfield", C.c_void_p), ("stream", C.c_void_p)]


class IbmContact(C.Structure):
    _fields_ = [("a", C.c_double), ("n", C.c_double), ("rcut", C.c_double), ("roff", C.c_double),
                ("dmin", C.c_double), ("cell_cell", C.c_int32), ("nplanes", C.c_int32), ("planes", C.c_void_p),
                ("ncyl", C.c_int32), ("cyl", C.c_void_p), ("cyl_off", C.c_void_p), ("nspheres", C.c_int32),
                ("spheres", C.c_void_p)]


class IbmMesh(C.Structure):
    _fields_ = [("ncells", C.c_int32), ("nverts", C.c_int32), ("ntris", C.c_int32), ("nedges", C.c_int32),
                ("vert_off", C.c_void_p), ("tri_off", C.c_void_p), ("edge_off", C.c_void_p),
                ("tri", C.c_void_p), ("hinge", C.c_void_p), ("anchor", C.c_void_p), ("cell_chan", C.c_void_p),
                ("x", C.c_void_p), ("v", C.c_void_p), ("f_el", C.c_void_p), ("moduli", C.c_void_p),
                ("l0", C.c_void_p), ("a0", C.c_void_p), ("th0", C.c_void_p), ("a0c", C.c_void_p),
                ("v0c", C.c_void_p), ("avert", C.c_void_p), ("vtri_off", C.c_void_p), ("vtri", C.c_void_p),
                ("vedge_off", C.c_void_p), ("vedge", C.c_void_p), ("xi", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
                ("contact", C.POINTER(IbmContact)), ("stretch_law", C.c_int32), ("max_cell_verts", C.c_int32), ("max_cell_tris", C.c_int32), ("max_cell_edges", C.c_int32),
                ("checked", C.c_uint32)]


class MagParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("nsheets", C.c_int32), ("sheets", (C.c_double * 6) * MAG_MAX_SHEETS),
                ("bias", C.c_double * 3), ("a", C.c_double), ("chi", C.c_double), ("eta", C.c_double),
                ("dt", C.c_double), ("rep_a", C.c_double), ("rep_n", C.c_double), ("rep_cut", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic", C.c_int32 * 3),
                ("walls_z", C.c_int32), ("stream", C.c_void_p)]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load liblbmibm.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it first (python -m paper_1110_0995_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.lbm_plane_stride.argtypes = [C.c_int64, C.c_int32]
    L.lbm_plane_stride.restype = C.c_int64
    L.lbm_workspace_bytes.argtypes = [C.POINTER(LbmParams)]
    L.lbm_workspace_bytes.restype = C.c_int64
    L.lbm_init.argtypes = [C.POINTER(LbmParams), C.POINTER(vp)]
    L.lbm_init_channels.argtypes = [C.POINTER(LbmParams), C.c_int32, C.POINTER(C.c_int32), C.POINTER(vp)]
    L.lbm_workspace_bytes_channels.argtypes = [C.POINTER(LbmParams), C.c_int32, C.POINTER(C.c_int32)]
    L.lbm_workspace_bytes_channels.restype = C.c_int64
    L.lbm_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
    L.lbm_set_ibm_overlap.argtypes = [vp, C.c_int32]
    L.lbm_set_node_records.argtypes = [vp, C.c_int32]
    L.lbm_node_records_used.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lbm_check_finite.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lbm_run.argtypes = [vp, C.POINTER(IbmMesh), C.c_int32, C.c_int32]
    L.lbm_step.argtypes = [vp, C.c_int32]
    L.lbm_step_timed.argtypes = [vp, vp, vp]
    L.ibm_rest_shape.argtypes = [vp, C.POINTER(IbmMesh)]
    L.ibm_couple.argtypes = [vp, C.POINTER(IbmMesh)]
    L.lbm_read_fields.argtypes = [vp, vp, vp, C.POINTER(C.c_double)]
    L.lbm_current.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_int64)]
    L.lbm_store_f64.argtypes = [vp, vp]
    L.lbm_load_f64.argtypes = [vp, vp]
    L.ibm_force_jvp.argtypes = [vp, C.POINTER(IbmMesh), vp, vp, vp, vp]
    L.lbm_adjoint_step.argtypes = [vp, C.POINTER(IbmMesh), vp, vp, vp, vp, vp, vp, vp, vp]
    L.lbm_run_record.argtypes = [vp, C.POINTER(IbmMesh), C.c_int32, vp, vp, vp, C.c_int32]
    L.lbm_adjoint_run.argtypes = [vp, C.POINTER(IbmMesh), C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    mp = C.POINTER(MagParams)
    L.mag_workspace_bytes.argtypes = [mp]
    L.mag_workspace_bytes.restype = C.c_int64
    L.mag_field.argtypes = [mp, vp, C.c_int32, vp, vp]
    L.mag_forces.argtypes = [mp, vp, vp, vp, vp]
    L.mag_run.argtypes = [mp, vp, C.c_int32, vp]
    L.mag_run_static.argtypes = [mp, vp, C.c_int32]
    L.mag_freeze.argtypes = [mp, vp, vp]
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = C.c_char_p
    for name in ("lbm_init", "lbm_init_channels", "lbm_set_launch", "lbm_set_ibm_overlap", "lbm_set_node_records",
                 "lbm_node_records_used", "lbm_run", "lbm_check_finite", "lbm_step",
                 "lbm_step_timed", "ibm_rest_shape", "ibm_couple", "lbm_read_fields", "lbm_current", "lbm_store_f64", "lbm_load_f64", "ibm_force_jvp",
                 "lbm_adjoint_step", "lbm_run_record", "lbm_adjoint_run", "mag_field", "mag_forces", "mag_run", "mag_run_static",
                 "mag_freeze"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error().decode())
