"""ctypes declarations of liblbm355.so (the C ABI of include/lbm355.h).

Loading requires torch to be imported first: the library then binds to the
HIP runtime torch already loaded, so device pointers and streams are shared.
There is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM355_LIB selects an alternative build of the same library (measurements of build variants)
LIB_PATH = os.environ.get("LBM355_LIB") or os.path.join(HERE, "liblbm355.so")

LBM_OK, LBM_E_ARG, LBM_E_STATE, LBM_E_HIP, LBM_E_UNSUPPORTED, LBM_E_DIVERGED = 0, -1, -2, -3, -4, -5
DIRECT, INDIRECT = 0, 1
SOA, AOS = 0, 1
F64, F32, F16S, F32S = 0, 1, 2, 3
TS, OS_PUSH, OS_PULL, AA, ET, OS_NT, CG, SWAP = range(8)
IDENTITY, BGK, TRT = 0, 1, 2
OPT_XCD_REMAP = 1
OPT_PITCH_PAD = 2
OPT_WG_LDS = 3
OPT_ROW_STAGE = 4
OPT_PAIR = 5
OPT_BAND = 6
OPT_SLAB_ORDER = 7
OPT_RANK_LOOKUP = 8
OPT_SOA_BLOCK = 9
NOALLOC_MAX_NODES = 1 << 26   # LBM_NOALLOC_MAX_NODES

SCHEMES = {"ts": TS, "os_push": OS_PUSH, "os_pull": OS_PULL, "aa": AA, "et": ET,
           "os_nt": OS_NT, "cg": CG, "swap": SWAP}
ADDRESSING = {"direct": DIRECT, "indirect": INDIRECT}
LAYOUTS = {"soa": SOA, "aos": AOS}
PRECISIONS = {"f64": F64, "f32": F32, "f16s": F16S, "f32s": F32S}
COLLIDERS = {"identity": IDENTITY, "bgk": BGK, "trt": TRT}
BC_WALL, BC_VELOCITY, BC_PRESSURE = 0, 1, 2
BC_KINDS = {"wall": BC_WALL, "velocity": BC_VELOCITY, "pressure": BC_PRESSURE}


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("addressing", ctypes.c_int32), ("layout", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("wall_z", ctypes.c_int32), ("et_ghosts", ctypes.c_int32),
                ("omega", ctypes.c_double), ("g", ctypes.c_double * 3), ("f16_scale", ctypes.c_double),
                ("brick", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32), ("trt_lambda", ctypes.c_double)]


class Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_cells", "n_nodes", "n_ghost", "pitch", "idx_pitch", "pdf_bytes", "pdf1_bytes", "idx_bytes",
        "aux_bytes", "scratch_bytes", "cellmap_bytes", "build_scratch_bytes")]


EXPORTS = [
    "lbm_last_error", "lbm_version", "lbm_lattice", "lbm_create_grid", "lbm_destroy_grid", "lbm_set_params",
    "lbm_set_boundary",
    "lbm_set_option", "lbm_set_block_order", "lbm_query_sizes", "lbm_build_idx", "lbm_bind", "lbm_set_pdfs", "lbm_get_pdfs",
    "lbm_init_equilibrium", "lbm_step", "lbm_time", "lbm_reduce_moments", "lbm_reduce_moments_noalloc", "lbm_stream_copy", "lbm_model_bytes",
    "lbm_rank_lookup_active", "lbm_lattice_block",
    "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_destroy", "lbm_batch_add", "lbm_batch_remove",
    "lbm_batch_run", "lbm_batch_sync", "lbm_batch_moments",
]

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm355 error {code}: {msg}")
        self.code = code


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python paper_1111_0922_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    gp = ctypes.c_void_p
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = []
    lib.lbm_version.argtypes = []
    lib.lbm_lattice.argtypes = [vp, vp, vp]
    lib.lbm_create_grid.argtypes = [ctypes.POINTER(GridDesc), ctypes.POINTER(gp)]
    lib.lbm_destroy_grid.argtypes = [gp]
    lib.lbm_set_params.argtypes = [gp, dbl, ctypes.POINTER(dbl)]
    lib.lbm_set_boundary.argtypes = [gp, ctypes.c_int32, ctypes.c_int32, dbl, ctypes.POINTER(dbl)]
    lib.lbm_set_option.argtypes = [gp, i32, i64]
    lib.lbm_set_block_order.argtypes = [gp, vp, i64]
    lib.lbm_query_sizes.argtypes = [gp, i32, ctypes.POINTER(Sizes)]
    lib.lbm_build_idx.argtypes = [gp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp]
    lib.lbm_bind.argtypes = [gp, i32, vp, vp, vp, vp, vp]
    lib.lbm_set_pdfs.argtypes = [gp, vp, vp]
    lib.lbm_get_pdfs.argtypes = [gp, vp, vp]
    lib.lbm_init_equilibrium.argtypes = [gp, vp, vp]
    lib.lbm_step.argtypes = [gp, i32, i32, i64, vp]
    lib.lbm_time.argtypes = [gp]
    lib.lbm_time.restype = i64
    lib.lbm_reduce_moments.argtypes = [gp, vp, vp]
    lib.lbm_reduce_moments_noalloc.argtypes = [gp, vp, vp]
    lib.lbm_stream_copy.argtypes = [vp, vp, i64, vp]
    lib.lbm_model_bytes.argtypes = [i32, i32, i32, i32]
    lib.lbm_model_bytes.restype = dbl
    lib.lbm_rank_lookup_active.argtypes = [gp]
    lib.lbm_lattice_block.argtypes = [gp]
    lib.lbm_batch_workspace_bytes.argtypes = [i32, i64, ctypes.POINTER(i64)]
    lib.lbm_batch_create.argtypes = [i32, i64, i32, vp, ctypes.POINTER(gp)]
    lib.lbm_batch_destroy.argtypes = [gp]
    lib.lbm_batch_add.argtypes = [gp, gp, ctypes.POINTER(i32)]
    lib.lbm_batch_remove.argtypes = [gp, i32]
    lib.lbm_batch_run.argtypes = [gp, i32, vp, i32, vp]
    lib.lbm_batch_sync.argtypes = [gp, vp, vp]
    lib.lbm_batch_moments.argtypes = [gp, vp, vp]
    _lib = lib
    return lib


def check(rc):
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error().decode())
    return rc
