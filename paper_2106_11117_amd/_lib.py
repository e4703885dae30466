"""ctypes declarations of the C ABI in include/lfltsmc.h (marshalling only).

Loads ``liblfltsmc.so`` from this package directory.  There is no fallback:
if the library is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblfltsmc.so")

LTS_OK, LTS_ERR_ARG, LTS_ERR_HIP, LTS_ERR_OOM, LTS_ERR_UNSTABLE, LTS_ERR_STATE = 0, -1, -2, -3, -4, -5
LTS_FP64, LTS_FP32_STEP = 0, 1
LTS_PTR_HOST, LTS_PTR_DEVICE = 0, 1
LTS_NODE_DOF, LTS_NODE_P, LTS_NODE_FPLUS = 1, 2, 4
LTS_RULE_BOX, LTS_RULE_GRADED_L, LTS_RULE_LF = 0, 1, 0x100
LTS_BATCH_GRAPH = 1
LTS_BATCH_FP32 = 2
LTS_BATCH_PERSIST = 4
LTS_BATCH_SB1 = 8
LTS_BATCH_SB2 = 16
LTS_BATCH_SB_MASK = 24
LTS_BATCH_AUTO = 32
LTS_BATCH_MLTS = 64
LTS_MESH_REGION_CAP = 2048
LTS_MLTS_MAX_TIERS = 5
LTS_MLTS_MAX_P = 16
LTS_MESH_MAX_DEGREE = 12
LTS_MLMC_BATCHED, LTS_MLMC_PLAIN = 0, 1
LTS_FINE_HALF_H, LTS_FINE_TIERS, LTS_FINE_QOPT = 0, 1, 2
LTS_LINE_KL, LTS_LINE_JUMP = 0, 1
LTS_MAX_LEVELS = 8
LTS_NOALLOC_SCRATCH_BYTES = 64 << 20

_ERR_NAMES = {LTS_ERR_ARG: "LTS_ERR_ARG", LTS_ERR_HIP: "LTS_ERR_HIP", LTS_ERR_OOM: "LTS_ERR_OOM",
              LTS_ERR_UNSTABLE: "LTS_ERR_UNSTABLE", LTS_ERR_STATE: "LTS_ERR_STATE"}

dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int32)
u8p = C.POINTER(C.c_uint8)
u64p = C.POINTER(C.c_uint64)


class GridDesc(C.Structure):
    _fields_ = [("nx_cells", C.c_int32), ("ny_cells", C.c_int32), ("x", dp), ("y", dp),
                ("cell_active", u8p), ("cell_block", ip), ("cell_fine", u8p), ("cell_qoi", u8p),
                ("n_blocks", C.c_int32), ("h", C.c_double), ("p", C.c_int32), ("nu", C.c_double)]


class RectRule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lo", C.c_double), ("hi", C.c_double), ("n_base", C.c_int32),
                ("box_lo", C.c_double), ("box_hi", C.c_double), ("ref", C.c_int32),
                ("layers", C.c_int32), ("nbx", C.c_int32), ("nby", C.c_int32),
                ("qx_lo", C.c_double), ("qx_hi", C.c_double), ("qy_lo", C.c_double),
                ("qy_hi", C.c_double), ("p", C.c_int32), ("nu", C.c_double),
                ("fine_rule", C.c_int32), ("fine_tiers", C.c_int32), ("p_max", C.c_int32)]


class LevelInfo(C.Structure):
    _fields_ = [("nx_nodes", C.c_int32), ("ny_nodes", C.c_int32), ("n_dof", C.c_int32),
                ("n_P", C.c_int32), ("n_Fplus", C.c_int32), ("p", C.c_int32),
                ("n_blocks", C.c_int32), ("h", C.c_double), ("nu", C.c_double),
                ("delta", C.c_double), ("omega", C.c_double), ("tile_x", C.c_int32),
                ("tile_y", C.c_int32), ("tile_rect", C.c_int32), ("tuned", C.c_int32),
                ("halo_ratio", C.c_double), ("tuned_ms", C.c_double)]


class TilingInfo(C.Structure):
    _fields_ = [("n_fine", C.c_int32), ("n_coarse", C.c_int32), ("tile_x", C.c_int32),
                ("tile_y", C.c_int32), ("tile_rect", C.c_int32), ("max_region", C.c_int32),
                ("regions_exact", C.c_int32), ("threads", C.c_int32), ("halo_ratio", C.c_double)]


class SampleRule(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("sigma", C.c_double), ("px_lo", C.c_double),
                ("px_hi", C.c_double), ("py_lo", C.c_double), ("py_hi", C.c_double),
                ("width", C.c_double), ("T", C.c_double), ("cfl", C.c_double)]


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tris", C.c_int32), ("n_blocks", C.c_int32),
                ("xy", C.c_void_p), ("tri", C.c_void_p), ("dirichlet", C.c_void_p), ("tri_block", C.c_void_p),
                ("tri_fine", C.c_void_p), ("qoi_w", C.c_void_p), ("h", C.c_double), ("p", C.c_int32),
                ("nu", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tris", C.c_int32), ("n_dof", C.c_int32), ("n_P", C.c_int32),
                ("n_Fplus", C.c_int32), ("n_edges", C.c_int32), ("max_degree", C.c_int32),
                ("n_tiles", C.c_int32), ("max_region", C.c_int32), ("p", C.c_int32), ("n_blocks", C.c_int32),
                ("h", C.c_double), ("nu", C.c_double), ("delta", C.c_double), ("omega", C.c_double),
                ("halo_ratio", C.c_double)]


class MltsDesc(C.Structure):
    _fields_ = [("n_tiers", C.c_int32), ("p", C.c_int32 * LTS_MLTS_MAX_TIERS), ("cell_tier", C.c_void_p),
                ("max_region", C.c_int32)]


class MltsInfo(C.Structure):
    _fields_ = [("n_tiers", C.c_int32), ("p", C.c_int32 * LTS_MLTS_MAX_TIERS),
                ("n_P", C.c_int32 * LTS_MLTS_MAX_TIERS), ("phases", C.c_int32), ("n_tiles", C.c_int32),
                ("max_region", C.c_int32), ("threads", C.c_int32), ("halo_ratio", C.c_double),
                ("updates_per_step", C.c_double)]


class Samples(C.Structure):
    _fields_ = [("n", C.c_int32), ("ptr_kind", C.c_int32), ("kappa", C.c_void_p), ("x0", C.c_void_p),
                ("n_steps", C.c_void_p), ("dt", C.c_void_p), ("width", C.c_double), ("g", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("level", C.c_int32), ("samples", Samples), ("q_offset", C.c_int32)]


class MLMCOpts(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level_ids", C.c_int32 * LTS_MAX_LEVELS),
                ("rule", SampleRule), ("seed", C.c_uint64), ("eps", C.c_double),
                ("alpha", C.c_double), ("L_start", C.c_int32),
                ("N_init", C.c_int32 * LTS_MAX_LEVELS), ("mode", C.c_int32),
                ("max_total_samples", C.c_int32), ("n_levels_max", C.c_int32), ("gen_rule", RectRule),
                ("level_kind", C.c_int32), ("gen_mlts", MltsDesc)]


class MLMCResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("L", C.c_int32), ("N", C.c_int32 * LTS_MAX_LEVELS),
                ("mean", C.c_double * LTS_MAX_LEVELS), ("var", C.c_double * LTS_MAX_LEVELS),
                ("cost", C.c_double * LTS_MAX_LEVELS), ("bias", C.c_double), ("rmse", C.c_double),
                ("converged", C.c_int32), ("seconds", C.c_double),
                ("level_ids", C.c_int32 * LTS_MAX_LEVELS)]


class LineRule(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("H", C.c_double), ("fine_lo", C.c_double),
                ("fine_hi", C.c_double), ("h_fine", C.c_double), ("nu", C.c_double), ("lf", C.c_int32)]


class LineInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_P", C.c_int32), ("p", C.c_int32), ("f0", C.c_int32),
                ("n_fplus", C.c_int32), ("H", C.c_double), ("nu", C.c_double)]


class LineSampleRule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("jump_lo", C.c_double), ("jump_hi", C.c_double), ("c_left", C.c_double),
                ("c_right", C.c_double), ("pulse_x", C.c_double), ("pulse_w2", C.c_double), ("T", C.c_double),
                ("cfl", C.c_double)]


class LineMLMCOpts(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("line_ids", C.c_int32 * LTS_MAX_LEVELS), ("rule", LineSampleRule),
                ("seed", C.c_uint64), ("eps", C.c_double), ("alpha", C.c_double), ("L_start", C.c_int32),
                ("N_init", C.c_int32 * LTS_MAX_LEVELS)]


class LineMLMCResult(C.Structure):
    _fields_ = [("L", C.c_int32), ("N", C.c_int32 * LTS_MAX_LEVELS), ("var", C.c_double * LTS_MAX_LEVELS),
                ("mean_norm", C.c_double * LTS_MAX_LEVELS), ("cost", C.c_double * LTS_MAX_LEVELS),
                ("bias", C.c_double), ("rmse", C.c_double), ("converged", C.c_int32), ("n_nodes", C.c_int32),
                ("seconds", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("step_kernel_ms", C.c_double), ("step_launches", C.c_int64), ("total_ms", C.c_double),
                ("dof_updates", C.c_double), ("alg_bytes", C.c_double), ("batch_form", C.c_int32),
                ("batch_sb_cap", C.c_int32)]


# (name, restype, argtypes) of every exported entry point of include/lfltsmc.h
SIGNATURES = [
    ("lts_create", C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    ("lts_destroy", C.c_int32, [C.c_void_p]),
    ("lts_last_error", C.c_char_p, [C.c_void_p]),
    ("lts_add_level", C.c_int32, [C.c_void_p, C.POINTER(GridDesc), ip]),
    ("lts_build_rect_level", C.c_int32, [C.c_void_p, C.POINTER(RectRule), ip]),
    ("lts_level_info_get", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(LevelInfo)]),
    ("lts_level_arrays", C.c_int32, [C.c_void_p, C.c_int32, dp, dp, u8p, dp, dp, ip]),
    ("lts_gen_samples", C.c_int32, [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.POINTER(SampleRule),
                                    C.c_double, dp, dp, dp, ip, dp]),
    ("lts_philox4x64_10", C.c_int32, [u64p, u64p, u64p]),
    ("lts_rect_level_host", C.c_int32, [C.POINTER(RectRule), C.POINTER(LevelInfo), dp, dp, u8p, dp, dp,
                                        ip]),
    ("lts_tiling_host", C.c_int32, [C.POINTER(RectRule), C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(TilingInfo), ip]),
    ("lts_cheb_constants", C.c_int32, [C.c_int32, C.c_double, C.c_double, dp, dp, dp, dp, dp]),
    ("lts_forward", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_int32, C.c_void_p]),
    ("lts_forward_plain", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_int32, C.c_void_p]),
    ("lts_forward_noalloc", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_int32, C.c_void_p]),
    ("lts_forward_coupled", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Samples),
                                        C.POINTER(Samples), C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    ("lts_batch_run", C.c_int32, [C.c_void_p, C.POINTER(Job), C.c_int32, C.c_int32, C.c_void_p]),
    ("lts_autotune", C.c_int32, [C.c_void_p, C.c_int32]),
    ("lts_set_tiling", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("lts_moments", C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, dp]),
    ("lts_backward", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_void_p, C.c_int32,
                                 C.c_void_p, C.c_void_p]),
    ("lts_mlmc", C.c_int32, [C.c_void_p, C.POINTER(MLMCOpts), C.POINTER(MLMCResult)]),
    ("lts_mlmc_grad", C.c_int32, [C.c_void_p, C.POINTER(MLMCOpts), C.c_int32, C.POINTER(MLMCResult), dp, dp,
                                  dp]),
    ("lts_build_line_level", C.c_int32, [C.c_void_p, C.POINTER(LineRule), ip]),
    ("lts_line_level_host", C.c_int32, [C.POINTER(LineRule), C.POINTER(LineInfo), dp, dp, u8p]),
    ("lts_gen_line_samples", C.c_int32, [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.POINTER(LineSampleRule),
                                         C.POINTER(LineRule), dp, ip, dp]),
    ("lts_line_forward", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(LineSampleRule), C.c_void_p]),
    ("lts_line_mlmc", C.c_int32, [C.c_void_p, C.POINTER(LineMLMCOpts), C.POINTER(LineMLMCResult), dp]),
    ("lts_set_timing", C.c_int32, [C.c_void_p, C.c_int32]),
    ("lts_get_timing", C.c_int32, [C.c_void_p, C.POINTER(Timing)]),
    ("lts_set_barrier_timeout", C.c_int32, [C.c_void_p, C.c_double]),
    ("lts_add_mesh", C.c_int32, [C.c_void_p, C.POINTER(MeshDesc), ip]),
    ("lts_mesh_info_get", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(MeshInfo)]),
    ("lts_mesh_host", C.c_int32, [C.POINTER(MeshDesc), C.POINTER(MeshInfo), u8p, dp]),
    ("lts_mesh_forward", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_int32, C.c_void_p]),
    ("lts_mesh_forward_coupled", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Samples),
                                             C.POINTER(Samples), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lts_set_mlts", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(MltsDesc)]),
    ("lts_mlts_info_get", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(MltsInfo)]),
    ("lts_mlts_host", C.c_int32, [C.c_void_p, C.POINTER(MltsDesc), C.POINTER(MltsInfo), u8p]),
    ("lts_mlts_forward", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Samples), C.c_int32, C.c_void_p]),
]

_lib = None


class LtsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


def load() -> C.CDLL:
    """Load the shared library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2106_11117_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
