"""ctypes declarations of the C ABI in include/lbm.h, include/lbm_mlp.h and
include/lbm3d.h (argument marshalling only).

Loading fails loudly when ``liblbm.so`` has not been built: there is no
fallback implementation of any entry point.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
STATUS_NAMES = {0: "LBM_OK", 1: "LBM_ERR_INVALID", 2: "LBM_ERR_DEVICE", 3: "LBM_ERR_OOM",
                4: "LBM_ERR_UNSTABLE", 5: "LBM_ERR_BUDGET", 6: "LBM_ERR_UNSUPPORTED"}

GEOM_BOX, GEOM_CHANNEL, GEOM_MASK = 0, 1, 2
INIT_UNIFORM, INIT_DROPLET, INIT_LAYERS, INIT_SLUG = 0, 1, 2, 3
STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2

# Every symbol include/lbm.h declares.
EXPORTED = [
    "lbm_last_error", "lbm_version", "lbm_required_bytes", "lbm_init", "lbm_step",
    "lbm_time", "lbm_set_fluid", "lbm_moments", "lbm_monitors", "lbm_get_populations",
    "lbm_fluid_mask", "lbm_set_tiling", "lbm_get_tiling", "lbm_destroy", "lbm_set_active",
    "lbm_snapshot_save", "lbm_snapshot_restore", "lbm_cp_default_options",
    "lbm_cp_required_bytes", "lbm_critical_pressure", "lbm_cp_drive",
    "lbm_set_instance_tiling", "lbm_get_instance_tiling", "lbm_autotune",
    "lbm_mlp_workspace_bytes", "lbm_mlp_forward", "lbm_mlp_backward", "lbm_mlp_adam",
    "lbm3d_required_bytes", "lbm3d_init", "lbm3d_step", "lbm3d_time", "lbm3d_set_fluid",
    "lbm3d_moments", "lbm3d_monitors", "lbm3d_get_populations", "lbm3d_fluid_mask",
    "lbm3d_set_tiling", "lbm3d_get_tiling", "lbm3d_snapshot_save", "lbm3d_snapshot_restore",
    "lbm3d_destroy", "lbm3d_cp_required_bytes", "lbm3d_critical_pressure",
    "lbm_stream_copy", "lbm_mlp_gradient_noalloc",
]

GEOM3_BOX, GEOM3_TUBE, GEOM3_MASK = 0, 1, 2
INIT3_UNIFORM, INIT3_DROPLET, INIT3_SLUG = 0, 1, 3

OPT_SNAPSHOT = 0x100
CP_UNDECIDED, CP_UNSTABLE, CP_WIDENED, CP_NOT_CONVERGED = 1, 2, 4, 8
MAX_SLUGS = 8
CP_BISECT, CP_RAMP = 0, 1


class LbmTuneReport(ctypes.Structure):
    _fields_ = [("buckets", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("ms_before", ctypes.c_double),
                ("ms_after", ctypes.c_double)]


class LbmGeom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("wall_interp", ctypes.c_int32), ("lam", ctypes.c_double),
                ("h0", ctypes.c_double), ("a", ctypes.c_double),
                ("mask", ctypes.POINTER(ctypes.c_uint8)), ("y_offset", ctypes.c_double),
                ("island_h", ctypes.c_double), ("island_len", ctypes.c_double)]


class LbmFluid(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double * 2), ("G", ctypes.c_double),
                ("rho_s", ctypes.c_double * 2), ("g", ctypes.c_double * 2),
                ("reg_order", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LbmInitFields(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("wall_rows", ctypes.c_int32),
                ("core_species", ctypes.c_int32), ("n_slugs", ctypes.c_int32),
                ("rho_hi", ctypes.c_double), ("rho_lo", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("r", ctypes.c_double),
                ("x0", ctypes.c_double), ("length", ctypes.c_double),
                ("slugs", ctypes.POINTER(ctypes.c_double)), ("width", ctypes.c_double)]


class LbmMonitor(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 2), ("momentum", ctypes.c_double * 2),
                ("oil_flux", ctypes.c_double), ("oil_cos", ctypes.c_double),
                ("oil_sin", ctypes.c_double), ("bad_nodes", ctypes.c_double)]


class LbmCpProblem(ctypes.Structure):
    _fields_ = [("geom", LbmGeom), ("fluid", LbmFluid), ("init", LbmInitFields),
                ("sigma", ctypes.c_double), ("rho_bar", ctypes.c_double),
                ("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double),
                ("equil_steps", ctypes.c_int64), ("max_steps", ctypes.c_int64),
                ("min_steps", ctypes.c_int64)]


class LbmCpOptions(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("move_frac", ctypes.c_double),
                ("creep_frac", ctypes.c_double), ("still_frac", ctypes.c_double),
                ("chunk_steps", ctypes.c_int32), ("still_chunks", ctypes.c_int32),
                ("max_probes", ctypes.c_int32), ("verify_bracket", ctypes.c_int32),
                ("min_steps", ctypes.c_int64), ("storage", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("protocol", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("ramp_dg", ctypes.c_double),
                ("ramp_steps", ctypes.c_int64)]


class LbmCpResult(ctypes.Structure):
    _fields_ = [("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double),
                ("g_crit", ctypes.c_double), ("bo_crit", ctypes.c_double),
                ("probes", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("steps", ctypes.c_int64)]


class Lbm3dGeom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("lam", ctypes.c_double), ("r0", ctypes.c_double),
                ("a", ctypes.c_double), ("mask", ctypes.POINTER(ctypes.c_uint8)),
                ("wall_interp", ctypes.c_int32)]


class Lbm3dFluid(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double * 2), ("G", ctypes.c_double),
                ("rho_s", ctypes.c_double * 2), ("g", ctypes.c_double * 3)]


class Lbm3dInitFields(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_slugs", ctypes.c_int32),
                ("rho_hi", ctypes.c_double), ("rho_lo", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double),
                ("r", ctypes.c_double), ("x0", ctypes.c_double), ("length", ctypes.c_double),
                ("slugs", ctypes.POINTER(ctypes.c_double)), ("width", ctypes.c_double)]


class Lbm3dCpProblem(ctypes.Structure):
    _fields_ = [("geom", Lbm3dGeom), ("fluid", Lbm3dFluid), ("init", Lbm3dInitFields),
                ("sigma", ctypes.c_double), ("rho_bar", ctypes.c_double),
                ("g_lo", ctypes.c_double), ("g_hi", ctypes.c_double),
                ("equil_steps", ctypes.c_int64), ("max_steps", ctypes.c_int64),
                ("min_steps", ctypes.c_int64)]


CP_BEGIN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double)
CP_ADVANCE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8),
                              ctypes.c_int64)
CP_MONITORS = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(LbmMonitor))
CP_SET_FORCING = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double)


class LbmCpEngine(ctypes.Structure):
    _fields_ = [("begin_probe", CP_BEGIN), ("advance", CP_ADVANCE), ("monitors", CP_MONITORS),
                ("user", ctypes.c_void_p), ("set_forcing", CP_SET_FORCING)]


_LIB = None


def load():
    """Load liblbm.so (raises if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    # PyTorch (which provides device memory and streams) ships a HIP runtime;
    # load it first so that the library binds to the same runtime instance
    # instead of bringing in a second one.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (expected at %s); run "
                          "paper_1601_00918_amd/build.py or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = []
    lib.lbm_version.restype = ctypes.c_char_p
    lib.lbm_version.argtypes = []
    lib.lbm_required_bytes.argtypes = [ctypes.POINTER(LbmGeom), i32, i32, ctypes.POINTER(sz)]
    lib.lbm_init.argtypes = [ctypes.POINTER(LbmGeom), ctypes.POINTER(LbmFluid),
                             ctypes.POINTER(LbmInitFields), i32, i32, vp, sz, vp,
                             ctypes.POINTER(vp)]
    lib.lbm_step.argtypes = [vp, i64]
    lib.lbm_time.argtypes = [vp]
    lib.lbm_time.restype = i64
    lib.lbm_set_fluid.argtypes = [vp, i32, ctypes.POINTER(LbmFluid)]
    lib.lbm_moments.argtypes = [vp, i32, dp, dp, dp, ctypes.POINTER(LbmMonitor)]
    lib.lbm_monitors.argtypes = [vp, ctypes.POINTER(LbmMonitor)]
    lib.lbm_get_populations.argtypes = [vp, i32, dp]
    lib.lbm_fluid_mask.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint8)]
    lib.lbm_set_tiling.argtypes = [vp, i32, i32]
    lib.lbm_get_tiling.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
    lib.lbm_set_instance_tiling.argtypes = [vp, i32, i32, i32]
    lib.lbm_get_instance_tiling.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.lbm_autotune.argtypes = [vp, i32, ctypes.POINTER(LbmTuneReport)]
    lib.lbm_set_active.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
    lib.lbm_snapshot_save.argtypes = [vp]
    lib.lbm_snapshot_restore.argtypes = [vp, i32]
    lib.lbm_cp_default_options.argtypes = [ctypes.POINTER(LbmCpOptions)]
    lib.lbm_cp_default_options.restype = None
    lib.lbm_cp_required_bytes.argtypes = [ctypes.POINTER(LbmCpProblem), i32, ctypes.POINTER(sz)]
    lib.lbm_critical_pressure.argtypes = [ctypes.POINTER(LbmCpProblem), i32,
                                          ctypes.POINTER(LbmCpOptions), vp, sz, vp,
                                          ctypes.POINTER(LbmCpResult)]
    lib.lbm_cp_drive.argtypes = [ctypes.POINTER(LbmCpEngine), ctypes.POINTER(LbmCpProblem), i32,
                                 ctypes.POINTER(LbmCpOptions), ctypes.POINTER(LbmCpResult)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_mlp_workspace_bytes.argtypes = [i32]
    lib.lbm_mlp_workspace_bytes.restype = sz
    lib.lbm_mlp_forward.argtypes = [vp, vp, i32, vp, vp, sz, vp]
    lib.lbm_mlp_backward.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]
    fl = ctypes.c_float
    lib.lbm_mlp_adam.argtypes = [vp, vp, vp, vp, i32, fl, fl, fl, fl, vp]
    lib.lbm3d_required_bytes.argtypes = [ctypes.POINTER(Lbm3dGeom), i32, ctypes.POINTER(sz)]
    lib.lbm3d_init.argtypes = [ctypes.POINTER(Lbm3dGeom), ctypes.POINTER(Lbm3dFluid),
                               ctypes.POINTER(Lbm3dInitFields), i32, vp, sz, vp,
                               ctypes.POINTER(vp)]
    lib.lbm3d_step.argtypes = [vp, i64]
    lib.lbm3d_time.argtypes = [vp]
    lib.lbm3d_time.restype = i64
    lib.lbm3d_set_fluid.argtypes = [vp, ctypes.POINTER(Lbm3dFluid)]
    lib.lbm3d_moments.argtypes = [vp, dp, dp, dp, ctypes.POINTER(LbmMonitor)]
    lib.lbm3d_monitors.argtypes = [vp, ctypes.POINTER(LbmMonitor)]
    lib.lbm3d_get_populations.argtypes = [vp, dp]
    lib.lbm3d_fluid_mask.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
    lib.lbm3d_set_tiling.argtypes = [vp, i32, i32, i32]
    lib.lbm3d_get_tiling.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.lbm3d_snapshot_save.argtypes = [vp]
    lib.lbm3d_snapshot_restore.argtypes = [vp]
    lib.lbm3d_cp_required_bytes.argtypes = [ctypes.POINTER(Lbm3dCpProblem), i32, i32,
                                            ctypes.POINTER(sz)]
    lib.lbm3d_critical_pressure.argtypes = [ctypes.POINTER(Lbm3dCpProblem), i32,
                                            ctypes.POINTER(LbmCpOptions), vp, sz, vp,
                                            ctypes.POINTER(LbmCpResult)]
    lib.lbm3d_destroy.argtypes = [vp]
    lib.lbm_stream_copy.argtypes = [vp, vp, sz, sz, vp]
    lib.lbm_mlp_gradient_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    lib.lbm3d_destroy.restype = None
    for name in EXPORTED:
        if name not in ("lbm_last_error", "lbm_version", "lbm_time", "lbm_destroy",
                        "lbm_cp_default_options", "lbm_mlp_workspace_bytes", "lbm3d_time",
                        "lbm3d_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


class LbmError(RuntimeError):
    def __init__(self, status, where):
        msg = load().lbm_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, where):
    if status != LBM_OK:
        raise LbmError(status, where)
