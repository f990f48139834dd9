"""ctypes loader for libcosmo_unroll.so (the C ABI in include/cosmo_unroll.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Importing this module does not touch the GPU; loading fails loudly
when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcosmo_unroll.so")

COSMO_OK, COSMO_EINVAL, COSMO_ENOMEM, COSMO_EHIP, COSMO_EUNSUPPORTED = 0, -1, -2, -3, -4
COSMO_PSD_STATIC_SCRATCH_BYTES = 64 << 20   # include/cosmo_unroll.h
COSMO_F32, COSMO_F64 = 0, 1
CONE_CODES = {"zero": 0, "nonneg": 1, "soc": 2, "psd": 3}

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTED = [
    "cosmo_status_string", "cosmo_last_error", "cosmo_abi_version",
    "cosmo_plan_create", "cosmo_plan_destroy", "cosmo_workspace_size", "cosmo_tape_offsets",
    "cosmo_unroll_forward", "cosmo_unroll_backward", "cosmo_residual_loss",
    "cosmo_proj_workspace_size", "psd_proj", "psd_proj_static_scratch", "psd_proj_vjp", "socp_proj", "socp_proj_vjp",
    "cosmo_plan_set_profiling", "cosmo_plan_profile_read", "cosmo_plan_set_tap",
    "cosmo_plan_set_pcg_form", "cosmo_plan_get_pcg_form", "cosmo_plan_autotune",
    "cosmo_plan_set_graph", "cosmo_plan_get_graph",
    "cosmo_plan_set_psd_schedule", "cosmo_plan_get_psd_schedule", "cosmo_plan_psd_tune_ms",
    "cosmo_plan_get_schedule", "cosmo_plan_set_schedule", "cosmo_plan_signature",
    "cosmo_schedule_cache_load", "cosmo_schedule_cache_store", "cosmo_plan_autotune_cached",
    "psd_proj_vjp_rule", "psd_ns_tape_size", "psd_proj_ns", "psd_proj_ns_vjp",
    "cosmo_policy_sizes", "cosmo_policy_forward", "cosmo_policy_backward",
    "cosmo_solve_size", "cosmo_solve",
]

# The learned policy's flat parameter vector (include/cosmo_unroll.h)
COSMO_POLICY_PARAMS = 2631

PSD_RULES = {"dk": 0, "naive": 1, "tikhonov": 2}


DENSE_MAX_PLACEMENTS = 4
DENSE_MAX_COLS = 1024


class CosmoDenseBlock(ctypes.Structure):
    _fields_ = [
        ("val", ctypes.c_void_p),
        ("rows", ctypes.c_int32),
        ("cols", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("col0", ctypes.c_int64),
        ("n_place", ctypes.c_int32),
        ("val_f32", ctypes.c_int32),
        ("row0", ctypes.c_int64 * DENSE_MAX_PLACEMENTS),
        ("scale", ctypes.c_double * DENSE_MAX_PLACEMENTS),
    ]


class CosmoProblem(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int32),
        ("n_off", ctypes.POINTER(ctypes.c_int64)),
        ("m_off", ctypes.POINTER(ctypes.c_int64)),
        ("A_rowptr", ctypes.c_void_p),
        ("A_col", ctypes.c_void_p),
        ("A_val", ctypes.c_void_p),
        ("A_nnz", ctypes.c_int64),
        ("P_rowptr", ctypes.c_void_p),
        ("P_col", ctypes.c_void_p),
        ("P_val", ctypes.c_void_p),
        ("P_nnz", ctypes.c_int64),
        ("q", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("n_cones", ctypes.c_int32),
        ("cone_kind", ctypes.POINTER(ctypes.c_int32)),
        ("cone_size", ctypes.POINTER(ctypes.c_int32)),
        ("n_dense", ctypes.c_int32),
        ("dense", ctypes.POINTER(CosmoDenseBlock)),
    ]


class CosmoOptions(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("cg_tol", ctypes.c_double),
        ("cg_max_iter", ctypes.c_int32),
        ("eig_max_sweeps", ctypes.c_int32),
        ("eig_tol", ctypes.c_double),
        ("eig_refine", ctypes.c_int32),
        ("eig_warm_start", ctypes.c_int32),
    ]


class CosmoSolveOptions(ctypes.Structure):
    _fields_ = [
        ("rho0", ctypes.c_double),
        ("eq_scale", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("eps_abs", ctypes.c_double),
        ("eps_rel", ctypes.c_double),
        ("tol_factor", ctypes.c_double),
        ("rho_min", ctypes.c_double),
        ("rho_max", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("interval", ctypes.c_int32),
        ("adapt", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class CosmoStats(ctypes.Structure):
    _fields_ = [("cg_iters_max", ctypes.c_int32), ("cg_not_converged", ctypes.c_int32),
                ("eig_sweeps_max", ctypes.c_int32), ("eig_not_converged", ctypes.c_int32),
                ("nonfinite", ctypes.c_int32), ("eig_sweeps_total", ctypes.c_int32),
                ("eig_solves", ctypes.c_int32), ("cg_iters_total", ctypes.c_int32),
                ("cg_passes_total", ctypes.c_int32), ("eig_refine_steps_total", ctypes.c_int32)]


class CosmoSchedule(ctypes.Structure):
    _fields_ = [("pcg_form", ctypes.c_int32), ("graph", ctypes.c_int32), ("eig_threads", ctypes.c_int32 * 4),
                ("vjp_threads", ctypes.c_int32)]

    def as_dict(self):
        return {"pcg_form": self.pcg_form, "graph": bool(self.graph), "eig_threads": list(self.eig_threads),
                "vjp_threads": self.vjp_threads}


STATS_FIELDS = ["cg_iters_max", "cg_not_converged", "eig_sweeps_max", "eig_not_converged", "nonfinite",
                "eig_sweeps_total", "eig_solves", "cg_iters_total",
                "cg_passes_total", "eig_refine_steps_total"]
STATS_INTS = len(STATS_FIELDS)

_lib = None


class CosmoError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _sig(lib):
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P32 = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    lib.cosmo_status_string.restype = ctypes.c_char_p
    lib.cosmo_status_string.argtypes = [ctypes.c_int]
    lib.cosmo_last_error.restype = ctypes.c_char_p
    lib.cosmo_last_error.argtypes = []
    lib.cosmo_abi_version.restype = i32
    lib.cosmo_plan_create.restype = ctypes.c_int
    lib.cosmo_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(CosmoProblem), ctypes.POINTER(CosmoOptions)]
    lib.cosmo_plan_destroy.restype = ctypes.c_int
    lib.cosmo_plan_destroy.argtypes = [vp]
    lib.cosmo_workspace_size.restype = ctypes.c_int
    lib.cosmo_workspace_size.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.cosmo_tape_offsets.restype = ctypes.c_int
    lib.cosmo_tape_offsets.argtypes = [vp, i32] + [ctypes.POINTER(sz)] * 5
    lib.cosmo_unroll_forward.restype = ctypes.c_int
    lib.cosmo_unroll_forward.argtypes = [vp] * 13
    lib.cosmo_unroll_backward.restype = ctypes.c_int
    lib.cosmo_unroll_backward.argtypes = [vp] * 15
    lib.cosmo_residual_loss.restype = ctypes.c_int
    lib.cosmo_residual_loss.argtypes = [vp] * 10
    lib.cosmo_proj_workspace_size.restype = sz
    lib.cosmo_proj_workspace_size.argtypes = [i32, P32]
    lib.cosmo_plan_set_tap.restype = ctypes.c_int
    lib.cosmo_plan_set_tap.argtypes = [vp, vp]
    lib.cosmo_policy_sizes.restype = ctypes.c_int
    lib.cosmo_policy_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.cosmo_policy_forward.restype = ctypes.c_int
    lib.cosmo_policy_forward.argtypes = [vp] * 17
    lib.cosmo_policy_backward.restype = ctypes.c_int
    lib.cosmo_policy_backward.argtypes = [vp] * 16
    lib.cosmo_solve_size.restype = ctypes.c_int
    lib.cosmo_solve_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.cosmo_solve.restype = ctypes.c_int
    lib.cosmo_solve.argtypes = [vp, ctypes.POINTER(CosmoSolveOptions), vp, vp, vp, P32,
                                ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp]
    lib.psd_proj.restype = ctypes.c_int
    lib.psd_proj.argtypes = [i32, P32, P64, ctypes.c_int, vp, vp, vp, vp, i32, dbl, i32, vp, vp]
    lib.psd_proj_static_scratch.restype = ctypes.c_int
    lib.psd_proj_static_scratch.argtypes = [i32, P32, P64, ctypes.c_int, vp, vp, vp, vp, i32, dbl, i32, vp]
    lib.psd_proj_vjp.restype = ctypes.c_int
    lib.psd_proj_vjp.argtypes = [i32, P32, P64, ctypes.c_int, vp, vp, vp, vp, vp, vp]
    lib.psd_proj_vjp_rule.restype = ctypes.c_int
    lib.psd_proj_vjp_rule.argtypes = [i32, P32, P64, ctypes.c_int, i32, dbl, vp, vp, vp, vp, vp, vp]
    lib.psd_ns_tape_size.restype = sz
    lib.psd_ns_tape_size.argtypes = [i32, P32, ctypes.c_int, i32]
    lib.psd_proj_ns.restype = ctypes.c_int
    lib.psd_proj_ns.argtypes = [i32, P32, P64, ctypes.c_int, i32, vp, vp, vp, vp]
    lib.psd_proj_ns_vjp.restype = ctypes.c_int
    lib.psd_proj_ns_vjp.argtypes = [i32, P32, P64, ctypes.c_int, i32, vp, vp, vp, vp]
    lib.socp_proj.restype = ctypes.c_int
    lib.socp_proj.argtypes = [i32, P32, P64, ctypes.c_int, vp, vp, vp, vp]
    lib.socp_proj_vjp.restype = ctypes.c_int
    lib.socp_proj_vjp.argtypes = [i32, P32, P64, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.cosmo_plan_set_profiling.restype = ctypes.c_int
    lib.cosmo_plan_set_profiling.argtypes = [vp, i32]
    lib.cosmo_plan_profile_read.restype = ctypes.c_int
    lib.cosmo_plan_profile_read.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    lib.cosmo_plan_set_pcg_form.restype = ctypes.c_int
    lib.cosmo_plan_set_pcg_form.argtypes = [vp, i32]
    lib.cosmo_plan_get_pcg_form.restype = ctypes.c_int
    lib.cosmo_plan_get_pcg_form.argtypes = [vp, ctypes.POINTER(i32)]
    lib.cosmo_plan_set_graph.restype = ctypes.c_int
    lib.cosmo_plan_set_graph.argtypes = [vp, i32]
    lib.cosmo_plan_get_graph.restype = ctypes.c_int
    lib.cosmo_plan_get_graph.argtypes = [vp, ctypes.POINTER(i32)]
    lib.cosmo_plan_autotune.restype = ctypes.c_int
    lib.cosmo_plan_autotune.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.cosmo_plan_set_psd_schedule.restype = ctypes.c_int
    lib.cosmo_plan_set_psd_schedule.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.cosmo_plan_get_psd_schedule.restype = ctypes.c_int
    lib.cosmo_plan_get_psd_schedule.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.cosmo_plan_psd_tune_ms.restype = ctypes.c_int
    lib.cosmo_plan_psd_tune_ms.argtypes = [vp, ctypes.POINTER(dbl)]
    sp = ctypes.POINTER(CosmoSchedule)
    lib.cosmo_plan_get_schedule.restype = ctypes.c_int
    lib.cosmo_plan_get_schedule.argtypes = [vp, sp]
    lib.cosmo_plan_set_schedule.restype = ctypes.c_int
    lib.cosmo_plan_set_schedule.argtypes = [vp, sp]
    lib.cosmo_plan_signature.restype = ctypes.c_int
    lib.cosmo_plan_signature.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    lib.cosmo_schedule_cache_load.restype = ctypes.c_int
    lib.cosmo_schedule_cache_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p, sp, ctypes.POINTER(i32)]
    lib.cosmo_schedule_cache_store.restype = ctypes.c_int
    lib.cosmo_schedule_cache_store.argtypes = [ctypes.c_char_p, ctypes.c_char_p, sp]
    lib.cosmo_plan_autotune_cached.restype = ctypes.c_int
    lib.cosmo_plan_autotune_cached.argtypes = [vp, vp, vp, vp, vp, ctypes.c_char_p, ctypes.POINTER(i32)]


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2606_13825_amd.build.build() "
                               "(the HIP library is required; there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        _sig(L)
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != COSMO_OK:
        L = lib()
        msg = L.cosmo_last_error().decode(errors="replace")
        raise CosmoError(status, where, msg or L.cosmo_status_string(status).decode())
