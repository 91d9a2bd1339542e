"""ctypes binding of the C-ABI declared in include/lbm_pp.h (argument
marshalling only: every step of the method runs in the HIP library)."""
import ctypes
import os

from .build import LIB_PATH

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                   ctypes.c_size_t, ctypes.c_void_p)

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_HIP, LBM_E_STATE, LBM_E_DOMAIN, LBM_E_UNSUPPORTED = range(7)
LBM_FP64, LBM_FP32_SHIFTED = 0, 1
T_FREE, T_DIRICHLET, T_ADIABATIC = 0, 1, 2
LBM_WALL_PSI_BASED, LBM_WALL_MODIFIED_PSI = 0, 1  # contact-angle models (lbm_params.wall_model)


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("precision", c_int32), ("walls", c_int32),
        ("thermal", c_int32), ("n_iso", c_int32), ("t_side_dirichlet", c_int32),
        ("tile_y", c_int32),
        ("a", c_double), ("b", c_double), ("R", c_double), ("omega", c_double), ("G", c_double),
        ("sigma", c_double), ("kappa", c_double),
        ("s_rho", c_double), ("s_e", c_double), ("s_zeta", c_double), ("s_j", c_double),
        ("s_q", c_double),
        ("eta_l", c_double), ("eta_v", c_double), ("rho_l", c_double), ("rho_v", c_double),
        ("gy", c_double), ("cv", c_double), ("lambda_l", c_double), ("lambda_v", c_double),
        ("t_side_val", c_double), ("rho_ref", c_double),
        ("xcd_remap", c_int32), ("strip_waves", c_int32), ("wall_model", c_int32), ("outflow_top", c_int32), ("reserved_i", c_int32 * 4), ("reserved_d", c_double * 8),
    ]


class LbmNorms(ctypes.Structure):
    _fields_ = [
        ("mass", c_double), ("rho_mean", c_double), ("umax", c_double), ("q_bottom", c_double),
        ("q_heater", c_double),
        ("l1_rho", c_double), ("l2_rho", c_double), ("linf_rho", c_double),
        ("l1_T", c_double), ("l2_T", c_double), ("linf_T", c_double),
        ("nonfinite", c_int64), ("n_heater", c_int64), ("step", c_int64),
    ]


class LbmLevel(ctypes.Structure):
    _fields_ = [(k, c_double) for k in ("dx", "a", "Tc", "T", "rho_v", "rho_l", "p_sat", "sigma",
                                        "kappa", "gamma", "gy")] + [("steps", c_int64)]


# (name, restype, argtypes) of every exported symbol of include/lbm_pp.h
P = ctypes.POINTER
_DP = P(c_double)
SIGNATURES = [
    ("lbm_status_string", ctypes.c_char_p, [c_int32]),
    ("lbm_last_error", ctypes.c_char_p, [c_void_p]),
    ("lbm_default_params", None, [P(LbmParams), c_int32, c_int32]),
    ("lbm_validate", c_int32, [P(LbmParams)]),
    ("lbm_buffer_bytes", c_int32, [P(LbmParams), P(c_size_t)]),
    ("lbm_create", c_int32, [P(LbmParams), c_void_p, c_size_t, c_void_p, P(c_void_p)]),
    ("lbm_destroy", None, [c_void_p]),
    ("lbm_set_boundary", c_int32, [c_void_p, _DP, _DP, P(c_int32), _DP, P(c_int32), _DP]),
    ("lbm_init_fields", c_int32, [c_void_p, _DP, _DP, _DP, _DP]),
    ("lbm_step", c_int32, [c_void_p, c_int64]),
    ("lbm_read_fields", c_int32, [c_void_p, _DP, _DP, _DP, _DP]),
    ("lbm_read_populations", c_int32, [c_void_p, _DP]),
    ("lbm_norms", c_int32, [c_void_p, P(LbmNorms)]),
    ("lbm_norms_device", c_int32, [c_void_p, c_void_p]),
    ("lbm_state_bytes", c_int32, [c_void_p, P(c_size_t)]),
    ("lbm_save_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("lbm_load_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("lbm_sync", c_int32, [c_void_p]),
    ("lbm_step_count", c_int64, [c_void_p]),
    ("lbm_last_step_time", c_int32, [c_void_p, _DP]),
    ("lbm_kernel_timing", c_int32, [c_void_p, c_int32]),
    ("lbm_set_tile_y", c_int32, [c_void_p, c_int32]),
    ("lbm_get_tile_y", c_int32, [c_void_p]),
    ("lbm_set_strip_waves", c_int32, [c_void_p, c_int32]),
    ("lbm_get_strip_waves", c_int32, [c_void_p]),
    ("lbm_batch_bytes", c_int32, [c_int32, P(c_size_t)]),
    ("lbm_batch_create", c_int32, [P(c_void_p), c_int32, c_void_p, c_size_t, c_void_p, P(c_void_p)]),
    ("lbm_batch_destroy", None, [c_void_p]),
    ("lbm_batch_last_error", ctypes.c_char_p, [c_void_p]),
    ("lbm_batch_run", c_int32, [c_void_p, P(c_int64), c_int32]),
    ("lbm_batch_prepare", c_int32, [c_void_p, P(c_int64), c_int32]),
    ("lbm_batch_last_time", c_int32, [c_void_p, _DP, P(c_int64), P(c_int64)]),
    ("lbm_autotune_tile_y", c_int32, [c_void_p, P(c_int32), c_int32, c_int32, P(c_int32), _DP]),
    ("lbm_tile_candidates", c_int32, [c_void_p, c_int32, P(c_int32), c_int32, P(c_int32)]),
    ("lbm_refinement_level", c_int32, [c_double] * 9 + [c_int64, P(LbmLevel)]),
    ("lbm_adjoint_bytes", c_int32, [P(LbmParams), c_int32, c_int32, P(c_size_t)]),
    ("lbm_adjoint_create", c_int32, [c_void_p, c_int32, c_int32, c_double, c_double, c_void_p, c_size_t,
                                     P(c_void_p)]),
    ("lbm_adjoint_destroy", None, [c_void_p]),
    ("lbm_adjoint_forward", c_int32, [c_void_p, _DP]),
    ("lbm_adjoint_backward", c_int32, [c_void_p, c_double, _DP]),
    ("lbm_adjoint_timing", c_int32, [c_void_p, _DP, _DP]),
    ("lbm_kernel_times", c_int32, [c_void_p, _DP, P(c_int64)]),
    ("lbm_pr_critical_temperature", c_double, [c_double, c_double, c_double]),
    ("lbm_pr_maxwell", c_int32, [c_double, c_double, c_double, c_double, c_double, _DP, _DP, _DP]),
    ("lbm_fit_sigma", c_int32, [c_double, c_double, c_double, c_double, c_double, c_double, _DP]),
    ("lbm_planar_gamma", c_int32, [c_double, c_double, c_double, c_double, c_double, c_double,
                                   c_double, _DP]),
    ("lbm_pr_latent_heat", c_int32, [c_double] * 7 + [_DP]),
    ("lbm_stefan_beta", c_int32, [c_double, _DP]),
]

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is missing: build it with "
                              "`python -m paper_2201_04560_amd.build` (or __graft_entry__.build())")
        # PyTorch bundles its own HIP runtime (soname libamdhip64.so.7); load
        # it first so that the library binds to the same runtime instance
        # instead of pulling a second copy from the ROCm install
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        l = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status, ctx=None, what=""):
    if status != LBM_OK:
        l = lib()
        detail = l.lbm_last_error(ctx)
        detail = detail.decode() if detail else ""
        raise LbmError(status, f"{what}: {l.lbm_status_string(status).decode()}: {detail}")
