"""ctypes declarations of the C ABI in include/chisao.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchisao.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_RANGE = 0, -1, -2, -3, -4, -5
GAUSS, STUDENT_T = 0, 1
RASTRIGIN, ACKLEY, SCHWEFEL, STYBLINSKI_TANG, MICHALEWICZ, TRID, BUKIN6 = 2, 3, 4, 5, 6, 7, 8
GRAD_FD, GRAD_ADJOINT = 0, 1
FLAG_NO_GRAPH = 1
FLAG_NO_AUTOTUNE = 2
FLAG_RAY_SEEDING = 4
FLAG_HALF_TILES = 8
TUNE_VARIANTS = 4


class Problem(C.Structure):
    _fields_ = [("family", C.c_int32), ("d", C.c_int32), ("K", C.c_int32), ("nu", C.c_float),
                ("log_w", C.c_void_p), ("mu", C.c_void_p), ("prec", C.c_void_p), ("lo", C.c_void_p),
                ("hi", C.c_void_p), ("noise_sigma", C.c_float)]


class Config(C.Structure):
    _fields_ = [("N", C.c_int32), ("m", C.c_int32), ("n_osc", C.c_int32), ("n_conv", C.c_int32),
                ("n_anti", C.c_int32), ("n_cloud", C.c_int32), ("M", C.c_int32), ("eps_grad", C.c_float),
                ("eps_dup", C.c_float), ("log_delta", C.c_float), ("momentum", C.c_float), ("alpha", C.c_float),
                ("sigma", C.c_float), ("sigma_c", C.c_float), ("grad_mode", C.c_int32), ("fd_h", C.c_float),
                ("ls_c1", C.c_float), ("ls_max", C.c_int32), ("curv_eps", C.c_float), ("gate_reps", C.c_int32),
                ("phase_mask", C.c_uint32), ("seed", C.c_uint64), ("problem_id", C.c_uint32),
                ("flags", C.c_uint32)]


class CycleStats(C.Structure):
    _fields_ = [("k", C.c_int32), ("f_max", C.c_float), ("n_stuck", C.c_int32), ("K_lost", C.c_int32),
                ("n_modes", C.c_int32), ("reseed_kind", C.c_int32), ("n_free", C.c_int32),
                ("n_unfrozen", C.c_int32), ("n_active", C.c_int32), ("sigma", C.c_float), ("alpha_c", C.c_float),
                ("alpha_a", C.c_float), ("ls_fail", C.c_int32), ("n_nonfinite", C.c_int32),
                ("evals", C.c_int64)]


class State(C.Structure):
    _fields_ = [("X", C.c_void_p), ("F", C.c_void_p), ("G", C.c_void_p), ("stuck", C.c_void_p),
                ("active", C.c_void_p), ("stuck_pre", C.c_void_p), ("removed", C.c_void_p), ("trace", C.c_void_p),
                ("k", C.c_int32), ("gr_disabled", C.c_int32), ("gr_fail", C.c_int32), ("gr_used_last", C.c_int32),
                ("gr_prev_modes", C.c_int32), ("S", C.c_void_p), ("Y", C.c_void_p), ("rho", C.c_void_p),
                ("head", C.c_void_p), ("cnt", C.c_void_p), ("conv", C.c_void_p), ("Fg", C.c_void_p),
                ("Wd", C.c_void_p), ("wvalid", C.c_void_p)]


class TuningEntry(C.Structure):
    _fields_ = [("padded_d", C.c_int32), ("family", C.c_int32), ("grad_mode", C.c_int32),
                ("n_problems", C.c_int32), ("order", C.c_int32), ("grid_cap", C.c_int32),
                ("ms", C.c_float * 4), ("tile_points", C.c_int32), ("ms_half_tiles", C.c_float), ("ms_full_tiles", C.c_float),
                ("probe_order", C.c_int32), ("probe_grid_cap", C.c_int32), ("ms_probe", C.c_float * 4),
                ("trial_grid_cap", C.c_int32)]


class Peaks(C.Structure):
    _fields_ = [("fp32_mfma_tflops", C.c_double), ("mfma_flops", C.c_double), ("mfma_ms", C.c_double),
                ("hbm_copy_gbs", C.c_double), ("copy_bytes", C.c_double), ("copy_ms", C.c_double)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int32), ("ms", C.c_double), ("points", C.c_int64)]


PROF_CLASSES = 8
PROF_NAMES = ("eval_direct", "eval_trial", "eval_probe", "eval_fd", "lbfgs", "lbfgs_pairs", "unused6", "unused7")

EXPORTS = ("chisao_init", "chisao_init_batched", "chisao_profile", "chisao_cycle", "chisao_modes",
           "chisao_mode_widths", "chisao_get_state", "chisao_set_state", "chisao_run_phases", "chisao_eval",
           "chisao_destroy", "chisao_last_error", "chisao_tuning", "chisao_eval_static",
           "chisao_measure_peaks")

_lib = None


def load(path: str = LIB_PATH):
    """Load libchisao.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2606_26164_amd.build`")
    L = C.CDLL(path)
    P = C.POINTER
    L.chisao_init.argtypes = [P(C.c_void_p), P(Problem), P(Config), C.c_void_p, C.c_void_p]
    L.chisao_init.restype = C.c_int
    L.chisao_init_batched.argtypes = [P(C.c_void_p), C.c_int, P(Problem), P(Config), P(C.c_void_p), C.c_void_p]
    L.chisao_init_batched.restype = C.c_int
    L.chisao_cycle.argtypes = [C.c_void_p, C.c_int, P(CycleStats)]
    L.chisao_cycle.restype = C.c_int
    L.chisao_modes.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, P(C.c_int)]
    L.chisao_modes.restype = C.c_int
    L.chisao_mode_widths.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, P(C.c_int)]
    L.chisao_mode_widths.restype = C.c_int
    L.chisao_get_state.argtypes = [C.c_void_p, C.c_int, P(State)]
    L.chisao_get_state.restype = C.c_int
    L.chisao_set_state.argtypes = [C.c_void_p, C.c_int, P(State)]
    L.chisao_set_state.restype = C.c_int
    L.chisao_run_phases.argtypes = [C.c_void_p, C.c_uint32]
    L.chisao_run_phases.restype = C.c_int
    L.chisao_eval.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
    L.chisao_eval.restype = C.c_int
    L.chisao_eval_static.argtypes = [P(Problem), C.c_float, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                     C.c_void_p]
    L.chisao_eval_static.restype = C.c_int
    L.chisao_measure_peaks.argtypes = [P(Peaks), C.c_size_t, C.c_void_p]
    L.chisao_measure_peaks.restype = C.c_int
    L.chisao_profile.argtypes = [C.c_void_p, C.c_int, P(KernelProfile)]
    L.chisao_profile.restype = C.c_int
    L.chisao_destroy.argtypes = [C.c_void_p]
    L.chisao_destroy.restype = None
    L.chisao_tuning.argtypes = [C.c_void_p, P(TuningEntry), C.c_int, P(C.c_int)]
    L.chisao_tuning.restype = C.c_int
    L.chisao_last_error.argtypes = []
    L.chisao_last_error.restype = C.c_char_p
    _lib = L
    return L


class ChisaoError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().chisao_last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def check(code: int, where: str):
    if code != OK:
        raise ChisaoError(code, where)
