"""ctypes view of libpr.so (the C ABI declared in include/pr.h).

Loading fails loudly when the library has not been built: there is no
fallback of any kind.
"""

from __future__ import annotations

import ctypes as C
import os

from .build import LIB

PR_OK, PR_ERR_INVALID_ARG, PR_ERR_UNSUPPORTED, PR_ERR_WORKSPACE, PR_ERR_DEVICE, \
    PR_ERR_NUMERIC, PR_NOT_CONVERGED = range(7)
PR_F64, PR_F32, PR_BF16, PR_BF16X2 = 0, 1, 2, 3
PR_G_SCHEME, PR_G_CNN = 0, 1
PR_ACT_GELU, PR_ACT_TANH = 0, 1
PR_SCHEME_SSI, PR_SCHEME_CN = 0, 1
PR_LAP_FD5, PR_LAP_SPECTRAL = 0, 1

EXPORTED = [
    "pr_fine_workspace_bytes", "pr_fine_propagate", "pr_fine_propagate_noalloc",
    "pr_coarse_workspace_bytes", "pr_coarse_apply",
    "pr_cnn_backward_workspace_bytes", "pr_cnn_backward",
    "pr_scheme_loss_workspace_bytes", "pr_scheme_loss",
    "pr_correct",
    "pr_solve_workspace_bytes", "pr_solve",
    "pr_solve_many_workspace_bytes", "pr_solve_many",
    "pr_serial_workspace_bytes", "pr_serial_fine",
    "pr_set_fine_plan", "pr_get_fine_plan", "pr_autotune_fine", "pr_set_graphs", "pr_get_graphs",
    "pr_set_coarse_plan", "pr_get_coarse_plan", "pr_autotune_coarse",
    "pr_set_coarse_tile", "pr_get_coarse_tile", "pr_set_fft_split", "pr_get_fft_split",
    "pr_set_overlap", "pr_get_overlap", "pr_set_fine_working_set", "pr_get_fine_working_set",
    "pr_set_fine_queue", "pr_get_fine_queue", "pr_get_fine_queue_choice",
    "pr_status_string", "pr_last_error", "pr_abi_version",
]
PR_PLAN_AUTO, PR_PLAN_STREAM, PR_PLAN_RESIDENT = 0, 1, 2
PR_CNN_PLAN_AUTO, PR_CNN_PLAN_LAYERED, PR_CNN_PLAN_FUSED, PR_CNN_PLAN_FOLDED = 0, 1, 2, 3
PR_CNN_TILE_AUTO, PR_CNN_TILE_8X32, PR_CNN_TILE_16X16 = 0, 1, 2
PR_FFT_SPLIT_AUTO, PR_FFT_SPLIT_R8, PR_FFT_SPLIT_R4_TAIL = 0, 1, 2


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("length", C.c_double),
                ("eps", C.c_double), ("conservative", C.c_int32), ("stab", C.c_double),
                ("dt", C.c_double), ("steps", C.c_int32), ("fine_prec", C.c_int32),
                ("f32_iters", C.c_int32), ("scheme", C.c_int32), ("picard_iters", C.c_int32),
                ("laplacian", C.c_int32)]


class Coarse(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dt", C.c_double), ("steps", C.c_int32),
                ("prec", C.c_int32), ("n_layers", C.c_int32), ("channels", C.c_int32),
                ("weights", C.c_void_p), ("biases", C.c_void_p), ("act", C.c_int32),
                ("residual", C.c_int32), ("mass_fix", C.c_int32), ("limiter", C.c_int32),
                ("lim_lo", C.c_double), ("lim_hi", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_converged", C.c_int32),
                ("ic_iterations", C.POINTER(C.c_int32)), ("history", C.POINTER(C.c_double)),
                ("fine_ms", C.c_double), ("sweep_ms", C.c_double)]


class Job(C.Structure):
    _fields_ = [("problem", Problem), ("coarse", Coarse), ("n_ics", C.c_int64),
                ("n_slices", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("u0", C.c_void_p), ("U", C.c_void_p), ("stats", C.POINTER(Stats)),
                ("status", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(
                f"{LIB} is not built; run paper_2510_07672_amd.build.build() "
                "(hipcc --offload-arch=gfx950) first")
        L = C.CDLL(LIB)
        P, G, S = C.POINTER(Problem), C.POINTER(Coarse), C.POINTER(Stats)
        Jp = C.POINTER(Job)
        vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
        sig = {
            "pr_fine_workspace_bytes": (sz, [P, i64]),
            "pr_fine_propagate": (C.c_int, [P, i64, vp, vp, C.c_int, vp, sz, vp]),
            "pr_fine_propagate_noalloc": (C.c_int, [P, i64, vp, vp, C.c_int, vp]),
            "pr_coarse_workspace_bytes": (sz, [P, G, i64]),
            "pr_coarse_apply": (C.c_int, [P, G, i64, vp, vp, vp, sz, vp]),
            "pr_cnn_backward_workspace_bytes": (sz, [P, G, i64]),
            "pr_cnn_backward": (C.c_int, [P, G, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
            "pr_scheme_loss_workspace_bytes": (sz, [P, i64]),
            "pr_scheme_loss": (C.c_int, [P, C.c_double, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
            "pr_correct": (C.c_int, [i64, i32, vp, C.c_int, vp, vp, vp, vp, i32, vp]),
            "pr_solve_workspace_bytes": (sz, [P, G, i64, i32]),
            "pr_solve": (C.c_int, [P, G, i64, i32, vp, vp, C.c_double, i32, S, vp, sz, vp]),
            "pr_solve_many_workspace_bytes": (sz, [i32, Jp]),
            "pr_solve_many": (C.c_int, [i32, Jp, vp, sz, vp]),
            "pr_serial_workspace_bytes": (sz, [P, i64]),
            "pr_serial_fine": (C.c_int, [P, i64, i32, vp, vp, vp, sz, vp]),
            "pr_set_fine_plan": (C.c_int, [i32, C.c_int, i32]),
            "pr_get_fine_plan": (i32, [i32, C.c_int]),
            "pr_autotune_fine": (C.c_int, [P, i64, vp, vp, vp, sz, vp, C.POINTER(i32)]),
            "pr_set_graphs": (None, [i32]),
            "pr_set_coarse_plan": (C.c_int, [i32]),
            "pr_set_overlap": (C.c_int, [i32]),
            "pr_set_fine_working_set": (C.c_int, [i64]),
            "pr_get_fine_working_set": (i64, [i32, C.c_int]),
            "pr_get_overlap": (i32, []),
            "pr_set_fine_queue": (C.c_int, [i32]),
            "pr_get_fine_queue": (i32, []),
            "pr_get_fine_queue_choice": (i32, [i32, i32]),
            "pr_get_coarse_plan": (i32, [G, i32]),
            "pr_set_coarse_tile": (C.c_int, [i32]),
            "pr_set_fft_split": (C.c_int, [i32, C.c_int, i32]),
            "pr_get_fft_split": (i32, [i32, C.c_int]),
            "pr_get_coarse_tile": (i32, [G, i32]),
            "pr_autotune_coarse": (C.c_int, [P, G, i64, vp, vp, vp, sz, vp, C.POINTER(i32)]),
            "pr_get_graphs": (i32, []),
            "pr_status_string": (C.c_char_p, [C.c_int]),
            "pr_last_error": (C.c_char_p, []),
            "pr_abi_version": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PrError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        self.status = status
        msg = L.pr_last_error().decode()
        super().__init__(f"{where}: {L.pr_status_string(status).decode()}: {msg}")


def check(status: int, where: str, allow=(PR_OK,)) -> int:
    if status not in allow:
        raise PrError(status, where)
    return status
