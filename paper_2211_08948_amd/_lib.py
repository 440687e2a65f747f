"""ctypes view of include/leja.h: struct mirrors and function prototypes.

Loading fails loudly (LejaLibraryError) when libleja.so has not been built;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleja.so")

LJ_OK, LJ_ENOTCONV, LJ_EINVAL, LJ_EHIP, LJ_ENOMEM = 0, 1, -1, -2, -3
LJ_MAX_K = 4
LJ_MAX_L = 4
LJ_MAX_POINTS = 100
LJ_NOALLOC_SCRATCH_BYTES = 32 << 20
LJ_NFEATURES = 16
LJ_MLP_NPARAM = 5378
LJ_MLP_MODEL_FLOATS = 5414
LJ_PROPOSAL_MARGIN = 1.02

(LJ_OP_DIAG, LJ_OP_ADVDIFF2D, LJ_OP_ALLENCAHN2D, LJ_OP_BRUSSELATOR2D, LJ_OP_BURGERS2D, LJ_OP_GRAYSCOTT2D,
 LJ_OP_ADR2D) = range(7)
LJ_EXPRB2, LJ_EXPRB43_U3, LJ_EXPRB43, LJ_EPIRK4S3, LJ_EPIRK4S3_LEKRY, LJ_EPIRK4S3A, LJ_EPIRK4S3A_LEKRY = 1, 2, 3, 4, 5, 6, 7


class LejaLibraryError(RuntimeError):
    pass


class lj_operator(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("ncomp", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("coef", C.c_double * 8), ("state", C.c_void_p),
    ]


# user-operator callbacks (lj_rhs_fn, lj_jv_fn)
lj_rhs_fn = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p)
lj_jv_fn = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p)


class lj_user_operator(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("rhs", lj_rhs_fn), ("jv", lj_jv_fn), ("user", C.c_void_p), ("state", C.c_void_p),
    ]


class lj_krylov_options(C.Structure):
    _fields_ = [("krylov_dim", C.c_int32), ("window", C.c_int32), ("max_substeps", C.c_int32),
                ("reserved", C.c_int32)]


class lj_options(C.Structure):
    _fields_ = [
        ("safety", C.c_double), ("power_iters", C.c_int32), ("max_points", C.c_int32),
        ("hump_max", C.c_double), ("max_substeps", C.c_int32), ("relative_tol", C.c_int32),
        ("bound", C.c_double), ("substeps", C.c_int32), ("power_seed", C.c_uint64),
        ("pi_start", C.c_void_p), ("use_proposal", C.c_int32), ("reserved", C.c_int32),
        ("bound_device", C.c_void_p),
    ]


class lj_stats(C.Structure):
    _fields_ = [
        ("m_star", C.c_int32 * LJ_MAX_K), ("substeps", C.c_int32 * LJ_MAX_K),
        ("err_est", C.c_double * LJ_MAX_K), ("iters_total", C.c_int32), ("power_iters", C.c_int32),
        ("rejections", C.c_int32), ("converged", C.c_int32), ("bound", C.c_double),
        ("c", C.c_double), ("gamma", C.c_double), ("fallbacks", C.c_int32),
        ("proposal_substeps", C.c_int32), ("proposal_bound", C.c_double),
    ]

    def as_dict(self, K: int = LJ_MAX_K) -> dict:
        return {
            "m_star": list(self.m_star)[:K], "substeps": list(self.substeps)[:K],
            "err_est": list(self.err_est)[:K], "iters_total": self.iters_total,
            "power_iters": self.power_iters, "rejections": self.rejections,
            "converged": bool(self.converged), "bound": self.bound, "c": self.c, "gamma": self.gamma,
            "fallbacks": self.fallbacks, "proposal_substeps": self.proposal_substeps,
            "proposal_bound": self.proposal_bound,
        }


class lj_timing(C.Structure):
    _fields_ = [
        ("launches", C.c_int64), ("iterations", C.c_int64), ("point_iters", C.c_int64),
        ("accum_point_iters", C.c_int64), ("power_point_iters", C.c_int64), ("tiled_launches", C.c_int64),
        ("kernel_ms", C.c_double), ("aborts", C.c_int64),
    ]


class lj_integrate_stats(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("rejected", C.c_int32), ("products", C.c_int64), ("t", C.c_double),
                ("dt_next", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class lj_step_record(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("err", C.c_double), ("products", C.c_int32),
                ("accepted", C.c_int32)]

    def as_dict(self) -> dict:
        return {"t": self.t, "dt": self.dt, "err": self.err, "products": self.products,
                "accepted": bool(self.accepted)}


class lj_batch_info_t(C.Structure):
    _fields_ = [
        ("schedule", C.c_int32), ("block_size", C.c_int32), ("blocks", C.c_int32),
        ("largest_first", C.c_int32), ("nschedules", C.c_int32), ("team", C.c_int32),
        ("tune_ms", C.c_float * 8), ("total_values", C.c_int64), ("alg_bytes", C.c_double),
    ]


_P = C.c_void_p
_PROTOS = {
    "lj_create": (C.c_int, [C.POINTER(_P), C.c_int]),
    "lj_destroy": (None, [_P]),
    "lj_last_error": (C.c_char_p, [_P]),
    "lj_default_options": (None, [C.POINTER(lj_options)]),
    "lj_version": (C.c_char_p, []),
    "lj_leja_points": (C.c_int, [C.POINTER(C.c_double), C.c_int]),
    "lj_spectral_bound": (C.c_int, [_P, C.POINTER(lj_operator), C.c_int, C.c_uint64, _P,
                                    C.POINTER(C.c_double), _P]),
    "lj_divided_differences": (C.c_int, [_P, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int,
                                         C.POINTER(C.c_double), _P]),
    "lj_rhs": (C.c_int, [_P, C.POINTER(lj_operator), _P, _P, _P]),
    "lj_jv": (C.c_int, [_P, C.POINTER(lj_operator), _P, _P, _P]),
    "lj_measure_bandwidth": (C.c_int, [C.c_longlong, C.POINTER(C.c_double)]),
    "lj_measure_bandwidth_shape": (C.c_int, [C.c_longlong, C.c_int, C.c_int, C.c_int, C.c_int,
                                             C.POINTER(C.c_double)]),
    "lj_default_krylov_options": (None, [C.POINTER(lj_krylov_options)]),
    "lj_phi_combination": (C.c_int, [_P, C.POINTER(lj_operator), C.c_int, C.POINTER(_P), C.c_double, C.c_double,
                                     _P, C.POINTER(lj_krylov_options), C.POINTER(lj_stats), _P]),
    "lj_user_phi_combination": (C.c_int, [_P, C.POINTER(lj_user_operator), C.c_int, C.POINTER(_P), C.c_double,
                                          C.c_double, _P, C.POINTER(lj_krylov_options), C.POINTER(lj_stats), _P]),
    "lj_user_phi_action": (C.c_int, [_P, C.POINTER(lj_user_operator), _P, _P, C.c_int, C.c_double, C.c_double,
                                     C.POINTER(lj_options), C.POINTER(lj_stats), _P]),
    "lj_user_phi_vertical": (C.c_int, [_P, C.POINTER(lj_user_operator), _P, C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(C.c_double), C.c_double, C.c_double, C.POINTER(_P),
                                       C.POINTER(lj_options), C.POINTER(lj_stats), _P]),
    "lj_user_step": (C.c_int, [_P, C.c_int, C.POINTER(lj_user_operator), C.c_double, C.c_double, _P, _P,
                               C.POINTER(lj_options), C.POINTER(lj_stats), C.c_int, C.POINTER(C.c_int), _P]),
    "lj_phi_action": (C.c_int, [_P, C.POINTER(lj_operator), _P, _P, C.c_int, C.c_double, C.c_double,
                                C.POINTER(lj_options), C.POINTER(lj_stats), _P]),
    "lj_defer_begin": (C.c_int, [_P]),
    "lj_defer_end": (C.c_int, [_P, _P]),
    "lj_bound_device": (C.c_void_p, [_P]),
    "lj_phi_action_noalloc": (C.c_int, [_P, C.POINTER(lj_operator), _P, _P, C.c_int, C.c_double, C.c_double,
                                        C.POINTER(lj_options), C.POINTER(lj_stats), _P]),
    "lj_phi_vertical": (C.c_int, [_P, C.POINTER(lj_operator), _P, C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(C.c_double), C.c_double, C.c_double, C.POINTER(_P),
                                  C.POINTER(lj_options), C.POINTER(lj_stats), _P]),
    "lj_step": (C.c_int, [_P, C.c_int, C.POINTER(lj_operator), C.c_double, C.c_double, _P, _P,
                          C.POINTER(lj_options), C.POINTER(lj_stats), C.c_int, C.POINTER(C.c_int), _P]),
    "lj_integrate": (C.c_int, [_P, C.c_int, C.POINTER(lj_operator), C.c_double, C.c_double, C.c_double,
                               C.c_double, _P, C.POINTER(lj_options), C.POINTER(lj_integrate_stats),
                               C.POINTER(lj_step_record), C.c_int, C.c_int, _P]),
    "lj_user_integrate": (C.c_int, [_P, C.c_int, C.POINTER(lj_user_operator), C.c_double, C.c_double, C.c_double,
                                    C.c_double, _P, C.POINTER(lj_options), C.POINTER(lj_integrate_stats),
                                    C.POINTER(lj_step_record), C.c_int, C.c_int, _P]),
    "lj_last_trace": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int]),
    "lj_last_profile": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "lj_timing_enable": (C.c_int, [_P, C.c_int]),
    "lj_timing_read": (C.c_int, [_P, C.POINTER(lj_timing), C.c_int]),
    "lj_batch_create": (C.c_int, [_P, C.POINTER(lj_operator), C.c_int, C.POINTER(_P), C.POINTER(C.c_double),
                                  C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_double,
                                  C.POINTER(_P), C.POINTER(C.c_double), C.POINTER(lj_options), C.POINTER(_P)]),
    "lj_batch_run": (C.c_int, [_P, _P]),
    "lj_batch_stats": (C.c_int, [_P, C.POINTER(lj_stats), _P]),
    "lj_batch_info": (C.c_int, [_P, C.POINTER(lj_batch_info_t)]),
    "lj_batch_timeline": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lj_batch_destroy": (None, [_P]),
    "lj_features": (C.c_int, [_P, C.POINTER(lj_operator), C.c_double, C.c_int, _P, _P]),
    "lj_gershgorin_bound": (C.c_int, [_P, C.POINTER(lj_operator), C.POINTER(C.c_double), _P]),
    "lj_proposal_record": (C.c_int, [_P, C.POINTER(lj_operator), C.c_double, C.c_int, C.c_double, C.c_int, _P, _P,
                                     _P]),
    "lj_mlp_init": (C.c_int, [_P, C.c_uint64]),
    "lj_mlp_train": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_float, C.c_int, C.POINTER(C.c_float), _P]),
    "lj_mlp_predict": (C.c_int, [_P, _P, C.c_int, _P, _P]),
    "lj_mlp_grad": (C.c_int, [_P, _P, _P, C.c_int, _P, C.POINTER(C.c_float), _P]),
    "lj_mlp_get": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "lj_mlp_set": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "lj_mlp_save": (C.c_int, [_P, C.c_char_p]),
    "lj_mlp_load": (C.c_int, [_P, C.c_char_p]),
}

_lib = None


def load() -> C.CDLL:
    """The loaded library (built by paper_2211_08948_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LejaLibraryError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2211_08948_amd.build` "
                "(the library has no non-HIP fallback)")
        # PyTorch brings its own HIP runtime (soname libamdhip64.so.7).  Loading
        # torch first makes this library bind to that same runtime instance;
        # loaded the other way round the process would hold two HIP runtimes
        # and torch's streams and allocations would be foreign to ours.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
