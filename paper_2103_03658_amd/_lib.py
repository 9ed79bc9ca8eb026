"""ctypes binding of libfl.so (the C ABI declared in include/fl.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  The library must be built in-tree
(python -m paper_2103_03658_amd.build); there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfl.so")

FL_OK = 0
FL_E_INVAL = 1
FL_E_UNSUPPORTED = 2
FL_E_NOMEM = 3
FL_E_DEVICE = 4
FL_E_NOCONV = 5
FL_E_BREAKDOWN = 6
STATUS_NAMES = {0: "FL_OK", 1: "FL_E_INVAL", 2: "FL_E_UNSUPPORTED", 3: "FL_E_NOMEM",
                4: "FL_E_DEVICE", 5: "FL_E_NOCONV", 6: "FL_E_BREAKDOWN"}

FL_KERNEL_FRACTIONAL = 0
FL_KERNEL_TEMPERED = 1
FL_MAX_KERNEL_TERMS = 16
FL_NOALLOC_SCRATCH_MIB = 128


class FlInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("converged", ctypes.c_int), ("status", ctypes.c_int),
                ("relres_rec", ctypes.c_double), ("relres_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# fl_alloc_fn / fl_release_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# name -> (restype, argtypes); mirrors include/fl.h
_P = ctypes.c_void_p
_SIGS = {
    "fl_weights": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_double, _P, ctypes.POINTER(_P)]),
    "fl_weights_gamma": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, _P, ctypes.POINTER(_P)]),
    "fl_generator": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "fl_symbol": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "fl_embedding": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "fl_query": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_int)] * 4),
    "fl_query_axes": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_int)] * 3),
    "fl_weights_box": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, _P,
                                      ctypes.POINTER(_P)]),
    "fl_weights_expsum": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_double, _P,
                                         ctypes.POINTER(_P)]),
    "fl_set_allocator": (ctypes.c_int, [ALLOC_FN, RELEASE_FN, _P]),
    "fl_solve_async": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P,
                                      ctypes.c_int, _P, ctypes.POINTER(_P)]),
    "fl_poll": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "fl_wait": (ctypes.c_int, [_P, ctypes.POINTER(FlInfo)]),
    "fl_apply": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P]),
    "fl_apply_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P]),
    "fl_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int, _P,
                                ctypes.c_int, ctypes.POINTER(FlInfo), _P]),
    "fl_set_refinement": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    "fl_set_schedule": (ctypes.c_int, [_P, ctypes.c_int] + [ctypes.c_int] * 6),
    "fl_get_schedule": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "fl_set_precond_schedule": (ctypes.c_int, [_P, ctypes.c_int] + [ctypes.c_int] * 6),
    "fl_get_precond_schedule": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "fl_profile_apply": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
    "fl_profile_precond": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]),
    "fl_set_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "fl_set_preconditioner": (ctypes.c_int, [_P, ctypes.c_int]),
    "fl_get_preconditioner": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "fl_apply_precond": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P]),
    "fl_exterior": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P]),
    "fl_destroy": (None, [_P]),
    "fl_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libfl.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run "
                               "`python -m paper_2103_03658_amd.build` first")
        # PyTorch provides the device memory and streams the library works
        # on; load its HIP runtime first so that both share one runtime.
        import torch  # noqa: F401
        handle = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status):
    if status != FL_OK:
        msg = lib().fl_last_error()
        raise FlError(status, msg.decode() if msg else "")
    return status
