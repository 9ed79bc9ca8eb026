"""The C ABI library loads, exports every symbol the header declares, and
rejects invalid arguments before touching a device (CPU only)."""

import ctypes

import numpy as np
import os
import re

import pytest

import paper_2103_03658_amd as fl
from paper_2103_03658_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fl_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_header_symbols():
    lib = _lib.lib()
    names = declared_symbols()
    assert {"fl_weights", "fl_apply", "fl_solve", "fl_destroy"} <= names
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's functions
    assert set(_lib._SIGS) == names


@pytest.mark.parametrize("args,code", [
    ((0, 1.0, 1, 0.25), _lib.FL_E_INVAL),        # d
    ((4, 1.0, 1, 0.25), _lib.FL_E_INVAL),
    ((2, 0.0, 1, 0.25), _lib.FL_E_INVAL),        # alpha
    ((2, 2.0, 1, 0.25), _lib.FL_E_INVAL),
    ((2, float("nan"), 1, 0.25), _lib.FL_E_INVAL),
    ((2, 1.0, 3, 0.25), _lib.FL_E_INVAL),        # degree
    ((2, 1.0, 1, 0.3), _lib.FL_E_INVAL),         # 2/h not an integer
    ((2, 1.0, 1, -0.25), _lib.FL_E_INVAL),
    ((2, 1.0, 1, 1.0), _lib.FL_E_INVAL),         # N = 2 < 4
    ((2, 1.0, 2, 2.0 / 9), _lib.FL_E_INVAL),     # p = 2, N odd
    ((2, 1.0, 1, 2.0 / 1025), _lib.FL_E_UNSUPPORTED),  # M = 4096
    ((1, 1.0, 1, 2.0 / 2048), _lib.FL_E_UNSUPPORTED),  # M = 4096
])
def test_fl_weights_validation(args, code):
    lib = _lib.lib()
    h = ctypes.c_void_p()
    st = lib.fl_weights(*args, 0, 0.0, None, ctypes.byref(h))
    assert st == code
    assert lib.fl_last_error()
    assert h.value is None


def test_tempered_lambda_validation():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.fl_weights(2, 1.0, 1, 0.25, 1, -1.0, None, ctypes.byref(h)) == _lib.FL_E_INVAL
    assert lib.fl_weights(2, 1.0, 1, 0.25, 7, 0.0, None, ctypes.byref(h)) == _lib.FL_E_INVAL


def test_null_handle_errors():
    lib = _lib.lib()
    assert lib.fl_apply(None, None, None, 1, 0, None) == _lib.FL_E_INVAL
    assert lib.fl_solve(None, None, None, 1e-10, 10, 0, None, 1, None, None) == _lib.FL_E_INVAL
    assert lib.fl_set_refinement(None, 0.1, 1e-3, 3) == _lib.FL_E_INVAL
    kind = ctypes.c_int(-1)
    assert lib.fl_get_preconditioner(None, ctypes.byref(kind)) == _lib.FL_E_INVAL
    assert kind.value == -1
    assert lib.fl_set_preconditioner(None, 2) == _lib.FL_E_INVAL
    lib.fl_destroy(None)  # accepted


def test_error_raises_in_binding():
    with pytest.raises(fl.FlError) as ei:
        fl.Operator(2, 1.0, 2, N=9)
    assert ei.value.status == _lib.FL_E_INVAL


def test_request_stream_is_seeded_and_shaped():
    from paper_2103_03658_amd import inputs
    a = inputs.request_stream(256, seed=0)
    b = inputs.request_stream(256, seed=0)
    assert a == b
    ns = [r["N"] - 1 for r in a]
    assert set(ns) <= {63, 127, 255, 511}
    assert all(0.2 - 1e-12 <= r["alpha"] <= 1.9 + 1e-12 and r["degree"] in (0, 1, 2) and 1 <= r["nrhs"] <= 8
               for r in a)
    t = [r["t_arrive"] for r in a]
    assert all(x < y for x, y in zip(t, t[1:]))
    rate = len(t) / t[-1]
    assert 150 < rate < 260                         # Poisson arrivals at 200 / s
    f = inputs.request_rhs(a[0])
    assert f.shape == (a[0]["nrhs"], ns[0], ns[0]) and np.abs(f).max() <= 1


def test_manufactured_rhs_matches_closed_form():
    """The 2D benchmark right-hand side inside the unit disk is the closed
    form of (-Delta)^{alpha/2} (1-|x|^2)_+^{1+alpha/2}."""
    import oracle.exact as ex
    from paper_2103_03658_amd import inputs
    for alpha in (0.5, 1.0, 1.5):
        f = inputs.manufactured_rhs_disk(32, alpha)
        X0, X1 = inputs.interior_coords(2, 32)
        r2 = X0 ** 2 + X1 ** 2
        inside = r2 < 1
        ref = ex.frac_lap_ball_power(r2[inside], 1 + alpha / 2, alpha, 2)
        np.testing.assert_allclose(f[inside], ref, rtol=1e-13)
        assert (f[~inside] == 0).all()


def test_exterior_null_and_unsupported():
    lib = _lib.lib()
    assert lib.fl_exterior(None, None, None, None, 1, None) == _lib.FL_E_INVAL


@pytest.mark.parametrize("gamma", [0.5, 1.0, 2.5, float("nan")])
def test_fl_weights_gamma_validation(gamma):
    lib = _lib.lib()
    h = ctypes.c_void_p()
    st = lib.fl_weights_gamma(2, 1.0, 1, 0.25, 0, 0.0, gamma, None, ctypes.byref(h))
    assert st == _lib.FL_E_INVAL
    assert h.value is None


def test_fl_weights_expsum_validation():
    """Bad kernel terms are rejected before any device work."""
    lib = _lib.lib()
    h = ctypes.c_void_p()
    iv = (ctypes.c_int * 3)(8, 8, 8)

    def call(coef, rate, nterm=None, intervals=iv):
        n = len(coef) if nterm is None else nterm
        c = (ctypes.c_double * max(len(coef), 1))(*coef)
        r = (ctypes.c_double * max(len(rate), 1))(*rate)
        return lib.fl_weights_expsum(2, 1.0, 1, intervals, n, c, r, 2.0, None, ctypes.byref(h))

    assert call([1.0, -0.1], [0.0, 1.0]) == _lib.FL_E_INVAL          # negative coefficient
    assert call([1.0], [-1.0]) == _lib.FL_E_INVAL                     # negative rate
    assert call([0.0, 0.0], [1.0, 2.0]) == _lib.FL_E_INVAL            # K = 0
    assert call([1.0], [float("inf")]) == _lib.FL_E_INVAL
    assert call([float("nan")], [1.0]) == _lib.FL_E_INVAL
    assert call([1.0] * 17, [0.0] * 17) == _lib.FL_E_INVAL            # too many terms
    assert call([1.0], [0.0], nterm=0) == _lib.FL_E_INVAL
    assert call([1.0], [0.0], intervals=None) == _lib.FL_E_INVAL
    assert _lib.FL_MAX_KERNEL_TERMS == 16


def test_allocator_and_async_argument_checks():
    """fl_set_allocator needs both callbacks or neither; the request calls
    reject null handles; fl_solve_async validates like fl_solve (no device
    work happens in any of these)."""
    lib = _lib.lib()
    alloc = _lib.ALLOC_FN(lambda n, ctx: None)
    assert lib.fl_set_allocator(alloc, _lib.RELEASE_FN(), None) == _lib.FL_E_INVAL
    assert lib.fl_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == _lib.FL_OK
    flag = ctypes.c_int(7)
    assert lib.fl_poll(None, ctypes.byref(flag)) == _lib.FL_E_INVAL
    assert lib.fl_wait(None, None) == _lib.FL_E_INVAL
    req = ctypes.c_void_p()
    assert lib.fl_solve_async(None, None, None, 1e-10, 10, 0, None, 1, None,
                              ctypes.byref(req)) == _lib.FL_E_INVAL
    assert req.value is None
