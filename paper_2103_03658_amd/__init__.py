"""Fractional Laplacian on MI355X: operator-factorization discretization
(Wu & Zhang, arXiv 2103.03658) applied by circulant-embedded FFT and solved
by conjugate gradients in hand-written HIP kernels for gfx950.

Thin Python layer over the C ABI (include/fl.h): it converts arguments and
hands device pointers of torch tensors to the library.  torch provides device
memory and streams only.
"""

import ctypes

from ._lib import (ALLOC_FN, FL_KERNEL_FRACTIONAL, FL_KERNEL_TEMPERED, RELEASE_FN, FlError, FlInfo,
                   check, lib)

# Callbacks handed to fl_set_allocator.  Blocks keep the allocator that made
# them until the library releases them, so no registered pair is ever freed.
_allocator_refs = []


def set_allocator(alloc, release):
    """Route the library's device allocations through alloc(nbytes) -> int
    device pointer (0 on failure) and release(ptr) (fl_set_allocator);
    set_allocator(None, None) restores hipMalloc / hipFree."""
    if alloc is None and release is None:
        check(lib().fl_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        return
    a = ALLOC_FN(lambda nbytes, ctx: alloc(nbytes) or None)
    r = RELEASE_FN(lambda ptr, ctx: release(ptr))
    _allocator_refs.append((a, r))
    check(lib().fl_set_allocator(a, r, None))


def use_torch_allocator():
    """Take operator memory from torch's caching allocator (current device)."""
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  torch.cuda.caching_allocator_delete)

__all__ = ["Operator", "FlError", "FlInfo", "lib"]


def _stream_ptr(stream):
    """hipStream_t of `stream`, or torch's current stream, or NULL (the
    default stream) when no device is visible (argument checks still run)."""
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(None)
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class SolveRequest:
    """A submitted solve (Operator.solve_async): done() polls, wait() blocks
    and returns (u, per-RHS info dicts) like Operator.solve."""

    def __init__(self, op, handle, nrhs, tensors):
        self._op, self._h, self._nrhs, self._tensors = op, handle, nrhs, tensors

    def done(self):
        flag = ctypes.c_int()
        check(self._op._lib.fl_poll(self._h, ctypes.byref(flag)))
        return bool(flag.value)

    def wait(self, raise_on_fail=True):
        if self._h is None:
            raise RuntimeError("request already waited for")
        info = (FlInfo * self._nrhs)()
        st = self._op._lib.fl_wait(self._h, info)
        self._h = None
        infos = [i.as_dict() for i in info]
        if raise_on_fail:
            check(st)
        return self._tensors[2], infos


class Operator:
    """The discrete operator A (g = 0 part of (-Delta)^{alpha/2}_h) on (-1,1)^d,
    or with box=(N_0, .., N_{d-1}) on the box whose longest axis spans (-1, 1)
    with N = max N_s intervals and axis s has N_s.

    Built on the current CUDA/HIP device by fl_weights_gamma / fl_weights_box
    (splitting parameter gamma in (alpha, 2], default 2).  kernel="expsum"
    with terms=[(coef, rate), ...] takes K(r) = sum coef exp(-rate r)
    (fl_weights_expsum; the cube, or the box given).  Vectors are torch
    tensors on that device holding nrhs * prod(n_s) values (any shape with
    that many elements, contiguous; row-major over `shape`)."""

    def __init__(self, d, alpha, degree, N=None, h=None, kernel="fractional", lam=0.0,
                 stream=None, gamma=2.0, box=None, terms=None):
        self._h = ctypes.c_void_p()
        self._lib = lib()
        if kernel == "expsum":
            # K(r) = sum coef exp(-rate r) over terms = [(coef, rate), ...]
            if not terms:
                raise ValueError("kernel 'expsum' needs terms=[(coef, rate), ...]")
            if box is None:
                if N is None:
                    if h is None:
                        raise ValueError("give N, h or box")
                    N = int(round(2.0 / h))
                box = (N,) * d
            if len(box) != d:
                raise ValueError("box needs d interval counts")
            arr = (ctypes.c_int * 3)(*[int(b) for b in box])
            coef = (ctypes.c_double * len(terms))(*[float(t[0]) for t in terms])
            rate = (ctypes.c_double * len(terms))(*[float(t[1]) for t in terms])
            check(self._lib.fl_weights_expsum(int(d), float(alpha), int(degree), arr, len(terms),
                                              coef, rate, float(gamma), _stream_ptr(stream),
                                              ctypes.byref(self._h)))
        elif box is not None:
            kind = {"fractional": FL_KERNEL_FRACTIONAL, "tempered": FL_KERNEL_TEMPERED}[kernel]
            if len(box) != d:
                raise ValueError("box needs d interval counts")
            arr = (ctypes.c_int * 3)(*[int(b) for b in box])
            check(self._lib.fl_weights_box(int(d), float(alpha), int(degree), arr, kind,
                                           float(lam), float(gamma), _stream_ptr(stream),
                                           ctypes.byref(self._h)))
        else:
            kind = {"fractional": FL_KERNEL_FRACTIONAL, "tempered": FL_KERNEL_TEMPERED}[kernel]
            if h is None:
                if N is None:
                    raise ValueError("give N or h")
                h = 2.0 / N
            check(self._lib.fl_weights_gamma(int(d), float(alpha), int(degree), float(h), kind,
                                             float(lam), float(gamma), _stream_ptr(stream),
                                             ctypes.byref(self._h)))
        q = [ctypes.c_int() for _ in range(4)]
        check(self._lib.fl_query(self._h, *[ctypes.byref(x) for x in q]))
        self.d, self.N = q[0].value, q[1].value
        ax = [(ctypes.c_int * 3)() for _ in range(3)]
        check(self._lib.fl_query_axes(self._h, *ax))
        self.intervals = tuple(ax[0][s] for s in range(self.d))
        self.shape = tuple(ax[1][s] for s in range(self.d))      # interior points per axis
        self.Ms = tuple(ax[2][s] for s in range(self.d))         # embedding length per axis
        self.M = max(self.Ms)
        self.n = self.shape[0] if len(set(self.shape)) == 1 else None
        self.alpha, self.degree, self.kernel, self.lam = float(alpha), int(degree), kernel, lam
        self.terms = [tuple(map(float, t)) for t in terms] if kernel == "expsum" else None
        self.gamma = float(gamma)
        self.nd = 1
        for v in self.shape:
            self.nd *= v
        kind = ctypes.c_int(0)
        check(self._lib.fl_get_preconditioner(self._h, ctypes.byref(kind)))
        self.precond_kind = kind.value   # the library's default (tau where available)

    # -- host copies (test hooks) ------------------------------------------
    def _host(self, fn, count):
        import numpy as np
        out = np.empty(count, dtype=np.float64)
        check(fn(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), count))
        return out

    def generator(self):
        return self._host(self._lib.fl_generator, (self.N + 1) ** self.d).reshape(
            (self.N + 1,) * self.d)

    def symbol(self):
        """Folded symbol lambda-hat on prod [0, M_s/2] (N + 1 per axis when M = 2N)."""
        shp = tuple(m // 2 + 1 for m in self.Ms)
        cnt = 1
        for v in shp:
            cnt *= v
        return self._host(self._lib.fl_symbol, cnt).reshape(shp)

    def embedding(self):
        cnt = 1
        for v in self.Ms:
            cnt *= v
        return self._host(self._lib.fl_embedding, cnt).reshape(self.Ms)

    # -- compute ----------------------------------------------------------------
    def _nrhs(self, t):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if t.numel() % self.nd:
            raise ValueError(f"size {t.numel()} is not a multiple of n^d = {self.nd}")
        return t.numel() // self.nd

    def apply(self, u, out=None, stream=None):
        """y = A u; FP32 transforms when u is float32, FP64 when float64."""
        import torch
        if u.dtype not in (torch.float32, torch.float64):
            raise TypeError("u must be float32 or float64")
        nrhs = self._nrhs(u)
        if out is None:
            out = torch.empty_like(u)
        if out.dtype != u.dtype or out.numel() != u.numel() or not out.is_contiguous():
            raise ValueError("out must match u")
        check(self._lib.fl_apply(self._h, ctypes.c_void_p(u.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), nrhs,
                                 1 if u.dtype == torch.float32 else 0, _stream_ptr(stream)))
        return out

    def apply_noalloc(self, u, out, stream=None):
        """y = A u through fl_apply_noalloc: the product of apply() with the
        transform intermediates in the library's fixed scratch area (no
        device allocation; out must be given)."""
        import torch
        if u.dtype not in (torch.float32, torch.float64):
            raise TypeError("u must be float32 or float64")
        nrhs = self._nrhs(u)
        if out.dtype != u.dtype or out.numel() != u.numel() or not out.is_contiguous():
            raise ValueError("out must match u")
        check(self._lib.fl_apply_noalloc(self._h, ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), nrhs,
                                         1 if u.dtype == torch.float32 else 0,
                                         _stream_ptr(stream)))
        return out

    def exterior(self, g_lat, tail=None, out=None, stream=None):
        """Exterior-data term b (fl_exterior): g_lat holds g on the node
        lattice, [-N, N_s + N] along axis s (N_s = N on the cube), shape
        (nrhs, N_0 + 2N + 1, ...); tail the far-field integrals per interior
        point (nrhs, n_0, ...) or None."""
        import torch
        if g_lat.dtype != torch.float64 or not g_lat.is_contiguous():
            raise TypeError("g_lat must be a contiguous float64 tensor")
        lat = 1
        for v in self.intervals:
            lat *= v + 2 * self.N + 1
        if g_lat.numel() % lat:
            raise ValueError(f"g_lat must hold nrhs * {lat} values")
        nrhs = g_lat.numel() // lat
        if tail is not None and (tail.dtype != torch.float64 or tail.numel() != nrhs * self.nd
                                 or not tail.is_contiguous()):
            raise ValueError("tail must be a contiguous float64 tensor of nrhs * n^d values")
        if out is None:
            out = torch.empty((nrhs,) + self.shape, dtype=torch.float64, device=g_lat.device)
        check(self._lib.fl_exterior(self._h, ctypes.c_void_p(g_lat.data_ptr()),
                                    ctypes.c_void_p(tail.data_ptr()) if tail is not None
                                    else None, ctypes.c_void_p(out.data_ptr()), nrhs,
                                    _stream_ptr(stream)))
        return out

    def solve(self, f, tol=1e-10, maxiter=20000, mixed=False, out=None, stream=None,
              raise_on_fail=True, b=None):
        """u with A u = f - b by CG (b: the exterior-data term from exterior(),
        or None for g = 0).  mixed: False/0 FP64; True/1 FP32 CG with FP64
        reliable updates; 2 FP32 inner solves with FP64 iterative refinement.
        Returns (u, list of per-RHS info dicts)."""
        import torch
        if f.dtype != torch.float64:
            raise TypeError("f must be float64")
        nrhs = self._nrhs(f)
        if b is not None and (b.dtype != torch.float64 or b.shape != f.shape
                              or not b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 tensor shaped like f")
        if out is None:
            out = torch.empty_like(f)
        info = (FlInfo * nrhs)()
        st = self._lib.fl_solve(self._h, ctypes.c_void_p(f.data_ptr()),
                                ctypes.c_void_p(b.data_ptr()) if b is not None else None,
                                float(tol),
                                int(maxiter), int(mixed), ctypes.c_void_p(out.data_ptr()),
                                nrhs, info, _stream_ptr(stream))
        infos = [i.as_dict() for i in info]
        if raise_on_fail:
            check(st)
        return out, infos

    def solve_async(self, f, tol=1e-10, maxiter=20000, mixed=False, out=None, stream=None,
                    b=None):
        """Submit the solve of solve() without waiting (fl_solve_async).  f, b
        and out must stay alive and f, b unchanged until the returned
        request's wait()."""
        import torch
        if f.dtype != torch.float64:
            raise TypeError("f must be float64")
        nrhs = self._nrhs(f)
        if b is not None and (b.dtype != torch.float64 or b.shape != f.shape
                              or not b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 tensor shaped like f")
        if out is None:
            out = torch.empty_like(f)
        req = ctypes.c_void_p()
        check(self._lib.fl_solve_async(self._h, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(b.data_ptr()) if b is not None else None,
                                       float(tol), int(maxiter), int(mixed),
                                       ctypes.c_void_p(out.data_ptr()), nrhs,
                                       _stream_ptr(stream), ctypes.byref(req)))
        return SolveRequest(self, req, nrhs, (f, b, out))

    def profile_apply(self, u, out=None, reps=20, stream=None):
        """Mean milliseconds per kernel of y = A u (HIP events between the
        kernels, on the stream the kernels run on)."""
        return self._profile(self._lib.fl_profile_apply, u, out, reps, stream)

    def profile_precond(self, u, out=None, reps=20, stream=None):
        """Mean milliseconds per kernel of the preconditioner y = P u."""
        return self._profile(self._lib.fl_profile_precond, u, out, reps, stream)

    def profile_apply_each(self, u, out=None, reps=20, stream=None):
        """(back-to-back means, single-dispatch means) in milliseconds per
        kernel of y = A u: every launch also timed between its own events."""
        return self._profile(self._lib.fl_profile_apply, u, out, reps, stream, each=True)

    def profile_precond_each(self, u, out=None, reps=20, stream=None):
        return self._profile(self._lib.fl_profile_precond, u, out, reps, stream, each=True)

    def _profile(self, fn, u, out, reps, stream, each=False):
        import torch
        nrhs = self._nrhs(u)
        if out is None:
            out = torch.empty_like(u)
        npass_d = 1 if self.d == 1 else (3 if self.d == 2 else 5)   # kernels per product
        cap = 2 * npass_d if each else npass_d
        ms = (ctypes.c_double * cap)()
        npass = ctypes.c_int()
        check(fn(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), nrhs,
                 1 if u.dtype == torch.float32 else 0, int(reps), _stream_ptr(stream), ms, cap,
                 ctypes.byref(npass)))
        k = npass.value
        if each:
            return [ms[i] for i in range(k)], [ms[k + i] for i in range(k)]
        return [ms[i] for i in range(k)]

    def set_refinement(self, delta=1e-5, inner_tol=1e-4, max_outer=40):
        check(self._lib.fl_set_refinement(self._h, float(delta), float(inner_tol),
                                          int(max_outer)))

    def set_schedule(self, fp32, e_first=0, e_mid=0, e_c2c=0, w_first=0, w_c2c=0, lpb_mid=0,
                     precond=False):
        """Launch schedule of the product's passes, or with precond=True of
        the preconditioner's passes (0 keeps a value)."""
        fn = self._lib.fl_set_precond_schedule if precond else self._lib.fl_set_schedule
        check(fn(self._h, int(bool(fp32)), e_first, e_mid, e_c2c, w_first, w_c2c, lpb_mid))

    def set_preconditioner(self, kind):
        """2: tau preconditioner (default), 1: restricted inverse of the
        embedding circulant, 0: plain CG."""
        check(self._lib.fl_set_preconditioner(self._h, int(kind)))
        self.precond_kind = int(kind)

    def apply_precond(self, u, out=None, stream=None):
        """y = P u with the selected preconditioner (2: tau inverse by sine
        transforms, 1: restricted inverse of the embedding circulant)."""
        import torch
        nrhs = self._nrhs(u)
        if out is None:
            out = torch.empty_like(u)
        check(self._lib.fl_apply_precond(self._h, ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), nrhs,
                                         1 if u.dtype == torch.float32 else 0,
                                         _stream_ptr(stream)))
        return out

    def set_graphs(self, enable):
        """1 / True: capture CG chunks as HIP graphs at their first launch
        (default); 2: capture them when they come a second time (operators
        solved once pay nothing for capture); 0 / False: direct launches."""
        check(self._lib.fl_set_graphs(self._h, int(enable)))

    def get_schedule(self, fp32, precond=False):
        s = (ctypes.c_int * 6)()
        fn = self._lib.fl_get_precond_schedule if precond else self._lib.fl_get_schedule
        check(fn(self._h, int(bool(fp32)), s))
        return dict(zip(["e_first", "e_mid", "e_c2c", "w_first", "w_c2c", "lpb_mid"], list(s)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.fl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
