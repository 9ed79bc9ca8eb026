"""fl_apply_noalloc, the product for callers that cannot allocate device
memory, against fl_apply through the C ABI: the same kernels and schedule
with the transform intermediates in the library's fixed scratch area, so
the same bits.  Two calls in a row, the second on a smaller input (fewer
right-hand sides, a smaller operator), then the largest product the area
holds and the first one it does not.
"""

import ctypes

import numpy as np
import pytest

from paper_2103_03658_amd import _lib, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ops():
    import paper_2103_03658_amd as fl
    return fl


def _abi_apply(op, fn, u, out):
    nrhs = u.numel() // op.nd
    return fn(op._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), nrhs,
              1 if u.dtype == torch.float32 else 0, None)


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_matches_apply_twice(fp32):
    fl = _ops()
    lib = fl.lib()
    dt = torch.float32 if fp32 else torch.float64
    cases = [(2, 1.3, 2, 128, 5), (2, 0.7, 1, 64, 2), (3, 1.0, 1, 32, 3), (3, 1.6, 0, 16, 1),
             (1, 1.5, 1, 1024, 3), (1, 0.4, 2, 64, 1)]
    for d, alpha, p, N, nrhs in cases:
        print(f"[noalloc] d={d} alpha={alpha} p={p} N={N} nrhs={nrhs} fp32={fp32}", flush=True)
        op = fl.Operator(d, alpha, p, N=N)
        u = torch.from_numpy(inputs.uniform_rhs(d, N, nrhs, seed=N + nrhs)).to(dt).cuda()
        y_ref = torch.empty_like(u)
        y = torch.full_like(u, float("nan"))
        assert _abi_apply(op, lib.fl_apply, u, y_ref) == _lib.FL_OK
        assert _abi_apply(op, lib.fl_apply_noalloc, u, y) == _lib.FL_OK
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), (d, N, nrhs)
        # second call on the same operator with fewer right-hand sides
        if nrhs > 1:
            u2 = u[:nrhs - 1].contiguous() * 0.5
            y2_ref, y2 = torch.empty_like(u2), torch.full_like(u2, float("nan"))
            assert _abi_apply(op, lib.fl_apply, u2, y2_ref) == _lib.FL_OK
            assert _abi_apply(op, lib.fl_apply_noalloc, u2, y2) == _lib.FL_OK
            torch.cuda.synchronize()
            assert torch.equal(y2, y2_ref), (d, N, nrhs - 1)
        op.close()


def test_noalloc_against_oracle():
    """The product itself: 2D p = 2 against the oracle's dense product."""
    import oracle
    fl = _ops()
    d, alpha, p, N = 2, 1.5, 2, 32
    op = fl.Operator(d, alpha, p, N=N)
    u = inputs.uniform_rhs(d, N, 3, seed=4)
    y = op.apply_noalloc(torch.from_numpy(u).cuda(), torch.empty(u.shape, dtype=torch.float64,
                                                                  device="cuda")).cpu().numpy()
    G = oracle.generator(d, alpha, p, N)
    for r in range(3):
        ref = oracle.apply(G, u[r])
        scale = np.abs(oracle.apply(np.abs(G), np.abs(u[r]))).max()
        assert np.abs(y[r] - ref).max() <= 1e-12 * scale


def test_noalloc_largest_and_rejected():
    """2D N = 512 FP64 needs 513 * 511 * 16 bytes per right-hand side: 32
    fill the 128 MiB area to within 512 bytes (the area's end is used), 33 are
    rejected before any launch."""
    fl = _ops()
    lib = fl.lib()
    assert _lib.FL_NOALLOC_SCRATCH_MIB == 128
    op = fl.Operator(2, 1.0, 2, N=512)
    per = 513 * 511 * 16
    assert 32 * per <= (128 << 20) < 33 * per
    u = torch.from_numpy(inputs.uniform_rhs(2, 512, 32, seed=11)).cuda()
    y_ref, y = torch.empty_like(u), torch.full_like(u, float("nan"))
    assert _abi_apply(op, lib.fl_apply, u, y_ref) == _lib.FL_OK
    assert _abi_apply(op, lib.fl_apply_noalloc, u, y) == _lib.FL_OK
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref)
    u33 = torch.zeros((33, 511, 511), dtype=torch.float64, device="cuda")
    y33 = torch.empty_like(u33)
    assert _abi_apply(op, lib.fl_apply_noalloc, u33, y33) == _lib.FL_E_UNSUPPORTED
    assert b"fixed scratch area" in lib.fl_last_error()
    # a smaller call after the rejected one still works
    u1 = u[:1].contiguous()
    y1_ref, y1 = torch.empty_like(u1), torch.full_like(u1, float("nan"))
    assert _abi_apply(op, lib.fl_apply, u1, y1_ref) == _lib.FL_OK
    assert _abi_apply(op, lib.fl_apply_noalloc, u1, y1) == _lib.FL_OK
    torch.cuda.synchronize()
    assert torch.equal(y1, y1_ref)
    op.close()
