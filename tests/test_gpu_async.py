"""The asynchronous solve (fl_solve_async / fl_poll / fl_wait) and the
caller's device allocator (fl_set_allocator).

An asynchronous solve gives the bits of the blocking one (same operator,
same input, same graphs), while several run at once on different operators
and queue on one; its failures come back through fl_wait.  With torch's
caching allocator registered, the operator's memory comes from torch and
goes back to it, and the results are the bits of a default operator.
Operators created concurrently from several threads (one shared setup
scratch area per device) equal those created one at a time.
"""

import time

import numpy as np
import pytest

from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make_op(alpha, N=128, p=1):
    import paper_2103_03658_amd as fl
    return fl.Operator(2, alpha, p, N=N)


def wait_all(reqs, limit_s=60.0):
    t0 = time.time()
    while not all(r.done() for r in reqs):
        assert time.time() - t0 < limit_s, "asynchronous solves did not finish"
        time.sleep(0.002)
    return [r.wait() for r in reqs]


@pytest.mark.parametrize("mixed", [0, 1])
def test_async_matches_blocking(mixed):
    print(f"[async] mixed={mixed}", flush=True)
    ops = [make_op(a) for a in (0.5, 1.0, 1.5)]
    fs = [torch.from_numpy(inputs.uniform_rhs(2, 128, 3, seed=40 + i)).cuda() for i in range(3)]
    ref = [op.solve(f, tol=1e-10, mixed=mixed) for op, f in zip(ops, fs)]
    # three operators at once, and a second request queued on the first one
    f4 = torch.from_numpy(inputs.uniform_rhs(2, 128, 3, seed=77)).cuda()
    ref4 = ops[0].solve(f4, tol=1e-10, mixed=mixed)
    reqs = [op.solve_async(f, tol=1e-10, mixed=mixed) for op, f in zip(ops, fs)]
    reqs.append(ops[0].solve_async(f4, tol=1e-10, mixed=mixed))
    got = wait_all(reqs)
    for (u, info), (ur, infor) in zip(got, ref + [ref4]):
        assert torch.equal(u, ur)
        assert [i["iters"] for i in info] == [i["iters"] for i in infor]
        assert all(i["converged"] == 1 for i in info)


def test_async_orders_after_the_callers_stream():
    """The solve starts after the work queued on the given stream: a right-hand
    side still being written there is the one solved."""
    op = make_op(1.2)
    s = torch.cuda.Stream()
    f = torch.zeros((2, 127, 127), dtype=torch.float64, device="cuda")
    src = torch.from_numpy(inputs.uniform_rhs(2, 128, 2, seed=5)).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        torch.cuda._sleep(2_000_000)          # keep the stream busy first
        f.copy_(src)
    req = op.solve_async(f, tol=1e-10, stream=s)
    u, info = req.wait()
    ur, _ = op.solve(src, tol=1e-10)
    assert torch.equal(u, ur)


def test_async_failure_comes_back_through_wait():
    import paper_2103_03658_amd as fl
    op = make_op(1.5)
    f = torch.from_numpy(inputs.uniform_rhs(2, 128, 2, seed=9)).cuda()
    req = op.solve_async(f, tol=1e-14, maxiter=2)
    with pytest.raises(fl.FlError):
        req.wait()
    u, info = op.solve_async(f, tol=1e-14, maxiter=2).wait(raise_on_fail=False)
    assert all(i["converged"] == 0 and i["iters"] <= 2 for i in info)


def test_torch_allocator_holds_operator_memory():
    import paper_2103_03658_amd as fl
    made, returned = [], []

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n)
        made.append(p)
        return p

    def release(p):
        returned.append(p)
        torch.cuda.caching_allocator_delete(p)

    f = torch.from_numpy(inputs.uniform_rhs(2, 128, 3, seed=2)).cuda()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    fl.set_allocator(alloc, release)
    try:
        op = make_op(0.8)
        u, info = op.solve(f, tol=1e-10)
        y = op.apply(f)
        held = torch.cuda.memory_allocated() - before
    finally:
        fl.set_allocator(None, None)
    ref = make_op(0.8)
    ur, _ = ref.solve(f, tol=1e-10)
    assert torch.equal(u, ur) and torch.equal(y, ref.apply(f))
    # the generator and symbols alone are (N+1)^2 + 4 (M/2+1)^2 values
    assert held >= 129 * 129 * 8 and len(made) > 5
    assert set(returned) <= set(made)
    op.close()
    torch.cuda.synchronize()
    assert sorted(returned) == sorted(made)


def test_concurrent_setup_matches_sequential():
    """Operators created at once from several threads (sharing the device's
    setup scratch area, which grows on the way: N = 32 ... 512, p = 0 ... 2)
    hold the generator and symbol of operators created one at a time."""
    import threading
    import paper_2103_03658_amd as fl
    shapes = [(2, 0.3 + 0.1 * i, i % 3, (32, 64, 128, 256, 512)[i % 5]) for i in range(12)]
    shapes.append((3, 0.9, 1, 32))
    ref = []
    for d, a, p, N in shapes:
        op = fl.Operator(d, a, p, N=N)
        ref.append((op.generator(), op.symbol()))
        op.close()
    got = [None] * len(shapes)
    errs = []

    def make(i):
        try:
            d, a, p, N = shapes[i]
            got[i] = fl.Operator(d, a, p, N=N)
        except Exception as exc:   # surfaced by the assertion below
            errs.append(repr(exc))

    threads = [threading.Thread(target=make, args=(i,)) for i in range(len(shapes))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(120)
    assert not errs and all(g is not None for g in got), errs
    for (G, lam), op in zip(ref, got):
        assert np.array_equal(op.generator(), G) and np.array_equal(op.symbol(), lam)
        op.close()


@pytest.mark.parametrize("mixed", [0, 1])
def test_calls_during_async_solve_wait_for_it(mixed):
    """Calls on a handle whose asynchronous solve is running wait for it (the
    handle's lock): an apply with more right-hand sides than the solve (its
    transform workspace must grow, which would free the solve's) and a
    schedule change, issued right after the submission, leave the solve's
    bits those of the blocking solve, and the apply's those of an apply on a
    fresh operator."""
    print(f"[async lock] mixed={mixed}", flush=True)
    op = make_op(1.1)
    ref_op = make_op(1.1)
    f = torch.from_numpy(inputs.uniform_rhs(2, 128, 2, seed=31)).cuda()
    big = torch.from_numpy(inputs.uniform_rhs(2, 128, 12, seed=32)).cuda()
    ur, infor = ref_op.solve(f, tol=1e-10, mixed=mixed)
    yr = ref_op.apply(big)
    torch.cuda.synchronize()
    req = op.solve_async(f, tol=1e-10, mixed=mixed)
    y = op.apply(big)
    sched = op.get_schedule(False)
    op.set_schedule(False, **sched)          # same values: results unchanged
    u, info = req.wait()
    torch.cuda.synchronize()
    assert torch.equal(u, ur)
    assert [i["iters"] for i in info] == [i["iters"] for i in infor]
    assert torch.equal(y, yr)
