"""Host logic of the serving loop on the CPU, with a stand-in operator in
place of the library's: requests for one operator merge into one batch up to
max_batch_rhs, every request gets back its own rows, oversize requests are
rejected, the operator cache evicts least recently used idle operators and
closes them, and each worker warms up on every given shape first."""

import threading

import pytest

torch = pytest.importorskip("torch")

import paper_2103_03658_amd as fl  # noqa: E402
from paper_2103_03658_amd import serve  # noqa: E402


class FakeOperator:
    made, closed, solves = [], [], []
    lock = threading.Lock()

    def __init__(self, d, alpha, degree, N=None, kernel="fractional", lam=0.0):
        self.key = (d, N, alpha, degree)
        with FakeOperator.lock:
            FakeOperator.made.append(self.key)

    def solve(self, f, tol=None, mixed=0, maxiter=None, stream=None, raise_on_fail=True):
        with FakeOperator.lock:
            FakeOperator.solves.append((self.key, int(f.shape[0]), mixed))
        info = [{"iters": 1, "converged": 1, "relres_true": 0.0} for _ in range(f.shape[0])]
        return 2.0 * f, info

    def close(self):
        with FakeOperator.lock:
            FakeOperator.closed.append(self.key)

    def set_graphs(self, mode):
        self.graphs = mode


class HostServer(serve.Server):
    def _open_stream(self):
        return None

    def _device_bytes_in_use(self):
        return 0

    def _tensor_device(self):
        return "cpu"


@pytest.fixture(autouse=True)
def fake_operator(monkeypatch):
    for lst in (FakeOperator.made, FakeOperator.closed, FakeOperator.solves):
        lst.clear()
    monkeypatch.setattr(fl, "Operator", FakeOperator)


def req(i, N, alpha, p, nrhs, t=0.0):
    f = torch.full((nrhs, N - 1, N - 1), float(i + 1), dtype=torch.float64)
    return serve.Request(i, 2, N, alpha, p, f, t_arrive=t)


def test_merging_and_results():
    reqs = [req(0, 16, 1.0, 1, 3), req(1, 16, 1.0, 1, 2), req(2, 32, 0.5, 0, 1),
            req(3, 16, 1.0, 1, 4), req(4, 16, 1.0, 1, 1)]
    srv = HostServer(workers=1, cache_bytes=1 << 40, max_batch_rhs=6, keep_solutions=True)
    st = srv.run(reqs, realtime=False)
    assert st["served"] == 5 and st["ok"] == 5 and st["rejected"] == 0
    for r in reqs:                                  # each request its own rows back
        assert torch.equal(r.u, 2.0 * r.f), r.id
    sizes = [n for key, n, _ in FakeOperator.solves if key[1] == 16]
    assert max(sizes) <= 6 and sum(sizes) == 10 and len(sizes) >= 2
    assert FakeOperator.made.count((2, 16, 1.0, 1)) == 1      # one operator, shared
    assert all(m == 0 for _, _, m in FakeOperator.solves)     # FP64 by default


def test_admission_rejects_what_never_fits():
    srv = HostServer(workers=2, hbm_budget=1024, cache_bytes=1 << 40)
    st = srv.run([req(0, 16, 1.0, 1, 1), req(1, 32, 1.0, 1, 2)], realtime=False)
    assert st["rejected"] == 2 and st["served"] == 0 and not FakeOperator.solves


def test_lru_eviction_closes_idle_operators():
    one = serve.op_bytes(2, 16) + serve.batch_bytes(2, 16, 1)
    srv = HostServer(workers=1, cache_bytes=2 * one)          # room for two operators
    alphas = [0.3, 0.4, 0.3, 0.5, 0.6]
    # arrivals 50 ms apart: one batch per request, in order
    st = srv.run([req(i, 16, a, 0, 1, t=0.05 * i) for i, a in enumerate(alphas)])
    assert st["served"] == 5 and st["batches"] == 5
    # 0.3 was used again before 0.5 arrived, so 0.4 went first, then 0.3
    assert FakeOperator.closed == [(2, 16, 0.4, 0), (2, 16, 0.3, 0)]
    assert [k[2] for k in srv._ops] == [0.5, 0.6]
    assert srv._cached <= 2 * one
    assert FakeOperator.made.count((2, 16, 0.3, 0)) == 1


def test_every_worker_warms_up_first():
    warm = [(2, 16, 0), (2, 32, 2)]
    srv = HostServer(workers=3, cache_bytes=1 << 40, warm=warm)
    st = srv.run([req(0, 16, 1.0, 1, 1)], realtime=False)
    assert st["served"] == 1 and st["warmup_s"] >= 0 and not st["errors"]
    warm_solves = [s for s in FakeOperator.solves if s[0][2] == 1.0 and s[0][1] in (16, 32)
                   and s[0][3] in (0, 2)]
    assert len(warm_solves) == 3 * len(warm)
    assert FakeOperator.closed.count((2, 16, 1.0, 0)) == 3     # warm-up operators closed
