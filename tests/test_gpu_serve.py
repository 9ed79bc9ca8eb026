"""Serving loop on the GPU: results are the same alone and in the mix, the
HBM budget is enforced, operators are shared through the cache."""

import numpy as np
import pytest

from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests(specs, seed=0):
    from paper_2103_03658_amd.serve import Request
    out = []
    for i, (N, alpha, p, nrhs) in enumerate(specs):
        f = np.stack([np.random.default_rng([seed, i, j]).uniform(-1, 1, (N - 1, N - 1))
                      for j in range(nrhs)])
        out.append(Request(i, 2, N, alpha, p, torch.from_numpy(f).cuda(), t_arrive=0.0))
    return out


SPECS = [(32, 1.0, 1, 2), (16, 0.5, 0, 1), (32, 1.0, 1, 3), (64, 1.7, 2, 2), (32, 1.0, 1, 1),
         (16, 1.9, 2, 4), (64, 0.3, 1, 1), (32, 1.2, 0, 2), (16, 0.5, 0, 2), (64, 1.7, 2, 1)]


def test_results_same_alone_and_in_mix():
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd.serve import Server
    reqs = _requests(SPECS)
    srv = Server(workers=3, keep_solutions=True)
    st = srv.run(reqs, realtime=False)
    assert st["served"] == len(SPECS) and st["ok"] == len(SPECS), st
    assert st["max_relres_true"] <= 1e-10
    assert st["mean_requests_per_batch"] > 1.0          # shared operators were merged
    for r in reqs:
        op = fl.Operator(2, r.alpha, r.degree, N=r.N)
        u, info = op.solve(r.f, tol=1e-10, mixed=srv.mixed)
        assert torch.equal(u, r.u), r.id
        op.close()


def test_hbm_budget_admission():
    from paper_2103_03658_amd.serve import Server, batch_bytes, op_bytes
    reqs = _requests(SPECS[:4], seed=1)
    need = max(op_bytes(2, r.N) + batch_bytes(2, r.N, r.nrhs) for r in reqs)
    srv = Server(workers=3, hbm_budget=need)           # one batch at a time at most
    st = srv.run(reqs, realtime=False)
    assert st["served"] == 4 and st["rejected"] == 0
    tiny = Server(workers=2, hbm_budget=1024)
    st2 = tiny.run(_requests(SPECS[:3], seed=2), realtime=False)
    assert st2["rejected"] == 3 and st2["served"] == 0


def test_cache_eviction_keeps_results_and_budget():
    """A cache budget of about one operator: idle operators are closed as new
    ones arrive (outside the server's lock), and every result is still the
    one of a fresh operator.  The workers warm up first without errors."""
    import paper_2103_03658_amd as fl
    from paper_2103_03658_amd.serve import Server, batch_bytes, op_bytes
    reqs = _requests(SPECS, seed=3)
    budget = op_bytes(2, 64) + batch_bytes(2, 64, 4)
    srv = Server(workers=3, cache_bytes=budget, keep_solutions=True, warm=[(2, 16, 0), (2, 32, 1)])
    st = srv.run(reqs, realtime=False)
    assert st["served"] == len(SPECS) and st["ok"] == len(SPECS), st
    assert st["warmup_s"] > 0 and not st["errors"], st
    assert srv._cached <= budget or len(srv._ops) == 1
    assert len(srv._ops) < len({r.key for r in reqs})
    for r in reqs:
        op = fl.Operator(2, r.alpha, r.degree, N=r.N)
        u, info = op.solve(r.f, tol=1e-10, mixed=srv.mixed)
        assert torch.equal(u, r.u), r.id
        op.close()
