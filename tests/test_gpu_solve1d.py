"""The 1D FP64 solve, which runs the whole PCG in one launch (one workgroup
per right-hand side): its solutions against Cholesky for each
preconditioner, and the stopping rules it shares with the multi-kernel
solve (iteration cap, zero right-hand side, iteration counts)."""

import numpy as np
import pytest

import oracle
from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make_op(alpha, p, N):
    import paper_2103_03658_amd as fl
    return fl.Operator(1, alpha, p, N=N)


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("alpha,p,N", [(1.5, 1, 1024), (0.6, 2, 64), (1.1, 0, 100), (1.9, 1, 8)])
def test_one_launch_solve_matches_cholesky(alpha, p, N, kind):
    import paper_2103_03658_amd as fl
    op = make_op(alpha, p, N)
    if kind == 2 and op.precond_kind != 2:
        # the tau preconditioner needs 2N without prime factors above 7 (with
        # 2N not a power of two it runs the multi-kernel iteration)
        with pytest.raises(fl.FlError) as exc:
            op.set_preconditioner(kind)
        assert exc.value.status == 2              # FL_E_UNSUPPORTED
        return
    op.set_preconditioner(kind)
    f = inputs.uniform_rhs(1, N, 3, seed=12)
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-12)
    G = oracle.generator(1, alpha, p, N)
    for r in range(3):
        assert info[r]["converged"] == 1 and info[r]["relres_true"] <= 2e-12
        uc = oracle.solve_cholesky(G, f[r])
        assert np.abs(u[r].cpu().numpy() - uc).max() <= 1e-9 * np.abs(uc).max()


def test_one_launch_solve_stopping_rules():
    import paper_2103_03658_amd as fl
    op = make_op(1.5, 1, 256)
    op.set_preconditioner(0)
    f = torch.from_numpy(inputs.uniform_rhs(1, 256, 2, seed=3)).cuda()
    f[1].zero_()
    u, info = op.solve(f, tol=1e-14, maxiter=5, raise_on_fail=False)
    assert info[0]["iters"] == 5 and info[0]["converged"] == 0
    assert info[0]["status"] == 5                      # FL_E_NOCONV
    assert info[1]["iters"] == 0 and info[1]["converged"] == 1
    assert torch.count_nonzero(u[1]) == 0
    with pytest.raises(fl.FlError):
        op.solve(f, tol=1e-14, maxiter=5)
    # the same counts as a loose solve stopped by the tolerance
    op.set_preconditioner(1)
    _, i1 = op.solve(f[:1].contiguous(), tol=1e-6)
    _, i2 = op.solve(f[:1].contiguous(), tol=1e-6, maxiter=i1[0]["iters"])
    assert i2[0]["converged"] == 1 and i2[0]["iters"] == i1[0]["iters"]
