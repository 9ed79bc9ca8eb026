"""Splitting parameter gamma < 2 on the GPU (fl_weights_gamma): generator,
product and solve against the oracle's scheme with the same gamma, and the
convergence rate the paper states for gamma = 1 + alpha/2 (phi^0, phi^1)."""

import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make_op(d, alpha, p, N, gamma, lam=0.0):
    import paper_2103_03658_amd as fl
    if lam:
        return fl.Operator(d, alpha, p, N=N, kernel="tempered", lam=lam, gamma=gamma)
    return fl.Operator(d, alpha, p, N=N, gamma=gamma)


CASES = [(1, 0.6, 0, 64, 1.3, 0.0), (1, 1.5, 2, 64, 1.75, 0.0), (1, 1.0, 1, 32, 1.2, 2.0),
         (2, 1.0, 1, 16, 1.5, 0.0), (2, 0.4, 2, 16, 1.0, 0.0), (2, 1.2, 1, 16, 1.6, 1.0),
         (3, 1.0, 1, 8, 1.5, 0.0), (3, 0.5, 0, 4, 1.9, 0.0)]


@pytest.mark.parametrize("d,alpha,p,N,gamma,lam", CASES)
def test_generator_gamma_parity(d, alpha, p, N, gamma, lam):
    op = make_op(d, alpha, p, N, gamma, lam)
    Go = oracle.generator(d, alpha, p, N, lam=lam, gamma=gamma)
    err = np.abs(op.generator() - Go)
    assert (err <= 1e-12 * np.abs(Go).max() + 1e-10 * np.abs(Go)).all(), \
        float((err / np.abs(Go).max()).max())


@pytest.mark.parametrize("d,alpha,p,N,gamma,lam", CASES[:6])
def test_apply_and_solve_gamma_parity(d, alpha, p, N, gamma, lam):
    op = make_op(d, alpha, p, N, gamma, lam)
    G = oracle.generator(d, alpha, p, N, lam=lam, gamma=gamma)
    f = inputs.uniform_rhs(d, N, 2, seed=17)
    y = op.apply(torch.from_numpy(f).cuda()).cpu().numpy()
    for r in range(2):
        ref = oracle.apply(G, f[r])
        scale = float(np.abs(oracle.apply(np.abs(G), np.abs(f[r]))).max())
        assert np.abs(y[r] - ref).max() <= 1e-12 * scale
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-11)
    for r in range(2):
        uc = oracle.solve_cholesky(G, f[r])
        assert np.abs(u[r].cpu().numpy() - uc).max() <= 1e-8 * np.abs(uc).max()


@pytest.mark.parametrize("p", [0, 1])
def test_gamma_rate_on_gpu(p):
    """gamma = 1 + alpha/2, alpha = 0.6: error decays like h^{2-alpha}."""
    alpha = 0.6
    gamma = 1.0 + alpha / 2
    s = 2.1 + alpha
    errs = []
    for N in (128, 256, 512):
        op = make_op(1, alpha, p, N, gamma)
        x = oracle.grid_points(N)
        y = op.apply(torch.from_numpy(((1 - x * x) ** s)[None].copy()).cuda()).cpu().numpy()[0]
        errs.append(np.abs(y - exact.frac_lap_ball_power(x * x, s, alpha, 1)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - (2.0 - alpha)) <= 0.05 for r in rates), rates
