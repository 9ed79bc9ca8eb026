"""Kernels K(r) = sum_i c_i exp(-lambda_i r) (Remark 2.2) on the GPU
(fl_weights_expsum): the weight integrals and the far-field constant of each
term, scaled by c_i and summed, then one origin rule and one set of a_k, a_0.

Parity against the oracle's generator for the same kernel (d = 1, 2, 3,
p = 0, 1, 2), one-term kernels bit-identical to the fractional and tempered
entry points, FP64/FP32 products on a cube and a box, solves against
Cholesky, and a 1D solve whose error falls at second order towards the exact
solution of the continuous problem with that K (right-hand side by the
oracle's quadrature of the operator).
"""

import math

import numpy as np
import pytest

import oracle
from oracle import continuous as C
from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

A = [(0.5, 0.0), (0.3, 1.0), (0.2, 4.0)]
B = [(0.7, 0.2), (0.1, 8.0), (2.0, 0.0), (0.05, 30.0)]
S = [(1.0, 0.0), (1e-3, 0.5)]   # a small tempered part on top of K = 1

_ORC = {}


def orc_gen(d, alpha, p, N, terms):
    key = (d, alpha, p, N, tuple(terms))
    if key not in _ORC:
        _ORC[key] = oracle.generator_expsum(d, alpha, p, N, terms)
    return _ORC[key]


def make_op(d, alpha, p, N, terms, box=None):
    import paper_2103_03658_amd as fl
    return fl.Operator(d, alpha, p, N=N, kernel="expsum", terms=terms, box=box)


def abs_scale(G, u):
    return float(np.abs(oracle.apply(np.abs(G), np.abs(u))).max())


GEN_CASES = [(1, 1.3, 1, 64, A), (1, 0.5, 2, 32, B), (1, 1.9, 0, 16, S), (2, 1.2, 1, 16, A),
             (2, 0.7, 2, 16, B), (2, 1.6, 0, 8, A), (3, 1.0, 1, 4, A), (3, 0.4, 2, 4, S)]


@pytest.mark.parametrize("d,alpha,p,N,terms", GEN_CASES)
def test_expsum_generator_parity(d, alpha, p, N, terms):
    print(f"[expsum gen] d={d} alpha={alpha} p={p} N={N} terms={terms}", flush=True)
    Gg = make_op(d, alpha, p, N, terms).generator()
    Go = orc_gen(d, alpha, p, N, terms)
    err = np.abs(Gg - Go)
    bound = 1e-12 * np.abs(Go).max() + 1e-10 * np.abs(Go)
    assert (err <= bound).all(), float((err / np.abs(Go).max()).max())


@pytest.mark.parametrize("d,N", [(1, 64), (2, 16), (3, 8)])
def test_one_term_is_the_fractional_or_tempered_operator(d, N):
    import paper_2103_03658_amd as fl
    frac = fl.Operator(d, 1.1, 1, N=N)
    temp = fl.Operator(d, 1.1, 1, N=N, kernel="tempered", lam=2.5)
    assert np.array_equal(make_op(d, 1.1, 1, N, [(1.0, 0.0)]).generator(), frac.generator())
    one = make_op(d, 1.1, 1, N, [(1.0, 2.5)])
    assert np.array_equal(one.generator(), temp.generator())
    assert np.array_equal(one.symbol(), temp.symbol())


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("d,alpha,p,N,terms,box", [(2, 1.2, 1, 32, A, None),
                                                   (2, 0.7, 2, 16, B, (16, 10)),
                                                   (3, 1.0, 1, 8, A, (8, 5, 6)),
                                                   (1, 1.5, 1, 1024, B, None)])
def test_expsum_apply_parity(d, alpha, p, N, terms, box, fp32):
    print(f"[expsum apply] d={d} N={N} box={box} fp32={fp32}", flush=True)
    op = make_op(d, alpha, p, N, terms, box=box)
    u = inputs.uniform_grid(op.shape, 2, seed=21)
    ut = torch.from_numpy(u.astype(np.float32) if fp32 else u).cuda()
    y = op.apply(ut).double().cpu().numpy()
    G = orc_gen(d, alpha, p, op.N, terms)
    tol = 5e-6 if fp32 else 1e-12
    for r in range(2):
        ur = ut[r].double().cpu().numpy()
        assert np.abs(y[r] - oracle.apply(G, ur)).max() <= tol * abs_scale(G, ur), r


@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("d,alpha,p,N,terms,box", [(2, 1.2, 1, 16, A, None),
                                                   (2, 1.7, 1, 16, B, (16, 12)),
                                                   (3, 0.8, 1, 8, A, None)])
def test_expsum_solve_matches_cholesky(d, alpha, p, N, terms, box, mixed):
    op = make_op(d, alpha, p, N, terms, box=box)
    f = inputs.uniform_grid(op.shape, 2, seed=8)
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10, mixed=mixed)
    u = u.cpu().numpy()
    G = orc_gen(d, alpha, p, op.N, terms)
    for r in range(2):
        assert info[r]["converged"] == 1
        assert info[r]["relres_true"] <= 2e-10
        uc = oracle.solve_cholesky(G, f[r])
        assert np.abs(u[r] - uc).max() <= 1e-8 * np.abs(uc).max()


def test_expsum_solve_second_order_1d():
    alpha = 1.2

    def K(r):
        return sum(c * math.exp(-lam * r) for c, lam in A)

    errs = []
    for N in (128, 256, 512, 1024):
        x = oracle.grid_points(N)
        f = C.nonlocal_1d(C.BumpSquared, x, alpha, K)
        op = make_op(1, alpha, 1, N, A)
        u, info = op.solve(torch.from_numpy(f[None].copy()).cuda(), tol=1e-12)
        assert info[0]["converged"] == 1
        errs.append(np.abs(u[0].cpu().numpy() - C.BumpSquared.value(x)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.85 <= r <= 2.5 for r in rates), (errs, rates)
