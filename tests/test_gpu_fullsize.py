"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (tuned schedules, batched right-hand
sides), on outputs the oracle can compute one by one:

* 2D N = 512, p = 2 (the 511^2 headline solve) and the tempered 2D N = 1024
  grid (1023^2, linear basis): products at sampled rows against the oracle's
  exact row sums, and solved systems' true residuals with the oracle's
  block-Toeplitz product;
* 3D N = 128 (127^3): the whole oracle lattice is out of reach, so sampled
  generator entries come from the oracle's per-node quadrature, the diagonal
  from the full-stencil identity sum_k G = c 2^d T_d, and the product is
  checked by properties that hold at any size (columns of A e_j against the
  generator, symmetry u.Av = v.Au, FP32 against FP64).
"""

import math

import numpy as np
import pytest

import oracle
from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_ORC = {}


def orc_gen(d, alpha, p, N, lam=0.0):
    key = (d, alpha, p, N, lam)
    if key not in _ORC:
        _ORC[key] = oracle.generator(d, alpha, p, N, lam=lam)
    return _ORC[key]


def make_op(d, alpha, p, N, lam=0.0):
    import paper_2103_03658_amd as fl
    if lam:
        return fl.Operator(d, alpha, p, N=N, kernel="tempered", lam=lam)
    return fl.Operator(d, alpha, p, N=N)


def tuned(op, nrhs):
    from paper_2103_03658_amd import tune
    for fp32 in (True, False):
        tune.tune(op, nrhs, fp32, use_cache=False)


def sample_rows(n, d, k, seed):
    rng = np.random.default_rng(seed)
    edge = [[0] * d, [n - 1] * d, [n // 2] * d, [0] + [n - 1] * (d - 1), [n - 1] + [0] * (d - 1)]
    rnd = rng.integers(0, n, size=(k, d)).tolist()
    return np.array(edge + rnd, dtype=np.int64)


# (d, alpha, p, N, lam, nrhs): the 511^2 headline batch and the tempered 1023^2 batch
FULL2D = [(2, 1.5, 2, 512, 0.0, 17), (2, 1.2, 1, 1024, 1.0, 64)]


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("d,alpha,p,N,lam,nrhs", FULL2D)
def test_fullsize_2d_apply_sampled_rows(d, alpha, p, N, lam, nrhs, fp32):
    print(f"[full2d apply] N={N} p={p} alpha={alpha} lam={lam} nrhs={nrhs} fp32={fp32}",
          flush=True)
    op = make_op(d, alpha, p, N, lam)
    tuned(op, nrhs)
    u = inputs.uniform_rhs(d, N, nrhs, seed=21)
    if fp32:
        u = u.astype(np.float32)
    y = op.apply(torch.from_numpy(u).cuda()).double().cpu().numpy()
    G = orc_gen(d, alpha, p, N, lam)
    tol = 5e-6 if fp32 else 1e-12
    for r in (0, nrhs - 1):
        ur = u[r].astype(np.float64)
        rows = sample_rows(N - 1, d, 8, seed=r)
        ref = oracle.apply_rows(G, ur, rows)
        scale = oracle.apply_rows(np.abs(G), np.abs(ur), rows)
        got = y[r][tuple(rows.T)]
        assert (np.abs(got - ref) <= tol * scale).all(), float((np.abs(got - ref) / scale).max())


@pytest.mark.parametrize("mixed", [0, 1])
def test_fullsize_headline_solve_true_residual(mixed):
    """511^2, p = 2, alpha = 1: the benchmark's 17-RHS batch (manufactured f
    plus 16 uniform RHS) to 1e-10; the oracle's product gives the true
    residual of two of them."""
    N, alpha = 512, 1.0
    print(f"[full2d solve] N={N} mixed={mixed}", flush=True)
    op = make_op(2, alpha, 2, N)
    tuned(op, 17)
    f = np.concatenate([inputs.manufactured_rhs_disk(N, alpha)[None],
                        inputs.uniform_rhs(2, N, 16, seed=0)])
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10, mixed=mixed)
    u = u.cpu().numpy()
    G = orc_gen(2, alpha, 2, N)
    for r in (0, 16):
        assert info[r]["converged"] == 1
        res = f[r] - oracle.apply_bttb(G, u[r])
        rel = np.linalg.norm(res) / np.linalg.norm(f[r])
        print(f"  rhs {r}: iters {info[r]['iters']} oracle relres {rel:.2e} "
              f"gpu relres_true {info[r]['relres_true']:.2e}")
        assert rel <= 2e-10


def test_fullsize_tempered_solve_true_residual():
    """Tempered 1023^2 (lambda = 1, alpha = 1.2, p = 1): 64 N(0,1) RHS in one
    batched mixed-precision solve to 1e-10; oracle true residual of two."""
    N, alpha, lam = 1024, 1.2, 1.0
    print(f"[full tempered solve] N={N} lam={lam}", flush=True)
    op = make_op(2, alpha, 1, N, lam)
    tuned(op, 64)
    f = inputs.normal_rhs(2, N, 64, seed=0)
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10, mixed=1)
    assert all(i["converged"] == 1 for i in info)
    u = u.cpu().numpy()
    G = orc_gen(2, alpha, 1, N, lam)
    for r in (0, 63):
        rel = np.linalg.norm(f[r] - oracle.apply_bttb(G, u[r])) / np.linalg.norm(f[r])
        print(f"  rhs {r}: iters {info[r]['iters']} oracle relres {rel:.2e}")
        assert rel <= 2e-10


def _lattice_multiplicity(N, d):
    k = np.indices((N + 1,) * d).reshape(d, -1).T
    return 2.0 ** (d - (k == 0).sum(axis=1))


def test_fullsize_3d_generator_sampled_and_stencil_identity():
    """127^3 (N = 128, p = 1, alpha = 1): sampled entries against the
    oracle's per-node quadrature; the diagonal through sum_k G = c 2^3 T_3."""
    N, alpha = 128, 1.0
    op = make_op(3, alpha, 1, N)
    Gg = op.generator()
    rng = np.random.default_rng(5)
    nodes = [[3, 0, 0], [0, 0, 128], [128, 128, 128], [64, 1, 1], [1, 1, 1], [2, 1, 0]]
    nodes += rng.integers(0, N + 1, size=(8, 3)).tolist()
    nodes = np.array([k for k in nodes if sum(k) > 2], dtype=np.int64)
    Go = oracle.generator_at(3, alpha, 1, N, nodes)
    got = Gg[tuple(nodes.T)]
    assert (np.abs(got - Go) <= 1e-12 * np.abs(Gg).max() + 1e-10 * np.abs(Go)).all()
    total = math.fsum(_lattice_multiplicity(N, 3) * Gg.reshape(-1))
    ref = oracle.c_dalpha(3, alpha) * 8 * oracle.far_field_T(3, alpha, L=2.0)
    assert abs(total - ref) <= 1e-10 * np.abs(Gg).max()


def test_fullsize_3d_apply_properties():
    """127^3 products: A e_j equals the generator column at every sampled
    row, u.Av = v.Au, and the FP32 product agrees with the FP64 one."""
    N, alpha, n = 128, 1.0, 127
    op = make_op(3, alpha, 1, N)
    tuned(op, 1)
    Gg = op.generator()
    js = [(0, 0, 0), (63, 63, 63), (126, 0, 126), (5, 90, 33)]
    E = np.zeros((len(js), n, n, n))
    for m, j in enumerate(js):
        E[m][j] = 1.0
    Y = op.apply(torch.from_numpy(E).cuda()).cpu().numpy()
    rows = sample_rows(n, 3, 12, seed=7)
    for m, j in enumerate(js):
        off = np.abs(rows - np.array(j))
        ref = Gg[tuple(off.T)]
        assert np.abs(Y[m][tuple(rows.T)] - ref).max() <= 1e-12 * np.abs(Gg).max()
    uv = inputs.normal_rhs(3, N, 2, seed=3)
    Au = op.apply(torch.from_numpy(uv).cuda()).cpu().numpy()
    a = float(np.vdot(uv[1], Au[0]))
    b = float(np.vdot(uv[0], Au[1]))
    assert abs(a - b) <= 1e-12 * float(np.abs(uv[0]).sum() * np.abs(Au[1]).max())
    A32 = op.apply(torch.from_numpy(uv.astype(np.float32)).cuda()).double().cpu().numpy()
    assert np.abs(A32 - Au).max() <= 1e-5 * np.abs(Au).max()


def test_fullsize_3d_mixed_solve_matches_fp64():
    """127^3, alpha = 1, p = 1, N(0,1) RHS seed 3: the mixed-precision solve
    reaches the 1e-10 true residual and agrees with the FP64 GPU solve."""
    N = 128
    op = make_op(3, 1.0, 1, N)
    tuned(op, 1)
    f = torch.from_numpy(inputs.normal_rhs(3, N, 1, seed=3)).cuda()
    u1, i1 = op.solve(f, tol=1e-10, mixed=1)
    u0, i0 = op.solve(f, tol=1e-10, mixed=0)
    print(f"  mixed iters {i1[0]['iters']} outer {i1[0]['outer_iters']} relres "
          f"{i1[0]['relres_true']:.2e}; fp64 iters {i0[0]['iters']} relres {i0[0]['relres_true']:.2e}")
    assert i1[0]["converged"] == 1 and i0[0]["converged"] == 1
    assert i1[0]["relres_true"] <= 1e-10
    d = (u1 - u0).abs().max().item() / u0.abs().max().item()
    assert d <= 1e-8, d
