"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.

Tolerances (FP64):
  * generator G_k: |G_gpu - G_orc| <= 1e-12 max|G| + 1e-10 |G_orc| (both are
    ~1e-15-accurate quadratures of the same integrals; a_0 sums (N+1)^d terms);
  * symbol: <= 1e-12 max|lambda-hat|;
  * product y = A u: max_i |y_gpu - y_orc|_i <= 1e-12 max_i (|A| |u|)_i.
    y itself cancels heavily (|A||u| / |Au| reaches ~1e4), so the bound is
    taken relative to the magnitude of the summed terms;
  * FP32 product: 5e-6 max_i (|A||u|)_i (float rounding of a length-M^d
    transform pair, ~log2(M^d) * 6e-8 * growth);
  * solves: the oracle-evaluated residual ||f - A u||_2 / ||f||_2 <= tol +
    1e-12 (the FP64 solves stop on the recursive residual, which the true one
    follows to ~kappa eps; the oracle's own product adds ~eps |A||u|/|f|),
    and the forward error against the oracle's Cholesky solve
    ||u - u_c||_2 / ||u_c||_2 <= kappa_2(A) (residual + 1e-15), the bound
    that the residual implies (kappa from the oracle's eigvalsh; the 1e-15
    covers the Cholesky solve's own error).
Index maps (the embedding) are compared bit for bit.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2103_03658_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fl():
    import paper_2103_03658_amd as fl
    return fl


_ORC = {}


def orc_gen(d, alpha, p, N, lam=0.0):
    key = (d, alpha, p, N, lam)
    if key not in _ORC:
        _ORC[key] = oracle.generator(d, alpha, p, N, lam=lam)
    return _ORC[key]


def make_op(d, alpha, p, N, lam=0.0):
    fl = _fl()
    if lam:
        return fl.Operator(d, alpha, p, N=N, kernel="tempered", lam=lam)
    return fl.Operator(d, alpha, p, N=N)


_KAPPA = {}


def kappa2(d, alpha, p, N):
    """2-norm condition number of the dense A (oracle, eigvalsh)."""
    key = (d, alpha, p, N)
    if key not in _KAPPA:
        ev = np.linalg.eigvalsh(oracle.dense_matrix(orc_gen(d, alpha, p, N)))
        _KAPPA[key] = float(ev[-1] / ev[0])
    return _KAPPA[key]


def abs_scale(G, u):
    """max_i (|A| |u|)_i by the oracle's dense/block product."""
    return float(np.abs(oracle.apply(np.abs(G), np.abs(u))).max())


GEN_CASES = [
    (1, 1.5, 1, 1024, 0.0), (1, 0.5, 0, 64, 0.0), (1, 1.7, 2, 64, 0.0), (1, 0.3, 2, 8, 0.0),
    (2, 1.5, 2, 32, 0.0), (2, 0.5, 1, 16, 0.0), (2, 1.0, 0, 16, 0.0), (2, 1.9, 1, 8, 0.0),
    (3, 1.0, 1, 8, 0.0), (3, 1.5, 2, 8, 0.0), (3, 0.4, 0, 4, 0.0),
    (1, 1.2, 1, 64, 5.0), (2, 1.2, 1, 16, 0.5), (2, 1.2, 1, 16, 5.0), (2, 1.2, 2, 16, 1.0),
]


@pytest.mark.parametrize("d,alpha,p,N,lam", GEN_CASES)
def test_generator_parity(d, alpha, p, N, lam):
    print(f"[gen] d={d} alpha={alpha} p={p} N={N} lam={lam}", flush=True)
    op = make_op(d, alpha, p, N, lam)
    Gg = op.generator()
    Go = orc_gen(d, alpha, p, N, lam)
    err = np.abs(Gg - Go)
    bound = 1e-12 * np.abs(Go).max() + 1e-10 * np.abs(Go)
    assert (err <= bound).all(), float((err / np.abs(Go).max()).max())


@pytest.mark.parametrize("d,N,p", [(1, 8, 1), (1, 64, 2), (2, 8, 1), (2, 16, 2), (3, 4, 1),
                                   (3, 8, 0)])
def test_embedding_index_map_bit_exact(d, N, p):
    op = make_op(d, 0.9, p, N)
    Gg = op.generator()
    c = op.embedding()
    M = 2 * N
    j = np.arange(M)
    m = np.minimum(j, M - j)
    keep = m <= N - 2
    exp = Gg[np.ix_(*([m] * d))].copy()
    mask = keep
    for _ in range(1, d):
        mask = np.multiply.outer(mask, keep)
    exp[~mask] = 0.0
    assert np.array_equal(c, exp)
    # the zero pattern matches the oracle's embedding of its own generator
    co = oracle.embed_generator(orc_gen(d, 0.9, p, N))
    assert np.array_equal(c == 0.0, co == 0.0)


@pytest.mark.parametrize("d,alpha,p,N", [(1, 1.5, 1, 1024), (2, 1.5, 2, 32), (2, 0.5, 1, 16),
                                         (3, 1.0, 1, 8)])
def test_symbol_parity(d, alpha, p, N):
    op = make_op(d, alpha, p, N)
    lg = op.symbol()
    lo, imag = oracle.symbol(orc_gen(d, alpha, p, N))
    lo = lo[(slice(0, N + 1),) * d]
    assert np.abs(lg - lo).max() <= 1e-12 * np.abs(lo).max()


APPLY_CASES = [
    (1, 1.5, 1, 1024, 1, 0.0), (1, 0.7, 2, 8, 3, 0.0), (1, 1.1, 0, 64, 2, 0.0),
    (2, 1.5, 2, 32, 1, 0.0), (2, 0.5, 1, 64, 3, 0.0), (2, 1.0, 0, 8, 2, 0.0),
    (2, 1.9, 1, 128, 1, 0.0), (2, 1.2, 1, 16, 2, 5.0),
    (3, 1.0, 1, 8, 2, 0.0), (3, 1.5, 2, 16, 1, 0.0), (3, 0.6, 1, 4, 1, 0.0),
]


@pytest.mark.parametrize("d,alpha,p,N,nrhs,lam", APPLY_CASES)
def test_apply_fp64_parity(d, alpha, p, N, nrhs, lam):
    print(f"[apply64] d={d} alpha={alpha} p={p} N={N} nrhs={nrhs} lam={lam}", flush=True)
    op = make_op(d, alpha, p, N, lam)
    u = inputs.uniform_rhs(d, N, nrhs, seed=11)
    y = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    G = orc_gen(d, alpha, p, N, lam)
    for r in range(nrhs):
        ref = oracle.apply(G, u[r])
        assert np.abs(y[r] - ref).max() <= 1e-12 * abs_scale(G, u[r])


@pytest.mark.parametrize("d,alpha,p,N,nrhs,lam", APPLY_CASES)
def test_apply_fp32_parity(d, alpha, p, N, nrhs, lam):
    op = make_op(d, alpha, p, N, lam)
    u = inputs.uniform_rhs(d, N, nrhs, seed=12).astype(np.float32)
    y = op.apply(torch.from_numpy(u).cuda()).cpu().numpy().astype(np.float64)
    G = orc_gen(d, alpha, p, N, lam)
    for r in range(nrhs):
        ref = oracle.apply(G, u[r].astype(np.float64))
        assert np.abs(y[r] - ref).max() <= 5e-6 * abs_scale(G, u[r].astype(np.float64))


@pytest.mark.parametrize("d,N", [(1, 64), (2, 32), (3, 8)])
def test_apply_batch_invariance_bitwise(d, N):
    """A right-hand side gives the same bits alone and inside a batch."""
    op = make_op(d, 1.3, 1, N)
    u = torch.from_numpy(inputs.uniform_rhs(d, N, 3, seed=5)).cuda()
    yb = op.apply(u)
    for r in range(3):
        ya = op.apply(u[r].contiguous())
        assert torch.equal(ya, yb[r])


def test_apply_ragged_and_edge_sizes():
    """Smallest grid (N = 4: n = 3, M = 8) and odd column counts."""
    for d in (1, 2, 3):
        op = make_op(d, 1.0, 1, 4)
        u = inputs.uniform_rhs(d, 4, 1, seed=3)
        y = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
        G = orc_gen(d, 1.0, 1, 4)
        assert np.abs(y[0] - oracle.apply(G, u[0])).max() <= 1e-12 * abs_scale(G, u[0])


@pytest.mark.parametrize("pc", [2, 1, 0])
@pytest.mark.parametrize("d,alpha,p,N,mixed", [
    (1, 1.5, 1, 256, 0), (2, 1.5, 1, 16, 0), (2, 0.5, 2, 32, 0), (3, 1.0, 1, 8, 0),
    (2, 1.5, 1, 16, 1), (2, 1.0, 2, 32, 1), (3, 1.0, 1, 8, 1), (1, 1.5, 1, 256, 1),
    (2, 1.9, 2, 64, 1), (2, 1.5, 1, 16, 2), (2, 1.0, 2, 32, 2), (3, 1.0, 1, 8, 2),
    (1, 1.5, 1, 256, 2),
])
def test_solve_parity(d, alpha, p, N, mixed, pc):
    print(f"[solve] d={d} alpha={alpha} p={p} N={N} mixed={mixed} pc={pc}", flush=True)
    op = make_op(d, alpha, p, N)
    op.set_preconditioner(pc)
    f = inputs.uniform_rhs(d, N, 2, seed=0)
    tol = 1e-10
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=tol, mixed=mixed)
    u = u.cpu().numpy()
    G = orc_gen(d, alpha, p, N)
    kap = kappa2(d, alpha, p, N)
    for r in range(2):
        assert info[r]["converged"] == 1
        res = f[r] - oracle.apply(G, u[r])
        rel = np.linalg.norm(res) / np.linalg.norm(f[r])
        uc = oracle.solve_cholesky(G, f[r])
        fwd = np.linalg.norm(u[r] - uc) / np.linalg.norm(uc)
        print(f"  rhs {r}: iters={info[r]['iters']} outer={info[r]['outer_iters']} "
              f"relres={rel:.2e} fwd_err={fwd:.2e} kappa={kap:.3g} "
              f"bound={kap * (rel + 1e-15):.2e}")
        assert rel <= tol + 1e-12, rel
        assert fwd <= kap * (rel + 1e-15), (fwd, kap, rel)


def test_solve_c1_paper_grid():
    """1D, alpha = 1.5, linear basis, N = 1024 (h = 1/512): f = Gamma(2.5)
    (exact u = (1-x^2)_+^{3/4}) and f ~ U[-1,1] (seed 0), tolerance 1e-12."""
    op = make_op(1, 1.5, 1, 1024)
    f = np.stack([np.full(1023, math.gamma(2.5)), inputs.uniform_rhs(1, 1024, 1, seed=0)[0]])
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-12, maxiter=20000)
    u = u.cpu().numpy()
    G = orc_gen(1, 1.5, 1, 1024)
    for r in range(2):
        uc = oracle.solve_cholesky(G, f[r])
        assert np.abs(u[r] - uc).max() <= 1e-9 * np.abs(uc).max()
    x = oracle.grid_points(1024)
    err = np.abs(u[0] - (1 - x * x) ** 0.75).max()
    # Table 3.2.1 (alpha = 1.5, linear basis, h = 1/512) scaled by f = Gamma(2.5)
    assert abs(err - math.gamma(2.5) * 1.1717e-3) <= 1e-7


def test_solve_batch_invariance_bitwise():
    op = make_op(2, 1.2, 1, 32)
    f = torch.from_numpy(inputs.uniform_rhs(2, 32, 3, seed=9)).cuda()
    ub, _ = op.solve(f, tol=1e-10)
    for r in range(3):
        ua, _ = op.solve(f[r].contiguous(), tol=1e-10)
        assert torch.equal(ua, ub[r])


def test_solve_zero_rhs_and_maxiter():
    fl = _fl()
    op = make_op(2, 1.0, 1, 16)
    f = torch.zeros((2, 15, 15), dtype=torch.float64, device="cuda")
    f[1] = torch.from_numpy(inputs.uniform_rhs(2, 16, 1, seed=1)[0])
    u, info = op.solve(f, tol=1e-12, maxiter=3, raise_on_fail=False)
    assert torch.count_nonzero(u[0]) == 0 and info[0]["converged"] == 1
    assert info[1]["status"] == fl._lib.FL_E_NOCONV and info[1]["iters"] == 3
    with pytest.raises(fl.FlError):
        op.solve(f, tol=1e-12, maxiter=3)


@pytest.mark.parametrize("d,N,fp32", [(2, 64, False), (2, 64, True), (3, 16, False),
                                      (3, 16, True), (1, 256, True), (2, 512, False),
                                      (2, 512, True)])
def test_schedules_give_same_product(d, N, fp32):
    """Every launch schedule the tuner may pick computes the same product
    (radix 8/16/32 register stages, 1..16 lines per block; the bench's
    1024-point lines at N = 512)."""
    from paper_2103_03658_amd import tune
    op = make_op(d, 1.1, 1, N)
    u = inputs.uniform_rhs(d, N, 3, seed=21)
    ut = torch.from_numpy(u.astype(np.float32) if fp32 else u).cuda()
    G = orc_gen(d, 1.1, 1, N)
    scales = [abs_scale(G, u[r]) for r in range(3)]
    refs = [oracle.apply(G, ut[r].double().cpu().numpy()) for r in range(3)]
    tol = 5e-6 if fp32 else 1e-12
    base = op.get_schedule(fp32)
    tried = 0
    for E, W in tune.candidates(op.M, fp32):
        for ek, wk in (("e_first", "w_first"), ("e_mid", "lpb_mid"), ("e_c2c", "w_c2c")):
            if d == 1 and ek != "e_mid":
                continue
            s = dict(base)
            s[ek], s[wk] = E, W
            try:
                op.set_schedule(fp32, **s)
            except Exception:
                continue
            y = op.apply(ut).double().cpu().numpy()
            for r in range(3):
                assert np.abs(y[r] - refs[r]).max() <= tol * scales[r], (ek, E, wk, W)
            tried += 1
    assert tried >= 5


def test_mixed_solve_batch_invariance_bitwise():
    """Mixed-precision solve: a right-hand side gives the same bits alone and
    inside a batch (reliable updates are decided per right-hand side)."""
    op = make_op(2, 1.5, 2, 32)
    f = torch.from_numpy(inputs.uniform_rhs(2, 32, 3, seed=19)).cuda()
    ub, ib = op.solve(f, tol=1e-10, mixed=1)
    for r in range(3):
        ua, ia = op.solve(f[r].contiguous(), tol=1e-10, mixed=1)
        assert torch.equal(ua, ub[r])
        assert ia[0]["iters"] == ib[r]["iters"]


def test_mixed_maxiter_reports_noconv():
    fl = _fl()
    op = make_op(2, 1.5, 1, 32)
    f = torch.from_numpy(inputs.uniform_rhs(2, 32, 1, seed=2)).cuda()
    u, info = op.solve(f, tol=1e-12, maxiter=5, mixed=1, raise_on_fail=False)
    assert info[0]["status"] == fl._lib.FL_E_NOCONV
    assert info[0]["iters"] == 5
    # the reported residual is the FP64 residual of the returned iterate
    G = orc_gen(2, 1.5, 1, 32)
    fn = f.cpu().numpy()[0]
    rel = np.linalg.norm(fn - oracle.apply(G, u.cpu().numpy()[0])) / np.linalg.norm(fn)
    assert abs(rel - info[0]["relres_true"]) <= 1e-6 * rel


@pytest.mark.parametrize("mixed", [0, 1])
def test_graph_replays_match_eager(mixed):
    """Captured CG chunks replayed several times, with eager solves in
    between, give the same bits as launching every kernel directly."""
    op = make_op(2, 1.3, 2, 32)
    f = torch.from_numpy(inputs.uniform_rhs(2, 32, 2, seed=31)).cuda()
    op.set_graphs(False)
    ue, ie = op.solve(f, tol=1e-10, mixed=mixed)
    op.set_graphs(True)
    for rep in range(3):
        ug, ig = op.solve(f, tol=1e-10, mixed=mixed)      # capture, then replays
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
        assert [i["iters"] for i in ig] == [i["iters"] for i in ie]
        op.set_graphs(False)
        ux, _ = op.solve(f, tol=1e-10, mixed=mixed)        # eager work in between
        assert torch.equal(ux, ue)
        op.set_graphs(True)


@pytest.mark.parametrize("mixed", [0, 1])
def test_graph_capture_at_second_use_matches_eager(mixed):
    """fl_set_graphs(2): the first solve launches directly, the second
    captures, the later ones replay; every one gives the eager bits."""
    import paper_2103_03658_amd as fl
    op = make_op(2, 1.1, 1, 32)
    f = torch.from_numpy(inputs.uniform_rhs(2, 32, 3, seed=33)).cuda()
    op.set_graphs(0)
    ue, ie = op.solve(f, tol=1e-10, mixed=mixed)
    op.set_graphs(2)
    for rep in range(4):
        ug, ig = op.solve(f, tol=1e-10, mixed=mixed)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
        assert [i["iters"] for i in ig] == [i["iters"] for i in ie]
    with pytest.raises(fl.FlError):
        op.set_graphs(3)


@pytest.mark.parametrize("d,N,fp32", [(1, 64, False), (2, 32, False), (2, 32, True),
                                      (3, 8, False)])
def test_precond_apply_parity(d, N, fp32):
    op = make_op(d, 1.5, 2 if N % 2 == 0 else 1, N)
    op.set_preconditioner(1)
    u = inputs.uniform_rhs(d, N, 2, seed=41)
    ut = torch.from_numpy(u.astype(np.float32) if fp32 else u).cuda()
    y = op.apply_precond(ut).double().cpu().numpy()
    G = orc_gen(d, 1.5, 2 if N % 2 == 0 else 1, N)
    for r in range(2):
        ref = oracle.precond_apply(G, ut[r].double().cpu().numpy())
        tol = 1e-5 if fp32 else 1e-12
        assert np.abs(y[r] - ref).max() <= tol * np.abs(ref).max()


def test_precond_cuts_iterations():
    op = make_op(2, 1.5, 1, 64)
    f = torch.from_numpy(inputs.uniform_rhs(2, 64, 1, seed=4)).cuda()
    op.set_preconditioner(0)
    _, i0 = op.solve(f, tol=1e-10)
    op.set_preconditioner(1)
    _, i1 = op.solve(f, tol=1e-10)
    assert i1[0]["iters"] * 3 < i0[0]["iters"], (i0, i1)


@pytest.mark.parametrize("d,alpha,p,N", [(1, 1.5, 1, 256), (2, 1.0, 2, 64), (2, 1.9, 1, 32),
                                         (3, 0.7, 1, 16)])
def test_fp64_pcg_follows_oracle_pcg(d, alpha, p, N):
    """FP64 preconditioned CG on the GPU takes the oracle's PCG steps: same
    iteration count (within one, for rounding at the threshold) and the same
    iterate to round-off growth."""
    op = make_op(d, alpha, p, N)
    op.set_preconditioner(1)
    f = inputs.uniform_rhs(d, N, 1, seed=12)
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10, mixed=0)
    G = orc_gen(d, alpha, p, N)
    ur, it, rel = oracle.solve_cg(G, f[0], tol=1e-10,
                                  precond=lambda v: oracle.precond_apply(G, v))
    print(f"  gpu iters {info[0]['iters']}, oracle iters {it}")
    assert abs(info[0]["iters"] - it) <= 1
    assert np.abs(u[0].cpu().numpy() - ur).max() <= 1e-8 * np.abs(ur).max()


@pytest.mark.parametrize("d,N,p,fp32", [(1, 64, 1, False), (1, 1024, 1, False), (2, 32, 2, False),
                                        (2, 32, 2, True), (2, 16, 0, False), (3, 8, 1, False),
                                        (3, 16, 2, True), (2, 256, 1, False), (3, 32, 1, False),
                                        (2, 4, 1, False)])
def test_tau_precond_apply_parity(d, N, p, fp32):
    """fl_apply_precond with the tau preconditioner (odd-extended passes)
    against the oracle's dense sine-transform form."""
    op = make_op(d, 1.3, p, N)
    op.set_preconditioner(2)
    u = inputs.uniform_rhs(d, N, 3, seed=43)
    ut = torch.from_numpy(u.astype(np.float32) if fp32 else u).cuda()
    y = op.apply_precond(ut).double().cpu().numpy()
    G = orc_gen(d, 1.3, p, N)
    for r in range(3):
        v = ut[r].double().cpu().numpy()
        ref = oracle.tau_precond_apply(G, v)
        sc = tau_scale(G, v, N, d)
        tol = 1e-5 if fp32 else 1e-12
        assert np.abs(y[r] - ref).max() <= tol * sc, (r, float(np.abs(y[r] - ref).max() / sc))


def tau_scale(G, v, N, d):
    """Rounding of the tau product acts on the magnitudes
    (2/N)^d |S|..(|1/lam| (|S|..|v|)); the largest of them."""
    n = N - 1
    k = np.arange(1, n + 1)
    S = np.abs(np.sin(np.pi * np.outer(k, k) / N))
    inv = 1.0 / np.abs(oracle.tau_symbol(G))
    sc = np.abs(v)
    for ax in range(d):
        sc = np.moveaxis(np.tensordot(S, sc, axes=([1], [ax])), 0, ax)
    sc = sc * inv
    for ax in range(d):
        sc = np.moveaxis(np.tensordot(S, sc, axes=([1], [ax])), 0, ax)
    return sc.max() * (2.0 / N) ** d


@pytest.mark.parametrize("d,N,fp32", [(2, 64, False), (2, 64, True), (3, 16, False),
                                      (2, 512, False), (2, 512, True)])
def test_tau_every_precond_schedule(d, N, fp32):
    """Every schedule the tuner may give the preconditioner's sine passes
    (radix 8/16/32 stages, 1..16 column pairs or line pairs per block,
    ragged last tiles; the bench's 1024-point lines at N = 512) computes the
    same tau product, against the oracle."""
    from paper_2103_03658_amd import tune
    op = make_op(d, 1.2, 1, N)
    u = inputs.uniform_rhs(d, N, 3, seed=47)
    ut = torch.from_numpy(u.astype(np.float32) if fp32 else u).cuda()
    G = orc_gen(d, 1.2, 1, N)
    refs = [oracle.tau_precond_apply(G, ut[r].double().cpu().numpy()) for r in range(3)]
    scs = [tau_scale(G, ut[r].double().cpu().numpy(), N, d) for r in range(3)]
    tol = 1e-5 if fp32 else 1e-12
    base = op.get_schedule(fp32, precond=True)
    tried = 0
    for E, W in tune.candidates(op.M, fp32):
        for ek, wk in (("e_first", "w_first"), ("e_mid", "lpb_mid"), ("e_c2c", "w_c2c")):
            s = dict(base)
            s[ek], s[wk] = E, W
            try:
                op.set_schedule(fp32, precond=True, **s)
            except Exception:
                continue
            y = op.apply_precond(ut).double().cpu().numpy()
            for r in range(3):
                assert np.abs(y[r] - refs[r]).max() <= tol * scs[r], (ek, E, wk, W)
            tried += 1
    assert tried >= 5


@pytest.mark.parametrize("mixed", [0, 1])
def test_precond_schedule_of_its_own_in_solves(mixed):
    """Preconditioned solves whose preconditioner tiles differ from the
    product's (so the r.z partials come in another count) agree with the
    solve on equal schedules."""
    N = 64
    op = make_op(2, 1.3, 1, N)
    f = torch.from_numpy(inputs.uniform_rhs(2, N, 3, seed=12)).cuda()
    fp32 = bool(mixed)
    op.set_schedule(fp32, e_first=8, w_first=4)
    op.set_schedule(fp32, precond=True, e_first=8, w_first=4)
    u0, i0 = op.solve(f, tol=1e-10, mixed=mixed)
    op.set_schedule(fp32, precond=True, e_first=16, w_first=1, e_mid=8, lpb_mid=2)
    u1, i1 = op.solve(f, tol=1e-10, mixed=mixed)
    for a, b in zip(i0, i1):
        assert a["converged"] == 1 and b["converged"] == 1
        assert abs(a["iters"] - b["iters"]) <= 1
    d = (u1 - u0).abs().max().item() / u0.abs().max().item()
    assert d <= 1e-8, d


@pytest.mark.parametrize("d,alpha,p,N", [(1, 1.5, 1, 256), (2, 1.0, 2, 64), (2, 1.9, 1, 32),
                                         (3, 0.7, 1, 16)])
def test_fp64_tau_pcg_follows_oracle(d, alpha, p, N):
    op = make_op(d, alpha, p, N)
    op.set_preconditioner(2)
    f = inputs.uniform_rhs(d, N, 1, seed=12)
    u, info = op.solve(torch.from_numpy(f).cuda(), tol=1e-10, mixed=0)
    G = orc_gen(d, alpha, p, N)
    ur, it, rel = oracle.solve_cg(G, f[0], tol=1e-10,
                                  precond=lambda v: oracle.tau_precond_apply(G, v))
    print(f"  gpu iters {info[0]['iters']}, oracle iters {it}")
    assert abs(info[0]["iters"] - it) <= 1
    assert np.abs(u[0].cpu().numpy() - ur).max() <= 1e-8 * np.abs(ur).max()


def test_tau_cuts_iterations_at_high_alpha():
    op = make_op(2, 1.9, 1, 128)
    f = torch.from_numpy(inputs.uniform_rhs(2, 128, 1, seed=4)).cuda()
    its = {}
    for kind in (1, 2):
        op.set_preconditioner(kind)
        its[kind] = op.solve(f, tol=1e-10)[1][0]["iters"]
    assert its[2] * 3 < its[1], its


@pytest.mark.parametrize("d,N,npass", [(1, 64, 1), (2, 32, 3), (3, 16, 5)])
@pytest.mark.parametrize("kind", [1, 2])
def test_profile_precond_runs_the_preconditioner(d, N, npass, kind):
    """fl_profile_precond times the preconditioner's own kernels (one per
    sine or transform pass) and leaves y = P u, bit for bit as
    fl_apply_precond; with kind 0 it is an error."""
    import paper_2103_03658_amd as fl
    op = make_op(d, 1.1, 1, N)
    op.set_preconditioner(kind)
    u = torch.from_numpy(inputs.uniform_rhs(d, N, 2, seed=8)).cuda()
    y = torch.empty_like(u)
    ms = op.profile_precond(u, out=y, reps=2)
    assert len(ms) == npass and all(m > 0 for m in ms)
    assert torch.equal(y, op.apply_precond(u))
    op.set_preconditioner(0)
    with pytest.raises(fl.FlError):
        op.profile_precond(u, out=y, reps=1)
