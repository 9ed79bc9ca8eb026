"""Pins of the CPU oracle by mathematics rather than printed numbers (CPU).

Independent checks: known constants, the far-field integral and the weight
moments by a different integration (scipy quadrature in cone coordinates),
a brute-force evaluation of the scheme straight from the sum over sign
patterns, the paper's own 2D case list for a_kl, structure (symmetry,
positive definiteness), the identity of the p=0 and p=1 matrices at
alpha = 1 in 1D, and the circulant embedding.
"""

import itertools
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle.constants import c_dalpha, far_field_T
from oracle.weights import weights


def test_c_dalpha_cauchy_values():
    # alpha = 1: c_{d,1} = Gamma((d+1)/2) / pi^{(d+1)/2}
    assert math.isclose(c_dalpha(1, 1.0), 1 / math.pi, rel_tol=1e-15)
    assert math.isclose(c_dalpha(2, 1.0), 1 / (2 * math.pi), rel_tol=1e-15)
    assert math.isclose(c_dalpha(3, 1.0), 1 / math.pi ** 2, rel_tol=1e-15)


@pytest.mark.parametrize("alpha", [0.3, 1.0, 1.7])
@pytest.mark.parametrize("lam", [0.0, 2.0])
def test_far_field_T_cartesian(alpha, lam):
    L = 2.0
    K = (lambda r: math.exp(-lam * r)) if lam else (lambda r: 1.0)
    if lam == 0:
        assert math.isclose(far_field_T(1, alpha), 1 / (alpha * L ** alpha), rel_tol=1e-14)
    else:
        ref = integrate.quad(lambda t: K(t) * t ** (-1 - alpha), L, np.inf,
                             epsrel=1e-13, epsabs=0)[0]
        assert math.isclose(far_field_T(1, alpha, lam=lam), ref, rel_tol=1e-10)
    # 2D: R^2_+ minus [0,L]^2 = {xi1 > L} u {xi1 < L, xi2 > L}
    f2 = lambda y, x: K(math.hypot(x, y)) * (x * x + y * y) ** (-1 - alpha / 2)
    a = integrate.dblquad(f2, L, np.inf, 0, np.inf, epsabs=0, epsrel=1e-11)[0]
    b = integrate.dblquad(f2, 0, L, L, np.inf, epsabs=0, epsrel=1e-11)[0]
    assert math.isclose(far_field_T(2, alpha, lam=lam), a + b, rel_tol=1e-8)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5])
def test_far_field_T3_closed_form(alpha):
    """K = 1, d = 3: integrating the radial tail (cos theta / L)^alpha / alpha
    over the part of the octant where e_3 is largest (times 3 by symmetry)
    leaves 6/(alpha (alpha+1) L^alpha) int_0^{pi/4} (1 - (cos p / sqrt(1 +
    cos^2 p))^{alpha+1}) dp."""
    L = 2.0
    f = lambda p: 1.0 - (math.cos(p) / math.sqrt(1.0 + math.cos(p) ** 2)) ** (alpha + 1)
    ref = 6.0 / (alpha * (alpha + 1) * L ** alpha) * integrate.quad(
        f, 0, math.pi / 4, epsabs=0, epsrel=1e-13)[0]
    assert math.isclose(far_field_T(3, alpha), ref, rel_tol=1e-12)


def _moment_reference(d, alpha, js, L, lam):
    """int_{[0,L]^d} prod xi_s^{j_s} K(|xi|) |xi|^{2-d-alpha} dxi in cone
    coordinates: for the region where xi_t is the largest component,
    xi = r (w, 1)/|(w, 1)| with w in [0,1]^{d-1}, r in [0, L |(w,1)|]."""
    J = sum(js)
    total = 0.0
    for t in range(d):
        others = [s for s in range(d) if s != t]

        def integrand(*w):
            rho = math.sqrt(1.0 + sum(x * x for x in w))
            e = {t: 1.0 / rho}
            for s, x in zip(others, w):
                e[s] = x / rho
            P = 1.0
            for s in range(d):
                P *= e[s] ** js[s]
            R = L * rho
            q = J + 2.0 - alpha            # r^{J} r^{2-d-alpha} r^{d-1}
            if lam:
                # int_0^R r^{q-1} e^{-lam r} dr = Gamma(q) P(q, lam R) / lam^q
                rad = special.gamma(q) * special.gammainc(q, lam * R) / lam ** q
            else:
                rad = R ** q / q
            return P * rad * rho ** (-d)       # dOmega = dw / rho^d
        if d == 2:
            total += integrate.quad(integrand, 0, 1, epsabs=0, epsrel=1e-13)[0]
        else:
            total += integrate.dblquad(lambda y, x: integrand(x, y), 0, 1, 0, 1,
                                       epsabs=0, epsrel=1e-11)[0]
    return total


@pytest.mark.parametrize("d,N", [(1, 16), (2, 8), (3, 4)])
@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("alpha", [0.4, 1.3])
@pytest.mark.parametrize("lam", [0.0, 1.5])
def test_weight_moments(d, N, p, alpha, lam):
    """sum_k omega_k prod_s xi_{k_s}^{j_s} equals the moment of the weight
    function for every j_s <= p (the basis reproduces such polynomials):
    partition of unity for all p, plus linear / quadratic reproduction."""
    L, h = 2.0, 2.0 / N
    om = weights(d, alpha, p, N, h=h, lam=lam)
    xi = h * np.arange(N + 1)
    for js in itertools.product(range(p + 1), repeat=d):
        if d == 1:
            q = js[0] + 2.0 - alpha
            if lam:
                ref = integrate.quad(lambda r: r ** (q - 1) * math.exp(-lam * r), 0, L,
                                     epsabs=0, epsrel=1e-13)[0]
            else:
                ref = L ** q / q
        else:
            ref = _moment_reference(d, alpha, js, L, lam)
        mono = np.ones_like(om)
        for s in range(d):
            shp = [1] * d
            shp[s] = N + 1
            mono = mono * (xi ** js[s]).reshape(shp)
        got = math.fsum((om * mono).ravel())
        assert math.isclose(got, ref, rel_tol=1e-10), (js, got, ref)


def _brute_force_apply(d, W, T, alpha, u, N):
    """(-Delta)_h u at every interior node, summing the sign patterns of the
    reformulated integral one by one: -c [ sum_{k != 0} W_k/|xi_k|^2
    sum_m (u(x_i + (-1)^m o xi_k) - u(x_i)) - 2^d T u_i ], u = 0 outside."""
    h = 2.0 / N
    n = N - 1
    c = c_dalpha(d, alpha)
    U = np.zeros((N + 1,) * d)
    U[(slice(1, N),) * d] = u
    out = np.zeros((n,) * d)
    for i in itertools.product(range(1, N), repeat=d):
        terms = []
        for k in itertools.product(range(N + 1), repeat=d):
            if not any(k):
                continue
            wk = W[k] / (h * h * sum(kk * kk for kk in k))
            for m in itertools.product((1, -1), repeat=d):
                j = tuple(ii + mm * kk for ii, mm, kk in zip(i, m, k))
                inside = all(0 <= jj <= N for jj in j)
                uj = U[j] if inside else 0.0
                terms.append(wk * (uj - U[i]))
        terms.append(-(2 ** d) * T * U[i])
        out[tuple(ii - 1 for ii in i)] = -c * math.fsum(terms)
    return out


@pytest.mark.parametrize("d,N", [(1, 8), (2, 4), (2, 6), (3, 4)])
@pytest.mark.parametrize("p", [1, 2])
def test_brute_force_sign_pattern_sum(d, N, p):
    alpha = 0.8
    G, parts = oracle.generator(d, alpha, p, N, return_parts=True)
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, (N - 1,) * d)
    ref = _brute_force_apply(d, parts["W"], parts["T"], alpha, u, N)
    got = oracle.apply_dense(G, u)
    scale = np.abs(oracle.dense_matrix(G)).sum(axis=1).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale


def test_2d_case_list():
    """The paper's a_kl case list for d = 2 (with reading R3: a_11 carries
    no omega_00 term) against the general-d formula."""
    alpha, p, N = 1.3, 1, 8
    h = 2.0 / N
    G, parts = oracle.generator(2, alpha, p, N, return_parts=True)
    om, T = parts["omega"], parts["T"]
    a = np.zeros_like(om)
    for k in range(N + 1):
        for l in range(N + 1):
            if k == l == 0:
                continue
            r2 = h * h * (k * k + l * l)
            if (k, l) in ((0, 1), (1, 0)):
                a[k, l] = (2 * om[k, l] + om[0, 0]) / r2
            elif k == 0 or l == 0:
                a[k, l] = 2 * om[k, l] / r2
            else:
                a[k, l] = om[k, l] / r2
    a[0, 0] = (-2 * (a[1:, 0].sum() + a[0, 1:].sum()) - 4 * a[1:, 1:].sum() - 4 * T)
    np.testing.assert_allclose(parts["a"], a, rtol=1e-13, atol=0)
    np.testing.assert_allclose(G, -c_dalpha(2, alpha) * a, rtol=1e-13)


@pytest.mark.parametrize("d,N", [(1, 32), (2, 12), (3, 6)])
@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("alpha,lam", [(0.3, 0.0), (1.0, 0.0), (1.9, 0.0), (1.2, 3.0)])
def test_symmetric_positive_definite(d, N, p, alpha, lam):
    G = oracle.generator(d, alpha, p, N, lam=lam)
    A = oracle.dense_matrix(G)
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("N", [16, 64, 256])
def test_p0_equals_p1_at_alpha_one(N):
    """Example 3.2.1: at alpha = 1 the constant and linear bases give the
    same 1D differentiation matrix."""
    G0 = oracle.generator(1, 1.0, 0, N)
    G1 = oracle.generator(1, 1.0, 1, N)
    np.testing.assert_allclose(G0, G1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("d,N,p,M", [(1, 64, 1, None), (2, 16, 2, None), (2, 32, 1, None),
                                     (3, 8, 1, None), (1, 50, 1, 128), (1, 50, 2, 97),
                                     (2, 12, 2, 32), (2, 12, 1, 21), (3, 6, 1, 16), (3, 5, 0, 9)])
def test_circulant_embedding_product(d, N, p, M):
    """The embedded circulant product restricted to the interior equals the
    dense Toeplitz product, for M = 2N and for any M >= 2N - 3 (no
    wrap-around of the offsets -(N-2)..N-2): what a non-power-of-two N
    padded to a power-of-two embedding relies on."""
    G = oracle.generator(d, 0.9, p, N)
    lam, imag = oracle.symbol(G, M)
    assert imag < 1e-13 * np.abs(lam).max()
    M = M or 2 * N
    assert lam.shape == (M,) * d
    n = N - 1
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, (n,) * d)
    z = np.zeros((M,) * d)
    z[(slice(0, n),) * d] = u
    y = np.fft.ifftn(lam * M ** d * np.fft.fftn(z)).real[(slice(0, n),) * d]
    ref = oracle.apply(G, u)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(oracle.dense_matrix(G)).sum(axis=1).max()


def test_embedding_too_short_is_rejected():
    G = oracle.generator(2, 0.9, 1, 12)
    with pytest.raises(ValueError):
        oracle.embed_generator(G, 20)      # 2N - 3 = 21


def test_tempered_reduces_to_fractional():
    for d, N in ((1, 32), (2, 8)):
        G0 = oracle.generator(d, 1.1, 1, N)
        Gt = oracle.generator(d, 1.1, 1, N, lam=1e-9)
        np.testing.assert_allclose(Gt, G0, rtol=1e-7)


def test_bttb_block_product_matches_dense():
    rng = np.random.default_rng(3)
    for d, N in ((2, 20), (3, 8)):
        G = oracle.generator(d, 1.4, 1, N)
        u = rng.uniform(-1, 1, (N - 1,) * d)
        np.testing.assert_allclose(oracle.apply_bttb(G, u), oracle.apply_dense(G, u),
                                   rtol=0, atol=1e-12 * np.abs(G).sum() * 4)


def test_apply_rows_matches_dense():
    rng = np.random.default_rng(4)
    G = oracle.generator(2, 0.7, 2, 16)
    u = rng.uniform(-1, 1, (15, 15))
    y = oracle.apply_dense(G, u)
    rows = np.array([[0, 0], [3, 7], [14, 14], [14, 0]])
    got = oracle.apply_rows(G, u, rows)
    np.testing.assert_allclose(got, y[tuple(rows.T)], rtol=1e-12)


def test_cg_matches_cholesky():
    rng = np.random.default_rng(5)
    G = oracle.generator(2, 1.5, 1, 16)
    f = rng.uniform(-1, 1, (15, 15))
    u1 = oracle.solve_cholesky(G, f)
    u2, it, rel = oracle.solve_cg(G, f, tol=1e-13)
    assert rel <= 1e-13
    assert np.abs(u1 - u2).max() <= 1e-10 * np.abs(u1).max()


@pytest.mark.parametrize("d,N,alpha", [(1, 64, 1.5), (2, 16, 1.5), (2, 16, 0.5), (3, 6, 1.0)])
def test_pcg_matches_cholesky_in_fewer_iterations(d, N, alpha):
    """Preconditioned CG reaches the Cholesky solution, and the circulant
    preconditioner cuts the iteration count of plain CG."""
    rng = np.random.default_rng(6)
    G = oracle.generator(d, alpha, 1, N)
    f = rng.uniform(-1, 1, (N - 1,) * d)
    u1 = oracle.solve_cholesky(G, f)
    u0, it0, _ = oracle.solve_cg(G, f, tol=1e-12)
    u2, it2, rel = oracle.solve_cg(G, f, tol=1e-12,
                                   precond=lambda v: oracle.precond_apply(G, v))
    assert rel <= 1e-12
    assert np.abs(u1 - u2).max() <= 1e-9 * np.abs(u1).max()
    assert it2 < it0


def test_pcg_identity_preconditioner_is_cg():
    """P = I reproduces plain CG step for step."""
    rng = np.random.default_rng(7)
    G = oracle.generator(2, 1.2, 1, 12)
    f = rng.uniform(-1, 1, (11, 11))
    a = oracle.solve_cg(G, f, tol=1e-12)
    b = oracle.solve_cg(G, f, tol=1e-12, precond=lambda v: v.copy())
    assert a[1] == b[1]
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("d,N,M", [(1, 16, None), (2, 8, None), (3, 4, None), (1, 12, 32),
                                   (2, 6, 16)])
def test_precond_fft_matches_dense_circulant_inverse(d, N, M):
    """The FFT form of R C^{-1} R^T against a dense inverse of the dense
    embedding circulant (C_{jk} = c_{(j-k) mod M}), M = 2N or padded."""
    G = oracle.generator(d, 1.3, 1, N)
    c = oracle.embed_generator(G, M)
    lam, _ = oracle.symbol(G, M)
    M = M or 2 * N
    n = N - 1
    idx = np.indices((M,) * d).reshape(d, -1)
    diff = tuple((idx[s][:, None] - idx[s][None, :]) % M for s in range(d))
    C = c[diff]
    rng = np.random.default_rng(8)
    v = rng.uniform(-1, 1, (n,) * d)
    z = np.zeros((M,) * d)
    z[(slice(0, n),) * d] = v
    y = np.linalg.solve(C, z.reshape(-1)).reshape((M,) * d)[(slice(0, n),) * d]
    if lam.min() <= 1e-12 * lam.max():
        pytest.skip("floored symbol: the dense inverse is not the preconditioner")
    np.testing.assert_allclose(oracle.precond_apply(G, v, M=M), y, rtol=1e-10,
                               atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("d,N", [(2, 8), (2, 12), (3, 4), (3, 6)])
@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("lam", [0.0, 1.5])
def test_weights_at_matches_full_lattice(d, N, p, lam):
    """Per-node weights (for sampled checks at large N) equal the whole-lattice
    computation at every node, origin element included."""
    om = weights(d, 0.9, p, N, lam=lam)
    nodes = np.indices((N + 1,) * d).reshape(d, -1).T
    got = oracle.weights_at(d, 0.9, p, N, nodes, lam=lam)
    np.testing.assert_allclose(got, om.reshape(-1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("d,N,p", [(2, 16, 2), (3, 6, 1)])
def test_generator_at_matches_generator(d, N, p):
    G = oracle.generator(d, 1.3, p, N, lam=0.7)
    nodes = np.array([k for k in np.indices((N + 1,) * d).reshape(d, -1).T if k.sum() > 2])
    got = oracle.generator_at(d, 1.3, p, N, nodes, lam=0.7)
    np.testing.assert_allclose(got, G[tuple(nodes.T)], rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        oracle.generator_at(d, 1.3, p, N, np.array([[1] + [0] * (d - 1)]))


@pytest.mark.parametrize("d,N,p,lam", [(1, 64, 1, 0.0), (2, 16, 2, 0.0), (2, 16, 1, 2.0),
                                       (3, 6, 1, 0.0)])
def test_full_stencil_sum_is_far_field(d, N, p, lam):
    """Summing G over the whole symmetric stencil [-N, N]^d leaves only the
    far-field term: c_{d,alpha} 2^d T_d (the scheme annihilates constants
    except for the part of the kernel outside the truncation box)."""
    alpha = 1.1
    G = oracle.generator(d, alpha, p, N, lam=lam)
    k = np.indices((N + 1,) * d).reshape(d, -1).T
    mult = 2.0 ** (d - (k == 0).sum(axis=1))
    total = math.fsum(mult * G.reshape(-1))
    ref = c_dalpha(d, alpha) * 2 ** d * far_field_T(d, alpha, L=2.0, lam=lam)
    scale = np.abs(G).max()
    assert abs(total - ref) <= 1e-12 * scale * len(mult) ** 0.5


def _hankel_tau_1d(t):
    """tau(T) = T - H from the definition: H_{ij} = t_{i+j+2} (first row
    t_2 .. t_{n-1}, 0, 0) plus its persymmetric image t_{2n-i-j} (last row
    0, 0, t_{n-1} .. t_2), 0-based indices, t_k = 0 for k > n - 1."""
    n = len(t)
    T = np.array([[t[abs(i - j)] for j in range(n)] for i in range(n)])
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i + j + 2 <= n - 1:
                H[i, j] += t[i + j + 2]
            if 2 * n - i - j <= n - 1:
                H[i, j] += t[2 * n - i - j]
    return T - H


@pytest.mark.parametrize("alpha,p,N", [(0.5, 1, 16), (1.5, 2, 16), (1.9, 0, 16), (1.2, 1, 12),
                                       (0.7, 2, 10), (1.6, 1, 21)])
def test_tau_symbol_1d_is_spectrum_of_t_minus_hankel(alpha, p, N):
    """Any N, also where 2N is not a power of two (the GPU's mixed-radix
    sine passes are checked against this oracle form there)."""
    G = oracle.generator(1, alpha, p, N)
    n = N - 1
    tau = _hankel_tau_1d(G[:n])
    lam = oracle.tau_symbol(G)
    k = np.arange(1, n + 1)
    S = np.sin(np.pi * np.outer(k, k) / N) * np.sqrt(2.0 / N)   # orthogonal
    np.testing.assert_allclose(S @ np.diag(lam) @ S, tau, atol=1e-12 * np.abs(tau).max())
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(tau)), np.sort(lam),
                               rtol=1e-11, atol=1e-12 * lam.max())


@pytest.mark.parametrize("N,shape", [(8, None), (6, None), (10, (9, 4)), (12, (5, 11))])
def test_tau_symbol_2d_is_spectrum_of_tensor_tau(N, shape):
    """2-level: tau(T) = sum_ab t_ab tau(B_a) (x) tau(B_b), B_a the Toeplitz
    basis matrix of offset a (size n_s of its axis), built densely; its
    eigen-decomposition in the 2D sine basis has the oracle's eigenvalues.
    Cubes and boxes, 2N a power of two or not."""
    alpha = 1.2
    G = oracle.generator(2, alpha, 1, N)
    n0, n1 = shape if shape else (N - 1, N - 1)

    def basis(n):
        out = []
        for a in range(n):
            e = np.zeros(n)
            e[a] = 1.0
            out.append(_hankel_tau_1d(e))
        return out

    t0, t1 = basis(n0), basis(n1)
    tau = sum(G[a, b] * np.kron(t0[a], t1[b]) for a in range(n0) for b in range(n1))

    def sine(n):
        k = np.arange(1, n + 1)
        return np.sin(np.pi * np.outer(k, k) / (n + 1)) * np.sqrt(2.0 / (n + 1))

    S2 = np.kron(sine(n0), sine(n1))
    lam = oracle.tau_symbol(G, (n0, n1)).reshape(-1)
    np.testing.assert_allclose(S2 @ np.diag(lam) @ S2, tau, atol=1e-12 * np.abs(tau).max())


@pytest.mark.parametrize("d,N", [(1, 32), (2, 16), (3, 8)])
def test_tau_precond_inverts_tau(d, N):
    G = oracle.generator(d, 1.3, 1, N)
    n = N - 1
    rng = np.random.default_rng(2)
    v = rng.uniform(-1, 1, (n,) * d)
    z = oracle.tau_precond_apply(G, v)
    # apply tau(T) to z through its spectrum with an independent FFT-free path:
    # tau(T) z = (2/N)^d S (lam * S z)
    lam = oracle.tau_symbol(G)
    k = np.arange(1, n + 1)
    S = np.sin(np.pi * np.outer(k, k) / N)
    y = z
    for ax in range(d):
        y = np.moveaxis(np.tensordot(S, y, axes=([1], [ax])), 0, ax)
    y = y * lam
    for ax in range(d):
        y = np.moveaxis(np.tensordot(S, y, axes=([1], [ax])), 0, ax)
    np.testing.assert_allclose(y * (2.0 / N) ** d, v, atol=1e-10)


@pytest.mark.parametrize("d,N,alpha", [(1, 64, 1.5), (2, 16, 1.9), (2, 32, 1.0), (3, 8, 1.5)])
def test_tau_pcg_matches_cholesky(d, N, alpha):
    rng = np.random.default_rng(9)
    G = oracle.generator(d, alpha, 1, N)
    f = rng.uniform(-1, 1, (N - 1,) * d)
    u1 = oracle.solve_cholesky(G, f)
    u2, it, rel = oracle.solve_cg(G, f, tol=1e-12,
                                  precond=lambda v: oracle.tau_precond_apply(G, v))
    assert rel <= 1e-12
    assert np.abs(u1 - u2).max() <= 1e-9 * np.abs(u1).max()
    _, it_emb, _ = oracle.solve_cg(G, f, tol=1e-12,
                                   precond=lambda v: oracle.precond_apply(G, v))
    assert it <= it_emb + 1


@pytest.mark.parametrize("d,N", [(1, 24), (2, 12), (3, 6)])
def test_tau_symbol_cosine_series_equals_sine_quotient(d, N):
    """The cosine-series eigenvalues equal (S..S c) / prod sin(theta), c the
    Hankel-corrected first column, evaluated with dense sine matrices."""
    G = oracle.generator(d, 0.8, 1, N, lam=1.0)
    n = N - 1
    c = G[(slice(0, n),) * d].copy()
    for ax in range(d):
        a = [slice(None)] * d
        b = [slice(None)] * d
        a[ax] = slice(0, n - 2)
        b[ax] = slice(2, n)
        c2 = c.copy()
        c2[tuple(a)] -= c[tuple(b)]
        c = c2
    k = np.arange(1, n + 1)
    S = np.sin(np.pi * np.outer(k, k) / N)
    y = c
    for ax in range(d):
        y = np.moveaxis(np.tensordot(S, y, axes=([1], [ax])), 0, ax)
    den = np.ones((n,) * d)
    for ax in range(d):
        shp = [1] * d
        shp[ax] = n
        den = den * S[:, 0].reshape(shp)
    lam = oracle.tau_symbol(G)
    np.testing.assert_allclose(lam, y / den, rtol=1e-10, atol=1e-12 * np.abs(lam).max())


def test_gamma_two_is_the_default_scheme():
    for d, p, N in ((1, 2, 16), (2, 1, 8)):
        assert np.array_equal(oracle.generator(d, 0.7, p, N),
                              oracle.generator(d, 0.7, p, N, gamma=2.0))


@pytest.mark.parametrize("d,N", [(1, 16), (2, 8)])
@pytest.mark.parametrize("p", [0, 1, 2])
def test_weight_moments_gamma(d, N, p):
    """sum_k omega_k xi_k^j equals the moment of |xi|^{gamma-d-alpha} for
    gamma = 1 + alpha/2 (omega_0 included)."""
    alpha = 1.2
    gamma = 1.0 + alpha / 2
    L, h = 2.0, 2.0 / N
    om = weights(d, alpha, p, N, h=h, gamma=gamma)
    xi = h * np.arange(N + 1)
    for js in itertools.product(range(p + 1), repeat=d):
        J = sum(js)
        if d == 1:
            q = J + gamma - alpha
            ref = L ** q / q
        else:
            # cone coordinates as in _moment_reference, radial power J + gamma - alpha
            total = 0.0
            for t in range(d):
                def integrand(w):
                    rho = math.sqrt(1.0 + w * w)
                    e = [0.0, 0.0]
                    e[t] = 1.0 / rho
                    e[1 - t] = w / rho
                    P = e[0] ** js[0] * e[1] ** js[1]
                    qq = J + gamma - alpha
                    return P * (L * rho) ** qq / qq * rho ** (-2)
                total += integrate.quad(integrand, 0, 1, epsabs=0, epsrel=1e-13)[0]
            ref = total
        mono = np.ones_like(om)
        for s in range(d):
            shp = [1] * d
            shp[s] = N + 1
            mono = mono * (xi ** js[s]).reshape(shp)
        got = math.fsum((om * mono).ravel())
        assert math.isclose(got, ref, rel_tol=1e-10), (js, got, ref)


@pytest.mark.parametrize("d,N", [(1, 8), (2, 4)])
@pytest.mark.parametrize("p", [1, 2])
def test_gamma_brute_force_sign_pattern_sum(d, N, p):
    """gamma < 2: the scheme summed sign pattern by sign pattern with
    Phi = second difference / |xi|^gamma and no origin term."""
    alpha, gamma = 0.8, 1.5
    G, parts = oracle.generator(d, alpha, p, N, return_parts=True, gamma=gamma)
    om, T = parts["omega"], parts["T"]
    h = 2.0 / N
    c = c_dalpha(d, alpha)
    rng = np.random.default_rng(8)
    u = rng.uniform(-1, 1, (N - 1,) * d)
    U = np.zeros((N + 1,) * d)
    U[(slice(1, N),) * d] = u
    ref = np.zeros((N - 1,) * d)
    for i in itertools.product(range(1, N), repeat=d):
        terms = []
        for k in itertools.product(range(N + 1), repeat=d):
            if not any(k):
                continue
            wk = om[k] / (h * math.sqrt(sum(kk * kk for kk in k))) ** gamma
            for m in itertools.product((1, -1), repeat=d):
                j = tuple(ii + mm * kk for ii, mm, kk in zip(i, m, k))
                uj = U[j] if all(0 <= jj <= N for jj in j) else 0.0
                terms.append(wk * (uj - U[i]))
        terms.append(-(2 ** d) * T * U[i])
        ref[tuple(ii - 1 for ii in i)] = -c * math.fsum(terms)
    got = oracle.apply_dense(G, u)
    scale = np.abs(oracle.dense_matrix(G)).sum(axis=1).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("alpha", [0.6, 1.0, 1.5])
@pytest.mark.parametrize("p", [0, 1, 2])
def test_gamma_convergence_rate(alpha, p):
    """gamma = 1 + alpha/2: the error of the product on u = (1-x^2)_+^{2.1+alpha}
    decays like h^{2-alpha} for phi^0 and phi^1, as Sec. 3.1 states.  For
    phi^2 the scheme as written (Phi(x, 0) = 0, no origin term) also gives
    h^{2-alpha}: near xi = 0, Phi(x, xi) ~ u''(x) xi^{2-gamma} is not smooth,
    and its interpolation error on the first element limits every degree."""
    from oracle import exact
    gamma = 1.0 + alpha / 2
    s = 2.1 + alpha
    errs = []
    for N in (64, 128, 256):
        G = oracle.generator(1, alpha, p, N, gamma=gamma)
        x = oracle.grid_points(N)
        y = oracle.apply(G, (1 - x * x) ** s)
        errs.append(np.abs(y - exact.frac_lap_ball_power(x * x, s, alpha, 1)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - (2.0 - alpha)) <= 0.05 for r in rates), rates


# ---------------------------------------------------------------------------
# boxes (Sec. 2.2: Upsilon = [0, L]^d with L the longest side, N_s <= N
# intervals on axis s): the cube's generator on the box's interior points
# ---------------------------------------------------------------------------

BOXES = [(2, 12, (11, 5)), (2, 8, (3, 7)), (3, 6, (5, 2, 4)), (1, 10, (6,))]


@pytest.mark.parametrize("d,N,shape", BOXES)
def test_box_matrix_is_cube_matrix_restricted(d, N, shape):
    """The box occupies the first n_s interior points of each axis of the
    cube's grid (axis s spans (-1, -1 + N_s h)), so its matrix is the cube's
    restricted to those rows and columns."""
    G = oracle.generator(d, 1.1, 1, N)
    A = oracle.dense_matrix(G)
    n = N - 1
    sel = np.ravel_multi_index(np.indices(shape).reshape(d, -1), (n,) * d)
    np.testing.assert_array_equal(oracle.dense_matrix(G, shape), A[np.ix_(sel, sel)])
    assert np.linalg.eigvalsh(oracle.dense_matrix(G, shape)).min() > 0.0


@pytest.mark.parametrize("d,N,shape", BOXES)
def test_box_products_agree(d, N, shape):
    """Box products: materialised, block form, sampled rows and the per-axis
    padded circulant embedding all give the same y."""
    G = oracle.generator(d, 0.7, 2, N)
    rng = np.random.default_rng(4)
    u = rng.uniform(-1, 1, shape)
    y = oracle.apply_dense(G, u)
    np.testing.assert_allclose(oracle.apply_bttb(G, u), y, atol=1e-13 * np.abs(y).max())
    rows = np.array([[0] * d, [s - 1 for s in shape]])
    np.testing.assert_allclose(oracle.apply_rows(G, u, rows), y[tuple(rows.T)],
                               atol=1e-13 * np.abs(y).max())
    intervals = tuple(s + 1 for s in shape)
    for M in (None, tuple(max(8, 1 << (2 * i - 1).bit_length()) for i in intervals)):
        lam, _ = oracle.symbol(G, M, intervals)
        z = np.zeros(lam.shape)
        z[tuple(slice(0, s) for s in shape)] = u
        yf = np.fft.ifftn(lam * lam.size * np.fft.fftn(z)).real[tuple(slice(0, s) for s in shape)]
        np.testing.assert_allclose(yf, y, atol=1e-13 * np.abs(G).sum() * np.abs(u).max())


def test_box_tau_is_tensor_tau_2d():
    """2-level tau on a box: sum_ab t_ab tau_{n0}(B_a) (x) tau_{n1}(B_b), built
    densely; tau_precond_apply inverts it."""
    N, shape = 10, (9, 5)
    G = oracle.generator(2, 1.3, 1, N)
    n0, n1 = shape

    def basis(n):
        out = []
        for a in range(n):
            e = np.zeros(n)
            e[a] = 1.0
            out.append(_hankel_tau_1d(e))
        return out

    t0, t1 = basis(n0), basis(n1)
    tau = sum(G[a, b] * np.kron(t0[a], t1[b]) for a in range(n0) for b in range(n1))
    v = np.random.default_rng(6).uniform(-1, 1, shape)
    z = oracle.tau_precond_apply(G, v)
    np.testing.assert_allclose(tau @ z.reshape(-1), v.reshape(-1), atol=1e-10)


@pytest.mark.parametrize("d,N,shape", BOXES)
def test_box_pcg_matches_cholesky(d, N, shape):
    G = oracle.generator(d, 1.4, 1, N)
    f = np.random.default_rng(11).uniform(-1, 1, shape)
    uc = oracle.solve_cholesky(G, f)
    for P in (lambda v: oracle.tau_precond_apply(G, v), lambda v: oracle.precond_apply(G, v)):
        u, it, rel = oracle.solve_cg(G, f, tol=1e-12, precond=P)
        assert rel <= 1e-12
        assert np.abs(u - uc).max() <= 1e-9 * np.abs(uc).max()
