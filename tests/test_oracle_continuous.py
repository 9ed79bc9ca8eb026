"""Pins of the continuous 1D operator (oracle.continuous) and, through it, of
the tempered weights (Remark 2.2, reading R6) beyond the lambda -> 0 limit.

* K = 1: the real-space quadrature reproduces the closed forms of
  (-Delta)^{alpha/2} for (1 - x^2)_+^2 (eq. (fun0) family) and exp(-x^2).
* K = exp(-lambda r): it reproduces the Fourier side.  The operator's symbol
  is 2 c int_0^inf (1 - cos k xi) e^{-lambda xi} xi^{-1-alpha} d xi, which is
  2 c Gamma(-alpha) [lambda^alpha - (lambda^2 + k^2)^{alpha/2} cos(alpha atan(k/lambda))]
  for alpha != 1 (the regularised Laplace transform of xi^{-1-alpha}), and
  2 c [k atan(k/lambda) - (lambda/2) log(1 + k^2/lambda^2)] for alpha = 1
  (integrate d/dk = atan(k/lambda) from 0).  Applied to the Gaussian
  (transform sqrt(pi) e^{-k^2/4}) by a quadrature over k.
* The tempered scheme is consistent with that operator: for u = (1-x^2)_+^2
  (C^{1,1} at the boundary) the product error falls like h^{2-alpha}
  (reached from below by N = 1024), which a
  wrong rate scaling or a far-field constant without K would stop at O(1).
* Example 3.2.2: the tempered solve with u = (1-x^2)_+^2 converges at second
  order, with errors insensitive to lambda (the paper's figure; no printed
  numbers, so the rate and the lambda ratio are the pins).
"""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import continuous as C
from oracle import exact
from oracle.constants import c_dalpha

X = np.array([0.0, 0.3, -0.55, 0.77, -0.95, 0.998046875])


@pytest.mark.parametrize("alpha", [0.3, 0.6, 1.0, 1.5, 1.9])
def test_fractional_bump_closed_form(alpha):
    v = C.nonlocal_1d(C.BumpSquared, X, alpha, lambda r: 1.0)
    ref = exact.frac_lap_ball_power(X * X, 2.0, alpha, 1)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [0.4, 1.0, 1.7])
def test_fractional_gaussian_closed_form(alpha):
    x = np.array([0.0, 0.5, 1.2, 2.5])
    v = C.nonlocal_1d(C.Gaussian, x, alpha, lambda r: 1.0)
    ref = exact.frac_lap_gaussian(x * x, alpha, 1)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()


def tempered_symbol(k, alpha, lam):
    c = c_dalpha(1, alpha)
    if alpha == 1.0:
        return 2.0 * c * (k * math.atan(k / lam) - 0.5 * lam * math.log1p((k / lam) ** 2))
    return 2.0 * c * math.gamma(-alpha) * (
        lam ** alpha - (lam * lam + k * k) ** (alpha / 2.0) * math.cos(alpha * math.atan(k / lam)))


def fourier_side(x, alpha, lam):
    return np.array([integrate.quad(
        lambda k: math.sqrt(math.pi) * math.exp(-k * k / 4.0) * tempered_symbol(k, alpha, lam)
        * math.cos(k * x0), 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=200)[0] / math.pi
        for x0 in x])


@pytest.mark.parametrize("alpha", [0.2, 0.6, 1.0, 1.5, 1.9])
@pytest.mark.parametrize("lam", [0.5, 1.0, 3.0])
def test_tempered_gaussian_fourier_side(alpha, lam):
    x = np.array([0.0, 0.4, 1.3])
    v = C.nonlocal_1d(C.Gaussian, x, alpha, C.tempered_kernel(lam))
    ref = fourier_side(x, alpha, lam)
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tempered_symbol_limits():
    # lambda -> 0 gives |k|^alpha (the normalisation c_{1,alpha}); the alpha = 1
    # form is the limit of the general one
    for alpha in (0.5, 1.0, 1.5):
        assert abs(tempered_symbol(2.0, alpha, 1e-16) - 2.0 ** alpha) <= 1e-7
    s1 = tempered_symbol(1.7, 1.0, 0.8)
    assert abs(tempered_symbol(1.7, 1.0 + 1e-7, 0.8) - s1) <= 1e-6 * s1


@pytest.mark.parametrize("alpha", [0.6, 1.0])
@pytest.mark.parametrize("lam", [0.5, 3.0])
def test_tempered_scheme_consistency(alpha, lam):
    errs = []
    for N in (256, 512, 1024):
        x = oracle.grid_points(N)
        G = oracle.generator(1, alpha, 1, N, lam=lam)
        f = C.nonlocal_1d(C.BumpSquared, x, alpha, C.tempered_kernel(lam))
        errs.append(np.abs(oracle.apply(G, C.BumpSquared.value(x)) - f).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # the rate approaches 2 - alpha from below (more slowly for larger lambda)
    assert errs[-1] <= 5e-5
    assert rates[0] <= rates[1] + 0.02 and rates[1] >= 2.0 - alpha - 0.15, (errs, rates)


def example_3_2_2_errors(alpha, lam, Ns):
    out = []
    for N in Ns:
        x = oracle.grid_points(N)
        G = oracle.generator(1, alpha, 1, N, lam=lam)
        f = C.nonlocal_1d(C.BumpSquared, x, alpha, C.tempered_kernel(lam))
        out.append(np.abs(oracle.solve_cholesky(G, f) - C.BumpSquared.value(x)).max())
    return out


@pytest.mark.parametrize("alpha", [0.6, 1.0, 1.5])
def test_example_3_2_2_second_order_and_lambda_insensitive(alpha):
    e = {lam: example_3_2_2_errors(alpha, lam, (64, 128, 256)) for lam in (0.5, 1.0)}
    for lam, errs in e.items():
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(1.85 <= r <= 2.5 for r in rates), (lam, errs, rates)
    ratio = [a / b for a, b in zip(e[0.5], e[1.0])]
    assert all(1.0 / 2.5 <= q <= 2.5 for q in ratio), ratio


# ---------------------------------------------------------------------------
# sums of exponentials (Remark 2.2 with K(r) = sum c_i exp(-lambda_i r))
# ---------------------------------------------------------------------------

TERMS = [(0.5, 0.0), (0.3, 1.0), (0.2, 4.0)]


def expsum_kernel(terms):
    return lambda r: sum(c * math.exp(-lam * r) for c, lam in terms)


@pytest.mark.parametrize("d,p,N", [(1, 1, 32), (1, 2, 16), (2, 1, 8), (2, 2, 8)])
def test_expsum_reductions(d, p, N):
    """One term is the fractional or tempered generator; equal rates add."""
    G0 = oracle.generator(d, 1.1, p, N)
    G1 = oracle.generator(d, 1.1, p, N, lam=1.5)
    assert np.array_equal(oracle.generator_expsum(d, 1.1, p, N, [(1.0, 0.0)]), G0)
    assert np.array_equal(oracle.generator_expsum(d, 1.1, p, N, [(1.0, 1.5)]), G1)
    G2 = oracle.generator_expsum(d, 1.1, p, N, [(0.25, 1.5), (0.75, 1.5)])
    assert np.abs(G2 - G1).max() <= 1e-14 * np.abs(G1).max()
    G3 = oracle.generator_expsum(d, 1.1, p, N, [(2.0, 0.0), (3.0, 1.5)])
    assert np.abs(G3 - (2.0 * G0 + 3.0 * G1)).max() <= 1e-14 * np.abs(G3).max()


@pytest.mark.parametrize("alpha,Ns", [(0.6, (256, 512)), (1.0, (256, 512, 1024))])
def test_expsum_scheme_consistency(alpha, Ns):
    """The scheme with a three-term kernel converges to the continuous operator
    with that K at the rate 2 - alpha of the one-term kernels."""
    K = expsum_kernel(TERMS)
    errs = []
    for N in Ns:
        x = oracle.grid_points(N)
        G = oracle.generator_expsum(1, alpha, 1, N, TERMS)
        f = C.nonlocal_1d(C.BumpSquared, x, alpha, K)
        errs.append(np.abs(oracle.apply(G, C.BumpSquared.value(x)) - f).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(Ns) - 1)]
    assert errs[-1] <= 5e-5
    assert rates[-1] >= 2.0 - alpha - 0.15, (errs, rates)


def test_expsum_solve_second_order():
    alpha = 1.2
    K = expsum_kernel(TERMS)
    errs = []
    for N in (64, 128, 256):
        x = oracle.grid_points(N)
        G = oracle.generator_expsum(1, alpha, 1, N, TERMS)
        f = C.nonlocal_1d(C.BumpSquared, x, alpha, K)
        errs.append(np.abs(oracle.solve_cholesky(G, f) - C.BumpSquared.value(x)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 <= r <= 2.5 for r in rates), (errs, rates)
