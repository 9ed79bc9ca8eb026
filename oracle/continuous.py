"""The continuous nonlocal operator of Remark 2.2 in 1D, by adaptive quadrature
(test infrastructure; see package header).

    L u(x) = c_{1,alpha} int_R (u(x) - u(y)) K(|x - y|) |x - y|^{-1-alpha} dy

with the normalisation c-bar = c_{1,alpha} (reading R6); K = 1 is the
fractional Laplacian (definition (fL-nD)), K(r) = exp(-lambda r) the tempered
operator of Example 3.2.2.  Folding y = x - xi and y = x + xi together,

    L u(x) = c int_0^inf D(x, xi) K(xi) xi^{1-alpha} d xi,
    D(x, xi) = (2 u(x) - u(x + xi) - u(x - xi)) / xi^2,

where D stays bounded as xi -> 0 (it tends to -u''(x)).  Each test function
supplies D in a form that does not cancel at small xi, and the points where
D has a kink.  The weight xi^{1-alpha} is integrated on the first piece by
QUADPACK's rule for algebraic end-point singularities.

Used for the right-hand side of Example 3.2.2 (u = (1 - x^2)_+^2, whose
tempered f the paper does not print) and for the consistency pins of the
tempered weights.
"""

import math

import numpy as np
from scipy import integrate

from .constants import c_dalpha


class BumpSquared:
    """u(x) = (1 - x^2)_+^2 (Example 3.2.2's exact solution)."""

    @staticmethod
    def value(x):
        x = np.asarray(x, dtype=np.float64)
        return np.maximum(1.0 - x * x, 0.0) ** 2

    @staticmethod
    def D(x, xi):
        # While x -+ xi both stay in the support, u is the quartic
        # 1 - 2x^2 + x^4 there and its even Taylor terms give exactly
        # u(x+xi) + u(x-xi) - 2u(x) = u''(x) xi^2 + 2 xi^4, u'' = 12x^2 - 4.
        # Beyond that, xi >= 1 - |x| and the direct quotient does not cancel.
        if abs(x) < 1.0 and xi <= 1.0 - abs(x):   # also the limit xi -> 0
            return (4.0 - 12.0 * x * x) - 2.0 * xi * xi
        val = 2.0 * (1.0 - x * x) ** 2 if abs(x) < 1.0 else 0.0
        for y in (x + xi, x - xi):
            if abs(y) < 1.0:
                val -= (1.0 - y * y) ** 2
        return val / (xi * xi)

    @staticmethod
    def kinks(x):
        return sorted({1.0 - abs(x), 1.0 + abs(x)})


class Gaussian:
    """u(x) = exp(-x^2)."""

    @staticmethod
    def value(x):
        return np.exp(-np.asarray(x, dtype=np.float64) ** 2)

    @staticmethod
    def D(x, xi):
        # 2 - e^{-xi^2}(e^{2 x xi} + e^{-2 x xi}) = -2 [e^{-xi^2} 2 sinh^2(x xi) + expm1(-xi^2)]
        if xi == 0.0:
            return (2.0 - 4.0 * x * x) * math.exp(-x * x)   # -u''(x)
        if xi > 1.0:   # no cancellation left
            return (2.0 * math.exp(-x * x) - math.exp(-(x + xi) ** 2)
                    - math.exp(-(x - xi) ** 2)) / (xi * xi)
        s = math.sinh(x * xi)
        return -2.0 * math.exp(-x * x) * (math.exp(-xi * xi) * 2.0 * s * s
                                          + math.expm1(-xi * xi)) / (xi * xi)

    @staticmethod
    def kinks(x):
        return [1.0]


def _quad(func, a, b, **kw):
    """scipy's QUADPACK call that fails loudly on a poor error estimate.

    QUADPACK flags round-off whenever its estimate reaches the FP64 noise
    floor (at points where L u crosses zero, say), so its warning is not
    used; the estimate itself must stay below 1e-12 (values are O(1))."""
    out = integrate.quad(func, a, b, epsabs=1e-15, epsrel=1e-12, full_output=1, **kw)
    val, err = out[0], out[1]
    if not err <= 1e-12 * max(1.0, abs(val)):
        raise ArithmeticError(f"quadrature on [{a}, {b}] estimates error {err:.3e}")
    return val


def nonlocal_1d(u, x, alpha, K):
    """L u at the points x for the kernel K (a callable of r >= 0).

    u: a test-function class above.  Accuracy about 1e-12 absolute on O(1)
    values (each piece's QUADPACK estimate is checked)."""
    c = c_dalpha(1, alpha)
    out = np.empty(len(x))
    for i, xi0 in enumerate(np.asarray(x, dtype=np.float64)):
        xi0 = float(xi0)
        br = [b for b in u.kinks(xi0) if b > 0.0]
        f = lambda t: u.D(xi0, t) * K(t)
        total = _quad(f, 0.0, br[0], weight="alg", wvar=(1.0 - alpha, 0.0), limit=200)
        g = lambda t: u.D(xi0, t) * K(t) * t ** (1.0 - alpha)
        for a, b in zip(br[:-1], br[1:]):
            total += _quad(g, a, b, limit=200)
        total += _quad(g, br[-1], np.inf, limit=400)
        out[i] = c * total
    return out


def tempered_kernel(lam):
    """K(r) = exp(-lam r)."""
    return lambda r: math.exp(-lam * r)
