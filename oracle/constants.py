"""Scalar constants of the scheme (test infrastructure; see package header).

c_{d,alpha}: the normalisation constant of the hypersingular-integral form of
(-Delta)^{alpha/2} (Sec. 1, definition (fL-nD) and the constant beneath it).

T_d: the far-field integral  int_{Upsilon^c_+} K(|xi|) |xi|^{-d-alpha} d xi,
with Upsilon = [0, L]^d and Upsilon^c_+ = R^d_+ minus Upsilon (Sec. 2,
eq. (FL30) and (L2)); K = 1 for the fractional Laplacian and
K(r) = exp(-lambda r) for the tempered operator (Remark 2.2).  It multiplies
-2^d u(x) in (L2) and therefore enters the diagonal coefficient a_0
(Sec. 2.1: a_0 = -2(sum a_j + 1/(alpha L^alpha)); Sec. 2.2: the last term of
a_00).  In 1D with K = 1 it is the paper's 1/(alpha L^alpha).
"""

import functools
import math

import mpmath


def c_dalpha(d, alpha):
    """c_{d,alpha} = 2^{alpha-1} alpha Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1-alpha/2))."""
    return (2.0 ** (alpha - 1.0) * alpha * math.gamma((d + alpha) / 2.0)
            / (math.pi ** (d / 2.0) * math.gamma(1.0 - alpha / 2.0)))


def K_ball(d, alpha):
    """Value of (-Delta)^{alpha/2} (1-|x|^2)_+^{alpha/2} inside the unit ball.

    2^alpha Gamma(1+alpha/2) Gamma((d+alpha)/2) / Gamma(d/2); for d=1 this is
    eq. (fun0) at s = alpha/2 (where 2F1 with a zero parameter is 1)."""
    return (2.0 ** alpha * math.gamma(1.0 + alpha / 2.0)
            * math.gamma((d + alpha) / 2.0) / math.gamma(d / 2.0))


def _radial_tail(R, alpha, lam):
    """F(R) = int_R^inf K(r) r^{-1-alpha} dr as an mpmath number."""
    R = mpmath.mpf(R)
    if lam == 0:
        return R ** (-alpha) / alpha
    lam = mpmath.mpf(lam)
    # int_R^inf e^{-lam r} r^{-1-alpha} dr = lam^alpha Gamma(-alpha, lam R)
    return lam ** alpha * mpmath.gammainc(-alpha, lam * R)


@functools.lru_cache(maxsize=None)   # pure function of its arguments; slow in 3D
def far_field_T(d, alpha, L=2.0, lam=0.0, dps=30):
    """T_d = int over R^d_+ \\ [0,L]^d of K(|xi|) |xi|^{-d-alpha} d xi.

    Polar form: the boundary of [0,L]^d in direction e (a unit vector of the
    positive orthant) is at r = L / max_s e_s, so
    T_d = int_{orthant of S^{d-1}} F(L / max_s e_s) dOmega(e),
    F(R) = int_R^inf K(r) r^{-1-alpha} dr.  Evaluated with mpmath.quad.
    """
    alpha = float(alpha)
    with mpmath.workdps(dps):
        a = mpmath.mpf(alpha)
        if d == 1:
            val = _radial_tail(L, a, lam)
        elif d == 2:
            # theta in [0, pi/2]; max(cos, sin) = cos on [0, pi/4]; symmetric.
            f = lambda th: _radial_tail(L / mpmath.cos(th), a, lam)
            val = 2 * mpmath.quad(f, [0, mpmath.pi / 4])
        elif d == 3:
            # Region where e_3 = cos(theta) is the largest component, times 3;
            # within it, phi in [0, pi/2] is symmetric about pi/4.
            def inner(ph):
                tmax = mpmath.atan(1 / mpmath.cos(ph))
                g = lambda th: _radial_tail(L / mpmath.cos(th), a, lam) * mpmath.sin(th)
                return mpmath.quad(g, [0, tmax])
            val = 6 * mpmath.quad(inner, [0, mpmath.pi / 4])
        else:
            raise ValueError("d must be 1, 2 or 3")
        return float(val)
