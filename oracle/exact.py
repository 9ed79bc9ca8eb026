"""Closed forms of the continuous operator used as pins (test infrastructure).

* (1-|x|^2)_+^s on the unit ball: for |x| < 1
    (-Delta)^{alpha/2} u = 2^alpha Gamma((d+alpha)/2) Gamma(s+1)
                            / (Gamma(d/2) Gamma(s+1-alpha/2))
                            * 2F1((d+alpha)/2, alpha/2 - s; d/2; |x|^2).
  For d = 1 this is eq. (fun0) (Example 3.2.1); for s = alpha/2 it is the
  constant K_d(alpha) = 2^alpha Gamma(1+alpha/2) Gamma((d+alpha)/2)/Gamma(d/2).
* Gaussian exp(-|x|^2):
    (-Delta)^{alpha/2} u = 2^alpha Gamma((d+alpha)/2)/Gamma(d/2)
                            * 1F1((d+alpha)/2; d/2; -|x|^2)
  (Example 3.2.3 prints the d = 2 case).
* u = 1/(1+x^2) in 1D (Example 3.1.3): from the Fourier transform
  pi exp(-|k|) and the symbol |k|^alpha (definition (pseudo)),
    (-Delta)^{alpha/2} u = Gamma(1+alpha) cos((1+alpha) arctan x)
                            / (1+x^2)^{(1+alpha)/2}.
* Benchmark solution of Example 3.2.1 (f = 1, g = 0):
    u = (1-x^2)_+^{alpha/2} / Gamma(1+alpha)   (printed with a wrong sign; the
  constant K_1(alpha) = Gamma(1+alpha) fixes it as +).
"""

import math

import numpy as np
from scipy.special import hyp2f1, hyp1f1


def frac_lap_ball_power(x2, s, alpha, d):
    """(-Delta)^{alpha/2} (1-|x|^2)_+^s at |x|^2 = x2 < 1."""
    x2 = np.asarray(x2, dtype=np.float64)
    pref = (2.0 ** alpha * math.gamma((d + alpha) / 2.0) * math.gamma(s + 1.0)
            / (math.gamma(d / 2.0) * math.gamma(s + 1.0 - alpha / 2.0)))
    return pref * hyp2f1((d + alpha) / 2.0, alpha / 2.0 - s, d / 2.0, x2)


def frac_lap_gaussian(x2, alpha, d):
    """(-Delta)^{alpha/2} exp(-|x|^2) at |x|^2 = x2."""
    x2 = np.asarray(x2, dtype=np.float64)
    return (2.0 ** alpha * math.gamma((d + alpha) / 2.0) / math.gamma(d / 2.0)
            * hyp1f1((d + alpha) / 2.0, d / 2.0, -x2))


def frac_lap_cauchy_1d(x, alpha):
    """(-Delta)^{alpha/2} 1/(1+x^2) in 1D."""
    x = np.asarray(x, dtype=np.float64)
    return (math.gamma(1.0 + alpha) * np.cos((1.0 + alpha) * np.arctan(x))
            / (1.0 + x * x) ** ((1.0 + alpha) / 2.0))


def benchmark_solution_1d(x, alpha):
    """Solution of (-Delta)^{alpha/2} u = 1 on (-1,1), u = 0 outside."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(1.0 - x * x, 0.0) ** (alpha / 2.0) / math.gamma(1.0 + alpha)
