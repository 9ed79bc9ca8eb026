"""Weight integrals omega_k^p (test infrastructure; see package header).

Definition (Sec. 2.1 eq. (wi-1D); Sec. 2.2 eq. (2D-scheme0); Remark 2.2):

    omega_k^p = int_{[0,L]^d} phi_k(xi) K(|xi|) |xi|^{gamma-d-alpha} d xi,

phi_k the tensor-product Lagrange basis of degree p on the xi-lattice
xi_k = k h, k in {0..N}^d, gamma = 2 (reading R5), K = 1 (fractional
Laplacian) or K(r) = exp(-lambda r) (tempered, Remark 2.2).

Bases (Appendix): p = 0 the indicator of [xi_{k-1/2}, xi_{k+1/2}] cut to
[0, L]; p = 1 hats on [xi_k, xi_{k+1}]; p = 2 quadratic Lagrange on the
elements [xi_{2m}, xi_{2m+2}] (N even).

1D: the integrals are evaluated exactly: each basis function is a polynomial on
each element, and int_a^b xi^{j+s-1} dxi (or its tempered counterpart, an
incomplete gamma function) is taken in mpmath at 50 digits, which removes the
cancellation of the Appendix closed forms in FP64.  Reading R1: the Appendix
p=2 formulas are replaced by the exact integral of the quadratic basis.

2D/3D: the paper computes them by quadrature without naming the rule.  Here:
tensor Gauss-Legendre on every element that avoids the origin (the integrand
is analytic there), and on the element touching the origin a Duffy split into
d pyramids xi = r (.., 1, ..) with Gauss-Jacobi in r for the weight r^{1-alpha}
(Jacobian r^{d-1} times |xi|^{2-d-alpha}) and Gauss-Legendre in the remaining
cone coordinates.
"""

import itertools
import math

import mpmath
import numpy as np
from scipy.special import roots_jacobi


# ---------------------------------------------------------------------------
# element structure on the lattice xi = 0..N (lattice units)
# ---------------------------------------------------------------------------

def _elements_1d(p, N):
    """List of (lo, hi, [(node, poly coefficients low->high in xi)])."""
    out = []
    if p == 0:
        for k in range(N + 1):
            lo, hi = max(k - 0.5, 0.0), min(k + 0.5, float(N))
            out.append((lo, hi, [(k, [1.0])]))
    elif p == 1:
        for e in range(N):
            out.append((float(e), float(e + 1),
                        [(e, [float(e + 1), -1.0]), (e + 1, [-float(e), 1.0])]))
    elif p == 2:
        if N % 2:
            raise ValueError("p = 2 needs an even N")
        for m in range(N // 2):
            nodes = [2 * m, 2 * m + 1, 2 * m + 2]
            basis = []
            for a in range(3):
                others = [nodes[b] for b in range(3) if b != a]
                den = float((nodes[a] - others[0]) * (nodes[a] - others[1]))
                # (xi - o0)(xi - o1) = xi^2 - (o0+o1) xi + o0 o1
                coef = [others[0] * others[1] / den,
                        -(others[0] + others[1]) / den, 1.0 / den]
                basis.append((nodes[a], coef))
            out.append((float(2 * m), float(2 * m + 2), basis))
    else:
        raise ValueError("p must be 0, 1 or 2")
    return out


def _weights_1d(alpha, p, N, h, lam, gamma=2.0):
    """Exact 1D weights in mpmath, returned as float64 (length N+1)."""
    with mpmath.workdps(50):
        s0 = mpmath.mpf(gamma) - mpmath.mpf(alpha)   # sigma_0 = gamma - alpha
        lam_l = mpmath.mpf(lam) * mpmath.mpf(h)   # kernel rate in lattice units

        def moment(j, a, b):
            # int_a^b t^{j + s0 - 1} K(h t) dt in lattice units
            s = s0 + j
            a, b = mpmath.mpf(a), mpmath.mpf(b)
            if lam == 0:
                return (b ** s - a ** s) / s
            return lam_l ** (-s) * mpmath.gammainc(s, lam_l * a, lam_l * b)

        om = [mpmath.mpf(0)] * (N + 1)
        for lo, hi, basis in _elements_1d(p, N):
            for node, coef in basis:
                om[node] += sum(mpmath.mpf(c) * moment(j, lo, hi)
                                for j, c in enumerate(coef) if c != 0)
        scale = mpmath.mpf(h) ** s0
        return np.array([float(w * scale) for w in om])


# ---------------------------------------------------------------------------
# 2D / 3D by quadrature
# ---------------------------------------------------------------------------

def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _poly_eval(coef, x):
    return sum(c * x ** j for j, c in enumerate(coef))


def _dim_tables(p, N, Q):
    """Per-element 1D quadrature tables: positions X[e,q], weighted basis
    WB[e,a,q] = w_q * (hi-lo)/2 * phi_a(X[e,q]), first node index of e, step."""
    els = _elements_1d(p, N)
    x, w = _gl(Q)
    nb = len(els[0][2])
    E = len(els)
    X = np.empty((E, Q))
    WB = np.empty((E, nb, Q))
    first = np.empty(E, dtype=np.int64)
    for e, (lo, hi, basis) in enumerate(els):
        X[e] = lo + (hi - lo) * (x + 1.0) / 2.0
        for a, (node, coef) in enumerate(basis):
            WB[e, a] = w * (hi - lo) / 2.0 * _poly_eval(coef, X[e])
        first[e] = basis[0][0]
    return X, WB, first, els


def _origin_element(d, alpha, p, h, lam, els, nr=24, nt=40, gamma=2.0):
    """Local integrals over the element touching xi = 0 (lattice units):
    I[a_1..a_d] = int_{[0,H]^d} prod_j phi_{a_j}(xi_j) g(xi) dxi,
    g(xi) = K(h|xi|) |xi|^{gamma-d-alpha}, via d Duffy pyramids."""
    lo, H, basis = els[0]
    assert lo == 0.0
    nb = len(basis)
    # Gauss-Jacobi on [0,H] with weight r^{gamma-alpha-1}: r = H(1+x)/2
    xj, wj = roots_jacobi(nr, 0.0, gamma - alpha - 1.0)
    r = H * (1.0 + xj) / 2.0
    wr = wj * (H / 2.0) ** (gamma - alpha)
    xt, wt = _gl(nt)
    t = (xt + 1.0) / 2.0
    wt = wt / 2.0
    I = np.zeros((nb,) * d)
    # cone coordinates t_j in [0,1]^{d-1}
    if d == 2:
        T = [t]
        WT = wt
    else:
        T = [np.repeat(t, nt), np.tile(t, nt)]
        WT = np.repeat(wt, nt) * np.tile(wt, nt)
    rho = np.sqrt(1.0 + sum(tt ** 2 for tt in T))
    for s in range(d):                          # pyramid where xi_s is largest
        # xi coordinates at every (r, t) point: shape (nr, nT)
        coords = []
        ti = 0
        for j in range(d):
            if j == s:
                coords.append(np.outer(r, np.ones_like(rho)))
            else:
                coords.append(np.outer(r, T[ti]))
                ti += 1
        R = np.outer(r, rho)
        kern = np.exp(-lam * h * R) if lam else 1.0
        g = kern * rho[None, :] ** (gamma - d - alpha)   # r^{gamma-alpha-1} in weight
        wgt = np.outer(wr, WT) * g
        vals = [[_poly_eval(coef, coords[j]) for (_, coef) in basis]
                for j in range(d)]
        for idx in np.ndindex(*(nb,) * d):
            prod = wgt.copy()
            for j in range(d):
                prod = prod * vals[j][idx[j]]
            I[idx] += prod.sum()
    return I


def _weights_nd(d, alpha, p, N, h, lam, Q=None, gamma=2.0):
    if Q is None:
        Q = 20 if d == 2 else 14
    X, WB, first, els = _dim_tables(p, N, Q)
    E, nb = WB.shape[0], WB.shape[1]
    step = 2 if p == 2 else 1
    ex = gamma - d - alpha

    def g_of(r2):
        r = np.sqrt(r2)
        out = r ** ex
        if lam:
            out = out * np.exp(-lam * h * r)
        return out

    om = np.zeros((N + 1,) * d)
    if d == 2:
        X2 = X ** 2
        for e1 in range(E):
            # G[e2, q1, q2]
            G = g_of(X2[e1][None, :, None] + X2[:, None, :])
            if e1 == 0:
                G[0] = 0.0            # origin element handled separately
            I = np.einsum('jqr,aq,jbr->jab', G, WB[e1], WB)
            for a in range(nb):
                for b in range(nb):
                    om[first[e1] + a, b: b + step * E: step] += I[:, a, b]
    elif d == 3:
        X2 = X ** 2
        for e1 in range(E):
            for e2 in range(E):
                G = g_of(X2[e1][None, :, None, None] + X2[e2][None, None, :, None]
                         + X2[:, None, None, :])
                if e1 == 0 and e2 == 0:
                    G[0] = 0.0
                I = np.einsum('kqrs,aq,br,kcs->kabc', G, WB[e1], WB[e2], WB)
                for a in range(nb):
                    for b in range(nb):
                        for c in range(nb):
                            om[first[e1] + a, first[e2] + b,
                               c: c + step * E: step] += I[:, a, b, c]
    else:
        raise ValueError("d must be 2 or 3 here")
    I0 = _origin_element(d, alpha, p, h, lam, els, gamma=gamma)
    for idx in np.ndindex(*(nb,) * d):
        om[tuple(first[0] + i for i in idx)] += I0[idx]
    return om * h ** (gamma - alpha)


def weights_at(d, alpha, p, N, nodes, h=None, lam=0.0, Q=None, gamma=2.0):
    """omega^p_k at selected multi-indices `nodes` (integer array (m, d)),
    d = 2 or 3, by the same element quadrature as weights(): the sum over
    the elements touching node k of int phi_k g.  For sampled checks at
    sizes where the whole lattice is out of reach."""
    if h is None:
        h = 2.0 / N
    if Q is None:
        Q = 20 if d == 2 else 14
    X, WB, first, els = _dim_tables(p, N, Q)
    E, nb = WB.shape[0], WB.shape[1]
    ex = gamma - d - alpha
    I0 = _origin_element(d, alpha, p, h, lam, els, gamma=gamma)
    X2 = X ** 2
    out = np.zeros(len(nodes))
    for m, k in enumerate(np.asarray(nodes, dtype=np.int64)):
        # per axis: the (element, local basis index) pairs whose node is k_s
        per = [[(e, a) for e in range(E) for a in range(nb) if first[e] + a == k[s]]
               for s in range(d)]
        total = 0.0
        for combo in itertools.product(*per):
            es = [e for e, _ in combo]
            if all(e == 0 for e in es):
                total += I0[tuple(a for _, a in combo)]
                continue
            r2 = X2[es[0]][:, None] + X2[es[1]][None, :]
            if d == 3:
                r2 = r2[:, :, None] + X2[es[2]][None, None, :]
            r = np.sqrt(r2)
            g = r ** ex
            if lam:
                g = g * np.exp(-lam * h * r)
            wb = [WB[e, a] for e, a in combo]
            if d == 2:
                total += np.einsum("qr,q,r->", g, wb[0], wb[1])
            else:
                total += np.einsum("qrs,q,r,s->", g, wb[0], wb[1], wb[2])
        out[m] = total
    return out * h ** (gamma - alpha)


def weights(d, alpha, p, N, h=None, lam=0.0, Q=None, gamma=2.0):
    """omega^p_k for k in {0..N}^d as an FP64 array of shape (N+1,)*d, with
    the splitting parameter gamma in (alpha, 2] (weight |xi|^{gamma-d-alpha}).

    h defaults to L/N with L = 2 (Omega = (-1,1)^d)."""
    if h is None:
        h = 2.0 / N
    if p == 2 and N % 2:
        raise ValueError("p = 2 needs an even N")
    if not (alpha < gamma <= 2.0):
        raise ValueError("gamma must lie in (alpha, 2]")
    if d == 1:
        return _weights_1d(alpha, p, N, h, lam, gamma=gamma)
    return _weights_nd(d, alpha, p, N, h, lam, Q=Q, gamma=gamma)
