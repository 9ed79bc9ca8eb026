"""Coefficients, generator, dense operator and exterior-data term
(test infrastructure; see package header).

Notation follows Sec. 2: lattice x_i = -1 + i h (Omega = (-1,1)^d, L = 2,
h = L/N), interior indices i in {1..N-1}^d (n = N-1 unknowns per axis; nodes
with a component 0 or N carry u = g, as in the sums for b in eq. (1D-scheme)
and (2D-scheme)), offsets k in {0..N}^d, xi_k = h k.

Scheme, written for general d (Sec. 2.1 eq. (L1h), (1D-scheme); Sec. 2.2
eq. (2D-scheme); the 3D case is said to follow the 2D lines):

  (-Delta)_h u_i = -c_{d,alpha} [ a_0 u_i + sum_{k != 0, |k_s| <= N} a_{|k|} u_{i+k} + (far field of g) ]

  a_k = 2^{z(k)} W_k / |xi_k|^gamma          (k != 0, z(k) = # zero entries)
  a_0 = - sum_{k != 0} 2^{d - z(k)} a_k - 2^d T_d

W is omega with the origin value redistributed (origin_rule).  The factor
2^{z(k)} counts the sign patterns m of (FL1) that land on the same lattice
neighbour; 2^{d-z(k)} counts the distinct neighbours with offset pattern |k|,
each of which subtracts u_i once per sign pattern.  For d = 1 this is the
paper's a_1 = (zeta omega_0 + omega_1)/xi_1^gamma, a_j = omega_j/xi_j^gamma,
a_0 = -2 (sum a_j + 1/(alpha L^alpha)); for d = 2 it is the case list under
(2D-scheme) with reading R3 for the origin.

The matrix on the interior unknowns is A = [G_{|i-j|}] with G = -c a
(symmetric Toeplitz A^(1), BTTB A^(2), and the 3-level analogue).
"""

import math

import numpy as np
from scipy.linalg import toeplitz

from .constants import c_dalpha, far_field_T
from .weights import weights as _weights

GAMMA = 2.0


def grid_points(N, d=1):
    """Interior coordinates x_i = -1 + i h, i = 1..N-1 (one axis)."""
    h = 2.0 / N
    return -1.0 + h * np.arange(1, N)


def origin_rule(om, d, p, gamma=2.0):
    """Redistribute omega_0 (the weight of Phi(x, 0), a limit) to the axis
    offsets.  gamma = 2: Phi(x, 0) = u''-type limit, replaced by the average
    over axes s of Phi(x, h e_s) (p <= 1; the paper's 1D rule
    Phi(x, xi_0) ~ Phi(x, xi_1), reading R3 in 2D) or of the Richardson
    combination (4 Phi(x, h e_s) - Phi(x, 2h e_s))/3 (p = 2, readings R2, R4).
    """
    W = np.array(om, dtype=np.float64, copy=True)
    zero = (0,) * d
    w0 = W[zero]
    W[zero] = 0.0
    if gamma < 2.0:
        # gamma < 2: Phi(x, 0) = 0 (eq. (gamma2)), the origin weight drops out
        return W
    c1, c2 = (1.0, 0.0) if p <= 1 else (4.0 / 3.0, -1.0 / 3.0)
    for s in range(d):
        e1 = tuple(1 if j == s else 0 for j in range(d))
        e2 = tuple(2 if j == s else 0 for j in range(d))
        W[e1] += w0 * c1 / d
        if c2:
            W[e2] += w0 * c2 / d
    return W


def _offset_tables(N, d):
    k = np.indices((N + 1,) * d).reshape(d, -1).T          # all offsets
    z = (k == 0).sum(axis=1)
    norm = np.sqrt((k.astype(np.float64) ** 2).sum(axis=1))
    return k, z, norm


def coefficients(W, d, h, T, gamma=GAMMA):
    """a_k for k in {0..N}^d from the origin-corrected weights W."""
    N = W.shape[0] - 1
    k, z, norm = _offset_tables(N, d)
    Wf = W.reshape(-1)
    a = np.zeros_like(Wf)
    nz = norm > 0
    a[nz] = (2.0 ** z[nz]) * Wf[nz] / (h * norm[nz]) ** gamma
    # a_0: compensated sum over all neighbours, then the far field
    terms = list((2.0 ** (d - z[nz])) * a[nz])
    a[~nz] = -math.fsum(terms) - (2.0 ** d) * T
    return a.reshape(W.shape)


def generator(d, alpha, p, N, lam=0.0, return_parts=False, gamma=2.0):
    """G_k = -c_{d,alpha} a_k on {0..N}^d (FP64).

    lam > 0 selects the tempered kernel exp(-lam r) (Remark 2.2, reading R6:
    same normalisation constant c_{d,alpha}).  gamma in (alpha, 2] is the
    splitting parameter (Sec. 2.1: Phi = second difference / |xi|^gamma;
    gamma < 2 has no origin term)."""
    h = 2.0 / N
    om = _weights(d, alpha, p, N, h=h, lam=lam, gamma=gamma)
    W = origin_rule(om, d, p, gamma=gamma)
    T = far_field_T(d, alpha, L=2.0, lam=lam)
    a = coefficients(W, d, h, T, gamma=gamma)
    G = -c_dalpha(d, alpha) * a
    if return_parts:
        return G, dict(omega=om, W=W, T=T, a=a)
    return G


def generator_expsum(d, alpha, p, N, terms, gamma=2.0):
    """G_k = -c_{d,alpha} a_k for K(r) = sum_i c_i exp(-lambda_i r), terms = [(c_i, lambda_i)].

    Remark 2.2: K enters mu_gamma, hence only the weight integrals omega_k,
    and the far-field constant T of a_0; both are integrals against K, so
    they are the c_i-weighted sums of the one-exponential ones (lambda_i = 0
    is K = 1).  The origin rule and a_k, a_0 are then formed once, as for
    any kernel."""
    h = 2.0 / N
    om = sum(c * _weights(d, alpha, p, N, h=h, lam=lam, gamma=gamma) for c, lam in terms)
    T = sum(c * far_field_T(d, alpha, L=2.0, lam=lam) for c, lam in terms)
    W = origin_rule(om, d, p, gamma=gamma)
    a = coefficients(W, d, h, T, gamma=gamma)
    return -c_dalpha(d, alpha) * a


def generator_at(d, alpha, p, N, nodes, lam=0.0):
    """G_k = -c_{d,alpha} 2^{z(k)} omega_k / |xi_k|^2 at selected offsets
    away from the origin correction (every node with |k|_1 > 2), d = 2, 3;
    the same definitions as generator(), for sampled checks at large N."""
    from .weights import weights_at
    nodes = np.asarray(nodes, dtype=np.int64)
    if (np.abs(nodes).sum(axis=1) <= 2).any():
        raise ValueError("generator_at: offsets with |k|_1 <= 2 carry origin corrections")
    h = 2.0 / N
    om = weights_at(d, alpha, p, N, nodes, h=h, lam=lam)
    z = (nodes == 0).sum(axis=1)
    norm2 = (h * h) * (nodes.astype(np.float64) ** 2).sum(axis=1)
    return -c_dalpha(d, alpha) * (2.0 ** z) * om / norm2 ** (GAMMA / 2.0)


# ---------------------------------------------------------------------------
# dense operator
# ---------------------------------------------------------------------------

def grid_shape(G, shape=None):
    """Interior points per axis: n = N-1 on every axis of the cube, or the
    given box shape (Sec. 2.2: the weights live on Upsilon = [0, L]^d with L
    the longest side, so a box with N_s <= N intervals on axis s uses the
    cube's generator on its own n_s = N_s - 1 interior points)."""
    d = G.ndim
    n = G.shape[0] - 2
    if shape is None:
        return (n,) * d
    shape = tuple(int(v) for v in shape)
    if len(shape) != d or min(shape) < 1 or max(shape) > n:
        raise ValueError("box shape must give 1 <= n_s <= N - 1 on each axis")
    return shape


def dense_matrix(G, shape=None):
    """Materialise A_{ij} = G_{|i-j|} on the interior grid (n = N-1 per axis,
    or the box `shape`)."""
    d = G.ndim
    shp = grid_shape(G, shape)
    idx = np.indices(shp).reshape(d, -1)
    diff = [np.abs(idx[s][:, None] - idx[s][None, :]) for s in range(d)]
    return G[tuple(diff)]


def apply_dense(G, u):
    """y = A u with A materialised (small grids); the grid is u's first d
    axes (the cube's or a box's), trailing axes are right-hand sides."""
    d = G.ndim
    shp = u.shape
    A = dense_matrix(G, shp[:d])
    ub = u.reshape((-1,) + shp[d:]) if u.ndim > d else u.reshape(-1)
    return (A @ ub).reshape(shp)


def apply_bttb(G, u):
    """y = A u without an FFT: y[i0] = sum_{j0} A_{|i0-j0|} u[j0], each
    block applied as a dense (d-1)-level Toeplitz product.  O(n^{2d}).  The
    grid is u's shape (the cube's or a box's)."""
    d = G.ndim
    shp = grid_shape(G, u.shape)
    n0 = shp[0]
    if d == 1:
        T = toeplitz(G[:n0])
        return T @ u
    if d == 2:
        # y[i0] = sum_m ( Z_m[i0 - m] + Z_m[i0 + m] ), Z_m[j0] = T_m u[j0],
        # T_m[i1, j1] = G[m, |i1 - j1|] (symmetric Toeplitz block)
        n1 = shp[1]
        y = np.zeros(shp)
        for m in range(n0):
            Z = u @ toeplitz(G[m, :n1])
            y[m:] += Z[:n0 - m]
            if m:
                y[:n0 - m] += Z[m:]
        return y
    if d == 3:
        y = np.zeros(shp)
        rest = shp[1] * shp[2]
        # V[m, j0] = A2(G[m]) u[j0]
        A2 = [dense_matrix(G[m], shp[1:]) for m in range(n0)]
        U = u.reshape(n0, rest)
        V = np.stack([U @ A2[m].T for m in range(n0)])   # (m, j0, n1 n2)
        for i0 in range(n0):
            m = np.abs(i0 - np.arange(n0))
            y[i0] = V[m, np.arange(n0)].sum(axis=0).reshape(shp[1:])
        return y
    raise ValueError("d must be 1, 2 or 3")


def apply(G, u):
    """Dense product, materialised when small, block form otherwise (grid:
    u's first d axes)."""
    if int(np.prod(u.shape[:G.ndim])) <= 4096:
        return apply_dense(G, u)
    return apply_bttb(G, u)


def apply_rows(G, u, rows):
    """Exact y_i = sum_j G_{|i-j|} u_j at selected interior multi-indices
    `rows` (array (m, d)), each by a compensated sum.  For sampled parity at
    sizes where the full product is out of reach."""
    d = G.ndim
    idx = np.indices(grid_shape(G, u.shape)).reshape(d, -1)
    uf = u.reshape(-1)
    out = np.empty(len(rows))
    for r, i in enumerate(rows):
        coef = G[tuple(np.abs(idx[s] - i[s]) for s in range(d))]
        out[r] = math.fsum(coef * uf)
    return out


# ---------------------------------------------------------------------------
# circulant embedding (what a fast product computes)
# ---------------------------------------------------------------------------

def embed_generator(G, M=None, intervals=None):
    """c on prod {0..M_s-1}: c[j] = G[m(j)], m(j_s) = min(j_s, M_s - j_s),
    zero wherever some m(j_s) > N_s - 2 (reading R7).  N_s: intervals of
    axis s (N for the cube; a box's axes, Sec. 2.2); M_s = 2 N_s unless
    given (an int for every axis, or one per axis).  The interior product
    uses offsets -(N_s-2)..N_s-2 only, so any M_s >= 2 N_s - 3 keeps them
    apart (no wrap-around) and gives the same restricted product."""
    d = G.ndim
    N = G.shape[0] - 1
    Ns = (N,) * d if intervals is None else tuple(int(v) for v in intervals)
    if len(Ns) != d or max(Ns) > N or min(Ns) < 2:
        raise ValueError("intervals must give 2 <= N_s <= N on each axis")
    if M is None:
        Ms = tuple(2 * v for v in Ns)
    elif np.ndim(M) == 0:
        Ms = (int(M),) * d
    else:
        Ms = tuple(int(v) for v in M)
    if any(Ms[s] < 2 * Ns[s] - 3 for s in range(d)):
        raise ValueError("embedding length M_s must be >= 2 N_s - 3")
    ms, keeps = [], []
    for s in range(d):
        j = np.arange(Ms[s])
        m = np.minimum(j, Ms[s] - j)
        ms.append(np.minimum(m, N))            # entries with m > N_s - 2 are zeroed below
        keeps.append(m <= Ns[s] - 2)
    c = G[np.ix_(*ms)].copy()
    mask = keeps[0]
    for s in range(1, d):
        mask = np.multiply.outer(mask, keeps[s])
    c[~mask] = 0.0
    return c


def symbol(G, M=None, intervals=None):
    """lambda-hat = DFT_M(c) / prod M_s, real part (c is real and even)."""
    c = embed_generator(G, M, intervals)
    lam = np.fft.fftn(c)
    return lam.real / c.size, float(np.abs(lam.imag).max() / c.size)


def precond_apply(G, v, floor_rel=1e-12, M=None):
    """y = R C^{-1} R^T v: the preconditioner the solver uses (not part of
    the paper, whose solver is unspecified).  C is the circulant embedding of
    A (symbol lambda-hat) of length M per axis (an int or one per axis; 2 N_s
    unless given, N_s = n_s + 1 for the grid of v), floored at floor_rel *
    max lambda-hat so that it is positive definite; R restricts to the
    interior grid of v."""
    d = G.ndim
    shp = grid_shape(G, v.shape)
    intervals = tuple(n + 1 for n in shp)
    if M is None:
        M = tuple(2 * i for i in intervals)
    lam, _ = symbol(G, M, intervals)
    Ms = lam.shape
    lam = np.maximum(lam, floor_rel * lam.max())
    z = np.zeros(Ms)
    z[tuple(slice(0, n) for n in shp)] = v
    y = np.fft.ifftn(np.fft.fftn(z) / (lam * np.prod(Ms))).real
    return y[tuple(slice(0, n) for n in shp)]


# ---------------------------------------------------------------------------
# exterior data g != 0 (the b term of the paper)
# ---------------------------------------------------------------------------

def tau_symbol(G, shape=None):
    """Eigenvalues of the natural tau approximation of the multilevel Toeplitz
    matrix A (entries G_{|i-j|}): tau(T) = T - H(T) on every level, H(T) the
    Hankel matrix with first row (t_2, ..., t_{n-1}, 0, 0) and last row its
    reverse.  tau(T) is diagonalised by the sine transform S_{jk} =
    sin(pi j k / (n+1)), j, k = 1..n, on each axis; with its first column
    c = t - (t shifted by two) on each level the eigenvalues are
    (S..S c)(k) / prod_s sin(theta_{k_s}), theta_k = pi k / (n+1), which
    telescopes (U_j - U_{j-2} = 2 cos(j theta) for the Chebyshev quotients
    U_j = sin((j+1) theta) / sin(theta)) into the truncated cosine series
        lam(k) = sum_{j in [0, n-1]^d} t_j prod_s w(j_s) cos(j_s theta_{k_s}),
    w(0) = 1, w(j) = 2; summed in this form (dense cosine matrices), which
    keeps its accuracy near theta = 0 and pi where the sine quotient loses
    digits.  Shape (n,)*d, or the box `shape` (n_s per axis, sine transform
    of length n_s + 1 on axis s)."""
    d = G.ndim
    shp = grid_shape(G, shape)
    t = np.array(G[tuple(slice(0, n) for n in shp)], dtype=np.float64)
    y = t
    for ax in range(d):
        n = shp[ax]
        k = np.arange(1, n + 1)
        j = np.arange(n)
        C = np.cos(np.pi * np.outer(k, j) / (n + 1)) * np.where(j == 0, 1.0, 2.0)[None, :]
        y = np.moveaxis(np.tensordot(C, y, axes=([1], [ax])), 0, ax)
    return y


def tau_precond_apply(G, v, floor_rel=1e-12):
    """tau(T)^{-1} v = prod_s (2/(n_s+1)) S..S diag(1/lam) S..S v with the
    dense sine matrices (S_s^2 = (n_s+1)/2 I) on v's grid (the cube's or a
    box's); lam floored at floor_rel * max lam."""
    d = G.ndim
    shp = grid_shape(G, v.shape)
    lam = tau_symbol(G, shp)
    lam = np.maximum(lam, floor_rel * lam.max())
    Ss = []
    for n in shp:
        k = np.arange(1, n + 1)
        Ss.append(np.sin(np.pi * np.outer(k, k) / (n + 1)))
    y = np.array(v, dtype=np.float64)
    for ax in range(d):
        y = np.moveaxis(np.tensordot(Ss[ax], y, axes=([1], [ax])), 0, ax)
    y = y / lam
    for ax in range(d):
        y = np.moveaxis(np.tensordot(Ss[ax], y, axes=([1], [ax])), 0, ax)
    return y * np.prod([2.0 / (n + 1) for n in shp])


def exterior_lattice_1d(G, g, intervals=None):
    """Lattice part of bold-b_i: sum over exterior nodes j (j <= 0 or j >= N_0,
    |j - i| <= N) of G_{|j-i|} g(x_j), x_j = -1 + j h (eq. (1D-scheme)); N_0 =
    intervals[0] intervals (N by default)."""
    N = G.shape[0] - 1
    Na = N if intervals is None else intervals[0]
    h = 2.0 / N
    out = np.zeros(Na - 1)
    for i in range(1, Na):
        s = 0.0
        for j in list(range(i - N, 1)) + list(range(Na, i + N + 1)):
            s += G[abs(j - i)] * g(-1.0 + j * h)
        out[i - 1] = s
    return out


def far_field_tail_1d(N, g, alpha, lam=0.0):
    """tail_i = int_L^inf [g(x_i - xi) + g(x_i + xi)] K(xi) xi^{-1-alpha} dxi,
    L = 2: the far-field integrals of bold-b_i (eq. (L2h))."""
    from scipy.integrate import quad
    h = 2.0 / N
    L = 2.0
    out = np.zeros(N - 1)
    for i in range(1, N):
        xi = -1.0 + i * h
        f = lambda t: (g(xi - t) + g(xi + t)) * t ** (-1.0 - alpha) * (
            math.exp(-lam * t) if lam else 1.0)
        out[i - 1] = quad(f, L, np.inf, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    return out


def exterior_b_1d(G, g, alpha, lam=0.0):
    """bold-b_i = lattice sum - c_{1,alpha} tail_i (eq. (1D-scheme) and the
    definition of b_i)."""
    N = G.shape[0] - 1
    return exterior_lattice_1d(G, g) - c_dalpha(1, alpha) * far_field_tail_1d(N, g, alpha, lam)


def exterior_lattice_2d(G, g, intervals=None):
    """Lattice part of bold-b_ij (eq. (2D-scheme)): for every interior node,
    the sum of G_{|k|} g(x_{i+k}) over the offsets k in [-N, N]^2 whose node
    i + k is outside the interior.  g must accept numpy arrays (x1, x2).
    intervals = (N_0, N_1) for a box (Sec. 2.2), the cube by default."""
    N = G.shape[0] - 1
    Na = (N, N) if intervals is None else tuple(intervals)
    nodes = [(i, jj) for i in range(1, Na[0]) for jj in range(1, Na[1])]
    return exterior_lattice_2d_at(G, g, nodes, Na).reshape(Na[0] - 1, Na[1] - 1)


def exterior_lattice_2d_at(G, g, nodes, intervals=None):
    """exterior_lattice_2d at the listed interior nodes (i, j), 1 <= i < N_0,
    1 <= j < N_1."""
    N = G.shape[0] - 1
    Na = (N, N) if intervals is None else tuple(intervals)
    h = 2.0 / N
    k = np.arange(-N, N + 1)
    Gs = G[np.abs(k)[:, None], np.abs(k)[None, :]]        # symmetric stencil
    out = np.zeros(len(nodes))
    for t, (i, jj) in enumerate(nodes):
        a0 = i + k
        a1 = jj + k
        inside = (((a0 >= 1) & (a0 <= Na[0] - 1))[:, None]
                  & ((a1 >= 1) & (a1 <= Na[1] - 1))[None, :])
        vals = g((-1.0 + a0 * h)[:, None], (-1.0 + a1 * h)[None, :])
        out[t] = math.fsum((Gs * vals)[~inside].ravel())
    return out


def exterior_lattice_3d(G, g, intervals=None):
    """Lattice part of the exterior-data term in 3D (the 2D definition of
    bold-b_ij, eq. (2D-scheme), taken over three axes: reading R4): for every
    interior node, the sum of G_{|k|} g(x_{i+k}) over the offsets k in
    [-N, N]^3 whose node i + k is outside the interior.  g must accept numpy
    arrays (x1, x2, x3).  intervals = (N_0, N_1, N_2) for a box."""
    N = G.shape[0] - 1
    Na = (N, N, N) if intervals is None else tuple(intervals)
    h = 2.0 / N
    k = np.arange(-N, N + 1)
    ak = np.abs(k)
    Gs = G[ak[:, None, None], ak[None, :, None], ak[None, None, :]]
    out = np.zeros(tuple(v - 1 for v in Na))
    for i0 in range(1, Na[0]):
        a0 = i0 + k
        in0 = (a0 >= 1) & (a0 <= Na[0] - 1)
        for i1 in range(1, Na[1]):
            a1 = i1 + k
            in1 = (a1 >= 1) & (a1 <= Na[1] - 1)
            for i2 in range(1, Na[2]):
                a2 = i2 + k
                in2 = (a2 >= 1) & (a2 <= Na[2] - 1)
                inside = in0[:, None, None] & in1[None, :, None] & in2[None, None, :]
                vals = g((-1.0 + a0 * h)[:, None, None], (-1.0 + a1 * h)[None, :, None],
                         (-1.0 + a2 * h)[None, None, :])
                out[i0 - 1, i1 - 1, i2 - 1] = math.fsum((Gs * vals)[~inside].ravel())
    return out


def far_field_tail_2d(N, g, alpha, nq=160):
    """tail_ij = sum_m int_{Upsilon^c_+} g(x + (-1)^m o xi) |xi|^{-2-alpha} dxi
    (the far-field integrals of bold-b_ij).  The region is split into
    {xi1 > L, xi2 < L}, {xi1 > L, xi2 > L}, {xi1 < L, xi2 > L}; on each
    unbounded axis xi = L/t, t in (0,1], and tensor Gauss-Legendre (nq points
    per axis) is applied."""
    h = 2.0 / N
    L = 2.0
    n = N - 1
    xg, wg = np.polynomial.legendre.leggauss(nq)
    sb = L * (xg + 1) / 2            # bounded axis [0, L]
    wb = wg * L / 2
    t = (xg + 1) / 2                 # unbounded axis xi = L/t: dxi = L/t^2 dt
    su = L / t
    wu = (wg / 2) * L / t ** 2
    pieces = [(su, wu, sb, wb), (su, wu, su, wu), (sb, wb, su, wu)]
    x = -1.0 + h * np.arange(N + 1)
    out = np.zeros((n, n))
    for i in range(1, N):
        for jj in range(1, N):
            tail = 0.0
            for (s1, w1, s2, w2) in pieces:
                X1, X2 = s1[:, None], s2[None, :]
                Wt = w1[:, None] * w2[None, :] * (X1 ** 2 + X2 ** 2) ** (-1.0 - alpha / 2)
                for m1 in (1.0, -1.0):
                    for m2 in (1.0, -1.0):
                        tail += float((Wt * g(x[i] + m1 * X1, x[jj] + m2 * X2)).sum())
            out[i - 1, jj - 1] = tail
    return out


def exterior_b_2d(G, g, alpha, nq=160):
    """2D analogue (eq. (2D-scheme), definition of b_ij): lattice sum minus
    c_{2,alpha} times the far-field integrals."""
    N = G.shape[0] - 1
    return exterior_lattice_2d(G, g) - c_dalpha(2, alpha) * far_field_tail_2d(N, g, alpha, nq)
