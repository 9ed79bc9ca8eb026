"""Seeded synthetic inputs (right-hand sides, request streams).

Holds none of the discretization's arithmetic: random draws, grid shapes and
one closed form of the continuous operator (the benchmark's disk right-hand
side, manufactured_rhs_disk).
Seeds follow one convention everywhere: numpy's PCG64 via
numpy.random.default_rng, FP64 draws in row-major order over the n^d
interior points; right-hand side j of a batch seeded s uses seed s + j.
"""

import numpy as np


def grid_shape(d, N):
    return (N - 1,) * d


def uniform_rhs(d, N, nrhs=1, seed=0):
    """nrhs arrays of i.i.d. U[-1, 1] values, shape (nrhs, n, ..., n)."""
    shp = grid_shape(d, N)
    return np.stack([np.random.default_rng(seed + j).uniform(-1.0, 1.0, shp)
                     for j in range(nrhs)])


def uniform_grid(shape, nrhs=1, seed=0):
    """nrhs arrays of i.i.d. U[-1, 1] values on a grid of any shape (a box's
    interior), shape (nrhs,) + shape."""
    return np.stack([np.random.default_rng(seed + j).uniform(-1.0, 1.0, tuple(shape))
                     for j in range(nrhs)])


def normal_rhs(d, N, nrhs=1, seed=0):
    """nrhs arrays of i.i.d. N(0, 1) values, shape (nrhs, n, ..., n)."""
    shp = grid_shape(d, N)
    return np.stack([np.random.default_rng(seed + j).standard_normal(shp)
                     for j in range(nrhs)])


def interior_coords(d, N):
    """Coordinates x_i = -1 + (i+1) h of the interior points, one array per axis."""
    h = 2.0 / N
    x = -1.0 + h * np.arange(1, N)
    return np.meshgrid(*([x] * d), indexing="ij")


def request_stream(n_requests=4096, rate=200.0, seed=0, alpha_round=0.01):
    """Serving workload: Poisson arrivals, d = 2 problems of mixed size.

    Each request: n in {63, 127, 255, 511} with probabilities 0.4/0.3/0.2/0.1
    (N = n + 1), alpha ~ U(0.2, 1.9) rounded to `alpha_round` (so that
    identical operators recur), degree in {0, 1, 2}, 1..8 right-hand sides
    of U[-1, 1] values drawn from default_rng([seed, request id, j])."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    ns = rng.choice([63, 127, 255, 511], size=n_requests, p=[0.4, 0.3, 0.2, 0.1])
    alphas = rng.uniform(0.2, 1.9, n_requests)
    if alpha_round:
        alphas = np.round(alphas / alpha_round) * alpha_round
    degrees = rng.integers(0, 3, n_requests)
    nrhs = rng.integers(1, 9, n_requests)
    reqs = []
    for i in range(n_requests):
        reqs.append(dict(id=i, t_arrive=float(t[i]), d=2, N=int(ns[i]) + 1,
                         alpha=float(alphas[i]), degree=int(degrees[i]),
                         nrhs=int(nrhs[i]), seed=[seed, i]))
    return reqs


def burst_stream(n_requests=512, rate=4000.0, seed=1):
    """Burst workload: requests for a few operators arriving faster than they
    are served, so that requests for the same operator queue and are merged:
    n in {127, 255}, alpha in {0.5, 1.0, 1.5}, degree 1 (six operators),
    1..8 right-hand sides, Poisson arrivals at `rate` per second."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    ns = rng.choice([127, 255], size=n_requests)
    alphas = rng.choice([0.5, 1.0, 1.5], size=n_requests)
    nrhs = rng.integers(1, 9, n_requests)
    return [dict(id=i, t_arrive=float(t[i]), d=2, N=int(ns[i]) + 1, alpha=float(alphas[i]),
                 degree=1, nrhs=int(nrhs[i]), seed=[seed, i]) for i in range(n_requests)]


def request_rhs(req):
    """Right-hand sides of one request, shape (nrhs, n, n)."""
    n = req["N"] - 1
    return np.stack([np.random.default_rng(list(req["seed"]) + [j]).uniform(-1.0, 1.0, (n, n))
                     for j in range(req["nrhs"])])


def manufactured_rhs_disk(N, alpha):
    """The benchmark's structured right-hand side on the 2D grid: inside the
    unit disk the closed-form image of u = (1-|x|^2)_+^{1+alpha/2},
    2^alpha Gamma(1+alpha/2) Gamma(2+alpha/2) (1 - (1+alpha/2)|x|^2),
    and zero in the corners |x| >= 1 of the square.  The image of u is
    negative there (it needs a singular quadrature per point), so this f is
    the image of no known solution on the square: a throughput input with the
    manufactured solution's shape, not an accuracy test.  Shape (n, n)."""
    import math
    X0, X1 = interior_coords(2, N)
    r2 = X0 * X0 + X1 * X1
    c = 2.0 ** alpha * math.gamma(1.0 + alpha / 2.0) * math.gamma(2.0 + alpha / 2.0)
    return np.where(r2 < 1.0, c * (1.0 - (1.0 + alpha / 2.0) * r2), 0.0)
