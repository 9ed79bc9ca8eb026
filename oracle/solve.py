"""Dense solves of A u = f (test infrastructure; see package header).

The paper only says the SPD multilevel-Toeplitz system can be solved with
fast FFT-based algorithms (Example 3.2.3); it names no solver.  A is
symmetric positive definite (Sec. 2.2), so the oracle uses a Cholesky
factorisation where A fits in memory and conjugate gradients on the block
product otherwise, optionally preconditioned by the restricted inverse of
the embedding circulant (operator.precond_apply).
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .operator import dense_matrix, apply


def solve_cholesky(G, f):
    """u = A^{-1} f by Cholesky of the materialised A (f may carry RHS as
    trailing axes beyond the grid axes)."""
    d = G.ndim
    shp = f.shape
    A = dense_matrix(G, shp[:d])   # the grid: f's first d axes (cube or box)
    fb = f.reshape((A.shape[0], -1)) if f.ndim > d else f.reshape(-1)
    u = cho_solve(cho_factor(A), fb)
    return u.reshape(shp)


def solve_cg(G, f, tol=1e-13, maxiter=100000, x0=None, precond=None):
    """Textbook CG (x0 = 0), stopping when ||r_k||_2 <= tol ||f||_2 on the
    recursively updated residual.  With `precond` (a callable z = P r for an
    SPD P) it is textbook preconditioned CG: rho = r.z drives alpha and beta,
    the stopping rule stays on ||r||_2.  Returns (u, iterations, rel. residual)."""
    P = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(f) if x0 is None else x0.copy()
    r = f - apply(G, x) if x0 is not None else f.copy()
    z = P(r)
    p = z.copy()
    rho = float(np.vdot(r, z))
    rr = float(np.vdot(r, r))
    fn = float(np.sqrt(np.vdot(f, f)))
    it = 0
    while np.sqrt(rr) > tol * fn and it < maxiter:
        q = apply(G, p)
        a = rho / float(np.vdot(p, q))
        x += a * p
        r -= a * q
        z = P(r)
        rho_new = float(np.vdot(r, z))
        p = z + (rho_new / rho) * p
        rho = rho_new
        rr = float(np.vdot(r, r))
        it += 1
    return x, it, np.sqrt(rr) / fn
