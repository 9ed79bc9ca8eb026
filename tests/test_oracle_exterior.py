"""Pins of the exterior-data lattice sums (the terms of eq. (1D-scheme) and
eq. (2D-scheme) that carry g, and their 3D form under reading R4).

* g = 1 on every exterior node: the lattice sum plus A 1 is the sum of G over
  the whole offset box [-N, N]^d, which the definition of a_0 fixes to
  c_{d,alpha} 2^d T_d (the far-field constant); a wrong exterior mask, offset
  or stencil range breaks it.
* g = the indicator of one exterior node j: b_i = G_{|j - i|} when
  |j - i|_inf <= N, else 0 (brute force on tiny grids).
* g even in every coordinate and symmetric under coordinate swaps: b has the
  same symmetries.
The first two also on boxes (axis s with N_s <= N intervals, Sec. 2.2).
"""

import numpy as np
import pytest

import oracle


def lattice(d):
    f = {1: oracle.exterior_lattice_1d, 2: oracle.exterior_lattice_2d,
         3: oracle.exterior_lattice_3d}[d]
    return lambda G, g, box=None: f(G, g, box)


def ones(d):
    if d == 1:
        return lambda x: np.ones_like(np.asarray(x, dtype=float))
    return lambda *xs: np.ones(np.broadcast(*xs).shape)


@pytest.mark.parametrize("d,alpha,p,N", [(1, 1.3, 1, 12), (2, 1.3, 1, 8), (2, 0.6, 2, 8),
                                         (3, 0.7, 1, 6), (3, 1.6, 2, 6), (3, 1.0, 0, 5)])
def test_unit_data_fills_the_offset_box(d, alpha, p, N):
    G = oracle.generator(d, alpha, p, N)
    b = lattice(d)(G, ones(d))
    n = N - 1
    a1 = oracle.apply(G, np.ones((n,) * d))
    full = oracle.c_dalpha(d, alpha) * 2 ** d * oracle.far_field_T(d, alpha)
    scale = np.abs(G).max() * (2 * N + 1) ** d
    assert np.abs(a1 + b - full).max() <= 1e-13 * scale


@pytest.mark.parametrize("d,N,node", [(2, 5, (-2, 3)), (2, 5, (7, 0)), (3, 4, (-1, 2, 5)),
                                      (3, 4, (0, 0, 0)), (3, 5, (2, 6, 3))])
def test_single_exterior_node(d, N, node):
    G = oracle.generator(d, 1.1, 1, N)
    h = 2.0 / N
    xj = [-1.0 + j * h for j in node]

    def g(*xs):
        m = np.ones(np.broadcast(*xs).shape, dtype=bool)
        for x, c in zip(xs, xj):
            m &= np.isclose(x, c, rtol=0.0, atol=1e-12)
        return m.astype(float)

    b = lattice(d)(G, g)
    exp = np.zeros((N - 1,) * d)
    for i in np.ndindex(*exp.shape):
        off = [abs(j - (ii + 1)) for j, ii in zip(node, i)]
        if max(off) <= N:
            exp[i] = G[tuple(off)]
    assert np.array_equal(b, exp)


def test_symmetries_3d():
    N = 6
    G = oracle.generator(3, 0.9, 1, N)
    b = oracle.exterior_lattice_3d(G, lambda a, c, e: np.exp(-(a * a + c * c + e * e)))
    tol = 1e-14 * np.abs(b).max()
    for ax in range(3):
        assert np.abs(b - np.flip(b, axis=ax)).max() <= tol
    assert np.abs(b - np.transpose(b, (1, 0, 2))).max() <= tol
    assert np.abs(b - np.transpose(b, (2, 1, 0))).max() <= tol


@pytest.mark.parametrize("d,N,box", [(1, 12, (7,)), (2, 8, (8, 5)), (2, 9, (4, 9)),
                                     (3, 6, (6, 3, 4))])
def test_unit_data_identity_on_boxes(d, N, box):
    """On a box (axis s with N_s <= N intervals) every interior node still sees
    the whole offset box [-N, N]^d, so b(1) + A 1 = c_{d,alpha} 2^d T_d."""
    alpha = 1.2
    G = oracle.generator(d, alpha, 1, N)
    b = lattice(d)(G, ones(d), box)
    a1 = oracle.apply(G, np.ones(tuple(v - 1 for v in box)))
    full = oracle.c_dalpha(d, alpha) * 2 ** d * oracle.far_field_T(d, alpha)
    scale = np.abs(G).max() * (2 * N + 1) ** d
    assert b.shape == a1.shape
    assert np.abs(a1 + b - full).max() <= 1e-13 * scale


@pytest.mark.parametrize("d,N,box,node", [(2, 6, (6, 3), (1, 3)), (2, 6, (4, 6), (5, -2)),
                                          (3, 4, (4, 2, 3), (1, 2, 1))])
def test_single_exterior_node_on_boxes(d, N, box, node):
    G = oracle.generator(d, 0.8, 1, N)
    h = 2.0 / N
    xj = [-1.0 + j * h for j in node]

    def g(*xs):
        m = np.ones(np.broadcast(*xs).shape, dtype=bool)
        for x, c in zip(xs, xj):
            m &= np.isclose(x, c, rtol=0.0, atol=1e-12)
        return m.astype(float)

    b = lattice(d)(G, g, box)
    exp = np.zeros(tuple(v - 1 for v in box))
    for i in np.ndindex(*exp.shape):
        off = [abs(j - (ii + 1)) for j, ii in zip(node, i)]
        if max(off) <= N:
            exp[i] = G[tuple(off)]
    assert np.array_equal(b, exp)
