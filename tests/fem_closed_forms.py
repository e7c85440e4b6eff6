"""Closed forms for trilinear (Q1) elements on a uniform grid, built from the
tensor-product structure of Q1: every matrix entry between an interior node a
and a node b = a + (ox, oy, oz) is a product of 1-D integrals of piecewise
linear hats of spacing h.  These are textbook values, independent of any
quadrature code:

    m(0) = 2h/3, m(+-1) = h/6             int phi_a phi_b
    k(0) = 2/h,  k(+-1) = -1/h            int phi_a' phi_b'
    c(-1) = 1/2, c(0) = 0, c(+1) = -1/2   int phi_a' phi_b
    d(o) = c(-o)                          int phi_a phi_b'
"""
import itertools

import numpy as np


def m1(o, h):
    return {0: 2 * h / 3, -1: h / 6, 1: h / 6}.get(o, 0.0)


def k1(o, h):
    return {0: 2 / h, -1: -1 / h, 1: -1 / h}.get(o, 0.0)


def c1(o, h):
    return {0: 0.0, -1: 0.5, 1: -0.5}.get(o, 0.0)


def d1(o, h):
    return c1(-o, h)


def offsets():
    return list(itertools.product((-1, 0, 1), repeat=3))


def mass(o, h):
    return m1(o[0], h) * m1(o[1], h) * m1(o[2], h)


def _f(i, j, o, h):
    """int dN_a/dx_i dN_b/dx_j for i, j in {0,1,2}."""
    val = 1.0
    for ax in range(3):
        if ax == i and ax == j:
            val *= k1(o[ax], h)
        elif ax == i:
            val *= c1(o[ax], h)
        elif ax == j:
            val *= d1(o[ax], h)
        else:
            val *= m1(o[ax], h)
    return val


def grad_grad(i, j, o, h):
    return _f(i, j, o, h)


def stiffness(o, h):
    return sum(_f(i, i, o, h) for i in range(3))


def n_dN(j, o, h):
    """int N_a dN_b/dx_j."""
    val = 1.0
    for ax in range(3):
        val *= d1(o[ax], h) if ax == j else m1(o[ax], h)
    return val


def dN_n(j, o, h):
    """int dN_a/dx_j N_b."""
    val = 1.0
    for ax in range(3):
        val *= c1(o[ax], h) if ax == j else m1(o[ax], h)
    return val


def lattice_index(nodes_int, level):
    """idx[i, j, k] -> node id on a uniform mesh of the given level."""
    N = 2 ** level
    idx = -np.ones((N + 1, N + 1, N + 1), dtype=np.int64)
    idx[nodes_int[:, 0], nodes_int[:, 1], nodes_int[:, 2]] = np.arange(nodes_int.shape[0])
    assert (idx >= 0).all()
    return idx


# ------------------------------------------------ exact 1-D hat integrals --
# Hats of a uniform grid of spacing h: node i at x_i = i h.  The integrals
# below are computed cell by cell with exact polynomial antiderivatives (no
# quadrature rule), optionally with a polynomial weight w(x) given by its
# coefficients in increasing powers of x.
def _hat_piece(i, cell, h, deriv):
    """Polynomial coefficients, in the local coordinate s = x - x_cell in
    [0, h], of hat i (or its derivative) on cell [x_cell, x_cell + h]."""
    if cell == i - 1:      # rising part: s / h
        return np.array([1.0 / h]) if deriv else np.array([0.0, 1.0 / h])
    if cell == i:          # falling part: (h - s) / h
        return np.array([-1.0 / h]) if deriv else np.array([1.0, -1.0 / h])
    return np.array([0.0])


def hat_integral(ia, da, ib, db, h, weight=(1.0,)):
    """int w(x) hat_ia^(da)(x) hat_ib^(db)(x) dx over the real line (da, db in
    {0, 1}: value or first derivative)."""
    P = np.polynomial.polynomial
    total = 0.0
    for cell in (ia - 1, ia):
        if cell not in (ib - 1, ib):
            continue
        # the weight in the local coordinate: w(x_cell + s)
        w = np.polynomial.Polynomial(np.asarray(weight, float))(
            np.polynomial.Polynomial([cell * h, 1.0])).coef
        f = P.polymul(P.polymul(_hat_piece(ia, cell, h, da), _hat_piece(ib, cell, h, db)), w)
        total += P.polyval(h, P.polyint(f))
    return total


def tensor_integral(a, da, b, db, h, weights=None):
    """int prod_ax w_ax(x_ax) d^da N_a d^db N_b over R^3 for lattice nodes a, b
    (index triples); da, db are derivative axes (None for the value); weights
    maps an axis to polynomial coefficients of a weight along that axis."""
    val = 1.0
    for ax in range(3):
        w = (weights or {}).get(ax, (1.0,))
        val *= hat_integral(a[ax], int(da == ax), b[ax], int(db == ax), h, w)
    return val
