"""Exact integrals of the 1D quadratic (cG(2)) basis functions against
polynomials, for closed-form checks of the oracle's triquadratic CH rows.

On a uniform grid of cells of side h over [0, L], the nodes sit at multiples
of h/2.  Node m (position m h/2) is a cell vertex for even m, with support on
the two cells around it, and a cell midpoint for odd m, with support on its
cell.  On a cell [x0, x0 + h] with local coordinate t = (x - x0)/h the three
basis functions are l0 = 2(t - 1/2)(t - 1), l1 = -4t(t - 1), l2 = 2t(t - 1/2).
Integrals are taken exactly with numpy's polynomial arithmetic in t, so no
quadrature rule is involved.
"""
import numpy as np

_L = [np.poly1d([2.0, -3.0, 1.0]),   # 2(t - 1/2)(t - 1)
      np.poly1d([-4.0, 4.0, 0.0]),   # -4t(t - 1)
      np.poly1d([2.0, -1.0, 0.0])]   # 2t(t - 1/2)


def _pieces(m, h, length):
    """(cell origin, local basis index) pairs of node m's support."""
    x = m * h / 2.0
    if m % 2:
        return [(x - h / 2.0, 1)]
    out = []
    if x - h >= -1e-12:
        out.append((x - h, 2))
    if x + h <= length + 1e-12:
        out.append((x, 0))
    return out


def hat_integral(m, h, length, f, deriv=0):
    """Integral over [0, length] of n_m^(deriv)(x) f(x), f a numpy poly1d in x,
    n_m the quadratic basis function of node m (deriv 0 or 1)."""
    s = 0.0
    for x0, i in _pieces(m, h, length):
        g = f(np.poly1d([h, x0]))          # f(x0 + h t) as a polynomial in t
        b = _L[i] if deriv == 0 else np.polyder(_L[i]) / h
        p = np.polyint(b * g)
        s += h * (p(1.0) - p(0.0))
    return s


def poly(*coeffs_low_first):
    """poly1d from coefficients in increasing powers."""
    return np.poly1d(list(coeffs_low_first)[::-1])
