"""The lane algebra of the element kernels, restated in numpy: eight lanes per
element, lane l standing for corner (bx, by, bz) with l = bx ^ 2 by ^ 7 bz,
partners l ^ 1, l ^ 2, l ^ 7 along x, y, z.  The evaluation butterfly and
both forms of the transposed butterfly (the generic one, and the FP64 one
that sends each partner share once) are checked against the explicit
trilinear shape functions at the 2 x 2 x 2 Gauss points of a cube of side h:
  value and gradient of u at the lane's Gauss point,
  sum over Gauss points of N_a c_q + grad N_a . F_q on the lane of corner a.
The kernels' own results are checked against the oracle by the GPU tests."""
import numpy as np
import pytest

G = 1.0 / np.sqrt(3.0)
B = 0.5 * (1.0 - G)
A = 0.5 * (1.0 + G)


def lane_signs(h):
    """Per lane: corner index and the signs s/h along each axis."""
    corner, sx, sy, sz = [], [], [], []
    for l in range(8):
        bz = l >> 2
        t = (l ^ 7) if bz else l
        bx, by = t & 1, (t >> 1) & 1
        corner.append(bx + 2 * by + 4 * bz)
        sx.append((1 if bx else -1) / h)
        sy.append((1 if by else -1) / h)
        sz.append((1 if bz else -1) / h)
    return np.array(corner), np.array(sx), np.array(sy), np.array(sz)


def xchg(v, m):
    return v[np.arange(8) ^ m]


def eval_vg(u, sx, sy, sz):
    d1 = xchg(u, 1) - u
    v = u + B * d1
    dx = -sx * d1
    d2, e2 = xchg(v, 2) - v, xchg(dx, 2) - dx
    v2 = v + B * d2
    dy = -sy * d2
    dx2 = dx + B * e2
    d3, e3, f3 = xchg(v2, 7) - v2, xchg(dx2, 7) - dx2, xchg(dy, 7) - dy
    return v2 + B * d3, dx2 + B * e3, dy + B * f3, -sz * d3


def contract_generic(c, Fx, Fy, Fz, sx, sy, sz):
    c1 = c + B * (xchg(c, 7) - c) + sz * (Fz + xchg(Fz, 7))
    Fx1 = Fx + B * (xchg(Fx, 7) - Fx)
    Fy1 = Fy + B * (xchg(Fy, 7) - Fy)
    c2 = c1 + B * (xchg(c1, 2) - c1) + sy * (Fy1 + xchg(Fy1, 2))
    Fx2 = Fx1 + B * (xchg(Fx1, 2) - Fx1)
    return c2 + B * (xchg(c2, 1) - c2) + sx * (Fx2 + xchg(Fx2, 1))


def contract_fp64(c, Fx, Fy, Fz, sx, sy, sz):
    c1 = A * c + sz * Fz + xchg(B * c - sz * Fz, 7)
    Fx1 = A * Fx + xchg(B * Fx, 7)
    Fy1 = A * Fy + xchg(B * Fy, 7)
    c2 = A * c1 + sy * Fy1 + xchg(B * c1 - sy * Fy1, 2)
    Fx2 = A * Fx1 + xchg(B * Fx1, 2)
    return A * c2 + sx * Fx2 + xchg(B * c2 - sx * Fx2, 1)


def shape(h):
    """N[q, a] and dN[q, a, d] at Gauss point q (the point with corner q's sign
    pattern) for corner a of [0, h]^3."""
    pts = [((1 + (1 if (q & 1) else -1) * G) / 2, (1 + (1 if (q & 2) else -1) * G) / 2,
            (1 + (1 if (q & 4) else -1) * G) / 2) for q in range(8)]
    N = np.zeros((8, 8))
    dN = np.zeros((8, 8, 3))
    for q, (x, y, z) in enumerate(pts):
        for a in range(8):
            fx = x if a & 1 else 1 - x
            fy = y if a & 2 else 1 - y
            fz = z if a & 4 else 1 - z
            gx = 1 if a & 1 else -1
            gy = 1 if a & 2 else -1
            gz = 1 if a & 4 else -1
            N[q, a] = fx * fy * fz
            dN[q, a] = (gx * fy * fz / h, fx * gy * fz / h, fx * fy * gz / h)
    return N, dN


@pytest.mark.parametrize("level", [0, 3, 10])
def test_evaluation_butterfly_is_trilinear_interpolation(level):
    h = 2.0 ** -level
    corner, sx, sy, sz = lane_signs(h)
    N, dN = shape(h)
    rng = np.random.default_rng(level)
    for _ in range(20):
        uc = rng.normal(0.0, 1.0, 8)  # values at corners 0..7
        v, dx, dy, dz = eval_vg(uc[corner], sx, sy, sz)
        # lane l's Gauss point has corner l's sign pattern
        q = corner
        assert np.allclose(v, N[q] @ uc, rtol=0, atol=1e-14)
        assert np.allclose(dx, dN[q, :, 0] @ uc, rtol=1e-13, atol=1e-12 / h)
        assert np.allclose(dy, dN[q, :, 1] @ uc, rtol=1e-13, atol=1e-12 / h)
        assert np.allclose(dz, dN[q, :, 2] @ uc, rtol=1e-13, atol=1e-12 / h)


@pytest.mark.parametrize("form", [contract_generic, contract_fp64])
@pytest.mark.parametrize("level", [0, 4, 9])
def test_transposed_butterfly_is_the_test_function_contraction(form, level):
    h = 2.0 ** -level
    corner, sx, sy, sz = lane_signs(h)
    N, dN = shape(h)
    rng = np.random.default_rng(100 + level)
    for _ in range(20):
        c, Fx, Fy, Fz = (rng.normal(0.0, 1.0, 8) for _ in range(4))  # per lane, i.e. per Gauss point
        r = form(c, Fx, Fy, Fz, sx, sy, sz)
        q = corner  # Gauss point of each lane
        ref = np.zeros(8)
        for l in range(8):
            a = corner[l]
            ref[l] = sum(N[q[m], a] * c[m] + dN[q[m], a] @ np.array([Fx[m], Fy[m], Fz[m]]) for m in range(8))
        assert np.allclose(r, ref, rtol=1e-13, atol=1e-13 / h)


def test_partner_signs_differ_in_one_axis():
    _, sx, sy, sz = lane_signs(1.0)
    for l in range(8):
        assert sz[l ^ 7] == -sz[l] and sx[l ^ 7] == sx[l] and sy[l ^ 7] == sy[l]
        assert sy[l ^ 2] == -sy[l] and sx[l ^ 2] == sx[l] and sz[l ^ 2] == sz[l]
        assert sx[l ^ 1] == -sx[l] and sy[l ^ 1] == sy[l] and sz[l ^ 1] == sz[l]
