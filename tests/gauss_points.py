"""Values of a nodal field at the 2x2x2 Gauss points of every leaf of an
oracle mesh (numpy, from the mesh arrays: corners through their constraint
rows, then the trilinear interpolant), and the rows an element set touches.
Used to find the points where a floating-point decision (the pull-back of
phi at |phi| = 1) can fall differently in FP32 and FP64."""
import numpy as np

G = 1.0 / np.sqrt(3.0)


def corner_values(m, u):
    """(E, 8) corner values of the nodal field u (hanging corners through
    their constraint rows)."""
    nh = m.hang_xyz.shape[0]
    if nh == 0:
        return u[m.elem]
    hv = np.zeros(nh)
    for h in range(nh):
        a, b = m.hang_off[h], m.hang_off[h + 1]
        hv[h] = (m.hang_w[a:b] * u[m.hang_ids[a:b]]).sum()
    return np.where(m.elem >= 0, u[np.maximum(m.elem, 0)], hv[np.maximum(-1 - m.elem, 0)])


def gauss_values(m, u):
    """(E, 8) values at the Gauss points, point q = i + 2j + 4k at
    ((-1)^(i+1), (-1)^(j+1), (-1)^(k+1)) / sqrt(3) on the reference cube."""
    cv = corner_values(m, u)
    out = np.zeros_like(cv)
    for q in range(8):
        xi = [G if (q >> d) & 1 else -G for d in range(3)]
        for c in range(8):
            w = 1.0
            for d in range(3):
                s = 1.0 if (c >> d) & 1 else -1.0
                w *= 0.5 * (1 + s * xi[d])
            out[:, q] += w * cv[:, c]
    return out


def touched_rows(m, elems):
    """Independent nodes touched by the listed elements, directly or as
    constraint parents of their hanging corners."""
    rows = set()
    for e in np.nonzero(elems)[0]:
        for r in m.elem[e]:
            if r >= 0:
                rows.add(int(r))
            else:
                h = -1 - r
                rows.update(int(i) for i in m.hang_ids[m.hang_off[h]:m.hang_off[h + 1]])
    return np.array(sorted(rows), dtype=np.int64)


def near_pullback(m, U1, width=1e-5):
    """Elements with a Gauss point where |phi^{k+1}| is within `width` of 1,
    and the rows they touch."""
    phq = gauss_values(m, U1[:, 0])
    el = (np.abs(np.abs(phq) - 1.0) < width).any(axis=1)
    return el, touched_rows(m, el)
