"""Independent 2x2x2 Gauss quadrature of Q1 fields on a uniform lattice
(numpy, tensor-product 1-D hats), used to evaluate the energy functional and
the other integrals of the discrete energy identity."""
import numpy as np

G = 1.0 / np.sqrt(3.0)


def _lattice(u, idx):
    return u[idx]


def qp_fields(u, idx, h):
    """Values and gradients of the Q1 field with nodal values u at the 8 Gauss
    points of every cell: returns val (8, N, N, N), grad (8, 3, N, N, N)."""
    U = _lattice(u, idx)
    N = U.shape[0] - 1
    xi = (-G, G)
    s = (-1.0, 1.0)
    b = [[0.5 * (1 + s[c] * xi[q]) for c in range(2)] for q in range(2)]
    db = [[s[c] / h for c in range(2)] for q in range(2)]
    corner = {}
    for cx in range(2):
        for cy in range(2):
            for cz in range(2):
                corner[(cx, cy, cz)] = U[cx:cx + N, cy:cy + N, cz:cz + N]
    vals, grads = [], []
    for qz in range(2):
        for qy in range(2):
            for qx in range(2):
                v = 0.0
                g = [0.0, 0.0, 0.0]
                for (cx, cy, cz), C in corner.items():
                    v = v + b[qx][cx] * b[qy][cy] * b[qz][cz] * C
                    g[0] = g[0] + db[qx][cx] * b[qy][cy] * b[qz][cz] * C
                    g[1] = g[1] + b[qx][cx] * db[qy][cy] * b[qz][cz] * C
                    g[2] = g[2] + b[qx][cx] * b[qy][cy] * db[qz][cz] * C
                vals.append(v)
                grads.append(np.stack(g))
    return np.stack(vals), np.stack(grads)


def integrate(f, h):
    """Sum over cells and Gauss points of f (8, N, N, N) with weight h^3/8."""
    return float(f.sum() * h ** 3 / 8.0)
