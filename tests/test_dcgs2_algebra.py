"""The algebra of the GMRES that the library runs on the device: right-
preconditioned restarted GMRES with classical Gram-Schmidt twice, the second
pass of each basis vector delayed into the next Arnoldi step, the provisional
vector stored unscaled, the stored preconditioned vectors those of the
provisional vectors (solution update through R^-1 y), and the column test on
provisional entries with the exact test at the end of the cycle.

Restated here in numpy, step for step as the control kernels order it, and
checked against textbook GMRES with CGS2 on seeded nonsymmetric systems:
same iteration counts, same iterates to rounding, an orthonormal basis.  The
GPU solver itself is checked against the oracle's steps by the GPU tests."""
import numpy as np
import pytest


def gmres_cgs2(A, M, b, m, max_it, rtol):
    """Textbook right-preconditioned GMRES(m), CGS2, stored Z = M^-1 V."""
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    its = 0
    while its < max_it:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= rtol * bn:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        e = np.zeros(m + 1)
        e[0] = beta
        done = False
        for k in range(m):
            z = M @ V[k]
            Z.append(z)
            w = A @ z
            Q = np.array(V)
            h1 = Q @ w
            w = w - Q.T @ h1
            h2 = Q @ w
            w = w - Q.T @ h2
            H[:k + 1, k] = h1 + h2
            H[k + 1, k] = np.linalg.norm(w)
            V.append(w / H[k + 1, k])
            its += 1
            y = np.linalg.lstsq(H[:k + 2, :k + 1], e[:k + 2], rcond=None)[0]
            res = np.linalg.norm(e[:k + 2] - H[:k + 2, :k + 1] @ y)
            if res <= rtol * bn or its >= max_it:
                done = True
                break
        x = x + np.array(Z).T @ y
        if done and res <= rtol * bn:
            break
    return x, its


def gmres_delayed(A, M, b, m, max_it, rtol):
    """The device scheme: one dot sweep and one update sweep per step."""
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    its = 0
    V = np.zeros((m + 1, n))
    Zt = np.zeros((m, n))
    Hr = np.zeros((m + 1, m))
    R = np.zeros((m + 1, m + 1))
    r = b.copy()
    beta = bn
    while True:
        V[0] = r / beta  # unit: the stored norm b of V_0 is 1
        bprov = 1.0
        g = np.zeros(m + 2)
        g[0] = beta
        cs = np.zeros(m + 1)
        sn = np.zeros(m + 1)
        H = np.zeros((m + 1, m + 1))
        kcols = 0
        finished = False

        def close(j):
            nonlocal its, kcols, finished
            col = Hr[:j + 2, j].copy()
            hn = col[j + 1]
            for i in range(j):
                a, c = col[i], col[i + 1]
                col[i], col[i + 1] = cs[i] * a + sn[i] * c, -sn[i] * a + cs[i] * c
            den = np.hypot(col[j], col[j + 1])
            cs[j], sn[j] = (col[j] / den, col[j + 1] / den) if den > 0 else (1.0, 0.0)
            col[j] = den
            H[:j + 1, j] = col[:j + 1]
            g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
            its += 1
            kcols = j + 1
            if abs(g[j + 1]) <= rtol * bn or den == 0 or hn == 0 or its >= max_it:
                finished = True

        def reorth(k, S, Sig):
            """Second pass of the stored provisional vector k (sums S, Sig of
            the stored vector, bprov times the unit one)."""
            s = S / bprov
            alpha = np.sqrt(Sig / bprov ** 2 - s @ s)
            R[:k, k] = S
            R[k, k] = bprov * alpha
            if k == 0:
                g[0] *= alpha
            else:
                hk = Hr[k, k - 1]
                Hr[:k, k - 1] += hk * s
                Hr[k, k - 1] = hk * alpha
                close(k - 1)
            return s, alpha

        provisional = False
        for k in range(m):
            Zt[k] = M @ V[k]
            w = A @ Zt[k]
            # dot sweep: the stored vector's sums, divided by bprov below
            S, T = V[:k] @ V[k], V[:k] @ w
            Sig, Tau = V[k] @ V[k], V[k] @ w
            provisional = False
            s, alpha = reorth(k, S, Sig)
            if finished:
                break
            t = T / bprov
            c = Hr[:k + 1, :k] @ s
            tk = (Tau / bprov ** 2 - s @ t) / alpha
            h = np.append(t - c[:k], tk - c[k]) / alpha
            cg = c / alpha + h
            # update sweep: the final v_k and the unscaled next provisional vector
            vk = (V[k] / bprov - V[:k].T @ s) / alpha
            wn = w / (bprov * alpha) - V[:k].T @ cg[:k] - cg[k] * vk
            V[k] = vk
            V[k + 1] = wn
            Hr[:k + 1, k] = h
            hn = np.linalg.norm(wn)
            Hr[k + 1, k] = hn
            if hn == 0:
                close(k)
                break
            bprov = hn
            provisional = True
            # the column test on provisional entries stops the steps early
            col = Hr[:k + 2, k].copy()
            for i in range(k):
                a, cc = col[i], col[i + 1]
                col[i], col[i + 1] = cs[i] * a + sn[i] * cc, -sn[i] * a + cs[i] * cc
            den = np.hypot(col[k], col[k + 1])
            if abs(col[k + 1] / den * g[k]) <= rtol * bn or its + 1 >= max_it:
                break
        if provisional:  # the cycle's last pass closes the provisional column
            kf = kcols + 1
            reorth(kf, V[:kf] @ V[kf], V[kf] @ V[kf])
        y = np.linalg.solve(np.triu(H[:kcols, :kcols]), g[:kcols])
        yp = np.linalg.solve(np.triu(R[:kcols, :kcols]), y)  # Z = Z~ R^-1
        x = x + Zt[:kcols].T @ yp
        if finished:
            break
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= rtol * bn:
            break
    return x, its, V[:kcols]


@pytest.mark.parametrize("seed,n,m", [(1, 200, 8), (2, 300, 20), (3, 120, 40), (4, 250, 60)])
def test_delayed_cgs2_gmres_matches_cgs2_gmres(seed, n, m):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 2.0 + rng.normal(0.0, 1.5 / np.sqrt(n), (n, n))
    M = np.diag(1.0 / np.diag(A)) + rng.normal(0.0, 0.01 / np.sqrt(n), (n, n))
    b = rng.normal(0.0, 1.0, n)
    rtol = 1e-10
    x1, i1 = gmres_cgs2(A, M, b, m, 2000, rtol)
    x2, i2, V = gmres_delayed(A, M, b, m, 2000, rtol)
    assert i1 == i2
    assert np.linalg.norm(x2 - x1) <= 1e-12 * np.linalg.norm(x1)
    assert np.linalg.norm(b - A @ x2) <= 1.01 * rtol * np.linalg.norm(b)
    # the last cycle's final basis vectors are orthonormal to working precision
    assert len(V) >= 1
    assert np.abs(V @ V.T - np.eye(len(V))).max() < 1e-13


def test_delayed_cgs2_iteration_cap_and_happy_breakdown():
    rng = np.random.default_rng(5)
    n = 150
    A = np.eye(n) * 2.0 + rng.normal(0.0, 1.5 / np.sqrt(n), (n, n))
    M = np.eye(n)
    b = rng.normal(0.0, 1.0, n)
    # the cap stops both at the same iterate
    x1, i1 = gmres_cgs2(A, M, b, 10, 37, 1e-14)
    x2, i2, _ = gmres_delayed(A, M, b, 10, 37, 1e-14)
    assert i1 == i2 == 37
    assert np.linalg.norm(x2 - x1) <= 1e-12 * np.linalg.norm(x1)
    # a right-hand side in a 3-dimensional invariant subspace: the Krylov space
    # closes after 3 steps and the solve is exact
    Q = np.linalg.qr(rng.normal(0.0, 1.0, (n, n)))[0]
    D = np.diag(np.concatenate([[1.0, 2.0, 3.0], rng.uniform(4.0, 5.0, n - 3)]))
    A2 = Q @ D @ Q.T
    b2 = Q[:, :3] @ np.array([1.0, -2.0, 0.5])
    x3, i3, _ = gmres_delayed(A2, np.eye(n), b2, 20, 100, 1e-15)
    assert i3 <= 4
    assert np.linalg.norm(b2 - A2 @ x3) <= 1e-12 * np.linalg.norm(b2)
