"""Pins of the oracle's cG(2) blocks (27-node leaves, 3x3x3 Gauss rule,
quadratic hanging constraints), against facts fixed by the mathematics:

* the triquadratic numbering of a uniform mesh has (2^(L+1) + 1)^3 nodes and
  no hanging node;
* on adaptive meshes the constraint rows reproduce any triquadratic
  polynomial at the hanging nodes (continuity of the cG(2) space across a
  2:1 face or edge, Sec. 4 "Handling hanging nodes" carried over to Q2);
* on a uniform mesh, with states whose integrands are polynomials of degree
  at most 5 per axis (so the 3-point rule is exact), every CH row and every
  JVP row equals its integral taken exactly (tests/q2_closed_forms.py); the
  rows follow Def. 2's chemical-potential and CH equations (eqns
  mu_eqn_var_semi_disc, phi_eqn_var_semi_disc) with the Crank-Nicolson
  midpoints of the cG(1) oracle;
* on adaptive meshes the phi rows sum to the integral of (phi^{k+1} -
  phi^k)/dt and the mu rows to that of psi'(phi~) - mu~ (partition of unity);
* the JVP is the derivative of the residual (central differences);
* NS block (the VMS form of Def. 2 with the cG(1) oracle's readings, and the
  second-derivative terms of R_m that trilinear leaves do not have): for a
  Poiseuille profile with its balancing pressure, and for a quadratic phase
  whose capillary divergence (Laplacian part included) a quadratic pressure
  balances, R_m = R_c = 0 and every row equals its Galerkin integral; at rest
  (hydrostatic) tau_m and tau_c are constants of the leaf size and every JVP
  row in a polynomial direction equals its exact integral, the Laplacian of
  the direction included.  Mutations of either Laplacian, the grad-div and
  continuity stabilisation terms, the basis' second derivatives, the pressure
  term and the wall rows each fail one of these.
"""
import numpy as np
import pytest

import oracle
from paper_1912_12453_amd import workloads as W
from tests.q2_closed_forms import hat_integral, poly

P = dict(Cn=0.3, Pe=2.0, Re=7.0, We=3.0, Fr=1.5, rho_minus=0.25, eta_minus=0.4, dt=0.05)


def params():
    return oracle.Params.make(**P)


def uniform(level):
    m = oracle.Mesh((1, 1, 1), level, level)
    return m, m.q2()


@pytest.mark.parametrize("level,trees", [(1, (1, 1, 1)), (2, (1, 1, 1)), (1, (2, 1, 1))])
def test_uniform_numbering(level, trees):
    m = oracle.Mesh(trees, level, level)
    q = m.q2()
    k = 2 ** (level + 1)
    assert q.n_nodes == (trees[0] * k + 1) * (trees[1] * k + 1) * (trees[2] * k + 1)
    assert q.hang_xyz.shape[0] == 0
    assert m.n_leaves == trees[0] * trees[1] * trees[2] * 8 ** level
    assert np.all(q.elem >= 0)


def _adaptive_meshes():
    out = []
    for seed, (lmin, lmax) in ((7, (2, 4)), (11, (1, 4)), (5, (2, 5))):
        leaves = W.random_leaves((1, 1, 1), lmax, seed, p_split=0.35, level_min=lmin)
        out.append(oracle.Mesh((1, 1, 1), 0, lmax, leaves=leaves))
    drops = [(np.array([0.4, 0.45, 0.5]), 0.2)]
    out.append(oracle.Mesh((1, 1, 1), 2, 5, W.drops_phi(drops, 0.05, -1.0), 0.9))
    return out


def _tri(x, c):
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * X + c[5] * Y * Y + c[6] * Z * Z
            + c[7] * X * Y + c[8] * Y * Z + c[9] * X * Z + c[10] * X * X * Y * Y * Z * Z
            + c[11] * X * Y * Z + c[12] * X * X * Y * Z)


def test_constraints_reproduce_triquadratics():
    rng = np.random.default_rng(3)
    seen_hanging = 0
    for m in _adaptive_meshes():
        q = m.q2()
        nh = q.hang_xyz.shape[0]
        seen_hanging += nh
        w = np.add.reduceat(q.hang_w, q.hang_off[:-1]) if nh else np.zeros(0)
        assert np.allclose(w, 1.0, atol=1e-14)
        c = rng.normal(size=13)
        u = _tri(q.node_xyz(), c)
        for i in range(nh):
            s = slice(q.hang_off[i], q.hang_off[i + 1])
            got = np.dot(q.hang_w[s], u[q.hang_ids[s]])
            assert abs(got - _tri(q.hang_coords()[i:i + 1], c)[0]) < 1e-13
    assert seen_hanging > 1000


def _tables(n1d, h, funcs):
    """1D integrals for lattice indices 0..n1d-1: key -> array."""
    out = {}
    for key, (f, d) in funcs.items():
        out[key] = np.array([hat_integral(m, h, 1.0, f, d) for m in range(n1d)])
    return out


def _lattice(q, level):
    # node coordinates in doubled units are the lattice indices (h/2 = 2^-(level+1))
    return q.nodes[:, 0], q.nodes[:, 1], q.nodes[:, 2]


A, B, DELTA = 0.2, 0.7, 0.3
C0, C1, C2 = 0.4, -0.9, 0.6
V = (0.5, -0.3, 0.8)


def _state(q):
    x = q.node_xyz()
    U1 = np.zeros((q.n_nodes, 6))
    U0 = np.zeros((q.n_nodes, 6))
    lin = A + B * x[:, 0]
    U1[:, 0], U0[:, 0] = lin + DELTA / 2, lin - DELTA / 2
    mu = C0 + C1 * x[:, 0] * x[:, 1] + C2 * x[:, 1] ** 2
    U1[:, 1] = U0[:, 1] = mu
    for d in range(3):
        U1[:, 2 + d] = U0[:, 2 + d] = V[d]
    U1[:, 5], U0[:, 5] = 0.37, -0.2  # pressure does not enter the CH rows
    return U1, U0


@pytest.mark.parametrize("level", [1, 2])
def test_residual_closed_form(level):
    m, q = uniform(level)
    h = 2.0 ** -level
    n1d = 2 ** (level + 1) + 1
    one, x1, x2 = poly(1.0), poly(0.0, 1.0), poly(0.0, 0.0, 1.0)
    phit = poly(A, B)
    psi1 = phit ** 3 - phit
    T = _tables(n1d, h, {"I0": (one, 0), "I1": (x1, 0), "I2": (x2, 0), "D0": (one, 1),
                         "D1": (x1, 1), "Nphi": (phit, 0), "Dphi": (phit, 1), "Npsi": (psi1, 0)})
    ix, iy, iz = _lattice(q, level)
    g = lambda k, i: T[k][i]
    kd, cn2, dt = 1.0 / (P["Pe"] * P["Cn"]), P["Cn"] ** 2, P["dt"]
    r_phi = (DELTA / dt * g("I0", ix) * g("I0", iy) * g("I0", iz)
             - (V[0] * g("Dphi", ix) * g("I0", iy) * g("I0", iz)
                + V[1] * g("Nphi", ix) * g("D0", iy) * g("I0", iz)
                + V[2] * g("Nphi", ix) * g("I0", iy) * g("D0", iz))
             + kd * (C1 * g("D0", ix) * g("I1", iy) * g("I0", iz)
                     + (C1 * g("I1", ix) * g("D0", iy) + 2 * C2 * g("I0", ix) * g("D1", iy)) * g("I0", iz)))
    r_mu = (g("Npsi", ix) * g("I0", iy) * g("I0", iz)
            - (C0 * g("I0", ix) * g("I0", iy) + C1 * g("I1", ix) * g("I1", iy)
               + C2 * g("I0", ix) * g("I2", iy)) * g("I0", iz)
            + cn2 * B * g("D0", ix) * g("I0", iy) * g("I0", iz))
    U1, U0 = _state(q)
    R = q.residual(params(), U1, U0)
    scale = max(np.abs(r_phi).max(), np.abs(r_mu).max())
    assert np.abs(R[:, 0] - r_phi).max() <= 1e-13 * scale
    assert np.abs(R[:, 1] - r_mu).max() <= 1e-13 * scale
    assert np.all(R[:, 2:] == 0.0)


@pytest.mark.parametrize("level", [1, 2])
def test_jvp_closed_form(level):
    m, q = uniform(level)
    h = 2.0 ** -level
    n1d = 2 ** (level + 1) + 1
    E_, F_, G_ = 0.3, -0.5, 0.8  # d phi = E + F z, d mu = G x^2
    one, x1 = poly(1.0), poly(0.0, 1.0)
    phit = poly(A, B)
    dpsi2 = 3 * phit ** 2 - 1
    dphi = poly(E_, F_)
    T = _tables(n1d, h, {"I0": (one, 0), "D0": (one, 1), "X2": (poly(0.0, 0.0, 1.0), 0),
                         "Dx2": (2 * x1, 1), "Ndp": (dphi, 0), "Ddp": (dphi, 1), "Npp": (dpsi2, 0)})
    ix, iy, iz = _lattice(q, level)
    g = lambda k, i: T[k][i]
    kd, cn2, dt = 1.0 / (P["Pe"] * P["Cn"]), P["Cn"] ** 2, P["dt"]
    j_phi = (g("I0", ix) * g("I0", iy) * g("Ndp", iz) / dt
             - 0.5 * (V[0] * g("D0", ix) * g("I0", iy) * g("Ndp", iz)
                      + V[1] * g("I0", ix) * g("D0", iy) * g("Ndp", iz)
                      + V[2] * g("I0", ix) * g("I0", iy) * g("Ddp", iz))
             + kd * 0.5 * G_ * g("Dx2", ix) * g("I0", iy) * g("I0", iz))
    j_mu = (0.5 * g("Npp", ix) * g("I0", iy) * g("Ndp", iz)
            - 0.5 * G_ * g("X2", ix) * g("I0", iy) * g("I0", iz)
            + cn2 * 0.5 * F_ * g("I0", ix) * g("I0", iy) * g("D0", iz))
    U1, U0 = _state(q)
    x = q.node_xyz()
    dU = np.zeros_like(U1)
    dU[:, 0] = E_ + F_ * x[:, 2]
    dU[:, 1] = G_ * x[:, 0] ** 2
    dU[:, 2:] = 0.9  # velocity and pressure directions do not enter the CH block's JVP
    J = q.jvp(params(), U1, U0, dU)
    scale = max(np.abs(j_phi).max(), np.abs(j_mu).max())
    assert np.abs(J[:, 0] - j_phi).max() <= 1e-13 * scale
    assert np.abs(J[:, 1] - j_mu).max() <= 1e-13 * scale
    assert np.all(J[:, 2:] == 0.0)


def test_row_sums_on_adaptive_meshes():
    for m in _adaptive_meshes():
        q = m.q2()
        U1, U0 = _state(q)
        R = q.residual(params(), U1, U0)
        # sum_a N_a = 1 and sum_a grad N_a = 0 on every leaf, through the constraints too
        assert abs(R[:, 0].sum() - DELTA / P["dt"]) < 1e-11
        psi = np.polyint(poly(A, B) ** 3 - poly(A, B))
        mu_int = C0 + C1 * 0.25 + C2 / 3.0
        assert abs(R[:, 1].sum() - (psi(1.0) - psi(0.0) - mu_int)) < 1e-12


def test_jvp_is_the_derivative_of_the_residual():
    m = _adaptive_meshes()[0]
    q = m.q2()
    rng = np.random.default_rng(9)
    n = q.n_nodes
    U0 = np.zeros((n, 6))
    U0[:, 0] = rng.uniform(-1.1, 1.1, n)
    U0[:, 1] = rng.normal(0, 0.5, n)
    U0[:, 2:5] = rng.normal(0, 0.3, (n, 3))
    U1 = U0 + rng.normal(0, 0.05, U0.shape)
    dU = rng.normal(0, 1.0, U0.shape)
    J = q.jvp(params(), U1, U0, dU)
    e = 1e-6
    dC = dU.copy()
    dC[:, 2:] = 0.0
    fd = (q.residual(params(), U1 + e * dC, U0) - q.residual(params(), U1 - e * dC, U0)) / (2 * e)
    err = np.linalg.norm(J[:, :2] - fd[:, :2]) / np.linalg.norm(fd[:, :2])
    assert err < 1e-8, err


# --------------------------------------------------------------- NS block --
NS = oracle.BLOCK_NS
PHI_C = 0.3  # constant phase inside (-1, 1): rho, eta constant, grad eta = 0


def _ns_params(g=(0.0, -1.0, 0.0)):
    return oracle.Params.make(**dict(P, g=g))


def _mixture():
    rho = 0.5 * (1 - P["rho_minus"]) * PHI_C + 0.5 * (1 + P["rho_minus"])
    eta = 0.5 * (1 - P["eta_minus"]) * PHI_C + 0.5 * (1 + P["eta_minus"])
    return rho, eta


def _interior(q):
    return (q.bflags & 1) == 0


@pytest.mark.parametrize("level", [1, 2])
def test_ns_poiseuille_closed_form(level):
    """v = (U(y), 0, 0) with U quadratic and the pressure that balances its
    viscous term and gravity: the strong residuals R_m (with the Laplacian of
    v, which trilinear leaves do not have) and R_c vanish at every point, so
    every VMS term drops out and the rows are the Galerkin integrals."""
    m, q = uniform(level)
    h = 2.0 ** -level
    n1d = 2 ** (level + 1) + 1
    rho, eta = _mixture()
    Re, We, Fr = P["Re"], P["We"], P["Fr"]
    c0, c1, c2 = 0.2, 0.5, -0.8
    Px = We * 2 * eta * c2 / Re        # (1/We) dp/dx = (1/Re) eta U''
    Py = -We * rho / Fr                # (1/We) dp/dy = rho g_y / Fr, g = (0, -1, 0)
    P0 = 0.4
    x = q.node_xyz()
    U = np.zeros((q.n_nodes, 6))
    U[:, 0] = PHI_C
    U[:, 1] = 0.7
    U[:, 2] = c0 + c1 * x[:, 1] + c2 * x[:, 1] ** 2
    U[:, 5] = P0 + Px * x[:, 0] + Py * x[:, 1]
    R = q.residual(_ns_params(), U, U.copy(), block=NS)
    one, y1 = poly(1.0), poly(0.0, 1.0)
    T = _tables(n1d, h, {"I0": (one, 0), "D0": (one, 1), "Dp": (poly(P0, Px), 1), "Np": (poly(P0, Px), 0),
                         "Y1": (y1, 0), "DY1": (y1, 1), "DUp": (poly(c1, 2 * c2), 1)})
    ix, iy, iz = _lattice(q, level)
    g = lambda k, i: T[k][i]
    rx = eta / Re * g("I0", ix) * g("DUp", iy) * g("I0", iz) - (
        g("Dp", ix) * g("I0", iy) + Py * g("D0", ix) * g("Y1", iy)) * g("I0", iz) / We
    ry = -(g("Np", ix) * g("D0", iy) + Py * g("I0", ix) * hat_y_deriv(T, iy)) * g("I0", iz) / We \
        + rho / Fr * g("I0", ix) * g("I0", iy) * g("I0", iz)
    rz = -(g("Np", ix) * g("I0", iy) + Py * g("I0", ix) * g("Y1", iy)) * g("D0", iz) / We
    inner = _interior(q)
    scale = max(np.abs(rx).max(), np.abs(ry).max(), np.abs(rz).max())
    for f, ref in ((2, rx), (3, ry), (4, rz)):
        assert np.abs(R[inner, f] - ref[inner]).max() <= 1e-12 * scale, f
    assert np.abs(R[(q.bflags & 2) == 0, 5]).max() <= 1e-12 * scale  # continuity rows vanish
    assert np.all(R[q.bflags == 1, 2:5] == 0.0)  # walls held: v^{k+1} - v^k


def hat_y_deriv(T, iy):
    """integral of n_j'(y) * y over the support (from the table of y n')."""
    return T["DY1"][iy]


@pytest.mark.parametrize("level", [1, 2])
def test_ns_jvp_closed_form_at_rest(level):
    """At rest (v = 0, constant phase, hydrostatic pressure) R_m = R_c = 0 and
    tau_m, tau_c are constants of the leaf size, so the Jacobian applied to a
    polynomial direction (dv quadratic with a Laplacian, dp linear) is a sum
    of exact polynomial integrals: the time term, pressure, viscous and
    grad-div (tau_c) terms in the momentum rows, the divergence and the
    tau_m-weighted linearised R_m (with the Laplacian of dv) in the
    continuity rows."""
    m, q = uniform(level)
    h = 2.0 ** -level
    n1d = 2 ** (level + 1) + 1
    rho, eta = _mixture()
    Re, We, Fr, dt, C_I = P["Re"], P["We"], P["Fr"], P["dt"], 6.0
    G = 4.0 / h ** 2
    nu = eta / (rho * Re)
    tau_m = (4.0 / dt ** 2 + C_I * nu * nu * 3 * G * G) ** -0.5
    tau_c = 1.0 / (3 * G * tau_m)
    x = q.node_xyz()
    U = np.zeros((q.n_nodes, 6))
    U[:, 0] = PHI_C
    U[:, 1] = 0.7
    U[:, 5] = 0.4 - We * rho / Fr * x[:, 1]
    dU = np.zeros_like(U)
    dU[:, 0:2] = 0.6  # CH fields: not unknowns of the NS block
    dU[:, 2] = x[:, 0] ** 2
    dU[:, 3] = x[:, 1] * x[:, 2]
    dU[:, 4] = x[:, 0]
    dU[:, 5] = 1 + 2 * x[:, 0] - x[:, 1]
    J = q.jvp(_ns_params(), U, U.copy(), dU, block=NS)
    one, x1, x2 = poly(1.0), poly(0.0, 1.0), poly(0.0, 0.0, 1.0)
    T = _tables(n1d, h, {"I0": (one, 0), "D0": (one, 1), "X1": (x1, 0), "X2": (x2, 0), "DX1": (x1, 1),
                         "DX2": (x2, 1), "Dp": (poly(1.0, 2.0), 1), "Np": (poly(1.0, 2.0), 0)})
    ix, iy, iz = _lattice(q, level)
    g = lambda k, i: T[k][i]
    I = lambda a, b, c: g(a, ix) * g(b, iy) * g(c, iz)
    # integrals of N_a dv_i, of d_i N_a dp, of d_i N_a div dv (div dv = 2x + z),
    # of grad N_a . grad dv_i
    Ndv = [I("X2", "I0", "I0"), I("I0", "X1", "X1"), I("X1", "I0", "I0")]
    Ddp = [I("Dp", "I0", "I0") - I("D0", "X1", "I0"), I("Np", "D0", "I0") - I("I0", "DX1", "I0"),
           I("Np", "I0", "D0") - I("I0", "X1", "D0")]
    Ddiv = [2 * I("DX1", "I0", "I0") + I("D0", "I0", "X1"), 2 * I("X1", "D0", "I0") + I("I0", "D0", "X1"),
            2 * I("X1", "I0", "D0") + I("I0", "I0", "DX1")]
    Lap = [2 * I("DX1", "I0", "I0"), I("I0", "D0", "X1") + I("I0", "X1", "D0"), I("D0", "I0", "I0")]
    mom = [rho / dt * Ndv[i] - Ddp[i] / (2 * We) + rho * tau_c / (2 * We) * Ddiv[i] + eta / (2 * Re) * Lap[i]
           for i in range(3)]
    Ndiv = 2 * I("X1", "I0", "I0") + I("I0", "I0", "X1")
    Gdv = I("DX2", "I0", "I0") + I("I0", "DX1", "X1") + I("X1", "I0", "D0")  # grad N . dv
    Gdp = 2 * I("D0", "I0", "I0") - I("I0", "D0", "I0")                      # grad N . grad dp
    GLap = 2 * I("D0", "I0", "I0")                                           # grad N . lap dv
    cont = 0.5 * Ndiv + tau_m / rho * (rho / dt * Gdv + Gdp / (2 * We) - eta / (2 * Re) * GLap)
    inner = _interior(q)
    scale = max(max(np.abs(r).max() for r in mom), np.abs(cont).max())
    for i in range(3):
        assert np.abs(J[inner, 2 + i] - mom[i][inner]).max() <= 1e-12 * scale, i
    free = (q.bflags & 2) == 0
    assert np.abs(J[free, 5] - cont[free]).max() <= 1e-12 * scale
    assert np.all(J[:, 0:2] == 0.0)


def test_ns_jvp_is_the_derivative_of_the_residual():
    m = _adaptive_meshes()[0]
    q = m.q2()
    rng = np.random.default_rng(12)
    n = q.n_nodes
    U0 = np.zeros((n, 6))
    U0[:, 0] = rng.uniform(-1.1, 1.1, n)
    U0[:, 1] = rng.normal(0, 0.5, n)
    U0[:, 2:5] = rng.normal(0, 0.3, (n, 3))
    U0[:, 5] = rng.normal(0, 1.0, n)
    U1 = U0 + rng.normal(0, 0.05, U0.shape)
    dU = rng.normal(0, 1.0, U0.shape)
    p = _ns_params()
    J = q.jvp(p, U1, U0, dU, block=NS)
    e = 1e-6
    dN = dU.copy()
    dN[:, :2] = 0.0
    fd = (q.residual(p, U1 + e * dN, U0, block=NS) - q.residual(p, U1 - e * dN, U0, block=NS)) / (2 * e)
    err = np.linalg.norm(J[:, 2:] - fd[:, 2:]) / np.linalg.norm(fd[:, 2:])
    assert err < 1e-7, err


@pytest.mark.parametrize("level", [1, 2])
def test_ns_capillary_balance_closed_form(level):
    """At rest with phi~ = b x + c x^2 inside (-1, 1), no gravity and constant
    mu, the strong capillary divergence (Cn/We) d/dx (dphi~/dx)^2 = (Cn/We) 2
    phi' phi'' (its Laplacian part included) is balanced by a quadratic
    pressure, so R_m = R_c = 0 and the rows are the Galerkin capillary and
    pressure integrals."""
    m, q = uniform(level)
    h = 2.0 ** -level
    n1d = 2 ** (level + 1) + 1
    Cn, We = P["Cn"], P["We"]
    b, c, P0 = 0.3, 0.2, 0.1
    # (1/We) p' = -(Cn/We) 2 phi' phi'' = -(Cn/We) 4c (b + 2c x)
    pc = poly(P0, -Cn * 4 * c * b, -Cn * 4 * c * c)
    x = q.node_xyz()
    U = np.zeros((q.n_nodes, 6))
    U[:, 0] = b * x[:, 0] + c * x[:, 0] ** 2
    U[:, 1] = 0.7
    U[:, 5] = pc(x[:, 0])
    R = q.residual(_ns_params(g=(0.0, 0.0, 0.0)), U, U.copy(), block=NS)
    dphi2 = poly(b, 2 * c) ** 2
    one = poly(1.0)
    T = _tables(n1d, h, {"I0": (one, 0), "D0": (one, 1), "Dcap": (dphi2, 1), "Dp": (pc, 1), "Np": (pc, 0)})
    ix, iy, iz = _lattice(q, level)
    g = lambda k, i: T[k][i]
    rx = -(Cn / We) * g("Dcap", ix) * g("I0", iy) * g("I0", iz) - g("Dp", ix) * g("I0", iy) * g("I0", iz) / We
    ry = -g("Np", ix) * g("D0", iy) * g("I0", iz) / We
    rz = -g("Np", ix) * g("I0", iy) * g("D0", iz) / We
    inner = _interior(q)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for f, ref in ((2, rx), (3, ry), (4, rz)):
        assert np.abs(R[inner, f] - ref[inner]).max() <= 1e-12 * scale, f
    assert np.abs(R[(q.bflags & 2) == 0, 5]).max() <= 1e-12 * scale
