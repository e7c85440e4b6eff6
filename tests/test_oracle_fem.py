"""Pins of the oracle's element loop (Sec. 3 and 3.4) against closed forms,
exact algebraic identities and finite differences.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or coefficient, a transposed index, the wrong time level) fails
at least one of them."""
import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W
from tests import fem_closed_forms as CF
from tests import uniform_quadrature as UQ

CH, NS = 0, 1


def P(orc, **kw):
    base = dict(Cn=0.3, Pe=2.0, Re=7.0, We=3.0, Fr=1.5, rho_minus=0.25, eta_minus=0.4,
                dt=0.05, g=(0.0, -1.0, 0.0), C_I=6.0, flux_mode=0)
    base.update(kw)
    return orc.Params.make(**base)


@pytest.fixture(scope="module")
def uni3(orc):
    m = orc.Mesh((1, 1, 1), 3, 3)
    return m, CF.lattice_index(m.nodes, 3)


@pytest.fixture(scope="module")
def adaptive(orc):
    leaves = W.random_leaves((1, 1, 1), 4, 7, p_split=0.3, level_min=2)
    m = orc.Mesh((1, 1, 1), 0, 4, leaves=leaves)
    assert m.hang_xyz.shape[0] > 50
    return m


def interior_centre(idx):
    c = idx.shape[0] // 2
    return c, c, c


# ------------------------------------------------------- Q1 stencils ------
def test_mass_stencil(orc, uni3):
    """(q, (phi^{k+1}-phi^k)/dt) with phi^{k+1} = dt e_n is the mass matrix
    column: h^3 * (8/27, 2/27, 1/54, 1/216) for centre, face, edge, corner."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc)
    i, j, k = interior_centre(idx)
    n = idx[i, j, k]
    U1 = np.zeros((m.n_nodes, 6))
    U1[n, 0] = p.dt
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    expect = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for o in CF.offsets():
        nb = idx[i + o[0], j + o[1], k + o[2]]
        assert R[nb, 0] == pytest.approx(expect[sum(map(abs, o))] * h ** 3, rel=1e-14)
        assert R[nb, 0] == pytest.approx(CF.mass(o, h), rel=1e-14)
    assert R[:, 0].sum() == pytest.approx(h ** 3, rel=1e-14)


def test_stiffness_stencil(orc, uni3):
    """1/(Pe Cn) (dq/dx_i, dmu~/dx_i) with mu~ = e_n and Pe Cn = 1 is the
    stiffness column: (8/3, 0, -1/6, -1/12) h; row sum 0."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, Cn=0.5, Pe=2.0)
    i, j, k = interior_centre(idx)
    n = idx[i, j, k]
    U1 = np.zeros((m.n_nodes, 6))
    U1[n, 1] = 2.0
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    expect = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}
    for o in CF.offsets():
        nb = idx[i + o[0], j + o[1], k + o[2]]
        assert R[nb, 0] == pytest.approx(expect[sum(map(abs, o))] * h, rel=1e-13, abs=1e-15)
    assert abs(R[:, 0].sum()) < 1e-14


def test_cahn_number_and_mass_in_mu_row(orc, uni3):
    """mu row: -(q, mu~) + Cn^2 (dq/dx_i, dphi~/dx_i); at phi~ = e_n the psi'
    term contributes (q, phi~^3 - phi~) evaluated at the Gauss points."""
    m, idx = uni3
    h = 1 / 8
    Cn = 0.3
    p = P(orc, Cn=Cn)
    i, j, k = interior_centre(idx)
    n = idx[i, j, k]
    U1 = np.zeros((m.n_nodes, 6))
    U1[n, 1] = 2.0   # mu~ = e_n
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    for o in CF.offsets():
        nb = idx[i + o[0], j + o[1], k + o[2]]
        assert R[nb, 1] == pytest.approx(-CF.mass(o, h), rel=1e-14)
    U1[:] = 0
    U1[n, 0] = 2e-6  # phi~ = 1e-6 e_n: psi' ~ -phi~ (cubic part 1e-18)
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    for o in CF.offsets():
        nb = idx[i + o[0], j + o[1], k + o[2]]
        exp = 1e-6 * (Cn ** 2 * CF.stiffness(o, h) - CF.mass(o, h))
        assert R[nb, 1] == pytest.approx(exp, rel=1e-9, abs=1e-22)


# ----------------------------------------- hanging-node gather/scatter ----
def test_partition_of_unity_adaptive(orc, adaptive):
    m = adaptive
    p = P(orc)
    U1 = np.zeros((m.n_nodes, 6))
    U1[:, 0] = p.dt
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    assert R[:, 0].sum() == pytest.approx(1.0, rel=1e-14)
    assert (R[:, 0] > 0).all()


def test_patch_test_adaptive(orc, adaptive):
    """For a linear mu~ the stiffness rows of interior nodes vanish on a 2:1
    mesh with hanging nodes (the constrained space reproduces linears)."""
    m = adaptive
    p = P(orc, Cn=1.0, Pe=1.0)
    x = m.node_xyz()
    U1 = np.zeros((m.n_nodes, 6))
    U1[:, 1] = 2 * (0.3 + 1.7 * x[:, 0] - 0.6 * x[:, 1] + 2.2 * x[:, 2])
    R = m.residual(p, CH, U1, np.zeros_like(U1))
    interior = (m.bflags & 1) == 0
    assert interior.sum() > 100
    assert np.abs(R[interior, 0]).max() < 1e-13
    assert np.abs(R[~interior, 0]).max() > 1e-3


# ------------------------------------------------ CH block identities ----
def random_ch_state(m, seed, amp=0.8):
    rng = np.random.default_rng(seed)
    n = m.n_nodes
    U0 = np.zeros((n, 6))
    U1 = np.zeros((n, 6))
    U0[:, 0] = rng.uniform(-amp, amp, n)
    U1[:, 0] = U0[:, 0] + rng.normal(0, 0.1, n)
    U0[:, 1] = rng.normal(0, 0.5, n)
    U1[:, 1] = rng.normal(0, 0.5, n)
    U0[:, 2:5] = rng.normal(0, 0.3, (n, 3))
    U1[:, 2:5] = rng.normal(0, 0.3, (n, 3))
    U0[:, 5] = rng.normal(0, 1, n)
    U1[:, 5] = rng.normal(0, 1, n)
    return U1, U0


def test_ch_constant_state(orc, adaptive):
    m = adaptive
    p = P(orc)
    c = 0.37
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = c
    U[:, 1] = c ** 3 - c
    R = m.residual(p, CH, U, U)
    assert np.abs(R).max() < 1e-15


def test_ch_mass_identity(orc, adaptive):
    """Testing with q = 1 (Prop. 1): the phi rows sum to the change of the
    integral of phi over dt, for any states; the integral of a trilinear
    field over a cube of side h is h^3 times the mean of its corner values."""
    m = adaptive
    p = P(orc)
    U1, U0 = random_ch_state(m, 3)
    R = m.residual(p, CH, U1, U0)

    def integral(u):
        hv = np.array([(m.hang_w[m.hang_off[i]:m.hang_off[i + 1]] *
                        u[m.hang_ids[m.hang_off[i]:m.hang_off[i + 1]]]).sum()
                       for i in range(m.hang_xyz.shape[0])])
        cv = np.where(m.elem >= 0, u[np.maximum(m.elem, 0)], hv[np.maximum(-1 - m.elem, 0)])
        h = 2.0 ** (-m.leaves[:, 3].astype(float))
        return float((h ** 3 * cv.mean(axis=1)).sum())

    lhs = R[:, 0].sum()
    rhs = (integral(U1[:, 0]) - integral(U0[:, 0])) / p.dt
    assert lhs == pytest.approx(rhs, rel=1e-12)
    mass1, _ = m.diagnostics(p, U1)
    assert mass1 == pytest.approx(integral(U1[:, 0]), rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_ch_energy_identity(orc, uni3, seed):
    """dt mu~^T R_phi + (phi^{k+1}-phi^k)^T R_mu equals
    F(phi^{k+1}) - F(phi^k) - int phi~/4 (dphi)^3 - dt int grad mu~ . v~ phi~
    + dt/(Pe Cn) ||grad mu~||^2 with F = int psi + Cn^2/2 |grad phi|^2.
    This is the energy argument of Sec. 3.2 (Prop. 2 is exact for the quartic
    psi with the midpoint): it holds for any states, at quadrature level."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, Cn=0.3, Pe=2.0, dt=0.05)
    U1, U0 = random_ch_state(m, 10 + seed)
    R = m.residual(p, CH, U1, U0)
    mut = 0.5 * (U1[:, 1] + U0[:, 1])
    dphi = U1[:, 0] - U0[:, 0]
    lhs = p.dt * (mut * R[:, 0]).sum() + (dphi * R[:, 1]).sum()

    def F(phi):
        v, g = UQ.qp_fields(phi, idx, h)
        return UQ.integrate(0.25 * (v ** 2 - 1) ** 2 + 0.5 * p.Cn ** 2 * (g ** 2).sum(axis=1), h)

    pt, _ = UQ.qp_fields(0.5 * (U1[:, 0] + U0[:, 0]), idx, h)
    dp, _ = UQ.qp_fields(dphi, idx, h)
    _, gmu = UQ.qp_fields(mut, idx, h)
    vt = [UQ.qp_fields(0.5 * (U1[:, 2 + d] + U0[:, 2 + d]), idx, h)[0] for d in range(3)]
    adv = UQ.integrate(sum(gmu[:, d] * vt[d] for d in range(3)) * pt, h)
    rhs = (F(U1[:, 0]) - F(U0[:, 0]) - UQ.integrate(pt / 4 * dp ** 3, h)
           - p.dt * adv + p.dt / (p.Pe * p.Cn) * UQ.integrate((gmu ** 2).sum(axis=1), h))
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-14)


# ------------------------------------------------ NS block special cases --
@pytest.mark.parametrize("phi,g", [(1.0, (0.0, -1.0, 0.0)), (-1.0, (0.0, -1.0, 0.0)),
                                   (1.0, (0.0, 0.0, -1.0)), (-1.3, (0.6, 0.0, -0.8))])
def test_ns_hydrostatic(orc, adaptive, phi, g):
    """v = 0, constant phi (rho constant, pulled back when |phi| > 1), constant
    mu (J = 0) and p = (We/Fr) rho g.x at both time levels: (1/We) grad p =
    rho g / Fr, so R_m = R_c = 0 and every row vanishes."""
    m = adaptive
    p = P(orc, g=g)
    rho_m = p.rho_minus
    rho = 0.5 * (1 - rho_m) * np.clip(phi, -1, 1) + 0.5 * (1 + rho_m)
    x = m.node_xyz()
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = phi
    U[:, 1] = 0.7
    U[:, 5] = (p.We / p.Fr) * rho * (x @ np.array(g))
    R = m.residual(p, NS, U, U)
    assert np.abs(R[:, 2:]).max() < 1e-13
    # with the gravity term dropped from the pressure the rows do not vanish
    U2 = U.copy()
    U2[:, 5] = 0
    R2 = m.residual(p, NS, U2, U2)
    assert np.abs(R2[:, 2:]).max() > 1e-4


def test_ns_uniform_velocity(orc, adaptive):
    """A uniform velocity at both time levels (boundary rows carry it) on top of
    the hydrostatic state: every convective term vanishes."""
    m = adaptive
    p = P(orc)
    x = m.node_xyz()
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 1.0
    U[:, 2:5] = [0.3, -0.2, 0.5]
    U[:, 5] = (p.We / p.Fr) * (x @ np.array(p.g[:]))
    R = m.residual(p, NS, U, U)
    assert np.abs(R[:, 2:]).max() < 1e-13


def _tau_m(p, h, v=(0.0, 0.0, 0.0), rho=1.0, eta=1.0, J=(0.0, 0.0, 0.0)):
    G = 4 / h ** 2
    v = np.array(v)
    br = (4 / p.dt ** 2 + G * v @ v + G * (v @ np.array(J)) / (rho * p.Pe)
          + p.C_I * (eta / (rho * p.Re)) ** 2 * 3 * G ** 2)
    return br ** -0.5


def test_ns_capillary_closed_form(orc, uni3):
    """phi~ = xy (phi^k = 2xy - 3, phi^{k+1} = 3 pulled back to 1, so rho = eta = 1),
    v = p = 0, no gravity: the capillary divergence is (Cn/We)(x, y, 0) and, by
    exact integration by parts on interior rows,
      R_v,a = [Cn/We + 3 tau_m^2 (Cn/We)^2] (x_a, y_a, 0) h^3,
      R_p,a = -2 tau_m (Cn/We) h^3.
    Pins the capillary Galerkin term (with phi~), the strong capillary term,
    the continuity stabilisation sign and the tau_m^2 R R term."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, g=(0.0, 0.0, 0.0))
    x = m.node_xyz()
    U1 = np.zeros((m.n_nodes, 6))
    U0 = np.zeros((m.n_nodes, 6))
    U1[:, 0] = 3.0
    U0[:, 0] = 2 * x[:, 0] * x[:, 1] - 3.0
    R = m.residual(p, NS, U1, U0)
    tm = _tau_m(p, h)
    cw = p.Cn / p.We
    inner = np.all((m.nodes > 0) & (m.nodes < 8), axis=1)
    a = np.nonzero(inner)[0]
    np.testing.assert_allclose(R[a, 2], (cw + 3 * tm ** 2 * cw ** 2) * x[a, 0] * h ** 3, rtol=1e-12)
    np.testing.assert_allclose(R[a, 3], (cw + 3 * tm ** 2 * cw ** 2) * x[a, 1] * h ** 3, rtol=1e-12)
    assert np.abs(R[a, 4]).max() < 1e-17
    np.testing.assert_allclose(R[a, 5], -2 * tm * cw * h ** 3, rtol=1e-12)


def _jvp_closed_form(p, h, o, c, J, rho=1.0):
    """Interior-row JVP entries for dv = e_x at node b = a + o, around a base
    state with R_m = R_c = 0, uniform velocity c, constant flux J, constant
    rho and eta = 1 (terms proportional to the base residuals vanish):
      x-row: M/dt + rho/2 C_c + 1/(2Pe) C_J + (1/(2 Re)) K
             + tau_m (c.grad N_a)(rho N_b/dt + rho/2 c.grad N_b + 1/(2Pe) J.grad N_b)
             + (1/Pe)(tau_m/rho)(J.grad N_a)(rho N_b/dt + ...)
             + (rho tau_c/(2 We)) dN_a/dx dN_b/dx
      y,z rows: (rho tau_c/(2 We)) dN_a/dx_i dN_b/dx
      p row: (N_a, dN_b/dx)/2 + (tau_m/rho)(dN_a/dx, rho N_b/dt + ...)"""
    tm = _tau_m(p, h, v=c, rho=rho, J=J)
    tc = h ** 2 / (12 * tm)
    c = np.array(c)
    J = np.array(J)
    M = CF.mass(o, h)
    conv = lambda w: sum(w[j] * CF.n_dN(j, o, h) for j in range(3))          # (N_a, w.grad N_b)
    supg_m = lambda w: sum(w[j] * CF.dN_n(j, o, h) for j in range(3))        # (w.grad N_a, N_b)
    supg_k = lambda w1, w2: sum(w1[j] * w2[k] * CF.grad_grad(j, k, o, h)
                                for j in range(3) for k in range(3))
    # dR_m,x tested against (c.grad N_a) tau_m and (J.grad N_a) tau_m / (rho Pe)
    def tested(w, coeff):
        return coeff * (rho * supg_m(w) / p.dt + 0.5 * rho * supg_k(w, c)
                        + 0.5 / p.Pe * supg_k(w, J))
    row_x = (rho * M / p.dt + 0.5 * rho * conv(c) + 0.5 / p.Pe * conv(J)
             + 0.5 / p.Re * CF.stiffness(o, h)
             + tested(c, tm) + tested(J, tm / (rho * p.Pe))
             + rho * tc / (2 * p.We) * CF.grad_grad(0, 0, o, h))
    row_y = rho * tc / (2 * p.We) * CF.grad_grad(1, 0, o, h)
    row_z = rho * tc / (2 * p.We) * CF.grad_grad(2, 0, o, h)
    e_x = np.array([1.0, 0.0, 0.0])
    row_p = (0.5 * CF.n_dN(0, o, h)
             + (tm / rho) * (rho * CF.dN_n(0, o, h) / p.dt + 0.5 * rho * supg_k(e_x, c)
                             + 0.5 / p.Pe * supg_k(e_x, J)))
    return np.array([row_x, row_y, row_z, row_p])


@pytest.mark.parametrize("case", ["rest", "uniform_flow", "flux", "both"])
def test_ns_jvp_closed_form(orc, uni3, case):
    """Linearisation about states where R_m = R_c = 0 (so every term that
    multiplies a base residual, including d tau_m, drops out): the JVP rows of
    interior nodes are tensor-product closed forms.  'uniform_flow' pins the
    Galerkin and fine-scale convection terms with tau_m(v); 'flux' pins the
    mass-flux terms with J = -(alpha/Cn) grad mu~."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, dt=0.02, rho_minus=0.25)
    x = m.node_xyz()
    c = {"rest": (0, 0, 0), "uniform_flow": (0.4, -0.3, 0.25), "flux": (0, 0, 0),
         "both": (0.2, 0.1, -0.3)}[case]
    grad_mu = {"rest": (0, 0, 0), "uniform_flow": (0, 0, 0), "flux": (0.5, 0.8, -0.3),
               "both": (-0.4, 0.3, 0.6)}[case]
    alpha = 0.5 * (1 - p.rho_minus)
    J = tuple(-alpha / p.Cn * gm for gm in grad_mu)
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 1.0
    U[:, 1] = x @ np.array(grad_mu, float)
    U[:, 2:5] = c
    U[:, 5] = (p.We / p.Fr) * (x @ np.array(p.g[:]))
    i, j, k = interior_centre(idx)
    b = idx[i, j, k]
    dU = np.zeros_like(U)
    dU[b, 2] = 1.0
    out = m.jvp(p, NS, U, U, dU)
    for o in CF.offsets():
        a = idx[i - o[0], j - o[1], k - o[2]]   # b = a + o
        exp = _jvp_closed_form(p, h, o, c, J)
        np.testing.assert_allclose(out[a, 2:], exp, rtol=1e-11, atol=1e-14 * np.abs(exp).max())


# ------------------------------------------- Jacobian-vector products ----
def random_state(m, seed):
    rng = np.random.default_rng(seed)
    n = m.n_nodes
    U0 = np.zeros((n, 6))
    U0[:, 0] = rng.uniform(-1.1, 1.1, n)
    U0[:, 1] = rng.normal(0, 0.5, n)
    U0[:, 2:5] = rng.normal(0, 0.3, (n, 3))
    U0[:, 5] = rng.normal(0, 1, n)
    U1 = U0 + rng.normal(0, 0.05, U0.shape)
    return U1, U0


@pytest.mark.parametrize("block", [CH, NS])
@pytest.mark.parametrize("meshkind", ["uniform4", "adaptive"])
def test_jvp_matches_central_differences(orc, adaptive, block, meshkind):
    m = orc.Mesh((1, 1, 1), 2, 2) if meshkind == "uniform4" else adaptive
    p = P(orc, dt=0.05)
    U1, U0 = random_state(m, 5)
    f = slice(0, 2) if block == CH else slice(2, 6)
    dU = np.zeros_like(U1)
    dU[:, f] = np.random.default_rng(6).normal(0, 1, (U1.shape[0], f.stop - f.start))
    Jd = m.jvp(p, block, U1, U0, dU)
    eps = 1e-6 * np.linalg.norm(U1) / np.linalg.norm(dU)
    Rp = m.residual(p, block, U1 + eps * dU, U0)
    Rm = m.residual(p, block, U1 - eps * dU, U0)
    fd = (Rp - Rm) / (2 * eps)
    err = np.linalg.norm(fd[:, f] - Jd[:, f]) / np.linalg.norm(Jd[:, f])
    assert err < 1e-7
    other = slice(2, 6) if block == CH else slice(0, 2)
    assert np.abs(Jd[:, other]).max() == 0.0


@pytest.mark.parametrize("block", [CH, NS])
def test_jvp_linearity(orc, adaptive, block):
    m = adaptive
    p = P(orc)
    U1, U0 = random_state(m, 8)
    rng = np.random.default_rng(9)
    d1, d2 = rng.normal(size=U1.shape), rng.normal(size=U1.shape)
    a, b = 0.7, -1.9
    lhs = m.jvp(p, block, U1, U0, a * d1 + b * d2)
    rhs = a * m.jvp(p, block, U1, U0, d1) + b * m.jvp(p, block, U1, U0, d2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


@pytest.mark.parametrize("block", [CH, NS])
def test_diag_blocks_are_jacobian_diagonal(orc, block):
    """Node-block diagonal vs. columns of the Jacobian probed with unit
    directions, on a small 2:1 mesh."""
    leaves = W.random_leaves((1, 1, 1), 3, 2, p_split=0.4, level_min=1)
    m = orc.Mesh((1, 1, 1), 0, 3, leaves=leaves)
    assert m.hang_xyz.shape[0] > 0
    p = P(orc)
    U1, U0 = random_state(m, 12)
    B = m.diag_blocks(p, block, U1, U0)
    f0, nf = (0, 2) if block == CH else (2, 4)
    rng = np.random.default_rng(0)
    for n in rng.choice(m.n_nodes, 12, replace=False):
        for fc in range(nf):
            dU = np.zeros_like(U1)
            dU[n, f0 + fc] = 1.0
            col = m.jvp(p, block, U1, U0, dU)
            np.testing.assert_allclose(B[n, :, fc], col[n, f0:f0 + nf], rtol=1e-12, atol=1e-14)


def test_boundary_rows(orc, adaptive):
    m = adaptive
    p = P(orc)
    U1, U0 = random_state(m, 13)
    R = m.residual(p, NS, U1, U0)
    b = (m.bflags & 1) != 0
    np.testing.assert_array_equal(R[b, 2:5], U1[b, 2:5] - U0[b, 2:5])
    assert R[0, 5] == U1[0, 5] - U0[0, 5]
    assert np.abs(R[:, :2]).max() == 0.0


def test_tau_bracket_error(orc, uni3):
    """A velocity against a strong flux makes v.G.J negative enough to turn the
    tau_m bracket non-positive: reported as an error, not a NaN."""
    m, _ = uni3
    p = P(orc, dt=10.0, Re=1e6)
    x = m.node_xyz()
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 0.0
    U[:, 1] = 50.0 * x[:, 0]           # J = -(alpha/Cn) * 50 e_x
    U[:, 2] = 1.0                       # v along +x: v.G.J < 0
    with pytest.raises(RuntimeError, match="tau_m"):
        m.residual(p, NS, U, U)


@pytest.mark.parametrize("block", [CH, NS])
@pytest.mark.parametrize("meshkind", ["uniform4", "adaptive"])
def test_full_jvp_matches_central_differences(orc, adaptive, block, meshkind):
    """The block's rows of the coupled Jacobian (derivatives with respect to
    all six fields, the cross terms included) against central differences of
    the residual; with the other block's seeds zero it is the block JVP."""
    m = orc.Mesh((1, 1, 1), 2, 2) if meshkind == "uniform4" else adaptive
    p = P(orc, dt=0.05)
    U1, U0 = random_state(m, 15)
    f = slice(0, 2) if block == CH else slice(2, 6)
    other = slice(2, 6) if block == CH else slice(0, 2)
    dU = np.random.default_rng(16).normal(0, 1, U1.shape)
    Jd = m.jvp_full(p, block, U1, U0, dU)
    eps = 1e-6 * np.linalg.norm(U1) / np.linalg.norm(dU)
    fd = (m.residual(p, block, U1 + eps * dU, U0) - m.residual(p, block, U1 - eps * dU, U0)) / (2 * eps)
    err = np.linalg.norm(fd[:, f] - Jd[:, f]) / np.linalg.norm(Jd[:, f])
    assert err < 1e-7, err
    assert np.abs(Jd[:, other]).max() == 0.0
    # the cross part is there, and without it the block JVP comes back
    dB = np.zeros_like(dU)
    dB[:, f] = dU[:, f]
    assert np.array_equal(m.jvp_full(p, block, U1, U0, dB), m.jvp(p, block, U1, U0, dB))
    cross = Jd[:, f] - m.jvp(p, block, U1, U0, dB)[:, f]
    assert np.linalg.norm(cross) > 1e-3 * np.linalg.norm(Jd[:, f])


@pytest.mark.parametrize("block", [CH, NS])
def test_thread_count_does_not_change_results(orc, adaptive, block):
    """Element vectors are added in element order after the parallel loop, so
    the residual, the JVP and the diagonal blocks are bitwise the same on one
    thread and on all of them (the CPU baseline times both)."""
    m = adaptive
    p = P(orc)
    U1, U0 = random_state(m, 10)
    d = np.random.default_rng(11).normal(size=U1.shape)
    cores = orc.num_threads()
    try:
        orc.set_num_threads(1)
        one = (m.residual(p, block, U1, U0), m.jvp(p, block, U1, U0, d), m.diag_blocks(p, block, U1, U0))
    finally:
        orc.set_num_threads(cores)
    many = (m.residual(p, block, U1, U0), m.jvp(p, block, U1, U0, d), m.diag_blocks(p, block, U1, U0))
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


# ------------------- linearisation about a state with R_m != 0, grad eta != 0 --
def _jvp_rows_general(p, h, a, b, m, c, J, bvec, rho, eta_w, e, d0):
    """Interior-row JVP entries (momentum x, y, z and continuity rows of node a)
    for the direction dv = N_b e_m, about a base state with uniform velocity
    c (grad v~ = 0), constant mass flux J, constant density rho, a constant
    strong momentum residual R_m = bvec, R_c = 0, and a viscosity that is
    linear along axis d0 (weight coefficients eta_w, gradient e); tau_m is
    constant (C_I = 0 when eta varies).  The derivative of each term of Def. 2
    (with readings A2, A3, A6, A7) is written out:
      dR_m,i = delta_im L_b,  L_b = rho N_b/dt + rho/2 c.grad N_b
                                   + 1/(2Pe) J.grad N_b - 1/(2Re) e.grad N_b
      d tau_m = D N_b,        D = -tau_m^3 G (c_m + J_m/(2 rho Pe)) / 2
      dR_c = dN_b/dx_m / 2.
    Every integral is an exact tensor product of 1-D hat integrals."""
    eta_const = eta_w[0] if len(eta_w) == 1 else None
    G = 4 / h ** 2
    c, J, bvec, e = (np.asarray(v, float) for v in (c, J, bvec, e))
    visc = 0.0 if eta_const is None else p.C_I * (eta_const / (rho * p.Re)) ** 2 * 3 * G ** 2
    assert eta_const is not None or p.C_I == 0.0
    T0 = (4 / p.dt ** 2 + G * c @ c + G * (c @ J) / (rho * p.Pe) + visc) ** -0.5
    tc = 1.0 / (3 * G * T0)
    D = -0.5 * T0 ** 3 * G * (c[m] + J[m] / (2 * rho * p.Pe))

    def I(A, B, w=None):
        return CF.tensor_integral(a, A, b, B, h, None if w is None else {d0: w})

    def IL(A):   # int A L_b
        return (rho / p.dt * I(A, None)
                + sum((0.5 * rho * c[k] + 0.5 / p.Pe * J[k] - 0.5 / p.Re * e[k]) * I(A, k)
                      for k in range(3)))

    rows = np.zeros(4)
    for i in range(3):
        t = 0.0
        if i == m:
            t += rho / p.dt * I(None, None)                                  # (w, rho dv/dt)
            t += sum(0.5 * rho * c[j] * I(None, j) for j in range(3))        # Galerkin convection
            t += sum(0.5 / p.Pe * J[j] * I(None, j) for j in range(3))       # (w, J.grad v)/Pe
            t -= sum(0.5 * T0 * bvec[j] * I(None, j) for j in range(3))      # -(w_i, tau R_m,j d_j v_i)
            t += 0.5 / p.Re * sum(I(k, k, eta_w) for k in range(3))          # (grad w, eta grad v)/Re
            t += T0 * sum(c[j] * IL(j) for j in range(3))                    # SUPG: tau c.grad w dR_m
            t -= T0 ** 2 / rho * sum(bvec[j] * IL(j) for j in range(3))
            t += T0 / (rho * p.Pe) * sum(J[j] * IL(j) for j in range(3))
        t += 0.5 * T0 * bvec[i] * I(m, None)                                 # dv~_j tau R_m,i
        t += D * bvec[i] * sum(c[j] * I(j, None) for j in range(3))          # c_j d tau R_m,i
        t -= 2 * T0 * D / rho * bvec[i] * sum(bvec[j] * I(j, None) for j in range(3))
        t -= T0 ** 2 / rho * bvec[i] * IL(m)
        t += D / (rho * p.Pe) * bvec[i] * sum(J[j] * I(j, None) for j in range(3))
        t += rho * tc / (2 * p.We) * I(i, m)                                 # grad-div (tau_c R_c)
        rows[i] = t
    rows[3] = (0.5 * I(None, m) + D / rho * sum(bvec[j] * I(j, None) for j in range(3))
               + T0 / rho * IL(m))
    return rows


@pytest.mark.parametrize("m_axis", [0, 1, 2])
def test_ns_jvp_closed_form_with_momentum_residual(orc, uni3, m_axis):
    """phi = 1 (rho = eta = 1), uniform v~ = c, mu~ linear (constant J), and a
    pressure gradient that does not balance gravity, so R_m is a nonzero
    constant b.  Pins the fine-scale convection term -(w_i, tau_m R_m,j
    dv~_i/dx_j) with its index order (reading A3), d tau_m, and the products of
    R_m with the SUPG and PSPG test functions."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, dt=0.02, rho_minus=0.25, Cn=0.3, Pe=2.0, We=3.0, Fr=1.5)
    x = m.node_xyz()
    c = np.array([0.3, -0.2, 0.45])
    grad_mu = np.array([0.5, -0.7, 0.2])
    bvec = np.array([0.7, -0.4, 0.9])
    alpha = 0.5 * (1 - p.rho_minus)
    J = -(alpha / p.Cn) * grad_mu
    g = np.array(p.g[:])
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 1.0
    U[:, 1] = x @ grad_mu
    U[:, 2:5] = c
    U[:, 5] = p.We * (x @ (bvec + g / p.Fr))     # (1/We) grad p - g/Fr = b
    i, j, k = interior_centre(idx)
    bnode = idx[i, j, k]
    dU = np.zeros_like(U)
    dU[bnode, 2 + m_axis] = 1.0
    out = m.jvp(p, NS, U, U, dU)
    for o in CF.offsets():
        a = (i - o[0], j - o[1], k - o[2])
        exp = _jvp_rows_general(p, h, a, (i, j, k), m_axis, c, J, bvec, 1.0, (1.0,), (0, 0, 0), 0)
        np.testing.assert_allclose(out[idx[a], 2:], exp, rtol=1e-11, atol=1e-13 * np.abs(exp).max())


@pytest.mark.parametrize("m_axis", [0, 1, 2])
def test_ns_jvp_closed_form_with_viscosity_gradient(orc, uni3, m_axis):
    """Density ratio 1 (rho = 1, J = 0), viscosity ratio 0.3 and phi linear
    inside (-1, 1), so eta is linear and grad eta = gamma grad phi^{k+1}
    (reading A22); C_I = 0 keeps tau_m constant.  Pins the -(1/Re) grad eta .
    grad v~ term of R_m (through the stabilised test functions) and the
    Galerkin viscous term with a varying eta, next to R_m = b != 0."""
    m, idx = uni3
    h = 1 / 8
    p = P(orc, dt=0.02, rho_minus=1.0, eta_minus=0.3, Re=0.8, C_I=0.0)
    x = m.node_xyz()
    c = np.array([0.25, 0.4, -0.3])
    bvec = np.array([-0.5, 0.6, 0.8])
    d0, s, phic = 0, 1.2, 0.1                          # phi = phic + s (x - 1/2)
    gamma, xi = 0.5 * (1 - p.eta_minus), 0.5 * (1 + p.eta_minus)
    eta_w = (xi + gamma * (phic - 0.5 * s), gamma * s)
    e = np.zeros(3)
    e[d0] = gamma * s
    g = np.array(p.g[:])
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = phic + s * (x[:, d0] - 0.5)
    U[:, 1] = 0.3
    U[:, 2:5] = c
    U[:, 5] = p.We * (x @ (bvec + g / p.Fr))
    i, j, k = interior_centre(idx)
    bnode = idx[i, j, k]
    dU = np.zeros_like(U)
    dU[bnode, 2 + m_axis] = 1.0
    out = m.jvp(p, NS, U, U, dU)
    for o in CF.offsets():
        a = (i - o[0], j - o[1], k - o[2])
        exp = _jvp_rows_general(p, h, a, (i, j, k), m_axis, c, (0, 0, 0), bvec, 1.0, eta_w, e, d0)
        np.testing.assert_allclose(out[idx[a], 2:], exp, rtol=1e-11, atol=1e-13 * np.abs(exp).max())


# ------------------------------------------------------------ energy --------
def _psi_integral_gauss(a, s, h):
    """int_0^1 psi(a + s y) dy for psi = (phi^2 - 1)^2 / 4 as the per-cell
    two-point Gauss rule computes it: the exact integral minus the rule's
    error, which for a quartic is exactly h^5/4320 times the fourth
    derivative on each cell of width h (the textbook Gauss-Legendre error
    term), with d^4 psi/dy^4 = 6 s^4."""
    F = lambda ph: (ph ** 5 / 5 - 2 * ph ** 3 / 3 + ph) / 4
    exact = (F(a + s) - F(a)) / s
    n = round(1 / h)
    return exact - n * h ** 5 * 6 * s ** 4 / 4320


@pytest.mark.parametrize("phi,gdir,trees", [(1.0, (0, -1, 0), (1, 1, 1)), (-1.0, (0, -1, 0), (1, 1, 1)),
                                            (1.3, (0, 0, -1), (1, 1, 2)), (-1.0, (0.6, 0.0, -0.8), (2, 1, 1))])
def test_energy_uniform_flow(orc, phi, gdir, trees):
    """E_tot (Sec. 2, eqn energy_functional; readings A10, A11) of a uniform
    phase with a uniform velocity: the kinetic energy 1/2 rho(phi*) |v|^2 |Omega|,
    the free energy (1/(Cn We)) psi(phi) |Omega| (psi of the unclamped phi,
    zero at +-1), and the potential (1/Fr) rho(phi*) int -g.x, outside the
    1/(Cn We) factor."""
    m = orc.Mesh(trees, 2, 2)
    p = P(orc, g=gdir, Cn=0.3, We=3.0, Fr=1.5)
    v = np.array([0.3, -0.7, 0.45])
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = phi
    U[:, 2:5] = v
    U[:, 5] = 0.77
    _, E = m.diagnostics(p, U)
    rho = 0.5 * (1 - p.rho_minus) * np.clip(phi, -1, 1) + 0.5 * (1 + p.rho_minus)
    vol = float(np.prod(trees))
    centroid = 0.5 * np.array(trees, float)
    psi = 0.25 * (phi ** 2 - 1) ** 2
    expect = (0.5 * rho * v @ v * vol + psi * vol / (p.Cn * p.We)
              + rho / p.Fr * (-(np.array(gdir) @ centroid)) * vol)
    assert E == pytest.approx(expect, rel=1e-14)


def test_energy_linear_phase_field(orc):
    """phi = a + s y inside (-1, 1), v uniform, gravity along -y: the kinetic
    and potential integrals are polynomials the rule integrates exactly, the
    gradient energy is (Cn^2/2) s^2, and the quartic psi(phi) is integrated
    with the two-point rule's known error."""
    lev = 3
    m = orc.Mesh((1, 1, 1), lev, lev)
    h = 2.0 ** -lev
    p = P(orc, g=(0.0, -1.0, 0.0), Cn=0.3, We=3.0, Fr=1.5, rho_minus=0.25)
    a, s = -0.6, 1.3
    x = m.node_xyz()
    v = np.array([0.2, 0.5, -0.1])
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = a + s * x[:, 1]
    U[:, 2:5] = v
    _, E = m.diagnostics(p, U)
    alpha, beta = 0.5 * (1 - p.rho_minus), 0.5 * (1 + p.rho_minus)
    int_rho = alpha * (a + s / 2) + beta                       # int rho
    int_rho_y = alpha * (a / 2 + s / 3) + beta / 2             # int rho y
    free = _psi_integral_gauss(a, s, h) + 0.5 * p.Cn ** 2 * s ** 2
    expect = 0.5 * (v @ v) * int_rho + free / (p.Cn * p.We) + int_rho_y / p.Fr
    assert E == pytest.approx(expect, rel=1e-13)


def test_gauss_point_helper_reproduces_trilinear_fields(orc, adaptive):
    """tests/gauss_points.py (which locates the phi pull-back kink for the FP32
    comparisons) evaluates a field that is trilinear on the whole domain
    exactly at the oracle's Gauss points, hanging corners included."""
    from tests import gauss_points as GP
    m = adaptive
    x = m.node_xyz()
    f = lambda P: 0.3 + P[..., 0] - 2 * P[..., 1] + 0.5 * P[..., 2] + 1.5 * P[..., 0] * P[..., 1] * P[..., 2]
    got = GP.gauss_values(m, f(x))
    np.testing.assert_allclose(got, f(m.qp_coords()), rtol=1e-13, atol=1e-14)
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 1.0
    el, rows = GP.near_pullback(m, U, 1e-6)
    assert el.all() and rows.size == m.n_nodes
