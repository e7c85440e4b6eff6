"""The manufactured solution of Sec. 5.1 (eqn manufac_exact), extended to
three dimensions with fields independent of z and w = 0, and the forcing
that makes it an exact solution of the CHNS system of Sec. 2.

The forcing is the strong operator of each equation applied to the exact
fields, written with the same sign conventions as the weak forms the
residual tests against (Def. 1 and Def. 2):

  f_phi = d phi/dt + div(v phi) - 1/(Pe Cn) lap mu
  f_mu  = -mu + psi'(phi) - Cn^2 lap phi,            psi'(phi) = phi^3 - phi
  f_m,i = rho (d v_i/dt + v_j d_j v_i) + (1/Pe) J_j d_j v_i
          + (Cn/We) d_j(d_i phi d_j phi) + (1/We) d_i p
          - (1/Re) d_k(eta d_k v_i) - rho g_i / Fr
  f_c   = div v

with rho = alpha phi + beta, eta = gamma phi + xi (phi stays in [-1, 1]) and
J = -(alpha/Cn) grad mu.  All derivatives are written out by hand below and
checked against central differences of the exact fields in the tests.
"""
import numpy as np

PI = np.pi


def params(Re=10.0, We=1.0, Cn=1.0, Pe=3.0, Fr=1.0, rho_minus=0.85, eta_minus=1.0):
    """The non-dimensional numbers of Sec. 5.1; the viscosity ratio is not
    stated there and is taken as 1."""
    return dict(Cn=Cn, Pe=Pe, Re=Re, We=We, Fr=Fr, rho_minus=rho_minus, eta_minus=eta_minus,
                g=(0.0, -1.0, 0.0), C_I=6.0, flux_mode=0)


def fields(x, t):
    """Exact fields at points x (..., 3) and time t: dict of arrays with
    values, first derivatives d[f][k] and the second derivatives needed."""
    X, Y = PI * x[..., 0], PI * x[..., 1]
    sX, cX, sY, cY = np.sin(X), np.cos(X), np.sin(Y), np.cos(Y)
    st, ct = np.sin(t), np.cos(t)
    z = np.zeros_like(X)
    out = {}
    # velocity
    u = sX * cY * st
    v = -cX * sY * st
    out["v"] = np.stack([u, v, z], -1)
    out["v_t"] = np.stack([sX * cY * ct, -cX * sY * ct, z], -1)
    # grad v: gv[..., i, k] = d v_i / d x_k
    gv = np.zeros(x.shape[:-1] + (3, 3))
    gv[..., 0, 0] = PI * cX * cY * st
    gv[..., 0, 1] = -PI * sX * sY * st
    gv[..., 1, 0] = PI * sX * sY * st
    gv[..., 1, 1] = -PI * cX * cY * st
    out["gv"] = gv
    out["lap_v"] = np.stack([-2 * PI ** 2 * u, -2 * PI ** 2 * v, z], -1)
    # pressure
    out["p"] = sX * sY * ct
    out["gp"] = np.stack([PI * cX * sY * ct, PI * sX * cY * ct, z], -1)
    # phase field and chemical potential (the same function)
    phi = cX * cY * st
    out["phi"] = phi
    out["mu"] = phi.copy()
    out["phi_t"] = cX * cY * ct
    gphi = np.stack([-PI * sX * cY * st, -PI * cX * sY * st, z], -1)
    out["gphi"] = gphi
    out["gmu"] = gphi.copy()
    H = np.zeros(x.shape[:-1] + (3, 3))
    H[..., 0, 0] = -PI ** 2 * phi
    H[..., 1, 1] = -PI ** 2 * phi
    H[..., 0, 1] = H[..., 1, 0] = PI ** 2 * sX * sY * st
    out["Hphi"] = H
    out["lap_phi"] = -2 * PI ** 2 * phi
    out["lap_mu"] = out["lap_phi"].copy()
    return out


def forcing_at(x, t, prm):
    """Forcing (..., 6) in the residual's field order (phi-eq, mu-eq,
    momentum x, y, z, continuity) at points x and time t."""
    F = fields(x, t)
    alpha = 0.5 * (1 - prm["rho_minus"])
    beta = 0.5 * (1 + prm["rho_minus"])
    gamma = 0.5 * (1 - prm["eta_minus"])
    xi = 0.5 * (1 + prm["eta_minus"])
    Cn, Pe, Re, We, Fr = prm["Cn"], prm["Pe"], prm["Re"], prm["We"], prm["Fr"]
    g = np.array(prm["g"])
    phi, v, gv = F["phi"], F["v"], F["gv"]
    rho = alpha * phi + beta
    eta = gamma * phi + xi
    geta = gamma * F["gphi"]
    J = -(alpha / Cn) * F["gmu"]
    out = np.zeros(x.shape[:-1] + (6,))
    div_vphi = np.einsum("...k,...k->...", v, F["gphi"]) + phi * np.einsum("...kk->...", gv)
    out[..., 0] = F["phi_t"] + div_vphi - F["lap_mu"] / (Pe * Cn)
    out[..., 1] = -F["mu"] + phi ** 3 - phi - Cn ** 2 * F["lap_phi"]
    conv = np.einsum("...j,...ij->...i", v, gv)
    flux = np.einsum("...j,...ij->...i", J, gv)
    cap = F["gphi"] * F["lap_phi"][..., None] + np.einsum("...j,...ij->...i", F["gphi"], F["Hphi"])
    visc = np.einsum("...k,...ik->...i", geta, gv) + eta[..., None] * F["lap_v"]
    out[..., 2:5] = (rho[..., None] * (F["v_t"] + conv) + flux / Pe + (Cn / We) * cap
                     + F["gp"] / We - visc / Re - rho[..., None] * g / Fr)
    out[..., 5] = np.einsum("...kk->...", gv)
    return out


def state(xyz, t):
    """Nodal state (n, 6) [phi, mu, u, v, w, p] of the exact solution."""
    F = fields(xyz, t)
    U = np.zeros((xyz.shape[0], 6))
    U[:, 0] = F["phi"]
    U[:, 1] = F["mu"]
    U[:, 2:5] = F["v"]
    U[:, 5] = F["p"]
    return U


def l2_error(U, nodes_int, level, t, field):
    """|| u_h - u ||_{L2(unit cube)} of field `field` of the nodal state U on
    a uniform mesh of the given level, with the 2x2x2 Gauss rule per cell
    (values at the points from tests/uniform_quadrature.py)."""
    from tests import fem_closed_forms as CF
    from tests import uniform_quadrature as UQ
    h = 2.0 ** -level
    N = 2 ** level
    idx = CF.lattice_index(nodes_int, level)
    val, _ = UQ.qp_fields(U[:, field], idx, h)
    g = 1.0 / np.sqrt(3.0)
    off = [0.5 * h * (1 + s * g) for s in (-1.0, 1.0)]
    cells = np.arange(N) * h
    e2, q = 0.0, 0
    for qz in range(2):
        for qy in range(2):
            for qx in range(2):
                X, Y, Z = np.meshgrid(cells + off[qx], cells + off[qy], cells + off[qz], indexing="ij")
                P = np.stack([X, Y, Z], -1).reshape(-1, 3)
                ex = state(P, t)[:, field].reshape(N, N, N)
                e2 += ((val[q] - ex) ** 2).sum() * h ** 3 / 8
                q += 1
    return float(np.sqrt(e2))


def run(m, prm, dt, T, opts):
    """CN steps of the oracle from the exact state at t = 0 to T, with the
    forcing at t^{k+1/2} and the exact wall velocity at t^{k+1}."""
    import oracle
    xyz, qp = m.node_xyz(), m.qp_coords()
    p = oracle.Params.make(dt=dt, **prm)
    U = state(xyz, 0.0)
    for k in range(int(round(T / dt))):
        U, st = m.step(p, opts, U, forcing=forcing_at(qp, (k + 0.5) * dt, prm), bc=state(xyz, (k + 1) * dt))
        assert st.converged == 1
    return U
