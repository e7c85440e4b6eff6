"""GPU parity under the physics of the Rayleigh-Taylor brick and of the
serving stream's droplets, through the C ABI, against the oracle.

* RT (Sec. 5.6): gravity along -z, density ratio rho_-/rho_+ = 3 (alpha < 0:
  the phase phi = -1 is the heavy one), viscosity ratio 1, Re = We = 1000,
  Cn = 0.0025, Pe = 1/(3 Cn^2), dt = 2.5e-4, on the 1x1x4 brick refined to
  level 5 around the perturbed interface;
* droplets: density ratio 500 and viscosity ratio 50 (droplet heavier and
  more viscous than the outer fluid), Cn = 0.01, Re 35, We 10, on a unit
  cube refined to level 6 around two drops.

FP64 residuals, JVPs (direct and from the cached linearisation), diagonal
blocks and coupled Jacobian rows agree with the oracle to 1e-12 relative.
FP32 results agree within tests/fp32_bound.py's bound: 100 FP32 unit
roundoffs (6e-6), or 20 times the change of the oracle's FP64 result under
FP32-size perturbations of its inputs where the physics makes the rows more
sensitive than that (density ratio 500)."""
import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W
from tests.fp32_bound import compare_fp32_coupled, fp32_tolerance

pytestmark = pytest.mark.gpu

CH, NS = 0, 1
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "a GPU is required"
    return t


@pytest.fixture(scope="module")
def chns():
    from paper_1912_12453_amd import chns as c
    c.lib()
    return c


def droplets(level=6):
    Cn = 0.01
    drops = [(np.array([0.35, 0.4, 0.5]), 0.15), (np.array([0.68, 0.62, 0.45]), 0.12)]
    return W.Workload(
        name="droplets", mesh=W.MeshSpec((1, 1, 1), 3, level, W.drops_phi(drops, Cn, -1.0), 0.9),
        physics=W.Physics(Cn=Cn, Pe=1.0 / (3 * Cn * Cn), Re=35.0, We=10.0, Fr=1.0, rho_minus=500.0,
                          eta_minus=50.0, dt=5e-4),
        steps=1, seeds={}, description="two heavy, viscous droplets")


CASES = {"rt5": lambda: W.rt(level_max=5), "droplets6": droplets}
_cache = {}


def case(chns, orc, name):
    if name not in _cache:
        w = CASES[name]()
        ms = w.mesh
        pm = chns.Mesh.from_spec(ms)
        om = orc.Mesh(ms.trees, ms.level_min, ms.level_max, ms.phi0, ms.band)
        assert (pm.n_leaves, pm.n_nodes) == (om.n_leaves, om.n_nodes)
        xyz, bf = pm.nodes()
        states = {"workload": W.state_for(w, xyz, bf),
                  "random": W.random_state(pm.n_nodes, 77)}
        _cache[name] = (w, pm, om, states)
    return _cache[name]


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def compare(gpu, ref, fields, tol, label):
    g, r = gpu[:, fields], ref[:, fields]
    e = relerr(g, r)
    emax = np.abs(g - r).max() / max(np.abs(r).max(), 1e-300)
    print(f"{label}: rel2 {e:.2e} relmax {emax:.2e}", flush=True)
    assert e <= tol and emax <= tol * 10, (e, emax)
    return e


def dev(torch, a, dtype=None):
    return torch.tensor(a, dtype=dtype or torch.float64, device="cuda:0").contiguous()


PARAMS = [(c, s) for c in CASES for s in ("workload", "random")]


@pytest.mark.parametrize("name,state", PARAMS)
@pytest.mark.parametrize("block", [CH, NS])
def test_residual_and_jvp(torch, chns, orc, name, state, block):
    w, pm, om, states = case(chns, orc, name)
    print(f"case {name} {state} block {block} E={pm.n_leaves}", flush=True)
    U1, U0 = states[state]
    dU = W.direction(pm.n_nodes, 900 + block)
    p, po = chns.make_params(w.physics), orc.Params.make(**vars(w.physics))
    d1, d0, dd = dev(torch, U1), dev(torch, U0), dev(torch, dU)
    fs = slice(0, 2) if block == CH else slice(2, 6)
    R = pm.residual(p, block, d1, d0).cpu().numpy()
    compare(R, om.residual(po, block, U1, U0), fs, TOL, f"residual {name} {state} {block}")
    ref = om.jvp(po, block, U1, U0, dU)
    compare(pm.jvp(p, block, d1, d0, dd).cpu().numpy(), ref, fs, TOL, f"jvp64 {name} {state} {block}")
    TOL32, ch = fp32_tolerance(lambda a, b, c: om.jvp(po, block, a, b, c), U1, U0, dU, fields=fs)
    print(f"fp32 bound {TOL32:.1e} (oracle change under FP32 perturbations {ch:.1e})", flush=True)
    J32 = pm.jvp(p, block, d1, d0, dev(torch, dU, torch.float32), prec=chns.CHNS_F32)
    compare(J32.cpu().numpy().astype(np.float64), ref, fs, TOL32, f"jvp32 {name} {state} {block}")
    pm.linearize(p, block, d1, d0)
    compare(pm.jvp_lin(p, block, dd).cpu().numpy(), ref, fs, TOL, f"jvp_lin64 {name} {state} {block}")
    pm.linearize(p, block, d1, d0, prec=chns.CHNS_F32)
    J32l = pm.jvp_lin(p, block, dev(torch, dU, torch.float32), prec=chns.CHNS_F32)
    compare(J32l.cpu().numpy().astype(np.float64), ref, fs, TOL32, f"jvp_lin32 {name} {state} {block}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("block", [CH, NS])
def test_diag_blocks(torch, chns, orc, name, block):
    w, pm, om, states = case(chns, orc, name)
    U1, U0 = states["workload"]
    p, po = chns.make_params(w.physics), orc.Params.make(**vars(w.physics))
    D = pm.diag_blocks(p, block, dev(torch, U1), dev(torch, U0)).cpu().numpy()
    ref = om.diag_blocks(po, block, U1, U0)
    nf = 2 if block == CH else 4
    compare(D.reshape(-1, nf * nf), ref.reshape(-1, nf * nf), slice(0, nf * nf), TOL, f"diag {name} {block}")


@pytest.mark.parametrize("name", list(CASES))
def test_coupled_rows_and_diagnostics(torch, chns, orc, name):
    w, pm, om, states = case(chns, orc, name)
    U1, U0 = states["workload"]
    dU = W.direction(pm.n_nodes, 950)
    p, po = chns.make_params(w.physics), orc.Params.make(**vars(w.physics))
    ref = np.zeros_like(U1)
    ref[:, 0:2] = om.jvp_full(po, CH, U1, U0, dU)[:, 0:2]
    ref[:, 2:6] = om.jvp_full(po, NS, U1, U0, dU)[:, 2:6]
    d1, d0 = dev(torch, U1), dev(torch, U0)
    J = pm.jvp_full(p, d1, d0, dev(torch, dU)).cpu().numpy()
    compare(J, ref, slice(0, 2), TOL, f"jvp_full64 CH rows {name}")
    compare(J, ref, slice(2, 6), TOL, f"jvp_full64 NS rows {name}")
    def full(a, b, c):
        out = np.zeros_like(a)
        out[:, 0:2] = om.jvp_full(po, CH, a, b, c)[:, 0:2]
        out[:, 2:6] = om.jvp_full(po, NS, a, b, c)[:, 2:6]
        return out
    TOL32, ch = fp32_tolerance(full, U1, U0, dU)
    print(f"fp32 bound {TOL32:.1e} (oracle change under FP32 perturbations {ch:.1e})", flush=True)
    J32 = pm.jvp_full(p, d1, d0, dev(torch, dU, torch.float32), prec=chns.CHNS_F32).cpu().numpy()
    compare_fp32_coupled(om, U1, J32, ref, TOL32, f"jvp_full32 {name}")
    m_ref, e_ref = om.diagnostics(po, U1)
    m, e = pm.diagnostics(p, d1)
    print(f"diagnostics {name}: mass {m:.15e} / {m_ref:.15e}, energy {e:.15e} / {e_ref:.15e}", flush=True)
    assert m == pytest.approx(m_ref, rel=1e-12, abs=1e-14)
    assert e == pytest.approx(e_ref, rel=1e-12)
