"""Intergrid transfer on the device (chns_mesh_interpolate) after remeshing:
every field equals the old trilinear field at the new nodes (independent
numpy evaluation on the oracle's mesh arrays), the mass-conserving form only
shifts phi by the constant that restores its integral, and the solver runs
on the new mesh."""
import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W
from tests.test_remesh_host import field_evaluator

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def chns():
    from paper_1912_12453_amd import chns as c
    c.lib()
    return c


def test_remesh_transfer_and_step(torch, chns, orc):
    print("case remesh transfer bubble5", flush=True)
    w = W.bubble(level_max=5, level_min=2)
    ms = w.mesh
    old_o = orc.Mesh(ms.trees, ms.level_min, ms.level_max, ms.phi0, ms.band)
    old_p = chns.Mesh.from_spec(ms)
    moved = W.sphere_phi((0.5, 0.4, 0.5), 0.15, 0.02, inside=-1.0)
    xo = old_o.node_xyz()
    U = np.random.default_rng(12).normal(0.0, 0.1, (old_p.n_nodes, 6))
    U[:, 0] = moved(xo)
    U[:, 1] = U[:, 0] ** 3 - U[:, 0]
    new_p = old_p.remesh(U, 2, 5, 0.9)
    print(f"old {old_p.n_nodes} nodes, new {new_p.n_nodes} nodes", flush=True)
    d = torch.tensor(U, device="cuda:0")
    Un = old_p.interpolate(new_p, d).cpu().numpy()
    xn, _ = new_p.nodes()
    for f in range(6):
        ref = field_evaluator(old_o, U[:, f])(xn)
        assert np.allclose(Un[:, f], ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max())), f
    # mass-conserving transfer: phi shifted by one constant, integral restored
    ph = W.moderate_physics()
    p = chns.make_params(ph)
    m_old, _ = old_p.diagnostics(p, d)
    Uc = old_p.interpolate(new_p, d, params=p, conserve_mass=True)
    m_new, _ = new_p.diagnostics(p, Uc)
    m_plain, _ = new_p.diagnostics(p, torch.tensor(Un, device="cuda:0"))
    print(f"mass old {m_old:.15f} plain {m_plain:.15f} conserving {m_new:.15f}", flush=True)
    assert abs(m_new - m_old) <= 1e-13 * max(1.0, abs(m_old))
    Ucn = Uc.cpu().numpy()
    shift = Ucn[:, 0] - Un[:, 0]
    assert np.ptp(shift) <= 1e-15 and np.array_equal(Ucn[:, 1:], Un[:, 1:])
    # a step on the new mesh from the transferred state
    U0 = Ucn.copy()
    U0[:, 2:] = 0.0
    _, bf = new_p.nodes()
    dn = torch.tensor(U0, device="cuda:0")
    rc, st = new_p.step(chns.make_params(w.physics), chns.make_opts(precond=2, precision=1, gmres_rtol=1e-5), dn)
    print(st.as_dict(), flush=True)
    assert rc in (chns.CHNS_OK, chns.CHNS_NOT_CONVERGED) and np.isfinite(dn.cpu().numpy()).all()
    assert abs(st.mass - m_new) <= 1e-12 * max(1.0, abs(m_new))
