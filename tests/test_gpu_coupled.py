"""Fully coupled Newton (chns_solver_opts.coupled = 1): one Newton solve of
the whole 6-field system with the coupled Jacobian reaches the same discrete
solution as the block iteration of Fig. 1 and as the oracle's step, in FP64
and mixed precision, with either preconditioner; captured and launched
GMRES cycles agree bit for bit."""
import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W

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


from tests.tolerances import step_tol  # noqa: E402

def drop(chns, level):
    w = W.drop16(level=level)
    pm = chns.Mesh.from_spec(w.mesh)
    xyz, bf = pm.nodes()
    U = W.initial_state(xyz, W.sphere_phi((0.5, 0.5, 0.5), 0.25, w.physics.Cn), bf,
                        phi_noise=1e-3, seed=0)
    return w, pm, U


def field_err(a, b):
    return [float(np.linalg.norm(a[:, f] - b[:, f]) / max(np.linalg.norm(b[:, f]), 1e-300))
            for f in range(6)]


@pytest.mark.parametrize("precision,precond", [(0, 1), (0, 2), (1, 2)])
def test_coupled_step_matches_block_iteration(torch, chns, orc, precision, precond):
    w, pm, U = drop(chns, 4)
    print(f"case coupled drop16 precision={precision} precond={precond}", flush=True)
    p = chns.make_params(w.physics)
    grtol = 1e-7 if precision == 0 else 1e-5
    res = {}
    for coupled in (0, 1):
        d = torch.tensor(U, device="cuda:0")
        opts = chns.make_opts(precision=precision, precond=precond, gmres_rtol=grtol, coupled=coupled)
        rc, st = pm.step(p, opts, d)
        print(coupled, st.as_dict(), flush=True)
        assert rc == chns.CHNS_OK and st.converged
        res[coupled] = (d.cpu().numpy(), st)
    st = res[1][1]
    assert st.block_its == 1 and st.newton_its[0] == 0 and st.newton_its[1] > 0
    assert st.rel_res[0] <= 1e-6 and st.rel_res[1] <= 1e-6
    e = field_err(res[1][0], res[0][0])
    print("coupled vs block", ["%.1e" % v for v in e], flush=True)
    assert max(e[0], e[2], e[3], e[4]) < step_tol(precision)
    Uo, _ = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max).step(
        orc.Params.make(**vars(w.physics)), orc.SolverOpts.make(), U)
    eo = field_err(res[1][0], Uo)
    print("coupled vs oracle", ["%.1e" % v for v in eo], flush=True)
    assert max(eo[0], eo[2], eo[3], eo[4]) < step_tol(precision)
    m0, e0 = pm.diagnostics(p, torch.tensor(U, device="cuda:0"))
    assert abs(st.mass - m0) < 1e-12 and st.energy < e0


def test_coupled_graphs_match_launches(torch, chns):
    w, pm, U = drop(chns, 3)
    print("case coupled graphs", flush=True)
    p = chns.make_params(w.physics)
    out = []
    for graphs in (0, 1, 1):
        d = torch.tensor(U, device="cuda:0")
        opts = chns.make_opts(precision=1, precond=2, gmres_rtol=1e-5, coupled=1, graphs=graphs,
                              gmres_restart=40)
        rc, st = pm.step(p, opts, d)
        assert rc == chns.CHNS_OK
        torch.cuda.synchronize()
        out.append((d.cpu().numpy(), tuple(st.gmres_its)))
    for a in out[1:]:
        assert a[1] == out[0][1] and np.array_equal(a[0], out[0][0])
