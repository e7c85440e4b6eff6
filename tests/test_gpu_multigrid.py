"""The octree multigrid preconditioner (precond = 2) inside the GPU step: it
changes how GMRES gets there, not where: steps converge to the same
discrete solution as with node-block Jacobi and as the oracle's step, the
captured and launched forms agree bit for bit, and GMRES needs fewer
iterations."""
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


@pytest.mark.parametrize("precision", [0, 1])
def test_multigrid_step_matches_jacobi_and_oracle(torch, chns, orc, precision):
    w, pm, U = drop(chns, 4)
    print(f"case mg drop16 precision={precision}", flush=True)
    p = chns.make_params(w.physics)
    grtol = 1e-7 if precision == 0 else 1e-5
    res = {}
    for pc in (1, 2):
        d = torch.tensor(U, device="cuda:0")
        rc, st = pm.step(p, chns.make_opts(precision=precision, precond=pc, gmres_rtol=grtol), d)
        print(pc, st.as_dict(), flush=True)
        assert rc == chns.CHNS_OK and st.converged
        assert st.rel_res[0] <= 1e-8
        res[pc] = (d.cpu().numpy(), st)
    e = field_err(res[2][0], res[1][0])
    print("mg vs jacobi field errors", ["%.1e" % v for v in e], flush=True)
    assert max(e[0], e[2], e[3], e[4]) < step_tol(precision)
    assert sum(res[2][1].gmres_its) < sum(res[1][1].gmres_its)
    Uo, _ = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max).step(
        orc.Params.make(**vars(w.physics)), orc.SolverOpts.make(), U)
    eo = field_err(res[2][0], Uo)
    print("mg vs oracle field errors", ["%.1e" % v for v in eo], flush=True)
    assert max(eo[0], eo[2], eo[3], eo[4]) < step_tol(precision)


def test_multigrid_graphs_match_launches(torch, chns):
    w, pm, U = drop(chns, 4)
    print("case mg graphs", flush=True)
    p = chns.make_params(w.physics)
    out = []
    for graphs in (0, 1, 1):
        d = torch.tensor(U, device="cuda:0")
        opts = chns.make_opts(precision=1, precond=2, gmres_rtol=1e-5, graphs=graphs, gmres_restart=40)
        its = []
        for _ in range(2):
            rc, st = pm.step(p, opts, d)
            assert rc == chns.CHNS_OK
            its.append(tuple(st.gmres_its))
        torch.cuda.synchronize()
        out.append((d.cpu().numpy(), its))
    for a in out[1:]:
        assert a[1] == out[0][1]
        assert np.array_equal(a[0], out[0][0])


def test_multigrid_levels_and_options(torch, chns):
    """Explicit depths give converged steps; bad multigrid options are
    rejected before any work."""
    w, pm, U = drop(chns, 4)
    print("case mg options", flush=True)
    p = chns.make_params(w.physics)
    for lv in (2, 3):
        d = torch.tensor(U, device="cuda:0")
        rc, st = pm.step(p, chns.make_opts(precond=2, mg_levels=lv, gmres_rtol=1e-7), d)
        print(lv, st.as_dict(), flush=True)
        assert rc == chns.CHNS_OK
    d = torch.tensor(U, device="cuda:0")
    for bad in (dict(mg_omega=0.0), dict(mg_smooth=0), dict(mg_levels=-1), dict(precond=3)):
        kw = dict(precond=2)
        kw.update(bad)
        with pytest.raises(chns.ChnsError):
            pm.step(p, chns.make_opts(**kw), d)
