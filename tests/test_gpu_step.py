"""GPU Crank-Nicolson step (block iteration, Newton, GMRES, Jacobi) against the
oracle's step, plus the conservation and dissipation properties and the
failure paths of chns_step."""
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

def drop(chns, orc, level):
    w = W.drop16(level=level)
    pm = chns.Mesh.from_spec(w.mesh)
    om = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max)
    xyz, bf = pm.nodes()
    U = W.initial_state(xyz, W.sphere_phi((0.5, 0.5, 0.5), 0.25, w.physics.Cn), bf,
                        phi_noise=1e-3, seed=0)
    return w, pm, om, U


def field_err(a, b):
    return [float(np.linalg.norm(a[:, f] - b[:, f]) / max(np.linalg.norm(b[:, f]), 1e-300))
            for f in range(6)]


def test_step_matches_oracle_tight(torch, chns, orc):
    """Both solvers driven to tight tolerances reach the same discrete solution."""
    w, pm, om, U = drop(chns, orc, 3)
    print(f"case step-tight drop8 n={pm.n_nodes}", flush=True)
    kw = dict(newton_rtol=1e-11, newton_atol=1e-14, block_tol=1e-10, gmres_rtol=1e-11,
              block_max_it=30)
    Uo, st_o = om.step(orc.Params.make(**vars(w.physics)), orc.SolverOpts.make(**kw), U)
    d = torch.tensor(U, device="cuda:0")
    rc, st = pm.step(chns.make_params(w.physics), chns.make_opts(**kw), d)
    assert rc == chns.CHNS_OK and st.converged
    e = field_err(d.cpu().numpy(), Uo)
    print("field rel errors vs oracle", ["%.1e" % v for v in e], st.as_dict(), flush=True)
    # phi, v: well determined; mu, p are the CN end values of midpoint unknowns
    assert max(e[0], e[2], e[3], e[4]) < 1e-8
    assert max(e[1], e[5]) < 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_drop16_step(torch, chns, orc, precision):
    """One step of the 16^3 drop at the default tolerances (Newton 1e-8): FP64
    and mixed precision both converge, conserve the integral of phi and
    dissipate energy; fields agree with the oracle's step within the solver
    tolerance."""
    w, pm, om, U = drop(chns, orc, 4)
    print(f"case drop16 step precision={precision}", flush=True)
    p = chns.make_params(w.physics)
    d = torch.tensor(U, device="cuda:0")
    m0, e0 = pm.diagnostics(p, d)
    opts = chns.make_opts(precision=precision, gmres_rtol=1e-7 if precision == 0 else 1e-5)
    rc, st = pm.step(p, opts, d)
    print(st.as_dict(), flush=True)
    assert rc == chns.CHNS_OK and st.converged
    assert st.singular_blocks == 0
    # the CH block is solved last in the sweep: its residual meets the Newton
    # tolerance at the end state; the NS residual moves by the last CH update
    assert st.rel_res[0] <= 1e-8
    assert st.rel_res[1] <= 1e-3
    assert abs(st.mass - m0) < 1e-12
    assert st.energy < e0
    Uo, _ = om.step(orc.Params.make(**vars(w.physics)), orc.SolverOpts.make(), U)
    e = field_err(d.cpu().numpy(), Uo)
    print("field rel errors vs oracle", ["%.1e" % v for v in e], flush=True)
    assert max(e[0], e[2], e[3], e[4]) < step_tol(precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_short_restart_step_matches_oracle(torch, chns, orc, precision):
    """GMRES(8) under the multigrid V-cycle: every linear solve of the step
    runs several restart cycles, so the second Gram-Schmidt pass that closes
    each cycle and the R^-1 y update of the stored preconditioned vectors
    carry the result; the step still reaches the oracle's step (GMRES(30),
    Jacobi) within the solver tolerance."""
    w, pm, om, U = drop(chns, orc, 4)
    print(f"case drop16 GMRES(8) precision={precision}", flush=True)
    p = chns.make_params(w.physics)
    d = torch.tensor(U, device="cuda:0")
    opts = chns.make_opts(precision=precision, gmres_restart=8, gmres_max_it=5000, precond=2,
                          gmres_rtol=1e-7 if precision == 0 else 1e-5)
    rc, st = pm.step(p, opts, d)
    print(st.as_dict(), flush=True)
    assert rc == chns.CHNS_OK and st.converged
    assert st.newton_its[1] > 0 and st.gmres_its[1] > 8 * st.newton_its[1]  # restarted solves
    Uo, _ = om.step(orc.Params.make(**vars(w.physics)), orc.SolverOpts.make(), U)
    e = field_err(d.cpu().numpy(), Uo)
    print("field rel errors vs oracle", ["%.1e" % v for v in e], flush=True)
    assert max(e[0], e[2], e[3], e[4]) < step_tol(precision)


def test_energy_decays_over_steps(torch, chns, orc):
    w, pm, om, U = drop(chns, orc, 4)
    p = chns.make_params(w.physics)
    d = torch.tensor(U, device="cuda:0")
    m0, e0 = pm.diagnostics(p, d)
    es = [e0]
    for _ in range(3):
        rc, st = pm.step(p, chns.make_opts(precision=1, gmres_rtol=1e-5), d)
        assert rc == chns.CHNS_OK
        es.append(st.energy)
        assert abs(st.mass - m0) < 1e-12
    print("energy", es, flush=True)
    assert all(b < a for a, b in zip(es, es[1:]))


def test_not_converged_reports_stats(torch, chns, orc):
    w, pm, om, U = drop(chns, orc, 3)
    d = torch.tensor(U, device="cuda:0")
    rc, st = pm.step(chns.make_params(w.physics),
                     chns.make_opts(newton_max_it_ch=1, newton_max_it_ns=1, block_max_it=1), d)
    assert rc == chns.CHNS_NOT_CONVERGED
    assert st.converged == 0 and st.block_its == 1 and st.newton_its[1] == 1
    assert np.isfinite(d.cpu().numpy()).all()


def test_nonfinite_state_is_reported(torch, chns, orc):
    w, pm, om, U = drop(chns, orc, 2)
    U = U.copy()
    U[3, 0] = np.nan
    d = torch.tensor(U, device="cuda:0")
    with pytest.raises(chns.ChnsError) as ei:
        pm.step(chns.make_params(w.physics), chns.make_opts(), d)
    assert ei.value.code in (chns.CHNS_ENONFINITE, chns.CHNS_ETAU)


def test_graph_cycles_match_launches(torch, chns, orc):
    """GMRES restart cycles replayed as HIP graphs give bit-identical steps to
    the same kernels launched one by one, over several steps, both precisions
    on one mesh (the graph cache is reused), with eager library work between
    the replays."""
    w, pm, om, U = drop(chns, orc, 4)
    p = chns.make_params(w.physics)
    res = {}
    for graphs in (0, 1):
        for precision in (0, 1, 0):
            print(f"case graphs={graphs} precision={precision}", flush=True)
            d = torch.tensor(U, device="cuda:0")
            opts = chns.make_opts(precision=precision, gmres_restart=40,
                                  gmres_rtol=1e-7 if precision == 0 else 1e-5)
            traj = []
            for _ in range(3):
                rc, st = pm.step(p, opts, d)
                assert rc == chns.CHNS_OK, st.as_dict()
                R = pm.residual(p, chns.CHNS_BLOCK_CH, d, d)  # eager work between replays
                torch.cuda.synchronize()
                traj.append((d.cpu().numpy().copy(), tuple(st.gmres_its), R.cpu().numpy()))
            key = (graphs, precision)
            if key in res:  # the same run again on the warm cache
                for a, b in zip(res[key], traj):
                    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
            res[key] = traj
    for precision in (0, 1):
        for a, b in zip(res[(0, precision)], res[(1, precision)]):
            assert a[1] == b[1]
            assert np.array_equal(a[0], b[0])
            assert np.array_equal(a[2], b[2])
