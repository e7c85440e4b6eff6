"""Pins of the oracle's time step (Newton + GMRES + Jacobi inside the block
iteration of Fig. 1): mass conservation (Prop. 1), energy decay (Thm. 1 and
every experiment of Sec. 5), and second-order time accuracy of the
Crank-Nicolson Cahn-Hilliard block."""
import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W


@pytest.fixture(autouse=True)
def one_thread(orc):
    """These meshes have at most a few thousand elements: the oracle runs
    them faster on one thread than with a parallel loop's start-up cost per
    element pass (results do not depend on the thread count)."""
    cores = orc.num_threads()
    orc.set_num_threads(1)
    yield
    orc.set_num_threads(cores)


def drop_setup(orc, level=3):
    w = W.drop16(level=level)
    m = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max)
    ph = w.physics
    p = orc.Params.make(ph.Cn, ph.Pe, ph.Re, ph.We, ph.Fr, ph.rho_minus, ph.eta_minus, ph.dt, ph.g)
    U = W.initial_state(m.node_xyz(), W.sphere_phi((0.5, 0.5, 0.5), 0.25, ph.Cn), m.bflags,
                        phi_noise=1e-3, seed=0)
    return m, p, U


@pytest.mark.parametrize("precond", [0, 1])
def test_step_converges_conserves_mass_and_dissipates(orc, precond):
    m, p, U = drop_setup(orc)
    o = orc.SolverOpts.make(precond=precond)
    M0, E0 = m.diagnostics(p, U)
    Es = [E0]
    for _ in range(2):
        U, st = m.step(p, o, U)
        assert st.converged == 1
        assert st.block_its >= 2
        M, E = m.diagnostics(p, U)
        assert abs(M - M0) < 1e-12
        Es.append(E)
    assert all(b < a for a, b in zip(Es, Es[1:]))


def test_step_residuals_small_at_solution(orc):
    m, p, U0 = drop_setup(orc)
    o = orc.SolverOpts.make(newton_rtol=1e-10, block_tol=1e-9, block_max_it=20)
    U1, st = m.step(p, o, U0)
    assert st.converged == 1
    for block in (0, 1):
        R = m.residual(p, block, U1, U0)
        R0 = m.residual(p, block, U0, U0)
        f = slice(0, 2) if block == 0 else slice(2, 6)
        assert np.linalg.norm(R[:, f]) < 1e-6 * np.linalg.norm(R0[:, f])


@pytest.mark.slow
def test_cahn_hilliard_block_second_order_in_time(orc):
    """With capillary forcing and gravity switched off (We = Fr = 1e30) the
    velocity stays zero and the step reduces to the Crank-Nicolson CH scheme:
    the error of phi at a fixed time against a fine-step reference falls by
    ~4x per halving of dt."""
    m = orc.Mesh((1, 1, 1), 2, 2)
    x = m.node_xyz()

    def run(dt, T=0.1):
        p = orc.Params.make(0.2, 5.0, 10.0, 1e30, 1e30, 0.5, 0.5, dt, (0, -1, 0))
        U = np.zeros((m.n_nodes, 6))
        U[:, 0] = 0.6 * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])
        U[:, 1] = U[:, 0] ** 3 - U[:, 0]
        o = orc.SolverOpts.make(newton_rtol=1e-12, newton_atol=1e-14, block_tol=1e-11,
                                gmres_rtol=1e-12, block_max_it=30)
        for _ in range(int(round(T / dt))):
            U, st = m.step(p, o, U)
        assert np.abs(U[:, 2:5]).max() == 0.0
        return U

    ref = run(0.1 / 256)
    errs = [np.linalg.norm(run(0.1 / k)[:, 0] - ref[:, 0]) for k in (16, 32, 64)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 1.8, rates
    assert rates.min() > 1.8, rates
