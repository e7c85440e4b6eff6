"""The serving loop (chns_server_*): a request's result is the same alone and
in a mix with other requests admitted while it runs, admission respects the
HBM budget, and one failing request does not disturb the others."""
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


def request(level, drops, bubble, ratio, visc, steps=3, Cn=0.04):
    inside = -1.0
    return W.Workload(
        name=f"r{level}", mesh=W.MeshSpec((1, 1, 1), 3, level, W.drops_phi(drops, Cn, inside), 0.9),
        physics=W.Physics(Cn=Cn, Pe=1.0 / (3 * Cn * Cn), Re=35.0, We=10.0, Fr=1.0,
                          rho_minus=(1.0 / ratio) if bubble else ratio,
                          eta_minus=(1.0 / visc) if bubble else visc, dt=5e-4),
        steps=steps)


REQS = [
    request(5, [((0.5, 0.5, 0.5), 0.2)], True, 10.0, 5.0),
    request(4, [((0.3, 0.4, 0.5), 0.15), ((0.7, 0.6, 0.5), 0.12)], False, 3.0, 2.0, steps=4),
    request(5, [((0.4, 0.5, 0.6), 0.18)], False, 20.0, 10.0, steps=2),
]


def opts(chns, precond=1):
    return chns.make_opts(precision=1, gmres_rtol=1e-5, gmres_restart=60, precond=precond)


def drain(server, max_s=120.0):
    import time
    t0 = time.time()
    while time.time() - t0 < max_s:
        st = server.stats()
        if st.queued == 0 and st.ready == 0 and st.resident == 0:
            return
        if server.run_round() == 0:
            time.sleep(0.002)
    raise AssertionError("server did not drain")


@pytest.mark.parametrize("precond", [1, 2])
def test_alone_equals_mix(torch, chns, precond):
    """Request 0 run alone, and run while requests 1 and 2 arrive and leave
    around it, gives bit-identical final states and solver counts; both equal
    chns_step applied n_steps times to the same mesh and U^0."""
    print(f"case serving alone-vs-mix precond={precond}", flush=True)
    alone = chns.Server(1 << 34, 1, opts(chns, precond))
    t = alone.submit(REQS[0].mesh, REQS[0].physics, REQS[0].steps)
    drain(alone)
    ia, Ua, sa, _ = alone.poll(t, state=True, steps=True)
    assert ia.state == chns.CHNS_REQ_DONE, ia.status
    alone.close()

    mix = chns.Server(1 << 34, 3, opts(chns, precond))
    t1 = mix.submit(REQS[1].mesh, REQS[1].physics, REQS[1].steps)
    t0 = mix.submit(REQS[0].mesh, REQS[0].physics, REQS[0].steps)
    # let the first round start with what is built, then add the third
    import time
    time.sleep(0.2)
    mix.run_round()
    t2 = mix.submit(REQS[2].mesh, REQS[2].physics, REQS[2].steps)
    drain(mix)
    im, Um, sm, lat = mix.poll(t0, state=True, steps=True)
    assert im.state == chns.CHNS_REQ_DONE
    assert np.array_equal(Ua, Um)
    assert [list(s.gmres_its) for s in sa] == [list(s.gmres_its) for s in sm]
    assert len(lat) == REQS[0].steps and all(v > 0 for v in lat)
    for tk in (t1, t2):
        info, U, _, _ = mix.poll(tk, state=True)
        assert info.state == chns.CHNS_REQ_DONE and np.isfinite(U).all()
    mix.close()

    # the same steps through chns_step
    m = chns.Mesh.from_spec(REQS[0].mesh)
    xyz, bf = m.nodes()
    phi = REQS[0].mesh.phi0(xyz)
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = phi
    U[:, 1] = phi * phi * phi - phi
    d = torch.tensor(U, device="cuda:0")
    p = chns.make_params(REQS[0].physics)
    o = opts(chns, precond)
    for _ in range(REQS[0].steps):
        rc, st = m.step(p, o, d)
        assert rc in (chns.CHNS_OK, chns.CHNS_NOT_CONVERGED)
    assert np.array_equal(d.cpu().numpy(), Ua)


def test_admission_by_footprint(torch, chns):
    """A budget that holds one request at a time serialises them; all finish."""
    print("case serving admission", flush=True)
    probe = chns.Server(1 << 34, 4, opts(chns))
    tks = [probe.submit(r.mesh, r.physics, 1) for r in REQS]
    import time
    for _ in range(500):
        if all(probe.poll(t)[0].state >= chns.CHNS_REQ_READY for t in tks):
            break
        time.sleep(0.01)
    fps = [probe.poll(t)[0].footprint_bytes for t in tks]
    probe.close()
    assert all(f > 0 for f in fps)
    srv = chns.Server(max(fps) + 1, 4, opts(chns))
    tks = [srv.submit(r.mesh, r.physics, r.steps) for r in REQS]
    t0 = time.time()
    while time.time() - t0 < 120:
        st = srv.stats()
        assert st.resident <= 1 and st.bytes_in_use <= max(fps) + 1
        if st.done == len(REQS):
            break
        if srv.run_round() == 0:
            time.sleep(0.002)
    assert srv.stats().done == len(REQS)
    assert srv.stats().bytes_in_use == 0
    srv.close()


def test_oversized_request_fails_alone(torch, chns):
    """A request above the budget fails with a message; the others complete."""
    print("case serving oversized", flush=True)
    big = request(7, [((0.5, 0.5, 0.5), 0.3)], True, 10.0, 5.0, steps=1)
    small = REQS[1]
    srv = chns.Server(64 << 20, 2, opts(chns))
    tb = srv.submit(big.mesh, big.physics, 1)
    ts = srv.submit(small.mesh, small.physics, 2)
    drain(srv)
    ib = srv.poll(tb)[0]
    assert ib.state == chns.CHNS_REQ_FAILED and ib.status == chns.CHNS_EINVAL
    assert "budget" in chns.lib().chns_last_error().decode()
    assert srv.poll(ts)[0].state == chns.CHNS_REQ_DONE
    srv.close()


@pytest.mark.parametrize("precision,precond,coupled", [(1, 1, 0), (0, 2, 0), (1, 2, 1), (0, 1, 1)])
def test_footprint_bounds_device_bytes(torch, chns, precision, precond, coupled):
    """The footprint reserved at admission is at least what the request's mesh
    holds on the device after a step under the same options: mesh arrays,
    solver workspace, cached linearisations and the multigrid hierarchy.
    Without multigrid it is exactly that."""
    print(f"case serving footprint precision={precision} precond={precond} coupled={coupled}", flush=True)
    import time
    o = chns.make_opts(precision=precision, gmres_rtol=1e-5, gmres_restart=60, precond=precond,
                       coupled=coupled)
    reqs = REQS + [request(7, [((0.5, 0.5, 0.5), 0.25)], True, 10.0, 5.0, steps=1)]
    probe = chns.Server(1 << 36, 4, o)
    tks = [probe.submit(r.mesh, r.physics, 1) for r in reqs]
    for _ in range(3000):
        if all(probe.poll(t)[0].state >= chns.CHNS_REQ_READY for t in tks):
            break
        time.sleep(0.01)
    fps = [probe.poll(t)[0].footprint_bytes for t in tks]
    probe.close()
    for r, fp in zip(reqs, fps):
        m = chns.Mesh.from_spec(r.mesh)
        xyz, _ = m.nodes()
        phi = r.mesh.phi0(xyz)
        U = np.zeros((m.n_nodes, 6))
        U[:, 0] = phi
        U[:, 1] = phi * phi * phi - phi
        d = torch.tensor(U, device="cuda:0")
        rc, _ = m.step(chns.make_params(r.physics), o, d)
        torch.cuda.synchronize()
        assert rc in (chns.CHNS_OK, chns.CHNS_NOT_CONVERGED)
        held = chns.chns_mesh_info(m.h).device_bytes
        print(f"  {r.name}: nodes {m.n_nodes} held {held} footprint {fp} ratio {fp / held:.2f}", flush=True)
        assert 0 < held <= fp
        if precond != 2:  # no coarse levels to estimate: the reservation is exact
            assert held == fp
        m.close()
