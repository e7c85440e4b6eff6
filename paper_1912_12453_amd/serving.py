"""Request loop over the libchns server: replays a stream of timed requests
(workloads.serving_stream), submitting each when its arrival time has passed
and running rounds while anything is resident or waiting, then summarises
per-step latency and throughput.

Per-step latency runs from the moment the step became runnable (admission,
or the end of the request's previous step) to its end; the library measures
it.  A request that waits for the builder or for memory is not runnable yet:
that wait shows in its time to admission.
"""
import time

import numpy as np

from . import chns


def run_stream(server, requests, time_scale=1.0, log=None, max_wall_s=None):
    """Runs the requests (objects with .arrival_s, .workload, .kind) through
    `server` (a chns.Server).  Arrival times are multiplied by time_scale.
    Returns (summary dict, per-request list)."""
    pending = sorted(requests, key=lambda r: r.arrival_s)
    tickets = {}
    t0 = time.perf_counter()
    i = 0
    rounds = 0
    t_log = 0.0
    while True:
        now = time.perf_counter() - t0
        while i < len(pending) and pending[i].arrival_s * time_scale <= now:
            r = pending[i]
            tickets[r.rid] = (server.submit(r.workload.mesh, r.workload.physics, r.workload.steps), now)
            i += 1
        st = server.stats()
        if st.done + st.failed == len(pending):
            break
        if max_wall_s is not None and now > max_wall_s:
            if log:
                log(f"[serve] wall-clock limit {max_wall_s} s reached: {st.as_dict()}")
            break
        if log and now - t_log >= 2.0:
            t_log = now
            log(f"[serve] t={now:.1f}s submitted {i}: {st.as_dict()}")
        if st.resident or st.ready:
            server.run_round()  # admits, then waits up to a few ms for progress
            rounds += 1
            continue
        # nothing runnable: wait for the builder or the next arrival
        nxt = pending[i].arrival_s * time_scale - now if i < len(pending) else 0.002
        time.sleep(min(max(nxt, 0.0), 0.002))
    wall = time.perf_counter() - t0
    per = []
    lat = []
    dof_steps = 0
    conv = 0
    nsteps = 0
    missed = []  # steps that ended above the Newton tolerance, per request
    for r in pending:
        if r.rid not in tickets:
            continue
        t, t_arr = tickets[r.rid]
        info, U, stats, la = server.poll(t, steps=True)
        per.append({"rid": r.rid, "kind": r.kind, "state": int(info.state), "nodes": int(info.n_nodes),
                    "rho_minus": r.workload.physics.rho_minus,
                    "steps": int(info.steps_done), "arrival_s": t_arr,
                    "admit_wait_ms": float(info.t_admit_ms - info.t_submit_ms) if info.t_admit_ms else None,
                    "latency_ms": la, "converged": [bool(s.converged) for s in stats],
                    "gmres_its": [list(s.gmres_its) for s in stats]})
        lat += la
        dof_steps += 6 * int(info.n_nodes) * int(info.steps_done)
        conv += sum(1 for s in stats if s.converged)
        nsteps += len(stats)
        for k, s in enumerate(stats):
            if not s.converged:
                missed.append({"rid": r.rid, "step": k, "rel_res": [float(s.rel_res[0]), float(s.rel_res[1])],
                               "newton_its": list(s.newton_its), "gmres_its": list(s.gmres_its)})
    sst = server.stats().as_dict()
    summary = {"requests": len(pending), "done": sst["done"], "failed": sst["failed"],
               "unfinished": len(pending) - sst["done"] - sst["failed"],
               "rounds": sst["rounds"], "steps": nsteps, "wall_s": round(wall, 3),
               "steps_per_s": round(nsteps / wall, 3),
               "dof_steps_per_s": round(dof_steps / wall, 1),
               "p50_step_ms": round(float(np.percentile(lat, 50)), 3) if lat else None,
               "p99_step_ms": round(float(np.percentile(lat, 99)), 3) if lat else None,
               "converged_step_fraction": round(conv / nsteps, 4) if nsteps else None,
               "requests_all_steps_converged": sum(1 for p in per if all(p["converged"])),
               "unconverged_steps": missed}
    return summary, per
