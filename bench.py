"""Throughput of the matrix-free CHNS element loop on one MI355X.

Workload (default): the Rayleigh-Taylor brick of Sec. 5.6 at level 10 (1x1x4
unit trees, refined from level 4 to 10 around z = 2 + 0.05 cos(2 pi x)
cos(2 pi y): 15.1M leaves, 13.9M nodes, 83M DoF), density ratio 3 (Atwood
0.5), viscosity ratio 1, Re = We = 1000, Fr 1, Cn 0.0025, gravity along -z;
FP64.  Its working set is far above the 256 MB Infinity Cache, so HBM
figures are HBM figures.  Inputs are synthetic and seeded (workloads.py).

One timed step is one pass of the whole hot path over that input: for the
Navier-Stokes block and then the Cahn-Hilliard block, one Newton iteration
with a fixed-length GMRES(30) cycle (residual and its FP64 norm, node-block
diagonal and its inversion, 30 preconditioned JVPs with classical
Gram-Schmidt twice (second pass delayed) and FP64 dot products, the Newton update, the new
residual), followed by the integral of phi and the total energy.  `value`
counts the DoF that the 60 JVPs of a step touch (30 x 4 per node for NS,
30 x 2 per node for CH) per second of wall time: JVP GDoF/s inside the
solver.

The roofline object describes the NS JVP kernel the solver runs (from the
cached linearisation points), timed live with HIP events on the stream it is
launched on, with the algorithmic work per element of the measurement
accounting (8,900 flops and 170 B per element in FP64); the counted VALU
flops and the rocprofv3 traffic figures sit beside it.

cn_steps times full Crank-Nicolson steps to the 1e-8 relative Newton
residual, FP64 and mixed precision from the same U^0: the 16^3 drop, the
level-9 bubble (10 steps from rest, with the final step's residual checked
by the FP64 oracle on sampled rows) and the RT brick itself, with the block
iteration of Fig. 1 and with the fully coupled Newton solve.  serving runs
the 64-request stream of droplet and bubble problems through the server.
cpu_baseline is the FP64 oracle (test infrastructure) computing the 6-DoF
JVP on the RT brick at level 8 (the same workload, coarser).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
                       [--workload rt_l10|bubble_l9|drop16|...] [--no-cpu-baseline]
                       [--no-steps] [--no-serving] [--cn-steps K] ...
       python bench.py --serving [--serve-requests 64] ...   (serving stream only)
       python bench.py --probe KIND... [--workload W] [--kernel-reps R]
              single element-kernel launches and a 1 GiB copy, for rocprofv3 --pmc
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Work per element of the NS JVP kernel the solver runs, k_ns_jvp_lin (the
# JVP from the cached linearisation points).
# Algorithmic (the measurement accounting of the path, per element with one
# node per element): 8,900 flops; 170 B in FP64 (direction and result 4 + 4
# values, the 10-value state, the corner ids), 100 B with FP32 vectors.
ALG_NS_JVP_FLOPS_PER_ELEMENT = 8900
ALG_NS_JVP_BYTES_PER_ELEMENT = {"fp64": 170, "mixed": 100}
# Counted: floating-point operations the kernel executes per element (the
# SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 or _F32 counters of one launch on the
# level-10 RT brick: 64 x (2 FMA + ADD + MUL + TRANS) / leaves), and the bytes
# it must move as built (per element the NS_LIN cached values at each of the
# 8 Gauss points, the 8 corner ids and the level byte; per node the 4-value
# direction, the 4 cached nodal midpoints and the 4-value result).
NS_LIN = 7
NS_MID = 4
NS_JVP_FLOPS_PER_ELEMENT = {"fp64": 5260, "mixed": 5076}
NS_JVP_BYTES_PER_NODE = {"fp64": (4 + NS_MID + 4) * 8, "mixed": (4 + NS_MID + 4) * 4}
NS_JVP_BYTES_PER_ELEMENT = {"fp64": NS_LIN * 8 * 8 + 8 * 4 + 1, "mixed": NS_LIN * 8 * 4 + 8 * 4 + 1}

# The same for every element kernel bench.py times (both roofline fractions
# per kernel): flops per element (the NS cached JVP and linearisation from the
# VALU counters of one launch; the others 8 lanes x the static count of one
# lane's arithmetic in the kernel's gfx950 code) and bytes per node
# (state staged at both time levels, direction, result, nodal midpoints, at
# their widths) and per element (corner ids and level byte, cached values).
# Key: bench.py's kernel timing name; value: (flops, bytes/node, bytes/element,
# peak).  ns_lin_* also launches k_ns_mid (its reads and writes per node).
ELEMENT_KERNELS = {
    "ch_residual": (1592, (10 + 2) * 8, 33, "fp64"),
    "ns_residual": (4792, (12 + 4) * 8, 33, "fp64"),
    "ch_jvp_f64": (1640, (10 + 2 + 2) * 8, 33, "fp64"),
    "ch_jvp_f32": (1704, 10 * 8 + (2 + 2) * 4, 33, "mixed"),
    "ns_jvp_f64": (6544, (12 + 4 + 4) * 8, 33, "fp64"),
    "ns_jvp_f32": (6344, 12 * 8 + (4 + 4) * 4, 33, "mixed"),
    "ch_lin_f64": (568, 10 * 8, 33 + 4 * 8 * 8, "fp64"),
    "ch_lin_f32": (568, 10 * 8, 33 + 4 * 8 * 4, "mixed"),
    "ch_jvp_lin_f64": (1104, (2 + 2) * 8, 33 + 4 * 8 * 8, "fp64"),
    "ch_jvp_lin_f32": (1168, (2 + 2) * 4, 33 + 4 * 8 * 4, "mixed"),
    "ns_lin_f64": (2597, 12 * 8 + (8 + 4) * 8, 33 + NS_LIN * 8 * 8, "fp64"),
    "ns_lin_f32": (2455, 12 * 8 + 8 * 8 + 4 * 4, 33 + NS_LIN * 8 * 4, "mixed"),
    "ns_jvp_lin_f64": (NS_JVP_FLOPS_PER_ELEMENT["fp64"], NS_JVP_BYTES_PER_NODE["fp64"],
                       NS_JVP_BYTES_PER_ELEMENT["fp64"], "fp64"),
    "ns_jvp_lin_f32": (NS_JVP_FLOPS_PER_ELEMENT["mixed"], NS_JVP_BYTES_PER_NODE["mixed"],
                       NS_JVP_BYTES_PER_ELEMENT["mixed"], "mixed"),
}

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}  # FP64 vector; FP32 vector
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["kernels.hip", "element.hpp", "internal.hpp", "dual.hpp"]


def kernel_source_hash():
    """Hash of the element-kernel sources: counter figures taken on another
    build of the kernels are not reported as this build's."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_12453_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def kernel_roofline(kern, n, E):
    """Both roofline fractions of every timed element kernel (one launch)."""
    out = {}
    for key, (flops, bpn, bpe, peak) in ELEMENT_KERNELS.items():
        ms = kern.get(f"{key}_ms")
        if not ms:
            continue
        gbs = (n * bpn + E * bpe) / (ms * 1e-3) / 1e9
        tf = flops * E / (ms * 1e-3) / 1e12
        out[key] = {"ms": round(ms, 4), "GBps": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                    "TFLOPs": round(tf, 3), "alu_frac": round(tf / PEAK_TFLOPS[peak], 4)}
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cn_steps(chns, W, torch, dev, name, nsteps, precond, restart=120, coupled=0, mesh=None, keep=None):
    """Consecutive Crank-Nicolson steps to the 1e-8 relative Newton residual,
    FP64 and mixed precision from the same U^0: steps/s, p50/p99 step
    latency, solver counts, both blocks' end-of-step relative residuals, the
    energy trace, mass drift, and the field error of the mixed-precision
    trajectory against the FP64 one.  With `mesh` the caller's mesh is used
    (and kept); `keep` (a dict) receives the host states before and after the
    last step of each precision."""
    import numpy as np
    w = W.by_name(name)
    own = mesh is None
    if own:
        mesh = chns.Mesh.from_spec(w.mesh)
        mesh.upload()
    xyz, bf = mesh.nodes()
    if name.startswith("drop"):  # heavy drop at rest, phi perturbed (seed 0)
        U0 = W.initial_state(xyz, W.sphere_phi((0.5, 0.5, 0.5), 0.25, w.physics.Cn), bf,
                             phi_noise=1e-3, seed=0)
    else:  # physical start: v = 0, p = 0
        U0 = W.initial_state(xyz, w.mesh.phi0, bf)
    p = chns.make_params(w.physics)
    out = {"workload": name, "nodes": mesh.n_nodes, "leaves": mesh.n_leaves, "newton_rtol": 1e-8,
           "gmres_restart": restart,
           "newton": "fully coupled" if coupled else "block iteration (Fig. 1)",
           "precond": {1: "node-block Jacobi", 2: "octree multigrid V-cycle"}[precond], "steps": nsteps}
    finals = {}
    for prec, pname, grtol in ((0, "fp64", 1e-7), (1, "mixed", 1e-5)):
        opts = chns.make_opts(precision=prec, gmres_rtol=grtol, gmres_restart=restart, precond=precond,
                              coupled=coupled)
        U = torch.tensor(U0, device=dev)
        rc, st = mesh.step(p, opts, U)  # warm-up: workspace, hierarchy and graph capture
        log(f"[bench] cn warm-up {name} {pname}: rc {rc}, gmres {list(st.gmres_its)}")
        U.copy_(torch.tensor(U0, device=dev))
        mass0, e0 = mesh.diagnostics(p, U)
        torch.cuda.synchronize()
        lat, energy, conv, gits, rel = [], [e0], True, [0, 0], [0.0, 0.0]
        t0 = time.perf_counter()
        for k in range(nsteps):
            if keep is not None and k == nsteps - 1:
                prev = U.clone()
            ts = time.perf_counter()
            rc, st = mesh.step(p, opts, U)
            lat.append((time.perf_counter() - ts) * 1e3)
            if rc not in (chns.CHNS_OK, chns.CHNS_NOT_CONVERGED):
                raise RuntimeError(f"step failed with {rc}")
            conv = conv and rc == chns.CHNS_OK
            log(f"[bench] cn step {name} {pname}: {lat[-1]:.0f} ms, gmres {list(st.gmres_its)}, "
                f"rel_res {st.rel_res[0]:.1e} {st.rel_res[1]:.1e}, rc {rc}")
            energy.append(st.energy)
            gits = [gits[0] + st.gmres_its[0], gits[1] + st.gmres_its[1]]
            rel = [max(rel[0], st.rel_res[0]), max(rel[1], st.rel_res[1])]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        finals[pname] = U.cpu().numpy()
        if keep is not None:
            keep[pname] = (prev.cpu().numpy(), finals[pname])
            del prev
        out[pname] = {"steps_per_s": round(nsteps / t, 3),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "all_converged": bool(conv),
                      "max_rel_res_end_of_step": {"ch": rel[0], "ns": rel[1]},
                      "gmres_its_per_step": [g / nsteps for g in gits],
                      "energy_non_increasing": bool(all(b <= a for a, b in zip(energy, energy[1:]))),
                      "energy": [float(e) for e in energy],
                      "mass_drift": st.mass - mass0}
        log(f"[bench] cn steps {name} {pname}: {out[pname]}")
        del U
    out["mixed_speedup"] = round(out["mixed"]["steps_per_s"] / out["fp64"]["steps_per_s"], 3)
    ef, em = np.array(out["fp64"]["energy"]), np.array(out["mixed"]["energy"])
    out["energy_trace_max_rel_diff_mixed_vs_fp64"] = float(np.abs(em - ef).max() / np.abs(ef).max())
    a, b = finals["mixed"], finals["fp64"]
    out["mixed_vs_fp64_rel_l2"] = {f: float(np.linalg.norm(a[:, i] - b[:, i]) / max(np.linalg.norm(b[:, i]), 1e-300))
                                   for i, f in enumerate(("phi", "mu", "u", "v", "w", "p"))}
    if own:
        mesh.close()
    return out


def oracle_anchor(oracle, w, om, states, rows):
    """The FP64 oracle's residual of both blocks, on sampled rows, at the last
    step's result (U^{k+1}, U^k) of each precision, relative to the same rows'
    residual at the step's start (U^k, U^k): the precision's error against
    the oracle, measured in the oracle's own discrete equations."""
    import numpy as np
    op = oracle.Params.make(**vars(w.physics))
    res = {}
    for pname, (Uk, Uk1) in states.items():
        r = {}
        for blk, bname, f in ((0, "ch", slice(0, 2)), (1, "ns", slice(2, 6))):
            R1 = om.residual_rows(op, blk, Uk1, Uk, rows)[:, f]
            R0 = om.residual_rows(op, blk, Uk, Uk, rows)[:, f]
            r[bname] = float(np.linalg.norm(R1) / max(np.linalg.norm(R0), 1e-300))
        res[pname] = r
    return res


def q2_run(chns, W, torch, name, reps):
    """The cG(2) blocks (27-node leaves) on a workload's mesh: host build of
    the numbering, then the element pass and node gather of each block's
    residual and JVP, each timed over `reps` launches with HIP events on the
    launch stream.  Random state and direction (seeded)."""
    w = W.by_name(name)
    mesh = chns.Mesh.from_spec(w.mesh)
    mesh.upload()
    t0 = time.time()
    q = mesh.q2()
    t_build = time.time() - t0
    U1, U0 = W.random_state(q.n_nodes, 1)
    dU = W.direction(q.n_nodes, 2)
    d1, d0, dd = (torch.tensor(a, device="cuda:0") for a in (U1, U0, dU))
    out = torch.empty_like(dd)
    p = chns.make_params(w.physics)
    res = {"workload": name, "leaves": mesh.n_leaves, "nodes": q.n_nodes, "hanging": q.n_hanging,
           "constraint_entries": q.n_constraint, "host_build_s": round(t_build, 2),
           "device_bytes": q.device_bytes, "precision": "fp64"}
    stream = torch.cuda.current_stream()
    for block, bname, nf in ((0, "ch", 2), (1, "ns", 4)):
        for mode in ("residual", "jvp"):
            if mode == "residual":
                f = lambda: q.residual(p, d1, d0, block=block, out=out)
            else:
                f = lambda: q.jvp(p, d1, d0, dd, block=block, out=out)
            f()
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record(stream)
            for _ in range(reps):
                f()
            e.record(stream)
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            res[f"{bname}_{mode}"] = {"ms": round(ms, 4), "GDoF_per_s": round(nf * q.n_nodes / ms / 1e6, 4),
                                      "ns_per_leaf": round(ms * 1e6 / mesh.n_leaves, 2)}
    q.close()
    mesh.close()
    del d1, d0, dd, out
    torch.cuda.empty_cache()
    return res


def serving_run(args, chns, W):
    """The serving stream: Poisson arrivals of independent droplet / bubble
    problems (workloads.serving_stream), mixed precision with the
    multigrid-preconditioned fully coupled solver at the default tolerances
    (Newton 1e-8), admitted by footprint into an HBM budget.  Returns the
    summary and the per-request list."""
    from paper_1912_12453_amd import serving
    reqs = W.serving_stream(n_requests=args.serve_requests, rate_hz=20.0, seed=4,
                            level_range=(args.serve_level_min, args.serve_level_max),
                            steps=args.serve_steps)
    # per-step work is capped so that a hard request cannot hold the device
    # for minutes: such steps end NOT_CONVERGED and are counted as such
    opts = chns.make_opts(precision=1, gmres_rtol=1e-5, gmres_restart=60, precond=2,
                          gmres_max_it=args.serve_gmres_max_it, newton_max_it_ch=args.serve_newton_max_it,
                          newton_max_it_ns=args.serve_newton_max_it, block_max_it=3, coupled=args.serve_coupled)
    srv = chns.Server(args.serve_budget_gib << 30, args.serve_max_resident, opts)
    summ, per = serving.run_stream(srv, reqs, log=log, max_wall_s=args.serve_max_wall_s)
    srv.close()
    summ.update({"levels": [args.serve_level_min, args.serve_level_max], "rate_hz": 20.0,
                 "steps_per_request": args.serve_steps, "budget_gib": args.serve_budget_gib,
                 "max_resident": args.serve_max_resident, "gmres_max_it": args.serve_gmres_max_it,
                 "newton_max_it": args.serve_newton_max_it,
                 "newton": "fully coupled" if args.serve_coupled else "block iteration"})
    return summ, per


def serving_main(args):
    """bench.py --serving: the serving stream alone, as one JSON line."""
    import torch

    from paper_1912_12453_amd import chns
    from paper_1912_12453_amd import workloads as W

    torch.cuda.set_device(0)
    summ, per = serving_run(args, chns, W)
    res = {"metric": "serving CN steps/s with p50/p99 per-step latency", "value": summ["steps_per_s"],
           "unit": "steps/s", "n_gpus": 1, "steps": summ["steps"], "warmup": 0,
           "ms_per_step": round(1e3 * summ["wall_s"] / max(summ["steps"], 1), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
           "data": "synthetic",
           "config": {"workload": "serving_stream", "requests": args.serve_requests},
           "serving": summ,
           "largest_requests": sorted(({"nodes": p["nodes"], "latency_ms": [round(x, 1) for x in p["latency_ms"]]}
                                       for p in per), key=lambda d: -d["nodes"])[:3],
           "slowest_requests": sorted(({"nodes": p["nodes"], "rho_minus": p["rho_minus"], "kind": p["kind"],
                                        "latency_ms": [round(x, 1) for x in p["latency_ms"]],
                                        "converged": p["converged"]}
                                       for p in per), key=lambda d: -max(d["latency_ms"] or [0]))[:3]}
    print(json.dumps(res), flush=True)


def batching_main(args):
    """bench.py --batching K LEVEL: the serving operator (the coupled FP32
    JVP, chns_jvp_full) over K serving-size drop problems, applied (a) in one
    launch over a brick of K trees holding one problem each, (b) as K
    launches on one stream and (c) as K launches on K streams (the serving
    loop's design).  Seeded drops as in the serving stream (1-4 per problem,
    r ~ U(0.08, 0.2)), one physics for all."""
    import numpy as np
    import torch

    from paper_1912_12453_amd import chns
    from paper_1912_12453_amd import workloads as W
    K, lmax = args.batching
    reps = args.kernel_reps
    torch.cuda.set_device(0)
    rng = np.random.default_rng(4)
    Cn = 0.01
    probs = []
    for _ in range(K):
        nd, drops = int(rng.integers(1, 5)), []
        while len(drops) < nd:
            r = rng.uniform(0.08, 0.2)
            c = rng.uniform(r + 0.05, 1 - r - 0.05, 3)
            if all(np.linalg.norm(c - c2) > r + r2 + 4 * np.sqrt(2) * Cn for c2, r2 in drops):
                drops.append((c, r))
        probs.append(drops)
    ph = W.Physics(Cn=Cn, Pe=1 / (3 * Cn * Cn), Re=35.0, We=10.0, Fr=1.0, rho_minus=100.0, eta_minus=10.0,
                   dt=5e-4)
    p = chns.make_params(ph)
    meshes = []
    for drops in probs:
        m = chns.Mesh.from_spec(W.MeshSpec((1, 1, 1), 4, lmax, W.drops_phi(drops, Cn, -1.0), 0.9))
        m.upload()
        meshes.append(m)
    alld = [(np.array(c) + np.array([i, 0, 0]), r) for i, drops in enumerate(probs) for c, r in drops]
    big = chns.Mesh.from_spec(W.MeshSpec((K, 1, 1), 4, lmax, W.drops_phi(alld, Cn, -1.0), 0.9))
    big.upload()

    def tensors(m):
        U1, U0 = W.random_state(m.n_nodes, 3, mu_sigma=0.01)
        d = W.direction(m.n_nodes, 4)
        return (torch.tensor(U1, device="cuda:0"), torch.tensor(U0, device="cuda:0"),
                torch.tensor(d, dtype=torch.float32, device="cuda:0"),
                torch.empty((m.n_nodes, 6), dtype=torch.float32, device="cuda:0"))
    ts = [tensors(m) for m in meshes]
    tb = tensors(big)
    streams = [torch.cuda.Stream() for _ in meshes]

    def run_big():
        chns.chns_jvp_full(big.h, p, tb[0], tb[1], tb[2], tb[3], chns.CHNS_F32)

    def run_serial():
        for m, t in zip(meshes, ts):
            chns.chns_jvp_full(m.h, p, t[0], t[1], t[2], t[3], chns.CHNS_F32)

    def run_streams():
        cur = torch.cuda.current_stream()
        ev = torch.cuda.Event()
        ev.record(cur)
        for st, m, t in zip(streams, meshes, ts):
            st.wait_event(ev)
            chns.chns_jvp_full(m.h, p, t[0], t[1], t[2], t[3], chns.CHNS_F32, stream=st.cuda_stream)
        for st in streams:
            cur.wait_stream(st)
    out = {"problems": K, "level_max": lmax, "leaves": [m.n_leaves for m in meshes], "brick_leaves": big.n_leaves,
           "operator": "coupled FP32 JVP (chns_jvp_full)", "reps": reps}
    for key, f in (("one_launch_over_brick_ms", run_big), ("k_launches_one_stream_ms", run_serial),
                   ("k_launches_k_streams_ms", run_streams)):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        out[key] = round((time.perf_counter() - t0) / reps * 1e3, 4)
        log(f"[batching] {key}: {out[key]} ms")
    print(json.dumps(out), flush=True)


def probe_main(args):
    """bench.py --probe KIND...: launches single element kernels of a workload
    (the per-chunk element loop alone), and a device copy of known size, for
    hardware-counter collection with rocprofv3 --pmc.
    KIND: ns64 ns32 ch64 ch32 nsres chres nsdiag chdiag nslin64 nslin32 chlin64
    chlin32 copy.  The copy reads and writes 1 GiB; its FETCH_SIZE and
    WRITE_SIZE give the factors that turn the counters into HBM bytes."""
    import torch

    from paper_1912_12453_amd import chns
    from paper_1912_12453_amd import workloads as W

    log("probe: start")
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = W.by_name(args.workload)
    m = chns.Mesh.from_spec(w.mesh)
    m.upload()
    xyz, bf = m.nodes()
    U1h, U0h = W.state_for(w, xyz, bf)
    U1 = torch.tensor(U1h, device=dev)
    U0 = torch.tensor(U0h, device=dev)
    dU = torch.tensor(W.direction(m.n_nodes, 3), device=dev)
    dU32 = dU.float()
    p = chns.make_params(w.physics)
    reps = args.kernel_reps
    log(f"probe: {args.workload} {m.n_leaves} leaves {m.n_nodes} nodes, {reps} launches per kernel")
    table = {  # kind: (block, op, direction)
        "chres": (0, 0, None), "ch64": (0, 1, dU), "ch32": (0, 2, dU32), "chdiag": (0, 3, None),
        "nsres": (1, 0, None), "ns64": (1, 1, dU), "ns32": (1, 2, dU32), "nsdiag": (1, 3, None),
    }
    for k in args.probe:
        if k in ("nslin64", "nslin32", "chlin64", "chlin32"):  # linearise once, then the cached JVP
            blk = 1 if k.startswith("ns") else 0
            op = 4 if k.endswith("64") else 6
            d = dU if k.endswith("64") else dU32
            chns.chns_launch_element_loop(m.h, p, blk, op + 1, U1, U0, None, None, 1)
            chns.chns_launch_element_loop(m.h, p, blk, op, U1, U0, d, None, reps)
        elif k == "copy":
            src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
        elif k in table:
            blk, op, d = table[k]
            chns.chns_launch_element_loop(m.h, p, blk, op, U1, U0, d, None, reps)
        else:
            raise SystemExit(f"unknown probe kind {k}")
        torch.cuda.synchronize()
        log(f"probe: {k} done")
    log("probe: end")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", default="rt_l10")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workload", default="rt_l8")
    ap.add_argument("--cpu-reps", type=int, default=25)
    ap.add_argument("--cn-steps", type=int, default=10, help="steps of the 16^3 drop (config 1)")
    ap.add_argument("--cn-steps-bubble", type=int, default=10, help="steps of the level-9 bubble (config 3)")
    ap.add_argument("--cn-steps-large", type=int, default=20, help="coupled steps of the workload itself")
    ap.add_argument("--cn-steps-large-block", type=int, default=3,
                    help="block-iteration steps of the workload itself")
    ap.add_argument("--cn-restart", type=int, default=60)
    ap.add_argument("--anchor-rows", type=int, default=2000)
    ap.add_argument("--no-steps", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("--probe", nargs="+", metavar="KIND")
    ap.add_argument("--batching", nargs=2, type=int, metavar=("K", "LEVEL"),
                    help="serving operator over K problems: one launch vs K launches")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--serve-level-min", type=int, default=6)
    ap.add_argument("--serve-level-max", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=int, default=160)
    ap.add_argument("--serve-max-resident", type=int, default=16)
    ap.add_argument("--serve-gmres-max-it", type=int, default=60)
    ap.add_argument("--serve-newton-max-it", type=int, default=8)
    ap.add_argument("--serve-max-wall-s", type=float, default=300.0)
    ap.add_argument("--serve-coupled", type=int, default=1)
    ap.add_argument("--q2-workload", default="bubble_l9", help="mesh of the cG(2) CH block line")
    ap.add_argument("--no-q2", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        return probe_main(args)
    if args.batching:
        return batching_main(args)
    if args.serving:
        return serving_main(args)

    import numpy as np
    import torch

    from paper_1912_12453_amd import chns
    from paper_1912_12453_amd import workloads as W

    t_bench = time.time()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    name = args.workload
    w = W.by_name(name)

    t0 = time.time()
    mesh = chns.Mesh.from_spec(w.mesh)
    mesh.upload()
    t_mesh = time.time() - t0
    xyz, bf = mesh.nodes()
    n, E = mesh.n_nodes, mesh.n_leaves
    log(f"[bench] {name}: {E} leaves, {n} nodes, {mesh.stats.n_hanging} hanging; "
        f"mesh build + upload {t_mesh:.2f}s")
    U1h, U0h = W.state_for(w, xyz, bf)
    dUh = W.direction(n, w.seeds.get("direction", 3))
    p = chns.make_params(w.physics)
    U0 = torch.tensor(U0h, device=dev)
    U1 = torch.tensor(U1h, device=dev)
    dU = torch.tensor(dUh, device=dev)
    precision = 0 if args.precision == "fp64" else 1
    K_GMRES = 30
    opts = chns.make_opts(newton_max_it_ch=1, newton_max_it_ns=1, gmres_restart=K_GMRES,
                          gmres_max_it=K_GMRES, gmres_rtol=0.0, newton_rtol=0.0, block_max_it=1,
                          precision=precision, precond=1)
    U = U0.clone()

    def step():
        U.copy_(U0)
        rc, st = mesh.step(p, opts, U)
        if rc not in (chns.CHNS_OK, chns.CHNS_NOT_CONVERGED):
            raise RuntimeError(f"step failed with {rc}")
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = step()
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    gits = list(st.gmres_its)
    dof_per_step = (gits[0] * 2 + gits[1] * 4) * n
    value = dof_per_step * args.steps / t_total / 1e9
    log(f"[bench] {args.steps} steps in {t_total:.3f}s; gmres its per step {gits}")

    # ---- live kernel timing: the NS JVP kernel of the solver (from the cached
    # linearisation points), HIP events on the stream it is launched on
    stream = torch.cuda.current_stream()
    out = torch.zeros_like(U1)
    op = 4 if precision == 0 else 6
    chns.chns_launch_element_loop(mesh.h, p, chns.CHNS_BLOCK_NS, op + 1, U1, U0, None, None, 1)
    dUk = dU if precision == 0 else dU.float()
    outk = out if precision == 0 else out.float()
    # untimed launches first: the clocks settle after the host-side work above
    chns.chns_launch_element_loop(mesh.h, p, chns.CHNS_BLOCK_NS, op, U1, U0, dUk, outk, 10)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    grid = chns.chns_launch_element_loop(mesh.h, p, chns.CHNS_BLOCK_NS, op, U1, U0, dUk, outk,
                                         args.kernel_reps)
    ev1.record(stream)
    ev1.synchronize()
    ns_ms = ev0.elapsed_time(ev1) / args.kernel_reps
    kern = {}
    for blk, bname in ((chns.CHNS_BLOCK_CH, "ch"), (chns.CHNS_BLOCK_NS, "ns")):
        for o, oname in ((0, "residual"), (1, "jvp_f64"), (2, "jvp_f32")):
            dd = dU if o != 2 else dU.float()
            oo = out if o != 2 else out.float()
            chns.chns_launch_element_loop(mesh.h, p, blk, o, U1, U0, dd, oo, 1)
            ev0.record(stream)
            chns.chns_launch_element_loop(mesh.h, p, blk, o, U1, U0, dd, oo, 5)
            ev1.record(stream)
            ev1.synchronize()
            kern[f"{bname}_{oname}_ms"] = ev0.elapsed_time(ev1) / 5
    for blk, bname in ((chns.CHNS_BLOCK_CH, "ch"), (chns.CHNS_BLOCK_NS, "ns")):
        for o, oname in ((5, "lin_f64"), (4, "jvp_lin_f64"), (7, "lin_f32"), (6, "jvp_lin_f32")):
            dd = dU if o in (4, 5) else dU.float()
            chns.chns_launch_element_loop(mesh.h, p, blk, o, U1, U0, dd, None, 1)
            ev0.record(stream)
            chns.chns_launch_element_loop(mesh.h, p, blk, o, U1, U0, dd, None, 5)
            ev1.record(stream)
            ev1.synchronize()
            kern[f"{bname}_{oname}_ms"] = ev0.elapsed_time(ev1) / 5
    for bname, nf, names in (("ch", 2, ("jvp_f64", "jvp_f32", "jvp_lin_f64", "jvp_lin_f32")),
                             ("ns", 4, ("jvp_f64", "jvp_f32", "jvp_lin_f64", "jvp_lin_f32"))):
        for oname in names:
            kern[f"{bname}_{oname}_gdofs"] = n * nf / kern[f"{bname}_{oname}_ms"] / 1e6

    # diagonal-block kernels (once per Newton iteration)
    for blk, bname in ((chns.CHNS_BLOCK_CH, "ch"), (chns.CHNS_BLOCK_NS, "ns")):
        chns.chns_launch_element_loop(mesh.h, p, blk, 3, U1, U0, None, None, 1)
        ev0.record(stream)
        chns.chns_launch_element_loop(mesh.h, p, blk, 3, U1, U0, None, None, 2)
        ev1.record(stream)
        ev1.synchronize()
        kern[f"{bname}_diag_ms"] = ev0.elapsed_time(ev1) / 2
    log(f"[bench] kernel timing done ({time.time() - t_bench:.0f}s)")

    # ---- roofline of the dominant kernel: the algorithmic work per element
    prec = args.precision
    alg_flops = ALG_NS_JVP_FLOPS_PER_ELEMENT * E
    alg_bytes = ALG_NS_JVP_BYTES_PER_ELEMENT[prec] * E
    alg_tf = alg_flops / (ns_ms * 1e-3) / 1e12
    alg_gbs = alg_bytes / (ns_ms * 1e-3) / 1e9
    cnt_flops = NS_JVP_FLOPS_PER_ELEMENT[prec] * E
    cnt_bytes = n * NS_JVP_BYTES_PER_NODE[prec] + E * NS_JVP_BYTES_PER_ELEMENT[prec]
    cnt_tf = cnt_flops / (ns_ms * 1e-3) / 1e12
    kname = "k_ns_jvp_lin<double,double>" if precision == 0 else "k_ns_jvp_lin<float,float>"
    traffic = valu_busy = None
    traffic_note = "no counter pass of this kernel on this workload in profiles/traffic.json"
    src_hash = kernel_source_hash()
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get("kernels", {}).get(kname, {}).get(name)
        if ent and ent.get("leaves") == E:
            if ent.get("kernel_sources") == src_hash:
                traffic = ent["hbm_bytes_per_launch"]
                valu_busy = ent.get("valu_busy")
                traffic_note = ("rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes of this build's kernel on "
                                "this workload (profiles/traffic.json, " + ent.get("profile", "") + "), "
                                "scaled by the 1 GiB copy's factors; not measured in this run")
            else:
                traffic_note = "counters in profiles/traffic.json are of another build of the kernel"
    alu_frac, hbm_frac = alg_tf / PEAK_TFLOPS[prec], alg_gbs / PEAK_HBM_GBS
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(alg_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(alg_tf, 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    roof.update({"traffic": traffic, "traffic_source": traffic_note, "kernel": kname,
                 "avg_ms": round(ns_ms, 4), "grid": grid, "block": 256, "timing": "HIP events on the launch stream",
                 "units_per_launch": E, "unit_of_work": "leaf element",
                 "algorithmic_flops_per_unit": ALG_NS_JVP_FLOPS_PER_ELEMENT,
                 "algorithmic_bytes_per_unit": ALG_NS_JVP_BYTES_PER_ELEMENT[prec],
                 "algorithmic_TFLOPs": round(alg_tf, 3), "alu_frac": round(alu_frac, 4),
                 "algorithmic_GBps": round(alg_gbs, 1), "hbm_frac": round(hbm_frac, 4),
                 "counted": {"flops_per_element": NS_JVP_FLOPS_PER_ELEMENT[prec],
                             "TFLOPs": round(cnt_tf, 3), "alu_frac": round(cnt_tf / PEAK_TFLOPS[prec], 4),
                             "bytes_per_launch_as_built": cnt_bytes,
                             "GBps_as_built": round(cnt_bytes / (ns_ms * 1e-3) / 1e9, 1),
                             "traffic_over_algorithmic": (round(traffic / alg_bytes, 2) if traffic else None)},
                 "kernel_sources": src_hash})
    if valu_busy is not None:  # rocprofv3's VALUBusy of the same kernel (counter pass), as a fraction
        roof["counted"]["valu_busy"] = valu_busy

    # ---- full Crank-Nicolson steps at the 1e-8 Newton tolerance, FP64 vs mixed
    n_hanging = int(mesh.stats.n_hanging)
    del U1, U0, dU, out, dUk, outk, U
    torch.cuda.empty_cache()
    steps = None
    anchor = None
    if not args.no_steps:
        steps = {}
        # the workload itself on its own mesh (config 5 on the RT brick)
        steps[name + "_coupled"] = cn_steps(chns, W, torch, dev, name, args.cn_steps_large, 2, args.cn_restart,
                                            1, mesh=mesh)
        if args.cn_steps_large_block > 0:
            steps[name] = cn_steps(chns, W, torch, dev, name, args.cn_steps_large_block, 2, args.cn_restart,
                                   0, mesh=mesh)
        mesh.close()
        torch.cuda.empty_cache()
        log(f"[bench] {name} CN steps done ({time.time() - t_bench:.0f}s)")
        for coupled, tag in ((0, ""), (1, "_coupled")):
            steps["drop16" + tag] = cn_steps(chns, W, torch, dev, "drop16", args.cn_steps, 2, 120, coupled)
        if name != "bubble_l9" and args.cn_steps_bubble > 0:
            keep = {}
            for coupled, tag in ((0, ""), (1, "_coupled")):
                keep[tag] = {}
                steps["bubble_l9" + tag] = cn_steps(chns, W, torch, dev, "bubble_l9", args.cn_steps_bubble, 2,
                                                    120, coupled, keep=keep[tag])
            log(f"[bench] bubble CN steps done ({time.time() - t_bench:.0f}s)")
            if args.anchor_rows > 0:
                import oracle
                wb = W.by_name("bubble_l9")
                t0 = time.time()
                om = oracle.Mesh(wb.mesh.trees, wb.mesh.level_min, wb.mesh.level_max, wb.mesh.phi0, wb.mesh.band)
                rows = np.sort(np.random.default_rng(7).choice(om.n_nodes, args.anchor_rows, replace=False))
                anchor = {"what": "FP64 oracle residual of the last of the bubble's CN steps, on sampled rows, "
                                  "relative to the same rows at the step's start: each precision's error "
                                  "against the oracle in the oracle's discrete equations (block rel. 2-norm)",
                          "rows": int(args.anchor_rows)}
                for tag in ("", "_coupled"):
                    anchor["bubble_l9" + tag] = oracle_anchor(oracle, wb, om, keep[tag], rows)
                del om
                log(f"[bench] oracle anchor {anchor} ({time.time() - t0:.0f}s)")
    else:
        mesh.close()
        torch.cuda.empty_cache()

    # ---- serving stream (config 4)
    serving_summary = None
    if not args.no_serving:
        summ, _ = serving_run(args, chns, W)
        serving_summary = summ
        log(f"[bench] serving {summ} ({time.time() - t_bench:.0f}s)")

    # ---- cG(2) CH block
    q2 = None
    if not args.no_q2:
        q2 = q2_run(chns, W, torch, args.q2_workload, args.kernel_reps)
        log(f"[bench] q2 {q2} ({time.time() - t_bench:.0f}s)")

    # ---- CPU baseline: the oracle's 6-DoF JVP on the same workload at level 8
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        wc = W.by_name(args.cpu_workload)
        t0 = time.time()
        om = oracle.Mesh(wc.mesh.trees, wc.mesh.level_min, wc.mesh.level_max, wc.mesh.phi0, wc.mesh.band)
        log(f"[bench] oracle mesh {args.cpu_workload}: {om.n_leaves} leaves, {time.time() - t0:.1f}s")
        xc = om.node_xyz()
        U1c, U0c = W.state_for(wc, xc, om.bflags)
        dUc = W.direction(om.n_nodes, wc.seeds.get("direction", 3))
        op_ = oracle.Params.make(**vars(wc.physics))
        reps = args.cpu_reps
        t0 = time.perf_counter()
        for _ in range(reps):
            om.jvp(op_, 0, U1c, U0c, dUc)
            om.jvp(op_, 1, U1c, U0c, dUc)
        tc = time.perf_counter() - t0
        cores = oracle.num_threads()
        cpu = {"value": round(6 * om.n_nodes * reps / tc / 1e9, 6), "unit": "GDoF/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "sample": f"{reps} x (CH + NS JVP) over the {args.cpu_workload} mesh ({om.n_leaves} leaves, "
                         f"the same RT workload two levels coarser), {tc:.1f}s on {cores} threads"}
        log(f"[bench] cpu baseline {cpu}")
        # one pass on one thread
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        om.jvp(op_, 1, U1c, U0c, dUc)
        t1 = time.perf_counter() - t0
        oracle.set_num_threads(cores)
        cpu["value_1thread_ns"] = round(4 * om.n_nodes / t1 / 1e9, 6)
        cpu["sample_1thread_ns"] = f"1 x NS JVP over the same mesh on one thread, {t1:.1f}s"
        log(f"[bench] cpu baseline, one thread: {cpu['value_1thread_ns']} GDoF/s (NS)")

    res = {
        "metric": "CHNS JVP GDoF/s", "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_total / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": name, "leaves": E, "nodes": n, "hanging": n_hanging,
                   "precision": args.precision, "step": "in-solver Newton-GMRES(30) pass of both blocks",
                   "gmres_per_block": K_GMRES,
                   "p50_ms": round(float(np.percentile(lat, 50)), 3),
                   "p99_ms": round(float(np.percentile(lat, 99)), 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cn_steps": steps,
        "oracle_anchor": anchor,
        "serving": serving_summary,
        "q2_ch": q2,
        "kernels": {k: round(v, 4) for k, v in kern.items()},
        "kernel_roofline": kernel_roofline(kern, n, E),
        "bench_wall_s": round(time.time() - t_bench, 1),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
