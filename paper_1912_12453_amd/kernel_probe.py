"""Launches single element kernels of a workload, and a device copy of known
size, for hardware counter collection (rocprofv3 --pmc).

Usage: python kernel_probe.py [--workload bubble_l9] [--reps 5] KIND...
KIND: ns64 ns32 ch64 ch32 nsres chres nsdiag chdiag nslin64 nslin32 chlin64 chlin32 copy

The copy kernel reads and writes 1 GiB; its FETCH_SIZE and WRITE_SIZE give
the factors that turn the counters into HBM bytes.
"""
import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="bubble_l9")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("kinds", nargs="+")
    a = ap.parse_args()
    import torch

    from paper_1912_12453_amd import chns
    from paper_1912_12453_amd import workloads as W

    print("probe: start", flush=True)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = W.by_name(a.workload)
    m = chns.Mesh.from_spec(w.mesh)
    m.upload()
    xyz, bf = m.nodes()
    U1h, U0h = W.state_for(w, xyz, bf)
    U1 = torch.tensor(U1h, device=dev)
    U0 = torch.tensor(U0h, device=dev)
    dU = torch.tensor(W.direction(m.n_nodes, 3), device=dev)
    dU32 = dU.float()
    p = chns.make_params(w.physics)
    print(f"probe: {a.workload} {m.n_leaves} leaves {m.n_nodes} nodes", flush=True)
    table = {  # kind: (block, op, direction)
        "chres": (0, 0, None), "ch64": (0, 1, dU), "ch32": (0, 2, dU32), "chdiag": (0, 3, None),
        "nsres": (1, 0, None), "ns64": (1, 1, dU), "ns32": (1, 2, dU32), "nsdiag": (1, 3, None),
    }
    for k in a.kinds:
        if k in ("nslin64", "nslin32", "chlin64", "chlin32"):  # linearise once, then the cached JVP
            blk = 1 if k.startswith("ns") else 0
            op = 4 if k.endswith("64") else 6
            d = dU if k.endswith("64") else dU32
            chns.chns_launch_element_loop(m.h, p, blk, op + 1, U1, U0, None, None, 1)
            chns.chns_launch_element_loop(m.h, p, blk, op, U1, U0, d, None, a.reps)
        elif k == "copy":
            src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
        elif k in table:
            blk, op, d = table[k]
            chns.chns_launch_element_loop(m.h, p, blk, op, U1, U0, d, None, a.reps)
        else:
            raise SystemExit(f"unknown kind {k}")
        torch.cuda.synchronize()
        print(f"probe: {k} done", flush=True)
    print("probe: end", flush=True)


if __name__ == "__main__":
    main()
