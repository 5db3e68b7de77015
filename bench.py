"""Benchmark: FETI solves/s on one MI355X.

A step is one complete FETI solve of the workload with its inputs resident on
the device: assembly, batched factorisation of every subdomain (interior-first
Cholesky, regularised interface Schur complement and its inverse), coarse
problem, projected PCG to ||P r|| <= 1e-8 ||P r_0||, and recovery of the
displacements into a device buffer.

Default workload: unit cube of 32^3 Q1 elements in 4x4x4 all-floating
subdomains of 8^3 elements (2187 DOFs each), E = 1, nu per subdomain from
U[0.25, 0.35] (seed 0), body force (0, 0, -1), u = 0 on the boundary,
lumped preconditioner.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per solve, used for the roofline line:
# the dominant kernel is the batched left-looking tile update of the local
# Cholesky factorisation (MFMA FP64 / FP32).


def factor_flops(mesh_subs):
    """Sum over subdomains of n^3/3 (dense Cholesky) + 2 n_b^3/3 (interface inverse)."""
    tot = 0.0
    for n, nb in mesh_subs:
        tot += n ** 3 / 3.0 + 2.0 * nb ** 3 / 3.0
    return tot


def sub_sizes(mesh, variant="af"):
    """(n_i, n_b) per subdomain, from the mesh (host-side counting only)."""
    sizes = []
    node_subs = {}
    for e in range(mesh.n_elems):
        pass
    n_nodes = mesh.n_nodes
    copies = np.zeros(n_nodes, dtype=np.int64)
    sub_nodes = []
    for s in range(mesh.n_sub):
        nodes = np.unique(mesh.hex8[mesh.elem_sub == s])
        sub_nodes.append(nodes)
        copies[nodes] += 1
    dmask = np.zeros(mesh.n_dofs, dtype=bool)
    dmask[mesh.dir_dof] = True
    dnode = dmask.reshape(-1, 3).any(axis=1)
    for nodes in sub_nodes:
        iface = (copies[nodes] > 1) | (dnode[nodes] if variant == "af" else False)
        nb = 3 * int(iface.sum())
        sizes.append((3 * len(nodes), nb))
    return sizes


def cpu_baseline(mesh, budget_s=20.0):
    """Oracle (monolithic sparse direct FP64 solve) timed on the host."""
    from oracle import monolithic
    t0 = time.perf_counter()
    n = 0
    while True:
        monolithic.solve_linear(mesh)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 20:
            break
    dt = (time.perf_counter() - t0) / n
    return dict(value=1.0 / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} full monolithic solves of the same workload (assembly + SuperLU "
                       f"factor + solve, single-threaded), {dt:.2f} s each")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cube32_s4")
    ap.add_argument("--variant", default="af")
    ap.add_argument("--precond", default="lumped")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is "
              "described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from workloads import config_mesh
    from paper_1508_02599_amd.feti import Problem

    torch.cuda.set_device(0)
    mesh = config_mesh(args.config)
    stream = torch.cuda.current_stream()
    p = Problem(mesh, variant=args.variant, precond=args.precond, precision=args.precision,
                rtol=1e-8, device_ptrs=True, hip_stream=stream.cuda_stream)
    u = torch.empty(mesh.n_dofs, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        p.factor()
        p.solve(out=u)
    torch.cuda.synchronize()
    lat = []
    stats = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        p.factor()
        _, stats = p.solve(out=u)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # PCG-only throughput with the factors resident
    p.factor()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        p.solve(out=u)
    torch.cuda.synchronize()
    pcg_total = time.perf_counter() - t1
    value = args.steps / total
    sizes = sub_sizes(mesh, args.variant)
    fl = factor_flops(sizes)
    line = {
        "metric": "FETI PCG solves/s at 1e-8 residual (FP64 vs mixed); p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-local/f64-global",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: unit cube 32^3 Q1, 4x4x4 subdomains of 8^3 elements "
                               f"(2187 DOFs each), {args.variant}, {args.precond}, rtol 1e-8",
                   "subdomains": mesh.n_sub, "global_dofs": mesh.n_dofs},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "pcg_only_solves_per_s": args.steps / pcg_total,
        "iters": stats["iters"],
        "phase_s": {k: stats[k] for k in ("t_assemble", "t_factor", "t_pcg", "t_total")},
        "factor_flops": fl,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
