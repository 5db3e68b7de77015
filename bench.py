"""Benchmark: FETI solves/s on one MI355X.

A step is one complete FETI solve of the workload with its inputs resident on
the device: assembly, batched factorisation of every subdomain (interior-first
Cholesky, regularised interface Schur complement and its inverse), coarse
problem, projected PCG to ||P r|| <= 1e-8 ||P r_0||, and recovery of the
displacements into a device buffer.

Default workload (the largest single-GPU configuration): unit cube of 64^3 Q1
elements cut by seeded axis-aligned planes into 8x8x8 all-floating boxes of
630-5577 DOFs (823,875 DOFs, 484,956 multipliers), E = 1, nu = 0.3, u = 0 on
the boundary, smooth random body force, lumped preconditioner.  The 32^3 cube
in 4^3 boxes of 8^3 elements is `--config cube32_s4`.

The JSON line carries:
- a roofline object for the dominant kernel (the one with the larger device
  time per solve among the dual-operator interface GEMV and the factor's tile
  update), timed live with HIP events on the library stream in a second,
  profiled pass of the same steps;
- the mixed-precision path (FP32 local factors and GEMV values, FP64 dual
  iteration and coarse problem, flexible GMRES refinement against the FP64
  sparse operator) at the settings its parity test covers: first dual solve to
  --mixed-rtol, refinement to --mixed-ir-tol;
- accuracy against the oracle at these settings on the 40^3 cube in uneven
  boxes of the same sizes (stored sparse-direct solution): the displacement
  error of FP64 at rtol 1e-8 and of mixed, and the FP64 rtol that reaches
  1e-9;
- the CPU oracle timed on the host on a bounded sample of the workload.

Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--precision fp64|mixed]
  python bench.py --config tube_16x128x64          # HGO tube load path (exact Newton)
  python bench.py --copy-calibration                # plain 1 GiB device copy (HBM counter scale)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}   # dense FP64 / FP32 matrix peaks


def _sub_block(mesh, n_blk):
    """The corner block of n_blk^3 elements of a structured cube mesh as a mesh
    of its own (same elements, materials and body force, clamped on the
    block's boundary)."""
    from workloads.meshes import Mesh, _boundary_nodes_cube
    n_el = int(round(len(mesh.xyz) ** (1.0 / 3.0))) - 1
    idx = np.arange(mesh.n_nodes)
    i, j, k = idx % (n_el + 1), (idx // (n_el + 1)) % (n_el + 1), idx // (n_el + 1) ** 2
    keep_n = (i <= n_blk) & (j <= n_blk) & (k <= n_blk)
    new_id = -np.ones(mesh.n_nodes, dtype=np.int64)
    new_id[keep_n] = np.arange(int(keep_n.sum()))
    keep_e = keep_n[mesh.hex8].all(axis=1)
    hex8 = new_id[mesh.hex8[keep_e]]
    bnodes = _boundary_nodes_cube(n_blk, n_blk, n_blk)
    dir_dof = (3 * bnodes[:, None] + np.arange(3)[None, :]).ravel().astype(np.int64)
    return Mesh(xyz=mesh.xyz[keep_n], hex8=hex8, elem_sub=np.zeros(hex8.shape[0], dtype=np.int32), n_sub=1,
                mat=mesh.mat, elem_mat=mesh.elem_mat[keep_e], dir_dof=dir_dof, dir_val=np.zeros(dir_dof.size),
                body_force=None if mesh.body_force is None else mesh.body_force[keep_e], name="block")


def cpu_baseline(mesh, config, budget_s=20.0):
    """The oracle (monolithic sparse direct FP64 solve: NumPy assembly, SuperLU
    symmetric-mode factor and solve) on the host.  SuperLU runs on one thread.
    For the 64^3 workload a whole solve takes far longer than the benchmark's
    budget, so the sample is the corner block of 24^3 of its elements (same
    element size, material and body force, clamped on the block's boundary),
    and solves/s is scaled by the DOF ratio: an upper bound for the full
    workload, since a sparse direct solve grows faster than linearly."""
    from threadpoolctl import threadpool_limits
    from oracle import monolithic
    sample = mesh
    if config.startswith("random"):
        sample = _sub_block(mesh, 24)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n = 0
        while True:
            monolithic.solve_linear(sample)
            n += 1
            if time.perf_counter() - t0 > budget_s or n >= 20:
                break
        dt = (time.perf_counter() - t0) / n
    scale = sample.n_dofs / mesh.n_dofs
    if sample is mesh:
        what = f"{n} complete monolithic solves of the benchmark workload, {dt:.2f} s each"
    else:
        what = (f"{n} monolithic solves of the 24^3-element corner block of the workload "
                f"({sample.n_dofs} of {mesh.n_dofs} DOFs, clamped on the block boundary), {dt:.2f} s "
                f"each; solves/s scaled by the DOF ratio {scale:.4f} (an upper bound: a sparse direct "
                f"solve grows faster than linearly)")
    return dict(value=scale / dt, unit="solves/s", cores=1, host_cores=os.cpu_count(), kind="oracle",
                sample=what)


def _load_reference(case, mesh):
    """Oracle solution stored by tests/golden/make_fullsize_refs.py for this input, or None."""
    import importlib.util
    path = os.path.join(ROOT, "tests", "golden", "make_fullsize_refs.py")
    spec = importlib.util.spec_from_file_location("make_fullsize_refs", path)
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    f = mk.path_for(case, mk.fullsize_key(mesh))
    return np.load(f) if os.path.exists(f) else None


def accuracy(args):
    """Displacement error against the oracle at the benchmark's settings, on
    the 40^3 cube in uneven boxes of the 64^3 workload's sizes (450-5616 DOFs;
    the oracle's direct solve of the 64^3 cube itself is out of reach)."""
    from workloads import config_mesh
    from paper_1508_02599_amd.feti import Problem
    m = config_mesh("random_boxes_40")
    ref = _load_reference("random_boxes_40", m)
    if ref is None:
        return {"error": "no stored oracle solution for random_boxes_40"}

    def err(u):
        return max(float(np.linalg.norm(u - ref) / np.linalg.norm(ref)),
                   float(np.abs(u - ref).max() / np.abs(ref).max()))
    out = {"workload": "random_boxes_40: unit cube 40^3 Q1 elements in 5x5x5 all-floating boxes of "
                       "450-5616 DOFs (seed 0), lumped preconditioner; error = max(relative 2-norm, "
                       "element-wise max relative to max|u|) against the oracle's sparse direct solution"}
    fp64 = {}
    for rt in (1e-8, 1e-9, 1e-10, 1e-11):
        with Problem(m, variant=args.variant, precond=args.precond, precision="fp64", rtol=rt) as p:
            p.factor()
            u, st = p.solve()
        fp64[f"{rt:g}"] = {"err": err(u), "iters": st["iters"]}
    out["fp64_by_rtol"] = fp64
    out["fp64_err_at_rtol_1e-8"] = fp64["1e-08"]["err"]
    reach = [rt for rt in ("1e-08", "1e-09", "1e-10", "1e-11") if fp64[rt]["err"] <= 1e-9]
    out["fp64_rtol_reaching_1e-9"] = float(reach[0]) if reach else None
    with Problem(m, variant=args.variant, precond=args.precond, precision="mixed", rtol=args.mixed_rtol,
                 ir_tol=args.mixed_ir_tol) as p:
        p.factor()
        u, st = p.solve()
    out["mixed"] = {"err": err(u), "first_solve_rtol": args.mixed_rtol, "ir_tol": args.mixed_ir_tol,
                    "iters": st["iters"], "gmres_iterations": st["ir_sweeps"]}
    return out


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    try:
        rec = json.load(open(f)).get(kernel)
        if not rec:
            return None
        src = os.path.join(ROOT, rec["source"])
        if source_sha(src) != rec["source_sha"]:
            return None
        return rec["hbm_bytes_per_launch"]
    except Exception:
        return None


def copy_calibration():
    import torch
    n = 1 << 27   # 128 Mi doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}))


def run(args, precision, profile=True, rtol=1e-8, ir_tol=0.0):
    import torch
    from workloads import config_mesh
    from paper_1508_02599_amd.feti import AUTOTUNE_FACTORISATIONS, Problem

    mesh = config_mesh(args.config)
    p = Problem(mesh, variant=args.variant, precond=args.precond, precision=precision, rtol=rtol,
                ir_tol=ir_tol, device_ptrs=True, profile=profile)
    u = torch.empty(mesh.n_dofs, dtype=torch.float64, device="cuda")
    # the autotuner times the update forms in the first factorisations
    # (untimed set-up, before the warmup steps)
    for _ in range(AUTOTUNE_FACTORISATIONS):
        p.factor()
    for _ in range(args.warmup):
        p.factor()
        p.solve(out=u)
    torch.cuda.synchronize()
    lat, st_all = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        p.factor()
        _, st = p.solve(out=u)
        lat.append(time.perf_counter() - a)
        st_all.append(st)
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
    p.close()
    return mesh, total, pcg_total, lat, st_all


def roofline(st_all, precision):
    """Roofline of the dominant kernel from the live HIP-event timings: the F
    GEMV (mean of a back-to-back burst after each solve) and the factor's tile
    update (events around each launch)."""
    g_ms = float(np.mean([s["kernel_gemv_ms"] for s in st_all]))
    g_n = float(np.mean([s["kernel_gemv_launches"] for s in st_all]))
    u_ms = float(np.mean([s["kernel_update_ms"] for s in st_all]))
    u_n = float(np.mean([s["kernel_update_launches"] for s in st_all]))
    gb = st_all[-1]["gemv_bytes"]
    gemv = {"kernel": "k_symv_one", "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "achieved": gb / (g_ms * 1e-3) / 1e9 if g_ms > 0 else None,
            "avg_launch_ms": g_ms, "launches_per_solve": g_n,
            "algorithmic_bytes_per_launch": gb}
    uf = st_all[-1]["update_flops"] / max(u_n, 1)
    upd = {"kernel": "k_update", "bound": "mfma", "unit": "TFLOP/s",
           "peak": MFMA_PEAK_TFLOPS[precision],
           "achieved": uf / (u_ms * 1e-3) / 1e12 if u_ms > 0 else None,
           "avg_launch_ms": u_ms, "launches_per_solve": u_n,
           "algorithmic_flops_per_launch": uf}
    for r in (gemv, upd):
        r["frac"] = r["achieved"] / r["peak"] if r["achieved"] else None
        r["device_ms_per_solve"] = r["avg_launch_ms"] * r["launches_per_solve"]
    dom, other = (gemv, upd) if gemv["device_ms_per_solve"] >= upd["device_ms_per_solve"] else (upd, gemv)
    suffix = "_f32" if precision == "mixed" else ""
    for r in (dom, other):
        t = traffic_from_profiles(r["kernel"] + suffix)
        r["traffic"] = t
    return dom, other


def tube_load_path(args):
    """The HGO tube under its inner-pressure ramp to P mmHg (--end-mmhg,
    default 16) in load increments of P/n mmHg (n = --load-steps, default 40:
    0.4 mmHg; the paper
    likewise reports that its Newton method needs small pressure steps), each
    load step solved by Newton from the previous equilibrium
    (paper_1508_02599_amd.loadpath: inexact Newton forcing, load-step
    cutting), every Newton step the exact linearisation (FETI_LOAD_STIFFNESS:
    the follower-pressure load stiffness is kept, so Newton converges
    quadratically) until ||r|| <= newton_tol ||r_0|| of the load step.

    Each Newton step: assembly and factorisation at U_k with the kernels of
    the stressed floating subdomains (translations, and the rotations whose
    stress-induced stiffness ||K r|| is at most --kernel-tol ||K|| ||r||; the
    tangent solved is then approximate and refined below), one FETI solve
    warm-started from the previous step's multipliers (FETI_WARM_START) whose
    dual problem is solved by projected GMRES (FETI_DUAL_GMRES: the stressed
    local tangents are indefinite in rotation directions, so F is), then
    flexible GMRES on the assembled exact operator preconditioned by FETI
    solves.  The metric counts Newton steps (each one factorisation and its
    FETI-preconditioned solve) per second of the whole path, rejected
    attempts included in the time.  Returns the JSON line."""
    import torch
    from workloads import config_mesh
    from paper_1508_02599_amd.feti import AUTOTUNE_FACTORISATIONS, Problem
    from paper_1508_02599_amd.loadpath import run_load_path

    from workloads.meshes import MMHG
    mesh = config_mesh(args.config, pressure=args.end_mmhg * MMHG)
    n = mesh.n_dofs
    rtol = args.rtol if args.precision == "fp64" else args.mixed_rtol
    p = Problem(mesh, variant=args.variant, precond="dirichlet", precision=args.precision, rtol=rtol,
                ir_tol=args.newton_eta_max, ir_max=60, max_it=3000, device_ptrs=True, load_stiffness=True,
                warm_start=not args.cold_start, dual_gmres=args.dual == "gmres", kernel_tol=args.kernel_tol)
    U = torch.zeros(n, dtype=torch.float64, device="cuda")
    for _ in range(AUTOTUNE_FACTORISATIONS):      # autotuning factorisations (untimed)
        p.factor(U)
    torch.cuda.synchronize()
    r = run_load_path(p, U, args.load_steps, rtol=rtol, newton_tol=args.newton_tol, eta_max=args.newton_eta_max,
                      max_newton=args.max_newton, time_budget=args.time_budget)
    p.close()
    lat, its, gm = r["latency"], r["pcg"], r["gmres"]
    nsteps = len(lat)
    total = r["wall_s"]
    line = {
        "metric": "FETI Newton steps/s on the HGO tube load path (each step one factorisation and its "
                  "FETI-preconditioned exact solve)",
        "value": nsteps / total, "unit": "newton_steps/s", "n_gpus": 1, "steps": nsteps, "warmup": 0,
        "ms_per_step": 1e3 * total / max(1, nsteps), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32-local/f64-global",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: two-layer HGO tube, {mesh.meta['nr']}x{mesh.meta['nth']}x"
                               f"{mesh.meta['nz']} Q{mesh.order}-P0 elements in "
                               f"{mesh.n_sub} subdomains ({args.variant}, Dirichlet preconditioner, kernel "
                               f"tolerance {args.kernel_tol:g}, "
                               f"{'projected dual GMRES' if args.dual == 'gmres' else 'dual PCG'}, "
                               f"{'cold' if args.cold_start else 'warm'} starts), inner pressure to {args.end_mmhg:g} "
                               f"mmHg in increments of {args.end_mmhg / args.load_steps:g} mmHg (halved on failure), "
                               f"exact Newton "
                               f"(follower-load stiffness) to |r| <= {args.newton_tol:g} |r_0| per load step",
                   "global_dofs": n},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "pressure_reached_mmHg": args.end_mmhg * r["tau_reached"], "load_steps_done": len(r["taus"]),
        "newton_steps_per_load_step": r["newton_per_load"],
        "accepted_steps": r["accepted_steps"], "rejected_steps": r["rejected_steps"], "cuts": r["cuts"],
        "pcg_iterations": {"mean": float(np.mean(its)), "max": int(np.max(its)), "total": int(np.sum(its))},
        "gmres_iterations": {"mean": float(np.mean(gm)), "max": int(np.max(gm))},
        "final_relative_residuals": r["res"],
    }
    if r["error"]:
        line["error"] = r["error"]
    return line


def workload_text(args, mesh):
    """One-line description of a linear workload, with its sizes."""
    kind = "all-floating" if args.variant == "af" else "classical"
    tail = f"{args.precond} preconditioner, PCG rtol {args.rtol:g}"
    if args.config.startswith("random"):
        return (f"{args.config}: unit cube 64^3 Q1 elements in 8x8x8 {kind} boxes with seeded slab "
                f"widths in 4..12 elements ({mesh.n_sub} subdomains of 300-6000 DOFs), E = 1, nu = 0.3, "
                f"smooth random body force, {tail}")
    n_el, ns, q = mesh.meta["n_el"], mesh.meta["n_sub_axis"], mesh.order
    h = n_el // ns
    return (f"{args.config}: unit cube {n_el}^3 Q{q} elements in {ns}x{ns}x{ns} {kind} subdomains of {h}^3 "
            f"elements ({3 * (q * h + 1) ** 3} DOFs each), nu per subdomain ~ U[0.25,0.35] (seed 0), {tail}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="random_boxes_64")
    ap.add_argument("--variant", default=None,
                    help="af or classical (default: af; classical on the tube load path)")
    ap.add_argument("--dual", default="gmres", choices=("gmres", "pcg"),
                    help="tube load path: dual solver (projected GMRES or PCG)")
    ap.add_argument("--precond", default="lumped")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--mixed-rtol", type=float, default=1e-6,
                    help="PCG tolerance of the first dual solve of the mixed path")
    ap.add_argument("--mixed-ir-tol", type=float, default=1e-10,
                    help="refinement target of the mixed path, ||b - A u|| <= ir_tol ||b|| (FP64, assembled)")
    ap.add_argument("--newton-tol", type=float, default=1e-8,
                    help="tube load path: residual reduction (relative to the start of a load step) "
                         "that ends it")
    ap.add_argument("--max-newton", type=int, default=12, help="tube load path: Newton steps per load step")
    ap.add_argument("--newton-eta-max", type=float, default=1e-3,
                    help="tube load path: loosest GMRES target of a Newton step (inexact Newton)")
    ap.add_argument("--load-steps", type=int, default=40, help="tube load path: load increments to --end-mmhg")
    ap.add_argument("--end-mmhg", type=float, default=16.0, help="tube load path: end pressure (mmHg)")
    ap.add_argument("--cold-start", action="store_true", help="tube load path: no multiplier warm starts")
    ap.add_argument("--kernel-tol", type=float, default=1e-6,
                    help="tube load path: rotations with ||K r|| <= tol ||K|| ||r|| join the local kernels")
    ap.add_argument("--time-budget", type=float, default=240.0,
                    help="tube load path: wall-clock limit (s); a partial path is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.variant is None:
        args.variant = "classical" if args.config.startswith("tube") else "af"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding the subdomains "
              "over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.config.startswith("tube"):
        print(json.dumps(tube_load_path(args)))
        return
    mixed_kw = dict(rtol=args.mixed_rtol, ir_tol=args.mixed_ir_tol)
    kw = dict(rtol=args.rtol, ir_tol=0.0) if args.precision == "fp64" else mixed_kw
    mesh, total, pcg_total, lat, st_all = run(args, args.precision, profile=False, **kw)
    st = st_all[-1]
    # roofline pass: same workload, kernel timings with HIP events
    _, ptotal, _, _, pst = run(args, args.precision, profile=True, **kw)
    dom, other = roofline(pst, args.precision)
    dom["profiled_pass_ms_per_step"] = 1e3 * ptotal / args.steps
    res64 = pst[-1]["res_primal"]
    line = {
        "metric": "FETI PCG solves/s at 1e-8 residual (FP64 vs mixed); p50/p99 solve latency",
        "value": args.steps / total,
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
        "config": {"workload": workload_text(args, mesh),
                   "subdomains": mesh.n_sub, "global_dofs": mesh.n_dofs,
                   "multipliers": st["n_lambda"], "coarse_dim": st["n_coarse"]},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "pcg_only_solves_per_s": args.steps / pcg_total,
        "iters": st["iters"],
        "res_primal": res64,
        "phase_ms": {k: 1e3 * st[k] for k in ("t_assemble", "t_factor", "t_pcg")},
        "roofline": {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": {k: v for k, v in dom.items()
                            if k not in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_secondary": other,
    }
    tm = None
    if args.precision == "fp64" and not args.no_mixed:
        # mixed precision at the settings its parity test covers: FP32 local
        # factors, first dual solve to mixed_rtol, flexible GMRES refinement
        # against the FP64 sparse operator to mixed_ir_tol
        try:
            _, tm, pm, lm, sm = run(args, "mixed", profile=False, **mixed_kw)
            _, _, _, _, smp = run(args, "mixed", profile=True, **mixed_kw)
        except Exception as e:   # reported as unavailable, never as a number
            line["mixed"] = {"error": str(e)}
            tm = None
    if args.precision == "fp64" and not args.no_mixed and tm is not None:
        d2, o2 = roofline(smp, "mixed")
        line["mixed"] = {"value": args.steps / tm, "unit": "solves/s",
                         "speedup_vs_fp64": (args.steps / tm) / line["value"],
                         "first_solve_rtol": args.mixed_rtol, "ir_tol": args.mixed_ir_tol,
                         "res_primal": sm[-1]["res_primal"],
                         "latency_ms": {"p50": 1e3 * float(np.percentile(lm, 50)),
                                        "p99": 1e3 * float(np.percentile(lm, 99))},
                         "pcg_only_solves_per_s": args.steps / pm, "iters": sm[-1]["iters"],
                         "gmres_iterations": sm[-1]["ir_sweeps"],
                         "phase_ms": {k: 1e3 * sm[-1][k] for k in ("t_assemble", "t_factor", "t_pcg")},
                         "roofline": d2, "roofline_secondary": o2}
    if not args.no_accuracy and args.config.startswith("random"):
        line["accuracy"] = accuracy(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh, args.config)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
