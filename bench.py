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

The JSON line carries a roofline object for the dominant kernel (the one with
the larger device time per solve among the dual-operator interface GEMV and
the factor's tile update), timed live with HIP events on the library stream in
a second timed pass of the same steps, and the CPU oracle timed on the host.

The mixed-precision path (FP32 local factors and GEMV values, FP64 dual
iteration and coarse problem) is reported beside it at the same accuracy: its
first dual solve stops at --mixed-rtol, and the outer refinement runs until
the FP64 residual ||f - K u|| / ||f|| is no larger than the FP64 path's.

Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]
  python bench.py --copy-calibration     # plain 1 GiB device copy (HBM counter scale)
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


def cpu_baseline(mesh, budget_s=20.0):
    """The oracle (monolithic sparse direct FP64 solve) on the host, one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import monolithic
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n = 0
        while True:
            monolithic.solve_linear(mesh)
            n += 1
            if time.perf_counter() - t0 > budget_s or n >= 20:
                break
        dt = (time.perf_counter() - t0) / n
    return dict(value=1.0 / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} complete monolithic solves of the benchmark workload (NumPy assembly, "
                       f"SuperLU symmetric-mode factor and solve), {dt:.2f} s each")


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
    gemv = {"kernel": "k_symv_tiles", "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
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
    """The HGO tube under its inner-pressure ramp to 16 mmHg: tau = s/n,
    s = 1..n (n = --load-steps, default 40: 0.4 mmHg per load step; with 10
    steps of 1.6 mmHg Newton stalls on this mesh, as the oracle's Newton does
    on the 4x32x16 tube), each load step solved by Newton from the previous
    equilibrium, every Newton step one FETI solve (factor at U_k + dual PCG).
    A load step converges when the residual norm at U_k is at most
    newton_tol times its value at the start of the load step.  When no damped
    step decreases the residual any more before that (the floor of the
    inexact steps), the path stops there and the line says so: the states
    after it would not be equilibria.

    Kernels: all six rigid modes for every floating subdomain, as in the paper
    (FETI_KERNEL6): away from U = 0 the stressed local tangents of this mesh
    are indefinite in rotation directions (compressive stress), so each
    Newton step solves that approximate tangent system (an inexact Newton
    step; --exact-steps refines it against the exact sparse tangent).  The
    residual, and so the equilibrium reached, is exact either way.

    Damping (not in the paper's scheme): with kappa = 1000 c the first
    linearised step of a load step can overshoot into states where the
    tangent is indefinite (a non-positive pivot, or a PCG breakdown).  A trial point U + a dU (a = 1, 1/2, ...) is
    accepted when its FETI solve succeeds and its residual is smaller; that
    solve's increment is then the next Newton step, so an accepted full step
    costs no extra solve.  The metric counts accepted Newton steps (FETI
    solves) per second of the whole path, rejected trials included in the
    time.  Returns the JSON line."""
    import torch
    from workloads import config_mesh
    from paper_1508_02599_amd.feti import Problem, FetiError

    mesh = config_mesh(args.config)
    n = mesh.n_dofs
    rtol = args.rtol if args.precision == "fp64" else args.mixed_rtol
    p = Problem(mesh, variant=args.variant, precond="dirichlet", precision=args.precision, rtol=rtol,
                ir_tol=args.ir_tol if args.ir_tol > 0 else 1e-10, ir_max=20 if args.exact_steps else 0,
                max_it=3000, device_ptrs=True, kernel6=True)
    U = torch.zeros(n, dtype=torch.float64, device="cuda")
    for _ in range(2):      # autotuning factorisations (untimed)
        p.factor(U)
    lat, its, res_hist = [], [], []
    newton_per_load, rejected, accepted = [], 0, 0

    def step(Ux, tau):
        d = torch.empty_like(Ux)
        a = time.perf_counter()
        try:
            _, rn, st = p.newton_step(Ux, tau, out=d)
            ok = True
        except FetiError as e:
            # an indefinite tangent (non-positive pivot, or s.Fs <= 0 in the
            # dual iteration) or a dual iteration that does not converge
            # rejects a trial point
            if e.status not in (-4, -5, -7):
                raise
            rn, st, ok = float("inf"), {"iters": 0}, False
        lat.append(time.perf_counter() - a)
        its.append(st["iters"])
        print(f"tau={tau:.3f} solve {len(lat)}: ok={ok} res={rn:.3e} pcg_it={st['iters']} "
              f"sweeps={st.get('ir_sweeps', 0)} {1e3 * lat[-1]:.0f} ms", file=sys.stderr, flush=True)
        return ok, d, rn

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    failed = None
    nload = args.load_steps
    for s in range(1, nload + 1):
        tau = s / nload
        ok, dU, rn = step(U, tau)
        if not ok:
            failed = f"tangent not SPD at the start of load step {s}"
            break
        accepted += 1
        r_start = rn
        tol = args.newton_tol * rn
        k = 0
        while rn > tol and k < 30:
            if time.perf_counter() - t0 > args.time_budget:
                failed = f"time budget of {args.time_budget:g} s spent in load step {s}"
                break
            k += 1
            a = 1.0
            while True:
                Ut = U + a * dU
                ok_t, dUt, rn_t = step(Ut, tau)
                if ok_t and rn_t < rn:
                    U, dU, rn = Ut, dUt, rn_t
                    accepted += 1
                    break
                rejected += 1
                a *= 0.5
                if a < 1.0 / 256:
                    break
            if a < 1.0 / 256:
                # no descent left: the residual is at the floor of the inexact steps
                break
            if failed:
                break
        res_hist.append(rn / r_start)
        newton_per_load.append(k)
        if not failed and rn > tol:
            failed = (f"Newton stalled in load step {s} (tau = {tau:g}) at |r| = {rn / r_start:.2e} of its "
                      f"start value (tolerance {args.newton_tol:g})")
        if failed:
            break
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    p.close()
    nsteps = len(lat)
    done = len(res_hist) - (1 if failed else 0)
    line = {
        "metric": "FETI Newton steps/s on the HGO tube load path (each step one FETI solve)",
        "value": accepted / total, "unit": "newton_steps/s", "n_gpus": 1, "steps": accepted, "warmup": 0,
        "ms_per_step": 1e3 * total / max(1, accepted), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32-local/f64-global",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: two-layer HGO tube, 16x128x64 Q1-P0 elements in "
                               f"{mesh.n_sub} subdomains ({args.variant}, Dirichlet preconditioner, six-mode "
                               f"kernels), "
                               f"inner pressure 16 mmHg x s/{nload}, s = 1..{nload}, damped "
                               f"{'exact' if args.exact_steps else 'inexact'} Newton to "
                               f"|r| <= {args.newton_tol:g} |r_0| per load step",
                   "global_dofs": n},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "load_steps_done": done, "load_steps": nload, "pressure_reached_mmHg": 16.0 * done / nload,
        "newton_steps_per_load_step": newton_per_load,
        "feti_solves": nsteps, "rejected_trials": rejected,
        "pcg_iterations": {"mean": float(np.mean(its)), "max": int(np.max(its))},
        "final_relative_residuals": res_hist,
    }
    if failed:
        line["error"] = failed
    return line


def workload_text(args, mesh):
    """One-line description of a linear workload, with its sizes."""
    kind = "all-floating" if args.variant == "af" else "classical"
    tail = f"{args.precond} preconditioner, PCG rtol {args.rtol:g}"
    if args.config.startswith("random"):
        return (f"{args.config}: unit cube 64^3 Q1 elements in 8x8x8 {kind} boxes with seeded slab "
                f"widths in 4..12 elements ({mesh.n_sub} subdomains of 300-6000 DOFs), E = 1, nu = 0.3, "
                f"smooth random body force, {tail}")
    return (f"{args.config}: unit cube 32^3 Q1 elements in 4x4x4 {kind} subdomains of 8^3 elements "
            f"(2187 DOFs each), nu per subdomain ~ U[0.25,0.35] (seed 0), {tail}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cube32_s4")
    ap.add_argument("--variant", default="af")
    ap.add_argument("--precond", default="lumped")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--mixed-rtol", type=float, default=1e-6,
                    help="PCG tolerance of the first dual solve of the mixed path")
    ap.add_argument("--ir-tol", type=float, default=0.0,
                    help="--precision mixed: refinement target (0: library default)")
    ap.add_argument("--newton-tol", type=float, default=1e-3,
                    help="tube load path: residual reduction (relative to the start of a load step) "
                         "that ends it")
    ap.add_argument("--load-steps", type=int, default=40, help="tube load path: load increments to 16 mmHg")
    ap.add_argument("--exact-steps", action="store_true",
                    help="tube load path: refine each Newton step against the exact tangent")
    ap.add_argument("--time-budget", type=float, default=240.0,
                    help="tube load path: wall-clock limit (s); a partial path is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
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
    mesh, total, pcg_total, lat, st_all = run(args, args.precision, profile=False,
                                              rtol=args.rtol if args.precision == "fp64" else args.mixed_rtol,
                                              ir_tol=args.ir_tol)
    st = st_all[-1]
    # roofline pass: same workload, kernel timings with HIP events
    _, ptotal, _, _, pst = run(args, args.precision, profile=True,
                               rtol=args.rtol if args.precision == "fp64" else args.mixed_rtol,
                               ir_tol=args.ir_tol)
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
        # mixed precision at the same accuracy: FP32 local factors, first dual
        # solve to mixed_rtol, then refinement until the FP64 residual is no
        # larger than the FP64 path's
        ir_tol = max(res64, 1e-14)
        try:
            _, tm, pm, lm, sm = run(args, "mixed", profile=False, rtol=args.mixed_rtol, ir_tol=ir_tol)
            _, _, _, _, smp = run(args, "mixed", profile=True, rtol=args.mixed_rtol, ir_tol=ir_tol)
        except Exception as e:   # reported as unavailable, never as a number
            line["mixed"] = {"error": str(e)}
            tm = None
    if args.precision == "fp64" and not args.no_mixed and tm is not None:
        d2, o2 = roofline(smp, "mixed")
        line["mixed"] = {"value": args.steps / tm, "unit": "solves/s",
                         "speedup_vs_fp64": (args.steps / tm) / line["value"],
                         "first_solve_rtol": args.mixed_rtol, "ir_tol": ir_tol,
                         "res_primal": sm[-1]["res_primal"],
                         "latency_ms": {"p50": 1e3 * float(np.percentile(lm, 50)),
                                        "p99": 1e3 * float(np.percentile(lm, 99))},
                         "pcg_only_solves_per_s": args.steps / pm, "iters": sm[-1]["iters"],
                         "ir_sweeps": sm[-1]["ir_sweeps"],
                         "phase_ms": {k: 1e3 * sm[-1][k] for k in ("t_assemble", "t_factor", "t_pcg")},
                         "roofline": d2, "roofline_secondary": o2}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
