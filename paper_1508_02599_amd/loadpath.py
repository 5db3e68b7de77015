"""Load stepping of a nonlinear problem with Newton steps on the GPU.

The external load is ramped, tau = tau_done + dtau (eq. (loadStepping)), and
each load step is solved by Newton from the previous equilibrium (eqs.
(NewtonRecursion), (LGS)); every Newton step is one feti_newton_step of a
Problem, normally the exact linearisation (load_stiffness=True).

Control around the paper's scheme (none of it changes a Newton step):
- inexact Newton: each step's linear system is solved to the Eisenstat-Walker
  forcing term eta_k = 0.9 (|r_k| / |r_{k-1}|)^2, within [eta_floor, eta_max]
  with eta_floor = 0.1 newton_tol |r_0| / |r_k| (feti_set_tolerances), so the
  refinement never chases accuracy the load step does not need;
- load-step cutting: if a load step meets an element inverted by U, a local
  factor that fails, or no convergence within max_newton steps, the
  increment is halved and retried from the last equilibrium (down to 1/64 of
  the nominal increment); it doubles back after two accepted steps.
"""
from __future__ import annotations

import sys
import time


def run_load_path(p, U, n_inc, *, rtol=1e-8, newton_tol=1e-8, eta_max=1e-3, max_newton=12,
                  time_budget=float("inf"), record=None, log=sys.stderr, tau_end=1.0):
    """Ramp tau from 0 to tau_end in nominal increments of 1/n_inc on Problem
    p (device pointers) from the displacement tensor U (updated in place).

    record(tau, k, U): called with every Newton iterate of every accepted load
    step (k = 0: the previous equilibrium).  Returns a dict of the path's
    statistics (per Newton step: latency, PCG iterations, refinement
    iterations) and the load factor reached."""
    import torch
    from .feti import FetiError

    out = dict(latency=[], pcg=[], gmres=[], newton_per_load=[], taus=[], res=[],
               accepted_steps=0, rejected_steps=0, cuts=0, error=None)

    def step(Ux, tau):
        d = torch.empty_like(Ux)
        a = time.perf_counter()
        # a step whose refinement stopped short of its target is an inexact
        # Newton step: the next residual decides
        _, rn, st = p.newton_step(Ux, tau, out=d, allow_noconv=True)
        out["latency"].append(time.perf_counter() - a)
        out["pcg"].append(st["iters"])
        out["gmres"].append(st["ir_sweeps"])
        if log is not None:
            print(f"tau={tau:.5f} newton step {len(out['latency'])}: res={rn:.3e} pcg_it={st['iters']} "
                  f"gmres={st['ir_sweeps']} modified={st['modified_pivots']} {1e3 * out['latency'][-1]:.0f} ms",
                  file=log, flush=True)
        return d, rn

    t0 = time.perf_counter()
    nominal = 1.0 / n_inc
    dt, tau_done, streak = nominal, 0.0, 0
    while tau_done < tau_end - 1e-12:
        if time.perf_counter() - t0 > time_budget:
            out["error"] = f"time budget of {time_budget:g} s spent at tau = {tau_done:g}"
            break
        tau = min(tau_end, tau_done + dt)
        Ut = U.clone()
        iterates = [Ut.clone()]
        r_start, r_prev, k, ok, why, n_try = None, None, 0, False, "", 0
        eta = eta_max
        try:
            while True:
                p.set_tolerances(rtol, eta)
                dU, rn = step(Ut, tau)
                n_try += 1
                if r_start is None:
                    r_start = rn
                if rn <= newton_tol * r_start:
                    ok = True
                    break
                if k >= max_newton or rn > 1e6 * r_start:
                    why = f"no convergence ({rn / r_start:.1e} after {k} steps)"
                    break
                eta = eta_max if r_prev is None else min(eta_max, 0.9 * (rn / r_prev) ** 2)
                eta = min(eta_max, max(eta, 0.1 * newton_tol * r_start / max(rn, 1e-300), 1e-12))
                r_prev = rn
                Ut += dU
                k += 1
                iterates.append(Ut.clone())
        except FetiError as e:
            why = str(e)
        if ok:
            U.copy_(Ut)
            if record is not None:
                for kk, Uk in enumerate(iterates):
                    record(tau, kk, Uk)
            tau_done = tau
            out["accepted_steps"] += n_try
            out["newton_per_load"].append(k)
            out["res"].append(rn / r_start)
            out["taus"].append(tau)
            streak += 1
            if streak >= 2 and dt < nominal:
                dt, streak = min(nominal, 2.0 * dt), 0
        else:
            out["rejected_steps"] += n_try
            out["cuts"] += 1
            streak = 0
            dt *= 0.5
            if log is not None:
                print(f"tau={tau:.5f}: increment rejected ({why}); halved to {dt:.5f}", file=log, flush=True)
            if dt < nominal / 64:
                out["error"] = f"load increment below 1/64 of the nominal one at tau = {tau_done:g}: {why}"
                break
    torch.cuda.synchronize()
    out["wall_s"] = time.perf_counter() - t0
    out["tau_reached"] = tau_done
    return out


def trajectory_states(p, n_inc=40, n_steps=10, iterates=4, **kw):
    """Newton iterates along the converged load path of Problem p (device
    pointers): {(s, k): (tau, U)} for the load steps that end at
    tau = s / n_inc, s = 1..n_steps, and their iterates k = 0..iterates-1
    (k = 0: the equilibrium the load step starts from; U a host array).
    Keyword arguments go to run_load_path."""
    import numpy as np
    import torch

    states = {}

    def record(tau, k, Uk):
        s = tau * n_inc
        if abs(s - round(s)) < 1e-9 and k < iterates:
            states[(int(round(s)), k)] = (tau, Uk.double().cpu().numpy())

    U = torch.zeros(p.n_dof, dtype=torch.float64, device="cuda")
    r = run_load_path(p, U, n_inc, record=record, tau_end=n_steps / n_inc, **kw)
    if r["error"]:
        raise RuntimeError(f"load path stopped: {r['error']}")
    missing = [(s, k) for s in range(1, n_steps + 1) for k in range(iterates) if (s, k) not in states]
    if missing:
        raise RuntimeError(f"load path converged in fewer than {iterates} Newton steps at {missing[:4]}")
    return states
