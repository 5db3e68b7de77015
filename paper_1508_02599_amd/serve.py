"""Serving loop: FETI solves and Newton steps of different meshes on one GPU.

Requests arrive over time (open loop).  A request is admitted as soon as a
worker slot is free and the device memory it needs fits the budget: an idle
problem of the same mesh is reused (its device-resident decomposition, and for
linear problems its factors, are kept between requests); otherwise a new
problem is set up, after evicting idle problems of other meshes
(least recently used first) if the budget requires it.  Admitted requests run
concurrently, each problem on its own HIP stream, so work arriving while
others are on the GPU overlaps with them.  Every reduction of the library has a
fixed order and each problem owns its buffers, so a request's result does not
depend on what else runs.

    python -m paper_1508_02599_amd.serve [--requests 256] [--rate-multiples 0.25,0.5,1,2,4]
                                         [--precision fp64|mixed] [--workers 4]

computes the tube's load path once (the states of its Newton requests),
measures the saturation rate (every request at t = 0), then prints one JSON
line per arrival rate (multiples of the saturation rate): throughput
(requests/s), p50/p99 latency from arrival to result, and the mix of work
served.
"""
from __future__ import annotations

import argparse
import json
import sys
import threading
import time
from collections import OrderedDict

import numpy as np

from .feti import Problem


class Request:
    def __init__(self, rid, key, kind, param, arrival):
        self.rid, self.key, self.kind, self.param, self.arrival = rid, key, kind, param, arrival
        self.result = None
        self.error = None
        self.t_start = self.t_done = None
        self.iters = 0
        self.done = threading.Event()

    @property
    def latency(self):
        return self.t_done - self.arrival


class _Slot:
    """A set-up problem of one mesh: device memory held until evicted."""

    def __init__(self, key, problem, footprint):
        self.key, self.p, self.bytes = key, problem, footprint
        self.factored_linear = False
        self.busy = False


class Server:
    """Admission by slots and device memory; see the module docstring.

    mesh_fn(key) builds the mesh of a request key; options are passed to every
    problem (variant, precond, precision, rtol, ...); options_for(key) adds
    per-mesh options; states(key, param) gives the displacement and load
    factor of a Newton request (a state of a precomputed load path)."""

    def __init__(self, mesh_fn, workers=4, hbm_budget=200 << 30, options_for=None, states=None, **options):
        self.mesh_fn = mesh_fn
        self.states = states     # (key, param) -> (U, tau) of a Newton request; None: from rest at tau = param
        self.options = dict(variant="af", precond="lumped", rtol=1e-8, max_it=10000)
        self.options.update(options)
        self.options_for = options_for     # key -> overrides of the problem options
        self.budget = int(hbm_budget)
        self.held = 0
        self.slots: list[_Slot] = []
        self.lru: OrderedDict = OrderedDict()   # idle slots, oldest first
        self.meshes = {}
        self.est = {}                            # key -> footprint of a problem of that mesh
        self.pending: list[Request] = []
        self.lock = threading.Condition()
        self.closed = False
        self.nworkers = workers
        self.free_workers = workers
        self.jobs: list = []
        self.n_setup = 0        # problems set up (a new one for each request of a busy or absent mesh)
        self.n_evict = 0        # idle problems evicted for memory
        self.threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(workers)]
        for t in self.threads:
            t.start()

    # ------------------------------------------------------------------ public
    def submit(self, req: Request):
        with self.lock:
            self.pending.append(req)
            self._admit()
            self.lock.notify_all()

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for t in self.threads:
            t.join()
        for s in self.slots:
            s.p.close()
        self.slots.clear()

    def mesh(self, key):
        if key not in self.meshes:
            self.meshes[key] = self.mesh_fn(key)
        return self.meshes[key]

    # ---------------------------------------------------------------- internal
    def _estimate(self, key):
        """Device bytes of a new problem of this mesh: measured once a problem
        of it exists, else a bound from its subdomain sizes (dense tile arenas
        for the factor and for the interface inverse and its square)."""
        if key in self.est:
            return self.est[key]
        m = self.mesh(key)
        sub_nodes = np.zeros(m.n_sub)
        for s in range(m.n_sub):
            sub_nodes[s] = np.unique(m.hex8[m.elem_sub == s]).size
        nt = np.ceil(3 * sub_nodes / 64) + 2
        tiles = (nt * (nt + 1) / 2).sum()
        elt = 4 if self.options.get("precision") == "mixed" else 8
        # factor arena, plus the interface arenas (at most as large again),
        # plus sparse rows (81 entries of value and index per local DOF)
        return int(2.0 * tiles * 64 * 64 * elt + 81 * 12 * 3 * sub_nodes.sum())

    def _admit(self):
        """Start pending requests (in arrival order) while slots and memory allow."""
        i = 0
        while i < len(self.pending) and self.free_workers > 0:
            req = self.pending[i]
            slot = next((s for s in self.slots if s.key == req.key and not s.busy), None)
            need = 0 if slot else self._estimate(req.key)
            if slot is None and self.held + need > self.budget:
                # evict idle problems of other meshes, least recently used first
                for s in list(self.lru.values()):
                    if self.held + need <= self.budget:
                        break
                    if s.key != req.key:
                        self._evict(s)
            if slot is None and self.held + need > self.budget:
                if self.slots or self.held > 0:
                    i += 1      # wait for memory; later requests of resident meshes may still run
                    continue
                # nothing resident: try it (the measured footprint decides after setup)
                need = min(need, self.budget)
            self.pending.pop(i)
            if slot is not None:
                slot.busy = True
                self.lru.pop(id(slot), None)
            else:
                self.held += need
            self.free_workers -= 1
            self.jobs.append((req, slot, need))
            self.lock.notify_all()

    def _evict(self, s: _Slot):
        self.n_evict += 1
        self.lru.pop(id(s), None)
        self.slots.remove(s)
        self.held -= s.bytes
        s.p.close()

    def _worker(self):
        while True:
            with self.lock:
                while not self.jobs and not self.closed:
                    self.lock.wait()
                if not self.jobs:
                    return
                req, slot, reserved = self.jobs.pop(0)
            req.t_start = time.perf_counter()
            try:
                if slot is None:
                    opts = dict(self.options)
                    if self.options_for is not None:
                        opts.update(self.options_for(req.key))
                    p = Problem(self.mesh(req.key), **opts)
                    fp = p.footprint()
                    if fp > self.budget:
                        p.close()
                        with self.lock:
                            self.est[req.key] = fp
                        raise MemoryError(f"problem needs {fp} bytes, budget {self.budget}")
                    slot = _Slot(req.key, p, fp)
                    slot.busy = True
                    self.n_setup += 1
                    with self.lock:
                        self.est[req.key] = fp
                        self.held += fp - reserved
                        self.slots.append(slot)
                self._run(req, slot)
            except Exception as e:   # reported on the request
                req.error = f"{type(e).__name__}: {e}"
            req.t_done = time.perf_counter()
            with self.lock:
                if slot is not None and slot in self.slots:
                    slot.busy = False
                    self.lru[id(slot)] = slot
                elif slot is None:
                    self.held -= reserved
                self.free_workers += 1
                self._admit()
                self.lock.notify_all()
            req.done.set()

    def _run(self, req: Request, slot: _Slot):
        p = slot.p
        if req.kind == "solve":
            if not slot.factored_linear:
                p.factor()
                slot.factored_linear = True
            u, st = p.solve(load_factor=req.param)
        else:
            U, tau = self.states(req.key, req.param) if self.states else (np.zeros(p.n_dof), req.param)
            u, _, st = p.newton_step(U, tau)
            slot.factored_linear = False
        req.result = u
        req.iters = st["iters"]


def run_stream(server: Server, stream, t0=None, progress=None, stall_s=None):
    """Submit the requests of `stream` at their arrival times (relative to
    t0) and wait for all; returns the Request objects.  progress: a file to
    which a line is written every 32 submitted requests and every 10 s of
    waiting; stall_s: when no request finishes for that long, print the
    server's state, the running requests and every thread's stack, and end
    the process (exit status 3)."""
    t0 = time.perf_counter() if t0 is None else t0
    reqs = []
    for k, r in enumerate(stream):
        now = time.perf_counter() - t0
        if r["t"] > now:
            time.sleep(r["t"] - now)
        req = Request(k, r["key"], r["kind"], r["param"], t0 + r["t"])
        reqs.append(req)
        server.submit(req)
        if progress is not None and (k + 1) % 32 == 0:
            done = sum(q.done.is_set() for q in reqs)
            print(f"  submitted {k + 1}, done {done}, t = {time.perf_counter() - t0:.1f} s", file=progress, flush=True)
    last_done, last_t = -1, time.perf_counter()
    for r in reqs:
        while not r.done.wait(timeout=10.0):
            done = sum(q.done.is_set() for q in reqs)
            if progress is not None:
                print(f"  done {done} of {len(reqs)}, t = {time.perf_counter() - t0:.1f} s", file=progress,
                      flush=True)
            if done != last_done:
                last_done, last_t = done, time.perf_counter()
            elif stall_s is not None and time.perf_counter() - last_t > stall_s:
                # print what runs and end the process at once: worker threads
                # inside a library call cannot be joined
                import faulthandler
                import os
                now_t = time.perf_counter()
                with server.lock:
                    running = [(q.rid, q.key, q.kind, q.param, round(now_t - q.t_start, 1)) for q in reqs
                               if q.t_start is not None and not q.done.is_set()]
                    state = (f"pending {len(server.pending)}, jobs {len(server.jobs)}, free workers "
                             f"{server.free_workers}, held {server.held / 2**30:.2f} GiB, running "
                             f"(id, key, kind, param, seconds) {running}")
                print(f"no request finished for {stall_s:g} s: {state}", file=sys.stderr, flush=True)
                faulthandler.dump_traceback(file=sys.stderr, all_threads=True)
                sys.stderr.flush()
                os._exit(3)
    return reqs


def summary(reqs, wall):
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {"requests": len(reqs), "failed": len(reqs) - len(ok),
            "throughput_req_per_s": len(ok) / wall if wall > 0 else None,
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                           "p99": 1e3 * float(np.percentile(lat, 99)),
                           "mean": 1e3 * float(lat.mean())},
            "solves": sum(r.kind == "solve" for r in ok),
            "newton_steps": sum(r.kind == "newton" for r in ok),
            "pcg_iterations": int(sum(r.iters for r in ok)),
            "errors": sorted({r.error for r in reqs if r.error})[:3]}


def tube_options(key):
    """Options of tube requests (nearly incompressible HGO): classical FETI
    (the clamped ends stay in the local problems, whose floating versions lose
    definiteness under load), the Dirichlet preconditioner, the exact Newton
    step with the follower-load stiffness, rotations of small stress stiffness
    in the kernels, projected GMRES on the dual problem, and the refinement to
    1e-4 of the step's residual (an inexact Newton step's accuracy)."""
    if key[0].startswith("tube"):
        return dict(variant="classical", precond="dirichlet", load_stiffness=True, kernel_tol=1e-6,
                    dual_gmres=True, ir_tol=1e-4, ir_max=60)
    return {}


def tube_states(mesh, n_steps=10, n_inc=40, iterates=4, **options):
    """States (s, k) -> (tau, U) of the tube's converged load path (load
    steps of 1/n_inc of the full pressure, Newton iterates k < iterates),
    computed once on the GPU with the tube options (warm starts, inexact
    Newton forcing: paper_1508_02599_amd.loadpath)."""
    from .loadpath import trajectory_states
    opts = tube_options(("tube", 0))
    opts.update(dict(rtol=1e-8, max_it=3000, warm_start=True))
    opts.update(options)
    with Problem(mesh, device_ptrs=True, **opts) as p:
        return trajectory_states(p, n_inc=n_inc, n_steps=n_steps, iterates=iterates, log=None)


def state_fn(trajectories):
    """states(key, param) of a Server from {tube kind: tube_states(...)}."""
    def states(key, param):
        tau, U = trajectories[key[0]][tuple(param)]
        return U, tau
    return states


def main():
    from workloads import request_mesh, request_stream
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate-multiples", default="0.25,0.5,1,2,4",
                    help="arrival rates as multiples of the measured saturation rate")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--cube-k", default="2,8")
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    ck = tuple(int(x) for x in a.cube_k.split(","))
    kw = dict(precision=a.precision)
    if a.precision == "mixed":
        kw.update(rtol=1e-6, ir_tol=1e-10, ir_max=20)
    t0 = time.perf_counter()
    traj = {"tube": tube_states(request_mesh(("tube", 128)))}
    print(json.dumps({"trajectory_states": len(traj["tube"]), "trajectory_s": time.perf_counter() - t0}), flush=True)
    srv = Server(request_mesh, workers=a.workers, hbm_budget=int(a.budget_gib * 2**30),
                 options_for=tube_options, states=state_fn(traj), **kw)

    def measure(rate, label):
        stream = request_stream(a.requests, rate, seed=a.seed, cube_k=ck)
        t0 = time.perf_counter()
        reqs = run_stream(srv, stream, t0, progress=sys.stderr, stall_s=120.0)
        wall = max(r.t_done for r in reqs) - t0
        line = {"metric": "served FETI requests", "precision": a.precision, "arrival": label,
                "arrival_rate": rate, "workers": a.workers, "budget_gib": a.budget_gib, "wall_s": wall}
        line.update(summary(reqs, wall))
        line.update({"held_gib": srv.held / 2**30, "problems_resident": len(srv.slots),
                     "problems_set_up": srv.n_setup, "problems_evicted": srv.n_evict})
        print(json.dumps(line), flush=True)
        return line

    try:
        # warm-up (not timed): one request per distinct mesh sets up its problem
        seen = {}
        for r in request_stream(a.requests, 1.0, seed=a.seed, cube_k=ck):
            seen.setdefault(r["key"], dict(r, t=0.0))
        t0 = time.perf_counter()
        run_stream(srv, list(seen.values()))
        print(json.dumps({"warmup_meshes": len(seen), "warmup_s": time.perf_counter() - t0,
                          "held_gib": srv.held / 2**30}), flush=True)
        # saturation: every request arrives at once
        sat = measure(1e9, "all at t=0 (saturation)")["throughput_req_per_s"]
        for mult in (float(x) for x in a.rate_multiples.split(",") if x):
            measure(mult * sat, f"{mult:g} x saturation")
    finally:
        srv.close()


if __name__ == "__main__":
    main()
