"""Served mix of FETI solves and Newton steps (different meshes and subdomain
counts, running concurrently on their own streams; the Newton steps at states
of the tube's converged load path): every result equals the result of the
same request run alone, and admission under a small device memory budget
(evicting idle problems) serves every request."""
import numpy as np
import pytest

from workloads import request_mesh, request_stream

pytestmark = pytest.mark.gpu

KEYS = [("cube", 2), ("cube", 3), ("tube_small", 4), ("tube_small", 8)]


N_STEPS = 3
N_INC = 160   # load steps of 0.1 mmHg on the small tube


def _stream(n=12, seed=1):
    s = request_stream(n, rate=1e6, seed=seed, cube_k=(2, 3), tube_subs=(4, 8), tube_kind="tube_small",
                       n_steps=N_STEPS)
    return s


_TRAJ = {}


def _states():
    from paper_1508_02599_amd.serve import state_fn, tube_states
    if "tube_small" not in _TRAJ:
        _TRAJ["tube_small"] = tube_states(request_mesh(("tube_small", 4)), n_steps=N_STEPS, n_inc=N_INC)
    return state_fn(_TRAJ)


def _alone(stream, fps=None, **extra):
    from paper_1508_02599_amd.feti import Problem
    from paper_1508_02599_amd.serve import tube_options
    states = _states()
    out = []
    for r in stream:
        opts = dict(variant="af", precond="lumped", rtol=1e-8, max_it=10000)
        opts.update(extra)
        opts.update(tube_options(r["key"]))
        with Problem(request_mesh(r["key"]), **opts) as p:
            if fps is not None:
                fps.append(p.footprint())
            if r["kind"] == "solve":
                p.factor()
                u, _ = p.solve(load_factor=r["param"])
            else:
                U, tau = states(r["key"], r["param"])
                u, _, _ = p.newton_step(U, tau)
        out.append(u)
    return out


@pytest.mark.parametrize("tight,precision", [(False, "fp64"), (True, "fp64"), (False, "mixed")])
def test_served_results_equal_alone(tight, precision):
    """tight: the budget holds the largest problem with 20% to spare, so
    requests of other meshes wait and idle problems are evicted.  mixed: FP32
    local factors with the flexible GMRES refinement, whose host-side
    Arnoldi and dot products are as deterministic as the rest."""
    from paper_1508_02599_amd.serve import Server, run_stream, summary, tube_options
    stream = _stream()
    fps = []
    extra = dict(precision=precision) if precision == "fp64" else dict(precision="mixed", rtol=1e-6,
                                                                        ir_tol=1e-10, ir_max=20)
    ref = _alone(stream, fps, **extra)
    budget = int(1.2 * max(fps)) if tight else 64 << 30
    srv = Server(request_mesh, workers=3, hbm_budget=budget, options_for=tube_options, states=_states(),
                 **extra)
    try:
        reqs = run_stream(srv, stream)
        held_max = srv.held
    finally:
        srv.close()
    s = summary(reqs, max(r.t_done for r in reqs) - min(r.arrival for r in reqs))
    print(f"budget {budget / 2**30:.3f} GiB: {s}")
    assert s["failed"] == 0, s["errors"]
    for r, u in zip(reqs, ref):
        d = float(np.abs(r.result - u).max() / np.abs(u).max())
        assert d <= 1e-12, (r.key, r.kind, d)
